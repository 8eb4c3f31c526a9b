"""Pins of the oracle's task math against closed forms, invariants, library
routines and brute force (CPU only)."""

import math

import numpy as np
import pytest
from scipy import integrate, ndimage, sparse

from oracle import run as orun
from oracle import tasks as T
from paper_2012_09646_amd import workloads as W


def test_vec_square_is_ieee_single_product():
    x = W.uniform_f32(11, 4096)
    x = np.concatenate([x, np.float32([0.0, 1.0, 3.0, 1e-20, 1.5e-45, 3.4e38])])
    with np.errstate(over="ignore", under="ignore"):
        ref = x * x                      # numpy float32 multiply, IEEE rounding
    assert np.array_equal(T.vec_square(x).view(np.uint32), ref.view(np.uint32))
    assert T.vec_square(np.float32([3.0]))[0] == 9.0


def test_vec_sum_diff_closed_forms():
    n = 4096
    i = np.arange(n, dtype=np.float32)
    x = i / np.float32(1024.0)           # exact binary fractions
    y = np.zeros(n, np.float32)
    assert T.vec_sum_diff(x, y) == np.float32(n * (n - 1) / 2 / 1024.0)
    # difference order matters: sum(x - y) = -sum(y - x)
    assert T.vec_sum_diff(y, x) == -np.float32(n * (n - 1) / 2 / 1024.0)
    assert T.vec_sum_diff(x, x) == 0.0
    # cancellation: exact, unlike a float32 running sum
    x2 = np.float32([1e8, 1.0, -1e8, 1.0])
    assert T.vec_sum_diff(x2, np.zeros(4, np.float32)) == 2.0


def _bs_quadrature(S, K, r, sigma, T_):
    """Discounted expectation of (S_T - K)^+ under the lognormal law, by
    numerical integration over the standard normal variable."""
    mu = math.log(S) + (r - 0.5 * sigma * sigma) * T_
    sd = sigma * math.sqrt(T_)
    z0 = (math.log(K) - mu) / sd

    def f(z):
        return (math.exp(mu + sd * z) - K) * math.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)

    val, _ = integrate.quad(f, z0, z0 + 40.0, epsabs=1e-13, epsrel=1e-12, limit=200)
    return math.exp(-r * T_) * val


@pytest.mark.parametrize("S", [10.0, 17.5, 24.0, 25.0, 31.25, 42.0, 50.0])
def test_bs_call_matches_lognormal_quadrature(S):
    K, r, sig, T_ = W.BS_K, W.BS_R, W.BS_SIGMA, W.BS_T
    got = float(T.bs_call(np.float32([S]), K, r, sig, T_)[0])
    ref = _bs_quadrature(S, K, r, sig, T_)
    assert abs(got - ref) <= 2e-7 * max(ref, 1e-3) + 1e-9


def test_bs_call_other_parameters_quadrature():
    for (S, K, r, sig, T_) in [(42.0, 40.0, 0.1, 0.2, 0.5), (100.0, 90.0, 0.01, 0.6, 2.0)]:
        got = float(T.bs_call(np.float32([S]), K, r, sig, T_)[0])
        assert abs(got - _bs_quadrature(S, K, r, sig, T_)) < 2e-5


def test_bs_call_invariants():
    S = W.uniform_f32(1, 20000, 10.0, 50.0)
    K, r, sig, T_ = W.BS_K, W.BS_R, W.BS_SIGMA, W.BS_T
    C = T.bs_call(S, K, r, sig, T_).astype(np.float64)
    Sd = S.astype(np.float64)
    lower = np.maximum(Sd - K * math.exp(-r * T_), 0.0)
    assert np.all(C >= lower * (1 - 1e-6)) and np.all(C <= Sd)
    order = np.argsort(S)
    assert np.all(np.diff(C[order]) >= -1e-6)
    # vanishing volatility -> intrinsic value of the forward
    c0 = T.bs_call(np.float32([30.0, 20.0]), K, r, 1e-6, T_)
    assert abs(c0[0] - (30.0 - K * math.exp(-r * T_))) < 1e-5 and c0[1] < 1e-6


def test_gauss_weights():
    for k in (3, 7, 15):
        w = T.gauss_weights(k)
        s = k / 6.0
        assert w.size == k and abs(w.sum() - 1.0) < 1e-15
        assert np.allclose(w, w[::-1], rtol=0, atol=0)
        c = (k - 1) // 2
        assert abs(w[c + 1] / w[c] - math.exp(-1.0 / (2 * s * s))) < 1e-14


@pytest.mark.parametrize("k", [3, 7, 15])
def test_gauss_blur_vs_separable_library(k):
    img = W.uniform_f32(5, 37 * 29).reshape(29, 37)
    w = T.gauss_weights(k)
    ref = ndimage.correlate1d(img.astype(np.float64), w, axis=1, mode="nearest")
    ref = ndimage.correlate1d(ref, w, axis=0, mode="nearest")
    got = T.gauss_blur(img, k)
    assert np.array_equal(got, ref.astype(np.float32)) or \
        np.max(np.abs(got - ref) / np.abs(ref)) < 1.2e-7


def test_gauss_blur_constant_and_impulse():
    c = np.full((20, 24), 0.375, np.float32)
    assert np.all(T.gauss_blur(c, 15) == np.float32(0.375))
    imp = np.zeros((31, 31), np.float32)
    imp[15, 15] = 1.0
    w = T.gauss_weights(7)
    out = T.gauss_blur(imp, 7)
    assert np.allclose(out[12:19, 12:19], np.outer(w, w).astype(np.float32), rtol=1e-7, atol=0)
    assert out[:12].max() == 0.0


def test_sobel_vs_library_and_ramps():
    img = W.uniform_f32(6, 33 * 21).reshape(21, 33)
    a = img.astype(np.float64)
    gx = ndimage.correlate(a, T.SOBEL_X, mode="nearest")
    gy = ndimage.correlate(a, T.SOBEL_X.T, mode="nearest")
    ref = np.sqrt(gx * gx + gy * gy).astype(np.float32)
    assert np.array_equal(T.sobel(img), ref)
    yy, xx = np.mgrid[0:16, 0:16].astype(np.float32)
    assert np.all(T.sobel(xx)[1:-1, 1:-1] == 8.0)
    assert np.all(T.sobel(yy)[1:-1, 1:-1] == 8.0)
    assert np.all(T.sobel(3 * xx + 4 * yy)[1:-1, 1:-1] == 40.0)
    assert np.all(T.sobel(np.ones((5, 5), np.float32)) == 0.0)


def test_minmax_normalise():
    s = W.uniform_f32(7, 1000) * np.float32(3.0)
    mx, mn = T.minmax(s)
    assert mx == max(s.tolist()) and mn == min(s.tolist())
    nrm = T.normalise(s, mx, mn)
    assert nrm[np.argmax(s)] == 1.0 and nrm[np.argmin(s)] == 0.0
    assert np.all((nrm >= 0) & (nrm <= 1))
    assert np.all(T.normalise(np.full(9, 2.0, np.float32), 2.0, 2.0) == 0.0)
    assert T.normalise(np.float32([1.5]), 2.0, 1.0)[0] == 0.5


def test_unsharp_combine_hand_values():
    one = lambda v: np.float32([v])
    out = T.unsharp_combine(one(0.5), one(0.25), one(0.5), one(0.75), one(0.3), one(0.6), one(0.9))
    assert abs(out[0] - 0.7) < 1e-7
    # constant image -> unchanged, whatever the edge weight
    c = one(0.4)
    for e in (0.0, 0.5, 1.0):
        assert abs(T.unsharp_combine(c, c, c, c, one(e), one(e), one(e))[0] - 0.4) < 1e-7
    # clamped to [0, 1]
    assert T.unsharp_combine(one(1.0), one(0.0), one(0.0), one(0.0), one(1), one(1), one(1))[0] == 1.0
    assert T.unsharp_combine(one(0.0), one(1.0), one(0.0), one(0.0), one(1), one(1), one(1))[0] == 0.0


def test_spmv_vs_library_and_dense():
    src, dst = W.zipf_graph(9, 300, 5)
    rp, ci, va = W.csr(300, src, dst)
    va = W.uniform_f32(9, va.size)
    x = W.uniform_f32(10, 300)
    A = sparse.csr_matrix((va.astype(np.float64), ci, rp), shape=(300, 300))
    ref = (A @ x.astype(np.float64)).astype(np.float32)
    got = T.spmv(rp, ci, va, x)
    assert np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-30)) < 1.2e-7
    dense = A.toarray() @ x.astype(np.float64)
    assert np.allclose(got, dense, rtol=2e-7, atol=0)
    # empty rows give exact zeros
    assert np.all(got[np.diff(rp) == 0] == 0.0)


def test_sumsq_scale_closed_forms():
    v = np.arange(1, 1001, dtype=np.float32)
    assert T.sumsq(v) == 1000 * 1001 * 2001 / 6
    t = np.float32([3.0, 4.0])
    assert np.array_equal(T.scale_l2(t, T.sumsq(t)), np.float32([0.6, 0.8]))


def test_hits_converges_to_singular_vectors():
    n = 48
    src, dst = W.zipf_graph(12, n, 6)
    g = {}
    g["a_ptr"], g["a_col"], g["a_val"] = W.csr(n, src, dst)
    g["at_ptr"], g["at_col"], g["at_val"] = W.csr(n, dst, src)
    A = np.zeros((n, n))
    A[src, dst] = 1.0
    U, S, Vt = np.linalg.svd(A)
    assert S[0] > 1.05 * S[1]
    auth, hub = T.hits(g["a_ptr"], g["a_col"], g["a_val"], g["at_ptr"], g["at_col"], g["at_val"], 400)
    v = np.abs(Vt[0])
    u = np.abs(U[:, 0])
    assert np.allclose(auth, v, atol=2e-5) and np.allclose(hub, u, atol=2e-5)


def test_hits_even_steps_equal_sequential_hits():
    # both products read the previous iterate, so two steps of this form equal
    # one step of the textbook sequential update a <- A^T A a (normalised)
    n = 40
    src, dst = W.zipf_graph(13, n, 5)
    A = np.zeros((n, n))
    A[src, dst] = 1.0
    g = W.csr(n, src, dst) + W.csr(n, dst, src)
    auth, _ = T.hits(*g, 6)
    a = np.ones(n)
    for _ in range(3):
        a = A.T @ (A @ a)
        a /= np.linalg.norm(a)
    assert np.allclose(auth, a, rtol=1e-6, atol=1e-7)


def test_program_executor_vec_and_img():
    prog = W.vec_program(n=1000)
    bufs = W.initial_arrays(prog)
    x0 = bufs["x"].view(np.float32).copy()
    y0 = bufs["y"].view(np.float32).copy()
    reads = orun.execute(prog.ops, bufs)
    assert np.array_equal(bufs["x"].view(np.float32), x0 * x0)
    r = reads[0][2].view(np.float32)[0]
    assert r == T.vec_sum_diff(x0 * x0, y0 * y0)
    prog = W.img_program(side=24)
    bufs = W.initial_arrays(prog)
    orun.execute(prog.ops, bufs)
    img = prog.bufs["img"].init.reshape(24, 24)
    b7 = T.gauss_blur(img, 7)
    assert np.array_equal(bufs["B7"].view(np.float32).reshape(24, 24), b7)
    s7 = T.sobel(b7)
    m = bufs["M7"].view(np.float32)
    assert (m[0], m[1]) == T.minmax(s7)


def test_program_executor_copies():
    prog = W.bs_program(n=64, tasks=3)
    bufs = W.initial_arrays(prog)
    orun.execute(prog.ops, bufs)
    for i in range(3):
        S = prog.bufs["S%d" % i].init
        ref = T.bs_call(S, W.BS_K, W.BS_R, W.BS_SIGMA, W.BS_T)
        assert np.array_equal(bufs["C%d" % i].view(np.float32), ref)


# --------------------------------------------------------------------------
# ML ensemble
# --------------------------------------------------------------------------
def test_softmax_rows_against_scipy_and_invariants():
    from scipy import special
    g = np.random.default_rng(7)
    S = g.normal(size=(50, 10)) * 5 - 560.0          # naive-Bayes-like magnitudes
    P = T.softmax_rows(S)
    assert np.allclose(P, special.softmax(S, axis=1), rtol=1e-13, atol=0)
    assert np.allclose(P.sum(axis=1), 1.0, rtol=0, atol=1e-15 * 10)
    assert np.allclose(T.softmax_rows(S + 123.25), P, rtol=1e-12, atol=0)   # shift invariance
    assert np.array_equal(T.softmax_rows(np.full((3, 4), -7.0)), np.full((3, 4), 0.25))
    # two classes: the logistic function of the score difference
    d = g.normal(size=20)
    two = T.softmax_rows(np.stack([d, np.zeros(20)], axis=1))
    assert np.allclose(two[:, 0], 1.0 / (1.0 + np.exp(-d)), rtol=1e-14, atol=0)


def _fitted_categorical_nb(F, V, C, seed):
    """A categorical naive Bayes model fitted by scikit-learn on random data,
    its parameters rounded to float32 (the in-memory type of the workload)
    and written back so that both sides use identical values."""
    from sklearn.naive_bayes import CategoricalNB
    g = np.random.default_rng(seed)
    Xtr = g.integers(0, V, size=(400, F))
    Xtr[:V, :] = np.arange(V)[:, None]               # every category seen
    ytr = g.integers(0, C, size=400)
    ytr[:C] = np.arange(C)
    m = CategoricalNB(alpha=1.0).fit(Xtr, ytr)
    lt = np.stack([m.feature_log_prob_[f] for f in range(F)], axis=1).astype(np.float32)   # (C, F, V)
    lp = m.class_log_prior_.astype(np.float32)
    m.feature_log_prob_ = [lt[:, f, :].astype(np.float64) for f in range(F)]
    m.class_log_prior_ = lp.astype(np.float64)
    return m, lt, lp


def test_nb_posteriors_match_scikit_learn_categorical_nb():
    F, V, C = 12, 5, 4
    m, lt, lp = _fitted_categorical_nb(F, V, C, 3)
    Xte = np.random.default_rng(4).integers(0, V, size=(300, F))
    ref = m.predict_proba(Xte)
    got = T.nb_predict_proba(Xte.astype(np.float32), lt, lp)
    assert np.allclose(got, ref.astype(np.float32), rtol=2e-7, atol=0)
    J = T.nb_log_joint(Xte.astype(np.float32), lt, lp)
    assert np.array_equal(np.argmax(J, axis=1), m.predict(Xte))


def test_nb_posteriors_by_brute_force_products():
    """P(c | x) = pi_c prod_f theta[c, f, x_f] / sum over classes, with the
    probabilities themselves (no logarithms), in pure Python."""
    d = W.ml_inputs(21, 7, features=6, classes=3, categories=4)
    got = T.nb_predict_proba(d["X"], d["log_theta"], d["log_prior"])
    for r in range(7):
        joint = []
        for c in range(3):
            p = math.exp(float(d["log_prior"][c]))
            for f in range(6):
                p *= math.exp(float(d["log_theta"][c, f, int(d["X"][r, f])]))
            joint.append(p)
        tot = sum(joint)
        for c in range(3):
            assert abs(float(got[r, c]) - joint[c] / tot) <= 1e-6 * joint[c] / tot


def test_ridge_scores_match_scikit_learn_pipeline():
    from sklearn.linear_model import RidgeClassifier
    from sklearn.pipeline import make_pipeline
    from sklearn.preprocessing import StandardScaler
    g = np.random.default_rng(5)
    F, C = 15, 4
    Xtr = g.integers(0, 16, size=(500, F)).astype(np.float64)
    ytr = g.integers(0, C, size=500)
    pipe = make_pipeline(StandardScaler(), RidgeClassifier(alpha=1.0)).fit(Xtr, ytr)
    sc, clf = pipe[0], pipe[1]
    mean, scale = sc.mean_.astype(np.float32), sc.scale_.astype(np.float32)
    Wc, b = clf.coef_.astype(np.float32), clf.intercept_.astype(np.float32)
    sc.mean_, sc.scale_ = mean.astype(np.float64), scale.astype(np.float64)
    clf.coef_, clf.intercept_ = Wc.astype(np.float64), b.astype(np.float64)
    Xte = g.integers(0, 16, size=(200, F)).astype(np.float32)
    ref = pipe.decision_function(Xte.astype(np.float64))
    got = T.ridge_scores(Xte, mean, scale, Wc, b)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)
    assert np.array_equal(np.argmax(got, axis=1), pipe.predict(Xte))
    # a zero coefficient matrix gives the softmax of the intercepts in every row
    P0 = T.ridge_predict_proba(Xte, mean, scale, np.zeros_like(Wc), b)
    e = np.exp(b.astype(np.float64) - b.max())
    assert np.allclose(P0, (e / e.sum()).astype(np.float32)[None, :], rtol=1e-7, atol=0)


def test_ensemble_average_and_lowest_index_ties():
    p_nb = np.float32([[0.25, 0.75, 0.0], [0.5, 0.25, 0.25], [0.2, 0.3, 0.5]])
    p_rr = np.float32([[0.75, 0.25, 0.0], [0.0, 0.25, 0.75], [0.6, 0.3, 0.1]])
    avg, lab = T.ensemble_argmax(p_nb, p_rr)
    assert np.array_equal(avg, np.float32([[0.5, 0.5, 0.0], [0.25, 0.25, 0.5], [0.4, 0.3, 0.3]]))
    assert lab.tolist() == [0, 2, 0]                 # row 0: tie between 0 and 1 -> 0
    # the decision is taken on the exact float64 average, not on its float32 rounding
    a = np.float32(1.0) - np.float32(2.0 ** -24)     # largest float32 below 1
    nb = np.float32([[a, np.float32(1.0)]])
    rr = np.float32([[np.float32(1.0), a]])
    avg, lab = T.ensemble_argmax(nb, rr)
    assert lab[0] == 0 and avg[0, 0] == avg[0, 1]
    nb2 = np.float32([[a, 1.0]])
    rr2 = np.float32([[a, 1.0]])
    assert T.ensemble_argmax(nb2, rr2)[1][0] == 1


def test_ml_program_runs_in_program_order():
    prog = W.ml_program(n=257, seed=5, features=20, classes=10, categories=16)
    arrays = W.initial_arrays(prog)
    orun.execute(prog.ops, arrays)
    d = W.ml_inputs(5, 257, 20, 10, 16)
    pnb = T.nb_predict_proba(d["X"], d["log_theta"], d["log_prior"])
    prr = T.ridge_predict_proba(d["X"], d["mean"], d["scale"], d["W"], d["b"])
    avg, lab = T.ensemble_argmax(pnb, prr)
    assert np.array_equal(arrays["Pnb"].view(np.float32).reshape(257, 10), pnb)
    assert np.array_equal(arrays["label"].view(np.int32), lab)
    assert np.allclose(arrays["Pavg"].view(np.float32).reshape(257, 10).sum(axis=1), 1.0, atol=1e-6)


# --------------------------------------------------------------------------
# DL (Siamese CNN)
# --------------------------------------------------------------------------
def test_conv_relu_pool_against_pytorch_cpu():
    import torch
    F = torch.nn.functional
    g = np.random.default_rng(8)
    for cin, cout, h, w in ((1, 4, 8, 10), (3, 5, 6, 6), (8, 2, 12, 4)):
        x = g.random((cin, h, w), dtype=np.float32)
        wt = (g.random((cout, cin, 3, 3), dtype=np.float32) - 0.5)
        b = (g.random(cout, dtype=np.float32) - 0.5) * 0.1
        ref = F.max_pool2d(torch.relu(F.conv2d(torch.tensor(x, dtype=torch.float64)[None],
                                                torch.tensor(wt, dtype=torch.float64),
                                                torch.tensor(b, dtype=torch.float64), padding=1)), 2)[0]
        got = T.conv3x3_relu_pool(x, wt, b)
        assert got.shape == (cout, h // 2, w // 2)
        assert np.array_equal(got, ref.numpy().astype(np.float32))


def test_conv_relu_pool_brute_force():
    g = np.random.default_rng(9)
    cin, cout, h, w = 2, 2, 4, 6
    x = g.random((cin, h, w), dtype=np.float32)
    wt = g.random((cout, cin, 3, 3), dtype=np.float32) - 0.5
    b = np.float32([0.01, -0.02])
    got = T.conv3x3_relu_pool(x, wt, b)
    for o in range(cout):
        for py in range(h // 2):
            for px in range(w // 2):
                best = 0.0
                for yy in (2 * py, 2 * py + 1):
                    for xx in (2 * px, 2 * px + 1):
                        s = float(b[o])
                        for c in range(cin):
                            for dy in range(3):
                                for dx in range(3):
                                    iy, ix = yy + dy - 1, xx + dx - 1
                                    if 0 <= iy < h and 0 <= ix < w:
                                        s += float(wt[o, c, dy, dx]) * float(x[c, iy, ix])
                        best = max(best, s)
                assert abs(float(got[o, py, px]) - best) <= 1e-7 * max(abs(best), 1e-30)


def test_conv_relu_pool_special_cases():
    g = np.random.default_rng(10)
    x = g.random((2, 6, 8), dtype=np.float32) - 0.5
    ident = np.zeros((2, 2, 3, 3), np.float32)
    ident[0, 0, 1, 1] = 1.0                      # output 0 copies input channel 0
    ident[1, 1, 1, 1] = -1.0                     # output 1 negates input channel 1
    got = T.conv3x3_relu_pool(x, ident, np.zeros(2, np.float32))
    pooled = lambda a: np.maximum(a, 0).reshape(3, 2, 4, 2).max(axis=(1, 3))
    assert np.array_equal(got[0], pooled(x[0]))
    assert np.array_equal(got[1], pooled(-x[1]))
    zero = T.conv3x3_relu_pool(x, np.zeros((3, 2, 3, 3), np.float32), np.float32([0.25, -1.0, 0.0]))
    assert np.all(zero[0] == np.float32(0.25)) and np.all(zero[1] == 0) and np.all(zero[2] == 0)


def test_dense_and_combine_closed_forms():
    g = np.random.default_rng(11)
    x = g.random(50, dtype=np.float32)
    y = T.dense(x, np.ones((3, 50), np.float32), np.float32([0.0, 1.0, -2.0]))
    s = math.fsum(float(v) for v in x)
    assert np.allclose(y.astype(np.float64), [s, s + 1, s - 2], rtol=1e-7, atol=0)
    w = g.random((4, 7), dtype=np.float32) - 0.5
    x7 = g.random(7, dtype=np.float32)
    yb = T.dense(x7, w, np.zeros(4, np.float32))
    for j in range(4):
        ref = sum(float(w[j, i]) * float(x7[i]) for i in range(7))
        assert abs(float(yb[j]) - ref) <= 1e-7 * abs(ref)
    e1, e2 = g.random(5, dtype=np.float32), g.random(5, dtype=np.float32)
    assert T.siamese_combine(e1, e2, np.zeros(10, np.float32), np.float32(0.3)) == np.float32(1 / (1 + math.exp(-0.3)))
    u = g.random(5, dtype=np.float32)
    assert T.siamese_combine(e1, e1, np.concatenate([u, -u]), np.float32(0.0)) == np.float32(0.5)
    assert T.siamese_combine(e1, e2, np.float32([1] * 10), np.float32(-40.0)) < 1e-6


def test_dl_program_runs_in_program_order():
    prog = W.dl_program(side=16, seed=3, channels=(4, 6), embed=5)
    arrays = W.initial_arrays(prog)
    orun.execute(prog.ops, arrays)
    d = W.dl_inputs(3, 16, (4, 6), 5)
    a1 = T.conv3x3_relu_pool(d["img1"], d["w1"], d["b1"])
    f1 = T.conv3x3_relu_pool(a1, d["w2"], d["b2"])
    e1 = T.dense(f1.ravel(), d["we"].T, d["be"])
    a2 = T.conv3x3_relu_pool(d["img2"], d["w1"], d["b1"])
    e2 = T.dense(T.conv3x3_relu_pool(a2, d["w2"], d["b2"]).ravel(), d["we"].T, d["be"])
    assert np.array_equal(arrays["e1"].view(np.float32), e1)
    assert arrays["p"].view(np.float32)[0] == T.siamese_combine(e1, e2, d["wc"], d["bc"][0])
    assert f1.shape == (6, 4, 4)
