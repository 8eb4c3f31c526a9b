"""GPU parity of the ML ensemble workload: the naive Bayes and ridge
posteriors and their average within 1e-5 relative of the oracle; the
ensemble kernel bit-exact (average and label) when it reads the oracle's
posteriors; the labels of the whole pipeline equal to the oracle's except at
a near-tie, where the chosen class must be within the tolerance of the best."""

import sys

import numpy as np
import pytest

import gpu_util as G
from oracle import dag as odag
from paper_2012_09646_amd import dagrt as D
from paper_2012_09646_amd import runner
from paper_2012_09646_amd import workloads as W

pytestmark = pytest.mark.gpu


def banner(msg):
    print("[gpu] " + msg, flush=True)
    sys.stdout.flush()


def run(prog, launch=None):
    ctx = D.Context()
    try:
        for k, cfg in (launch or {}).items():
            ctx.set_launch(k, *cfg)
        b = runner.Bound(ctx, prog)
        b.run()
        outs = {name: b.read(name) for name in prog.outputs}
        edges = b.edges()
    finally:
        ctx.close()
    return outs, edges


def check_labels(lab_g, lab_o, avg_o, C):
    """Labels equal the oracle's; where they differ the oracle's average of
    the chosen class must be within 2e-5 of the row's largest (a near-tie
    that rounding may break either way)."""
    lab_g = lab_g.view(np.int32)
    lab_o = lab_o.view(np.int32)
    avg = avg_o.view(np.float32).reshape(-1, C).astype(np.float64)
    assert np.all((lab_g >= 0) & (lab_g < C))
    diff = np.nonzero(lab_g != lab_o)[0]
    for r in diff:
        assert avg[r, lab_g[r]] >= avg[r].max() * (1 - 2e-5), "row %d: label %d vs %d" % (r, lab_g[r], lab_o[r])
    return diff.size


@pytest.mark.parametrize("n,F,C,V", [(3000, 200, 10, 16), (1, 200, 10, 16), (777, 13, 3, 5),
                                     (1000, 128, 16, 16), (500, 1, 1, 1), (2049, 64, 7, 9)])
def test_ml_pipeline(n, F, C, V):
    banner("ml n=%d F=%d C=%d V=%d" % (n, F, C, V))
    prog = W.ml_program(n=n, seed=n + F, features=F, classes=C, categories=V)
    ref = G.oracle_run(prog)
    outs, edges = run(prog)
    assert edges == odag.build_dag(prog.ops).edges
    for name in ("Pnb", "Prr", "Pavg"):
        G.assert_close(prog, name, outs[name], ref[name])
    flips = check_labels(outs["label"], ref["label"], ref["Pavg"], C)
    print("[gpu] labels differing from the oracle's at near-ties: %d of %d rows" % (flips, n), flush=True)
    assert flips <= max(1, n // 100)  # near-ties are rare on these inputs


@pytest.mark.parametrize("C", [10, 16])
@pytest.mark.parametrize("launch", [
    {"nb_proba": (256, 3, 0), "ridge_proba": (512, 2, 0), "ensemble": (64, 5, 0)},
    {"nb_proba": (64, 0, 0), "ridge_proba": (64, 0, 0), "ensemble": (1024, 0, 0)},
    {"nb_proba": (512, 1, 0), "ridge_proba": (128, 1, 0), "ensemble": (128, 1, 0)},
    {"nb_proba": (1024, 256, 0), "ridge_proba": (256, 1024, 4), "ensemble": (256, 0, 0)},
    {"nb_proba": (1024, 256, 0), "ridge_proba": (64, 3, 4), "ensemble": (256, 0, 0)},
    {"nb_proba": (1024, 256, 0), "ridge_proba": (256, 1024, 2), "ensemble": (256, 0, 0)},
    {"nb_proba": (1024, 256, 0), "ridge_proba": (64, 5, 2), "ensemble": (256, 0, 0)},
])
def test_ml_launch_configurations(launch, C):
    """Grid-stride loops that wrap several times, single workgroups, small
    and large workgroups, one, two or four rows per thread: same results."""
    banner("ml launch %s C=%d" % (launch, C))
    F = 200 if C == 10 else 127
    # 5004 rows: a multiple of 4, so the two- and four-row variants run (5003 would fall back to one row)
    prog = W.ml_program(n=5004 if launch["ridge_proba"][2] in (2, 4) else 5003, seed=9, features=F, classes=C,
                        categories=16)
    ref = G.oracle_run(prog)
    outs, _ = run(prog, launch)
    for name in ("Pnb", "Prr", "Pavg"):
        G.assert_close(prog, name, outs[name], ref[name])
    check_labels(outs["label"], ref["label"], ref["Pavg"], C)


@pytest.mark.parametrize("n,C,tied", [(4099, 10, False), (4099, 10, True), (333, 1, True), (1000, 16, True)])
def test_ensemble_bit_exact_on_the_oracles_posteriors(n, C, tied):
    """The ensemble kernel alone, reading the same float32 inputs as the
    oracle: average and label bit-exact; with values drawn from a small set
    most rows hold ties, which must go to the lowest class index."""
    banner("ensemble n=%d C=%d tied=%d" % (n, C, tied))
    g = np.random.default_rng(n + C)
    if tied:
        a = g.choice(np.float32([0.0, 0.25, 0.5, 1.0]), size=(n, C)).astype(np.float32)
        b = g.choice(np.float32([0.0, 0.25, 0.5, 1.0]), size=(n, C)).astype(np.float32)
    else:
        a = g.random((n, C), dtype=np.float32)
        b = g.random((n, C), dtype=np.float32)
    bufs = {"Pnb": W.Buf(a.nbytes, init=a), "Prr": W.Buf(b.nbytes, init=b),
            "Pavg": W.Buf(4 * n * C), "label": W.Buf(4 * n)}
    ops = [W.K("ensemble", [("Pnb", "c"), ("Prr", "c"), ("Pavg", "m"), ("label", "m")],
               n=n, features=1, classes=C, categories=1), W.HR("label")]
    prog = W.Program("ens", bufs, ops, ["Pavg", "label"], "label")
    ref = G.oracle_run(prog)
    outs, _ = run(prog)
    assert np.array_equal(outs["Pavg"], ref["Pavg"])
    assert np.array_equal(outs["label"], ref["label"])
    if tied and C > 1:
        assert np.any(ref["label"].view(np.int32) > 0)


@pytest.mark.parametrize("ridge_launch", [None, (256, 1024, 2), (256, 4096, 4)])
def test_ml_full_size_sampled(ridge_launch):
    """The benchmark's shape (2^20 rows, 200 features, 10 classes, 16
    categories) in the default launch configuration and with the two- and
    four-row ridge kernels: 4096 sampled rows against the oracle computed for
    those rows alone (rows are independent)."""
    from oracle import tasks as T
    n = 1 << 20
    banner("ml full size n=%d ridge %s" % (n, ridge_launch))
    prog = W.ml_program(n=n, seed=5)
    outs, _ = run(prog, {"ridge_proba": ridge_launch} if ridge_launch else None)
    d = {k: prog.bufs[k].init for k in ("X", "log_theta", "log_prior", "mean", "scale", "W", "b")}
    rows = np.sort(np.random.default_rng(1).choice(n, 4096, replace=False))
    rows[0], rows[-1] = 0, n - 1
    X = d["X"][:, rows].T                        # stored feature-major
    pnb = T.nb_predict_proba(X, d["log_theta"], d["log_prior"])
    prr = T.ridge_predict_proba(X, d["mean"], d["scale"], d["W"], d["b"])
    avg, lab = T.ensemble_argmax(pnb, prr)
    g_nb = outs["Pnb"].view(np.float32).reshape(n, 10)[rows]
    g_rr = outs["Prr"].view(np.float32).reshape(n, 10)[rows]
    g_avg = outs["Pavg"].view(np.float32).reshape(n, 10)[rows]
    for g, o in ((g_nb, pnb), (g_rr, prr), (g_avg, avg)):
        assert np.all(np.abs(g.astype(np.float64) - o) <= 1e-5 * np.abs(o.astype(np.float64)))
    check_labels(np.ascontiguousarray(outs["label"].view(np.int32)[rows]), lab, avg, 10)


@pytest.mark.parametrize("F", [1, 3, 8, 9, 17])
@pytest.mark.parametrize("variant", [0, 2, 4])
def test_ridge_few_features(variant, F):
    """Ridge alone with fewer features than the loads kept in flight (and
    just above): the loads ahead stop at the last feature."""
    banner("ridge variant=%d F=%d" % (variant, F))
    from oracle import tasks as T
    n, C = 1004, 10
    g = np.random.default_rng(F + 10 * variant)
    X = (g.random((F, n), dtype=np.float32) * 4.0 - 2.0).astype(np.float32)    # feature-major
    mean = (g.random(F, dtype=np.float32) - 0.5).astype(np.float32)
    scale = (g.random(F, dtype=np.float32) + 0.5).astype(np.float32)
    Wt = (g.random((C, F), dtype=np.float32) - 0.5).astype(np.float32)
    b = (g.random(C, dtype=np.float32) - 0.5).astype(np.float32)
    ref = T.ridge_predict_proba(np.ascontiguousarray(X.T), mean, scale, Wt, b)
    ctx = D.Context(max_streams=1)
    try:
        ctx.set_launch("ridge_proba", 64, 3, variant)
        hs = [ctx.alloc(a.nbytes) for a in (X, mean, scale, Wt, b)]
        for h_, a in zip(hs, (X, mean, scale, Wt, b)):
            ctx.host_write(h_, a)
        hp = ctx.alloc(4 * n * C)
        ctx.kernel("ridge_proba", [(h_, "c") for h_ in hs] + [(hp, "m")], n=n, features=F, classes=C)
        P = np.zeros((n, C), np.float32)
        ctx.host_read(hp, P)
    finally:
        ctx.close()
    assert np.all(np.abs(P.astype(np.float64) - ref) <= 1e-5 * np.abs(ref.astype(np.float64)))


def test_ml_zero_rows():
    """n = 0: nothing is launched, the call succeeds."""
    banner("ml zero rows")
    ctx = D.Context()
    try:
        bufs = [ctx.alloc(4096) for _ in range(7)]
        ctx.kernel("nb_proba", [(bufs[0], "c"), (bufs[1], "c"), (bufs[2], "c"), (bufs[3], "m")],
                   n=0, features=4, classes=2, categories=2)
        ctx.kernel("ridge_proba", [(bufs[0], "c"), (bufs[1], "c"), (bufs[2], "c"), (bufs[4], "c"),
                                   (bufs[5], "c"), (bufs[6], "m")], n=0, features=20, classes=10)
        ctx.sync()
    finally:
        ctx.close()


@pytest.mark.parametrize("graph_mode", [0, 2])
def test_ml_graph_region_outputs_read_right_after_the_launch(graph_mode):
    """The ML DAG recorded as a hipGraph region (graph mode 0, and mode 2,
    which also makes it a graph since it has no host copies), replayed many
    times, then once more into cleared outputs: every output read right
    after that launch equals the eager run bit for bit."""
    banner("ml graph region reads graph_mode=%d" % graph_mode)
    n = 1 << 18
    prog = W.ml_program(n=n, seed=5)
    outs, _ = run(prog)
    ctx = D.Context(graph_mode=graph_mode)
    try:
        b = runner.Bound(ctx, prog, read_bytes=4)
        b.record(1)
        ctx.sync()
        for _ in range(30):
            b.replay(1, 1)
        for o in prog.outputs:
            ctx.host_write(b.h[o], np.zeros(prog.bufs[o].nbytes, np.uint8))
        b.replay(1, 1)
        for o in prog.outputs:
            assert np.array_equal(b.read(o), outs[o]), o
    finally:
        ctx.close()
