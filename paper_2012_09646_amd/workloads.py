"""Seeded synthetic inputs and task programs of the benchmark workloads.

This module is the only code shared by the product path and the CPU oracle.
It draws random numbers and lays out data; it holds none of the scheduler's
logic and none of the task kernels' arithmetic.

Random numbers come from numpy's Philox4x32-10 counter-based generator
(Salmon et al., SC'11), keyed by the workload seed.

A *program* is a list of operations in program order (dicts, see
``oracle.dag`` and ``runner``) plus a buffer table
``name -> Buf(nbytes, loc, init)`` where ``loc`` is ``'device'`` or
``'host'`` (pinned host memory) and ``init`` is a numpy array (or None for
zero-filled buffers).  Kernel argument order follows the kernel signatures
declared in ``include/dagrt.h``.
"""

from dataclasses import dataclass

import numpy as np

F32 = np.float32


def rng(seed):
    return np.random.Generator(np.random.Philox(key=int(seed)))


def uniform_f32(seed, n, lo=0.0, hi=1.0, stream=0):
    """n float32 values ~ U[lo, hi) from Philox(seed); ``stream`` selects an
    independent sub-sequence (jumped generator) for multi-array inputs."""
    g = np.random.Generator(np.random.Philox(key=int(seed)).jumped(int(stream)))
    u = g.random(int(n), dtype=np.float32)
    if lo == 0.0 and hi == 1.0:
        return u
    return (F32(lo) + F32(hi - lo) * u).astype(F32)


# ---------------------------------------------------------------------------
# Power-law graph: every source has `deg` distinct out-neighbours (no
# self-loops); targets follow a Zipf(alpha) rank distribution mapped through a
# seeded random permutation of vertex ids, so in-degrees are power-law.
# ---------------------------------------------------------------------------
def zipf_graph(seed, n, deg=20, alpha=1.5):
    """Return (src, dst) int64 arrays of n*deg edges."""
    g = rng(seed)
    ranks = np.arange(1, n + 1, dtype=np.float64)
    pmf = ranks ** (-alpha)
    cdf = np.cumsum(pmf)
    cdf /= cdf[-1]
    perm = g.permutation(n).astype(np.int64)

    def draw(k):
        u = g.random(k)
        r = np.searchsorted(cdf, u, side="right")
        return perm[np.minimum(r, n - 1)]

    src = np.repeat(np.arange(n, dtype=np.int64), deg).reshape(n, deg)
    dst = draw(n * deg).reshape(n, deg)
    todo = np.arange(n)
    while todo.size:
        sub = dst[todo]
        order = np.argsort(sub, axis=1, kind="stable")
        s = np.take_along_axis(sub, order, axis=1)
        dup_sorted = np.zeros_like(s, dtype=bool)
        dup_sorted[:, 1:] = s[:, 1:] == s[:, :-1]
        bad = np.zeros_like(dup_sorted)
        np.put_along_axis(bad, order, dup_sorted, axis=1)
        bad |= sub == src[todo]
        rows_bad = bad.any(axis=1)
        if not rows_bad.any():
            break
        todo = todo[rows_bad]
        bad = bad[rows_bad]
        sub = sub[rows_bad]
        sub[bad] = draw(int(bad.sum()))
        dst[todo] = sub
    return src.ravel(), dst.ravel()


def csr(nrows, rows, cols):
    """CSR (row_ptr int32, col int32, val float32 = 1) of the 0/1 matrix with
    ones at (rows, cols); column indices sorted within each row."""
    ncols = int(cols.max()) + 1 if cols.size else 1
    key = np.sort(rows.astype(np.int64) * ncols + cols.astype(np.int64))
    r = key // ncols
    c = (key - r * ncols).astype(np.int32)
    counts = np.bincount(r, minlength=nrows)
    row_ptr = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] > np.iinfo(np.int32).max:
        raise ValueError("nnz exceeds int32 indexing")
    return row_ptr.astype(np.int32), c, np.ones(c.size, dtype=F32)


# ---------------------------------------------------------------------------
# Programs
# ---------------------------------------------------------------------------
@dataclass
class Buf:
    nbytes: int
    loc: str = "device"
    init: object = None     # numpy array (any dtype) or None = zeros


@dataclass
class Program:
    name: str
    bufs: dict
    ops: list
    outputs: list           # buffer names whose final contents are checked
    result: str = ""        # the buffer a serving request returns


def K(kernel, args, **params):
    return {"kind": "kernel", "kernel": kernel, "params": params,
            "args": [tuple(a) for a in args]}


def COPY(dst, src, nbytes):
    return {"kind": "copy", "dst": dst, "src": src, "bytes": int(nbytes)}


def HR(buf):
    return {"kind": "host_read", "buf": buf}


def vec_program(n=1 << 20, seed=0):
    """Vector diamond: x <- x^2, y <- y^2 (independent), r = sum(x - y),
    host reads r."""
    x = uniform_f32(seed, n, stream=0)
    y = uniform_f32(seed, n, stream=1)
    bufs = {"x": Buf(4 * n, init=x), "y": Buf(4 * n, init=y), "r": Buf(4)}
    ops = [K("vec_square", [("x", "m")], n=n),
           K("vec_square", [("y", "m")], n=n),
           K("vec_sum_diff", [("x", "c"), ("y", "c"), ("r", "m")], n=n),
           HR("r")]
    return Program("vec", bufs, ops, ["x", "y", "r"], "r")


BS_K, BS_R, BS_SIGMA, BS_T = 25.0, 0.08, 0.3, 1.0


def bs_program(n=1 << 22, tasks=10, seed=1):
    """Black-Scholes fan-out: per task, pinned host spot prices are copied to
    the device, priced, and the call prices copied back; host reads at the
    end.  No edges between tasks."""
    bufs, ops = {}, []
    for i in range(tasks):
        bufs["S%d" % i] = Buf(4 * n, "host", uniform_f32(seed, n, 10.0, 50.0, stream=i))
        bufs["C%d" % i] = Buf(4 * n, "host")
        bufs["dS%d" % i] = Buf(4 * n)
        bufs["dC%d" % i] = Buf(4 * n)
    for i in range(tasks):
        ops.append(COPY("dS%d" % i, "S%d" % i, 4 * n))
        ops.append(K("bs_call", [("dS%d" % i, "c"), ("dC%d" % i, "m")],
                     n=n, K=BS_K, r=BS_R, sigma=BS_SIGMA, T=BS_T))
        ops.append(COPY("C%d" % i, "dC%d" % i, 4 * n))
    for i in range(tasks):
        ops.append(HR("C%d" % i))
    return Program("bs", bufs, ops, ["C%d" % i for i in range(tasks)], "C0")


IMG_KSIZES = (3, 7, 15)


def img_program(side=2048, seed=2, height=None):
    """Image pipeline: for k in (3, 7, 15): blur_k -> sobel_k -> minmax_k ->
    normalise_k, then one unsharp-mask combine of all branches; breadth-first
    submission order; host reads the output."""
    w = side
    h = side if height is None else height
    n = w * h
    bufs = {"img": Buf(4 * n, init=uniform_f32(seed, n)), "out": Buf(4 * n)}
    for k in IMG_KSIZES:
        for p in ("B", "S", "N"):
            bufs["%s%d" % (p, k)] = Buf(4 * n)
        bufs["M%d" % k] = Buf(8)
    ops = []
    for k in IMG_KSIZES:
        ops.append(K("gauss_blur", [("img", "c"), ("B%d" % k, "m")], w=w, h=h, ksize=k))
    for k in IMG_KSIZES:
        ops.append(K("sobel", [("B%d" % k, "c"), ("S%d" % k, "m")], w=w, h=h))
    for k in IMG_KSIZES:
        ops.append(K("minmax", [("S%d" % k, "c"), ("M%d" % k, "m")], n=n))
    for k in IMG_KSIZES:
        ops.append(K("normalise", [("S%d" % k, "c"), ("M%d" % k, "c"), ("N%d" % k, "m")], n=n))
    ops.append(K("unsharp_combine",
                 [("img", "c"), ("B3", "c"), ("B7", "c"), ("B15", "c"),
                  ("N3", "c"), ("N7", "c"), ("N15", "c"), ("out", "m")], n=n))
    ops.append(HR("out"))
    outs = ["B%d" % k for k in IMG_KSIZES] + ["S%d" % k for k in IMG_KSIZES] + \
           ["M%d" % k for k in IMG_KSIZES] + ["N%d" % k for k in IMG_KSIZES] + ["out"]
    return Program("img", bufs, ops, outs, "out")


def hits_graph(n=1 << 20, deg=20, seed=3, alpha=1.5):
    """CSR of A (rows = sources) and A^T (rows = targets) of the power-law
    graph: dict with a_ptr, a_col, a_val, at_ptr, at_col, at_val."""
    src, dst = zipf_graph(seed, n, deg, alpha)
    a_ptr, a_col, a_val = csr(n, src, dst)
    at_ptr, at_col, at_val = csr(n, dst, src)
    return dict(a_ptr=a_ptr, a_col=a_col, a_val=a_val,
                at_ptr=at_ptr, at_col=at_col, at_val=at_val)


def hits_iteration_ops(n, nnz):
    """A has a fixed out-degree, so its product uses the short-row SpMV;
    A^T has power-law rows and uses the merge-path SpMV."""
    sp = dict(nrows=n, ncols=n, nnz=nnz)
    return [
        K("spmv", [("at_ptr", "c"), ("at_col", "c"), ("at_val", "c"), ("h", "c"), ("at", "m")], **sp),
        K("spmv_rows", [("a_ptr", "c"), ("a_col", "c"), ("a_val", "c"), ("a", "c"), ("ht", "m")], **sp),
        K("sumsq", [("at", "c"), ("sa", "m")], n=n),
        K("sumsq", [("ht", "c"), ("sh", "m")], n=n),
        K("scale_l2", [("at", "c"), ("sa", "c"), ("a", "m")], n=n),
        K("scale_l2", [("ht", "c"), ("sh", "c"), ("h", "m")], n=n),
    ]


def hits_program(n=1 << 20, deg=20, iters=10, seed=3, graph=None):
    """HITS: per iteration auth_tmp = A^T hub, hub_tmp = A auth, their squared
    norms, and the normalised auth / hub (two chains with cross edges)."""
    gr = hits_graph(n, deg, seed) if graph is None else graph
    nnz = int(gr["a_ptr"][-1])
    bufs = {k: Buf(v.nbytes, init=v) for k, v in gr.items()}
    ones = np.ones(n, dtype=F32)
    bufs["a"] = Buf(4 * n, init=ones)
    bufs["h"] = Buf(4 * n, init=ones.copy())
    bufs["at"] = Buf(4 * n)
    bufs["ht"] = Buf(4 * n)
    bufs["sa"] = Buf(8)
    bufs["sh"] = Buf(8)
    ops = []
    for _ in range(iters):
        ops.extend(hits_iteration_ops(n, nnz))
    ops.append(HR("a"))
    ops.append(HR("h"))
    return Program("hits", bufs, ops, ["a", "h", "at", "ht", "sa", "sh"], "a")


ML_FEATURES, ML_CLASSES, ML_CATEGORIES = 200, 10, 16


def ml_inputs(seed, n, features=ML_FEATURES, classes=ML_CLASSES, categories=ML_CATEGORIES):
    """Synthetic data and random-initialised model parameters of the ML
    ensemble (nothing is trained; the paper uses random data):

    X          (n, F) float32 category codes, uniform over 0..V-1
    log_theta  (C, F, V) float32 log P(feature f = v | class c): each
               (c, f) row is a random distribution with weights U[0.5, 1)
    log_prior  (C,) float32 log class priors, weights U[0.5, 1)
    mean, scale (F,) float32 standardisation of the ridge branch, near the
               mean and standard deviation of a uniform code
    W          (C, F) float32 ridge coefficients U[-0.25, 0.25)
    b          (C,) float32 ridge intercepts U[-0.1, 0.1)
    """
    g = np.random.Generator(np.random.Philox(key=int(seed)))
    F, C, V = int(features), int(classes), int(categories)
    X = g.integers(0, V, size=(int(n), F)).astype(F32)
    wt = g.uniform(0.5, 1.0, size=(C, F, V))
    log_theta = np.log(wt / wt.sum(axis=2, keepdims=True)).astype(F32)
    wp = g.uniform(0.5, 1.0, size=C)
    log_prior = np.log(wp / wp.sum()).astype(F32)
    mu = (V - 1) / 2.0
    sd = np.sqrt((V * V - 1) / 12.0) if V > 1 else 1.0
    mean = (mu + g.uniform(-0.5, 0.5, size=F)).astype(F32)
    scale = (sd * g.uniform(0.9, 1.1, size=F)).astype(F32)
    W = g.uniform(-0.25, 0.25, size=(C, F)).astype(F32)
    b = g.uniform(-0.1, 0.1, size=C).astype(F32)
    return dict(X=X, log_theta=log_theta, log_prior=log_prior, mean=mean, scale=scale, W=W, b=b)


def ml_program(n=1 << 20, seed=5, features=ML_FEATURES, classes=ML_CLASSES, categories=ML_CATEGORIES):
    """ML ensemble: naive Bayes posteriors and ridge posteriors of the same
    rows (independent branches sharing the read-only X, stored feature-major
    so that the threads of a wave, one row each, read consecutive words),
    then their average and argmax; host reads the labels."""
    d = ml_inputs(seed, n, features, classes, categories)
    d["X"] = np.ascontiguousarray(d["X"].T)   # stored feature-major: feature f of row r at f*n + r
    C = int(classes)
    bufs = {k: Buf(v.nbytes, init=v) for k, v in d.items()}
    for name in ("Pnb", "Prr", "Pavg"):
        bufs[name] = Buf(4 * int(n) * C)
    bufs["label"] = Buf(4 * int(n))
    sz = dict(n=int(n), features=int(features), classes=C, categories=int(categories))
    ops = [K("nb_proba", [("X", "c"), ("log_theta", "c"), ("log_prior", "c"), ("Pnb", "m")], **sz),
           K("ridge_proba", [("X", "c"), ("mean", "c"), ("scale", "c"), ("W", "c"), ("b", "c"), ("Prr", "m")],
             **sz),
           K("ensemble", [("Pnb", "c"), ("Prr", "c"), ("Pavg", "m"), ("label", "m")], **sz),
           HR("label")]
    return Program("ml", bufs, ops, ["Pnb", "Prr", "Pavg", "label"], "label")


DL_CHANNELS = (16, 32)    # output channels of the two convolution layers
DL_EMBED = 16             # embedding size


def dl_inputs(seed, side=1024, channels=DL_CHANNELS, embed=DL_EMBED):
    """Two input images (1 channel, side x side, U[0,1)) and random-initialised
    weights of the network (nothing is trained): He-uniform convolution and
    dense weights, small uniform biases."""
    g = np.random.Generator(np.random.Philox(key=int(seed)))
    c1, c2 = int(channels[0]), int(channels[1])
    s = int(side)

    def he(shape, fan_in):
        a = np.sqrt(6.0 / fan_in)
        return g.uniform(-a, a, size=shape).astype(F32)

    d = {"img1": g.random((1, s, s), dtype=np.float32), "img2": g.random((1, s, s), dtype=np.float32),
         "w1": he((c1, 1, 3, 3), 9), "b1": g.uniform(-0.05, 0.05, size=c1).astype(F32),
         "w2": he((c2, c1, 3, 3), 9 * c1), "b2": g.uniform(-0.05, 0.05, size=c2).astype(F32)}
    n = c2 * (s // 4) * (s // 4)
    d["we"] = he((n, int(embed)), n)     # stored input-major: the weights of input i adjacent
    d["be"] = g.uniform(-0.05, 0.05, size=int(embed)).astype(F32)
    d["wc"] = he((2 * int(embed),), 2 * int(embed))
    d["bc"] = g.uniform(-0.05, 0.05, size=1).astype(F32)
    return d


def dl_program(side=1024, seed=6, channels=DL_CHANNELS, embed=DL_EMBED):
    """Siamese CNN: each image through conv(3x3)+ReLU+pool twice and a dense
    embedding (the two branches share the read-only weights), then one dense
    layer with a sigmoid combines the embeddings; host reads the output."""
    d = dl_inputs(seed, side, channels, embed)
    s, c1, c2, m = int(side), int(channels[0]), int(channels[1]), int(embed)
    bufs = {k: Buf(v.nbytes, init=v) for k, v in d.items()}
    for i in (1, 2):
        bufs["a%d" % i] = Buf(4 * c1 * (s // 2) * (s // 2))
        bufs["f%d" % i] = Buf(4 * c2 * (s // 4) * (s // 4))
        bufs["e%d" % i] = Buf(4 * m)
    bufs["p"] = Buf(4)
    n = c2 * (s // 4) * (s // 4)
    ops = []
    for i in (1, 2):
        ops.append(K("conv3x3_relu_pool", [("img%d" % i, "c"), ("w1", "c"), ("b1", "c"), ("a%d" % i, "m")],
                     cin=1, cout=c1, h=s, w=s))
    for i in (1, 2):
        ops.append(K("conv3x3_relu_pool", [("a%d" % i, "c"), ("w2", "c"), ("b2", "c"), ("f%d" % i, "m")],
                     cin=c1, cout=c2, h=s // 2, w=s // 2))
    for i in (1, 2):
        ops.append(K("dense", [("f%d" % i, "c"), ("we", "c"), ("be", "c"), ("e%d" % i, "m")], n=n, m=m))
    ops.append(K("siamese_combine", [("e1", "c"), ("e2", "c"), ("wc", "c"), ("bc", "c"), ("p", "m")], m=m))
    ops.append(HR("p"))
    return Program("dl", bufs, ops, ["a1", "a2", "f1", "f2", "e1", "e2", "p"], "p")


def initial_arrays(prog):
    """Fresh numpy arrays (uint8 views over the initial contents) for a program."""
    out = {}
    for name, b in prog.bufs.items():
        if b.init is None:
            out[name] = np.zeros(b.nbytes, dtype=np.uint8)
        else:
            arr = np.ascontiguousarray(b.init).view(np.uint8).ravel().copy()
            if arr.size != b.nbytes:
                raise ValueError("init size mismatch for %s" % name)
            out[name] = arr
    return out


# ---------------------------------------------------------------------------
# Serving mix: request shapes and arrival traces
# ---------------------------------------------------------------------------
SERVE_KS = (-4, -3, -2, -1, 0)


def img_side(k):
    """Image side for size scale 2^k (pixels scale with 2^k), rounded to 32."""
    return int(round(2048 * 2.0 ** (k / 2.0) / 32.0)) * 32


def serve_program(kind, k, seed=4, graphs=None):
    """Program of one request shape: workload `kind` at footprint scale 2^k."""
    if kind == "vec":
        return vec_program(n=1 << (20 + k), seed=seed)
    if kind == "bs":
        return bs_program(n=1 << (22 + k), tasks=10, seed=seed)
    if kind == "img":
        return img_program(side=img_side(k), seed=seed)
    if kind == "hits":
        n = 1 << (20 + k)
        g = graphs.get(n) if graphs is not None else None
        if g is None:
            g = hits_graph(n, 20, seed)
            if graphs is not None:
                graphs[n] = g
        return hits_program(n=n, iters=10, graph=g)
    raise ValueError(kind)


def poisson_trace(seed, n, rate_per_s, nshapes):
    """Open-loop arrivals: exponential inter-arrival times at `rate_per_s`,
    shapes uniform over range(nshapes).  Returns (arrival_ns int64, shape int32)."""
    g = rng(seed)
    gaps = g.exponential(1e9 / rate_per_s, size=n)
    arrival = np.cumsum(gaps).astype(np.int64)
    shape = g.integers(0, nshapes, size=n).astype(np.int32)
    return arrival, shape
