"""Execute a program strictly in program order on the CPU (test infrastructure).

Buffers are named 1-D numpy arrays.  Kernel operations name one of the task
kernels below and pass their arguments positionally; the order of the
arguments and their meaning is the kernel signature documented with each
entry of ``KERNELS``.  Copies move bytes; host reads snapshot a buffer; host
writes overwrite one.  Nothing runs concurrently and nothing is reordered.
"""

import numpy as np

from . import tasks


def _f32(a, n=None):
    v = a.view(np.float32)
    return v if n is None else v[:n]


def _k_vec_square(p, x):
    n = p["n"]
    _f32(x, n)[:] = tasks.vec_square(_f32(x, n))


def _k_vec_sum_diff(p, x, y, r):
    n = p["n"]
    _f32(r)[0] = tasks.vec_sum_diff(_f32(x, n), _f32(y, n))


def _k_bs_call(p, s, c):
    n = p["n"]
    _f32(c, n)[:] = tasks.bs_call(_f32(s, n), p["K"], p["r"], p["sigma"], p["T"])


def _img(a, p):
    return _f32(a, p["w"] * p["h"]).reshape(p["h"], p["w"])


def _k_gauss_blur(p, src, dst):
    _img(dst, p)[:] = tasks.gauss_blur(_img(src, p), p["ksize"])


def _k_sobel(p, src, dst):
    _img(dst, p)[:] = tasks.sobel(_img(src, p))


def _k_minmax(p, src, m):
    mx, mn = tasks.minmax(_f32(src, p["n"]))
    _f32(m)[0] = mx
    _f32(m)[1] = mn


def _k_normalise(p, s, m, out):
    n = p["n"]
    _f32(out, n)[:] = tasks.normalise(_f32(s, n), _f32(m)[0], _f32(m)[1])


def _k_unsharp_combine(p, img, b3, b7, b15, n3, n7, n15, out):
    n = p["n"]
    ins = [_f32(a, n) for a in (img, b3, b7, b15, n3, n7, n15)]
    _f32(out, n)[:] = tasks.unsharp_combine(*ins)


def _k_spmv(p, row_ptr, col, val, x, y):
    nr, nc, nnz = p["nrows"], p["ncols"], p["nnz"]
    rp = row_ptr.view(np.int32)[: nr + 1]
    ci = col.view(np.int32)[:nnz]
    _f32(y, nr)[:] = tasks.spmv(rp, ci, _f32(val, nnz), _f32(x, nc))


def _k_sumsq(p, v, s):
    s.view(np.float64)[0] = tasks.sumsq(_f32(v, p["n"]))


def _k_scale_l2(p, t, s, v):
    n = p["n"]
    _f32(v, n)[:] = tasks.scale_l2(_f32(t, n), s.view(np.float64)[0])


def _ml(p):
    return p["n"], p["features"], p["classes"], p["categories"]


def _rows(X, n, F):
    """The n x F matrix of a feature-major buffer (feature f of row r at f*n + r)."""
    return _f32(X, n * F).reshape(F, n).T


def _k_nb_proba(p, X, lt, lp, P):
    n, F, C, V = _ml(p)
    _f32(P, n * C).reshape(n, C)[:] = tasks.nb_predict_proba(
        _rows(X, n, F), _f32(lt, C * F * V).reshape(C, F, V), _f32(lp, C))


def _k_ridge_proba(p, X, mean, scale, W, b, P):
    n, F, C, _ = _ml(p)
    _f32(P, n * C).reshape(n, C)[:] = tasks.ridge_predict_proba(
        _rows(X, n, F), _f32(mean, F), _f32(scale, F), _f32(W, C * F).reshape(C, F), _f32(b, C))


def _k_ensemble(p, p_nb, p_rr, avg, label):
    n, _, C, _ = _ml(p)
    a, lab = tasks.ensemble_argmax(_f32(p_nb, n * C).reshape(n, C), _f32(p_rr, n * C).reshape(n, C))
    _f32(avg, n * C).reshape(n, C)[:] = a
    label.view(np.int32)[:n] = lab


def _k_conv3x3_relu_pool(p, x, w, b, y):
    cin, cout, h, wd = p["cin"], p["cout"], p["h"], p["w"]
    _f32(y, cout * (h // 2) * (wd // 2))[:] = tasks.conv3x3_relu_pool(
        _f32(x, cin * h * wd).reshape(cin, h, wd), _f32(w, cout * cin * 9).reshape(cout, cin, 3, 3),
        _f32(b, cout)).ravel()


def _k_dense(p, x, w, b, y):
    """W is stored input-major (n x m); the layer's matrix is its transpose."""
    n, m = p["n"], p["m"]
    _f32(y, m)[:] = tasks.dense(_f32(x, n), _f32(w, m * n).reshape(n, m).T, _f32(b, m))


def _k_siamese_combine(p, e1, e2, w, b, out):
    m = p["m"]
    _f32(out)[0] = tasks.siamese_combine(_f32(e1, m), _f32(e2, m), _f32(w, 2 * m), _f32(b)[0])


def _k_spin(p, *bufs):
    """Delay kernel used by the scheduler tests: no effect on data."""


# name -> function(params, *buffers) ; signature (argument order, mode):
KERNELS = {
    "vec_square": _k_vec_square,            # x:m
    "vec_sum_diff": _k_vec_sum_diff,        # x:c y:c r:m  (r float32 at [0])
    "bs_call": _k_bs_call,                  # S:c C:m
    "gauss_blur": _k_gauss_blur,            # in:c out:m
    "sobel": _k_sobel,                      # in:c out:m
    "minmax": _k_minmax,                    # in:c M:m     (M = [max, min])
    "normalise": _k_normalise,              # S:c M:c N:m
    "unsharp_combine": _k_unsharp_combine,  # img B3 B7 B15 N3 N7 N15 :c out:m
    "spmv": _k_spmv,                        # row_ptr col val x :c  y:m
    "spmv_rows": _k_spmv,                   # same product (an implementation choice of the caller)
    "sumsq": _k_sumsq,                      # v:c s:m      (s float64)
    "scale_l2": _k_scale_l2,                # t:c s:c v:m
    "spin": _k_spin,                        # any
    "nb_proba": _k_nb_proba,                # X lt lp :c P:m      (X feature-major; n x C posteriors)
    "ridge_proba": _k_ridge_proba,          # X mean scale W b :c P:m
    "ensemble": _k_ensemble,                # Pnb Prr :c avg:m label:m (int32)
    "conv3x3_relu_pool": _k_conv3x3_relu_pool,  # x w b :c y:m      (channel-major)
    "dense": _k_dense,                      # x W b :c y:m        (y = W x + b, W stored n x m)
    "siamese_combine": _k_siamese_combine,  # e1 e2 w b :c p:m    (p = sigmoid(w.[e1;e2] + b))
}


def execute(ops, buffers):
    """Run ``ops`` in program order over ``buffers`` (name -> 1-D array of any
    dtype; modified in place).  Returns the list of host-read snapshots as
    (position, name, bytes-array copy)."""
    bytes_of = {k: v.view(np.uint8) for k, v in buffers.items()}
    reads = []
    for pos, op in enumerate(ops, start=1):
        kind = op["kind"]
        if kind == "kernel":
            fn = KERNELS[op["kernel"]]
            fn(op.get("params", {}), *[bytes_of[b] for b, _ in op["args"]])
        elif kind == "copy":
            nb = op["bytes"]
            so, do = op.get("src_off", 0), op.get("dst_off", 0)
            src = bytes_of[op["src"]][so:so + nb].copy()
            bytes_of[op["dst"]][do:do + nb] = src
        elif kind == "host_read":
            reads.append((pos, op["buf"], bytes_of[op["buf"]].copy()))
        elif kind == "host_write":
            data = np.asarray(op["data"]).view(np.uint8).ravel()
            off = op.get("off", 0)
            bytes_of[op["buf"]][off:off + data.size] = data
        elif kind in ("sync", "macro"):
            if kind == "macro":
                raise ValueError("macro operations carry no math of their own")
        else:
            raise ValueError("unknown op kind %r" % (kind,))
    return reads
