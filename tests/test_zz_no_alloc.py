"""dag_launch_static, the launch that allocates nothing (its scratch is a
fixed device array), against dag_submit_kernel, which runs the same kernel
with a context's per-stream scratch: same inputs, same launch configuration,
outputs equal bit for bit.  Each kernel is called twice in a row through the
static entry point, the second time on a smaller input, so the second call
starts from the array as the first one left it."""

import numpy as np
import pytest

from paper_2012_09646_amd import dagrt as D
from paper_2012_09646_amd import workloads as W

pytestmark = pytest.mark.gpu


def banner(s):
    print("[no-alloc] " + s, flush=True)


class Case:
    """One kernel on device buffers of a context: the scheduler's result and
    the static launch's result for the same parameters."""

    def __init__(self, ctx, kernel, inputs, outputs):
        self.ctx = ctx
        self.kid = D.KERNEL_IDS[kernel]
        self.kernel = kernel
        self.inputs = inputs      # [(name, np array)]
        self.outputs = outputs    # [(name, nbytes)]
        self.h = {}
        for name, arr in inputs:
            self.h[name] = ctx.alloc(arr.nbytes)
            ctx.host_write(self.h[name], arr)
        for name, nb in outputs:
            self.h[name] = ctx.alloc(nb)
            self.h[name + "@static"] = ctx.alloc(nb)

    def args(self, static):
        names = [n for n, _ in self.inputs] + [n + ("@static" if static else "") for n, _ in self.outputs]
        return [self.h[n] for n in names]

    def scheduled(self, params):
        hs = self.args(False)
        mode = [D.DAG_CONST] * len(self.inputs) + [D.DAG_MUTABLE] * len(self.outputs)
        D.dag_submit_kernel(self.ctx.h, self.kid, params, list(zip(hs, mode)))
        out = {}
        for name, nb in self.outputs:
            out[name] = np.zeros(nb, np.uint8)
            self.ctx.host_read(self.h[name], out[name])
        return out

    def static(self, params):
        hs = self.args(True)
        ptrs, sizes = zip(*[self.ctx.ptr(h) for h in hs])
        cfg = D.dag_kernel_get_launch(self.ctx.h, self.kid)
        D.dag_launch_static(self.kid, params, list(ptrs), list(sizes), cfg=cfg,
                            stream=D.dag_stream_handle(self.ctx.h, 0))
        self.ctx.sync()  # waits for the context's streams, the static launch's included
        out = {}
        for name, nb in self.outputs:
            out[name] = np.zeros(nb, np.uint8)
            self.ctx.host_read(self.h[name + "@static"], out[name])
        return out


def run_twice(case, params_big, params_small):
    for tag, prm in (("first", params_big), ("second (smaller)", params_small)):
        want = case.scheduled(prm)
        got = case.static(prm)
        for name in want:
            assert np.array_equal(got[name], want[name]), "%s %s call: %s differs" % (case.kernel, tag, name)


def f32(seed, n, lo=0.0, hi=1.0):
    return W.uniform_f32(seed, n, lo, hi)


@pytest.mark.parametrize("variant", [0, 1])
def test_sum_diff(variant):
    banner("vec_sum_diff variant %d" % variant)
    n = (1 << 20) + 3
    with D.Context() as ctx:
        c = Case(ctx, "vec_sum_diff", [("x", f32(1, n)), ("y", f32(2, n))], [("r", 4)])
        cfg = D.dag_kernel_get_launch(ctx.h, c.kid)
        cfg.variant = variant
        D.dag_kernel_set_launch(ctx.h, c.kid, cfg)
        run_twice(c, D.dag_p_n(n), D.dag_p_n(1000))


def test_sumsq_and_minmax():
    banner("sumsq, minmax")
    n = (1 << 21) + 5
    v = f32(3, n, -1.0, 1.0)
    with D.Context() as ctx:
        run_twice(Case(ctx, "sumsq", [("v", v)], [("s", 8)]), D.dag_p_n(n), D.dag_p_n(777))
        run_twice(Case(ctx, "minmax", [("v", v)], [("M", 8)]), D.dag_p_n(n), D.dag_p_n(4099))


def test_spmv_merge_path():
    banner("spmv merge path")
    n = 1 << 15
    g = W.hits_graph(n=n, deg=20, seed=9)
    x = f32(4, n)
    nnz = int(g["at_ptr"][-1])
    with D.Context() as ctx:
        c = Case(ctx, "spmv", [("p", g["at_ptr"]), ("c", g["at_col"]), ("v", g["at_val"]), ("x", x)],
                 [("y", 4 * n)])
        run_twice(c, D.dag_p_csr(n, n, nnz), D.dag_p_csr(n // 4 + 3, n, int(g["at_ptr"][n // 4 + 3])))


def test_dense():
    banner("dense")
    n, m = 1 << 18, 16
    with D.Context() as ctx:
        c = Case(ctx, "dense", [("x", f32(5, n)), ("W", f32(6, n * m, -0.1, 0.1)), ("b", f32(7, m))],
                 [("y", 4 * m)])
        run_twice(c, D.dag_p_dense(n, m, 0), D.dag_p_dense(5000, 4, 0))
