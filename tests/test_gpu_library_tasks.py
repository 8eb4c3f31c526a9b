"""A library call (rocBLAS SGEMM) as a task between built-in kernels: the
scheduler infers its edges from the argument modes like for any task, and
the results equal numpy's."""

import sys

import numpy as np
import pytest

from oracle import tasks as T
from paper_2012_09646_amd import dagrt as D

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("m,n,k", [(64, 48, 200), (1000, 10, 200), (3, 5, 7)])
def test_sgemm_task_between_builtin_kernels(m, n, k):
    from paper_2012_09646_amd import library_tasks as L
    print("[gpu] sgemm task m=%d n=%d k=%d" % (m, n, k), flush=True)
    sys.stdout.flush()
    g = np.random.default_rng(m + n + k)
    a0 = g.random((m, k), dtype=np.float32)
    b = g.random((k, n), dtype=np.float32)
    ctx = D.Context()
    gemm = L.Sgemm(ctx)
    try:
        hA0, hA, hB, hC, hs = (ctx.alloc(a0.nbytes), ctx.alloc(a0.nbytes), ctx.alloc(b.nbytes),
                               ctx.alloc(4 * m * n), ctx.alloc(8))
        ctx.host_write(hA0, a0)
        ctx.host_write(hB, b)
        t1 = ctx.kernel("copy_f32", [(hA0, "c"), (hA, "m")], n=m * k)          # A = A0
        t2 = gemm.submit(hA, hB, hC, m, n, k)                                   # C = A B (library)
        t3 = ctx.kernel("sumsq", [(hC, "c"), (hs, "m")], n=m * n)              # s = sum C^2
        c = np.zeros(m * n, np.float32)
        s = np.zeros(1, np.float64)
        ctx.host_read(hC, c)
        ctx.host_read(hs, s)
        pairs = {(src, dst) for src, dst, _, _ in ctx.edges()}
        assert (t1, t2) in pairs and (t2, t3) in pairs and (t1, t3) not in pairs
        ref = a0.astype(np.float64) @ b.astype(np.float64)
        assert np.allclose(c.reshape(m, n), ref, rtol=1e-5, atol=1e-5 * k)     # fp32 accumulation in rocBLAS
        assert abs(s[0] - T.sumsq(c)) <= 1e-12 * T.sumsq(c)                    # our kernel on its output
        with pytest.raises(ValueError):
            gemm.submit(hA, hB, hC, m + 1, n, k)                                # buffers too small
    finally:
        gemm.close()
        ctx.close()
