"""Library calls as tasks: a rocBLAS single-precision GEMM registered as a
user kernel, so that the scheduler places it in the DAG like its own kernels
(the paper lets library functions that take a stream be computational
elements too, Sec. IV-A).

``Sgemm(ctx)`` registers the call; ``submit(A, B, C, m, n, k)`` adds
C = alpha * A B + beta * C (row-major m x k, k x n, m x n fp32 device
buffers; A and B read-only, C modified) as one task.  The launch callback
sets the task's HIP stream on a rocBLAS handle and calls rocblas_sgemm,
which enqueues the library's own kernels on that stream.
"""

import ctypes as C
import os

from . import dagrt as D

_ROCBLAS_OP_NONE = 111


class _Params(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("k", C.c_int32), ("reserved", C.c_int32),
                ("alpha", C.c_float), ("beta", C.c_float)]


def _rocblas():
    path = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib", "librocblas.so")
    lib = C.CDLL(path)
    lib.rocblas_create_handle.argtypes = [C.POINTER(C.c_void_p)]
    lib.rocblas_destroy_handle.argtypes = [C.c_void_p]
    lib.rocblas_set_stream.argtypes = [C.c_void_p, C.c_void_p]
    lib.rocblas_sgemm.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                  C.POINTER(C.c_float), C.c_void_p, C.c_int, C.c_void_p, C.c_int,
                                  C.POINTER(C.c_float), C.c_void_p, C.c_int]
    for f in ("rocblas_create_handle", "rocblas_destroy_handle", "rocblas_set_stream", "rocblas_sgemm"):
        getattr(lib, f).restype = C.c_int
    return lib


class Sgemm:
    """A rocBLAS SGEMM as a task kind of context `ctx` (not thread-safe, like
    the context)."""

    def __init__(self, ctx):
        self.ctx = ctx
        self.lib = _rocblas()
        self.handle = C.c_void_p()
        st = self.lib.rocblas_create_handle(C.byref(self.handle))
        if st != 0:
            raise RuntimeError("rocblas_create_handle failed (%d)" % st)
        self._fn = D.DAG_LAUNCH_FN(self._launch)   # kept alive as long as the object
        self.kid = D.dag_kernel_register(ctx.h, "rocblas_sgemm", self._fn)

    def _launch(self, stream, ptrs, nptrs, params, user):
        if nptrs != 3:
            return 1
        p = C.cast(params, C.POINTER(_Params)).contents
        if self.lib.rocblas_set_stream(self.handle, stream) != 0:
            return 2
        alpha, beta = C.c_float(p.alpha), C.c_float(p.beta)
        # row-major C = A B is column-major C^T = B^T A^T: pass B first
        st = self.lib.rocblas_sgemm(self.handle, _ROCBLAS_OP_NONE, _ROCBLAS_OP_NONE, p.n, p.m, p.k,
                                    C.byref(alpha), ptrs[1], p.n, ptrs[0], p.k, C.byref(beta), ptrs[2], p.n)
        return 0 if st == 0 else 3

    def submit(self, A, B, Cbuf, m, n, k, alpha=1.0, beta=0.0):
        # the library checks no sizes for user kernels: check them here, on the host
        if min(m, n, k) <= 0 or max(m, n, k) >= 1 << 31:
            raise ValueError("m, n, k must be in [1, 2^31)")
        for buf, need, what in ((A, 4 * m * k, "A"), (B, 4 * k * n, "B"), (Cbuf, 4 * m * n, "C")):
            if self.ctx.ptr(buf)[1] < need:
                raise ValueError("%s smaller than %d bytes" % (what, need))
        prm = _Params(m, n, k, 0, alpha, beta)
        self._prm = prm
        return D.dag_submit_kernel(self.ctx.h, self.kid, prm,
                                   [(A, D.DAG_CONST), (B, D.DAG_CONST), (Cbuf, D.DAG_MUTABLE)])

    def close(self):
        if self.handle:
            self.lib.rocblas_destroy_handle(self.handle)
            self.handle = C.c_void_p()
