"""ctypes binding of the C ABI declared in include/dagrt.h.

Every ``dag_*`` function of the header is exposed under the same name and
with the same arguments; these wrappers only marshal arguments and turn a
non-zero status into :class:`DagError`.  :class:`Context` is a small
convenience layer over the same calls.  All scheduling and all device work
happen in the native library (``_lib/libdagrt.so``); if it has not been
built this module raises instead of falling back to anything else.
"""

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libdagrt.so")

# ---- constants (mirror include/dagrt.h) --------------------------------------
DAG_OK = 0
STATUS = {0: "DAG_OK", -1: "DAG_E_INVAL", -2: "DAG_E_ALIAS", -3: "DAG_E_NOMEM", -4: "DAG_E_HIP",
          -5: "DAG_E_POISONED", -6: "DAG_E_BUSY", -7: "DAG_E_UNSUPPORTED", -8: "DAG_E_NOTFOUND",
          -9: "DAG_E_RANGE"}
DAG_E_INVAL, DAG_E_RANGE = -1, -9
DAG_CONST, DAG_MUTABLE = 0, 1
DAG_DEVICE, DAG_PINNED_HOST = 0, 1
DAG_SERIAL_SYNC, DAG_PARALLEL_ASYNC = 0, 1
DAG_WAIT_SIGNALS, DAG_WAIT_EVENTS = 0, 1
DAG_EDGE_RAW, DAG_EDGE_WAR, DAG_EDGE_WAW = 0, 1, 2
(DAG_TASK_KERNEL, DAG_TASK_COPY, DAG_TASK_HOST_READ, DAG_TASK_HOST_WRITE, DAG_TASK_SYNC,
 DAG_TASK_REGION, DAG_TASK_RELEASE) = range(7)
DAG_MAX_STREAMS = 64
DAG_K_USER_BASE = 1000

KERNEL_IDS = {
    "vec_square": 1, "vec_sum_diff": 2, "bs_call": 3, "gauss_blur": 4, "sobel": 5,
    "minmax": 6, "normalise": 7, "unsharp_combine": 8, "spmv": 9, "spmv_rows": 10, "sumsq": 11,
    "scale_l2": 12, "spin": 13, "copy_f32": 14,
    "nb_proba": 15, "ridge_proba": 16, "ensemble": 17,
    "conv3x3_relu_pool": 18, "dense": 19, "siamese_combine": 20,
}
KERNEL_NAMES = {v: k for k, v in KERNEL_IDS.items()}


class dag_config(C.Structure):
    _fields_ = [("policy", C.c_uint32), ("max_streams", C.c_uint32), ("trace", C.c_uint32),
                ("dry_run", C.c_uint32), ("device", C.c_int32), ("graph_mode", C.c_uint32),
                ("scratch_bytes", C.c_uint64), ("copy_streams", C.c_uint32),
                ("spin_wait", C.c_uint32), ("copy_lanes", C.c_uint32), ("own_queues", C.c_uint32),
                ("copy_engine", C.c_uint32), ("wait_mode", C.c_uint32)]


class dag_arg(C.Structure):
    _fields_ = [("buf", C.c_uint32), ("mode", C.c_uint32)]


class dag_edge(C.Structure):
    _fields_ = [("src", C.c_uint64), ("dst", C.c_uint64), ("buf", C.c_uint32), ("kind", C.c_uint32)]


class dag_task_info(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("stream", C.c_int32), ("vertex", C.c_uint32),
                ("active", C.c_uint32), ("nparents", C.c_uint32), ("nwaits", C.c_uint32),
                ("kernel_id", C.c_uint32), ("reserved", C.c_uint32),
                ("t_start_ms", C.c_double), ("t_end_ms", C.c_double)]


class dag_stats(C.Structure):
    _fields_ = [("tasks", C.c_uint64), ("vertices", C.c_uint64), ("edges", C.c_uint64),
                ("waits", C.c_uint64), ("host_waits", C.c_uint64), ("streams", C.c_uint32),
                ("active", C.c_uint32), ("submit_host_us", C.c_double),
                ("launch_host_us", C.c_double), ("spmv_plans", C.c_uint64), ("signals", C.c_uint64),
                ("signal_waits", C.c_uint64)]


class dag_launch(C.Structure):
    _fields_ = [("block", C.c_uint32), ("grid_cap", C.c_uint32), ("variant", C.c_uint32),
                ("reserved", C.c_uint32)]


class dag_op(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("kernel_id", C.c_uint32), ("params", C.c_void_p),
                ("params_bytes", C.c_size_t), ("args", C.POINTER(dag_arg)), ("nargs", C.c_uint32),
                ("dst", C.c_uint32), ("src", C.c_uint32), ("reserved", C.c_uint32),
                ("dst_off", C.c_size_t), ("src_off", C.c_size_t), ("bytes", C.c_size_t),
                ("host", C.c_void_p)]


class dag_p_n(C.Structure):
    _fields_ = [("n", C.c_uint64)]


class dag_p_bs(C.Structure):
    _fields_ = [("n", C.c_uint64), ("strike", C.c_double), ("rate", C.c_double),
                ("vol", C.c_double), ("years", C.c_double)]


class dag_p_img(C.Structure):
    _fields_ = [("w", C.c_uint32), ("h", C.c_uint32), ("ksize", C.c_uint32),
                ("reserved", C.c_uint32)]


class dag_p_csr(C.Structure):
    _fields_ = [("nrows", C.c_uint32), ("ncols", C.c_uint32), ("nnz", C.c_uint64)]


class dag_p_spin(C.Structure):
    _fields_ = [("ns", C.c_uint64)]


class dag_sched(C.Structure):
    _fields_ = [("stream", C.c_uint32), ("nwaits", C.c_uint32), ("waits", C.POINTER(C.c_uint32))]


class dag_p_conv(C.Structure):
    _fields_ = [("cin", C.c_uint32), ("cout", C.c_uint32), ("h", C.c_uint32), ("w", C.c_uint32)]


class dag_p_dense(C.Structure):
    _fields_ = [("n", C.c_uint64), ("m", C.c_uint32), ("reserved", C.c_uint32)]


class dag_p_combine(C.Structure):
    _fields_ = [("m", C.c_uint32), ("reserved", C.c_uint32)]


class dag_p_ml(C.Structure):
    _fields_ = [("n", C.c_uint64), ("features", C.c_uint32), ("classes", C.c_uint32),
                ("categories", C.c_uint32), ("reserved", C.c_uint32)]


class dag_shape_buf(C.Structure):
    _fields_ = [("buf", C.c_uint32), ("role", C.c_uint32), ("init_src", C.c_uint32),
                ("reserved", C.c_uint32)]


class dag_serve_config(C.Structure):
    _fields_ = [("budget_bytes", C.c_uint64), ("device_arena_bytes", C.c_uint64),
                ("host_arena_bytes", C.c_uint64), ("lanes", C.c_uint32), ("bypass", C.c_uint32),
                ("copy_lanes", C.c_uint32), ("transfer_lanes", C.c_uint32)]


class dag_request(C.Structure):
    _fields_ = [("shape", C.c_uint32), ("reserved", C.c_uint32), ("arrival_ns", C.c_uint64),
                ("result", C.c_void_p)]


class dag_serve_done(C.Structure):
    _fields_ = [("id", C.c_uint64), ("arrival_ns", C.c_uint64), ("admit_ns", C.c_uint64),
                ("done_ns", C.c_uint64), ("shape", C.c_uint32), ("lane", C.c_uint32)]


class dag_serve_summary(C.Structure):
    _fields_ = [("p50_ms", C.c_double), ("p99_ms", C.c_double), ("mean_ms", C.c_double),
                ("max_ms", C.c_double), ("req_per_s", C.c_double), ("wall_ms", C.c_double),
                ("peak_device_bytes", C.c_uint64), ("max_inflight", C.c_uint32),
                ("max_queued", C.c_uint32), ("completed", C.c_uint64)]


DAG_ROLE_SHARED, DAG_ROLE_PRIVATE, DAG_ROLE_INIT = 0, 1, 2
DAG_SERVE_CONCURRENT, DAG_SERVE_SERIAL = 0, 1
DAG_SERVE_NOW = (1 << 64) - 1

DAG_LAUNCH_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.POINTER(C.c_void_p), C.c_uint32, C.c_void_p,
                            C.c_void_p)

_ctx_t = C.c_void_p
_st = C.c_int32
_P = C.POINTER
_SIGS = {
    "dag_create": (_st, [_P(dag_config), _P(_ctx_t)]),
    "dag_destroy": (_st, [_ctx_t]),
    "dag_last_error": (C.c_char_p, [_ctx_t]),
    "dag_status_string": (C.c_char_p, [_st]),
    "dag_buffer_register": (_st, [_ctx_t, C.c_void_p, C.c_size_t, C.c_uint32, _P(C.c_uint32)]),
    "dag_buffer_alloc": (_st, [_ctx_t, C.c_size_t, C.c_uint32, _P(C.c_uint32)]),
    "dag_buffer_release": (_st, [_ctx_t, C.c_uint32]),
    "dag_buffer_ptr": (_st, [_ctx_t, C.c_uint32, _P(C.c_void_p), _P(C.c_size_t)]),
    "dag_kernel_get_launch": (_st, [_ctx_t, C.c_uint32, _P(dag_launch)]),
    "dag_launch_static": (_st, [C.c_uint32, C.c_void_p, C.c_size_t, _P(C.c_void_p), _P(C.c_size_t),
                                C.c_uint32, _P(dag_launch), C.c_void_p]),
    "dag_kernel_set_launch": (_st, [_ctx_t, C.c_uint32, _P(dag_launch)]),
    "dag_tune_kernel": (_st, [_ctx_t, C.c_uint32, C.c_void_p, C.c_size_t, _P(dag_arg), C.c_uint32,
                              _P(dag_launch), C.c_uint32, C.c_uint32, _P(C.c_uint32), _P(C.c_double)]),
    "dag_kernel_register": (_st, [_ctx_t, C.c_char_p, DAG_LAUNCH_FN, C.c_void_p, _P(C.c_uint32)]),
    "dag_submit_kernel": (_st, [_ctx_t, C.c_uint32, C.c_void_p, C.c_size_t, _P(dag_arg), C.c_uint32,
                                _P(C.c_uint64)]),
    "dag_submit_copy": (_st, [_ctx_t, C.c_uint32, C.c_size_t, C.c_uint32, C.c_size_t, C.c_size_t,
                              _P(C.c_uint64)]),
    "dag_host_read": (_st, [_ctx_t, C.c_uint32, C.c_size_t, C.c_void_p, C.c_size_t, _P(C.c_uint64)]),
    "dag_host_write": (_st, [_ctx_t, C.c_uint32, C.c_size_t, C.c_void_p, C.c_size_t, _P(C.c_uint64)]),
    "dag_sync": (_st, [_ctx_t]),
    "dag_submit_batch": (_st, [_ctx_t, _P(dag_op), C.c_uint32, _P(C.c_uint64), _P(C.c_uint32)]),
    "dag_region_begin": (_st, [_ctx_t, C.c_uint64]),
    "dag_region_end": (_st, [_ctx_t]),
    "dag_region_launch": (_st, [_ctx_t, C.c_uint64, _P(C.c_uint64)]),
    "dag_region_info": (_st, [_ctx_t, C.c_uint64, _P(C.c_uint32), _P(C.c_uint32)]),
    "dag_region_set_schedule": (_st, [_ctx_t, C.c_uint64, _P(dag_sched), C.c_uint32]),
    "dag_region_drop": (_st, [_ctx_t, C.c_uint64]),
    "dag_region_run_begin": (_st, [_ctx_t, C.c_uint64]),
    "dag_region_run_end": (_st, [_ctx_t, _P(C.c_uint64), _P(C.c_uint32)]),
    "dag_edges": (_st, [_ctx_t, _P(dag_edge), C.c_size_t, _P(C.c_size_t)]),
    "dag_task_waits": (_st, [_ctx_t, C.c_uint64, _P(C.c_uint64), C.c_uint32, _P(C.c_uint32)]),
    "dag_task_get_info": (_st, [_ctx_t, C.c_uint64, _P(dag_task_info)]),
    "dag_get_stats": (_st, [_ctx_t, _P(dag_stats)]),
    "dag_trace_reset": (_st, [_ctx_t]),
    "dag_stream_handle": (_st, [_ctx_t, C.c_uint32, _P(C.c_void_p)]),
    "dag_serve_create": (_st, [_ctx_t, _P(dag_serve_config), _P(C.c_void_p)]),
    "dag_serve_destroy": (_st, [C.c_void_p]),
    "dag_serve_add_shape": (_st, [C.c_void_p, C.c_uint64, _P(dag_shape_buf), C.c_uint32, C.c_uint32,
                                  C.c_size_t, C.c_uint64, _P(C.c_uint32)]),
    "dag_serve_shape_info": (_st, [C.c_void_p, C.c_uint32, _P(C.c_uint64), _P(C.c_uint64)]),
    "dag_serve_start": (_st, [C.c_void_p, C.c_uint32]),
    "dag_serve_submit": (_st, [C.c_void_p, C.c_uint32, C.c_uint64, C.c_void_p, _P(C.c_uint64)]),
    "dag_serve_close": (_st, [C.c_void_p]),
    "dag_serve_poll": (_st, [C.c_void_p, C.c_uint64, _P(dag_serve_done), C.c_uint32, _P(C.c_uint32),
                             _P(C.c_uint64)]),
    "dag_serve_stats": (_st, [C.c_void_p, _P(dag_serve_summary)]),
    "dag_serve_run": (_st, [C.c_void_p, _P(dag_request), C.c_uint32, C.c_uint32, _P(dag_serve_done),
                            _P(dag_serve_summary)]),
}

_lib = None


def lib():
    """Load libdagrt.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libdagrt.so is not built (python -m paper_2012_09646_amd.build)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class DagError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status
        self.name = STATUS.get(status, str(status))


def _check(ctx, st):
    if st != DAG_OK:
        m = lib().dag_last_error(ctx)
        raise DagError(st, m.decode() if m else "")


# ---- raw wrappers, one per C function ------------------------------------------
def dag_create(cfg=None):
    h = C.c_void_p()
    st = lib().dag_create(C.byref(cfg) if cfg is not None else None, C.byref(h))
    if st != DAG_OK:
        raise DagError(st, "dag_create failed")
    return h


def dag_destroy(ctx):
    _check(None, lib().dag_destroy(ctx))


def dag_last_error(ctx):
    return lib().dag_last_error(ctx).decode()


def dag_status_string(st):
    return lib().dag_status_string(st).decode()


def dag_buffer_register(ctx, ptr, nbytes, loc):
    out = C.c_uint32()
    _check(ctx, lib().dag_buffer_register(ctx, C.c_void_p(ptr), nbytes, loc, C.byref(out)))
    return out.value


def dag_buffer_alloc(ctx, nbytes, loc):
    out = C.c_uint32()
    _check(ctx, lib().dag_buffer_alloc(ctx, nbytes, loc, C.byref(out)))
    return out.value


def dag_buffer_release(ctx, buf):
    _check(ctx, lib().dag_buffer_release(ctx, buf))


def dag_buffer_ptr(ctx, buf):
    p, n = C.c_void_p(), C.c_size_t()
    _check(ctx, lib().dag_buffer_ptr(ctx, buf, C.byref(p), C.byref(n)))
    return p.value, n.value


def dag_kernel_get_launch(ctx, kid):
    out = dag_launch()
    _check(ctx, lib().dag_kernel_get_launch(ctx, kid, C.byref(out)))
    return out


def dag_kernel_set_launch(ctx, kid, cfg):
    _check(ctx, lib().dag_kernel_set_launch(ctx, kid, C.byref(cfg)))


def dag_tune_kernel(ctx, kid, params, args, candidates, reps=20):
    """candidates: [(block, grid_cap, variant)].  Returns (best index, [us])."""
    arr = _args_array(args)
    cands = (dag_launch * len(candidates))()
    for i, (b, g, v) in enumerate(candidates):
        cands[i] = dag_launch(b, g, v, 0)
    best = C.c_uint32()
    us = (C.c_double * len(candidates))()
    _check(ctx, lib().dag_tune_kernel(ctx, kid, C.byref(params), C.sizeof(params), arr, len(args), cands,
                                      len(candidates), reps, C.byref(best), us))
    return best.value, list(us)


def dag_kernel_register(ctx, name, fn, user=None):
    kid = C.c_uint32()
    _check(ctx, lib().dag_kernel_register(ctx, name.encode(), fn, user, C.byref(kid)))
    return kid.value


def _args_array(args):
    arr = (dag_arg * max(len(args), 1))()
    for i, (b, m) in enumerate(args):
        arr[i].buf = b
        arr[i].mode = m
    return arr


def dag_submit_kernel(ctx, kid, params, args):
    """params: a ctypes parameter struct (or None); args: [(buf, mode)]."""
    arr = _args_array(args)
    out = C.c_uint64()
    pp = C.byref(params) if params is not None else None
    pb = C.sizeof(params) if params is not None else 0
    _check(ctx, lib().dag_submit_kernel(ctx, kid, pp, pb, arr, len(args), C.byref(out)))
    return out.value


def dag_launch_static(kid, params, ptrs, sizes, cfg=None, stream=None):
    """params: a ctypes parameter struct (or None); ptrs: device addresses
    (ints) in the kernel's argument order; sizes: their sizes in bytes;
    cfg: a dag_launch (None = the kernel's default); stream: a hipStream_t
    as an int (None = the null stream)."""
    n = len(ptrs)
    if len(sizes) != n:
        raise ValueError("one size per pointer")
    pa = (C.c_void_p * max(n, 1))(*[C.c_void_p(int(p)) for p in ptrs])
    sa = (C.c_size_t * max(n, 1))(*[int(v) for v in sizes])
    pp = C.byref(params) if params is not None else None
    pb = C.sizeof(params) if params is not None else 0
    st = lib().dag_launch_static(kid, pp, pb, pa, sa, n, C.byref(cfg) if cfg is not None else None,
                                 C.c_void_p(int(stream)) if stream else None)
    _check(None, st)


def dag_submit_copy(ctx, dst, dst_off, src, src_off, nbytes):
    out = C.c_uint64()
    _check(ctx, lib().dag_submit_copy(ctx, dst, dst_off, src, src_off, nbytes, C.byref(out)))
    return out.value


def _host_ptr(arr):
    if arr is None:
        return None
    if not isinstance(arr, np.ndarray) or not arr.flags["C_CONTIGUOUS"]:
        raise ValueError("host buffer must be a C-contiguous numpy array")
    return arr.ctypes.data


def dag_host_read(ctx, buf, off=0, host_dst=None, nbytes=0):
    out = C.c_uint64()
    _check(ctx, lib().dag_host_read(ctx, buf, off, _host_ptr(host_dst), nbytes, C.byref(out)))
    return out.value


def dag_host_write(ctx, buf, off, host_src, nbytes):
    out = C.c_uint64()
    _check(ctx, lib().dag_host_write(ctx, buf, off, _host_ptr(host_src), nbytes, C.byref(out)))
    return out.value


def dag_sync(ctx):
    _check(ctx, lib().dag_sync(ctx))


def dag_submit_batch(ctx, ops):
    """ops: a ctypes array of dag_op (see Batch).  Returns the task ids."""
    n = len(ops)
    ids = (C.c_uint64 * max(n, 1))()
    done = C.c_uint32()
    _check(ctx, lib().dag_submit_batch(ctx, ops, n, ids, C.byref(done)))
    return list(ids[:n])


def dag_region_begin(ctx, key):
    _check(ctx, lib().dag_region_begin(ctx, key))


def dag_region_end(ctx):
    _check(ctx, lib().dag_region_end(ctx))


def dag_region_launch(ctx, key):
    out = C.c_uint64()
    _check(ctx, lib().dag_region_launch(ctx, key, C.byref(out)))
    return out.value


def dag_region_run_begin(ctx, key):
    _check(ctx, lib().dag_region_run_begin(ctx, key))


def dag_region_run_end(ctx):
    """Returns (task id or 0, replayed)."""
    out = C.c_uint64()
    rep = C.c_uint32()
    _check(ctx, lib().dag_region_run_end(ctx, C.byref(out), C.byref(rep)))
    return out.value, bool(rep.value)


def dag_region_info(ctx, key):
    a, b = C.c_uint32(), C.c_uint32()
    _check(ctx, lib().dag_region_info(ctx, key, C.byref(a), C.byref(b)))
    return a.value, b.value


def dag_region_set_schedule(ctx, key, sched):
    """sched: one (stream, [earlier call indices waited for]) per recorded call."""
    arr = (dag_sched * max(len(sched), 1))()
    keep = []
    for k, (stream, waits) in enumerate(sched):
        w = (C.c_uint32 * max(len(waits), 1))(*waits)
        keep.append(w)
        arr[k].stream = int(stream)
        arr[k].nwaits = len(waits)
        arr[k].waits = C.cast(w, _P(C.c_uint32))
    _check(ctx, lib().dag_region_set_schedule(ctx, key, arr, len(sched)))


def dag_region_drop(ctx, key):
    _check(ctx, lib().dag_region_drop(ctx, key))


def dag_edges(ctx):
    n = C.c_size_t()
    _check(ctx, lib().dag_edges(ctx, None, 0, C.byref(n)))
    arr = (dag_edge * max(n.value, 1))()
    _check(ctx, lib().dag_edges(ctx, arr, n.value, C.byref(n)))
    return [(e.src, e.dst, e.buf, e.kind) for e in arr[:n.value]]


def dag_task_waits(ctx, t):
    n = C.c_uint32()
    _check(ctx, lib().dag_task_waits(ctx, t, None, 0, C.byref(n)))
    arr = (C.c_uint64 * max(n.value, 1))()
    _check(ctx, lib().dag_task_waits(ctx, t, arr, n.value, C.byref(n)))
    return list(arr[:n.value])


def dag_task_get_info(ctx, t):
    out = dag_task_info()
    _check(ctx, lib().dag_task_get_info(ctx, t, C.byref(out)))
    return out


def dag_get_stats(ctx):
    out = dag_stats()
    _check(ctx, lib().dag_get_stats(ctx, C.byref(out)))
    return out


def dag_trace_reset(ctx):
    _check(ctx, lib().dag_trace_reset(ctx))


def dag_stream_handle(ctx, i):
    out = C.c_void_p()
    _check(ctx, lib().dag_stream_handle(ctx, i, C.byref(out)))
    return out.value


def dag_serve_create(ctx, cfg):
    out = C.c_void_p()
    _check(ctx, lib().dag_serve_create(ctx, C.byref(cfg), C.byref(out)))
    return out


def dag_serve_destroy(srv):
    lib().dag_serve_destroy(srv)


def dag_serve_add_shape(ctx, srv, key, bufs, result_buf, result_bytes, sim_ns=0):
    """bufs: [(handle, role, init_src)]; returns the shape id.  ctx is used
    for the error message."""
    arr = (dag_shape_buf * len(bufs))()
    for i, (b, role, src) in enumerate(bufs):
        arr[i].buf, arr[i].role, arr[i].init_src = b, role, src
    sid = C.c_uint32()
    _check(ctx, lib().dag_serve_add_shape(srv, key, arr, len(bufs), result_buf, result_bytes, sim_ns,
                                          C.byref(sid)))
    return sid.value


def dag_serve_shape_info(srv, shape):
    a, b = C.c_uint64(), C.c_uint64()
    st = lib().dag_serve_shape_info(srv, shape, C.byref(a), C.byref(b))
    if st != DAG_OK:
        raise DagError(st, "dag_serve_shape_info")
    return a.value, b.value


def dag_serve_start(ctx, srv, mode=DAG_SERVE_CONCURRENT):
    _check(ctx, lib().dag_serve_start(srv, mode))


def dag_serve_submit(srv, shape, arrival_ns=DAG_SERVE_NOW, result=None):
    """Thread-safe (no context message on failure).  result: a C-contiguous
    numpy array (kept alive by the caller until its completion is reported)
    or None.  Returns the request id."""
    rid = C.c_uint64()
    st = lib().dag_serve_submit(srv, int(shape), int(arrival_ns), _host_ptr(result), C.byref(rid))
    if st != DAG_OK:
        raise DagError(st, "dag_serve_submit")
    return rid.value


def dag_serve_close(srv):
    st = lib().dag_serve_close(srv)
    if st != DAG_OK:
        raise DagError(st, "dag_serve_close")


def dag_serve_poll(ctx, srv, wait_us=0, cap=256):
    """Returns (list of dag_serve_done, outstanding)."""
    arr = (dag_serve_done * max(cap, 1))()
    n = C.c_uint32()
    left = C.c_uint64()
    _check(ctx, lib().dag_serve_poll(srv, int(wait_us), arr, cap, C.byref(n), C.byref(left)))
    return [arr[i] for i in range(n.value)], left.value


def dag_serve_stats(srv):
    out = dag_serve_summary()
    st = lib().dag_serve_stats(srv, C.byref(out))
    if st != DAG_OK:
        raise DagError(st, "dag_serve_stats")
    return out


def dag_serve_run(ctx, srv, reqs, mode):
    """reqs: ctypes array of dag_request.  Returns (done array, summary)."""
    n = len(reqs)
    done = (dag_serve_done * max(n, 1))()
    stats = dag_serve_summary()
    _check(ctx, lib().dag_serve_run(srv, reqs, n, mode, done, C.byref(stats)))
    return done, stats


# ---- parameter blocks ------------------------------------------------------------
def make_params(kernel, p):
    """ctypes parameter block of a built-in kernel from a dict of values."""
    if kernel in ("vec_square", "vec_sum_diff", "minmax", "normalise", "unsharp_combine",
                  "sumsq", "scale_l2", "copy_f32"):
        return dag_p_n(int(p["n"]))
    if kernel == "bs_call":
        return dag_p_bs(int(p["n"]), float(p["K"]), float(p["r"]), float(p["sigma"]), float(p["T"]))
    if kernel in ("gauss_blur", "sobel"):
        return dag_p_img(int(p["w"]), int(p["h"]), int(p.get("ksize", 0)), 0)
    if kernel in ("spmv", "spmv_rows"):
        return dag_p_csr(int(p["nrows"]), int(p["ncols"]), int(p["nnz"]))
    if kernel == "spin":
        return dag_p_spin(int(p.get("ns", 0)))
    if kernel == "conv3x3_relu_pool":
        return dag_p_conv(int(p["cin"]), int(p["cout"]), int(p["h"]), int(p["w"]))
    if kernel == "dense":
        return dag_p_dense(int(p["n"]), int(p["m"]), 0)
    if kernel == "siamese_combine":
        return dag_p_combine(int(p["m"]), 0)
    if kernel in ("nb_proba", "ridge_proba", "ensemble"):
        return dag_p_ml(int(p["n"]), int(p["features"]), int(p["classes"]), int(p.get("categories", 1)), 0)
    raise KeyError(kernel)


class Context:
    """Convenience wrapper: one execution context with its buffers."""

    def __init__(self, policy=DAG_PARALLEL_ASYNC, max_streams=8, trace=0, dry_run=False,
                 device=0, graph_mode=0, scratch_bytes=0, copy_streams=0, spin_wait=0, copy_lanes=1,
                 own_queues=0, copy_engine=0, wait_mode=0):
        self.cfg = dag_config(policy, max_streams, int(trace), int(bool(dry_run)), device,
                              graph_mode, scratch_bytes, copy_streams, int(spin_wait), int(copy_lanes),
                              int(own_queues), int(copy_engine), int(wait_mode))
        self.h = dag_create(self.cfg)

    def close(self):
        if self.h:
            dag_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # buffers
    def alloc(self, nbytes, loc=DAG_DEVICE):
        return dag_buffer_alloc(self.h, int(nbytes), loc)

    def register(self, ptr, nbytes, loc=DAG_DEVICE):
        return dag_buffer_register(self.h, ptr, int(nbytes), loc)

    def release(self, buf):
        dag_buffer_release(self.h, buf)

    def ptr(self, buf):
        return dag_buffer_ptr(self.h, buf)

    # calls
    def kernel(self, kernel, args, **params):
        kid = KERNEL_IDS[kernel] if isinstance(kernel, str) else kernel
        prm = make_params(KERNEL_NAMES.get(kid, ""), params) if kid in KERNEL_NAMES else params.get("params")
        return dag_submit_kernel(self.h, kid, prm, [(b, DAG_MUTABLE if m in ("m", 1) else DAG_CONST)
                                                    for b, m in args])

    def copy(self, dst, src, nbytes, dst_off=0, src_off=0):
        return dag_submit_copy(self.h, dst, dst_off, src, src_off, int(nbytes))

    def host_read(self, buf, out=None, off=0):
        return dag_host_read(self.h, buf, off, out, 0 if out is None else out.nbytes)

    def host_write(self, buf, data, off=0):
        data = np.ascontiguousarray(data)
        return dag_host_write(self.h, buf, off, data, data.nbytes)

    def sync(self):
        dag_sync(self.h)

    # introspection
    def edges(self):
        return dag_edges(self.h)

    def waits(self, t):
        return dag_task_waits(self.h, t)

    def info(self, t):
        return dag_task_get_info(self.h, t)

    def stats(self):
        return dag_get_stats(self.h)

    def set_launch(self, kernel, block, grid_cap=0, variant=0):
        kid = KERNEL_IDS[kernel] if isinstance(kernel, str) else kernel
        dag_kernel_set_launch(self.h, kid, dag_launch(block, grid_cap, variant, 0))

    def get_launch(self, kernel):
        kid = KERNEL_IDS[kernel] if isinstance(kernel, str) else kernel
        l = dag_kernel_get_launch(self.h, kid)
        return l.block, l.grid_cap, l.variant
