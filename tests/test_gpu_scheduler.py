"""Scheduler behaviour on the MI355X: every edge is honoured in time
(timing events), randomly injected delays never change results, a
user-registered launcher takes part in the DAG, and releasing a buffer
waits for the tasks that use it."""

import ctypes as C
import random
import time

import numpy as np
import pytest

import gpu_util as G
from oracle import dag as odag
from paper_2012_09646_amd import dagrt as D
from paper_2012_09646_amd import runner
from paper_2012_09646_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("copy_streams", [0, 1])
def test_edges_are_honoured_in_time(copy_streams):
    print("[gpu] happens-before copy_streams=%d" % copy_streams, flush=True)
    for prog in (W.img_program(side=512, seed=41), W.hits_program(n=4000, iters=5, seed=42),
                 W.bs_program(n=1 << 18, tasks=6, seed=43)):
        ctx = D.Context(trace=1, copy_streams=copy_streams)
        b = runner.Bound(ctx, prog)
        D.dag_trace_reset(ctx.h)
        b.run()
        info = {p: ctx.info(b.base + p) for p in range(1, len(prog.ops) + 1)}
        checked = 0
        for s, d in {(s, d) for s, d, _, _ in b.edges()}:
            if info[s].stream >= 0 and info[d].stream >= 0:
                assert info[s].t_end_ms <= info[d].t_start_ms + 1e-6, (prog.name, s, d)
                checked += 1
        assert checked > 0
        ctx.close()


def test_gated_timing_in_the_serial_policy():
    """Trace mode 3 under the serial policy: tasks are timed one after the
    other (each starts after the previous one ends), every duration is
    positive and the outputs equal the oracle's."""
    print("[gpu] gated timing", flush=True)
    for prog in (W.img_program(side=300, height=200, seed=44), W.bs_program(n=1 << 16, tasks=3, seed=45)):
        ref = G.oracle_run(prog)
        ctx = D.Context(policy=D.DAG_SERIAL_SYNC, trace=3)
        b = runner.Bound(ctx, prog)
        D.dag_trace_reset(ctx.h)
        b.run()
        iv = []
        for p in range(1, len(prog.ops) + 1):
            inf = ctx.info(b.base + p)
            if inf.stream >= 0:
                assert inf.t_end_ms > inf.t_start_ms >= 0.0, (prog.name, p)
                iv.append((inf.t_start_ms, inf.t_end_ms))
        for (a0, a1), (b0, b1) in zip(iv, iv[1:]):
            assert a1 <= b0 + 1e-6
        for name in prog.outputs:
            G.assert_close(prog, name, b.read(name), ref[name])
        ctx.close()


@pytest.mark.parametrize("seed", range(4))
def test_delay_injection_keeps_results(seed):
    """Spin kernels of random length at random places (with random buffer
    arguments, so they also change the DAG) must not change any result."""
    print("[gpu] delay injection seed=%d" % seed, flush=True)
    rnd = random.Random(seed)
    base = [W.img_program(side=160, height=96, seed=50 + seed),
            W.hits_program(n=3000, iters=4, seed=60 + seed)][seed % 2]
    ref = G.oracle_run(base)
    names = list(base.bufs)
    ops = list(base.ops)
    for _ in range(6):
        pos = rnd.randrange(len(ops))
        args = [(rnd.choice(names), rnd.choice("cm")) for _ in range(rnd.randint(0, 2))]
        ops.insert(pos, W.K("spin", args, ns=rnd.randint(5_000, 300_000)))
    prog = W.Program(base.name, base.bufs, ops, base.outputs, base.result)
    g = odag.build_dag(prog.ops)
    for cs in (0, 1):
        ctx = D.Context(max_streams=rnd.choice([2, 4, 8]), copy_streams=cs)
        b = runner.Bound(ctx, prog)
        b.run()
        assert b.edges() == g.edges
        for name in prog.outputs:
            G.assert_close(base, name, b.read(name), ref[name])
        ctx.close()


def test_user_kernel_takes_part_in_the_dag():
    """A launcher registered from outside the library (here: a device memset
    through the HIP runtime) is scheduled like any other call."""
    print("[gpu] user kernel", flush=True)
    hip = C.CDLL("libamdhip64.so.7")
    hip.hipMemsetAsync.argtypes = [C.c_void_p, C.c_int, C.c_size_t, C.c_void_p]
    hip.hipMemsetAsync.restype = C.c_int

    @D.DAG_LAUNCH_FN
    def fill_ones(stream, ptrs, nptrs, params, user):
        nbytes = C.cast(params, C.POINTER(C.c_uint64))[0]
        return hip.hipMemsetAsync(ptrs[0], 0x3F, nbytes, stream)   # bytes 0x3F -> floats ~0.75

    ctx = D.Context()
    kid = D.dag_kernel_register(ctx.h, "fill", fill_ones)
    n = 1 << 16
    x, y, r = ctx.alloc(4 * n), ctx.alloc(4 * n), ctx.alloc(4)
    ctx.host_write(y, np.zeros(n, np.float32))
    nb = C.c_uint64(4 * n)
    t1 = D.dag_submit_kernel(ctx.h, kid, nb, [(x, D.DAG_MUTABLE)])
    t2 = ctx.kernel("vec_sum_diff", [(x, "c"), (y, "c"), (r, "m")], n=n)
    assert (t1, t2, D.DAG_EDGE_RAW) in {(s, d, k) for s, d, _, k in ctx.edges()}
    out = np.zeros(1, np.float32)
    ctx.host_read(r, out)
    v = np.frombuffer(bytes([0x3F] * 4), np.float32)[0]
    assert abs(out[0] - n * float(v)) <= 1e-5 * n * float(v)
    ctx.close()


def test_release_waits_for_active_users():
    print("[gpu] release while active", flush=True)
    ctx = D.Context()
    x = ctx.alloc(1024)
    ctx.kernel("spin", [(x, "m")], ns=20_000_000)
    t0 = time.perf_counter()
    ctx.release(x)
    assert time.perf_counter() - t0 > 0.015
    with pytest.raises(D.DagError):
        ctx.kernel("spin", [(x, "m")], ns=0)
    assert ctx.stats().active == 0
    ctx.close()
