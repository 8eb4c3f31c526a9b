"""Serving on the MI355X: every request's result is the same alone (serial
mode) and in the concurrent mix, and equals the oracle for its shape; a small
budget forces admission queueing without changing any result."""

import sys

import numpy as np
import pytest

import gpu_util as G
from paper_2012_09646_amd import dagrt as D
from paper_2012_09646_amd import serving
from paper_2012_09646_amd import workloads as W

pytestmark = pytest.mark.gpu


def shapes():
    return [W.vec_program(n=(1 << 12) + 3, seed=21), W.img_program(side=96, height=80, seed=22),
            W.hits_program(n=2000, iters=10, seed=23), W.bs_program(n=5001, tasks=10, seed=24),
            W.vec_program(n=1 << 15, seed=25)]


def expected(prog, tmpl):
    ref = G.oracle_run(prog)
    return ref[tmpl.result][:tmpl.result_bytes]


@pytest.mark.parametrize("budget_mult,lanes,copy_lanes", [(100, 4, 1), (2, 8, 2), (100, 4, 0)])
def test_alone_vs_mix_and_oracle(budget_mult, lanes, copy_lanes):
    print("[gpu] serving budget x%d lanes %d copy lanes %d" % (budget_mult, lanes, copy_lanes), flush=True)
    ctx = D.Context()
    progs = shapes()
    tmpls = [serving.ShapeTemplate(ctx, p, key=100 + i) for i, p in enumerate(progs)]
    probe = serving.Server(ctx, 1 << 34, host_arena_bytes=1 << 28, lanes=1)
    for t in tmpls:
        probe.add(t)
    biggest = max(probe.footprint(i)[0] for i in range(len(tmpls)))
    probe.close()
    srv = serving.Server(ctx, budget_mult * biggest, device_arena_bytes=budget_mult * biggest + (1 << 20),
                         host_arena_bytes=1 << 28, lanes=lanes, copy_lanes=copy_lanes)
    for t in tmpls:
        srv.add(t)
    arr, shp = W.poisson_trace(31, 150, 20_000, len(tmpls))
    mix, st_mix, res_mix = srv.run(arr, shp, keep_results=True)
    alone, st_alone, res_alone = srv.run(arr, shp, mode=D.DAG_SERVE_SERIAL, keep_results=True)
    refs = [expected(p, t) for p, t in zip(progs, tmpls)]
    for i in range(len(arr)):
        assert np.array_equal(res_mix[i], res_alone[i]), "request %d differs alone vs mix" % i
        tm = tmpls[shp[i]]
        got = res_mix[i]
        G.assert_close(tm.prog, tm.result, got, refs[shp[i]])
    assert st_alone.max_inflight == 1
    if budget_mult == 2:
        assert st_mix.peak_device_bytes <= 2 * biggest
    print("[gpu] mix p50 %.3f p99 %.3f ms inflight %d queued %d; serial p50 %.3f" % (
        st_mix.p50_ms, st_mix.p99_ms, st_mix.max_inflight, st_mix.max_queued, st_alone.p50_ms), flush=True)
    srv.close()
    ctx.close()


def test_online_producer_results_equal_serial_and_oracle():
    """A producer thread submits the trace while the main thread polls
    (dag_serve_submit / dag_serve_poll): every result equals the serial
    session's bit for bit and the oracle's."""
    print("[gpu] serving online producer", flush=True)
    ctx = D.Context()
    progs = shapes()
    tmpls = [serving.ShapeTemplate(ctx, p, key=200 + i) for i, p in enumerate(progs)]
    srv = serving.Server(ctx, 1 << 32, host_arena_bytes=1 << 28, lanes=4, copy_lanes=1, transfer_lanes=1)
    for t in tmpls:
        srv.add(t)
    arr, shp = W.poisson_trace(33, 200, 20_000, len(tmpls))
    recs, st_on, res_on = srv.run_online(arr, shp, keep_results=True, pace=True)
    _, st_ser, res_ser = srv.run(arr, shp, mode=D.DAG_SERVE_SERIAL, keep_results=True)
    refs = [expected(p, t) for p, t in zip(progs, tmpls)]
    for i in range(len(arr)):
        assert np.array_equal(res_on[i], res_ser[i]), "request %d differs online vs serial" % i
        tm = tmpls[shp[i]]
        G.assert_close(tm.prog, tm.result, res_on[i], refs[shp[i]])
        a, adm, done, sh, lane = recs[i]
        assert sh == shp[i] and adm >= a and done >= adm
    assert st_on.completed == len(arr)
    print("[gpu] online p50 %.3f ms p99 %.3f ms in flight %d" % (st_on.p50_ms, st_on.p99_ms, st_on.max_inflight),
          flush=True)
    srv.close()
    ctx.close()


def test_shape_pins_buffers_and_released_buffer_kills_region():
    """On the GPU: a buffer a serving shape uses cannot be released while the
    server exists; after the server is gone it can, and the region recorded
    on it can no longer be launched."""
    print("[gpu] serving pins and released-buffer regions", flush=True)
    ctx = D.Context()
    t = serving.ShapeTemplate(ctx, W.vec_program(n=4096, seed=3), key=300)
    srv = serving.Server(ctx, 1 << 24, host_arena_bytes=1 << 20, lanes=2)
    srv.add(t)
    with pytest.raises(D.DagError) as e:
        ctx.release(t.bound.h["x"])
    assert e.value.name == "DAG_E_BUSY"
    srv.close()
    D.dag_region_launch(ctx.h, 300)
    ctx.sync()
    ctx.release(t.bound.h["x"])
    with pytest.raises(D.DagError) as e:
        D.dag_region_launch(ctx.h, 300)
    assert e.value.name == "DAG_E_INVAL"
    ctx.close()
