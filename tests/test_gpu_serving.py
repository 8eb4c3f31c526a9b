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
