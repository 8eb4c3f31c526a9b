"""Run as a script (GPU_MAX_HW_QUEUES is read once when HIP starts, so the
benchmark's serving configuration needs a process of its own).

The benchmark's serving mix at full size: the 20 request shapes (vector
diamond, Black-Scholes fan-out, image pipeline and HITS at footprint scale
2^k, k = -4..0) on the benchmark's server (3 lanes, the first for requests
that copy between host and device, one copy stream per direction, SDMA
copies, 64 GB budget, tuned kernel launch configurations).  A seeded Poisson
trace at 2000 requests/s asks for every shape REPEATS times.  The trace runs
three ways: as one batch session (dag_serve_run), submitted online by a
producer thread pacing the arrivals while this thread polls, and serially
(one request at a time).  Every request's whole result must be bit-identical
in the three runs and equal to the oracle for its shape.

Usage: python tests/serving_mix_check.py [REPEATS]
Prints one line per step; exits 1 on any mismatch.
"""

import multiprocessing as mp
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

KINDS = ("vec", "bs", "img", "hits")
KS = (-4, -3, -2, -1, 0)


def oracle_shape(kind, k):
    """The oracle's result buffer for one shape, and the HITS graph it used."""
    import gpu_util as G
    from paper_2012_09646_amd import workloads as W
    graphs = {}
    prog = W.serve_program(kind, k, seed=4, graphs=graphs)
    ref = G.oracle_run(prog)
    return ref[prog.result], graphs


def log(*a):
    print("[serving-mix]", *a, flush=True)


def main():
    repeats = int(sys.argv[1]) if len(sys.argv) > 1 else 3
    t0 = time.time()
    # oracles in worker processes started before this process touches the GPU
    with ProcessPoolExecutor(max_workers=10, mp_context=mp.get_context("spawn")) as ex:
        futs = {(kind, k): ex.submit(oracle_shape, kind, k) for kind in KINDS for k in KS}
        refs, graphs = {}, {}
        for key, f in futs.items():
            refs[key], g = f.result()
            graphs.update(g)
    log("oracle of %d shapes in %.1f s" % (len(refs), time.time() - t0))

    import gpu_util as G
    from paper_2012_09646_amd import dagrt as D
    from paper_2012_09646_amd import serving
    from paper_2012_09646_amd import tune
    from paper_2012_09646_amd import workloads as W

    ctx = D.Context(copy_engine=0)
    path = os.path.join(os.path.dirname(HERE), "paper_2012_09646_amd", "tuning", "gfx950.json")
    tune.apply_kernels(ctx, tune.load(path).get("kernels", {}))
    tmpls = serving.mix_templates(ctx, graphs=graphs, result_bytes=None)
    srv = serving.mix_server(ctx, tmpls)
    log("%d shapes recorded, GPU_MAX_HW_QUEUES=%s" % (len(tmpls), os.environ.get("GPU_MAX_HW_QUEUES")))
    nshapes = len(tmpls)
    arr, _ = W.poisson_trace(44, repeats * nshapes, 2000.0, nshapes)
    shp = W.rng(45).permutation(np.repeat(np.arange(nshapes, dtype=np.int32), repeats))

    mix, st_mix, res_mix = srv.run(arr, shp, keep_results=True)
    log("batch session: p50 %.3f ms p99 %.3f ms, max in flight %d" % (st_mix.p50_ms, st_mix.p99_ms,
                                                                        st_mix.max_inflight))
    _, st_on, res_on = srv.run_online(arr, shp, keep_results=True, pace=True)
    log("online session (paced producer): p50 %.3f ms, max in flight %d" % (st_on.p50_ms, st_on.max_inflight))
    _, st_ser, res_ser = srv.run(arr, shp, mode=D.DAG_SERVE_SERIAL, keep_results=True)
    log("serial session: p50 %.3f ms" % st_ser.p50_ms)
    ok = st_ser.max_inflight == 1
    for i in range(len(arr)):
        t = tmpls[shp[i]]
        kind, k = KINDS[shp[i] // len(KS)], KS[shp[i] % len(KS)]
        if not (np.array_equal(res_mix[i], res_ser[i]) and np.array_equal(res_on[i], res_ser[i])):
            log("request %d (%s, k=%d): results differ between the sessions" % (i, kind, k))
            ok = False
            continue
        try:
            G.assert_close(t.prog, t.result, res_mix[i], refs[(kind, k)].view(np.uint8)[:t.result_bytes])
        except AssertionError as e:
            log("request %d (%s, k=%d): %s" % (i, kind, k, e))
            ok = False
    srv.close()
    ctx.close()
    log("%d requests over %d shapes: %s" % (len(arr), nshapes, "ok" if ok else "MISMATCH"))
    sys.exit(0 if ok else 1)


if __name__ == "__main__":
    main()
