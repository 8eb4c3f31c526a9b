#!/usr/bin/env python3
"""Makespan of the benchmark DAGs on one MI355X: the runtime DAG scheduler
against synchronous serial execution of the same calls, and against the
contention-free critical-path bound (paper Sec. V-C and V-E).

Workloads (seeded synthetic inputs, sizes of the benchmark configurations):
  vec   vector diamond, 2^20 fp32, 3 tasks + host read of r, 5 repeats
  bs    Black-Scholes fan-out: 10 x (H2D 16 MiB -> price 2^22 -> D2H 16 MiB)
  img   image pipeline 2048x2048: 3 blur/Sobel/minmax/normalise branches + combine
  hits  HITS on a 2^20-vertex power-law graph (20 out-links each), 10 iterations,
        eager DAG and one-iteration graph replay
  serve open-loop Poisson arrivals (2000/s) of request DAGs drawn uniformly from
        the four workloads at footprint scale 2^k, k in -4..0, admitted by a 64 GB
        device-memory budget; p50/p99 latency and req/s, concurrent vs serial

The headline line is the Black-Scholes fan-out.  Prints ONE JSON line on
stdout; progress goes to stderr.
"""

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DAG makespan speedup vs serial + % critical-path bound; serving p50/p99 ms"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6   # vector fp64: 256 CUs x 128 flop/clk (4 SIMDs x 16 lanes x FMA) x 2.4 GHz
# fp64 work of one Black-Scholes price: the SQ_INSTS_VALU_{FMA,ADD,MUL,TRANS}_F64 counters of the leanest kernel
# variant (2: own exp and log, one polynomial per CDF) give 86 FMA + 5 ADD + 19 MUL + 3 TRANS per element
# (FMA = 2 flops); that count is taken as the method's work for every variant (variant 1 executes
# 83 + 44 + 23 + 3, variant 0, the library erfc, 127 + 61 + 22 + 7).  VALU wave-lane instructions per element
# (all kinds) per variant:
BS_FLOPS_PER_ELEMENT = 2 * 86 + 5 + 19 + 3
BS_VALU_PER_ELEMENT = {0: 285.75, 1: 206.25, 2: 146.125}  # 0, 1: measured before the zero-spot select (+2)
# HBM bytes per bs_call launch (variant 2, 128 threads, grid cap 4096) from FETCH_SIZE / WRITE_SIZE, each divided
# by what the counter reads for a 256 MiB copy kernel (FETCH_SIZE 0.500054x, WRITE_SIZE 1.000x of the true
# bytes): 16.14 MiB in + 16.00 MiB out (the kernel with the zero-spot select)
TRAFFIC_BS_BYTES = int((8262.20625 / 0.5000536 + 16384.0 / 1.0) * 1024)
CUS, CLOCK_GHZ = 256, 2.4
SERVE_HW_QUEUES = 8


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="all", choices=["all", "vec", "bs", "img", "hits", "ml", "dl", "serve"])
    ap.add_argument("--requests", type=int, default=10000, help="serving: requests in the trace")
    ap.add_argument("--serve-lanes", type=int, default=3,
                    help="serving: lanes (HIP streams) requests spread over")
    ap.add_argument("--serve-copy-engine", type=int, default=0, choices=[-1, 0, 1, 2, 3],
                    help="serving: copy engine (as --copy-engine; -1 = the same as the DAGs); SDMA measured "
                         "best for the mix in a process of its own")
    ap.add_argument("--serve-copy-lanes", type=int, default=1, choices=[0, 1, 2, 3, 4],
                    help="serving: N = host<->device copies of all requests on N streams per direction")
    ap.add_argument("--serve-transfer-lanes", type=int, default=1,
                    help="serving: N >= 1 = requests that copy between host and device use the first N lanes "
                         "only, all others the remaining lanes (0 = any lane); 3 lanes with 1 for transfers "
                         "sustained the 2000/s mix (p50 1.7 ms) where 2 shared lanes saturated at ~1890/s")
    ap.add_argument("--rate", type=float, default=2000.0, help="serving: Poisson arrival rate per second")
    ap.add_argument("--capacity-rate", type=float, default=4000.0,
                    help="serving: an overload rate (half the requests, concurrent mode only) whose throughput "
                         "is the loop's capacity (0 = skip)")
    ap.add_argument("--low-rate", type=float, default=600.0,
                    help="serving: a second, lower arrival rate (half the requests; 0 = skip)")
    ap.add_argument("--tuned", default=os.path.join(ROOT, "paper_2012_09646_amd", "tuning", "gfx950.json"),
                    help="kernel launch configurations from the autotuner (ignored if missing)")
    ap.add_argument("--max-streams", type=int, default=0,
                    help="stream pool bound (0 = per workload from the tuning file, else 8)")
    ap.add_argument("--hw-queues", type=int, default=0,
                    help="GPU_MAX_HW_QUEUES for this process (0 = from the tuning file, else the runtime's)")
    ap.add_argument("--copy-streams", type=int, default=0, choices=[0, 1],
                    help="0: one FIFO stream per copy direction; 1: copies placed like kernels")
    ap.add_argument("--copy-lanes", type=int, default=0,
                    help="streams per copy direction (0 = from the tuning file, else 1)")
    ap.add_argument("--copy-engine", type=int, default=2, choices=[0, 1, 2, 3],
                    help="host<->device copies: 0 = SDMA, 1 = CU copy kernel, 2 = H2D SDMA + D2H kernel "
                         "(default: with SDMA both ways, some processes ran the two directions on one engine "
                         "and the fan-out at serial speed), 3 = H2D kernel + D2H SDMA")
    ap.add_argument("--spin-wait", type=int, default=0, choices=[0, 1],
                    help="1: host waits spin (hipDeviceScheduleSpin)")
    ap.add_argument("--wait-mode", type=int, default=0, choices=[0, 1],
                    help="cross-stream waits: 0 = device-side signal polls, 1 = HIP events")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-oracle", default="", help=argparse.SUPPRESS)  # internal: CPU baseline of one workload
    return ap.parse_args()


# ---- CPU baseline: the oracle timed on the host's cores ----------------------------------------------
# The oracle executes a DAG strictly in program order.  On one thread it runs unchanged (oracle.run.execute,
# BLAS limited to one thread).  On all cores, each task whose outputs are independent per element, per image
# row, per matrix row or per output channel is cut into ranges that forked worker processes compute with the
# same oracle function (the program's buffers live in shared anonymous memory, so the workers write the
# results in place); the reductions that return one correctly rounded sum (math.fsum), the dense layer and the
# final combination run whole in the parent.  The arithmetic per output is the oracle's; the outputs must equal
# the one-thread run's bit for bit (checked and reported).
CPU_POOL_CAP = 16  # worker processes at most (the host share of one GPU)
_CPU = {}          # the program being run: set before the pool forks, inherited by the workers

PER_ELEMENT = ("vec_square", "bs_call", "unsharp_combine", "minmax")
PER_ELEMENT_SCALAR2 = ("normalise", "scale_l2")  # argument 1 is a small whole buffer


def _cpu_units(op, bufs):
    k, p = op["kernel"], op.get("params", {})
    if k in PER_ELEMENT or k in PER_ELEMENT_SCALAR2:
        return int(p["n"])
    if k in ("gauss_blur", "sobel"):
        return int(p["h"])
    if k in ("spmv", "spmv_rows"):
        return int(p["nrows"])
    if k in ("nb_proba", "ridge_proba", "ensemble"):
        return int(p["n"])
    if k == "conv3x3_relu_pool":
        return int(p["cout"])
    return 0


def _cpu_ranges(op, bufs, units, pieces):
    """Unit ranges of about equal work (SpMV: rows + nonzeros, as a merge path)."""
    import numpy as np
    if op["kernel"] in ("spmv", "spmv_rows"):
        rp = bufs[op["args"][0][0]].view(np.int32)[:units + 1].astype(np.int64)
        path = rp + np.arange(units + 1)
        cuts = np.searchsorted(path, np.linspace(0, path[-1], pieces + 1)[1:-1])
    else:
        cuts = np.linspace(0, units, pieces + 1)[1:-1].round().astype(np.int64)
    edges = [0] + sorted(set(int(c) for c in cuts if 0 < c < units)) + [units]
    return list(zip(edges[:-1], edges[1:]))


def _cpu_worker_init():
    from threadpoolctl import threadpool_limits
    _CPU["limits"] = threadpool_limits(1)


def _cpu_chunk(task):
    """Worker: one range of one task through the oracle's own function."""
    import numpy as np
    from oracle import run as orun
    i, lo, hi = task
    op = _CPU["ops"][i]
    bufs = _CPU["bufs"]
    k, p = op["kernel"], dict(op.get("params", {}))
    a = [bufs[name] for name, _ in op["args"]]
    fn = orun.KERNELS[k]

    def f4(x, l, h):
        return x[4 * l:4 * h]
    if k == "minmax":
        p["n"] = hi - lo
        m = np.zeros(8, np.uint8)
        fn(p, f4(a[0], lo, hi), m)
        return m.view(np.float32).copy()
    if k in PER_ELEMENT:
        p["n"] = hi - lo
        fn(p, *[f4(x, lo, hi) for x in a])
    elif k in PER_ELEMENT_SCALAR2:
        p["n"] = hi - lo
        fn(p, f4(a[0], lo, hi), a[1], f4(a[2], lo, hi))
    elif k in ("gauss_blur", "sobel"):
        # rows lo..hi from the input rows they read (the stencil's halo; the image border stays the border)
        w, h = p["w"], p["h"]
        rad = (p["ksize"] - 1) // 2 if k == "gauss_blur" else 1
        r0, r1 = max(lo - rad, 0), min(hi + rad, h)
        p["h"] = r1 - r0
        tmp = np.zeros(4 * w * (r1 - r0), np.uint8)
        fn(p, a[0][4 * w * r0:4 * w * r1], tmp)
        a[1][4 * w * lo:4 * w * hi] = tmp[4 * w * (lo - r0):4 * w * (hi - r0)]
    elif k in ("spmv", "spmv_rows"):
        rp = a[0].view(np.int32)
        s0, s1 = int(rp[lo]), int(rp[hi])
        sub = (rp[lo:hi + 1] - s0).astype(np.int32)
        p.update(nrows=hi - lo, nnz=s1 - s0)
        fn(p, sub.view(np.uint8), f4(a[1], s0, s1), f4(a[2], s0, s1), a[3], f4(a[4], lo, hi))
    elif k in ("nb_proba", "ridge_proba"):
        n, F, C = p["n"], p["features"], p["classes"]
        X = np.ascontiguousarray(a[0].view(np.float32)[:n * F].reshape(F, n)[:, lo:hi])
        p["n"] = hi - lo
        fn(p, X.view(np.uint8).ravel(), *a[1:-1], a[-1][4 * C * lo:4 * C * hi])
    elif k == "ensemble":
        C = p["classes"]
        p["n"] = hi - lo
        fn(p, *[x[4 * C * lo:4 * C * hi] for x in a[:3]], f4(a[3], lo, hi))
    elif k == "conv3x3_relu_pool":
        cin, plane = p["cin"], (p["h"] // 2) * (p["w"] // 2)
        p["cout"] = hi - lo
        fn(p, a[0], a[1][36 * cin * lo:36 * cin * hi], f4(a[2], lo, hi), a[3][4 * plane * lo:4 * plane * hi])
    return None


def _cpu_execute(prog, bufs, pool, pieces):
    """Program order, each splittable task spread over the pool."""
    import numpy as np
    from oracle import run as orun
    for i, op in enumerate(prog.ops):
        kind = op["kind"]
        if kind == "kernel":
            units = _cpu_units(op, bufs)
            if pool is not None and units >= 2:
                ranges = _cpu_ranges(op, bufs, units, pieces)
                res = pool.map(_cpu_chunk, [(i, lo, hi) for lo, hi in ranges], chunksize=1)
                if op["kernel"] == "minmax":
                    m = bufs[op["args"][1][0]].view(np.float32)
                    m[0] = max(r[0] for r in res)
                    m[1] = min(r[1] for r in res)
            else:
                orun.KERNELS[op["kernel"]](op.get("params", {}), *[bufs[b] for b, _ in op["args"]])
        elif kind == "copy":
            nb, so, do = op["bytes"], op.get("src_off", 0), op.get("dst_off", 0)
            bufs[op["dst"]][do:do + nb] = bufs[op["src"]][so:so + nb]
        elif kind == "host_read":
            bufs[op["buf"]].copy()
        elif kind != "sync":
            raise ValueError(kind)


def cpu_workload_program(wl, quarter=False):
    """The workload's program; quarter=True: the same DAG on a quarter of the elements (pixels, vertices,
    rows), the one-thread sample of the heavy workloads."""
    from paper_2012_09646_amd import workloads as W
    q = 2 if quarter else 0
    return {"vec": lambda: W.vec_program(n=1 << (20 - q), seed=0),
            "bs": lambda: W.bs_program(n=1 << (22 - q), tasks=10, seed=1),
            "img": lambda: W.img_program(side=2048 >> (q // 2), seed=2),
            "hits": lambda: W.hits_program(n=1 << (20 - q), deg=20, iters=10, seed=3),
            "ml": lambda: W.ml_program(n=1 << (20 - q), seed=5),
            "dl": lambda: W.dl_program(side=1024 >> (q // 2), seed=6)}[wl]()


# one-thread runs of these take 7-40 s each at full size: timed on a quarter of the elements, times 4
CPU_ONE_THREAD_QUARTER = ("img", "hits", "ml", "dl")


def cpu_baseline(wl, budget_s=4.0):
    """The oracle on one thread and on all cores for one workload's DAG: ms per full DAG run (median of the
    runs that fit in budget_s per mode, at least one).  The all-cores result must equal the one-thread one
    bit for bit on the program the one-thread run executed."""
    import mmap
    import multiprocessing as mp
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import run as orun
    from paper_2012_09646_amd import workloads as W
    prog = cpu_workload_program(wl)
    quarter = wl in CPU_ONE_THREAD_QUARTER
    one = cpu_workload_program(wl, quarter=True) if quarter else prog
    init = W.initial_arrays(prog)
    init_one = W.initial_arrays(one) if quarter else init

    def timed(prepare, run):
        """Median ms of run(prepare()) over the runs that fit in budget_s (prepare is not timed)."""
        times, t_start = [], time.perf_counter()
        while not times or (time.perf_counter() - t_start < budget_s and len(times) < 5):
            state = prepare()
            t0 = time.perf_counter()
            run(state)
            times.append((time.perf_counter() - t0) * 1e3)
        return statistics.median(times), len(times), state

    def one_thread(arrays):
        with threadpool_limits(1):
            orun.execute(one.ops, arrays)
    t1, n1, serial = timed(lambda: {k: v.copy() for k, v in init_one.items()}, one_thread)
    cores = min(len(os.sched_getaffinity(0)), CPU_POOL_CAP)

    def all_cores(p, ini, timed_runs):
        bufs = {}
        for name, arr in ini.items():
            mm = mmap.mmap(-1, max(arr.nbytes, 1))
            bufs[name] = np.frombuffer(mm, dtype=np.uint8, count=arr.nbytes)
        _CPU.update(ops=p.ops, bufs=bufs)

        def reset():
            for name, arr in ini.items():
                bufs[name][:] = arr
            return bufs
        with mp.get_context("fork").Pool(cores, initializer=_cpu_worker_init) as pool:
            if timed_runs:
                res = timed(reset, lambda b: _cpu_execute(p, b, pool, 4 * cores))
            else:
                _cpu_execute(p, reset(), pool, 4 * cores)
                res = (None, 0, bufs)
        _CPU.clear()
        return res
    tp, n_p, par = all_cores(prog, init, True)
    if quarter:
        par = all_cores(one, init_one, False)[2]
    same = all(np.array_equal(par[o], serial[o]) for o in one.outputs)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"all_cores_ms": round(tp, 2), "one_thread_ms": round(t1 * (4 if quarter else 1), 2),
            "cores": cores, "affinity_cores": len(os.sched_getaffinity(0)), "cpu_model": model,
            "runs": [n_p, n1], "one_thread_sample": "a quarter of the elements, x4" if quarter else "full DAG",
            "matches_one_thread": bool(same)}


def orchestrate(args):
    """--workload all: every workload measured in a fresh child process, one
    after the other (this process never touches the GPU).  A process's copy
    engines and hardware queues are bound when it first uses them, and a
    measurement was seen to depend on what ran earlier in the same process;
    fresh processes make each figure independent of the others."""
    import subprocess
    fwd = ["--steps", str(args.steps), "--warmup", str(args.warmup), "--tuned", args.tuned,
           "--max-streams", str(args.max_streams), "--copy-streams", str(args.copy_streams),
           "--copy-lanes", str(args.copy_lanes), "--copy-engine", str(args.copy_engine),
           "--spin-wait", str(args.spin_wait), "--wait-mode", str(args.wait_mode), "--requests", str(args.requests),
           "--rate", str(args.rate),
           "--low-rate", str(args.low_rate), "--capacity-rate", str(args.capacity_rate),
           "--serve-lanes", str(args.serve_lanes),
           "--serve-copy-lanes", str(args.serve_copy_lanes), "--serve-copy-engine", str(args.serve_copy_engine),
           "--serve-transfer-lanes", str(args.serve_transfer_lanes)]
    if args.hw_queues:
        fwd += ["--hw-queues", str(args.hw_queues)]
    lines = {}
    for wl in ("bs", "vec", "img", "hits", "ml", "dl", "serve"):
        log("child process: --workload %s" % wl)
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--workload", wl, "--no-cpu-baseline"] + fwd,
                           stdout=subprocess.PIPE, text=True)
        if r.returncode != 0:
            log("workload %s failed with status %d" % (wl, r.returncode))
            sys.exit(r.returncode)
        lines[wl] = json.loads(r.stdout.strip().splitlines()[-1])
    line = lines["bs"]
    for wl in ("vec", "img", "hits", "ml", "dl"):
        line["workloads"][wl] = lines[wl]["workloads"][wl]
    line["serving"] = lines["serve"]["serving"]
    line["config"]["processes"] = "one per workload"
    if not args.no_cpu_baseline:
        # this process never touched the GPU, so it may fork the oracle's workers
        for wl in ("bs", "vec", "img", "hits", "ml", "dl"):
            log("cpu baseline: %s (oracle, one thread and all cores)" % wl)
            line["workloads"][wl]["cpu_oracle"] = cpu_baseline(wl)
        add_cpu_line(line)
    print(json.dumps(line), flush=True)


def add_cpu_line(line):
    """The headline's cpu_baseline entry: the Black-Scholes DAG on the oracle."""
    c = line["workloads"]["bs"]["cpu_oracle"]
    line["cpu_baseline"] = {
        "value": c["all_cores_ms"], "unit": "ms per DAG run", "cores": c["cores"], "kind": "oracle",
        "sample": "full runs of the 10-task Black-Scholes DAG (10 x 2^22 options), median of %d; each pricing "
                  "task cut into element ranges over %d worker processes, copies in the parent; outputs equal "
                  "the one-thread run's: %s" % (c["runs"][0], c["cores"], c["matches_one_thread"]),
        "value_one_thread": c["one_thread_ms"], "cpu_model": c["cpu_model"],
        "affinity_cores": c["affinity_cores"]}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the scheduler space-shares a single device; "
              "runs on more than one GPU are not supported (got --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if not args.hw_queues and args.tuned and os.path.exists(args.tuned) and args.workload != "all":
        # the workload's tuned hardware queue count (the serving loop: 8, which
        # its 3 lanes and 2 copy streams fit); HIP reads it once at start-up, so
        # it is set before anything touches the GPU
        if args.workload == "serve":
            args.hw_queues = SERVE_HW_QUEUES
        else:
            with open(args.tuned) as f:
                args.hw_queues = int(json.load(f).get("dag", {}).get(args.workload, {}).get("hw_queues", 0))
    if args.hw_queues:
        os.environ["GPU_MAX_HW_QUEUES"] = str(args.hw_queues)
    if args.cpu_oracle:
        print(json.dumps(cpu_baseline(args.cpu_oracle)), flush=True)
        return
    if args.workload == "all":
        orchestrate(args)
        return
    import numpy as np  # noqa: F401

    from paper_2012_09646_amd import dagrt as D
    from paper_2012_09646_amd import handwritten
    from paper_2012_09646_amd import metrics as M
    from paper_2012_09646_amd import runner
    from paper_2012_09646_amd import serving
    from paper_2012_09646_amd import tune
    from paper_2012_09646_amd import workloads as W

    tuned = {}
    tuned_dag = {}
    if args.tuned and os.path.exists(args.tuned):
        tdata = tune.load(args.tuned)
        tuned = tdata.get("kernels", {})
        tuned_dag = tdata.get("dag", {})
        log("kernel launch configurations from", args.tuned)
    if not args.copy_lanes:
        args.copy_lanes = int(tuned_dag.get("bs", {}).get("copy_lanes", 1))
    fixed_pool = args.max_streams

    def pool_for(name):
        return fixed_pool or int(tuned_dag.get(name, {}).get("max_streams", 8))

    def kernel_intervals(ctx, b, nops):
        iv = []
        for pos in range(1, nops + 1):
            inf = ctx.info(b.base + pos)
            if inf.stream < 0 or inf.t_start_ms < 0:
                continue
            kind = "C" if inf.kind in (D.DAG_TASK_KERNEL, D.DAG_TASK_REGION) else "T"
            iv.append((pos, kind, inf.t_start_ms, inf.t_end_ms))
        return iv

    def measure(name, prog, steps, warmup, restore=(), per_iter=None):
        """Timed parallel runs, serial runs, traced runs; returns a summary."""
        res = {"workload": name, "tasks": sum(1 for o in prog.ops if o["kind"] != "host_read")}
        pris = {}
        args.max_streams = pool_for(name)
        res["max_streams"] = args.max_streams
        res["kernel_overrides"] = tuned_dag.get(name, {}).get("kernels", {})
        res["hw_queues"] = int(os.environ.get("GPU_MAX_HW_QUEUES", "0") or 0)

        def make(policy, trace):
            ctx = D.Context(policy=policy, max_streams=args.max_streams, trace=trace,
                            copy_streams=args.copy_streams, spin_wait=args.spin_wait,
                            copy_lanes=args.copy_lanes, copy_engine=args.copy_engine, wait_mode=args.wait_mode)
            tune.apply_kernels(ctx, tuned)
            # near-tie kernel configurations the tuner chose for this DAG's makespan
            for k, cfg in tuned_dag.get(name, {}).get("kernels", {}).items():
                tune.set_launch(ctx, k, cfg)
            b = runner.Bound(ctx, prog, read_bytes=4)
            for dst in restore:
                if dst not in pris:
                    pris[dst] = prog.bufs[dst].init
                h0 = ctx.alloc(prog.bufs[dst].nbytes)
                ctx.host_write(h0, pris[dst])
                b.h[dst + "@0"] = h0
            ctx.sync()
            return ctx, b

        def reset(ctx, b):
            if restore:
                for dst in restore:
                    ctx.copy(b.h[dst], b.h[dst + "@0"], prog.bufs[dst].nbytes)
                ctx.sync()

        def timed(ctx, b, n, warm):
            ts = []
            for i in range(warm + n):
                reset(ctx, b)
                if i == warm:
                    timed.stats0 = ctx.stats()  # host times of the timed runs only (no first-launch code loads)
                t0 = time.perf_counter()
                b.run()
                t1 = time.perf_counter()
                if i >= warm:
                    ts.append((t1 - t0) * 1e3)
            return ts

        ctxP, bP = make(D.DAG_PARALLEL_ASYNC, False)
        log(name, "parallel")
        par = timed(ctxP, bP, steps, warmup)
        st, st0 = ctxP.stats(), timed.stats0
        res["makespan_ms"] = statistics.median(par)
        res["makespan_min_ms"] = min(par)
        ntimed = max(st.tasks - st0.tasks, 1)
        res["host_us_per_task"] = (st.submit_host_us - st0.submit_host_us) / ntimed
        res["launch_us_per_task"] = (st.launch_host_us - st0.launch_host_us) / ntimed
        res["streams"] = st.streams
        edges = sorted({(s, d) for s, d, _, _ in bP.edges()})
        res["edges"] = len(edges)
        res["event_waits_per_run"] = sum(len(w) for w in bP.waits().values())
        eager_out = {o: bP.read(o) for o in prog.outputs}  # outputs of the last timed run
        ctxP.close()

        # the same runs with timing events around every kernel (not copies):
        # in-DAG kernel durations for the roofline, measured on the kernels' streams
        ctxK, bK = make(D.DAG_PARALLEL_ASYNC, 2)
        log(name, "parallel, kernel timing events")
        ktimes = {}
        park = []
        for i in range(warmup + steps):
            reset(ctxK, bK)
            t0 = time.perf_counter()
            bK.run()
            t1 = time.perf_counter()
            if i < warmup:
                continue
            park.append((t1 - t0) * 1e3)
            for pos, kind, a, bb in kernel_intervals(ctxK, bK, len(prog.ops)):
                o = prog.ops[pos - 1]
                if o["kind"] == "kernel":
                    ktimes.setdefault(o["kernel"], []).append((bb - a, M.algorithmic_bytes(o["kernel"], o["params"])))
        res["makespan_kernel_events_ms"] = statistics.median(park)
        res["kernels_in_dag"] = {k: {"launches": len(v), "avg_us": 1e3 * sum(t for t, _ in v) / len(v),
                                     "gbs": sum(by for _, by in v) / sum(t for t, _ in v) / 1e6}
                                 for k, v in ktimes.items()}
        ctxK.close()

        ctxS, bS = make(D.DAG_SERIAL_SYNC, False)
        log(name, "serial")
        ser = timed(ctxS, bS, steps, warmup)
        res["serial_ms"] = statistics.median(ser)
        res["speedup"] = res["serial_ms"] / res["makespan_ms"]
        ctxS.close()

        # isolated task times: the serial policy (each task alone on the GPU)
        # with gated timing events (trace mode 3: the start marker and the
        # work are queued together, so the host's launch latency is not
        # counted).  Markers still add a few microseconds around a kernel, so
        # kernels are weighted by their back-to-back time instead (every
        # distinct call launched back to back alone, median of three batches
        # of 20, per launch): never above the time alone, which keeps the
        # critical path a lower bound.  Copies keep the gated marker times.
        ctxI, bI = make(D.DAG_SERIAL_SYNC, 3)
        log(name, "isolated")
        iso = {}
        for i in range(max(3, min(steps, 10))):
            reset(ctxI, bI)
            D.dag_trace_reset(ctxI.h)
            bI.run()
            for pos, kind, a, bb in kernel_intervals(ctxI, bI, len(prog.ops)):
                iso.setdefault(pos, []).append(bb - a)
        b2b = {}
        b2b_kernel = {}
        for pos in range(1, len(prog.ops) + 1):
            o = prog.ops[pos - 1]
            if o["kind"] != "kernel":
                continue
            key = (o["kernel"], tuple(sorted(o["params"].items())), tuple(o["args"]))
            if key not in b2b:
                prm = D.make_params(o["kernel"], o["params"])
                a = [(bI.h[n], D.DAG_MUTABLE if m == "m" else D.DAG_CONST) for n, m in o["args"]]
                _, us = D.dag_tune_kernel(ctxI.h, D.KERNEL_IDS[o["kernel"]], prm, a,
                                          [ctxI.get_launch(o["kernel"])], 20)
                b2b[key] = us[0]
                b2b_kernel.setdefault(o["kernel"], []).append(us[0])
        ctxI.close()
        res["kernels_back_to_back_us"] = {k: statistics.median(v) for k, v in b2b_kernel.items()}
        gated = {}
        for pos in range(1, len(prog.ops) + 1):
            o = prog.ops[pos - 1]
            if o["kind"] == "kernel":
                gated.setdefault(o["kernel"], []).extend(iso.get(pos, []))
                key = (o["kernel"], tuple(sorted(o["params"].items())), tuple(o["args"]))
                iso[pos] = [b2b[key] / 1e3]
        res["kernels_isolated_gated_us"] = {k: 1e3 * statistics.median(v) for k, v in gated.items() if v}
        w = {p: statistics.median(v) for p, v in iso.items()}
        cp, path = M.critical_path(len(prog.ops), edges, w)
        res["cp_bound_ms"] = cp
        res["cp_path"] = [prog.ops[p - 1].get("kernel", prog.ops[p - 1]["kind"]) for p in path]
        res["cp_frac"] = cp / res["makespan_ms"]
        h2d = sum(w[p] for p in w if prog.ops[p - 1]["kind"] == "copy" and prog.bufs[prog.ops[p - 1]["src"]].loc == "host")
        d2h = sum(w[p] for p in w if prog.ops[p - 1]["kind"] == "copy" and prog.bufs[prog.ops[p - 1]["dst"]].loc == "host")
        hbm = sum(M.algorithmic_bytes(o["kernel"], o["params"]) for o in prog.ops if o["kind"] == "kernel")
        res["resource_bound_ms"] = max(cp, h2d, d2h, hbm / HBM_PEAK_GBS / 1e6)
        res["resource_frac"] = res["resource_bound_ms"] / res["makespan_ms"]
        # context, not a bound: all tasks' isolated times added up (what one
        # stream would take with no launch gaps)
        res["sum_isolated_ms"] = sum(w.values())
        res["sum_isolated_frac"] = res["sum_isolated_ms"] / res["makespan_ms"]
        # per-kernel isolated bandwidth
        per = {}
        for p, t in w.items():
            o = prog.ops[p - 1]
            if o["kind"] != "kernel":
                continue
            k = o["kernel"]
            by = M.algorithmic_bytes(k, o["params"])
            e = per.setdefault(k, {"launches": 0, "ms": 0.0, "bytes": 0})
            e["launches"] += 1
            e["ms"] += t
            e["bytes"] += by
        res["kernels_isolated"] = {k: {"avg_us": 1e3 * e["ms"] / e["launches"],
                                       "gbs": e["bytes"] / e["ms"] / 1e6} for k, e in per.items()}

        # fully traced parallel runs (copies too): overlap figures
        ctxT, bT = make(D.DAG_PARALLEL_ASYNC, 1)
        log(name, "traced parallel")
        tr = []
        gap_us = {}
        for i in range(max(3, min(steps, 10))):
            reset(ctxT, bT)
            D.dag_trace_reset(ctxT.h)
            t0 = time.perf_counter()
            bT.run()
            tr.append((time.perf_counter() - t0) * 1e3)
            ivs = kernel_intervals(ctxT, bT, len(prog.ops))
            gaps = M.dependency_gaps({(s, d) for s, d, _, _ in bT.edges()}, bT.streams(),
                                     {pos: (a, bb) for pos, _, a, bb in ivs})
            for kind in ("same", "cross"):
                gap_us.setdefault(kind, []).extend(1e3 * g for g in gaps[kind])
        res["overlap"] = M.overlap([(k, a, bb) for _, k, a, bb in ivs])
        res["traced_makespan_ms"] = statistics.median(tr)
        # device idle time per dependency edge (last parent's end to the task's start), over the traced runs
        res["dependency_gap_us"] = {kind: {"edges": len(v), "median": statistics.median(v) if v else None,
                                           "mean": statistics.fmean(v) if v else None,
                                           "total_per_run": sum(v) / len(tr)}
                                    for kind, v in ((k, gap_us.get(k, [])) for k in ("same", "cross"))}
        ctxT.close()

        # graph form: the DAG (or one HITS iteration) recorded once and replayed
        # as one task per launch; no dependency work or per-task HIP calls
        forms = [(0, "graph", args.copy_engine), (1, "replay", args.copy_engine)]
        if any(o["kind"] == "copy" for o in prog.ops):
            # the graph with its host<->device copies as copy kernels on the CUs
            # (kernel nodes) instead of memcpy nodes
            forms.append((0, "graph_kernel_copies", 1))
        # the program as written, each iteration (or the whole DAG) bracketed by
        # dag_region_run_begin/end: recorded once, then replayed when every call
        # matches (graph mode 2: a hipGraph unless the region copies to or from the host)
        forms.append((2, "recurring", args.copy_engine))
        # hand-written schedules (streams and waits chosen by hand, checked
        # against the inferred edges): multi-stream replay and hipGraph, the
        # paper's hand-optimized baselines
        forms += [(1, "hand", args.copy_engine), (0, "hand_graph", args.copy_engine)]
        for gm, tag, engine in forms:
            ctxG = D.Context(policy=D.DAG_PARALLEL_ASYNC, max_streams=args.max_streams, graph_mode=gm,
                             copy_streams=args.copy_streams, spin_wait=args.spin_wait,
                             copy_lanes=args.copy_lanes, copy_engine=engine, wait_mode=args.wait_mode)
            tune.apply_kernels(ctxG, tuned)
            bG = runner.Bound(ctxG, prog, read_bytes=4)
            for dst in restore:
                h0 = ctxG.alloc(prog.bufs[dst].nbytes)
                ctxG.host_write(h0, pris[dst])
                bG.h[dst + "@0"] = h0
            reset(ctxG, bG)
            nsub = sum(1 for o in prog.ops if o["kind"] in ("kernel", "copy"))
            if tag == "recurring":
                go = lambda: bG.run_recurring(1, per_iter or nsub)
                go()  # records
            elif per_iter:
                bG.record(1, 0, per_iter)
                times = len(prog.ops) // per_iter
                go = lambda: bG.replay(1, times)
            else:
                bG.record(1)
                go = lambda: bG.replay(1, 1)
            if tag.startswith("hand"):
                handwritten.install(ctxG, 1, prog)
            ctxG.sync()
            log(name, tag)
            gt = []
            for i in range(warmup + steps):
                reset(ctxG, bG)
                t0 = time.perf_counter()
                go()
                t1 = time.perf_counter()
                if i >= warmup:
                    gt.append((t1 - t0) * 1e3)
            res[tag + "_ms"] = statistics.median(gt)
            res[tag + "_speedup"] = res["serial_ms"] / res[tag + "_ms"]
            res[tag + "_cp_frac"] = res["cp_bound_ms"] / res[tag + "_ms"]
            # one more replay into cleared outputs must reproduce the eager outputs bit for bit
            for o in prog.outputs:
                ctxG.host_write(bG.h[o], np.zeros(prog.bufs[o].nbytes, np.uint8))
            reset(ctxG, bG)
            go()
            got = {o: bG.read(o) for o in prog.outputs}
            res[tag + "_matches_eager"] = all(np.array_equal(got[o], eager_out[o]) for o in prog.outputs)
            if not res[tag + "_matches_eager"]:
                # which outputs differ (bytes differing, of them zero) and whether they still
                # differ after a full device synchronisation
                res[tag + "_mismatch"] = {o: [int(np.sum(got[o] != eager_out[o])),
                                              int(np.sum((got[o] != eager_out[o]) & (got[o] == 0)))]
                                          for o in prog.outputs if not np.array_equal(got[o], eager_out[o])}
                ctxG.sync()
                res[tag + "_matches_after_sync"] = all(np.array_equal(bG.read(o), eager_out[o])
                                                       for o in prog.outputs)
            ctxG.close()
        return res, ktimes

    def edge_cost(calls=64, gate_ns=2_000_000, reps=15):
        """Device cost of a dependency edge on this GPU.  A 2 ms delay kernel,
        then a chain of `calls` tiny kernels that each square the same 4 KiB
        vector (every call depends on the one before), recorded as a region
        and replayed (recorded multi-stream replay) with two hand-written
        schedules: all calls on one stream (edges through stream order), or
        consecutive calls alternating between two streams, each waiting on
        its predecessor's event.  The host enqueues the whole chain while the
        delay runs, so a replay's time minus the delay is the device's time
        for the chain; per call = that / calls."""
        n = 1024
        ones = np.ones(n, np.float32)
        ops = [W.K("spin", [("x", "m")], ns=gate_ns)] + [W.K("vec_square", [("x", "m")], n=n)] * calls
        prog = W.Program("chain", {"x": W.Buf(4 * n, init=ones)}, ops, ["x"])
        ctx = D.Context(graph_mode=1, max_streams=2)
        tune.apply_kernels(ctx, tuned)
        b = runner.Bound(ctx, prog, read_bytes=4)
        b.record(1)
        ctx.sync()
        out = {}
        scheds = {"same_stream": [(0, [])] * (calls + 1),
                  "cross_stream": [(0, [])] + [(k % 2, [k - 1]) for k in range(1, calls + 1)]}
        for name, sched in scheds.items():
            D.dag_region_set_schedule(ctx.h, 1, sched)
            ts = []
            for _ in range(reps + 2):
                t0 = time.perf_counter()
                D.dag_region_launch(ctx.h, 1)
                ctx.sync()
                ts.append((time.perf_counter() - t0) * 1e6)
            out[name] = statistics.median(ts[2:])
        # the delay alone (same context, one call)
        ctx2 = D.Context(max_streams=1)
        h = ctx2.alloc(4 * n)
        ts = []
        for _ in range(reps + 2):
            t0 = time.perf_counter()
            ctx2.kernel("spin", [(h, "m")], ns=gate_ns)
            ctx2.sync()
            ts.append((time.perf_counter() - t0) * 1e6)
        gate = statistics.median(ts[2:])
        ctx2.close()
        ctx.close()
        same = (out["same_stream"] - gate) / calls
        cross = (out["cross_stream"] - gate) / calls
        res = {"calls": calls, "same_stream_us_per_call": round(same, 3),
               "cross_stream_us_per_call": round(cross, 3), "cross_edge_extra_us": round(cross - same, 3),
               "method": "2 ms delay kernel, then a %d-call dependent chain of 4 KiB squares replayed from a "
                         "recorded region (event waits); (replay time - delay alone) / calls, median of %d"
                         % (calls, reps)}
        # The scheduler's own placement: after the delay, tiny kernels (zero
        # delays) over four rotating buffers; calls 0 and 1 each write one,
        # and from then on call k reads the outputs of calls k-1 and k-2 and
        # overwrites that of k-4.  Its parents are
        # k-3, k-2 and k-1; it joins the stream of k-2 (the oldest parent
        # that is still the last call on its stream) and waits for k-1 on the
        # other: every call is a cross-stream edge with max_streams=2, and
        # with max_streams=1 the same calls run in stream order.
        xs = {"o%d" % i: W.Buf(4 * n, init=ones) for i in range(4)}
        eops = [W.K("spin", [("o%d" % i, "m") for i in range(4)], ns=gate_ns),
                W.K("spin", [("o0", "m")], ns=0), W.K("spin", [("o1", "m")], ns=0)]
        for k in range(2, calls):
            eops.append(W.K("spin", [("o%d" % ((k - 1) % 4), "c"), ("o%d" % ((k - 2) % 4), "c"),
                                     ("o%d" % (k % 4), "m")], ns=0))
        eprog = W.Program("alternating", xs, eops, list(xs))
        for mode, label in ((D.DAG_WAIT_SIGNALS, "signals"), (D.DAG_WAIT_EVENTS, "events")):
            per = {}
            for ms in (1, 2):
                cx = D.Context(max_streams=ms, wait_mode=mode)
                tune.apply_kernels(cx, tuned)
                be = runner.Bound(cx, eprog, read_bytes=4)
                ts = []
                for _ in range(reps + 2):
                    t0 = time.perf_counter()
                    be.run()
                    cx.sync()
                    ts.append((time.perf_counter() - t0) * 1e6)
                st = cx.stats()
                cx.close()
                per[ms] = (statistics.median(ts[2:]) - gate) / calls
                if ms == 2:
                    assert st.streams == 2 and st.waits >= calls - 1, (st.streams, st.waits)
            res["eager_%s" % label] = {"same_stream_us_per_call": round(per[1], 3),
                                       "cross_stream_us_per_call": round(per[2], 3),
                                       "cross_edge_extra_us": round(per[2] - per[1], 3)}
        res["eager_method"] = ("2 ms delay kernel, then %d zero-delay kernels submitted as one batch that "
                               "alternate between two streams, each waiting for the previous one "
                               "(max_streams=2), against the same calls on one stream (max_streams=1); "
                               "(run time - delay alone) / calls, median of %d, per wait mode" % (calls, reps))
        return res

    def measure_serving(graphs):
        """Open-loop serving of the mixed trace, concurrent and serial."""
        ctx = D.Context(spin_wait=args.spin_wait,
                        copy_engine=args.copy_engine if args.serve_copy_engine < 0 else args.serve_copy_engine)
        tune.apply_kernels(ctx, tuned)
        tmpls = serving.mix_templates(ctx, graphs=graphs, result_bytes=64)
        budget = serving.MIX_BUDGET
        srv = serving.mix_server(ctx, tmpls, lanes=args.serve_lanes, copy_lanes=args.serve_copy_lanes,
                                 transfer_lanes=args.serve_transfer_lanes)
        foot = [srv.footprint(sid) for sid in range(len(tmpls))]
        def one_rate(rate, nreq, serial=True):
            arr, shp = W.poisson_trace(4, nreq, rate, len(tmpls))
            log("serving: %d requests at %g/s, %d shapes" % (len(arr), rate, len(tmpls)))
            mix, st, _ = srv.run(arr, shp)
            if not serial:
                return {"requests": len(arr), "rate_per_s": rate,
                        "concurrent": {"p50_ms": st.p50_ms, "p99_ms": st.p99_ms, "req_per_s": st.req_per_s,
                                       "max_inflight": st.max_inflight, "max_queued": st.max_queued}}
            log("serving: serial baseline")
            ser, st2, _ = srv.run(arr, shp, mode=D.DAG_SERVE_SERIAL)
            return {
                "requests": len(arr), "rate_per_s": rate,
                "mean_footprint_mb": float(np.mean([foot[i][0] for i in shp])) / 2 ** 20,
                "concurrent": {"p50_ms": st.p50_ms, "p99_ms": st.p99_ms, "mean_ms": st.mean_ms,
                               "req_per_s": st.req_per_s, "max_inflight": st.max_inflight,
                               "max_queued": st.max_queued, "peak_device_gb": st.peak_device_bytes / 2 ** 30},
                "serial": {"p50_ms": st2.p50_ms, "p99_ms": st2.p99_ms, "mean_ms": st2.mean_ms,
                           "req_per_s": st2.req_per_s, "max_queued": st2.max_queued},
                "throughput_gain": st.req_per_s / st2.req_per_s if st2.req_per_s else None,
            }

        out = one_rate(args.rate, args.requests)
        out.update({"shapes": len(tmpls), "budget_bytes": budget, "lanes": args.serve_lanes,
                    "copy_lanes": args.serve_copy_lanes, "transfer_lanes": args.serve_transfer_lanes,
                    "copy_engine": args.copy_engine if args.serve_copy_engine < 0 else args.serve_copy_engine})
        # a second, lower arrival rate at which the serial baseline is not overloaded
        if args.low_rate:
            out["low_rate"] = one_rate(args.low_rate, max(1, args.requests // 2))
        # an arrival rate past what the loop can serve: its throughput there is the capacity
        if args.capacity_rate:
            out["capacity"] = one_rate(args.capacity_rate, max(1, args.requests // 2), serial=False)
        srv.close()
        ctx.close()
        return out

    workloads = ["bs", "vec", "img", "hits", "ml", "dl", "serve"] if args.workload == "all" else [args.workload]
    results = {}
    graphs = {}
    kt_bs = None
    for wl in workloads:
        if wl == "vec":
            prog = W.vec_program(n=1 << 20, seed=0)
            results[wl], _ = measure(wl, prog, 5, args.warmup, restore=("x", "y"))
            log("vec: cost of a dependency edge")
            results[wl]["edge_cost"] = edge_cost()
        elif wl == "bs":
            prog = W.bs_program(n=1 << 22, tasks=10, seed=1)
            results[wl], kt_bs = measure(wl, prog, args.steps, args.warmup)
            bs_prog = prog
        elif wl == "img":
            prog = W.img_program(side=2048, seed=2)
            results[wl], _ = measure(wl, prog, args.steps, args.warmup)
        elif wl == "hits":
            log("hits: generating the graph")
            prog = W.hits_program(n=1 << 20, deg=20, iters=10, seed=3)
            results[wl], _ = measure(wl, prog, args.steps, args.warmup, restore=("a", "h"), per_iter=6)
        elif wl == "ml":
            prog = W.ml_program(n=1 << 20, seed=5)
            results[wl], _ = measure(wl, prog, args.steps, args.warmup)
        elif wl == "dl":
            prog = W.dl_program(side=1024, seed=6)
            results[wl], _ = measure(wl, prog, args.steps, args.warmup)
        elif wl == "serve":
            results[wl] = measure_serving(graphs)

    if "serve" in results and len(results) == 1:
        sv = results["serve"]
        print(json.dumps({"metric": METRIC, "value": round(sv["concurrent"]["p50_ms"], 4), "unit": "ms (p50 latency)",
                          "n_gpus": 1, "steps": sv["requests"], "warmup": 0, "ms_per_step": None,
                          "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
                          "data": "synthetic", "config": {"workload": "serving_mix_poisson_2000"}, "serving": sv}),
              flush=True)
        return
    head = results.get("bs") or results[workloads[0]]
    line = {
        "metric": METRIC,
        "value": round(head["speedup"], 4),
        "unit": "x (serial-sync makespan / DAG makespan)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["makespan_ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "bs_fanout_10x2^22" if "bs" in results else head["workload"],
                   "max_streams": head["max_streams"], "copy_streams": args.copy_streams,
                   "copy_lanes": args.copy_lanes,
                   "spin_wait": args.spin_wait, "copy_engine": args.copy_engine,
                   "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "0") or 0)},
        "makespan_ms": round(head["makespan_ms"], 4),
        "serial_ms": round(head["serial_ms"], 4),
        "cp_bound_ms": round(head["cp_bound_ms"], 4),
        "cp_frac": round(head["cp_frac"], 4),
        "resource_bound_ms": round(head["resource_bound_ms"], 4),
        "resource_frac": round(head["resource_frac"], 4),
        "overlap": head["overlap"],
        "graph_ms": round(head["graph_ms"], 4),
        "graph_speedup": round(head["graph_speedup"], 4),
        "replay_ms": round(head["replay_ms"], 4),
        "replay_speedup": round(head["replay_speedup"], 4),
        "recurring_ms": round(head["recurring_ms"], 4),
        "recurring_speedup": round(head["recurring_speedup"], 4),
        # hand-written streams and waits (multi-stream replay, hipGraph); the
        # scheduler's makespan relative to them (> 1: the scheduler is slower)
        "hand_ms": round(head["hand_ms"], 4),
        "hand_graph_ms": round(head["hand_graph_ms"], 4),
        "vs_hand": round(head["makespan_ms"] / head["hand_ms"], 4),
        "vs_hand_graph": round(head["makespan_ms"] / head["hand_graph_ms"], 4),
    }
    if "graph_kernel_copies_ms" in head:
        line["graph_kernel_copies_ms"] = round(head["graph_kernel_copies_ms"], 4)
        line["graph_kernel_copies_speedup"] = round(head["graph_kernel_copies_speedup"], 4)
    if "bs" in results:
        # the kernel alone on the GPU, launched back to back on its stream
        # between two events (per-launch median of three batches of 20)
        avg = results["bs"]["kernels_isolated"]["bs_call"]["avg_us"] / 1e3   # ms per launch
        op = next(o for o in bs_prog.ops if o["kind"] == "kernel")
        by = M.algorithmic_bytes("bs_call", op["params"])
        v = kt_bs["bs_call"]
        fl = BS_FLOPS_PER_ELEMENT * (by // 8)
        ach = fl / avg / 1e9                          # TFLOP/s
        variant = int(tuned.get("bs_call", {}).get("variant", 0))
        # share of the SIMDs' issue cycles taken by VALU instructions (a wave64
        # instruction occupies a 16-lane SIMD for 4 cycles; 4 SIMDs per CU)
        valu_busy = (BS_VALU_PER_ELEMENT[variant] * (by // 8) / 64 * 4) / (4 * CUS * CLOCK_GHZ * 1e9 * avg / 1e3)
        line["roofline"] = {"kernel": "bs_call", "bound": "alu", "achieved": round(ach, 2),
                            "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(ach / FP64_PEAK_TFLOPS, 4),
                            "traffic": TRAFFIC_BS_BYTES, "avg_us": round(avg * 1e3, 2), "flops_per_launch": fl,
                            "bytes_per_launch": by, "hbm_gbs": round(by / avg / 1e6, 1),
                            "timing": "launches back to back alone on the GPU, events on their stream, 3 x 20",
                            "avg_us_gated_events": round(results["bs"]["kernels_isolated_gated_us"]["bs_call"], 2),
                            "avg_us_in_dag_events": round(1e3 * sum(t for t, _ in v) / len(v), 2),
                            "variant": variant, "valu_busy": round(valu_busy, 3)}
    if "serve" in results:
        line["serving"] = results.pop("serve")
    line["workloads"] = results
    if not args.no_cpu_baseline:
        # in a child process that never touches the GPU (the oracle's workers are forked)
        import subprocess
        for wl in [w for w in results if w in ("bs", "vec", "img", "hits", "ml", "dl")]:
            log("cpu baseline: %s (oracle, one thread and all cores)" % wl)
            r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-oracle", wl],
                               stdout=subprocess.PIPE, text=True, check=True)
            results[wl]["cpu_oracle"] = json.loads(r.stdout.strip().splitlines()[-1])
        if "bs" in results:
            add_cpu_line(line)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
