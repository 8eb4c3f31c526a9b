"""Launch a workload's DAG a few times plus a plain copy kernel of known size,
for profiler runs (kernel traces, and hardware-counter passes that need a
reference kernel to calibrate byte counters against).

Usage (under a profiler):
  python3 -m paper_2012_09646_amd.profile_run --workload bs --runs 3 --copy-mib 256
Prints one JSON line describing what was launched.
"""

import argparse
import json
import os

from . import dagrt as D
from . import metrics as M
from . import runner
from . import tune
from . import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def spmv_bounds(args, n=1 << 20, deg=20):
    """The SpMV alone (its tuned launch configuration) on matrices with the
    same shape and nonzero count as HITS' but different column patterns:
    sequential columns (every gather of x coalesced: the streaming floor),
    uniformly random columns (every gather a separate cache line: the random
    gather bound), and A^T and A themselves.  Each matrix gets its own context; its
    SpMVs run back to back after one partition."""
    import numpy as np
    nnz = n * deg
    rp = np.arange(0, nnz + 1, deg, dtype=np.int32)
    g = np.random.Generator(np.random.Philox(key=17))
    mats = [("sequential", rp, (np.arange(nnz) % n).astype(np.int32)),
            ("uniform", rp, g.integers(0, n, nnz).astype(np.int32))]
    gr = W.hits_graph(n, deg, 3)
    mats.append(("hits_at", gr["at_ptr"], gr["at_col"]))
    mats.append(("hits_a", gr["a_ptr"], gr["a_col"]))
    val = np.ones(nnz, np.float32)
    x = W.uniform_f32(18, n)
    order = []
    for name, ptr, col in mats:
        bufs = {"rp": W.Buf(ptr.nbytes, init=ptr), "ci": W.Buf(col.nbytes, init=col),
                "va": W.Buf(val.nbytes, init=val), "x": W.Buf(x.nbytes, init=x), "y": W.Buf(4 * n)}
        ops = [W.K("spmv", [("rp", "c"), ("ci", "c"), ("va", "c"), ("x", "c"), ("y", "m")],
                   nrows=n, ncols=n, nnz=int(col.size))] * args.runs
        prog = W.Program("spmv_" + name, bufs, ops, ["y"])
        ctx = D.Context(policy=D.DAG_SERIAL_SYNC if args.serial else D.DAG_PARALLEL_ASYNC)
        if args.tuned and os.path.exists(args.tuned):
            tune.apply_kernels(ctx, tune.load(args.tuned).get("kernels", {}))
        for item in args.set:
            k, cfg = item.split("=")
            ctx.set_launch(k, *[int(v) for v in cfg.split(",")])
        b = runner.Bound(ctx, prog, read_bytes=4)
        b.run()
        ctx.sync()
        order.append({"matrix": name, "spmv_launches": args.runs, "launch": list(ctx.get_launch("spmv"))})
        ctx.close()
    ctx = D.Context()
    nc = copies(ctx, args)
    ctx.close()
    print(json.dumps({"workload": "spmv_bounds", "order": order, "nnz": nnz, "nrows": n,
                      "copy_f32_bytes_read": 4 * nc, "copies": args.copies}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="bs", choices=["vec", "bs", "img", "hits", "ml", "dl", "spmv_bounds"],
                    help="spmv_bounds: the SpMV kernel alone on three matrices of 2^20 rows x 20 nonzeros "
                         "(sequential columns, uniformly random columns, HITS' A^T and A), runs times each in "
                         "that order")
    ap.add_argument("--runs", type=int, default=3)
    ap.add_argument("--copy-mib", type=int, default=256)
    ap.add_argument("--copies", type=int, default=3)
    ap.add_argument("--serial", action="store_true", help="serial policy: every call alone on the GPU")
    ap.add_argument("--tuned", default=os.path.join(ROOT, "paper_2012_09646_amd", "tuning", "gfx950.json"))
    ap.add_argument("--set", action="append", default=[], metavar="KERNEL=BLOCK,CAP,VARIANT",
                    help="launch configuration override after the tuning file (repeatable)")
    ap.add_argument("--trace", type=int, default=0, choices=[0, 1],
                    help="1: timing events on every task; the library's overlap figures of each run are printed "
                         "(to compare with a profiler timeline of the same runs)")
    ap.add_argument("--copy-engine", type=int, default=0, choices=[0, 1, 2, 3])
    ap.add_argument("--max-streams", type=int, default=8)
    args = ap.parse_args()
    if args.workload == "spmv_bounds":
        spmv_bounds(args)
        return
    prog, _ = tune.workload_program(args.workload)
    ctx = D.Context(policy=D.DAG_SERIAL_SYNC if args.serial else D.DAG_PARALLEL_ASYNC, trace=args.trace,
                    copy_engine=args.copy_engine, max_streams=args.max_streams)
    if args.tuned and os.path.exists(args.tuned):
        tune.apply_kernels(ctx, tune.load(args.tuned).get("kernels", {}))
    for item in args.set:
        name, cfg = item.split("=")
        ctx.set_launch(name, *[int(v) for v in cfg.split(",")])
    b = runner.Bound(ctx, prog, read_bytes=4)
    lib_overlap = []
    for _ in range(args.runs):
        if args.trace:
            D.dag_trace_reset(ctx.h)
        b.run()
        if args.trace:
            iv = []
            for pos in range(1, len(prog.ops) + 1):
                inf = ctx.info(b.base + pos)
                if inf.stream < 0 or inf.t_start_ms < 0:
                    continue
                kind = "C" if inf.kind in (D.DAG_TASK_KERNEL, D.DAG_TASK_REGION) else "T"
                iv.append((kind, inf.t_start_ms, inf.t_end_ms))
            o = M.overlap(iv)
            o["span_ms"] = max(e for _, _, e in iv) - min(s0 for _, s0, _ in iv)
            lib_overlap.append(o)
    ctx.sync()
    n = copies(ctx, args)
    ctx.close()
    print(json.dumps({"workload": args.workload, "runs": args.runs, "set": args.set, "copy_f32_bytes_read": 4 * n,
                      "copy_f32_bytes_written": 4 * n, "copies": args.copies, "library_overlap": lib_overlap}),
          flush=True)


def copies(ctx, args):
    """The calibration kernel: copy_f32 over copy_mib MiB, `copies` times."""
    n = args.copy_mib << 18  # fp32 elements
    src = ctx.alloc(4 * n)
    dst = ctx.alloc(4 * n)
    for _ in range(args.copies):
        ctx.kernel("copy_f32", [(src, "c"), (dst, "m")], n=n)
    ctx.sync()
    return n


if __name__ == "__main__":
    main()
