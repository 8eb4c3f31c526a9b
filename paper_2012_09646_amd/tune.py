"""Autotuner: launch configurations of the task kernels and the scheduler's
DAG-level knobs.

Kernels are tuned alone on the GPU, as the paper tunes launch parameters for
serial execution (Sec. V-A): for every kernel a workload uses, each candidate
(threads per workgroup, grid cap, kernel variant) is timed by
``dag_tune_kernel`` on the workload's own buffers after one full run of the
workload (so every input holds realistic data), summed over the kernel's
occurrences, and the fastest is kept.  The DAG knobs (stream pool size, copy
placement, hardware queue count) are then chosen by the median makespan of
whole runs, and kernel configurations within 3 % of the fastest alone are
retried inside the DAG, kept only when they shorten it by more than 3 % (the fastest alone can take every CU's registers and
leave nothing for a kernel that could run beside it).  Each
GPU_MAX_HW_QUEUES value is tried in a process of its own, since HIP fixes it
at start-up (the orchestrating process never touches the GPU).  Results are
stored as JSON keyed by GPU architecture (and marked with the ROCm release),
kernel and problem size, and loaded with ``load``/``apply_kernels``.  Only
configurations from ``candidates`` are installed; the GPU test suite checks
every one of them against the oracle.

Usage: python -m paper_2012_09646_amd.tune --workload img --out tuned.json
"""

import argparse
import json
import os
import statistics
import time

from . import dagrt as D
from . import runner
from . import workloads as W

ARCH = "gfx950"
BLOCKS = (64, 128, 256, 512, 1024)
CAPS = (0, 1024, 4096)
NEAR_TIE = 0.03  # kernel configurations this close to the fastest alone are retried inside the DAG
# Grid caps of the resident SpMV (workgroups; uncapped it fills every wave slot of the GPU, eight workgroups
# per CU), and the kernels whose fastest capped form is always retried inside the DAG: a kernel that holds
# every CU slot for its whole run keeps a kernel on another stream from starting.
RESIDENT_CAPS = (1792, 1536, 1024)
LEAVES_ROOM = {"spmv": lambda cfg: cfg[2] & 0x500 == 0x500 and cfg[1] != 0,
               "gauss_blur": lambda cfg: cfg[2] in (9, 11) and cfg[1] != 0,
               "sobel": lambda cfg: cfg[2] in (9, 11) and cfg[1] != 0}
TILE_SHAPES = ((64, 16), (64, 8), (64, 4), (32, 8))  # stencil tiles, in the kernels' variant order


def candidates(kernel):
    """Candidate (block, grid_cap, variant) triples of a built-in kernel."""
    if kernel in ("vec_square", "normalise", "unsharp_combine", "scale_l2", "copy_f32"):
        return [(b, c, 0) for b in BLOCKS for c in CAPS]
    if kernel == "bs_call":
        return [(b, c, v) for b in BLOCKS for c in CAPS for v in (0, 1, 2)]
    if kernel in ("vec_sum_diff", "minmax", "sumsq"):
        return [(b, c, v) for b in (256, 512, 1024) for c in (64, 128, 256, 512, 1024, 2048) for v in (0, 1)]
    if kernel == "spmv":
        # merge-path items per thread, or 0x100 | nonzeros per thread of the row-window form (0x400: resident
        # grid loading each workgroup's next tile early; a grid cap leaves CU slots to other streams)
        return ([(256, 0, v) for v in (4, 8, 12, 16, 0x104, 0x108, 0x110, 0x504, 0x508)] +
                [(256, c, 0x504) for c in RESIDENT_CAPS])
    if kernel == "spmv_rows":
        return [(256, c, v) for v in (4, 8, 16, 32) for c in (0, 2048, 8192)]
    if kernel in ("gauss_blur", "sobel"):
        # variant bit 0: tile order (row-major, or one run per XCD); bits 1-2: tile shape 64x16, 64x8,
        # 64x4 or 32x8, whose workgroup is the tile's threads (four rows of one column each); 9 and 11:
        # 64x16 and 64x8 on a resident grid (grid cap: workgroups, 0 = as many as fit) that loads each
        # workgroup's next tile while it computes the current one
        return ([(tw * th // 4, 0, order | (shape << 1))
                 for shape, (tw, th) in enumerate(TILE_SHAPES) for order in (0, 1)] +
                [(256, c, 9) for c in (0, 1024, 512)] + [(128, c, 11) for c in (0, 2048, 1024)])
    if kernel == "nb_proba":
        # one workgroup per CU fits beside the 128 KB table: its size sets the waves per CU
        return [(b, c, 0) for b in (256, 512, 1024) for c in (0, 256, 512, 1024)]
    if kernel == "ridge_proba":
        # variant = rows per thread: 0 one, 2 two by 8-byte loads, 4 four by
        # 16-byte loads (workgroups up to 256 for 2 and 4)
        return [(b, c, v) for b in (64, 128, 256, 512) for c in CAPS for v in (0, 2, 4) if v == 0 or b <= 256]
    if kernel == "ensemble":
        return [(b, c, 0) for b in BLOCKS for c in CAPS]
    if kernel == "dense":
        # variant 0: one input per lane; 1, 2: whole 1 KB weight loads per wave,
        # 2 or 4 chunks of 64 inputs in flight; 3, 4: the same with the final
        # add in a second kernel
        return [(b, c, v) for b in (256, 512, 1024) for c in (128, 256, 512, 1024, 2048) for v in (0, 1, 2, 3, 4)]
    if kernel == "conv3x3_relu_pool":
        # variant 0: one input channel per barrier pair; 1: channels pipelined;
        # 2: pipelined with fp64 weights read as scalars; 3: implicit GEMM on
        # the fp64 matrix cores (where cin % 4 == 0 and cout % 16 == 0); 4: the
        # same with 16 output channels per workgroup (twice the workgroups)
        return [(256, 0, v) for v in (0, 1, 2, 3, 4)]
    return []  # the delay kernel


def size_key(op):
    p = op.get("params", {})
    return ",".join("%s=%s" % (k, p[k]) for k in sorted(p) if k in ("n", "w", "h", "nrows", "nnz", "ksize"))


ONE_LAUNCH_VARIANT = ("vec_sum_diff", "minmax", "sumsq")  # variant 0: two kernels, 1: one


def tune_kernels(ctx, prog, reps=20, log=None):
    """Tune every tunable kernel of `prog` in context `ctx`; installs the
    winners in ctx and returns {kernel: entry}."""
    b = runner.Bound(ctx, prog, read_bytes=0)
    b.run()
    ctx.sync()
    occ = {}
    for op in prog.ops:
        if op["kind"] == "kernel" and candidates(op["kernel"]):
            occ.setdefault(op["kernel"], []).append(op)
    out = {}
    for k, ops in occ.items():
        cands = candidates(k)
        default = ctx.get_launch(k)  # before tuning installs a winner
        total = [0.0] * len(cands)
        for op in ops:
            prm = D.make_params(k, op["params"])
            args = [(b.h[n], D.DAG_MUTABLE if m == "m" else D.DAG_CONST) for n, m in op["args"]]
            _, us = D.dag_tune_kernel(ctx.h, D.KERNEL_IDS[k], prm, args, cands, reps)
            total = [t + u if (t >= 0 and u >= 0) else -1.0 for t, u in zip(total, us)]
        valid = [i for i, t in enumerate(total) if t >= 0]
        best = min(valid, key=lambda i: total[i])
        di = cands.index(default) if default in cands else None
        set_launch(ctx, k, cands[best])
        # near-ties (within NEAR_TIE of the best alone), fastest first: the DAG
        # tuning picks among them by makespan, since the configuration that
        # is fastest alone may leave no room for a concurrent kernel
        near = sorted((i for i in valid if i != best and total[i] <= total[best] * (1 + NEAR_TIE)),
                      key=lambda i: total[i])[:3]
        # a reduction finished by its last workgroup (variant 1) saves a launch, which in a DAG of short
        # kernels can matter more than its time alone: its fastest form is always tried in the DAG
        if k in ONE_LAUNCH_VARIANT and cands[best][2] != 1:
            ones = [i for i in valid if cands[i][2] == 1]
            if ones:
                f = min(ones, key=lambda i: total[i])
                if f not in near:
                    near.append(f)
        # likewise the fastest form that leaves CU slots free for kernels on other streams
        if k in LEAVES_ROOM and not LEAVES_ROOM[k](cands[best]):
            room = [i for i in valid if LEAVES_ROOM[k](cands[i])]
            if room:
                f = min(room, key=lambda i: total[i])
                if f not in near:
                    near.append(f)
        out[k] = {"block": cands[best][0], "grid_cap": cands[best][1], "variant": cands[best][2],
                  "us": total[best] / len(ops), "size": size_key(ops[0]), "launches": len(ops),
                  "default_us": (total[di] / len(ops)) if di is not None and total[di] >= 0 else None,
                  "near": [list(cands[i]) + [total[i] / len(ops)] for i in near]}
        if log:
            log("tuned %s: %s %.2f us (default %s)" % (k, cands[best], out[k]["us"], out[k]["default_us"]))
    b.release()
    return out


def tune_dag(prog, kernels, pools=(1, 2, 4, 8, 16), copy_modes=((0, 1), (0, 2), (0, 3), (1, 1)), runs=15,
             restore=(), log=None, hw_queues=None):
    """Choose max_streams and copy placement (copy_streams, lanes per
    direction) by median makespan, among the configurations whose streams
    (plus the context's own) fit the hardware queues: with more streams than
    queues, HIP shares queues between streams in an order that changes from
    process to process, and the same configuration was measured 1.6x slower
    in one process than in the next."""
    table = []
    has_copies = any(o["kind"] == "copy" for o in prog.ops)
    for cm, lanes in copy_modes:
        if (cm == 1 or lanes > 1) and not has_copies:
            continue
        for ms in pools:
            m, streams = makespan(prog, kernels, {}, ms, cm, lanes, restore, runs)
            fits = hw_queues is None or streams + 1 <= hw_queues
            row = {"max_streams": ms, "copy_streams": cm, "copy_lanes": lanes, "ms": m, "streams": streams,
                   "fits": fits}
            table.append(row)
            if log:
                log("dag %s: max_streams=%d copy_streams=%d lanes=%d %.4f ms (%d streams%s)" % (
                    prog.name, ms, cm, lanes, m, streams, "" if fits else ", more than the queues"))
    ok = [r for r in table if r["fits"]] or table
    best = dict(min(ok, key=lambda r: r["ms"]))
    return best, table


def makespan(prog, kernels, overrides, ms, cm, lanes, restore=(), runs=15):
    """Median makespan (ms) of `runs` whole runs and the streams used, with
    the kernel table `kernels` and per-kernel (block, cap, variant)
    `overrides`."""
    ctx = D.Context(max_streams=ms, copy_streams=cm, copy_lanes=lanes)
    apply_kernels(ctx, kernels)
    for k, cfg in overrides.items():
        set_launch(ctx, k, cfg)
    b = runner.Bound(ctx, prog, read_bytes=4)
    pris = {}
    for dst in restore:
        pris[dst] = ctx.alloc(prog.bufs[dst].nbytes)
        ctx.host_write(pris[dst], prog.bufs[dst].init)
    ts = []
    for i in range(runs + 2):
        for dst in restore:
            ctx.copy(b.h[dst], pris[dst], prog.bufs[dst].nbytes)
        ctx.sync()
        t0 = time.perf_counter()
        b.run()
        if i >= 2:
            ts.append((time.perf_counter() - t0) * 1e3)
    streams = ctx.stats().streams
    ctx.close()
    return statistics.median(ts), streams


def break_ties(prog, kernels, best, restore=(), runs=15, rounds=3, log=None, measure=None):
    """For every kernel of `prog` with near-tie configurations, try each in
    the DAG (one kernel at a time, the others at their current choice) with
    the chosen pool and copy placement.  The current choice and the trial are
    measured alternately, `rounds` times each (makespans of separate contexts
    vary by several per cent), and the trial is kept if its median over the
    rounds is more than 3 % below the current one's.  Returns
    ({kernel: [block, cap, variant]}, makespan)."""
    measure = measure or makespan
    used = sorted({o["kernel"] for o in prog.ops if o["kind"] == "kernel"})
    cfg = (best["max_streams"], best["copy_streams"], best["copy_lanes"])
    chosen = {}
    cur = best["ms"]
    for k in used:
        for alt in (kernels.get(k) or {}).get("near", []):
            trial = dict(chosen, **{k: tuple(alt[:3])})
            mb, mt = [], []
            for _ in range(rounds):
                mb.append(measure(prog, kernels, chosen, *cfg, restore, runs)[0])
                mt.append(measure(prog, kernels, trial, *cfg, restore, runs)[0])
            base, m = statistics.median(mb), statistics.median(mt)
            if log:
                log("dag %s: %s=%s %.4f ms against %.4f" % (prog.name, k, tuple(alt[:3]), m, base))
            if m < base * 0.97:
                chosen, cur = trial, m
    return {k: list(v) for k, v in chosen.items()}, cur


def check_candidate(kernel, cfg):
    """Only configurations of candidates(kernel) are ever installed: that is
    the set the GPU parity sweep checks against the oracle."""
    cfg = tuple(int(v) for v in cfg)
    if cfg not in candidates(kernel):
        raise ValueError("%s: launch configuration %s is not one of the swept candidates" % (kernel, cfg))
    return cfg


def set_launch(ctx, kernel, cfg):
    ctx.set_launch(kernel, *check_candidate(kernel, cfg))


def apply_kernels(ctx, kernels):
    for k, e in (kernels or {}).items():
        set_launch(ctx, k, (e["block"], e["grid_cap"], e["variant"]))


def rocm_version():
    """ROCm release of this machine (from /opt/rocm/.info/version), '' if unknown."""
    for path in ("/opt/rocm/.info/version", "/opt/rocm/.info/version-dev"):
        try:
            with open(path) as f:
                return f.read().strip().split("-")[0]
        except OSError:
            pass
    return ""


def load(path):
    """The table for this architecture.  A table made under another ROCm
    release still loads (its configurations are all valid candidates) but is
    marked: data["rocm_matches"] is False and the caller reports it."""
    with open(path) as f:
        data = json.load(f)
    if data.get("arch") != ARCH:
        raise ValueError("tuning file is for %s, not %s" % (data.get("arch"), ARCH))
    for k, e in data.get("kernels", {}).items():
        check_candidate(k, (e["block"], e["grid_cap"], e["variant"]))
    for name, e in data.get("dag", {}).items():
        for k, cfg in e.get("kernels", {}).items():
            check_candidate(k, cfg)
    data["rocm_matches"] = data.get("rocm") == rocm_version()
    return data


def save(path, data):
    data = dict(data)
    data["arch"] = ARCH
    data["rocm"] = rocm_version()
    data.pop("rocm_matches", None)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def workload_program(name):
    if name == "vec":
        return W.vec_program(n=1 << 20, seed=0), ("x", "y")
    if name == "bs":
        return W.bs_program(n=1 << 22, tasks=10, seed=1), ()
    if name == "img":
        return W.img_program(side=2048, seed=2), ()
    if name == "hits":
        return W.hits_program(n=1 << 20, iters=10, seed=3), ("a", "h")
    if name == "ml":
        return W.ml_program(n=1 << 20, seed=5), ()
    if name == "dl":
        return W.dl_program(side=1024, seed=6), ()
    raise ValueError(name)


def _worker(args, log):
    """Runs inside one process (one GPU_MAX_HW_QUEUES setting)."""
    names = ["vec", "bs", "img", "hits", "ml", "dl"] if args.workload == "all" else [args.workload]
    out = {"kernels": {}, "dag": {}}
    if args.worker == "kernels":
        for name in names:
            prog, _ = workload_program(name)
            ctx = D.Context()
            ks = tune_kernels(ctx, prog, args.reps, log)
            ctx.close()
            for k, e in ks.items():
                prev = out["kernels"].get(k)
                if prev is None or e["launches"] >= prev.get("launches", 0):
                    out["kernels"][k] = e
    else:
        with open(args.kernels_json) as f:
            kernels = json.load(f)["kernels"]
        hwq = int(os.environ.get("GPU_MAX_HW_QUEUES", "0") or 0) or 4  # HIP's default is 4
        for name in names:
            prog, restore = workload_program(name)
            best, table = tune_dag(prog, kernels, restore=restore, log=log, hw_queues=hwq)
            over, ms = break_ties(prog, kernels, best, restore=restore, log=log)
            if over:
                best = dict(best, kernels=over, ms_alone_kernels=best["ms"], ms=ms)
            out["dag"][name] = dict(best, table=table)
    with open(args.worker_out, "w") as f:
        json.dump(out, f)


def _spawn(extra, out, hw_queues=None):
    """One worker process; the parent never touches the GPU (the hardware
    queue count is fixed when HIP starts, so each setting needs a process)."""
    import subprocess
    import sys
    env = dict(os.environ)
    if hw_queues:
        env["GPU_MAX_HW_QUEUES"] = str(hw_queues)
    cmd = [sys.executable, "-m", "paper_2012_09646_amd.tune"] + extra + ["--worker-out", out]
    subprocess.run(cmd, env=env, check=True)
    with open(out) as f:
        return json.load(f)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="all", choices=["all", "vec", "bs", "img", "hits", "ml", "dl"])
    ap.add_argument("--out", required=False)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--dag", action="store_true", help="also tune pool size, copy placement and hardware queues")
    ap.add_argument("--hw-queues", default="4,8,16",
                    help="GPU_MAX_HW_QUEUES values tried by --dag, one worker process each")
    ap.add_argument("--worker", choices=["kernels", "dag"], help=argparse.SUPPRESS)
    ap.add_argument("--worker-out", help=argparse.SUPPRESS)
    ap.add_argument("--kernels-json", help=argparse.SUPPRESS)
    args = ap.parse_args()
    log = lambda *a: print("[tune]", *a, flush=True)
    if args.worker:
        _worker(args, log)
        return
    if not args.out:
        ap.error("--out is required")
    tmp = args.out + ".part"
    common = ["--workload", args.workload, "--reps", str(args.reps)]
    data = _spawn(common + ["--worker", "kernels"], tmp)
    if args.dag:
        kfile = args.out + ".kernels"
        with open(kfile, "w") as f:
            json.dump({"kernels": data["kernels"]}, f)
        for hwq in [int(v) for v in args.hw_queues.split(",") if v]:
            log("dag knobs with GPU_MAX_HW_QUEUES=%d" % hwq)
            part = _spawn(common + ["--worker", "dag", "--kernels-json", kfile], tmp, hw_queues=hwq)
            for name, e in part["dag"].items():
                e = dict(e, hw_queues=hwq)
                for row in e["table"]:
                    row["hw_queues"] = hwq
                prev = data["dag"].get(name)
                if prev is None:
                    data["dag"][name] = e
                else:
                    table = prev["table"] + e["table"]
                    # a configuration that fits its queues beats one that does not
                    better = (e.get("fits", True), -e["ms"]) > (prev.get("fits", True), -prev["ms"])
                    data["dag"][name] = dict(e if better else prev, table=table)
        os.remove(kfile)
    if os.path.exists(tmp):
        os.remove(tmp)
    save(args.out, data)
    log("wrote", args.out)


if __name__ == "__main__":
    main()
