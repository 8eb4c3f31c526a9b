"""Measurement helpers over task intervals and the DAG.

critical_path  contention-free bound (paper Sec. V-E): the longest path of
               the DAG when every task takes its isolated time, i.e. the time
               it takes alone on the whole GPU (measured under the serial
               policy).
overlap        the four overlap figures of Sec. V-F over an execution
               timeline: CT (share of kernel time overlapping any transfer),
               TC (share of transfer time overlapping any kernel), CC (share
               of kernel time overlapping another kernel) and TOT (share of
               all busy time overlapping any other operation; an interval that
               overlaps several others is counted once, via the union).
"""


def critical_path(n, edges, weight):
    """Longest weighted path.  n tasks at positions 1..n, edges (src, dst)
    with src < dst, weight[pos] >= 0 (missing = 0).  Returns (length, path)."""
    parents = {}
    for s, d in edges:
        parents.setdefault(d, []).append(s)
    best = [0.0] * (n + 1)
    prev = [0] * (n + 1)
    for j in range(1, n + 1):
        w = float(weight.get(j, 0.0))
        b, arg = 0.0, 0
        for p in parents.get(j, ()):
            if best[p] > b:
                b, arg = best[p], p
        best[j] = b + w
        prev[j] = arg
    end = max(range(1, n + 1), key=lambda j: best[j]) if n else 0
    path = []
    j = end
    while j:
        path.append(j)
        j = prev[j]
    return (best[end] if n else 0.0), path[::-1]


def _union(iv):
    out = []
    for a, b in sorted(iv):
        if b <= a:
            continue
        if out and a <= out[-1][1]:
            out[-1][1] = max(out[-1][1], b)
        else:
            out.append([a, b])
    return out


def _covered(a, b, union):
    """Length of [a, b) covered by a sorted disjoint interval list."""
    tot = 0.0
    for x, y in union:
        lo, hi = max(a, x), min(b, y)
        if hi > lo:
            tot += hi - lo
    return tot


def overlap(intervals):
    """intervals: list of (kind, start, end) with kind 'C' (kernel) or 'T'
    (transfer).  Returns dict CT, TC, CC, TOT in [0, 1] (None when the
    denominator is empty)."""
    ks = [(a, b) for k, a, b in intervals if k == "C"]
    ts = [(a, b) for k, a, b in intervals if k == "T"]
    allv = ks + ts
    uk, ut = _union(ks), _union(ts)

    def frac(num, den):
        return None if den <= 0 else num / den

    def self_excl(items, idx_pool):
        num = 0.0
        for i, (a, b) in enumerate(items):
            others = _union([iv for j, iv in enumerate(idx_pool) if j != i])
            num += _covered(a, b, others)
        return num

    len_k = sum(b - a for a, b in ks)
    len_t = sum(b - a for a, b in ts)
    ct = frac(sum(_covered(a, b, ut) for a, b in ks), len_k)
    tc = frac(sum(_covered(a, b, uk) for a, b in ts), len_t)
    cc = frac(self_excl(ks, ks), len_k)
    tot = frac(self_excl(allv, allv), len_k + len_t)
    return {"CT": ct, "TC": tc, "CC": cc, "TOT": tot}


def dependency_gaps(edges, streams, times):
    """Idle time between a task's last-finishing parent and the task (the
    latency an edge costs on the device).  edges: (src, dst) positions;
    streams: {pos: stream}; times: {pos: (start, end)} for timed GPU tasks.
    For every timed task with timed parents, the parent that ends last is the
    one the task waited for; its gap start(task) - end(parent) goes to
    'same' when both ran on one stream (stream order) and to 'cross' when
    the parent ran on another stream (an event wait).  Returns
    {'same': [...], 'cross': [...]}, in the units of `times`."""
    parents = {}
    for s, d in edges:
        if s in times and d in times:
            parents.setdefault(d, []).append(s)
    out = {"same": [], "cross": []}
    for d, ps in sorted(parents.items()):
        p = max(ps, key=lambda q: times[q][1])
        gap = times[d][0] - times[p][1]
        out["same" if streams.get(p) == streams.get(d) else "cross"].append(gap)
    return out


def percentile(values, q):
    """Nearest-rank percentile (q in (0, 100])."""
    v = sorted(values)
    if not v:
        return None
    import math
    k = max(1, int(math.ceil(q / 100.0 * len(v))))
    return v[k - 1]


def algorithmic_bytes(kernel, p):
    """Compulsory HBM bytes of one launch of a built-in kernel: every input
    read once, every output written once (CSR SpMV: the matrix, one read of x
    and one write of y)."""
    if kernel == "vec_square":
        return 8 * p["n"]
    if kernel == "vec_sum_diff":
        return 8 * p["n"] + 4
    if kernel == "bs_call":
        return 8 * p["n"]
    if kernel in ("gauss_blur", "sobel"):
        return 8 * p["w"] * p["h"]
    if kernel == "minmax":
        return 4 * p["n"] + 8
    if kernel == "normalise":
        return 8 * p["n"] + 8
    if kernel == "unsharp_combine":
        return 32 * p["n"]
    if kernel in ("spmv", "spmv_rows"):
        return 4 * (p["nrows"] + 1) + 8 * p["nnz"] + 4 * p["ncols"] + 4 * p["nrows"]
    if kernel == "sumsq":
        return 4 * p["n"] + 8
    if kernel == "scale_l2":
        return 8 * p["n"] + 8
    if kernel == "copy_f32":
        return 8 * p["n"]
    if kernel == "nb_proba":
        n, F, C, V = p["n"], p["features"], p["classes"], p["categories"]
        return 4 * n * F + 4 * C * F * V + 4 * C + 4 * n * C
    if kernel == "ridge_proba":
        n, F, C = p["n"], p["features"], p["classes"]
        return 4 * n * F + 4 * (2 * F + C * F + C) + 4 * n * C
    if kernel == "ensemble":
        n, C = p["n"], p["classes"]
        return 12 * n * C + 4 * n
    if kernel == "conv3x3_relu_pool":
        cin, cout, h, w = p["cin"], p["cout"], p["h"], p["w"]
        return 4 * cin * h * w + 36 * cout * cin + 4 * cout + cout * h * w
    if kernel == "dense":
        return 4 * p["n"] * (p["m"] + 1) + 8 * p["m"]
    if kernel == "siamese_combine":
        return 16 * p["m"] + 8
    return 0


def rocprof_intervals(kernel_csv, copy_csv=None, name_filter=None):
    """(kind, start_ns, end_ns, name) from rocprofv3 --kernel-trace /
    --memory-copy-trace CSV files; kind 'C' for kernels, 'T' for copies
    between host and device (device-to-device copies count as kernels)."""
    import csv
    out = []
    with open(kernel_csv) as f:
        for r in csv.DictReader(f):
            if name_filter and not name_filter(r["Kernel_Name"]):
                continue
            out.append(("C", int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]))
    if copy_csv:
        with open(copy_csv) as f:
            for r in csv.DictReader(f):
                d = r["Direction"]
                kind = "T" if ("HOST_TO_DEVICE" in d or "DEVICE_TO_HOST" in d) else "C"
                out.append((kind, int(r["Start_Timestamp"]), int(r["End_Timestamp"]), d))
    out.sort(key=lambda e: e[1])
    return out


def split_runs(intervals, gap_ns):
    """Split a sorted timeline into runs separated by idle gaps > gap_ns."""
    runs, cur, end = [], [], None
    for e in intervals:
        if cur and e[1] - end > gap_ns:
            runs.append(cur)
            cur = []
        cur.append(e)
        end = e[2] if end is None or not cur[:-1] else max(end, e[2])
    if cur:
        runs.append(cur)
    return runs
