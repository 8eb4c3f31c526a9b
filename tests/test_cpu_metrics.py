"""Pins of the measurement helpers on hand-computed cases (CPU only)."""

from paper_2012_09646_amd import metrics as M


def test_critical_path_diamond():
    # VEC diamond: 1 -> 3, 2 -> 3; weights 2, 5, 1 -> path 2,3 = 6
    length, path = M.critical_path(3, [(1, 3), (2, 3)], {1: 2.0, 2: 5.0, 3: 1.0})
    assert length == 6.0 and path == [2, 3]


def test_critical_path_chain_and_isolated():
    length, path = M.critical_path(5, [(1, 2), (2, 4)], {1: 1, 2: 1, 3: 10, 4: 1, 5: 0.5})
    assert length == 10 and path == [3]
    length, path = M.critical_path(5, [(1, 2), (2, 4), (3, 4)], {1: 1, 2: 1, 3: 10, 4: 1, 5: 0.5})
    assert length == 11 and path == [3, 4]
    assert M.critical_path(0, [], {}) == (0.0, [])


def test_overlap_hand_values():
    # kernel [0,10), transfer [5,15), kernel [8,12)
    iv = [("C", 0, 10), ("T", 5, 15), ("C", 8, 12)]
    o = M.overlap(iv)
    # CT: kernel1 overlaps T on [5,10) = 5, kernel2 on [8,12) = 4 -> 9 / 14
    assert abs(o["CT"] - 9 / 14) < 1e-12
    # TC: T overlaps union of kernels [0,12) on [5,12) = 7 -> 7/10
    assert abs(o["TC"] - 0.7) < 1e-12
    # CC: k1 overlaps k2 on [8,10) = 2; k2 overlaps k1 on [8,10) = 2 -> 4/14
    assert abs(o["CC"] - 4 / 14) < 1e-12
    # TOT: k1 vs union(T,k2)=[5,15): 5; T vs union(k1,k2)=[0,12): 7; k2 vs [0,15): 4 -> 16/24
    assert abs(o["TOT"] - 16 / 24) < 1e-12


def test_overlap_serial_timeline_is_zero():
    iv = [("T", 0, 1), ("C", 1, 2), ("T", 2, 3), ("C", 3.5, 4)]
    o = M.overlap(iv)
    assert o == {"CT": 0.0, "TC": 0.0, "CC": 0.0, "TOT": 0.0}
    assert M.overlap([("C", 0, 1)])["CT"] == 0.0 and M.overlap([("C", 0, 1)])["TC"] is None


def test_percentile_nearest_rank():
    v = list(range(1, 101))
    assert M.percentile(v, 50) == 50 and M.percentile(v, 99) == 99 and M.percentile(v, 100) == 100
    assert M.percentile([3, 1, 2], 50) == 2


def test_rocprof_intervals_and_runs(tmp_path):
    k = tmp_path / "k.csv"
    c = tmp_path / "c.csv"
    k.write_text('"Kernel_Name","Start_Timestamp","End_Timestamp"\n"a",100,200\n"b",150,260\n"a",10000,10100\n')
    c.write_text('"Direction","Start_Timestamp","End_Timestamp"\n'
                 '"MEMORY_COPY_HOST_TO_DEVICE",50,120\n"MEMORY_COPY_DEVICE_TO_DEVICE",300,310\n')
    iv = M.rocprof_intervals(str(k), str(c))
    assert [(x[0], x[1]) for x in iv] == [("T", 50), ("C", 100), ("C", 150), ("C", 300), ("C", 10000)]
    runs = M.split_runs(iv, 1000)
    assert [len(r) for r in runs] == [4, 1]
    o = M.overlap([(x[0], x[1], x[2]) for x in runs[0]])
    # T [50,120) overlaps kernels on [100,120) = 20 of 70
    assert abs(o["TC"] - 20 / 70) < 1e-12


def test_dependency_gaps_take_the_last_parent_and_split_by_stream():
    # 1 and 2 on streams 0 and 1 end at 5 and 7; 3 (stream 0) starts at 9:
    # its last parent is 2 (cross-stream), gap 2; 4 follows 3 on stream 0
    edges = {(1, 3), (2, 3), (3, 4)}
    streams = {1: 0, 2: 1, 3: 0, 4: 0}
    times = {1: (0.0, 5.0), 2: (1.0, 7.0), 3: (9.0, 10.0), 4: (10.5, 11.0)}
    g = M.dependency_gaps(edges, streams, times)
    assert g == {"same": [0.5], "cross": [2.0]}
    # untimed tasks (host reads) are ignored
    assert M.dependency_gaps({(1, 5)}, streams, times) == {"same": [], "cross": []}


def test_trace_overlap_reads_a_rocprofv3_timeline(tmp_path):
    """The timeline reader behind the profile cross-check of the overlap
    figures: kernels by name, copy kernels and memory copies as transfers,
    runs split at the largest gaps between the library's task ranges."""
    import csv
    from paper_2012_09646_amd import trace_overlap as TO
    k = [("k_bs_call<2>", 100, 200), ("k_copy_bytes", 150, 300), ("other", 0, 1000), ("k_bs_call<2>", 2100, 2200)]
    with open(tmp_path / "p_kernel_trace.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writerows(k)
    with open(tmp_path / "p_memory_copy_trace.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Start_Timestamp", "End_Timestamp"])
        w.writerow([50, 120])
        w.writerow([2000, 2150])
    with open(tmp_path / "p_marker_api_trace.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Function", "Start_Timestamp", "End_Timestamp"])
        w.writerows([("dagrt task 1 copy stream 1 waits 0", 40, 45), ("dagrt task 2 bs_call stream 0 waits 1", 46, 50),
                     ("dagrt task 7 copy stream 1 waits 0", 1990, 1995)])
    ivs = TO.intervals(str(tmp_path), ["bs_call"], ["k_copy_bytes"])
    assert ivs == [("T", 50, 120), ("C", 100, 200), ("T", 150, 300), ("T", 2000, 2150), ("C", 2100, 2200)]
    runs = TO.split_runs(ivs, TO.task_ranges(str(tmp_path)), 2)
    assert [len(r) for r in runs] == [3, 2]
    o = M.overlap([(kind, a, b) for kind, a, b in runs[0]])
    # the kernel [100, 200) is covered by transfers on [100, 120) and [150, 200)
    assert abs(o["CT"] - 0.7) < 1e-12


def test_algorithmic_bytes_equal_the_argument_buffers():
    """The roofline's compulsory bytes of every kernel of every workload DAG
    equal what its arguments hold in the program: each buffer once, except a
    buffer the kernel both reads and writes (vec_square updates x in place),
    which moves twice."""
    from paper_2012_09646_amd import workloads as W
    in_place = {"vec_square"}
    progs = [W.vec_program(n=1000, seed=0), W.bs_program(n=1000, tasks=2, seed=1), W.img_program(side=64, seed=2),
             W.hits_program(n=500, iters=2, seed=3), W.ml_program(n=300, seed=5), W.dl_program(side=64, seed=6)]
    seen = set()
    for prog in progs:
        for o in prog.ops:
            if o["kind"] != "kernel":
                continue
            k = o["kernel"]
            held = sum(prog.bufs[b].nbytes * (2 if m == "m" and k in in_place else 1)
                       for b, m in dict(o["args"]).items())
            assert M.algorithmic_bytes(k, o["params"]) == held, (k, o["params"])
            seen.add(k)
    assert len(seen) == 18
