"""The native scheduler in schedule-only mode (no GPU: dry_run makes no HIP
call) against the oracle: edges, streams and event waits must be identical.
Also the C-ABI's argument checks and error conventions."""

import random

import numpy as np
import pytest

import dagcases
from oracle import dag as odag
from paper_2012_09646_amd import dagrt as D
from paper_2012_09646_amd import runner
from paper_2012_09646_amd import workloads as W


def run_dry(ops, max_streams):
    ctx = D.Context(dry_run=True, max_streams=max_streams, copy_streams=1)
    names = sorted({b for op in ops for b in
                    ([a for a, _ in op["args"]] if op["kind"] in ("kernel", "macro") else
                     [op["buf"]] if op["kind"] in ("host_read", "host_write") else [])})
    h = {n: ctx.alloc(256) for n in names}
    name_of = {v: k for k, v in h.items()}
    ids = []
    for op in ops:
        k = op["kind"]
        if k in ("kernel", "macro"):
            ids.append(ctx.kernel("spin", [(h[b], m) for b, m in op["args"]], ns=0))
        elif k == "host_read":
            ids.append(D.dag_host_read(ctx.h, h[op["buf"]]))
        elif k == "host_write":
            ids.append(D.dag_host_write(ctx.h, h[op["buf"]], 0, None, 0))
        elif k == "sync":
            ctx.sync()
            ids.append(ctx.stats().tasks)
    assert ids == list(range(1, len(ops) + 1))
    edges = {(s, d, name_of[b], kd) for s, d, b, kd in ctx.edges()}
    streams = {}
    waits = {}
    for i in ids:
        inf = ctx.info(i)
        if inf.stream >= 0:
            streams[i] = inf.stream
            waits[i] = ctx.waits(i)
    return ctx, edges, streams, waits


def check_against_oracle(ops, max_streams):
    g = odag.build_dag(ops)
    st, wt = odag.replay_streams(ops, g, max_streams)
    ctx, edges, streams, waits = run_dry(ops, max_streams)
    assert edges == g.edges
    assert streams == st
    assert waits == {k: v for k, v in wt.items()}
    for i in range(1, len(ops) + 1):
        inf = ctx.info(i)
        assert bool(inf.vertex) == g.vertex[i]
        assert bool(inf.active) == (i not in g.retired_by and ops[i - 1]["kind"] == "kernel")
    ctx.close()


CASES = dagcases.load_cases()


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_golden_cases_native(case):
    check_against_oracle(case["ops"], case["max_streams"])


@pytest.mark.parametrize("seed", range(150))
def test_random_programs_native(seed):
    rnd = random.Random(1000 + seed)
    ops = dagcases.random_program(rnd, rnd.randint(3, 45), rnd.randint(1, 6))
    check_against_oracle(ops, rnd.choice([1, 2, 3, 4, 8, 64]))


def test_many_readers_compaction():
    # long read-only runs with periodic host reads exercise reader-list compaction
    ops = []
    for i in range(120):
        ops.append({"kind": "kernel", "kernel": "spin", "params": {},
                    "args": [("A", "c"), ("B%d" % (i % 5), "m")]})
        if i % 17 == 3:
            ops.append({"kind": "host_read", "buf": "B%d" % (i % 5)})
    ops.append({"kind": "kernel", "kernel": "spin", "params": {}, "args": [("A", "m")]})
    check_against_oracle(ops, 8)


@pytest.mark.parametrize("maker,pool", [
    (lambda: W.vec_program(n=64), 8),
    (lambda: W.bs_program(n=64, tasks=10), 4),
    (lambda: W.bs_program(n=64, tasks=10), 16),
    (lambda: W.img_program(side=16), 8),
    (lambda: W.hits_program(n=64, deg=4, iters=10), 8),
    (lambda: W.hits_program(n=64, deg=4, iters=3), 1),
])
def test_workload_programs_native(maker, pool):
    prog = maker()
    g = odag.build_dag(prog.ops)
    st, wt = odag.replay_streams(prog.ops, g, pool)
    ctx = D.Context(dry_run=True, max_streams=pool, copy_streams=1)
    b = runner.Bound(ctx, prog, upload=False)
    b.run()
    assert b.edges() == g.edges
    assert b.streams() == st
    assert {k: v for k, v in b.waits().items() if k in st} == wt
    # the single-call path gives the same DAG as the batched one
    ctx2 = D.Context(dry_run=True, max_streams=pool, copy_streams=1)
    b2 = runner.Bound(ctx2, prog, upload=False)
    b2.run_calls()
    assert b2.edges() == g.edges and b2.streams() == st
    ctx.close()
    ctx2.close()


def test_region_replay_is_one_task_with_union_access():
    ctx = D.Context(dry_run=True)
    x, y, z = ctx.alloc(64), ctx.alloc(64), ctx.alloc(64)
    D.dag_region_begin(ctx.h, 7)
    t1 = ctx.kernel("spin", [(x, "c"), (y, "m")], ns=0)
    t2 = ctx.kernel("spin", [(y, "c"), (z, "m")], ns=0)
    D.dag_region_end(ctx.h)
    assert D.dag_region_info(ctx.h, 7) == (2, 1)
    t3 = D.dag_region_launch(ctx.h, 7)
    t4 = ctx.kernel("spin", [(z, "c")], ns=0)
    ops = [{"kind": "kernel", "args": [("x", "c"), ("y", "m")]},
           {"kind": "kernel", "args": [("y", "c"), ("z", "m")]},
           {"kind": "macro", "args": [("x", "c"), ("y", "m"), ("z", "m")]},
           {"kind": "kernel", "args": [("z", "c")]}]
    g = odag.build_dag(ops)
    name_of = {x: "x", y: "y", z: "z"}
    assert {(s, d, name_of[b], k) for s, d, b, k in ctx.edges()} == g.edges
    assert (t1, t2, t3, t4) == (1, 2, 3, 4)
    ctx.close()


# ---------------------------------------------------------------------------
# argument checks and error conventions
# ---------------------------------------------------------------------------
def _status(fn, *a, **k):
    try:
        fn(*a, **k)
    except D.DagError as e:
        return e.name
    return "DAG_OK"


def test_error_paths():
    ctx = D.Context(dry_run=True)
    x = ctx.alloc(4 * 100)
    r = ctx.alloc(4)
    p = ctx.alloc(400, D.DAG_PINNED_HOST)
    # unknown handle, bad mode, written argument passed as const
    assert _status(ctx.kernel, "vec_square", [(999, "m")], n=100) == "DAG_E_INVAL"
    assert _status(ctx.kernel, "vec_square", [(x, "c")], n=100) == "DAG_E_INVAL"
    # buffer too small for n, wrong arity, pinned host argument
    assert _status(ctx.kernel, "vec_square", [(x, "m")], n=101) == "DAG_E_INVAL"
    assert _status(ctx.kernel, "vec_sum_diff", [(x, "c"), (x, "c")], n=100) == "DAG_E_INVAL"
    assert _status(ctx.kernel, "vec_square", [(p, "m")], n=100) == "DAG_E_INVAL"
    assert _status(D.dag_submit_kernel, ctx.h, 77, None, []) == "DAG_E_NOTFOUND"
    # copies out of range
    assert _status(ctx.copy, x, p, 401) == "DAG_E_INVAL"
    assert _status(ctx.copy, x, x, 8, 0, 4) == "DAG_E_INVAL"
    # none of the failures consumed a task id
    t = ctx.kernel("vec_square", [(x, "m")], n=100)
    assert t == 1
    # aliasing registrations
    base, nbytes = ctx.ptr(x)
    assert _status(ctx.register, base + 16, 8) == "DAG_E_ALIAS"
    assert _status(ctx.register, base - 8, 16) == "DAG_E_ALIAS"
    ok = ctx.register(base + nbytes + (1 << 20), 8)
    assert ok > 0
    # host access / sync inside a region
    D.dag_region_begin(ctx.h, 1)
    assert _status(D.dag_host_read, ctx.h, r) == "DAG_E_BUSY"
    assert _status(ctx.sync) == "DAG_E_BUSY"
    assert _status(D.dag_region_begin, ctx.h, 2) == "DAG_E_BUSY"
    assert _status(D.dag_region_end, ctx.h) == "DAG_E_INVAL"  # empty region
    assert _status(D.dag_region_launch, ctx.h, 5) == "DAG_E_NOTFOUND"
    # released handles are invalid
    ctx.release(x)
    assert _status(ctx.kernel, "vec_square", [(x, "m")], n=100) == "DAG_E_INVAL"
    # launch configuration checks
    assert _status(ctx.set_launch, "vec_square", 96) == "DAG_E_INVAL"
    assert _status(ctx.set_launch, "spmv", 256, 0, 5) == "DAG_E_INVAL"
    ctx.set_launch("vec_square", 512, 64)
    assert ctx.get_launch("vec_square") == (512, 64, 0)
    ctx.close()


def test_recurring_region_replays_when_every_call_matches():
    """dag_region_run_*: the first HITS iteration is recorded, the next ones
    are replayed as one task each, chained through the vectors they write."""
    prog = W.hits_program(n=300, deg=5, iters=4, seed=7)
    ctx = D.Context(dry_run=True)
    b = runner.Bound(ctx, prog)
    before = ctx.stats().tasks  # the uploads
    res = b.run_recurring(1, 6)
    assert [r for _, r in res] == [False, True, True, True]
    assert res[0][0] == 0 and all(t > 0 for t, _ in res[1:])
    assert D.dag_region_info(ctx.h, 1)[0] == 6
    # one eager iteration, three replays, two host reads
    assert ctx.stats().tasks - before == 6 + 3 + 2
    # each replay depends on the previous one (both read and write a and h)
    edges = {(s, d) for s, d, _, _ in ctx.edges()}
    for prev, cur in zip(res[1:], res[2:]):
        assert (prev[0], cur[0]) in edges
    ctx.close()


def test_recurring_region_rerecords_on_a_difference():
    prog = W.hits_program(n=300, deg=5, iters=2, seed=7)
    ctx = D.Context(dry_run=True)
    b = runner.Bound(ctx, prog)
    b.run_recurring(1, 6, host_reads=False)
    before = ctx.stats().tasks
    # a different launch configuration of sumsq makes the third call differ
    ctx.set_launch("sumsq", 512, 256, 0)
    D.dag_region_run_begin(ctx.h, 1)
    ids = D.dag_submit_batch(ctx.h, b._sub(list(range(6))))
    t, rep = D.dag_region_run_end(ctx.h)
    assert not rep and t == 0
    assert ids[:2] == [0, 0] and all(i > 0 for i in ids[2:])  # matched prefix, then eager
    # the first two calls were run eagerly once the third differed: six new tasks in all
    assert ctx.stats().tasks - before == 6
    # the new sequence replays next time
    D.dag_region_run_begin(ctx.h, 1)
    D.dag_submit_batch(ctx.h, b._sub(list(range(6))))
    t, rep = D.dag_region_run_end(ctx.h)
    assert rep and t > 0
    # only a prefix: recorded anew with four calls
    D.dag_region_run_begin(ctx.h, 1)
    D.dag_submit_batch(ctx.h, b._sub(list(range(4))))
    t, rep = D.dag_region_run_end(ctx.h)
    assert not rep and D.dag_region_info(ctx.h, 1)[0] == 4
    # host access, sync, region launch and drop are refused inside
    D.dag_region_run_begin(ctx.h, 1)
    assert _status(ctx.sync) == "DAG_E_BUSY"
    assert _status(D.dag_region_launch, ctx.h, 1) == "DAG_E_BUSY"
    assert _status(D.dag_region_drop, ctx.h, 1) == "DAG_E_BUSY"
    assert _status(D.dag_region_run_begin, ctx.h, 2) == "DAG_E_BUSY"
    D.dag_submit_batch(ctx.h, b._sub(list(range(4))))
    assert D.dag_region_run_end(ctx.h)[1]
    assert _status(D.dag_region_run_end, ctx.h) == "DAG_E_BUSY"
    ctx.close()


def test_bad_config_rejected():
    with pytest.raises(D.DagError):
        D.Context(dry_run=True, max_streams=65)
    with pytest.raises(D.DagError):
        D.Context(dry_run=True, policy=7)
    with pytest.raises(D.DagError):
        D.Context(dry_run=True, own_queues=2)
    with pytest.raises(D.DagError) as e:
        D.Context(dry_run=True, own_queues=1)
    assert e.value.name == "DAG_E_UNSUPPORTED"
    with pytest.raises(D.DagError):
        D.Context(dry_run=True, copy_lanes=5)
    with pytest.raises(D.DagError) as e:
        D.Context(dry_run=True, wait_mode=2)
    assert e.value.name == "DAG_E_INVAL"
    for mode in (D.DAG_WAIT_SIGNALS, D.DAG_WAIT_EVENTS):  # both accepted; dry runs place no wait of either kind
        with D.Context(dry_run=True, wait_mode=mode) as ctx:
            assert ctx.stats().signals == 0


def test_serial_policy_computes_no_dependencies():
    ctx = D.Context(dry_run=True, policy=D.DAG_SERIAL_SYNC)
    x = ctx.alloc(64)
    ctx.kernel("spin", [(x, "m")], ns=0)
    ctx.kernel("spin", [(x, "m")], ns=0)
    assert ctx.edges() == []
    assert ctx.info(1).stream == ctx.info(2).stream == 0
    ctx.close()


@pytest.mark.parametrize("lanes", [2, 3])
def test_copy_lanes_rotate(lanes):
    prog = W.bs_program(n=64, tasks=10)
    g = odag.build_dag(prog.ops)
    ctx = D.Context(dry_run=True, max_streams=8, copy_streams=0, copy_lanes=lanes)
    b = runner.Bound(ctx, prog, upload=False)
    b.run()
    assert b.edges() == g.edges
    st, wt = b.streams(), b.waits()
    assert dagcases.uncovered_edges(g.edges, st, wt) == []
    h2d = [p for p, o in enumerate(prog.ops, 1) if o["kind"] == "copy" and o["src"].startswith("S")]
    d2h = [p for p, o in enumerate(prog.ops, 1) if o["kind"] == "copy" and o["dst"].startswith("C")]
    for copies in (h2d, d2h):
        seq = [st[p] for p in copies]
        assert len(set(seq)) == lanes and all(seq[i] == seq[i % lanes] for i in range(len(seq)))
    assert not set(st[p] for p in h2d) & set(st[p] for p in d2h)
    ctx.close()


@pytest.mark.parametrize("pool", [1, 4, 8])
def test_copy_lanes(pool):
    """Host<->device copies on one FIFO stream per direction: same edges as
    the oracle, every edge ordered by stream order + waits, copies of each
    direction on one lane in issue order, kernels never on a lane."""
    prog = W.bs_program(n=64, tasks=10)
    g = odag.build_dag(prog.ops)
    ctx = D.Context(dry_run=True, max_streams=pool, copy_streams=0)
    b = runner.Bound(ctx, prog, upload=False)
    b.run()
    assert b.edges() == g.edges
    st = b.streams()
    wt = b.waits()
    assert dagcases.uncovered_edges(g.edges, st, wt) == []
    h2d = [p for p, o in enumerate(prog.ops, 1) if o["kind"] == "copy" and o["src"].startswith("S")]
    d2h = [p for p, o in enumerate(prog.ops, 1) if o["kind"] == "copy" and o["dst"].startswith("C")]
    ker = [p for p, o in enumerate(prog.ops, 1) if o["kind"] == "kernel"]
    assert len({st[p] for p in h2d}) == 1 and len({st[p] for p in d2h}) == 1
    lanes = {st[h2d[0]], st[d2h[0]]}
    assert len(lanes) == 2 and not lanes & {st[p] for p in ker}
    assert len({st[p] for p in ker}) == min(pool, 10)
    ctx.close()


@pytest.mark.parametrize("seed", range(60))
def test_copy_lanes_random(seed):
    rnd = random.Random(77 + seed)
    ctx = D.Context(dry_run=True, max_streams=rnd.choice([1, 2, 4]), copy_streams=0)
    names = ["d%d" % i for i in range(4)] + ["h%d" % i for i in range(3)]
    h = {n: ctx.alloc(256, D.DAG_PINNED_HOST if n[0] == "h" else D.DAG_DEVICE) for n in names}
    ops = []
    for _ in range(rnd.randint(5, 40)):
        r = rnd.random()
        if r < 0.3:
            a, c = rnd.sample(names, 2)
            ops.append({"kind": "copy", "dst": a, "src": c, "bytes": 16})
            ctx.copy(h[a], h[c], 16)
        elif r < 0.4:
            bname = rnd.choice(names)
            ops.append({"kind": "host_read", "buf": bname})
            D.dag_host_read(ctx.h, h[bname])
        else:
            args = [(rnd.choice(names[:4]), rnd.choice("cm")) for _ in range(rnd.randint(1, 3))]
            ops.append({"kind": "kernel", "kernel": "spin", "params": {}, "args": args})
            ctx.kernel("spin", [(h[x], m) for x, m in args], ns=0)
    g = odag.build_dag(ops)
    name_of = {v: k for k, v in h.items()}
    assert {(s, d, name_of[bb], k) for s, d, bb, k in ctx.edges()} == g.edges
    st = {i: ctx.info(i).stream for i in range(1, len(ops) + 1) if ctx.info(i).stream >= 0}
    wt = {i: ctx.waits(i) for i in st}
    assert dagcases.uncovered_edges(g.edges, st, wt) == []
    ctx.close()


def test_injected_launch_failure_poisons_the_context(monkeypatch):
    monkeypatch.setenv("DAGRT_FAULT_LAUNCH", "3")
    ctx = D.Context(dry_run=True)
    monkeypatch.delenv("DAGRT_FAULT_LAUNCH")
    x = ctx.alloc(64)
    ctx.kernel("spin", [(x, "m")], ns=0)
    ctx.kernel("spin", [(x, "m")], ns=0)
    with pytest.raises(D.DagError) as e:
        ctx.kernel("spin", [(x, "m")], ns=0)
    assert e.value.name == "DAG_E_HIP" and "injected" in str(e.value)
    for call in (lambda: ctx.kernel("spin", [(x, "m")], ns=0), ctx.sync, lambda: ctx.alloc(64),
                 lambda: D.dag_host_read(ctx.h, x)):
        with pytest.raises(D.DagError) as e:
            call()
        assert e.value.name == "DAG_E_POISONED"
    # introspection still works on a poisoned context
    assert len(ctx.edges()) == 2 and ctx.stats().tasks == 3
    ctx.close()
    # a fresh context is unaffected
    ctx2 = D.Context(dry_run=True)
    y = ctx2.alloc(64)
    for _ in range(4):
        ctx2.kernel("spin", [(y, "m")], ns=0)
    ctx2.close()


def test_ml_kernel_argument_checks():
    """The ML kernels' sizes are validated on the host: class count 1..16,
    the naive Bayes table within its LDS capacity, the ridge weights within
    theirs, every buffer large enough, reserved zero."""
    ctx = D.Context(dry_run=True)
    big = ctx.alloc(1 << 22)
    b2 = ctx.alloc(1 << 22)
    out = ctx.alloc(1 << 22)
    lab = ctx.alloc(1 << 22)

    def nb(**p):
        q = dict(n=1000, features=200, classes=10, categories=16)
        q.update(p)
        return _status(ctx.kernel, "nb_proba", [(big, "c"), (b2, "c"), (b2, "c"), (out, "m")], **q)

    def ridge(**p):
        q = dict(n=1000, features=200, classes=10)
        q.update(p)
        return _status(ctx.kernel, "ridge_proba", [(big, "c"), (b2, "c"), (b2, "c"), (b2, "c"), (b2, "c"),
                                                   (out, "m")], **q)

    assert nb() == "DAG_OK" and ridge() == "DAG_OK"
    assert nb(classes=0) == "DAG_E_INVAL" and nb(classes=17) == "DAG_E_INVAL"
    assert nb(features=0) == "DAG_E_INVAL" and nb(categories=0) == "DAG_E_INVAL"
    assert nb(features=128, classes=16, categories=16) == "DAG_OK"          # 32768 table entries
    assert nb(features=129, classes=16, categories=16) == "DAG_E_INVAL"
    assert nb(n=6000) == "DAG_E_INVAL"                                       # X too small
    assert ridge(features=744, classes=10) == "DAG_OK"                       # 744 * 11 = 8184 <= 8192
    assert ridge(features=745, classes=10) == "DAG_E_INVAL"
    assert ridge(classes=17) == "DAG_E_INVAL" and ridge(n=6000) == "DAG_E_INVAL"
    assert _status(ctx.kernel, "ensemble", [(big, "c"), (b2, "c"), (out, "m"), (lab, "m")],
                   n=1000, features=1, classes=10) == "DAG_OK"
    assert _status(ctx.kernel, "ensemble", [(big, "c"), (b2, "c"), (out, "m"), (lab, "m")],
                   n=1 << 20, features=1, classes=10) == "DAG_E_INVAL"
    # written arguments passed as const are rejected
    assert _status(ctx.kernel, "ensemble", [(big, "c"), (b2, "c"), (out, "c"), (lab, "m")],
                   n=10, features=1, classes=10) == "DAG_E_INVAL"
    ctx.close()


@pytest.mark.parametrize("name", ["vec", "bs", "img", "hits", "ml", "dl"])
def test_hand_written_schedules_order_every_dependency(name):
    """Each workload's hand-written schedule passes the library's check
    against the inferred dependencies (schedule-only context)."""
    from paper_2012_09646_amd import handwritten as H
    small = {"vec": lambda: W.vec_program(n=1024), "bs": lambda: W.bs_program(n=1024, tasks=10),
             "img": lambda: W.img_program(side=64), "hits": lambda: W.hits_program(n=256, deg=4, iters=3),
             "ml": lambda: W.ml_program(n=100, features=8, classes=3, categories=4),
             "dl": lambda: W.dl_program(side=16, channels=(4, 4), embed=3)}
    prog = small[name]()
    ctx = D.Context(dry_run=True)
    b = runner.Bound(ctx, prog)
    if name == "hits":
        b.record(7, 0, H.HITS_CALLS_PER_ITERATION)
    else:
        b.record(7)
    H.install(ctx, 7, prog)
    n, ns = D.dag_region_info(ctx.h, 7)
    assert ns == max(s for s, _ in H.schedule(prog)) + 1
    ctx.close()


def test_hand_written_schedule_missing_a_wait_is_refused():
    ctx = D.Context(dry_run=True)
    prog = W.vec_program(n=1024)
    b = runner.Bound(ctx, prog)
    b.record(3)
    with pytest.raises(D.DagError) as e:        # the sum on stream 0 without waiting for y^2 on stream 1
        D.dag_region_set_schedule(ctx.h, 3, [(0, []), (1, []), (0, [])])
    assert e.value.name == "DAG_E_INVAL" and "call 2" in str(e.value)
    with pytest.raises(D.DagError):              # a wait on a later call
        D.dag_region_set_schedule(ctx.h, 3, [(0, [1]), (1, []), (0, [1])])
    with pytest.raises(D.DagError):              # wrong length
        D.dag_region_set_schedule(ctx.h, 3, [(0, []), (1, [])])
    with pytest.raises(D.DagError):              # stream out of range
        D.dag_region_set_schedule(ctx.h, 3, [(0, []), (64, []), (0, [1])])
    D.dag_region_set_schedule(ctx.h, 3, [(0, []), (0, []), (0, [])])   # one stream: program order suffices
    assert D.dag_region_info(ctx.h, 3) == (3, 1)
    D.dag_region_set_schedule(ctx.h, 3, [(0, []), (1, []), (2, [0, 1])])
    assert D.dag_region_info(ctx.h, 3) == (3, 3)
    ctx.close()


def test_dl_kernel_argument_checks():
    ctx = D.Context(dry_run=True)
    big = ctx.alloc(1 << 22)
    out = ctx.alloc(1 << 22)

    def conv(**p):
        q = dict(cin=2, cout=8, h=64, w=64)
        q.update(p)
        return _status(ctx.kernel, "conv3x3_relu_pool", [(big, "c"), (big, "c"), (big, "c"), (out, "m")], **q)

    assert conv() == "DAG_OK"
    assert conv(h=63) == "DAG_E_INVAL" and conv(w=0) == "DAG_E_INVAL" and conv(cin=0) == "DAG_E_INVAL"
    assert conv(cin=64, cout=64, h=512, w=512) == "DAG_E_INVAL"          # x and y too small
    assert _status(ctx.kernel, "dense", [(big, "c"), (big, "c"), (big, "c"), (out, "m")], n=1000, m=16) == "DAG_OK"
    assert _status(ctx.kernel, "dense", [(big, "c"), (big, "c"), (big, "c"), (out, "m")], n=1000, m=17) == "DAG_E_INVAL"
    assert _status(ctx.kernel, "dense", [(big, "c"), (big, "c"), (big, "c"), (out, "m")],
                   n=1 << 20, m=16) == "DAG_E_INVAL"                     # W too small
    assert _status(ctx.kernel, "siamese_combine", [(big, "c"), (big, "c"), (big, "c"), (big, "c"), (out, "m")],
                   m=32) == "DAG_OK"
    assert _status(ctx.kernel, "siamese_combine", [(big, "c"), (big, "c"), (big, "c"), (big, "c"), (out, "m")],
                   m=33) == "DAG_E_INVAL"
    assert _status(ctx.set_launch, "conv3x3_relu_pool", 128) == "DAG_E_INVAL"
    assert _status(ctx.set_launch, "conv3x3_relu_pool", 256, 0, 1) == "DAG_OK"
    assert _status(ctx.set_launch, "conv3x3_relu_pool", 256, 0, 2) == "DAG_OK"
    assert _status(ctx.set_launch, "conv3x3_relu_pool", 256, 0, 3) == "DAG_OK"
    assert _status(ctx.set_launch, "conv3x3_relu_pool", 256, 0, 4) == "DAG_OK"
    assert _status(ctx.set_launch, "conv3x3_relu_pool", 256, 0, 5) == "DAG_E_INVAL"
    assert _status(ctx.set_launch, "dense", 256, 1024, 2) == "DAG_OK"
    assert _status(ctx.set_launch, "dense", 256, 1024, 4) == "DAG_OK"
    assert _status(ctx.set_launch, "dense", 256, 1024, 5) == "DAG_E_INVAL"
    assert _status(ctx.set_launch, "conv3x3_relu_pool", 256, 64, 1) == "DAG_E_INVAL"
    assert _status(ctx.set_launch, "siamese_combine", 128) == "DAG_E_INVAL"
    ctx.close()


def test_history_is_compacted_once_everything_is_retired():
    """A context that has run more than 65,536 tasks drops the per-task
    records at the next point where every task is retired: ids stay
    monotonic, the totals in the statistics keep counting, the dropped ids
    are unknown to the introspection calls, and the DAG of a program run
    afterwards is still the oracle's edge for edge."""
    prog = W.vec_program(n=1024, seed=0)
    ctx = D.Context(dry_run=True)
    b = runner.Bound(ctx, prog)
    st0 = ctx.stats()  # the uploads are host writes
    runs = (1 << 16) // len(prog.ops) + 2
    for _ in range(runs):
        b.run()
    st = ctx.stats()
    assert st.tasks - st0.tasks == runs * len(prog.ops)
    assert st.edges - st0.edges == runs * 3 and st.vertices - st0.vertices == runs * len(prog.ops)
    assert _status(ctx.info, st0.tasks + 5) == "DAG_E_INVAL"  # compacted
    b.run()
    g = odag.build_dag(prog.ops)
    assert b.edges() == g.edges
    assert ctx.stats().tasks - st0.tasks == (runs + 1) * len(prog.ops)
    ctx.close()
