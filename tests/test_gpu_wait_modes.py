"""Waits between streams in both wait modes: device-side polls of completion
signals (DAG_WAIT_SIGNALS, the default) and HIP events (DAG_WAIT_EVENTS).
The same programs give the oracle's outputs and edges in both modes; in
signal mode the waits on tasks that ran on the CUs are polls, in event mode
none are; a slow producer holds back its consumer on another stream; and a
poll that gives up (its bound lowered from the host) poisons the context at
the next host wait instead of letting a wrong result through."""

import pytest

import gpu_util as G
from oracle import dag as odag
from paper_2012_09646_amd import dagrt as D
from paper_2012_09646_amd import runner
from paper_2012_09646_amd import workloads as W

pytestmark = pytest.mark.gpu

MODES = [D.DAG_WAIT_SIGNALS, D.DAG_WAIT_EVENTS]

# Small ragged programs; the Black-Scholes one runs its copies on the copy
# lanes, host->device by SDMA (events) and device->host by the copy kernel
# (signals), so both kinds of wait meet in one DAG.
PROGRAMS = {
    "vec": (lambda: W.vec_program(n=(1 << 20) + 3, seed=21), {}),
    "bs": (lambda: W.bs_program(n=(1 << 18) + 5, tasks=4, seed=22), dict(copy_streams=0, copy_engine=2)),
    "img": (lambda: W.img_program(side=257, height=131, seed=23), {}),
    "hits": (lambda: W.hits_program(n=(1 << 13) + 7, iters=4, seed=24), {}),
    "ml": (lambda: W.ml_program(n=3001, seed=25), {}),
    "dl": (lambda: W.dl_program(side=64, seed=26), {}),
}


def banner(s):
    print("[wait] " + s, flush=True)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("name", sorted(PROGRAMS))
def test_programs_in_both_modes(name, mode):
    banner("%s mode %d" % (name, mode))
    make, kw = PROGRAMS[name]
    prog = make()
    ref = G.oracle_run(prog)
    g = odag.build_dag(prog.ops)
    ctx, b, outs = G.gpu_run(prog, max_streams=8, wait_mode=mode, **kw)
    try:
        assert b.edges() == g.edges
        for out in prog.outputs:
            G.assert_close(prog, out, outs[out], ref[out])
        st = ctx.stats()
        if mode == D.DAG_WAIT_EVENTS:
            assert st.signals == 0 and st.signal_waits == 0
        else:
            # every signal poll had its value raised first, by at most one raise per task on the CUs
            gpu_tasks = sum(1 for o in prog.ops if o["kind"] in ("kernel", "copy"))
            sdma = sum(1 for o in prog.ops if o["kind"] == "copy" and
                       prog.bufs[o["src"]].loc == "host")  # host->device copies by SDMA
            assert st.signals <= gpu_tasks - sdma
            assert st.signal_waits <= st.waits
            assert (st.signals > 0) == (st.signal_waits > 0)
            if name in ("img", "hits"):  # every cross-stream parent is a kernel
                assert st.waits > 0 and st.signal_waits == st.waits
            if name == "bs":  # copies by SDMA (events) and by the copy kernel (signals)
                assert 0 < st.signal_waits < st.waits
    finally:
        ctx.close()


def _chain_program(spin_ns, n=(1 << 16) + 9, seed=27):
    """y <- y^2 on one stream; a delay then x <- x^2 on a second; r = sum(x - y)
    joins them on the first stream (its lowest parent's), behind a wait for
    the second."""
    base = W.vec_program(n=n, seed=seed)
    ops = [W.K("vec_square", [("y", "m")], n=n),
           W.K("spin", [("x", "m")], ns=spin_ns),
           W.K("vec_square", [("x", "m")], n=n),
           W.K("vec_sum_diff", [("x", "c"), ("y", "c"), ("r", "m")], n=n),
           W.HR("r")]
    return W.Program("chain", base.bufs, ops, base.outputs, "r")


@pytest.mark.parametrize("mode", MODES)
def test_slow_producer_holds_its_consumer(mode):
    banner("slow producer mode %d" % mode)
    prog = _chain_program(20_000_000)
    ref = G.oracle_run(prog)
    with D.Context(max_streams=4, wait_mode=mode) as ctx:
        b = runner.Bound(ctx, prog)
        b.run()
        st = b.streams()
        assert st[1] == st[4] != st[2] == st[3]
        for out in prog.outputs:
            G.assert_close(prog, out, b.read(out), ref[out])
        s = ctx.stats()
        assert s.waits == 1 and s.signal_waits == (1 if mode == D.DAG_WAIT_SIGNALS else 0)


def test_a_wait_that_gives_up_poisons_the_context(monkeypatch):
    """The poll's bound is lowered to 1 ms from the host while its producer
    runs 100 ms: the poll exits, and the host read that follows reports the
    failure (every kernel still ends normally)."""
    banner("poll bound 1 ms")
    monkeypatch.setenv("DAGRT_SIGNAL_TIMEOUT_MS", "1")
    prog = _chain_program(100_000_000)
    ctx = D.Context(max_streams=4)
    monkeypatch.delenv("DAGRT_SIGNAL_TIMEOUT_MS")
    try:
        b = runner.Bound(ctx, prog, upload=True)
        with pytest.raises(D.DagError) as ei:
            b.run()
        assert "gave up" in str(ei.value)
        with pytest.raises(D.DagError):
            ctx.sync()
    finally:
        ctx.close()


def test_one_stream_pool_raises_no_signal():
    """With one pool stream and no copy lane nothing waits across streams, so
    no signal is ever raised (the tasks' values stay pending)."""
    banner("one-stream pool")
    for prog in (W.vec_program(n=(1 << 18) + 1, seed=29), W.ml_program(n=2049, seed=30)):
        ref = G.oracle_run(prog)
        ctx, b, outs = G.gpu_run(prog, max_streams=1)
        try:
            for out in prog.outputs:
                G.assert_close(prog, out, outs[out], ref[out])
            st = ctx.stats()
            assert st.signals == 0 and st.waits == 0 and st.streams == 1
        finally:
            ctx.close()


def test_wide_join_waits_for_ten_streams():
    """A task that joins ten branches, each on its own stream, places nine
    waits: more than one poll kernel holds (eight), so two are queued.  The
    timing events show it starting after every branch ended (each branch is
    a delay of a different length, then x_i <- x_i^2), and the outputs equal
    the oracle's."""
    banner("ten-way join")
    n = (1 << 16) + 3
    bufs = {"x%d" % i: W.Buf(4 * n, init=W.uniform_f32(40 + i, n)) for i in range(10)}
    bufs.update(z=W.Buf(4), r=W.Buf(4))
    ops = []
    for i in range(10):
        ops += [W.K("spin", [("x%d" % i, "m")], ns=100_000 + 40_000 * ((7 * i) % 10)),
                W.K("vec_square", [("x%d" % i, "m")], n=n)]
    ops.append(W.K("spin", [("x%d" % i, "c") for i in range(10)] + [("z", "m")], ns=0))
    ops.append(W.K("vec_sum_diff", [("x0", "c"), ("x9", "c"), ("r", "m")], n=n))
    ops.append(W.HR("r"))
    prog = W.Program("join10", bufs, ops, ["x%d" % i for i in range(10)] + ["r"], "r")
    ref = G.oracle_run(prog)
    with D.Context(max_streams=16, trace=1) as ctx:
        b = runner.Bound(ctx, prog)
        D.dag_trace_reset(ctx.h)
        b.run()
        join = 21  # position of the joining task
        info = {p: ctx.info(b.base + p) for p in range(1, len(ops) + 1)}
        assert info[join].nwaits == 9
        assert len({info[2 * i + 2].stream for i in range(10)}) == 10
        last_branch_end = max(info[2 * i + 2].t_end_ms for i in range(10))
        assert info[join].t_start_ms >= last_branch_end - 1e-6
        assert ctx.stats().signal_waits >= 9
        for out in prog.outputs:
            G.assert_close(prog, out, b.read(out), ref[out])


@pytest.mark.parametrize("mode", MODES)
def test_a_consumer_on_another_stream_waits_for_a_replay(mode):
    """A recorded multi-stream replay (graph mode 1) of the vector diamond,
    then y <- y^2 (on the replay's stream: the replay is its tail) and x <-
    x^2, which joins another stream and must wait for the replay there. A
    replay whose tasks all ran on the CUs ends with a completion signal, so
    in signal mode that wait is a poll; the results equal the oracle's after
    every one of three rounds."""
    banner("consumer of a replay mode %d" % mode)
    n = (1 << 18) + 5
    base = W.vec_program(n=n, seed=31)
    # inputs in [0.9, 1): six squarings keep them normal
    base.bufs["x"] = W.Buf(4 * n, init=W.uniform_f32(31, n, 0.9, 1.0, stream=0))
    base.bufs["y"] = W.Buf(4 * n, init=W.uniform_f32(31, n, 0.9, 1.0, stream=1))
    region = [o for o in base.ops if o["kind"] == "kernel"]
    after = [W.K("vec_square", [("y", "m")], n=n), W.K("vec_square", [("x", "m")], n=n)]
    rounds = 3
    ref = G.oracle_run(W.Program("vec_rounds", base.bufs, (region + after) * rounds, base.outputs))
    prog = W.Program("vec_region", base.bufs, region + after, base.outputs)
    with D.Context(max_streams=4, graph_mode=1, wait_mode=mode) as ctx:
        b = runner.Bound(ctx, prog)
        b.record(1, 0, len(region))  # the region runs once while it is recorded
        tail = b._sub(list(range(len(region), len(region) + 2)))
        for k in range(rounds):
            ids = D.dag_submit_batch(ctx.h, tail)
            if k + 1 < rounds:
                D.dag_region_launch(ctx.h, 1)
        info = {t: ctx.info(t) for t in ids}
        assert info[ids[1]].stream != info[ids[0]].stream and info[ids[1]].nwaits >= 1
        for out in prog.outputs:
            G.assert_close(prog, out, b.read(out), ref[out])
        st = ctx.stats()
        if mode == D.DAG_WAIT_SIGNALS:
            assert st.signal_waits >= 1
        else:
            assert st.signals == 0 and st.signal_waits == 0
