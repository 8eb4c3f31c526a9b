"""Pins of the oracle's DAG and stream-policy replay (CPU only)."""

import random

import pytest

import dagcases
from oracle import dag as odag
from paper_2012_09646_amd import workloads as W

CASES = dagcases.load_cases()


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_golden_case(case):
    g = odag.build_dag(case["ops"])
    assert g.edges == case["edges"]
    st, wt = odag.replay_streams(case["ops"], g, case["max_streams"])
    n = len(case["ops"])
    assert [st.get(i) for i in range(1, n + 1)] == case["streams"]
    assert [wt.get(i, []) for i in range(1, n + 1)] == case["waits"]


def _edges_by_iteration(g, lo, hi):
    return sorted((s, d) for (s, d) in g.pair_edges() if lo <= d <= hi)


def test_hits_program_edges_and_streams():
    # Two HITS iterations written out by hand from the task list:
    # 1 at=A^T h, 2 ht=A a, 3 sa=|at|^2, 4 sh=|ht|^2, 5 a=at/sqrt(sa), 6 h=ht/sqrt(sh)
    prog = W.hits_program(n=8, deg=2, iters=10, graph=W.hits_graph(8, 2, seed=1))
    g = odag.build_dag(prog.ops)
    it1 = [(1, 3), (2, 4), (1, 5), (3, 5), (2, 5), (2, 6), (4, 6), (1, 6)]
    it2 = [(6, 7), (3, 7), (5, 7), (5, 8), (4, 8), (6, 8), (7, 9), (5, 9),
           (8, 10), (6, 10), (7, 11), (9, 11), (8, 11), (8, 12), (10, 12), (7, 12)]
    assert _edges_by_iteration(g, 1, 6) == sorted(it1)
    assert _edges_by_iteration(g, 7, 12) == sorted(it2)
    for it in range(2, 10):
        shift = 6 * (it - 1)
        assert _edges_by_iteration(g, 7 + shift, 12 + shift) == sorted((s + shift, d + shift) for s, d in it2)
    pairs = g.pair_edges()
    assert len([p for p in pairs if p[1] <= 60]) == 152
    assert (59, 61) in pairs and (60, 62) in pairs and len(pairs) == 154
    st, wt = odag.replay_streams(prog.ops, g, 8)
    assert [st[i] for i in range(1, 61)] == [0, 1] * 30
    assert wt[5] == [2] and wt[6] == [1]
    for it in range(1, 10):
        b = 6 * it
        assert (wt[b + 1], wt[b + 2], wt[b + 3], wt[b + 4], wt[b + 5], wt[b + 6]) == \
            ([b], [b - 1], [], [], [b + 2], [b + 1])


def test_img_program_edges_and_streams():
    prog = W.img_program(side=8)
    g = odag.build_dag(prog.ops)
    pairs = g.pair_edges()
    # blur_k(1..3) -> sobel_k(4..6) -> minmax_k(7..9); norm_k(10..12) <- sobel_k, minmax_k;
    # combine(13) <- blur_k, norm_k; host read(14) <- combine
    exp = [(1, 4), (2, 5), (3, 6), (4, 7), (5, 8), (6, 9), (4, 10), (7, 10), (5, 11), (8, 11),
           (6, 12), (9, 12), (1, 13), (2, 13), (3, 13), (10, 13), (11, 13), (12, 13), (13, 14)]
    assert pairs == sorted(exp)
    st, wt = odag.replay_streams(prog.ops, g, 8)
    assert [st[i] for i in range(1, 14)] == [0, 1, 2] * 4 + [0]
    assert wt[13] == [11, 12]
    assert all(wt[i] == [] for i in range(1, 13))


def test_vec_program():
    prog = W.vec_program(n=16)
    g = odag.build_dag(prog.ops)
    assert g.pair_edges() == [(1, 3), (2, 3), (3, 4)]
    st, wt = odag.replay_streams(prog.ops, g, 8)
    assert (st[1], st[2], st[3], wt[3]) == (0, 1, 0, [2])
    assert set(g.retired_by) == {1, 2, 3}


@pytest.mark.parametrize("pool", [1, 2, 3, 4, 10, 16])
def test_bs_program_streams(pool):
    prog = W.bs_program(n=4, tasks=10)
    g = odag.build_dag(prog.ops)
    # copy in -> price -> copy out per task; host reads wait on the copy out
    exp = []
    for i in range(10):
        a, b, c = 3 * i + 1, 3 * i + 2, 3 * i + 3
        exp += [(a, b), (b, c), (c, 31 + i)]
    assert g.pair_edges() == sorted(exp)
    st, wt = odag.replay_streams(prog.ops, g, pool)
    for i in range(10):
        assert st[3 * i + 1] == st[3 * i + 2] == st[3 * i + 3] == i % pool
    assert all(not w for w in wt.values())


# ---------------------------------------------------------------------------
# Invariants on random programs
# ---------------------------------------------------------------------------
def random_program(rnd, n_ops, n_bufs):
    bufs = ["b%d" % i for i in range(n_bufs)]
    ops = []
    for _ in range(n_ops):
        r = rnd.random()
        if r < 0.1:
            ops.append({"kind": "host_read", "buf": rnd.choice(bufs)})
        elif r < 0.15:
            ops.append({"kind": "host_write", "buf": rnd.choice(bufs)})
        elif r < 0.17:
            ops.append({"kind": "sync"})
        else:
            k = rnd.randint(1, 4)
            args = [(rnd.choice(bufs), rnd.choice("cm")) for _ in range(k)]
            ops.append({"kind": "kernel", "kernel": "spin", "params": {}, "args": args})
    return ops


def _reach(parents, src, dst):
    stack, seen = [dst], set()
    while stack:
        t = stack.pop()
        if t == src:
            return True
        if t not in seen:
            seen.add(t)
            stack.extend(parents.get(t, ()))
    return False


@pytest.mark.parametrize("seed", range(40))
def test_dag_invariants(seed):
    rnd = random.Random(seed)
    ops = random_program(rnd, rnd.randint(5, 40), rnd.randint(1, 5))
    g = odag.build_dag(ops)
    acc = [None] + [odag.accesses(o) for o in ops]
    for (s, d, b, k) in g.edges:
        assert s < d
        assert ops[s - 1]["kind"] == "kernel"
        a_s, a_d = acc[s][b], acc[d][b]
        assert "W" in (a_s, a_d)
        assert k == {("W", "R"): 0, ("R", "W"): 1, ("W", "W"): 2}[(a_s, a_d)]
    # every conflict between a call and an earlier call still active is ordered
    # through a path of edges
    for j in range(1, len(ops) + 1):
        for i in range(1, j):
            if ops[i - 1]["kind"] != "kernel":
                continue
            if g.retired_by.get(i, len(ops) + 1) < j:
                continue
            for b, a_j in acc[j].items():
                a_i = acc[i].get(b)
                if a_i and "W" in (a_i, a_j):
                    assert _reach(g.parents, i, j), (i, j, b)
    # the event waits plus stream order cover every edge between GPU calls
    for pool in (1, 2, 3, 8):
        st, wt = odag.replay_streams(ops, g, pool)
        hb = {}
        last = {}
        for j in range(1, len(ops) + 1):
            if j not in st:
                continue
            hb[j] = ([last[st[j]]] if st[j] in last else []) + wt[j]
            last[st[j]] = j
            assert set(wt[j]) <= set(g.parents[j])
        for (s, d, b, k) in g.edges:
            if d in st:
                assert _reach(hb, s, d), (pool, s, d)
