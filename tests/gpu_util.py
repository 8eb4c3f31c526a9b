"""Helpers of the GPU parity tests: run a program through the C ABI and
through the oracle, compare outputs at the stated tolerances."""

import numpy as np

from oracle import dag as odag
from oracle import run as orun
from paper_2012_09646_amd import dagrt as D
from paper_2012_09646_amd import runner
from paper_2012_09646_amd import workloads as W

RTOL = 1e-5  # fp32 outputs: |g - o| <= 1e-5 |o| (exact zeros must match)


def oracle_run(prog):
    arrays = W.initial_arrays(prog)
    orun.execute(prog.ops, arrays)
    return arrays


def gpu_run(prog, policy=D.DAG_PARALLEL_ASYNC, max_streams=8, batch=True, trace=0,
            graph_mode=0, outputs=None, copy_streams=1, own_queues=0, copy_engine=0, wait_mode=0):
    ctx = D.Context(policy=policy, max_streams=max_streams, trace=trace, graph_mode=graph_mode,
                    copy_streams=copy_streams, own_queues=own_queues, copy_engine=copy_engine,
                    wait_mode=wait_mode)
    b = runner.Bound(ctx, prog)
    if batch:
        b.run()
    else:
        b.run_calls()
    outs = {name: b.read(name) for name in (outputs or prog.outputs)}
    return ctx, b, outs


def kind_of(prog, name, _seen=None):
    """How a buffer is compared: 'exact' (bit-exact), 'f32', 'f64'.  A copy's
    destination is compared like its source (the Black-Scholes prices reach
    host memory by a copy)."""
    for op in prog.ops:
        if op["kind"] == "copy" and op["dst"] == name:
            seen = (_seen or set()) | {name}
            if op["src"] not in seen:
                return kind_of(prog, op["src"], seen)
        if op["kind"] != "kernel":
            continue
        for i, (b, m) in enumerate(op["args"]):
            if b != name or m != "m":
                continue
            k = op["kernel"]
            if k in ("vec_square", "minmax") or (k == "ensemble" and i == 3):
                return "exact"
            if k == "sumsq":
                return "f64"
            return "f32"
    return "exact"


def assert_close(prog, name, got, ref, rtol=RTOL):
    k = kind_of(prog, name)
    if k == "exact":
        assert np.array_equal(got, ref), "%s differs bitwise" % name
        return
    dt = np.float64 if k == "f64" else np.float32
    g = got.view(dt).astype(np.float64)
    o = ref.view(dt).astype(np.float64)
    tol = 1e-12 if k == "f64" else rtol
    nan_g, nan_o = np.isnan(g), np.isnan(o)
    assert np.array_equal(nan_g, nan_o), "%s: NaN at different places" % name
    g, o = g[~nan_o], o[~nan_o]
    with np.errstate(invalid="ignore"):
        bad = ~((g == o) | (np.abs(g - o) <= tol * np.abs(o)))
    if bad.any():
        i = int(np.argmax(bad))
        raise AssertionError("%s: %d of %d elements off; first at %d: gpu %r oracle %r" % (
            name, int(bad.sum()), bad.size, i, g[i], o[i]))


def check_program(prog, **kw):
    ref = oracle_run(prog)
    g = odag.build_dag(prog.ops)
    ctx, b, outs = gpu_run(prog, **kw)
    try:
        if kw.get("policy", D.DAG_PARALLEL_ASYNC) == D.DAG_PARALLEL_ASYNC:
            assert b.edges() == g.edges
            if kw.get("copy_streams", 1) == 1:
                st, wt = odag.replay_streams(prog.ops, g, kw.get("max_streams", 8))
                assert b.streams() == st
        for name in prog.outputs:
            assert_close(prog, name, outs[name], ref[name])
    finally:
        ctx.close()
    return outs
