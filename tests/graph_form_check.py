"""Run as a script (one process per GPU_MAX_HW_QUEUES setting, which HIP fixes
at start-up): the Black-Scholes fan-out recorded once and replayed, with every
result buffer cleared before each replay, so a host read that returned before
the replay finished would see zeros instead of prices.

Usage: python tests/graph_form_check.py GRAPH_MODE MAX_STREAMS N TASKS REPLAYS
Prints one line per replay; exits 1 on a mismatch with the oracle.
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

import gpu_util as G  # noqa: E402
from paper_2012_09646_amd import dagrt as D  # noqa: E402
from paper_2012_09646_amd import runner  # noqa: E402
from paper_2012_09646_amd import workloads as W  # noqa: E402


def main():
    gm, pool, n, tasks, replays = (int(v) for v in sys.argv[1:6])
    prog = W.bs_program(n=n, tasks=tasks, seed=17)
    ref = G.oracle_run(prog)
    ctx = D.Context(graph_mode=gm, max_streams=pool)
    b = runner.Bound(ctx, prog, read_bytes=4)
    b.record(1)
    ctx.sync()
    zeros = np.zeros(n, np.float32)
    ok = True
    for rep in range(replays):
        for name in prog.outputs:
            ctx.host_write(b.h[name], zeros)
        b.replay(1)  # then 4-byte host reads of every result: the program's sync points
        for name in prog.outputs:
            got = b.read(name)
            try:
                G.assert_close(prog, name, got, ref[name])
            except AssertionError as e:
                ok = False
                print("replay %d: %s" % (rep, e), flush=True)
        print("replay %d done (GPU_MAX_HW_QUEUES=%s)" % (rep, os.environ.get("GPU_MAX_HW_QUEUES")), flush=True)
    ctx.close()
    sys.exit(0 if ok else 1)


if __name__ == "__main__":
    main()
