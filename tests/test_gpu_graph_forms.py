"""Graph forms at the full Black-Scholes size under several hardware queue
counts: each configuration runs in a child process (GPU_MAX_HW_QUEUES is read
once when HIP starts), clears the results before every replay and checks them
against the oracle after the replay's host reads."""

import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("hw_queues", [4, 8])
@pytest.mark.parametrize("graph_mode,pool", [(0, 1), (0, 2), (0, 4), (1, 2)])
def test_replay_results_ready_at_host_read(hw_queues, graph_mode, pool):
    print("[gpu] graph form check hwq=%d graph_mode=%d pool=%d" % (hw_queues, graph_mode, pool), flush=True)
    env = dict(os.environ, GPU_MAX_HW_QUEUES=str(hw_queues))
    r = subprocess.run([sys.executable, os.path.join(HERE, "graph_form_check.py"), str(graph_mode), str(pool),
                        str(1 << 22), "10", "8"], env=env, capture_output=True, text=True, timeout=240)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0
