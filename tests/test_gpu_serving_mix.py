"""Serving parity at the benchmark's configuration (see serving_mix_check.py):
the 20 full-size request shapes of the mix on the benchmark's server, each
result bit-identical in a batch session, an online session fed by a producer
thread and a serial session, and equal to the oracle."""

import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.timeout(600)
def test_mix_shapes_alone_online_and_mixed_equal_the_oracle():
    print("[gpu] serving mix at the benchmark's 20 shapes (child process, GPU_MAX_HW_QUEUES=8)", flush=True)
    env = dict(os.environ, GPU_MAX_HW_QUEUES="8")
    r = subprocess.run([sys.executable, "-u", os.path.join(HERE, "serving_mix_check.py"), "3"], env=env,
                       capture_output=True, text=True, timeout=560)
    print(r.stdout[-4000:], r.stderr[-3000:], flush=True)
    assert r.returncode == 0
