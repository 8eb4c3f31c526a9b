"""GPU parity of the DL workload (Siamese CNN): convolution layers, dense
embeddings and the combining layer against the oracle at 1e-5 relative, the
DAG edge for edge; launch shapes with ragged tiles, one or several output
channels per workgroup, grid-stride dense reductions repeated on one stream."""

import sys

import numpy as np
import pytest

import gpu_util as G
from oracle import dag as odag
from oracle import tasks as T
from paper_2012_09646_amd import dagrt as D
from paper_2012_09646_amd import runner
from paper_2012_09646_amd import workloads as W

pytestmark = pytest.mark.gpu


def banner(msg):
    print("[gpu] " + msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("side,channels,embed", [(64, (16, 32), 16), (36, (4, 6), 5), (4, (8, 8), 1),
                                                 (100, (3, 5), 7), (256, (16, 32), 16)])
def test_dl_pipeline(side, channels, embed):
    banner("dl side=%d channels=%s embed=%d" % (side, channels, embed))
    G.check_program(W.dl_program(side=side, seed=side, channels=channels, embed=embed))


@pytest.mark.parametrize("m", [16, 7])
@pytest.mark.parametrize("block,cap", [(256, 1024), (64, 3), (1024, 1), (512, 0)])
def test_dense_reduction_launch_shapes(block, cap, m):
    """Dense layer alone with several launch shapes, launched three times in
    a row on one stream (the ticket counter must be back to zero each time)."""
    banner("dense block=%d cap=%d m=%d" % (block, cap, m))
    g = np.random.default_rng(block + cap + m)
    n = 300007
    x = g.random(n, dtype=np.float32) - 0.5
    w = g.random((n, m), dtype=np.float32) - 0.5      # stored input-major
    b = g.random(m, dtype=np.float32)
    ref = T.dense(x, w.T, b)
    ctx = D.Context(max_streams=1)
    try:
        ctx.set_launch("dense", block, cap, 0)
        hx, hw, hb, hy = ctx.alloc(x.nbytes), ctx.alloc(w.nbytes), ctx.alloc(b.nbytes), ctx.alloc(4 * m)
        ctx.host_write(hx, x)
        ctx.host_write(hw, w)
        ctx.host_write(hb, b)
        for _ in range(3):
            ctx.kernel("dense", [(hx, "c"), (hw, "c"), (hb, "c"), (hy, "m")], n=n, m=m)
            y = np.zeros(m, np.float32)
            ctx.host_read(hy, y)
            assert np.all(np.abs(y.astype(np.float64) - ref) <= 1e-5 * np.abs(ref.astype(np.float64))), (y, ref)
    finally:
        ctx.close()


def test_dl_full_size():
    """The benchmark's shape: two 1024 x 1024 images, 16 and 32 channels, 16-wide embeddings."""
    banner("dl full size")
    prog = W.dl_program(side=1024, seed=6)
    G.check_program(prog)
