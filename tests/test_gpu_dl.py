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


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("m", [16, 7, 8, 4])
@pytest.mark.parametrize("block,cap,n", [(256, 1024, 300007), (64, 3, 300007), (1024, 1, 300007), (512, 0, 300007),
                                         (256, 256, 37), (128, 5, 64 * 13), (256, 7, 64 * 29 + 1)])
def test_dense_reduction_launch_shapes(block, cap, n, m, variant):
    """Dense layer alone with several launch shapes and variants (one input
    per lane; whole 1 KB weight loads per wave with 2 or 4 chunks in flight,
    which apply to 4, 8 or 16 outputs, the last block adding the partials or
    a second kernel), inputs that leave a partial 64-input chunk or none,
    launched three times in a row on one stream (the ticket counter must be
    back to zero each time)."""
    banner("dense block=%d cap=%d n=%d m=%d variant=%d" % (block, cap, n, m, variant))
    g = np.random.default_rng(block + cap + m + n)
    x = g.random(n, dtype=np.float32) - 0.5
    w = g.random((n, m), dtype=np.float32) - 0.5      # stored input-major
    b = g.random(m, dtype=np.float32)
    ref = T.dense(x, w.T, b)
    ctx = D.Context(max_streams=1)
    try:
        ctx.set_launch("dense", block, cap, variant)
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


@pytest.mark.parametrize("variant,scratch", [(0, 0), (1, 0), (2, 0), (2, 4096), (3, 4096)])
@pytest.mark.parametrize("cin,cout,h,w", [(1, 16, 64, 64), (16, 32, 66, 98), (3, 8, 34, 36), (2, 4, 2, 2),
                                          (5, 3, 40, 30), (17, 8, 50, 70), (4, 12, 96, 32)])
def test_conv_launch_variants(variant, scratch, cin, cout, h, w):
    """One convolution layer alone in each launch variant (one channel at a
    time; channels pipelined through a double-buffered tile; pipelined with
    fp64 weights read as scalars, which falls back to the second where the
    stream scratch of 4096 bytes cannot hold the weight copy; the matrix-core
    variant falls back to the second in that case too): ragged tiles,
    odd and even channel counts, 8, 4 or 1 output channels per workgroup.
    Every variant must agree with the others bit for bit (same FMA order)."""
    banner("conv variant=%d scratch=%d cin=%d cout=%d h=%d w=%d" % (variant, scratch, cin, cout, h, w))
    g = np.random.default_rng(cin * 1000 + cout + h + w)
    x = (g.random((cin, h, w), dtype=np.float32) - 0.3).astype(np.float32)
    wt = ((g.random((cout, cin, 3, 3), dtype=np.float32) - 0.5) / (3.0 * np.sqrt(cin))).astype(np.float32)
    b = ((g.random(cout, dtype=np.float32) - 0.5) * 0.1).astype(np.float32)
    ref = T.conv3x3_relu_pool(x, wt, b)
    outs = {}
    ctx = D.Context(max_streams=1, scratch_bytes=scratch)
    try:
        hx, hw_, hb = ctx.alloc(x.nbytes), ctx.alloc(wt.nbytes), ctx.alloc(b.nbytes)
        hy = ctx.alloc(4 * cout * (h // 2) * (w // 2))
        ctx.host_write(hx, x)
        ctx.host_write(hw_, wt)
        ctx.host_write(hb, b)
        for v in [variant] + [u for u in (0, 1, 2) if u != variant]:
            ctx.set_launch("conv3x3_relu_pool", 256, 0, v)
            ctx.kernel("conv3x3_relu_pool", [(hx, "c"), (hw_, "c"), (hb, "c"), (hy, "m")],
                       cin=cin, cout=cout, h=h, w=w)
            y = np.zeros((cout, h // 2, w // 2), np.float32)
            ctx.host_read(hy, y)
            outs[v] = y
    finally:
        ctx.close()
    y = outs[variant]
    r = ref.astype(np.float64)
    assert np.all(np.abs(y.astype(np.float64) - r) <= 1e-5 * np.abs(r)), np.max(np.abs(y - ref))
    for v in (0, 1, 2):
        assert np.array_equal(outs[v].view(np.uint32), y.view(np.uint32)), v


@pytest.mark.parametrize("cin,cout,h,w", [(16, 32, 66, 98), (4, 16, 34, 36), (8, 48, 50, 70), (16, 16, 2, 2),
                                          (12, 32, 96, 32), (32, 16, 40, 30), (28, 32, 18, 46), (16, 32, 512, 512),
                                          (3, 8, 34, 36), (16, 12, 20, 20)])
def test_conv_matrix_core_variant(cin, cout, h, w):
    """Variant 3, the implicit GEMM on the fp64 matrix cores (16 x 16 tiles
    of convolution outputs, 16 or 32 output channels per workgroup), against
    the oracle at 1e-5: ragged tiles, several channel counts, one and two
    channel blocks, launched twice in a row (equal bit for bit); variant 4
    (always one block of 16 channels) equal to it bit for bit.  Where the channel counts do not
    allow it (cin % 4 != 0 or cout % 16 != 0) variant 1 runs instead and the
    result equals variant 1's bit for bit."""
    banner("conv mfma cin=%d cout=%d h=%d w=%d" % (cin, cout, h, w))
    g = np.random.default_rng(cin * 7919 + cout * 31 + h + w)
    x = (g.random((cin, h, w), dtype=np.float32) - 0.3).astype(np.float32)
    wt = ((g.random((cout, cin, 3, 3), dtype=np.float32) - 0.5) / (3.0 * np.sqrt(cin))).astype(np.float32)
    b = ((g.random(cout, dtype=np.float32) - 0.5) * 0.1).astype(np.float32)
    ref = T.conv3x3_relu_pool(x, wt, b)
    outs = {}
    ctx = D.Context(max_streams=1)
    try:
        hx, hw_, hb = ctx.alloc(x.nbytes), ctx.alloc(wt.nbytes), ctx.alloc(b.nbytes)
        hy = ctx.alloc(4 * cout * (h // 2) * (w // 2))
        ctx.host_write(hx, x)
        ctx.host_write(hw_, wt)
        ctx.host_write(hb, b)
        for v in (3, 3, 4, 1):
            ctx.host_write(hy, np.zeros(cout * (h // 2) * (w // 2), np.float32))
            ctx.set_launch("conv3x3_relu_pool", 256, 0, v)
            ctx.kernel("conv3x3_relu_pool", [(hx, "c"), (hw_, "c"), (hb, "c"), (hy, "m")],
                       cin=cin, cout=cout, h=h, w=w)
            y = np.zeros((cout, h // 2, w // 2), np.float32)
            ctx.host_read(hy, y)
            r = ref.astype(np.float64)
            assert np.all((y == ref) | (np.abs(y.astype(np.float64) - r) <= 1e-5 * np.abs(r))), \
                (v, np.max(np.abs(y - ref)))
            outs.setdefault(v, []).append(y)
    finally:
        ctx.close()
    assert np.array_equal(outs[3][0].view(np.uint32), outs[3][1].view(np.uint32))
    # variant 4 (one block of 16 channels per workgroup) sums every output in variant 3's order
    assert np.array_equal(outs[4][0].view(np.uint32), outs[3][0].view(np.uint32))
    if cin % 4 or cout % 16:
        assert np.array_equal(outs[3][0].view(np.uint32), outs[1][0].view(np.uint32))


@pytest.mark.parametrize("graph_mode", [0, 1])
@pytest.mark.parametrize("conv_variant,dense_variant", [(2, 3), (2, 4), (1, 1), (3, 4)])
def test_dl_region_replays_with_two_kernel_tasks(graph_mode, conv_variant, dense_variant):
    """The DL DAG recorded as a region (hipGraph, or recorded multi-stream
    replay) while its convolution and dense tasks launch two kernels each
    (an fp64 weight copy, then the convolution; partial sums, then the final
    add): three replays, the inputs uploaded again before each, every
    replay's outputs checked against the oracle."""
    from paper_2012_09646_amd import runner
    banner("dl region graph_mode=%d conv=%d dense=%d" % (graph_mode, conv_variant, dense_variant))
    prog = W.dl_program(side=96, seed=31, channels=(8, 16), embed=16)
    ref = G.oracle_run(prog)
    ctx = D.Context(graph_mode=graph_mode)
    try:
        ctx.set_launch("conv3x3_relu_pool", 256, 0, conv_variant)
        ctx.set_launch("dense", 256, 64, dense_variant)
        b = runner.Bound(ctx, prog)
        b.record(1)
        for _ in range(3):
            for name in prog.outputs:
                ctx.host_write(b.h[name], np.zeros(prog.bufs[name].nbytes, np.uint8))
            b.upload([n for n in prog.bufs if prog.bufs[n].init is not None])
            b.replay(1)
            for name in prog.outputs:
                G.assert_close(prog, name, b.read(name), ref[name])
    finally:
        ctx.close()


_FULL = {}


def _full_size_reference():
    if not _FULL:
        prog = W.dl_program(side=1024, seed=6)
        _FULL["prog"], _FULL["ref"] = prog, G.oracle_run(prog)
    return _FULL["prog"], _FULL["ref"]


def test_dl_full_size():
    """The benchmark's shape: two 1024 x 1024 images, 16 and 32 channels, 16-wide embeddings."""
    banner("dl full size")
    prog = W.dl_program(side=1024, seed=6)
    G.check_program(prog)


@pytest.mark.parametrize("conv_variant,dense_variant,dense_block,dense_cap",
                         [(0, 0, 256, 1024), (2, 3, 512, 256), (1, 4, 512, 512), (1, 2, 1024, 128),
                          (3, 4, 512, 512)])
def test_dl_full_size_launch_variants(conv_variant, dense_variant, dense_block, dense_cap):
    """The benchmark's shape in other launch variants of the convolution and
    dense kernels than the tuned ones: every output against the oracle."""
    banner("dl full size conv=%d dense=%d (%d, %d)" % (conv_variant, dense_variant, dense_block, dense_cap))
    prog, ref = _full_size_reference()
    ctx = D.Context()
    try:
        ctx.set_launch("conv3x3_relu_pool", 256, 0, conv_variant)
        ctx.set_launch("dense", dense_block, dense_cap, dense_variant)
        b = runner.Bound(ctx, prog)
        b.run()
        for name in prog.outputs:
            G.assert_close(prog, name, b.read(name), ref[name])
    finally:
        ctx.close()
