"""The autotuner's search space on the GPU: every candidate launch
configuration of every tunable kernel (tune.candidates, the only
configurations tune.py installs) runs its kernel inside a small ragged
workload DAG whose outputs must equal the oracle's; and dag_tune_kernel,
run on real arguments, installs the candidate it measured fastest, after
which the kernel still matches the oracle."""

import numpy as np
import pytest

import gpu_util as G
from paper_2012_09646_amd import dagrt as D
from paper_2012_09646_amd import runner
from paper_2012_09646_amd import tune
from paper_2012_09646_amd import workloads as W

pytestmark = pytest.mark.gpu


def banner(s):
    print("[tune] " + s, flush=True)


# Small programs with ragged sizes: several workgroups, tiles and grid-stride
# passes, and a partial last one.
PROGRAMS = {
    "vec": lambda: W.vec_program(n=(1 << 21) + 3, seed=11),
    "bs": lambda: W.bs_program(n=(1 << 18) + 5, tasks=1, seed=12),
    "img": lambda: W.img_program(side=197, height=131, seed=13),
    "hits": lambda: W.hits_program(n=(1 << 14) + 3, iters=2, seed=14),
    "ml": lambda: W.ml_program(n=4099, seed=15),
    "dl": lambda: W.dl_program(side=96, seed=16),
}


@pytest.mark.parametrize("name", sorted(PROGRAMS))
def test_every_candidate_matches_the_oracle(name):
    prog = PROGRAMS[name]()
    ref = G.oracle_run(prog)
    kernels = sorted({o["kernel"] for o in prog.ops if o["kind"] == "kernel" and tune.candidates(o["kernel"])})
    assert kernels
    with D.Context() as ctx:
        b = runner.Bound(ctx, prog, upload=False)
        for k in kernels:
            default = ctx.get_launch(k)
            for cand in tune.candidates(k):
                banner("%s %s %s" % (name, k, cand))
                tune.set_launch(ctx, k, cand)
                b.upload()
                b.run()
                for out in prog.outputs:
                    try:
                        G.assert_close(prog, out, b.read(out), ref[out])
                    except AssertionError as e:
                        raise AssertionError("%s with %s: %s" % (k, cand, e))
            ctx.set_launch(k, *default)


def test_copy_kernel_candidates():
    n = (1 << 20) + 7
    src = W.uniform_f32(17, n)
    with D.Context() as ctx:
        hs, hd = ctx.alloc(4 * n), ctx.alloc(4 * n)
        ctx.host_write(hs, src)
        for cand in tune.candidates("copy_f32"):
            tune.set_launch(ctx, "copy_f32", cand)
            ctx.host_write(hd, np.zeros(n, np.float32))
            ctx.kernel("copy_f32", [(hs, "c"), (hd, "m")], n=n)
            out = np.zeros(n, np.float32)
            ctx.host_read(hd, out)
            assert np.array_equal(out.view(np.uint32), src.view(np.uint32)), cand


@pytest.mark.parametrize("kernel,name", [("gauss_blur", "img"), ("sobel", "img"), ("sumsq", "hits"),
                                         ("spmv", "hits")])
def test_tune_kernel_installs_its_fastest_candidate(kernel, name):
    banner("dag_tune_kernel %s" % kernel)
    prog = PROGRAMS[name]()
    ref = G.oracle_run(prog)
    op = next(o for o in prog.ops if o["kind"] == "kernel" and o["kernel"] == kernel)
    cands = tune.candidates(kernel)
    with D.Context() as ctx:
        b = runner.Bound(ctx, prog)
        b.run()  # every input of the tuned call holds the program's data
        ctx.sync()
        args = [(b.h[n], D.DAG_MUTABLE if m == "m" else D.DAG_CONST) for n, m in op["args"]]
        best, us = D.dag_tune_kernel(ctx.h, D.KERNEL_IDS[kernel], D.make_params(kernel, op["params"]), args,
                                     cands, 5)
        valid = [i for i, t in enumerate(us) if t >= 0]
        assert len(valid) == len(cands), "the library rejected a candidate: %s" % us
        assert best == min(valid, key=lambda i: us[i])
        assert ctx.get_launch(kernel) == cands[best]
        b.upload()
        b.run()
        for out in prog.outputs:
            G.assert_close(prog, out, b.read(out), ref[out])
