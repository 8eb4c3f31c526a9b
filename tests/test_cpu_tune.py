"""Autotuner host logic: candidate sets are valid launch configurations,
the JSON round trip, and applying a tuning table to a context."""

import pytest

from paper_2012_09646_amd import dagrt as D
from paper_2012_09646_amd import tune
from paper_2012_09646_amd import workloads as W


@pytest.mark.parametrize("kernel", sorted(D.KERNEL_IDS))
def test_candidates_accepted_by_the_library(kernel):
    ctx = D.Context(dry_run=True)
    for c in tune.candidates(kernel):
        ctx.set_launch(kernel, *c)
        assert ctx.get_launch(kernel) == c
    ctx.close()


def test_json_round_trip_and_apply(tmp_path):
    data = {"kernels": {"bs_call": {"block": 512, "grid_cap": 1024, "variant": 0, "us": 40.0},
                        "spmv": {"block": 256, "grid_cap": 0, "variant": 16, "us": 30.0}},
            "dag": {"bs": {"max_streams": 4, "copy_streams": 0, "ms": 3.9}}}
    p = str(tmp_path / "t.json")
    tune.save(p, data)
    back = tune.load(p)
    assert back["arch"] == "gfx950" and back["kernels"] == data["kernels"]
    ctx = D.Context(dry_run=True)
    tune.apply_kernels(ctx, back["kernels"])
    assert ctx.get_launch("bs_call") == (512, 1024, 0) and ctx.get_launch("spmv") == (256, 0, 16)
    ctx.close()


def test_tune_kernel_needs_a_gpu():
    ctx = D.Context(dry_run=True)
    x = ctx.alloc(4096)
    with pytest.raises(D.DagError) as e:
        D.dag_tune_kernel(ctx.h, 1, D.dag_p_n(1024), [(x, D.DAG_MUTABLE)], [(256, 0, 0)])
    assert e.value.name == "DAG_E_UNSUPPORTED"
    ctx.close()


def test_hw_queue_sweep_merges_worker_results(tmp_path, monkeypatch):
    """The orchestrator runs one worker per GPU_MAX_HW_QUEUES value and keeps,
    per workload, the fastest configuration with its queue count."""
    calls = []
    times = {4: {"bs": 4.0, "img": 0.10}, 8: {"bs": 3.5, "img": 0.12}, 16: {"bs": 3.7, "img": 0.11}}

    def fake_spawn(extra, out, hw_queues=None):
        calls.append((extra[extra.index("--worker") + 1], hw_queues))
        if "kernels" in extra:
            return {"kernels": {"bs_call": {"block": 256, "grid_cap": 0, "variant": 1}}, "dag": {}}
        dag = {w: {"max_streams": 2, "copy_streams": 0, "copy_lanes": 1, "ms": t,
                   "table": [{"max_streams": 2, "ms": t}]} for w, t in times[hw_queues].items()}
        return {"kernels": {}, "dag": dag}

    monkeypatch.setattr(tune, "_spawn", fake_spawn)
    out = str(tmp_path / "t.json")
    monkeypatch.setattr("sys.argv", ["tune", "--out", out, "--dag", "--hw-queues", "4,8,16"])
    tune.main()
    data = tune.load(out)
    assert calls == [("kernels", None), ("dag", 4), ("dag", 8), ("dag", 16)]
    assert data["dag"]["bs"]["hw_queues"] == 8 and data["dag"]["bs"]["ms"] == 3.5
    assert data["dag"]["img"]["hw_queues"] == 4
    assert len(data["dag"]["bs"]["table"]) == 3
    assert {r["hw_queues"] for r in data["dag"]["bs"]["table"]} == {4, 8, 16}
    assert data["kernels"]["bs_call"]["variant"] == 1


def test_dag_choice_prefers_configurations_that_fit_the_queues(tmp_path, monkeypatch):
    def fake_spawn(extra, out, hw_queues=None):
        if "kernels" in extra:
            return {"kernels": {}, "dag": {}}
        # 4 queues: the fastest configuration needs 6 streams; 8 queues: it fits but is slower
        e = {4: {"max_streams": 4, "ms": 3.0, "fits": False, "table": [{"ms": 3.0}, {"ms": 3.5}]},
             8: {"max_streams": 1, "ms": 3.4, "fits": True, "table": [{"ms": 3.4}]}}[hw_queues]
        return {"kernels": {}, "dag": {"bs": e}}

    monkeypatch.setattr(tune, "_spawn", fake_spawn)
    out = str(tmp_path / "t.json")
    monkeypatch.setattr("sys.argv", ["tune", "--out", out, "--dag", "--hw-queues", "4,8", "--workload", "bs"])
    tune.main()
    d = tune.load(out)["dag"]["bs"]
    assert d["hw_queues"] == 8 and d["max_streams"] == 1


def test_near_ties_are_broken_by_makespan():
    """A kernel configuration within 3 % of the fastest alone is kept for a
    DAG when it shortens the makespan by more than 3 % against the current
    choice measured in the same rounds; one that does not is left out."""
    prog = W.ml_program(n=64, seed=1, features=8, classes=3, categories=4)
    kernels = {"nb_proba": {"block": 1024, "grid_cap": 256, "variant": 2,
                            "near": [[1024, 256, 0, 101.0], [512, 256, 0, 102.0]]},
               "ridge_proba": {"block": 256, "grid_cap": 0, "variant": 4, "near": [[256, 0, 0, 100.5]]}}
    best = {"max_streams": 2, "copy_streams": 0, "copy_lanes": 1, "ms": 0.50}
    seen = []

    def fake(prog_, kern, over, ms, cm, lanes, restore, runs):
        seen.append(dict(over))
        if over.get("nb_proba") == (1024, 256, 0):
            return (0.40 if "ridge_proba" not in over else 0.395), 2   # the second gain is below 3 %
        return 0.52, 2

    over, ms = tune.break_ties(prog, kernels, best, measure=fake)
    assert over == {"nb_proba": [1024, 256, 0]} and ms == 0.40
    assert {"nb_proba": (512, 256, 0)} in seen                      # every near tie was tried
    assert {"nb_proba": (1024, 256, 0), "ridge_proba": (256, 0, 0)} in seen


def test_shipped_table_holds_only_swept_candidates():
    """tune.load refuses a table with a configuration outside candidates();
    the shipped table loads and names its ROCm release."""
    import os
    path = os.path.join(os.path.dirname(tune.__file__), "tuning", "gfx950.json")
    data = tune.load(path)
    assert data["rocm"]
    for k, e in data["kernels"].items():
        assert (e["block"], e["grid_cap"], e["variant"]) in tune.candidates(k)


def test_unswept_configuration_is_refused(tmp_path):
    ctx = D.Context(dry_run=True)
    # a valid library configuration that is not a candidate (grid cap 2048 for an elementwise kernel)
    ctx.set_launch("vec_square", 256, 2048, 0)
    with pytest.raises(ValueError):
        tune.set_launch(ctx, "vec_square", (256, 2048, 0))
    ctx.close()
    p = str(tmp_path / "bad.json")
    tune.save(p, {"kernels": {"sobel": {"block": 256, "grid_cap": 0, "variant": 2, "us": 1.0}}, "dag": {}})
    with pytest.raises(ValueError):
        tune.load(p)


def test_stencil_tile_shapes_need_their_workgroup_size():
    ctx = D.Context(dry_run=True)
    # 9 and 11: the resident grids of 64x16 and 64x8 tiles, the only ones that take a grid cap
    for block, cap, variant, ok in [(256, 0, 0, True), (128, 0, 2, True), (64, 0, 4, True), (64, 0, 6, True),
                                    (64, 0, 7, True), (256, 0, 2, False), (128, 0, 4, False), (256, 0, 8, False),
                                    (256, 0, 9, True), (256, 1024, 9, True), (128, 0, 11, True),
                                    (128, 8, 11, True), (128, 0, 9, False), (256, 0, 11, False),
                                    (64, 0, 13, False), (64, 0, 15, False), (256, 1024, 1, False),
                                    (256, 0, 16, False)]:
        for k in ("gauss_blur", "sobel"):
            try:
                ctx.set_launch(k, block, cap, variant)
                assert ok, (k, block, cap, variant)
            except D.DagError:
                assert not ok, (k, block, cap, variant)
    ctx.close()


def test_spmv_grid_cap_only_for_the_resident_grid():
    ctx = D.Context(dry_run=True)
    for cap, variant, ok in [(0, 0x504, True), (1024, 0x504, True), (1, 0x508, True), (1024, 0x104, False),
                             (1024, 8, False), (1024, 0x304, False)]:
        try:
            ctx.set_launch("spmv", 256, cap, variant)
            assert ok, (cap, variant)
        except D.DagError:
            assert not ok, (cap, variant)
    ctx.close()


def test_resident_spmv_caps_are_candidates_and_tried_in_the_dag():
    cands = tune.candidates("spmv")
    for c in tune.RESIDENT_CAPS:
        assert (256, c, 0x504) in cands
    assert tune.LEAVES_ROOM["spmv"]((256, 1024, 0x504)) and not tune.LEAVES_ROOM["spmv"]((256, 0, 0x504))


def test_capped_resident_tiles_are_candidates():
    for k in ("gauss_blur", "sobel"):
        room = [c for c in tune.candidates(k) if tune.LEAVES_ROOM[k](c)]
        assert room and all(c[2] in (9, 11) and c[1] for c in room)


def test_the_fastest_capped_resident_form_is_retried_in_the_dag(monkeypatch):
    """tune_kernels (timings faked; schedule-only context): the uncapped
    resident SpMV wins alone, and the fastest capped form joins the
    configurations retried inside the DAG although it is not a near-tie; a
    reduction's one-launch form likewise."""
    def fake_tune(h, kid, prm, args, cands, reps=20):
        us = [200.0 + i for i in range(len(cands))]
        if kid == D.KERNEL_IDS["spmv"]:
            us[cands.index((256, 0, 0x504))] = 50.0
            for c, t in zip(tune.RESIDENT_CAPS, (61.0, 60.0, 70.0)):
                us[cands.index((256, c, 0x504))] = t
        return 0, us

    monkeypatch.setattr(tune.D, "dag_tune_kernel", fake_tune)
    ctx = D.Context(dry_run=True)
    out = tune.tune_kernels(ctx, W.hits_program(n=1000, iters=2, seed=3))
    ctx.close()
    e = out["spmv"]
    assert (e["block"], e["grid_cap"], e["variant"]) == (256, 0, 0x504)
    assert [256, tune.RESIDENT_CAPS[1], 0x504] in [n[:3] for n in e["near"]]
    assert any(n[2] == 1 for n in out["sumsq"]["near"])
