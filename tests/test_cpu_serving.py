"""The serving loop's admission logic, simulated on a virtual clock by a
schedule-only context (no GPU): budget, bypass, lanes, serial mode."""

import numpy as np
import pytest

from paper_2012_09646_amd import dagrt as D
from paper_2012_09646_amd import serving
from paper_2012_09646_amd import workloads as W


def make(budget, lanes=4, bypass=32):
    ctx = D.Context(dry_run=True)
    small = serving.ShapeTemplate(ctx, W.vec_program(n=1 << 10), key=1)
    big = serving.ShapeTemplate(ctx, W.img_program(side=256), key=2)
    srv = serving.Server(ctx, budget, host_arena_bytes=1 << 20, lanes=lanes, bypass=bypass)
    s0 = srv.add(small, sim_ns=10_000)
    s1 = srv.add(big, sim_ns=100_000)
    return ctx, srv, s0, s1


def test_roles_and_footprints():
    ctx, srv, s0, s1 = make(1 << 30)
    t = srv.shapes[0]
    roles = {t.bound.name_of[h]: r for h, r, _ in t.roles}
    assert roles == {"x": D.DAG_ROLE_INIT, "y": D.DAG_ROLE_INIT, "r": D.DAG_ROLE_PRIVATE}
    dev, host = srv.footprint(s0)
    assert dev == 2 * 4096 + 256 and host == 256   # x, y, r (256-aligned) + staged result
    roles1 = {srv.shapes[1].bound.name_of[h]: r for h, r, _ in srv.shapes[1].roles}
    assert roles1["img"] == D.DAG_ROLE_SHARED and roles1["out"] == D.DAG_ROLE_PRIVATE
    srv.close()
    ctx.close()


def test_budget_binds_and_everything_completes():
    ctx, srv, s0, s1 = make(1 << 30)
    big = srv.footprint(s1)[0]
    srv.close()
    ctx.close()
    ctx, srv, s0, s1 = make(2 * big + 1000, lanes=8)
    arr, shp = W.poisson_trace(7, 400, 50_000, 2)
    out, st, _ = srv.run(arr, shp)
    assert st.peak_device_bytes <= 2 * big + 1000
    assert st.max_queued > 0 and st.max_inflight >= 2
    assert np.all(out["admit_ns"] >= arr) and np.all(out["done_ns"] > out["admit_ns"])
    lat = np.sort((out["done_ns"] - arr) / 1e6)
    assert abs(st.p50_ms - lat[int(np.ceil(0.5 * len(lat))) - 1]) < 1e-9
    assert abs(st.p99_ms - lat[int(np.ceil(0.99 * len(lat))) - 1]) < 1e-9
    srv.close()
    ctx.close()


def test_small_requests_bypass_a_big_one_that_does_not_fit():
    ctx, srv, s0, s1 = make(1 << 30)
    big = srv.footprint(s1)[0]
    small = srv.footprint(s0)[0]
    srv.close()
    ctx.close()
    # budget fits one big request plus a few small ones, not two big ones
    ctx, srv, s0, s1 = make(big + 4 * small, lanes=4)
    arr = np.array([0, 1, 2, 3, 4], dtype=np.int64)
    shp = np.array([s1, s1, s0, s0, s0], dtype=np.int32)
    out, st, _ = srv.run(arr, shp)
    # the second big request waits for the first; the small ones do not wait for it
    assert out["admit_ns"][1] >= out["done_ns"][0]
    assert np.all(out["admit_ns"][2:] < out["done_ns"][0])
    srv.close()
    # without bypass the small ones queue behind the second big request
    ctx2, srv2, a0, a1 = make(big + 4 * small, lanes=4, bypass=1)
    out2, _, _ = srv2.run(arr, np.array([a1, a1, a0, a0, a0], dtype=np.int32))
    assert np.all(out2["admit_ns"][2:] >= out2["admit_ns"][1])
    srv2.close()
    ctx.close()
    ctx2.close()


def test_serial_mode_runs_one_at_a_time():
    ctx, srv, s0, s1 = make(1 << 30)
    arr, shp = W.poisson_trace(3, 60, 100_000, 2)
    out, st, _ = srv.run(arr, shp, mode=D.DAG_SERVE_SERIAL)
    order = np.argsort(out["admit_ns"], kind="stable")
    assert np.all(out["admit_ns"][order][1:] >= out["done_ns"][order][:-1])
    assert st.max_inflight == 1 and np.all(out["lane"] == 0)
    srv.close()
    ctx.close()


def test_lanes_share_load():
    ctx, srv, s0, s1 = make(1 << 30, lanes=4)
    arr = np.zeros(40, dtype=np.int64)
    shp = np.zeros(40, dtype=np.int32)
    out, st, _ = srv.run(arr, shp)
    assert sorted(np.bincount(out["lane"], minlength=4).tolist()) == [10, 10, 10, 10]
    assert st.max_inflight == 40
    srv.close()
    ctx.close()


def test_shape_validation():
    ctx = D.Context(dry_run=True)
    t = serving.ShapeTemplate(ctx, W.vec_program(n=256), key=3)
    srv = serving.Server(ctx, 1 << 20, host_arena_bytes=1 << 16, lanes=2)
    with pytest.raises(D.DagError):   # a buffer the region modifies declared shared
        D.dag_serve_add_shape(ctx.h, srv.h, 3, [(h, D.DAG_ROLE_SHARED, 0) for h, _, _ in t.roles],
                              t.bound.h["r"], 4, 0)
    with pytest.raises(D.DagError):   # a buffer of the region missing
        D.dag_serve_add_shape(ctx.h, srv.h, 3, t.roles[:1], 0, 0, 0)
    with pytest.raises(D.DagError):   # unknown region
        D.dag_serve_add_shape(ctx.h, srv.h, 99, t.roles, 0, 0, 0)
    small = serving.Server(ctx, 1024, host_arena_bytes=1 << 16, lanes=1)
    with pytest.raises(D.DagError):   # footprint beyond the budget
        small.add(t)
    small.close()
    srv.close()
    ctx.close()


def test_transfer_lanes_separate_link_bound_requests():
    """With transfer_lanes = 1, requests whose shape copies between host and
    device (the Black-Scholes fan-out) use lane 0 only and all others lanes
    1.. only; without it any lane takes any request."""
    ctx = D.Context(dry_run=True)
    comp = serving.ShapeTemplate(ctx, W.vec_program(n=1 << 10), key=11)
    link = serving.ShapeTemplate(ctx, W.bs_program(n=1 << 10, tasks=2), key=12)
    arr = np.zeros(32, dtype=np.int64)
    shp = np.array([i % 4 == 0 for i in range(32)], dtype=np.int32)   # every fourth request copies
    srv = serving.Server(ctx, 1 << 30, host_arena_bytes=1 << 24, lanes=3, transfer_lanes=1)
    a, b = srv.add(comp, sim_ns=10_000), srv.add(link, sim_ns=50_000)
    assert (a, b) == (0, 1)
    out, st, _ = srv.run(arr, shp)
    assert np.all(out["lane"][shp == 1] == 0)
    assert set(out["lane"][shp == 0].tolist()) == {1, 2}
    srv.close()
    srv = serving.Server(ctx, 1 << 30, host_arena_bytes=1 << 24, lanes=3, transfer_lanes=0)
    srv.add(comp, sim_ns=10_000)
    srv.add(link, sim_ns=50_000)
    out, _, _ = srv.run(arr, shp)
    assert set(out["lane"][shp == 1].tolist()) == {0, 1, 2}
    srv.close()
    for bad in (3, 4):
        with pytest.raises(D.DagError):
            serving.Server(ctx, 1 << 30, host_arena_bytes=1 << 24, lanes=3, transfer_lanes=bad)
    ctx.close()


def test_online_producer_gets_exactly_the_batch_schedule():
    """Requests submitted one by one by a producer thread while the loop
    polls (dag_serve_submit / dag_serve_poll) are admitted and completed on
    the virtual clock exactly as when the whole trace is known at the start
    (dag_serve_run), with the budget forcing queueing and bypass."""
    ctx, srv, s0, s1 = make(1 << 30)
    big, small = srv.footprint(s1)[0], srv.footprint(s0)[0]
    srv.close()
    ctx.close()
    ctx, srv, s0, s1 = make(2 * big + 3 * small, lanes=3, bypass=4)
    arr, shp = W.poisson_trace(11, 300, 40_000, 2)
    out, st, _ = srv.run(arr, shp)
    delays = W.rng(5).uniform(0, 2e-4, size=len(arr)) * (W.rng(6).random(len(arr)) < 0.2)
    recs, st2, _ = srv.run_online(arr, shp, pace=False, delays=delays)
    assert st.max_queued > 0
    for i, (a, adm, done, sh, lane) in enumerate(recs):
        assert (a, sh) == (arr[i], shp[i])
        assert (adm, done, lane) == (out["admit_ns"][i], out["done_ns"][i], out["lane"][i]), i
    for f in ("p50_ms", "p99_ms", "mean_ms", "req_per_s", "peak_device_bytes", "max_inflight", "max_queued"):
        assert getattr(st, f) == getattr(st2, f), f
    assert st2.completed == len(arr)
    srv.close()
    ctx.close()


def test_online_submission_rules():
    ctx, srv, s0, s1 = make(1 << 30)
    with pytest.raises(D.DagError) as e:   # no session yet
        srv.submit(s0, 0)
    assert e.value.name == "DAG_E_BUSY"
    srv.start()
    srv.submit(s0, 100)
    with pytest.raises(D.DagError) as e:   # arrivals must not go back in time
        srv.submit(s0, 99)
    assert e.value.name == "DAG_E_INVAL"
    with pytest.raises(D.DagError) as e:   # a virtual clock has no "now"
        srv.submit(s0)
    assert e.value.name == "DAG_E_INVAL"
    with pytest.raises(D.DagError):        # unknown shape
        srv.submit(7, 200)
    # the loop does not pass the latest arrival while more may come
    got, left = srv.poll()
    assert got == [] and left == 1
    with pytest.raises(D.DagError) as e:   # a new session while requests are outstanding
        srv.start()
    assert e.value.name == "DAG_E_BUSY"
    srv.close_session()
    with pytest.raises(D.DagError) as e:   # closed
        srv.submit(s0, 300)
    assert e.value.name == "DAG_E_BUSY"
    got, left = srv.poll()
    assert len(got) == 1 and left == 0
    d = got[0]
    assert (d.id, d.arrival_ns, d.admit_ns, d.done_ns) == (0, 100, 100, 100 + 10_000)
    assert srv.stats().completed == 1
    srv.start()   # a fresh session
    assert srv.stats().completed == 0
    srv.close_session()
    assert srv.poll() == ([], 0)
    srv.close()
    ctx.close()


def test_released_buffer_kills_the_regions_that_use_it():
    """A recorded region keeps its buffers' addresses: after one of them is
    released the region can no longer be launched (DAG_E_INVAL), and a
    recurring-region run records it anew instead of replaying it."""
    ctx = D.Context(dry_run=True)
    x, y = ctx.alloc(4096), ctx.alloc(4096)
    D.dag_region_begin(ctx.h, 5)
    ctx.kernel("vec_square", [(x, "m")], n=1024)
    D.dag_region_end(ctx.h)
    D.dag_region_begin(ctx.h, 6)
    ctx.kernel("vec_square", [(y, "m")], n=1024)
    D.dag_region_end(ctx.h)
    D.dag_region_launch(ctx.h, 5)
    ctx.release(x)
    with pytest.raises(D.DagError) as e:
        D.dag_region_launch(ctx.h, 5)
    assert e.value.name == "DAG_E_INVAL"
    D.dag_region_launch(ctx.h, 6)          # the other region is untouched
    x2 = ctx.alloc(4096)
    D.dag_region_run_begin(ctx.h, 5)       # the dead recording is replaced
    ctx.kernel("vec_square", [(x2, "m")], n=1024)
    assert D.dag_region_run_end(ctx.h) == (0, False)
    D.dag_region_run_begin(ctx.h, 5)
    ctx.kernel("vec_square", [(x2, "m")], n=1024)
    tid, replayed = D.dag_region_run_end(ctx.h)
    assert replayed and tid > 0
    ctx.close()


def test_serving_shape_pins_its_region_and_buffers():
    ctx = D.Context(dry_run=True)
    t = serving.ShapeTemplate(ctx, W.vec_program(n=256), key=3)
    srv = serving.Server(ctx, 1 << 20, host_arena_bytes=1 << 16, lanes=2)
    srv.add(t)
    for call in (lambda: D.dag_region_drop(ctx.h, 3), lambda: D.dag_region_begin(ctx.h, 3),
                 lambda: ctx.release(t.bound.h["x"]), lambda: ctx.release(t.pristine["x"])):
        with pytest.raises(D.DagError) as e:
            call()
        assert e.value.name == "DAG_E_BUSY"
    # a recurring run whose calls differ from the pinned recording runs
    # eagerly and leaves the recording as it is
    ntasks = D.dag_region_info(ctx.h, 3)[0]
    D.dag_region_run_begin(ctx.h, 3)
    tid = ctx.kernel("vec_square", [(t.bound.h["y"], "m")], n=7)
    assert tid > 0
    assert D.dag_region_run_end(ctx.h) == (0, False)
    assert D.dag_region_info(ctx.h, 3)[0] == ntasks
    srv.close()
    ctx.release(t.pristine["x"])
    ctx.release(t.bound.h["x"])
    D.dag_region_drop(ctx.h, 3)
    ctx.close()
