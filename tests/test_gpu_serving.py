"""Serving with continuous batching on the GPU: a request's result is the same
alone and in a mix of requests admitted at other times; admission respects
the HBM budget; latency statistics are reported."""
import numpy as np
import pytest

from paper_2605_01352_amd import scenegen as sg
from paper_2605_01352_amd import vuda
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def small_requests():
    specs = [sg.RequestSpec(0, 0.0, 5, 12, 64, 7), sg.RequestSpec(1, 0.0, 9, 20, 128, 11),
             sg.RequestSpec(2, 0.0, 4, 8, 64, 5), sg.RequestSpec(3, 0.0, 6, 30, 64, 9)]
    return specs, [sg.request_scene(r) for r in specs]


def server(**kw):
    args = dict(cap_envs=64, cap_bodies=1024, cap_cams=64, cap_pixels=64 * 128 * 128, keep_results=True)
    args.update(kw)
    return vuda.Server(**args)


def run_until_done(srv, n, max_ticks=500):
    done = {}
    for _ in range(max_ticks):
        srv.tick()
        for rid, lat in srv.completed():
            done[rid] = lat
        if len(done) >= n:
            return done
    raise AssertionError(f"only {len(done)} of {n} requests completed")


@pytest.mark.parametrize("schedule,split", [(vuda.SCHED_INTERSTEP, 2.0), (vuda.SCHED_INTERTRAJ, 0.5),
                                            (vuda.SCHED_PIPELINED, 2.0), (vuda.SCHED_SERIAL, 0.0)])
def test_request_same_alone_and_in_mix(schedule, split):
    specs, scenes = small_requests()
    with server(schedule=schedule, cu_split=split) as a:
        a.submit(0, scenes[0], specs[0].horizon)
        run_until_done(a, 1)
        alone = [a.result(0, k) for k in (vuda.FETCH_STATE, vuda.FETCH_RGB, vuda.FETCH_DEPTH)]
    with server(schedule=schedule, cu_split=split) as b:
        b.submit(1, scenes[1], specs[1].horizon)
        b.tick()
        b.tick()
        b.submit(0, scenes[0], specs[0].horizon)   # joins while request 1 is running
        b.tick()
        b.submit(2, scenes[2], specs[2].horizon)
        b.submit(3, scenes[3], specs[3].horizon)
        run_until_done(b, 4)
        mixed = [b.result(0, k) for k in (vuda.FETCH_STATE, vuda.FETCH_RGB, vuda.FETCH_DEPTH)]
        st = b.stats()
    for x, y in zip(alone, mixed):
        assert np.array_equal(x, y)
    assert st["completed"] == 4 and st["queued"] == 0 and st["active_requests"] == 0
    assert st["env_steps"] == sum(r.n_envs * r.horizon for r in specs)


def test_result_matches_a_plain_world():
    specs, scenes = small_requests()
    r = specs[1]
    with server() as srv:
        srv.submit(7, scenes[1], r.horizon)
        run_until_done(srv, 1)
        got = srv.result(7, vuda.FETCH_STATE)
    with vuda.World(scenes[1]) as w:
        for _ in range(r.horizon):
            w.step()
        w.wait()
        assert np.array_equal(w.fetch(vuda.FETCH_STATE), got)


def test_admission_waits_for_budget():
    specs, scenes = small_requests()
    # a budget that holds request 1 (the largest) but not two of them at once
    with server(hbm_budget=1, keep_results=False) as tiny:
        with pytest.raises(vuda.VudaError):
            tiny.submit(1, scenes[1], specs[1].horizon)  # can never fit
    with server(keep_results=False) as one:
        one.submit(10, scenes[1], specs[1].horizon)
        one.tick()
        need = one.stats()["reserved_bytes"]  # what one such request holds
    assert need > 9 * 128 * 128 * 7
    budget = need + need // 2
    with server(hbm_budget=budget, keep_results=False) as srv:
        for k in range(3):
            srv.submit(10 + k, scenes[1], specs[1].horizon)
        srv.tick()
        st = srv.stats()
        assert st["active_requests"] == 1 and st["queued"] == 2
        done = run_until_done(srv, 3)
        st = srv.stats()
        assert st["peak_reserved_bytes"] <= budget
        assert st["queue_p99_s"] > 0 and st["latency_p99_s"] >= st["latency_p50_s"] > 0
        say(f"budget-limited serving: {st}")
        assert sorted(done) == [10, 11, 12]


def test_slots_are_reused():
    specs, scenes = small_requests()
    with server(cap_envs=10, cap_bodies=200, cap_cams=10, cap_pixels=10 * 128 * 128,
                keep_results=False) as srv:
        for k in range(6):
            srv.submit(k, scenes[1], specs[1].horizon)  # 9 envs each: one at a time
        done = run_until_done(srv, 6, max_ticks=200)
        assert len(done) == 6


def test_box_request_matches_a_plain_world():
    """A request whose envs hold boxes (extents and moments copied with the
    request and uploaded at admission) ends as a plain world of them."""
    r = sg.RequestSpec(5, 0.0, 6, 20, 64, 9)
    scene = sg.with_boxes(sg.request_scene(r), every=1)
    assert np.count_nonzero(scene.btype == 2) > 0
    with server() as srv:
        srv.submit(5, scene, r.horizon)
        run_until_done(srv, 1)
        got = [srv.result(5, k) for k in (vuda.FETCH_STATE, vuda.FETCH_RGB, vuda.FETCH_DEPTH)]
    with vuda.World(scene) as w:
        for _ in range(r.horizon):
            w.step()
        w.render()
        w.wait()
        want = [w.fetch(k) for k in (vuda.FETCH_STATE, vuda.FETCH_RGB, vuda.FETCH_DEPTH)]
    for x, y in zip(want, got):
        assert np.array_equal(x, y)
    say("box request: state, rgb and depth equal to the plain world's")


_ORACLE_CHECKED = {}  # request id -> a plain world's results, checked against the oracle


@pytest.mark.parametrize("schedule,split", [(vuda.SCHED_INTERTRAJ, 0.5), (vuda.SCHED_PIPELINED, 2.0)])
def test_c5_shaped_requests_meet_the_oracle_gates(schedule, split):
    """Three requests of the serving workload's shape (16-24 envs of 12-64
    bodies, horizons 50-60, 64^2 and 128^2 frames) admitted at different
    ticks of one server, under a CU split and under the serving default (the
    pipelined schedule on streams over every CU).  Each served result (final
    state and its frame) equals a plain world's run of the request, and that
    run meets the oracle gates at every step (contact sets, state) and on the
    final frame (depth and winners bit-exact, RGB within 1)."""
    from tests.gpu_util import compare_render, compare_step
    specs = [sg.RequestSpec(100, 0.0, 16, 40, 64, 50), sg.RequestSpec(101, 0.0, 24, 12, 128, 60),
             sg.RequestSpec(102, 0.0, 20, 64, 64, 55)]
    scenes = [sg.request_scene(r) for r in specs]
    kinds = (vuda.FETCH_STATE, vuda.FETCH_RGB, vuda.FETCH_DEPTH)
    with server(cap_envs=96, cap_bodies=4096, cap_cams=96, cap_pixels=96 * 128 * 128,
                schedule=schedule, cu_split=split) as srv:
        srv.submit(100, scenes[0], specs[0].horizon)
        for _ in range(3):
            srv.tick()
        srv.submit(101, scenes[1], specs[1].horizon)
        for _ in range(7):
            srv.tick()
        srv.submit(102, scenes[2], specs[2].horizon)
        run_until_done(srv, 3)
        served = {r.rid: [srv.result(r.rid, k) for k in kinds] for r in specs}
    for r, sc in zip(specs, scenes):
        if r.rid not in _ORACLE_CHECKED:
            with vuda.World(sc, debug=True) as w:
                exact = 0
                for _ in range(r.horizon):
                    exact += compare_step(w, sc)["bitexact"]
                compare_render(w, sc)
                _ORACLE_CHECKED[r.rid] = ([w.fetch(k) for k in kinds], exact)
        want, exact = _ORACLE_CHECKED[r.rid]
        for x, y in zip(want, served[r.rid]):
            assert np.array_equal(x, y)
        say(f"request {r.rid} ({r.n_envs} envs x {r.n_bodies} bodies, {r.res}^2, horizon {r.horizon}), "
            f"{vuda.SCHED_NAMES[schedule]}@{split:g}: served result = plain world; oracle gates met at every "
            f"step ({exact} bit-exact) and on the frame")


def test_submit_refuses_requests_that_can_never_run():
    """Malformed requests and requests larger than the world are refused at
    submit, so that the FIFO never holds one that blocks the rest."""
    specs, scenes = small_requests()
    with server(cap_envs=8, cap_bodies=1024, cap_cams=8, cap_pixels=8 * 128 * 128) as srv:
        with pytest.raises(vuda.VudaError):
            srv.submit(1, scenes[1], specs[1].horizon)  # 9 envs > 8 slots
        bad = sg.request_scene(specs[0])
        bad.albedo[3] = 9  # palette has 8 entries
        with pytest.raises(vuda.VudaError):
            srv.submit(2, bad, specs[0].horizon)
        srv.submit(0, scenes[0], specs[0].horizon)  # still served
        done = run_until_done(srv, 1)
        assert list(done) == [0]
        assert srv.stats()["rejected"] == 0


@pytest.mark.parametrize("schedule", [vuda.SCHED_INTERSTEP, vuda.SCHED_PIPELINED])
def test_pipelined_ticks_keep_results_exact(schedule):
    """Ticks enqueue several iterations without waiting; requests with
    different horizons finish mid-stream and their slots are reused by
    later ones while others run.  Each result equals a plain world's."""
    specs = [sg.RequestSpec(20 + k, 0.0, 3 + k, 10 + 4 * k, 64, 9 + 5 * k) for k in range(5)]
    scenes = [sg.request_scene(r) for r in specs]
    with server(cap_envs=12, cap_bodies=600, cap_cams=12, cap_pixels=12 * 64 * 64, schedule=schedule) as srv:
        for r, sc in zip(specs, scenes):
            srv.submit(r.rid, sc, r.horizon)
        run_until_done(srv, len(specs))
        got = {r.rid: srv.result(r.rid, vuda.FETCH_STATE) for r in specs}
        st = srv.stats()
    assert st["env_steps"] == sum(r.n_envs * r.horizon for r in specs)
    for r, sc in zip(specs, scenes):
        with vuda.World(sc) as w:
            w.step(nsteps=r.horizon)
            w.wait()
            assert np.array_equal(w.fetch(vuda.FETCH_STATE), got[r.rid])
