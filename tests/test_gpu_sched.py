"""Scheduling obligations on the GPU (through the C ABI).

The paper's interface makes step and render asynchronous, binds a stream for
spatial co-execution and requires that binding/unbinding preserve the
applications's synchronisation and results (VUDA Programming Interface; System
Mechanisms, Correctness).  Here: asynchronous enqueue, bit-identical results
in every co-scheduling mode and schedule (inter-step, inter-trajectory),
toggling mid-run, the CU partition of the masked streams, checkpoint/resume,
the autotuner leaving results unchanged, and the error flags.
"""
import collections
import time

import numpy as np
import pytest

from paper_2605_01352_amd import scenegen as sg
from paper_2605_01352_amd import vuda
from tests.gpu_util import say
from tests.scenes import tiny_scene

pytestmark = pytest.mark.gpu


def outputs(w):
    return (w.fetch(vuda.FETCH_STATE), w.fetch(vuda.FETCH_RGB), w.fetch(vuda.FETCH_DEPTH))


def reference(scene, iters):
    with vuda.World(scene) as w:
        for _ in range(iters):
            w.step()
            w.render()
        w.wait()
        return outputs(w)


def assert_same(a, b, what=""):
    for x, y in zip(a, b):
        assert np.array_equal(x, y), what


def test_async_enqueue_returns_early():
    """step/render only enqueue: right after the calls return, the streams
    still hold the work."""
    import torch
    torch.cuda.init()
    dev = torch.device("cuda", 0)
    s = sg.config_scene(2, n_envs=1024)
    with vuda.World(s) as w:
        w.cosched(2.0)
        w.run(vuda.SCHED_INTERSTEP, 2)
        w.wait()
        streams = [torch.cuda.ExternalStream(w.stream(p), device=dev)
                   for p in (vuda.PHASE_STEP, vuda.PHASE_RENDER)]
        t0 = time.perf_counter()
        w.run(vuda.SCHED_INTERSTEP, 30)
        t_enqueue = time.perf_counter() - t0
        busy = not all(st.query() for st in streams)
        w.wait()
        t_total = time.perf_counter() - t0
        say(f"enqueue {t_enqueue*1e3:.2f} ms of {t_total*1e3:.2f} ms")
        assert busy and t_enqueue < t_total


@pytest.mark.parametrize("split", [2.0, 0.5])
def test_list_rebuild_does_not_wait_for_running_work(split):
    """A call that builds a new work list (here a step over an env range not
    stepped before) copies the list to the device while earlier iterations
    still run.  The co-scheduled streams are blocking streams, which a copy
    on the null stream would wait for: the call must return long before the
    running iterations end."""
    import torch
    torch.cuda.init()
    dev = torch.device("cuda", 0)
    s = sg.config_scene(2, n_envs=1024)
    with vuda.World(s) as w:
        w.cosched(split)
        w.run(vuda.SCHED_INTERSTEP, 2)
        w.wait()
        streams = [torch.cuda.ExternalStream(w.stream(p), device=dev)
                   for p in (vuda.PHASE_STEP, vuda.PHASE_RENDER)]
        t0 = time.perf_counter()
        w.run(vuda.SCHED_INTERSTEP, 100)
        t1 = time.perf_counter()
        w.step(lo=0, hi=384)  # a range with no list yet
        t_call = time.perf_counter() - t1
        busy = not all(st.query() for st in streams)
        w.wait()
        t_total = time.perf_counter() - t0
        say(f"split {split:g}: new-range step returned in {t_call * 1e3:.2f} ms; the running iterations took "
            f"{t_total * 1e3:.2f} ms")
        assert busy and t_call < 0.25 * t_total


@pytest.mark.parametrize("schedule", [vuda.SCHED_SERIAL, vuda.SCHED_INTERSTEP, vuda.SCHED_INTERTRAJ])
@pytest.mark.parametrize("split", [0.0, 2.0, 0.25, 0.625])
def test_schedules_and_modes_bit_identical(schedule, split):
    s = sg.config_scene(4, n_envs=40)
    iters = 12
    ref = reference(s, iters)
    with vuda.World(s) as w:
        w.cosched(split)
        w.run(schedule, iters)
        w.render()  # a frame of the final state in every schedule
        w.wait()
        got = outputs(w)
    assert_same(ref, got, f"schedule {schedule} split {split}")


def test_toggle_cosched_mid_run():
    s = sg.config_scene(2, n_envs=64)
    ref = reference(s, 16)
    with vuda.World(s) as w:
        for k, split in enumerate([0.5, 0.0, 2.0, 0.25]):
            w.cosched(split)
            w.run(vuda.SCHED_INTERSTEP if k % 2 == 0 else vuda.SCHED_INTERTRAJ, 4)
        w.cosched(0.0)
        w.render()
        w.wait()
        assert_same(ref, outputs(w))


def test_graphs_replayed_in_cosched_mode():
    s = sg.config_scene(2, n_envs=64)
    ref = reference(s, 20)
    with vuda.World(s) as w:
        w.set_tuning(vuda.TUNE_GRAPHS, 1)
        w.cosched(0.5)
        for _ in range(10):
            w.run(vuda.SCHED_INTERSTEP, 2)
            w.wait()  # the host's own synchronisation between replays
        w.render()
        w.wait()
        assert_same(ref, outputs(w))


def _iter_seconds(w, st, schedule, iters=20, windows=5):
    """Median wall time of `iters` iterations of `schedule` from state st."""
    dts = []
    for _ in range(windows):
        w.load_state(st)
        w.run(schedule, 3)
        w.wait()
        t0 = time.perf_counter()
        w.run(schedule, iters)
        w.wait()
        dts.append(time.perf_counter() - t0)
    return sorted(dts)[len(dts) // 2]


@pytest.mark.parametrize("schedule", [vuda.SCHED_INTERSTEP, vuda.SCHED_PIPELINED])
def test_graph_replay_leaves_cosched_streams_concurrent(schedule):
    """A graph capture must not leave a stream behind that shares a hardware
    queue with the co-scheduled streams: two streams on one queue run one
    after the other, which once cost a third of the co-scheduled throughput
    after any graph replay.  The same iterations are timed before and after
    replaying graphs (results are checked elsewhere); the margin is far
    wider than the run-to-run noise of a few percent."""
    s = sg.config_scene(2)
    with vuda.World(s) as w:
        w.step(nsteps=250)  # the settled pile the bench times
        w.wait()
        st = w.state()
        w.cosched(2.0)
        before = _iter_seconds(w, st, schedule)
        w.set_tuning(vuda.TUNE_GRAPHS, 1)
        for _ in range(3):
            w.run(schedule, 2)
            w.wait()
        w.set_tuning(vuda.TUNE_GRAPHS, 0)
        w.cosched(2.0)
        after = _iter_seconds(w, st, schedule)
        if after >= 1.15 * before:  # a second sample before failing: a slow window is not the defect
            after = min(after, _iter_seconds(w, st, schedule))
    say(f"{vuda.SCHED_NAMES[schedule]}@2, 1024 envs: {before / 20 * 1e6:.1f} us/iteration before graph replay, "
        f"{after / 20 * 1e6:.1f} after")
    assert after < 1.15 * before


def test_cu_mask_partition():
    s = sg.config_scene(1, n_envs=2)
    with vuda.World(s) as w:
        nc = None
        for split in (0.25, 0.5):
            w.cosched(split)
            a = w.probe_placement(vuda.PHASE_STEP, 4096, 300)
            b = w.probe_placement(vuda.PHASE_RENDER, 4096, 300)
            sa, sb = set(map(tuple, a.tolist())), set(map(tuple, b.tolist()))
            assert not (sa & sb), "the two streams share a CU"
            total = len(sa) + len(sb)
            assert abs(len(sa) / total - split) < 0.02, (len(sa), len(sb))
            # spread over every XCD
            assert len(collections.Counter(a[:, 0].tolist())) == len(collections.Counter(b[:, 0].tolist()))
            say(f"split {split}: step CUs {len(sa)}, render CUs {len(sb)}")


def test_external_stream_handles():
    import torch
    torch.cuda.init()
    s = sg.config_scene(1, n_envs=4)
    with vuda.World(s) as w:
        w.cosched(0.5)
        w.render()
        st = torch.cuda.ExternalStream(w.stream(vuda.PHASE_RENDER), device=torch.device("cuda", 0))
        ev = torch.cuda.Event()
        ev.record(st)
        ev.synchronize()
        assert ev.query() and st.query()


def test_checkpoint_resume():
    s = sg.config_scene(2, n_envs=32)
    ref = reference(s, 30)
    with vuda.World(s) as w:
        for _ in range(12):
            w.step()
            w.render()
        mid = w.state()
    resumed = sg.Scene(**{**s.__dict__, "pos": mid["pos"], "vel": mid["vel"], "quat": mid["quat"],
                          "omega": mid["omega"]})
    with vuda.World(resumed) as w:
        for _ in range(18):
            w.step()
            w.render()
        w.wait()
        assert_same(ref, outputs(w))


def test_autotune_leaves_results_unchanged(tmp_path):
    s = sg.config_scene(2, n_envs=128)
    ref = reference(s, 10)
    cache = str(tmp_path / "tune.txt")
    with vuda.World(s) as w:
        r = w.autotune(steps=5, cache=cache)
        say(f"autotune: {r}")
        assert r["trials"] > 10 and r["cosched_env_steps_per_s"] > 0
        w.run(r["schedule"], 10)
        w.render()
        w.wait()
        assert_same(ref, outputs(w))
        r2 = w.autotune(steps=5, cache=cache)
        assert r2["trials"] == 0 and r2["schedule"] == r["schedule"]


def test_nonfinite_state_is_reported():
    s = sg.config_scene(1, n_envs=3)
    with vuda.World(s) as w:
        st = w.state()
        st["vel"][9, 2] = np.nan  # a body of env 1
        w.load_state(st)
        w.step()
        with pytest.raises(vuda.VudaError) as e:
            w.wait()
        assert e.value.code == vuda.ENUMERIC
        flags = w.fetch(vuda.FETCH_FLAGS)
        assert flags[1] & 1 and not flags[0] & 1 and not flags[2] & 1


def test_contact_capacity_overflow_is_reported():
    bodies = [dict(type=1, size=0.1, pos=(0.0, 0.0, 1.0)) for _ in range(64)]
    s = tiny_scene(bodies)
    with vuda.World(s) as w:
        w.step()
        with pytest.raises(vuda.VudaError) as e:
            w.wait()
        assert e.value.code == vuda.EOVERFLOW


def test_invalid_calls():
    s = sg.config_scene(1, n_envs=2)
    with vuda.World(s) as w:
        for bad in (lambda: w.step(0, 3), lambda: w.render(-1, 1), lambda: w.cosched(1.5),
                    lambda: w.set_tuning(vuda.TUNE_RASTER_THREADS, 100), lambda: w.run(7, 1),
                    lambda: w.set_tuning(vuda.TUNE_PHYS_PERSISTENT, -2),
                    lambda: w.set_tuning(vuda.TUNE_RASTER_PERSISTENT, -2)):
            with pytest.raises(vuda.VudaError) as e:
                bad()
            assert e.value.code == vuda.EINVAL
        # mixed parity inside one range is refused
        w.step(0, 1)
        with pytest.raises(vuda.VudaError):
            w.step(0, 2)


def test_launch_timing_counts_and_leaves_results_unchanged():
    s = sg.config_scene(2, n_envs=64)
    ref = reference(s, 6)
    with vuda.World(s) as w:
        w.set_tuning(vuda.TUNE_TIMING, 1)
        w.cosched(0.5)
        for _ in range(6):
            w.step()
            w.render()
        w.wait()
        t = {k: w.kernel_times(k) for k in (vuda.KERNEL_PHYSICS, vuda.KERNEL_RASTER_SETUP,
                                             vuda.KERNEL_RASTER_TILES)}
        say(f"timing: {t}")
        # with presetup every step ends with the setup of its new state
        for v in t.values():
            assert v["launches"] == 6
            assert 0 < v["max_ms"] <= v["total_ms"] < 1e4
        assert w.kernel_times(vuda.KERNEL_PHYSICS)["launches"] == 0  # read resets the count
        w.set_tuning(vuda.TUNE_TIMING, 0)
        assert_same(ref, outputs(w))


@pytest.mark.parametrize("presetup", [0, 1])
def test_setup_placement_and_reloaded_state(presetup):
    """The raster setup in the step or in the render gives the same frames,
    also for a state loaded from the host (rendered with its own setup)."""
    s = sg.config_scene(4, n_envs=24)
    ref = reference(s, 5)
    with vuda.World(s) as w:
        w.set_tuning(vuda.TUNE_PRESETUP, presetup)
        w.cosched(2.0)
        for _ in range(5):
            w.step()
            w.render()
        w.wait()
        assert_same(ref, outputs(w))
        st = w.state()
        w.load_state(st)
        w.render()
        w.wait()
        assert_same(ref, outputs(w))
        w.step(0, 12)  # half the envs step (and set up), the other half keep their setup
        w.step(12, 24)
        w.render()
        w.wait()
        with vuda.World(s) as w2:
            for _ in range(6):
                w2.step()
            w2.render()
            w2.wait()
            assert_same(outputs(w2), outputs(w))
