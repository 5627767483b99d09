"""GPU parity with the oracle under every way the step loop can run.

The gates of the plain loop (contact-pair sets of every substep bit-exact,
state within 1e-5 relative from identical input, winners, coverage and depth
bit-exact, RGB within 1/255) are checked here at every iteration of:
  - the co-scheduled schedules on CU-masked streams (inter-trajectory at a
    37.5% split) and on two unmasked streams (inter-step, and
    inter-trajectory with raised step priority);
  - persistent launches with hipGraph replay (c2 and the uneven c4 mix);
  - the fused raster path (setup and tiles in one kernel);
  - the three-stage pipelined schedule, one iteration per call and many;
  - the configuration the autotuner picks;
  - the uniform-grid broadphase on settled piles of 100 and 128 bodies,
    automatic and forced, and its fallback for cells far from the origin;
  - the all-pairs broadphase's step candidate superset on a settled pile of
    64 bodies.
Each run starts from a state the GPU reached after a few hundred steps
(bodies resting in contact), not from the spawn.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2605_01352_amd import scenegen as sg
from paper_2605_01352_amd import vuda
from tests.gpu_util import (check_contacts, check_images, check_state, env_of_cam, oracle_step_many, say)
from tests.scenes import quat_axis_angle, tiny_scene

pytestmark = pytest.mark.gpu


def parity_iterations(w, scene, sched, iters, label):
    """`iters` iterations of schedule `sched` on world w (debug), each
    checked against the oracle from the GPU's own input state.  Returns the
    number of contact pairs seen."""
    n = scene.n_envs
    mid = (n + 1) // 2  # the inter-trajectory split of a world with every env active
    ecam = env_of_cam(scene)
    envs = range(n)
    pairs_seen = 0
    exact = 0
    worst = 0.0
    for t in range(iters):
        st_in = w.state()
        st_o, pairs_o = oracle_step_many(scene, st_in, envs)
        w.run(sched, 1)
        w.wait()
        st_g = w.state()
        pairs_seen += check_contacts(w.contacts(), pairs_o, envs, scene.substeps)
        err, ex = check_state(st_g, st_o, scene, envs)
        worst = max(worst, err)
        exact += ex
        # which state each image shows: rendered after its env's step (serial;
        # the first half of inter-trajectory) or before it
        after = np.zeros(n, bool)
        if sched == vuda.SCHED_SERIAL:
            after[:] = True
        elif sched == vuda.SCHED_INTERTRAJ:
            after[:mid] = True
        rgb, dep = w.images(vuda.FETCH_RGB), w.images(vuda.FETCH_DEPTH)
        win, cov = w.images(vuda.FETCH_WINNERS), w.images(vuda.FETCH_COVERAGE)
        states = {c: (st_g if after[ecam[c]] else st_in) for c in range(scene.n_cams)}
        check_images(scene, range(scene.n_cams), rgb, dep, states, win, cov)
    say(f"{label}: {iters} iterations, {pairs_seen} contact pairs, state bit-exact in {exact}/{iters}, "
        f"max err {worst:.3g}")
    assert pairs_seen > 0
    return pairs_seen


def settled_world(scene, settle, debug=True):
    """A world whose state is `settle` GPU steps past the spawn."""
    w = vuda.World(scene, debug=debug)
    if settle:
        w.step(nsteps=settle)
        w.wait()
    return w


C2 = dict(cfg=2, n_envs=48, settle=250)


@pytest.mark.parametrize("label,split,sched,knobs", [
    ("serialized", 0.0, vuda.SCHED_SERIAL, {}),
    ("CU-masked 0.375, inter-trajectory", 0.375, vuda.SCHED_INTERTRAJ, {}),
    ("CU-masked 0.5, inter-step", 0.5, vuda.SCHED_INTERSTEP, {}),
    ("unmasked, inter-step", 2.0, vuda.SCHED_INTERSTEP, {}),
    ("unmasked, inter-trajectory, step priority 3", 2.0, vuda.SCHED_INTERTRAJ, {vuda.TUNE_PHYS_PRIORITY: 3}),
    ("persistent launches + graphs, CU-masked 0.5, inter-step", 0.5, vuda.SCHED_INTERSTEP,
     {vuda.TUNE_PHYS_PERSISTENT: 24, vuda.TUNE_RASTER_PERSISTENT: 40, vuda.TUNE_GRAPHS: 1}),
    ("persistent launches + graphs, unmasked, inter-trajectory", 2.0, vuda.SCHED_INTERTRAJ,
     {vuda.TUNE_PHYS_PERSISTENT: 256, vuda.TUNE_RASTER_PERSISTENT: 256, vuda.TUNE_GRAPHS: 1}),
    ("persistent grids of the resident workgroups + graphs, unmasked, inter-step", 2.0, vuda.SCHED_INTERSTEP,
     {vuda.TUNE_PHYS_PERSISTENT: vuda.PERSISTENT_RESIDENT, vuda.TUNE_RASTER_PERSISTENT: vuda.PERSISTENT_RESIDENT,
      vuda.TUNE_GRAPHS: 1}),
    ("two envs per physics wave, unmasked, inter-step", 2.0, vuda.SCHED_INTERSTEP,
     {vuda.TUNE_PHYS_ENVS_PER_WAVE: 2}),
    ("two envs per physics wave, persistent, CU-masked 0.375, inter-trajectory", 0.375, vuda.SCHED_INTERTRAJ,
     {vuda.TUNE_PHYS_ENVS_PER_WAVE: 2, vuda.TUNE_PHYS_PERSISTENT: 7}),
    ("fused raster, unmasked, inter-step", 2.0, vuda.SCHED_INTERSTEP, {vuda.TUNE_RASTER_FUSED: 1}),
    ("setup workgroups of 128, tile workgroups of 2 waves, unmasked, inter-step", 2.0, vuda.SCHED_INTERSTEP,
     {vuda.TUNE_RASTER_THREADS: 128, vuda.TUNE_TILE_WAVES: 2}),
    ("tile workgroups of 1 wave, CU-masked 0.5, inter-trajectory", 0.5, vuda.SCHED_INTERTRAJ,
     {vuda.TUNE_TILE_WAVES: 1}),
    ("tile wave priority 1, setup workgroups of 128, unmasked, inter-step", 2.0, vuda.SCHED_INTERSTEP,
     {vuda.TUNE_TILE_PRIORITY: 1, vuda.TUNE_RASTER_THREADS: 128, vuda.TUNE_TILE_WAVES: 4}),
    ("pipelined, unmasked", 2.0, vuda.SCHED_PIPELINED, {}),
    ("pipelined, CU-masked 0.5", 0.5, vuda.SCHED_PIPELINED, {}),
    ("pipelined, persistent + graphs, setup workgroups of 128", 2.0, vuda.SCHED_PIPELINED,
     {vuda.TUNE_PHYS_PERSISTENT: 24, vuda.TUNE_RASTER_PERSISTENT: 40, vuda.TUNE_GRAPHS: 1,
      vuda.TUNE_RASTER_THREADS: 128}),
    ("pipelined with the fused raster (inter-step order)", 2.0, vuda.SCHED_PIPELINED, {vuda.TUNE_RASTER_FUSED: 1}),
    ("fused raster 512 threads, serialized", 0.0, vuda.SCHED_SERIAL,
     {vuda.TUNE_RASTER_FUSED: 1, vuda.TUNE_RASTER_THREADS: 512}),
    ("fused raster, persistent + graphs, CU-masked 0.375, inter-trajectory", 0.375, vuda.SCHED_INTERTRAJ,
     {vuda.TUNE_RASTER_FUSED: 1, vuda.TUNE_RASTER_PERSISTENT: 20, vuda.TUNE_GRAPHS: 1}),
    ("fused raster, resident persistent grid, two envs per physics wave on a resident grid", 2.0,
     vuda.SCHED_INTERSTEP, {vuda.TUNE_RASTER_FUSED: 1, vuda.TUNE_RASTER_PERSISTENT: vuda.PERSISTENT_RESIDENT,
                            vuda.TUNE_PHYS_ENVS_PER_WAVE: 2, vuda.TUNE_PHYS_PERSISTENT: vuda.PERSISTENT_RESIDENT}),
])
def test_c2_schedule_parity(label, split, sched, knobs):
    """48 envs of the 1024-env config, 250 steps past the spawn (a settled
    pile), then 6 co-scheduled iterations checked against the oracle."""
    oracle.lib()
    scene = sg.config_scene(C2["cfg"], n_envs=C2["n_envs"])
    with settled_world(scene, C2["settle"]) as w:
        for k, v in knobs.items():
            w.set_tuning(k, v)
        w.cosched(split)
        parity_iterations(w, scene, sched, 6, f"c2[0:48] @250, {label}")


@pytest.mark.parametrize("split,knobs", [
    (2.0, {}),
    (0.5, {}),
    (2.0, {vuda.TUNE_PHYS_PERSISTENT: 24, vuda.TUNE_RASTER_PERSISTENT: 40, vuda.TUNE_GRAPHS: 1}),
    (0.0, {}),
], ids=["unmasked", "cu-masked", "persistent-graphs", "one-stream"])
def test_pipelined_runs(split, knobs):
    """Many iterations in one pipelined call (the stages of consecutive
    iterations overlap): 11 iterations from a settled state, then 3 single
    iterations checked against the oracle, then a mix with plain step and
    render calls; state and frames bit-identical to a serialized world that
    made the same iterations."""
    oracle.lib()
    scene = sg.config_scene(C2["cfg"], n_envs=C2["n_envs"])
    with settled_world(scene, C2["settle"]) as w, settled_world(scene, C2["settle"]) as ref:
        for k, v in knobs.items():
            w.set_tuning(k, v)
        w.cosched(split)
        w.run(vuda.SCHED_PIPELINED, 11)
        parity_iterations(w, scene, vuda.SCHED_PIPELINED, 3, f"c2[0:48] @250, pipelined after 11, split {split}")
        w.run(vuda.SCHED_PIPELINED, 4)
        w.step()
        w.render()
        w.run(vuda.SCHED_PIPELINED, 2)
        w.wait()
        for _ in range(11 + 3 + 4):
            ref.render()
            ref.step()
        ref.step()
        ref.render()
        for _ in range(2):
            ref.render()
            ref.step()
        ref.wait()
        for what in (vuda.FETCH_STATE, vuda.FETCH_RGB, vuda.FETCH_DEPTH):
            assert np.array_equal(w.fetch(what), ref.fetch(what)), what
        say(f"pipelined, split {split} {knobs}: 25 iterations bit-identical to the serialized loop")


@pytest.mark.parametrize("phys_grid,raster_grid", [(32, 64), (vuda.PERSISTENT_RESIDENT, vuda.PERSISTENT_RESIDENT)],
                         ids=["fixed-grids", "resident-grids"])
def test_c4_persistent_graph_parity(phys_grid, raster_grid):
    """The uneven config as it is meant to run: one persistent launch per
    phase, hipGraph-captured steps, on CU-masked streams.  64 envs of 4..128
    bodies and 64^2..256^2 frames, 150 steps past the spawn; persistent grids
    of fixed sizes, or of the workgroups the GPU holds at once."""
    oracle.lib()
    scene = sg.config_scene(4, n_envs=64)
    with settled_world(scene, 150) as w:
        for k, v in ((vuda.TUNE_PHYS_PERSISTENT, phys_grid), (vuda.TUNE_RASTER_PERSISTENT, raster_grid),
                     (vuda.TUNE_GRAPHS, 1)):
            w.set_tuning(k, v)
        w.cosched(0.5)
        parity_iterations(w, scene, vuda.SCHED_INTERTRAJ, 5,
                          f"c4[0:64] @150, persistent grids {phys_grid}/{raster_grid} + graphs")


def test_autotuned_choice_parity():
    """Whatever the autotuner picks (schedule, split, launch shapes), the
    run under it meets the oracle's gates."""
    oracle.lib()
    scene = sg.config_scene(2, n_envs=64)
    with settled_world(scene, 200) as w:
        choice = w.autotune(steps=6)
        say(f"autotuned: {choice}")
        sched = int(choice["schedule"])
        parity_iterations(w, scene, sched, 4, f"c2[0:64] @200, autotuned {vuda.SCHED_NAMES[sched]}")


def _pile(n, seed, offset=(0.0, 0.0), mu=0.0):
    """n bodies (spheres and turned cubes alternating, sizes 3.5-5.5 cm) on a
    jittered lattice of 0.2 m, layers of 36, thrown toward the middle and
    settled by 600 oracle steps (2.5 s).  Without friction they slide apart
    into one layer with a few bodies touching; with mu = 0.6 they stay piled
    (about one body-body contact per body)."""
    rng = np.random.default_rng(seed)
    bodies = []
    for i in range(n):
        layer, k = divmod(i, 36)
        gx, gy = divmod(k, 6)
        a = float(rng.uniform(0.035, 0.055))
        pos = (-0.5 + 0.2 * gx + float(rng.uniform(-0.004, 0.004)) + offset[0],
               -0.5 + 0.2 * gy + float(rng.uniform(-0.004, 0.004)) + offset[1], 0.1 + 0.2 * layer)
        bodies.append(dict(type=i % 2, size=a, pos=pos,
                           quat=quat_axis_angle(rng.normal(size=3), float(rng.uniform(0, math.pi)))))
    sc = tiny_scene(bodies, res=64, mu=mu, vp=sg.view_proj((1.2 + offset[0], offset[1], 1.0),
                                                           target=(offset[0], offset[1], 0.2)))
    # lean the layers toward the middle so that the bodies meet
    sc.vel[:, 0] = -1.2 * (sc.pos[:, 0] - offset[0])
    sc.vel[:, 1] = -1.2 * (sc.pos[:, 1] - offset[1])
    st = sc.state()
    for _ in range(600):
        oracle.step_scene(sc, st)
    sc.pos[:], sc.vel[:], sc.quat[:], sc.omega[:] = st["pos"], st["vel"], st["quat"], st["omega"]
    return sc


@pytest.mark.parametrize("mu", [0.0, 0.6])
@pytest.mark.parametrize("n", [100, 128])
@pytest.mark.parametrize("broadphase", [0, 1, 2])
def test_grid_broadphase_settled_pile(n, broadphase, mu):
    """A settled pile of 100 or 128 bodies (two-wave workgroups), with and
    without friction: automatic (grid above 64 bodies), forced grid and
    forced all-pairs broadphase give the oracle's contact sets in every
    substep, body-body contacts among them."""
    oracle.lib()
    scene = _pile(n, 40 + n, mu=mu)
    st = scene.state()
    _, pr = oracle.step_env(scene, 0, st, record_pairs=True)
    body_pairs = int((pr[0][:, 1] != vuda.GROUND).sum())
    assert body_pairs >= (40 if mu else 5)
    with vuda.World(scene, debug=True) as w:
        w.set_tuning(vuda.TUNE_BROADPHASE, broadphase)
        parity_iterations(w, scene, vuda.SCHED_SERIAL, 5,
                          f"pile of {n}, mu {mu}, broadphase {broadphase} ({body_pairs} body pairs in contact)")


@pytest.mark.parametrize("broadphase", [0, 2])
def test_step_superset_settled_pile(broadphase):
    """A pile of 64 bodies settled with friction (one wave per env, the
    all-pairs broadphase with the step's candidate superset: substeps after
    the first retest only the pairs found within the margin at the step's
    start, while no body has moved a quarter of it -- every body here is
    slower than 1 m/s): contact sets of every substep and the state
    bit-exact with the oracle over 5 steps."""
    oracle.lib()
    scene = _pile(64, 104, mu=0.6)
    st = scene.state()
    _, pr = oracle.step_env(scene, 0, st, record_pairs=True)
    body_pairs = int((pr[0][:, 1] != vuda.GROUND).sum())
    assert body_pairs >= 5
    assert float(np.abs(scene.vel).max()) < 1.0
    with vuda.World(scene, debug=True) as w:
        w.set_tuning(vuda.TUNE_BROADPHASE, broadphase)
        parity_iterations(w, scene, vuda.SCHED_SERIAL, 5,
                          f"pile of 64, mu 0.6, broadphase {broadphase} ({body_pairs} body pairs in contact)")


def test_grid_far_from_origin_falls_back():
    """The same pile 600 m from the origin: its grid cells lie beyond +-1000
    cells, every wave of the env takes the all-pairs fallback together, and
    the contact sets stay the oracle's."""
    oracle.lib()
    scene = _pile(100, 140, offset=(600.0, -600.0), mu=0.6)
    with vuda.World(scene, debug=True) as w:
        w.set_tuning(vuda.TUNE_BROADPHASE, 1)
        parity_iterations(w, scene, vuda.SCHED_SERIAL, 4, "pile of 100 at (600, -600), forced grid")


@pytest.mark.parametrize("n_envs", [1, 7, 33])
def test_two_envs_per_wave_uneven(n_envs):
    """Two envs per physics wave over envs of 4..32 bodies of different
    sizes (the uneven config's small envs), an odd count leaving one half of
    the last wave empty, forced grid and all-pairs broadphase, friction."""
    oracle.lib()
    base = sg.config_scene(4, n_envs=200)
    small = [e for e in range(base.n_envs) if base.counts()[e] <= 32][:n_envs]
    scene = base.subset(small)
    for bp, mu in ((0, 0.0), (1, 0.0), (2, 0.5)):
        import dataclasses
        sc = dataclasses.replace(scene, mu=mu)
        with settled_world(sc, 120) as w:
            w.set_tuning(vuda.TUNE_PHYS_ENVS_PER_WAVE, 2)
            w.set_tuning(vuda.TUNE_BROADPHASE, bp)
            parity_iterations(w, sc, vuda.SCHED_SERIAL, 3, f"{n_envs} small envs, two per wave, broadphase {bp}, mu {mu}")
