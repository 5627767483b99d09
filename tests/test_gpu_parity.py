"""GPU parity: the HIP path against the CPU oracle, through the C ABI.

Gates: contact-pair sets (sorted, every substep) bit-exact; body state within
1e-5 relative per component (floor 1) per step from identical input state;
raster coverage, winners and depth bit-exact; RGB within 1/255.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2605_01352_amd import scenegen as sg
from paper_2605_01352_amd import vuda
from tests.gpu_util import compare_render, compare_step, say
from tests.scenes import quat_axis_angle, tiny_scene

pytestmark = pytest.mark.gpu


def run_parity(scene, steps, render_every=1, label=""):
    with vuda.World(scene, debug=True) as w:
        exact = 0
        worst = 0.0
        for t in range(steps):
            if render_every and t % render_every == 0:
                compare_render(w, scene)
            r = compare_step(w, scene)
            exact += r["bitexact"]
            worst = max(worst, r["max_err"])
        compare_render(w, scene)
        say(f"{label}: {steps} steps, bit-exact steps {exact}/{steps}, max state err {worst:.3g}")
        return exact, worst


def test_c1_full_parity():
    """16 envs x 8 spheres, 64x64, 100 steps: every step and every frame."""
    s = sg.config_scene(1)
    run_parity(s, 100, render_every=1, label="c1")


def test_c2_subset_parity():
    """32 envs of the 1024-env config (same content), 40 steps."""
    s = sg.config_scene(2, n_envs=32)
    run_parity(s, 40, render_every=8, label="c2[0:32]")


def test_c3_subset_parity():
    """4 envs of the 4096-env config: 64 bodies, two 256x256 ring cameras."""
    s = sg.config_scene(3, n_envs=4)
    run_parity(s, 6, render_every=3, label="c3[0:4]")


def test_c4_subset_parity():
    """48 envs of the uneven config: 4..128 bodies, mixed resolutions."""
    s = sg.config_scene(4, n_envs=48)
    run_parity(s, 5, render_every=2, label="c4[0:48]")


def test_settled_pile_parity():
    """A c2 env after 400 oracle steps (bodies resting in contact)."""
    s = sg.config_scene(2, n_envs=2)
    st = s.state()
    for _ in range(400):
        oracle.step_scene(s, st)
    for k, v in st.items():
        getattr(s, k if k != "omega" else "omega")[:] = v
    run_parity(s, 10, render_every=5, label="settled")


def test_edge_cases():
    """0 bodies, 1 body, 65 bodies (two-wave workgroup), 128 bodies, non-square
    and non-multiple-of-16 images, a camera inside the scene."""
    mk = lambda n, t=lambda i: i % 2: [dict(type=t(i), size=0.05 + 0.01 * (i % 5),
                                             pos=(0.3 * math.cos(i), 0.3 * math.sin(i), 0.1 + 0.06 * i))
                                        for i in range(n)]
    scenes = []
    for n in (1, 65, 128):
        sc = tiny_scene(mk(n), res=40)
        scenes.append(sc)
    base = sg.Scene.concat(scenes)
    # one env with no bodies (ground only)
    empty = sg.Scene.concat([tiny_scene(mk(1), res=24)]).subset([0])
    empty = sg.Scene(body_off=np.array([0, 0], np.int32), btype=empty.btype[:0], size=empty.size[:0],
                     rbound=empty.rbound[:0], inv_m=empty.inv_m[:0], inv_I=empty.inv_I[:0],
                     albedo=empty.albedo[:0], pos=empty.pos[:0], vel=empty.vel[:0],
                     quat=empty.quat[:0], omega=empty.omega[:0], cam_off=empty.cam_off,
                     cam_vp=empty.cam_vp, cam_w=np.array([37], np.int32), cam_h=np.array([23], np.int32))
    full = sg.Scene.concat([base, empty])
    # non-square image and a camera among the bodies
    full.cam_w[1], full.cam_h[1] = 100, 61
    full.cam_vp[0] = sg.view_proj((0.2, 0.1, 0.3), target=(0.0, 0.0, 0.2)).reshape(16)
    run_parity(full, 4, render_every=2, label="edge")


def test_unbinned_images_parity():
    """Images whose tile bins exceed the allowed entries are rendered with
    every tile testing every visible triangle; same bits as the oracle."""
    s = sg.config_scene(4, n_envs=12)
    with vuda.World(s, debug=True) as w:
        w.set_tuning(vuda.TUNE_REC_CAP, 1)
        compare_render(w, s)
        for _ in range(3):
            w.step()
        compare_render(w, s)


def test_bit_exact_and_deterministic():
    """Two runs give identical bits; GPU equals oracle bit for bit on c1."""
    s = sg.config_scene(1)
    outs = []
    for _ in range(2):
        with vuda.World(s) as w:
            for _ in range(20):
                w.step()
                w.render()
            w.wait()
            outs.append((w.fetch(vuda.FETCH_STATE), w.fetch(vuda.FETCH_RGB), w.fetch(vuda.FETCH_DEPTH)))
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_tuning_knobs_do_not_change_outputs():
    s = sg.config_scene(4, n_envs=24)
    ref = None
    for knobs in ({}, {vuda.TUNE_RASTER_THREADS: 64}, {vuda.TUNE_RASTER_THREADS: 1024},
                  {vuda.TUNE_REC_CAP: 64}, {vuda.TUNE_REC_CAP: 5000}, {vuda.TUNE_PHYS_PERSISTENT: 7, vuda.TUNE_RASTER_PERSISTENT: 5},
                  {vuda.TUNE_GRAPHS: 1}, {vuda.TUNE_BROADPHASE: 1}, {vuda.TUNE_BROADPHASE: 2},
                  {vuda.TUNE_PHYS_PRIORITY: 3}, {vuda.TUNE_PRESETUP: 0},
                  {vuda.TUNE_PRESETUP: 0, vuda.TUNE_GRAPHS: 1}, {vuda.TUNE_RASTER_PERSISTENT: 3},
                  {vuda.TUNE_PHYS_ENVS_PER_WAVE: 2}, {vuda.TUNE_PHYS_ENVS_PER_WAVE: 2, vuda.TUNE_PHYS_PERSISTENT: 5},
                  {vuda.TUNE_TILE_SIZE: 8}, {vuda.TUNE_TILE_SIZE: 32},
                  {vuda.TUNE_TILE_SIZE: 32, vuda.TUNE_REC_CAP: 64},
                  {vuda.TUNE_RASTER_FUSED: 1}, {vuda.TUNE_RASTER_FUSED: 1, vuda.TUNE_RASTER_THREADS: 1024},
                  {vuda.TUNE_RASTER_FUSED: 1, vuda.TUNE_FUSED_LDS_RECORDS: 60},
                  {vuda.TUNE_RASTER_FUSED: 1, vuda.TUNE_TILE_SIZE: 8, vuda.TUNE_RASTER_PERSISTENT: 5},
                  {vuda.TUNE_TILE_WAVES: 1}, {vuda.TUNE_TILE_WAVES: 2, vuda.TUNE_TILE_SIZE: 8},
                  {vuda.TUNE_TILE_WAVES: 2, vuda.TUNE_RASTER_THREADS: 128, vuda.TUNE_GRAPHS: 1},
                  {vuda.TUNE_TILE_PRIORITY: 2, vuda.TUNE_PHYS_PRIORITY: 3}):
        with vuda.World(s) as w:
            for k, v in knobs.items():
                w.set_tuning(k, v)
            for _ in range(3):
                w.render()
                w.step()
            w.render()
            w.wait()
            out = (w.fetch(vuda.FETCH_STATE), w.fetch(vuda.FETCH_RGB), w.fetch(vuda.FETCH_DEPTH))
        if ref is None:
            ref = out
        else:
            for a, b in zip(ref, out):
                assert np.array_equal(a, b), f"knobs {knobs}"
        say(f"knobs {knobs}: identical")


def test_datagen_camera_640x480_parity():
    """The paper's data-generation camera shape: 640x480 (4:3, 40 x 30 tiles)
    over 4 envs of the 1024-env config, 3 steps, every frame compared."""
    s = sg.config_scene(2, n_envs=4)
    s.cam_w[:] = 640
    s.cam_h[:] = 480
    s.cam_vp[:] = sg.view_proj(sg.FIXED_EYE, aspect=640.0 / 480.0).reshape(1, 16)
    run_parity(s, 3, render_every=1, label="c2[0:4] at 640x480")


def test_near_plane_clipping_parity():
    """Cameras a few centimetres above the ground and inside a pile of
    bodies: the ground quad and nearby faces cross the near plane.  With
    VUDA_FLAG_NEAR_CLIP they are cut along it (one or two pieces each),
    without it culled whole; winners, depth and coverage bit-exact either
    way."""
    s = sg.config_scene(2, n_envs=6)
    eyes = [((0.0, 0.0, 0.03), (1.0, 0.2, -0.01)), ((0.3, -0.2, 0.02), (-1.0, 0.5, 0.05)),
            ((0.0, 0.0, 0.4), (0.3, 0.1, 0.0)), ((0.1, 0.1, 0.15), (0.0, 0.0, 0.0)),
            ((-0.2, 0.0, 0.06), (0.5, 0.0, 0.1)), ((0.05, -0.05, 0.25), (0.0, 0.3, 0.2))]
    for c, (eye, tgt) in enumerate(eyes):
        s.cam_vp[c] = sg.view_proj(eye, target=tgt).reshape(16)
    run_parity(s, 3, render_every=1, label="near-plane cameras, culled whole")
    s.near_clip = True
    run_parity(s, 6, render_every=1, label="near-plane cameras, cut")


def test_near_plane_piece_overflow_is_reported():
    """More pieces of near-plane cuts than an image keeps (64): 30 small
    spheres straddling the near plane inside the view.  The render reports
    VUDA_EOVERFLOW instead of drawing an image with pieces missing."""
    rng = np.random.default_rng(5)
    bodies = [dict(type=0, size=0.006, pos=(float(x), float(y), 0.95)) for x, y in rng.uniform(-0.02, 0.02, (30, 2))]
    vp = sg.view_proj((0.0, 0.0, 1.0), target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0))
    s = tiny_scene(bodies, res=64, vp=vp)
    s.near_clip = True
    with vuda.World(s) as w:
        w.render()
        with pytest.raises(vuda.VudaError) as err:
            w.wait()
        assert err.value.code == vuda.EOVERFLOW


@pytest.mark.parametrize("tile", [8, 32])
def test_tile_sizes_against_the_oracle(tile):
    """Raster tiles of 8x8 and 32x32 pixels (16x16 is the default every
    other test uses): winners, coverage and depth bit-exact and RGB within 1
    on c1, envs of c2 (spawn and settled), c3's 256^2 ring cameras, c4's
    mixed sizes, 640x480, a 100x61 image, smooth shading, and the tile size
    switched between steps of one world."""
    import dataclasses
    cases = [sg.config_scene(1, n_envs=4), sg.config_scene(2, n_envs=8), sg.config_scene(3, n_envs=2),
             sg.config_scene(4, n_envs=16), dataclasses.replace(sg.config_scene(2, n_envs=3), smooth=True)]
    wide = sg.config_scene(2, n_envs=2)
    wide.cam_w[:] = [640, 100]
    wide.cam_h[:] = [480, 61]
    wide.cam_vp[0] = sg.view_proj(sg.FIXED_EYE, aspect=640.0 / 480.0).reshape(16)
    cases.append(wide)
    for sc in cases:
        with vuda.World(sc, debug=True) as w:
            w.set_tuning(vuda.TUNE_TILE_SIZE, tile)
            compare_render(w, sc)
            for _ in range(60):
                w.step()
            compare_render(w, sc)
            w.set_tuning(vuda.TUNE_TILE_SIZE, 16)
            w.step()
            compare_render(w, sc)
            w.set_tuning(vuda.TUNE_TILE_SIZE, tile)
            compare_render(w, sc)
        say(f"tile {tile}: {sc.name} {sc.n_cams} frames bit-exact")
