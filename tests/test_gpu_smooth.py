"""Smooth shading on the GPU (VUDA_FLAG_SMOOTH) against the oracle: the
vertex normals of each pixel's winning triangle interpolated
perspective-correctly and Lambert-shaded.  Winners, depth and coverage are
bit-exact (they are flat shading's), RGB within 1/255."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2605_01352_amd import scenegen as sg
from paper_2605_01352_amd import vuda
from tests.gpu_util import check_images, say
from tests.scenes import quat_axis_angle, tiny_scene

pytestmark = pytest.mark.gpu


def _frames_match(scene, steps=0):
    with vuda.World(scene, debug=True) as w:
        if steps:
            w.step(nsteps=steps)
            w.wait()
        st = w.state()
        w.render()
        w.wait()
        rgb, dep = w.images(vuda.FETCH_RGB), w.images(vuda.FETCH_DEPTH)
        win, cov = w.images(vuda.FETCH_WINNERS), w.images(vuda.FETCH_COVERAGE)
    cams = range(scene.n_cams)
    worst = check_images(scene, cams, rgb, dep, {c: st for c in cams}, win, cov)
    return worst, rgb


@pytest.mark.parametrize("cfg,n_envs,steps", [(2, 24, 0), (2, 24, 200), (3, 6, 60), (4, 24, 100)])
def test_smooth_config_parity(cfg, n_envs, steps):
    """Envs of the 1024-, 4096- and 2048-env configs, at the spawn and after
    the drop, every frame (two 256^2 ring cameras at c3, mixed sizes at c4)."""
    oracle.lib()
    scene = dataclasses.replace(sg.config_scene(cfg, n_envs=n_envs), smooth=True)
    worst, rgb = _frames_match(scene, steps)
    flat_scene = dataclasses.replace(scene, smooth=False)
    _, rgb_flat = _frames_match(flat_scene, steps)
    differ = sum(int(np.any(a != b)) for a, b in zip(rgb, rgb_flat))
    say(f"smooth c{cfg}[0:{n_envs}] @{steps}: {scene.n_cams} frames, winners/depth/coverage bit-exact, "
        f"rgb max diff {worst}; {differ} frames differ from flat shading")
    assert differ > 0


def test_smooth_close_sphere_and_boxes():
    """A sphere filling much of a 128^2 view (large, steep triangles) next to
    a box and a cube; a 100x61 image (ragged tiles)."""
    oracle.lib()
    bodies = [dict(type=0, size=0.3, pos=(0.0, 0.0, 0.3), quat=quat_axis_angle((0.2, 0.4, 1.0), 0.8)),
              dict(type=2, ext=(0.15, 0.06, 0.04), pos=(0.35, 0.2, 0.05), quat=quat_axis_angle((0, 0, 1), 0.4)),
              dict(type=1, size=0.07, pos=(-0.3, -0.25, 0.07))]
    sc = tiny_scene(bodies, res=128, vp=sg.view_proj((0.55, -0.5, 0.7), target=(0.0, 0.0, 0.25)), envs=2)
    sc.cam_w[1], sc.cam_h[1] = 100, 61
    sc.smooth = True
    worst, _ = _frames_match(sc)
    say(f"smooth close sphere, box, cube: rgb max diff {worst}")


def test_smooth_with_near_clip_is_refused():
    sc = dataclasses.replace(sg.config_scene(1, n_envs=2), smooth=True, near_clip=True)
    with pytest.raises(vuda.VudaError):
        vuda.World(sc)
