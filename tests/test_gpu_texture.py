"""Textures on the GPU (VUDA_FLAG_TEXTURE with VUDA_FLAG_SMOOTH) against the
oracle: the ground and cube and box faces take the texel (nearest,
repeating) at the perspective-correct texture coordinates of each pixel
centre.  Winners, depth and coverage are bit-exact, RGB within 1/255 (the
texel choice itself is exact: a different texel would show as a far larger
difference)."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2605_01352_amd import scenegen as sg
from paper_2605_01352_amd import vuda
from tests.gpu_util import check_images, say
from tests.scenes import quat_axis_angle, tiny_scene

pytestmark = pytest.mark.gpu


def _frames(scene, steps=0, knobs=None):
    with vuda.World(scene, debug=True) as w:
        for k, v in (knobs or {}).items():
            w.set_tuning(k, v)
        if steps:
            w.step(nsteps=steps)
            w.wait()
        st = w.state()
        w.render()
        w.wait()
        rgb, dep = w.images(vuda.FETCH_RGB), w.images(vuda.FETCH_DEPTH)
        win, cov = w.images(vuda.FETCH_WINNERS), w.images(vuda.FETCH_COVERAGE)
    return st, rgb, dep, win, cov


def _match(scene, steps=0, knobs=None):
    st, rgb, dep, win, cov = _frames(scene, steps, knobs)
    cams = range(scene.n_cams)
    worst = check_images(scene, cams, rgb, dep, {c: st for c in cams}, win, cov)
    return worst, rgb


@pytest.mark.parametrize("cfg,n_envs,steps", [(2, 24, 0), (2, 24, 200), (3, 6, 60), (4, 24, 100)])
def test_texture_config_parity(cfg, n_envs, steps):
    """Envs of the 1024-, 4096- and 2048-env configs with the procedural
    texture, at the spawn and after the drop, every frame."""
    oracle.lib()
    scene = sg.with_texture(sg.config_scene(cfg, n_envs=n_envs))
    worst, rgb = _match(scene, steps)
    plain = dataclasses.replace(scene, texture=None)
    _, rgb_plain, _, _, _ = _frames(plain, steps)
    differ = sum(int(np.any(a != b)) for a, b in zip(rgb, rgb_plain))
    say(f"texture c{cfg}[0:{n_envs}] @{steps}: {scene.n_cams} frames, winners/depth/coverage bit-exact, "
        f"rgb max diff {worst}; {differ} frames differ from untextured smooth shading")
    assert differ == scene.n_cams  # the ground is in every frame


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_texture_close_cubes_ragged_images(tile):
    """A turned cube and box close to an oblique camera over the textured
    ground (steep perspective), a 37 x 23 texture (not a power of two), a
    128^2 and a 100 x 61 image, at each tile size."""
    oracle.lib()
    bodies = [dict(type=1, size=0.2, pos=(0.0, 0.0, 0.2), quat=quat_axis_angle((0.2, 0.4, 1.0), 0.8)),
              dict(type=2, ext=(0.15, 0.06, 0.04), pos=(0.35, 0.2, 0.05), quat=quat_axis_angle((0, 0, 1), 0.4)),
              dict(type=0, size=0.07, pos=(-0.3, -0.25, 0.07))]
    sc = tiny_scene(bodies, res=128, vp=sg.view_proj((0.55, -0.5, 0.45), target=(0.0, 0.0, 0.1)), envs=2)
    sc.cam_w[1], sc.cam_h[1] = 100, 61
    sc = sg.with_texture(sc, sg.procedural_texture(37, 23, seed=7), ground_uv_scale=3.0)
    worst, _ = _match(sc, knobs={vuda.TUNE_TILE_SIZE: tile})
    say(f"texture close cube and box, tiles {tile}: rgb max diff {worst}")


def test_texture_is_refused_without_smooth_or_texels():
    sc = sg.config_scene(1, n_envs=2)
    with pytest.raises(vuda.VudaError) as e:
        vuda.World(dataclasses.replace(sc, smooth=False, texture=sg.procedural_texture()))
    assert e.value.code == vuda.EINVAL
    with pytest.raises(vuda.VudaError) as e:
        vuda.World(dataclasses.replace(sc, smooth=True, texture=np.zeros((0, 4, 3), np.uint8)))
    assert e.value.code == vuda.EINVAL
    with pytest.raises(vuda.VudaError) as e:
        vuda.World(sg.with_texture(sc, ground_uv_scale=float("inf")))
    assert e.value.code == vuda.EINVAL
