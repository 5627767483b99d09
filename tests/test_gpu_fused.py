"""GPU parity of the fused raster path (VUDA_TUNE_RASTER_FUSED: the setup and
the tiles of an image in one workgroup, its records, bins and tile table in
LDS) with the oracle, and with the two-kernel path.

Gates as for every render: winners, coverage and depth bit-exact, RGB within
1/255.  Covered: tile sizes 8, 16 and 32 and workgroups of 256 to 1024
threads; the configs' image shapes (64^2 to 256^2, ring cameras, mixed
sizes), 640x480 and a ragged 100x61 image; images whose records do not fit
the LDS share asked for (through the raster scratch, binned and unbinned);
persistent launches and graph replay; and the full 1024-env config bit for
bit against the two-kernel path.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2605_01352_amd import scenegen as sg
from paper_2605_01352_amd import vuda
from tests.gpu_util import compare_render, say

pytestmark = pytest.mark.gpu


def _cases():
    cases = [("c1", sg.config_scene(1, n_envs=4)), ("c2", sg.config_scene(2, n_envs=8)),
             ("c3", sg.config_scene(3, n_envs=2)), ("c4", sg.config_scene(4, n_envs=16))]
    wide = sg.config_scene(2, n_envs=2)
    wide.cam_w[:] = [640, 100]
    wide.cam_h[:] = [480, 61]
    wide.cam_vp[0] = sg.view_proj(sg.FIXED_EYE, aspect=640.0 / 480.0).reshape(16)
    cases.append(("640x480 + 100x61", wide))
    return cases


def _fused_world(sc, knobs):
    w = vuda.World(sc, debug=True)
    w.set_tuning(vuda.TUNE_RASTER_FUSED, 1)
    for k, v in knobs.items():
        w.set_tuning(k, v)
    return w


@pytest.mark.parametrize("tile,threads", [(16, 256), (16, 512), (16, 1024), (8, 512), (32, 256)])
def test_fused_against_the_oracle(tile, threads):
    """Every case at the spawn and 60 steps later (bodies at rest)."""
    oracle.lib()
    for name, sc in _cases():
        with _fused_world(sc, {vuda.TUNE_TILE_SIZE: tile, vuda.TUNE_RASTER_THREADS: threads}) as w:
            compare_render(w, sc)
            w.step(nsteps=60)
            worst = compare_render(w, sc)
        say(f"fused tile {tile} threads {threads}: {name} matches the oracle (rgb max diff {worst})")


@pytest.mark.parametrize("knobs", [
    {vuda.TUNE_FUSED_LDS_RECORDS: 1},
    {vuda.TUNE_FUSED_LDS_RECORDS: 150},
    {vuda.TUNE_FUSED_LDS_RECORDS: 1, vuda.TUNE_REC_CAP: 1},
    {vuda.TUNE_REC_CAP: 1},
    {vuda.TUNE_RASTER_PERSISTENT: 5},
    {vuda.TUNE_RASTER_PERSISTENT: 40, vuda.TUNE_GRAPHS: 1, vuda.TUNE_FUSED_LDS_RECORDS: 150},
], ids=["all-through-scratch", "some-through-scratch", "scratch-unbinned", "lds-unbinned",
        "persistent", "persistent-graphs-mixed"])
def test_fused_fallbacks_and_launch_modes(knobs):
    """Records past the LDS share go through the raster scratch (1: every
    image with a visible triangle; 150: the larger images only), bins past
    their cap leave an image unbinned, and persistent or graph launches
    pull the images from a queue."""
    oracle.lib()
    for name, sc in _cases()[1:4]:
        with _fused_world(sc, knobs) as w:
            compare_render(w, sc)
            w.step(nsteps=40)
            compare_render(w, sc)
            w.step()
            compare_render(w, sc)
        say(f"fused {knobs}: {name} matches the oracle")


def test_fused_equals_two_kernels_full_c2():
    """The full 1024-env config, 20 render/step iterations from a state 250
    steps past the spawn: the fused path's state, RGB and depth equal the
    two-kernel path's bit for bit, also when the path changes between
    iterations (a step without its raster setup, rendered by two kernels)."""
    sc = sg.config_scene(2)
    outs = []
    for plan in ("two-kernel", "fused", "alternating"):
        with vuda.World(sc) as w:
            w.step(nsteps=250)
            for t in range(20):
                if plan != "two-kernel":
                    w.set_tuning(vuda.TUNE_RASTER_FUSED, 1 if plan == "fused" or t % 2 == 0 else 0)
                w.render()
                w.step()
            w.render()
            w.wait()
            outs.append((w.fetch(vuda.FETCH_STATE), w.fetch(vuda.FETCH_RGB), w.fetch(vuda.FETCH_DEPTH)))
    for plan, out in zip(("fused", "alternating"), outs[1:]):
        for a, b in zip(outs[0], out):
            assert np.array_equal(a, b), plan
    say("fused: full c2, 20 iterations, bit-identical to the two-kernel path (also alternating)")


def test_fused_keeps_two_kernels_where_it_does_not_apply():
    """Smooth shading and near-plane clipping keep the two kernels: with the
    knob on, their frames still match the oracle."""
    oracle.lib()
    smooth = dataclasses.replace(sg.config_scene(2, n_envs=4), smooth=True)
    clip = dataclasses.replace(sg.config_scene(2, n_envs=4), near_clip=True)
    for name, sc in (("smooth", smooth), ("near clip", clip)):
        with _fused_world(sc, {}) as w:
            compare_render(w, sc)
            w.step(nsteps=20)
            compare_render(w, sc)
        say(f"fused knob with {name}: two-kernel path, matches the oracle")
