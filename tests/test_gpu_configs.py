"""GPU parity at the full sizes of the three batch configurations.

Each config runs on the GPU from its spawn for its whole horizon in the
product world (no debug outputs), in the co-scheduled launch configuration
the bench's headline usually picks: the pipelined schedule on streams over
every CU, step priority 3, tile priority 1, setup workgroups of 128 threads,
tile workgroups of 2 waves.  At the first, middle and last step of that
trajectory every env is checked against the oracle from the GPU's own state
S_t:
  - one physics step: state within 1e-5 relative, and (from a debug world
    loaded with S_t) the contact-pair sets of all four substeps bit-exact,
    the debug world's S_t+1 bit-identical to the product world's;
  - the frames of S_t: depth bit-exact, RGB within 1/255, for every camera
    of c2 and c4 and for 256 seeded cameras of c3 (8,192 in all).
"""
import os

import numpy as np
import pytest

import oracle
from paper_2605_01352_amd import scenegen as sg
from paper_2605_01352_amd import vuda
from tests.gpu_util import STATE_KEYS, check_contacts, check_images, check_state, oracle_step_many, say

pytestmark = pytest.mark.gpu


def _sample_cams(scene, cfg):
    if cfg != 3:
        return np.arange(scene.n_cams)
    rng = np.random.default_rng(3003)
    return np.sort(rng.choice(scene.n_cams, 256, replace=False))


def _images(w, scene, cams, what):
    """Images of the listed cameras, fetched env by env."""
    ecam = np.searchsorted(scene.cam_off, cams, side="right") - 1
    out = {}
    for e in np.unique(ecam):
        imgs = w.images(what, lo=int(e), hi=int(e) + 1)
        for k, c in enumerate(range(int(scene.cam_off[e]), int(scene.cam_off[e + 1]))):
            out[c] = imgs[k]
    return {c: out[c] for c in cams}


@pytest.mark.parametrize("cfg,horizon", [(2, 500), (3, 200), (4, 300)])
def test_full_config_samples(cfg, horizon):
    oracle.lib()
    scene = sg.config_scene(cfg, workers=min(16, os.cpu_count() or 1))
    n = scene.n_envs
    samples = (0, horizon // 2, horizon - 1)
    cams = _sample_cams(scene, cfg)
    envs = range(n)
    with vuda.World(scene) as w, vuda.World(scene, debug=True) as wd:
        for k, v in ((vuda.TUNE_RASTER_THREADS, 128), (vuda.TUNE_TILE_WAVES, 2), (vuda.TUNE_PHYS_PRIORITY, 3),
                     (vuda.TUNE_TILE_PRIORITY, 1)):
            w.set_tuning(k, v)
        w.cosched(2.0)
        t = 0
        for ts in samples:
            if ts > t:
                w.run(vuda.SCHED_PIPELINED, ts - t)  # ts - t steps, each state rendered
                t = ts
            w.wait()
            st_t = w.state()
            # frames of S_t in the product kernels
            w.render()
            w.wait()
            rgb = _images(w, scene, cams, vuda.FETCH_RGB)
            dep = _images(w, scene, cams, vuda.FETCH_DEPTH)
            worst_rgb = check_images(scene, cams, rgb, dep, {c: st_t for c in cams})
            # one step from S_t: oracle, product world, debug world
            st_o, pairs_o = oracle_step_many(scene, st_t, envs)
            w.step()
            t += 1
            w.wait()
            st_g = w.state()
            err, exact = check_state(st_g, st_o, scene, envs)
            wd.load_state(st_t)
            wd.step()
            wd.wait()
            st_d = wd.state()
            for k in STATE_KEYS:
                assert np.array_equal(st_d[k], st_g[k]), f"debug world differs from the product world in {k}"
            npairs = check_contacts(wd.contacts(), pairs_o, envs, scene.substeps)
            say(f"c{cfg} step {ts}: {n} envs, {npairs} contact pairs over 4 substeps, state "
                f"{'bit-exact' if exact else f'max err {err:.3g}'}; {len(cams)} frames, depth bit-exact, "
                f"rgb max diff {worst_rgb}")
