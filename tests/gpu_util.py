"""Helpers of the GPU parity tests: run the HIP path and the oracle from the
same input state and compare per the gates (contact sets and raster output
bit-exact, state within 1e-5 relative, colour within 1/255)."""
import sys

import numpy as np

import oracle
from paper_2605_01352_amd import vuda

STATE_KEYS = ("pos", "vel", "quat", "omega")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def state_close(g, o, rel=1e-5):
    """Per component |g - o| <= rel * max(|o|, 1); returns max normalised error."""
    worst = 0.0
    for k in STATE_KEYS:
        d = np.abs(g[k].astype(np.float64) - o[k].astype(np.float64))
        sc = np.maximum(np.abs(o[k].astype(np.float64)), 1.0)
        worst = max(worst, float((d / sc).max()) if d.size else 0.0)
    return worst


def state_equal(g, o):
    return all(np.array_equal(g[k], o[k]) for k in STATE_KEYS)


def oracle_step_from(scene, st_in, envs):
    """Oracle one step of `envs` from st_in (global arrays); returns (state, pairs)."""
    st = {k: v.copy() for k, v in st_in.items()}
    pairs = {}
    for e in envs:
        status, prs = oracle.step_env(scene, e, st, record_pairs=True)
        assert status == 0, f"oracle status {status} env {e}"
        pairs[e] = prs
    return st, pairs


def compare_step(world, scene, envs=None, rel=1e-5, expect_bitexact=True):
    """One GPU step of all envs vs the oracle from the same input state.

    Returns dict(max_err, bitexact).  Asserts contact sets equal and the
    state tolerance.
    """
    envs = range(scene.n_envs) if envs is None else envs
    st_in = world.state()
    st_o, pairs_o = oracle_step_from(scene, st_in, envs)
    world.step()
    world.wait()
    st_g = world.state()
    cts = world.contacts() if world.debug else None
    worst = 0.0
    exact = True
    for e in envs:
        b0, b1 = int(scene.body_off[e]), int(scene.body_off[e + 1])
        g = {k: st_g[k][b0:b1] for k in STATE_KEYS}
        o = {k: st_o[k][b0:b1] for k in STATE_KEYS}
        err = state_close(g, o)
        worst = max(worst, err)
        exact &= state_equal(g, o)
        if cts is not None:
            for s in range(scene.substeps):
                a = cts[e][s]
                b = pairs_o[e][s]
                assert a.shape == b.shape and np.array_equal(a, b), \
                    f"env {e} substep {s}: contact sets differ\nGPU {a.tolist()}\noracle {b.tolist()}"
    assert worst <= rel, f"state error {worst:.3g} > {rel}"
    return dict(max_err=worst, bitexact=exact, state_in=st_in, state_out=st_g)


def compare_render(world, scene, envs=None, state=None):
    """Render the world's current state on the GPU and with the oracle."""
    envs = range(scene.n_envs) if envs is None else list(envs)
    st = world.state() if state is None else state
    world.render()
    world.wait()
    rgb = world.images(vuda.FETCH_RGB)
    dep = world.images(vuda.FETCH_DEPTH)
    win = world.images(vuda.FETCH_WINNERS) if world.debug else None
    cov = world.images(vuda.FETCH_COVERAGE) if world.debug else None
    worst_rgb = 0
    for e in envs:
        for c in range(int(scene.cam_off[e]), int(scene.cam_off[e + 1])):
            ref = oracle.render_image(scene, st, c, e=e, debug=True)
            if win is not None:
                assert np.array_equal(cov[c].astype(np.int32), ref["cover"]), f"coverage env {e} cam {c}"
                assert np.array_equal(win[c].astype(np.int32), ref["winner"]), f"winners env {e} cam {c}"
            assert np.array_equal(dep[c], ref["depth"]), f"depth env {e} cam {c}"
            d = np.abs(rgb[c].astype(np.int32) - ref["rgb"].astype(np.int32)).max()
            assert d <= 1, f"rgb env {e} cam {c}: {d}"
            worst_rgb = max(worst_rgb, int(d))
    return worst_rgb


def _pool():
    from concurrent.futures import ThreadPoolExecutor
    import os
    return ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1))


def oracle_step_many(scene, st_in, envs):
    """oracle_step_from over many envs on a thread pool (the oracle's C
    calls release the interpreter lock; envs write disjoint slices)."""
    st = {k: v.copy() for k, v in st_in.items()}
    pairs = {}

    def one(e):
        status, prs = oracle.step_env(scene, e, st, record_pairs=True)
        assert status == 0, f"oracle status {status} env {e}"
        return e, prs

    with _pool() as ex:
        for e, prs in ex.map(one, list(envs)):
            pairs[e] = prs
    return st, pairs


def check_contacts(cts, pairs_o, envs, substeps, lo=0):
    """GPU contact sets (list indexed from env lo) against the oracle's."""
    n = 0
    for e in envs:
        for s in range(substeps):
            a, b = cts[e - lo][s], pairs_o[e][s]
            assert a.shape == b.shape and np.array_equal(a, b), \
                f"env {e} substep {s}: contact sets differ\nGPU {a.tolist()}\noracle {b.tolist()}"
            n += len(b)
    return n


def check_state(st_g, st_o, scene, envs, rel=1e-5):
    worst, exact = 0.0, True
    for e in envs:
        b0, b1 = int(scene.body_off[e]), int(scene.body_off[e + 1])
        g = {k: st_g[k][b0:b1] for k in STATE_KEYS}
        o = {k: st_o[k][b0:b1] for k in STATE_KEYS}
        worst = max(worst, state_close(g, o))
        exact &= state_equal(g, o)
    assert worst <= rel, f"state error {worst:.3g} > {rel}"
    return worst, exact


def check_images(scene, cams, rgb, dep, states, win=None, cov=None):
    """GPU images of cameras `cams` (dicts cam -> image) against oracle
    renders of states[cam] (the state each image shows): depth (and winners
    and coverage when given) bit-exact, RGB within 1."""
    def one(c):
        ref = oracle.render_image(scene, states[c], c, debug=win is not None)
        return c, ref

    worst = 0
    with _pool() as ex:
        for c, ref in ex.map(one, list(cams)):
            if win is not None:
                assert np.array_equal(cov[c].astype(np.int32), ref["cover"]), f"coverage cam {c}"
                assert np.array_equal(win[c].astype(np.int32), ref["winner"]), f"winners cam {c}"
            assert np.array_equal(dep[c], ref["depth"]), f"depth cam {c}"
            d = int(np.abs(rgb[c].astype(np.int32) - ref["rgb"].astype(np.int32)).max())
            assert d <= 1, f"rgb cam {c}: {d}"
            worst = max(worst, d)
    return worst


def env_of_cam(scene):
    return np.searchsorted(scene.cam_off, np.arange(scene.n_cams), side="right") - 1
