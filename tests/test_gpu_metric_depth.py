"""GPU metric depth (VUDA_FETCH_DEPTH_METRIC) against the oracle's
conversion of its own rendering of the same seeded state: identical
background, and the view depth within one float32 ulp elsewhere (both sides
evaluate beta / (D / (2^24 - 1) - alpha) in float64 and round once)."""
import numpy as np
import pytest

import oracle
from paper_2605_01352_amd import scenegen as sg
from paper_2605_01352_amd import vuda
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def check(scene, label):
    with vuda.World(scene) as w:
        w.render()
        w.wait()
        got = w.images(vuda.FETCH_DEPTH_METRIC)
        dep = w.images(vuda.FETCH_DEPTH)
        torch = pytest.importorskip("torch")
        dev = torch.empty(w.fetch_bytes(vuda.FETCH_DEPTH_METRIC) // 4, dtype=torch.float32, device="cuda")
        w.fetch(vuda.FETCH_DEPTH_METRIC, out=dev)
        assert np.array_equal(dev.cpu().numpy(), np.concatenate([g.reshape(-1) for g in got]))
    st = scene.state()
    worst = 0
    for e in range(scene.n_envs):
        for c in range(int(scene.cam_off[e]), int(scene.cam_off[e + 1])):
            ref = oracle.render_image(scene, st, c, e=e)
            assert np.array_equal(dep[c], ref["depth"]), f"camera {c}: depth images differ"
            exp = oracle.metric_depth(ref["depth"], scene.cam_vp[c])
            fin = np.isfinite(exp)
            assert np.array_equal(np.isfinite(got[c]), fin)
            assert np.all(np.isposinf(got[c][~fin]))
            ulps = np.abs(got[c][fin].view(np.int32).astype(np.int64) - exp[fin].view(np.int32).astype(np.int64))
            worst = max(worst, int(ulps.max(initial=0)))
    assert worst <= 1
    say(f"{label}: metric depth within {worst} ulp of the oracle")


def test_metric_depth_c2():
    check(sg.config_scene(2, n_envs=16), "c2[0:16]")


def test_metric_depth_ring_cameras_and_640x480():
    s = sg.config_scene(3, n_envs=2)  # two 256x256 ring cameras per env
    check(s, "c3[0:2]")
    s = sg.config_scene(2, n_envs=2)
    s.cam_w[:] = 640
    s.cam_h[:] = 480
    s.cam_vp[:] = sg.view_proj(sg.FIXED_EYE, aspect=640.0 / 480.0).reshape(1, 16)
    check(s, "c2[0:2] at 640x480")


def test_metric_depth_needs_a_perspective():
    s = sg.config_scene(1, n_envs=2)
    # an orthographic-style matrix: constant w
    s.cam_vp[1] = np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 0.1, 0.5, 0, 0, 0, 1], np.float32)
    with vuda.World(s) as w:
        w.render()
        w.fetch(vuda.FETCH_DEPTH_METRIC, 0, 1)  # env 0 is fine
        with pytest.raises(vuda.VudaError):
            w.fetch(vuda.FETCH_DEPTH_METRIC)
