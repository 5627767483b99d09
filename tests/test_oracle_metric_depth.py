"""Pins of the metric-depth reading (no GPU).

The stored depth is z_ndc = far (d - near) / (d (far - near)) of the view
distance d, quantized to 24 bits.  oracle.metric_depth recovers d from the
view-projection alone; here it is checked against depths placed by hand under
cameras at arbitrary poses and aspects, against the near and far planes, and
end to end against the ray-plane intersection of the ground seen through each
pixel of an oracle rendering.
"""
import math

import numpy as np

import oracle
from paper_2605_01352_amd import scenegen as sg
from tests.scenes import tiny_scene

N, F = sg.NEAR, sg.FAR


def stored(d):
    """24-bit depth of view distance d (the definition, rounded to nearest)."""
    z = F * (d - N) / (d * (F - N))
    return np.rint(z * (2 ** 24 - 1)).astype(np.uint32)


def test_depths_placed_by_hand():
    rng = np.random.default_rng(3)
    d = np.concatenate([[N, F], np.exp(rng.uniform(math.log(N), math.log(F), 2000))])
    for eye, target, aspect in (((1.5, 0.0, 1.0), (0.0, 0.0, 0.3), 1.0), ((-0.3, 2.0, 0.4), (0.1, -0.2, 0.0), 4 / 3),
                                ((0.2, 0.1, 3.0), (0.0, 0.0, 0.0), 0.5)):
        vp = sg.view_proj(eye, target=target, aspect=aspect)
        got = oracle.metric_depth(stored(d), vp).astype(np.float64)
        # d = beta / (z - alpha) with beta = -F N / (F - N), alpha = F / (F - N).
        # Rounding z to the 24-bit code moves it by up to 2^-25: dd = d^2 / |beta| 2^-25.
        # The float32 matrix moves alpha by about 2^-23 alpha (dd = d^2 / |beta| dalpha),
        # and beta, the difference of two translation terms of size |t|, by about
        # 2 |t| 2^-24 (dd = d dbeta / |beta|).
        beta = F * N / (F - N)
        m = vp.reshape(4, 4).astype(np.float64)
        dalpha = 2.0 ** -23 * F / (F - N)
        dbeta = 2.0 ** -24 * (abs(m[2, 3]) + F / (F - N) * abs(m[3, 3]))
        bound = 1.01 * (d ** 2 / beta * (2.0 ** -25 + dalpha) + d * dbeta / beta) + 1e-9
        assert np.all(np.abs(got - d) <= bound)
    assert np.isinf(oracle.metric_depth(np.array([0xFFFFFFFF], np.uint32), vp)[0])
    # the planes themselves
    assert abs(float(oracle.metric_depth(np.array([0], np.uint32), vp)[0]) - N) < 1e-7
    assert abs(float(oracle.metric_depth(np.array([2 ** 24 - 1], np.uint32), vp)[0]) - F) < 1e-4


def test_ground_seen_through_each_pixel():
    """An oracle rendering of the bare ground quad: at every covered pixel
    the metric depth is the camera-axis distance of the point where the ray
    through the pixel centre meets z = 0, within the depth quantization plus
    the 1/256-pixel vertex snap times the local depth gradient."""
    W = H = 48
    sc = tiny_scene([dict(type=0, size=0.02, pos=(5.0, 5.0, 0.02))], res=W)
    vp = sc.cam_vp[0].reshape(4, 4).astype(np.float64)
    ref = oracle.render_image(sc, sc.state(), 0, e=0)
    dep = oracle.metric_depth(ref["depth"], sc.cam_vp[0]).astype(np.float64)
    inv = np.linalg.inv(vp)
    exact = np.full((H, W), np.nan)
    for py in range(H):
        for px in range(W):
            nx = (px + 0.5) / W * 2.0 - 1.0
            ny = 1.0 - (py + 0.5) / H * 2.0
            a = inv @ np.array([nx, ny, 0.0, 1.0])
            b = inv @ np.array([nx, ny, 1.0, 1.0])
            a, b = a[:3] / a[3], b[:3] / b[3]
            if (a[2] - b[2]) <= 0:
                continue
            t = a[2] / (a[2] - b[2])
            p = a + t * (b - a)
            if abs(p[0]) > 1.0 or abs(p[1]) > 1.0:
                continue
            exact[py, px] = vp[3] @ np.append(p, 1.0)
    inner = np.zeros((H, W), bool)
    inner[1:-1, 1:-1] = np.isfinite(exact[1:-1, 1:-1]) & np.isfinite(exact[:-2, 1:-1]) & np.isfinite(exact[2:, 1:-1]) \
        & np.isfinite(exact[1:-1, :-2]) & np.isfinite(exact[1:-1, 2:])
    assert inner.sum() > 500
    gy, gx = np.gradient(np.where(np.isfinite(exact), exact, 0.0))
    bound = (np.abs(gx) + np.abs(gy)) / 256.0 + exact ** 2 * (F - N) / (F * N) * 2.0 ** -22 + 1e-6
    err = np.abs(dep - exact)
    assert np.all(err[inner] <= bound[inner])
