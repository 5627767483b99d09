"""Pins of near-plane clipping in the raster oracle (no GPU).

A triangle crossing the plane clip w = near is cut along it and the part in
front is drawn, as one or two triangles with the triangle's primitive id.
Checked against the geometry it must reproduce: a camera a few centimetres
above the ground quad sees exactly the pixels whose centre ray meets the
quad at a view depth of at least `near`, each covered once across the quad's
diagonal and the fan split (the cut point of a shared edge does not depend
on which triangle cuts it); and against the piece counts of the cases.
"""
import numpy as np

import oracle
from paper_2605_01352_amd import scenegen as sg
from tests.scenes import tiny_scene

N = sg.NEAR


def test_piece_counts():
    vp = sg.view_proj((0.0, 0.0, 1.0), target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0))
    a, b, c = (-0.3, -0.3, 0.0), (0.3, -0.3, 0.0), (0.0, 0.3, 0.0)
    full = oracle.setup_clipped(a, b, c, vp, 64, 64)
    ok, X, Y, z, A = oracle.setup_triangle(a, b, c, vp, 64, 64)
    assert ok and len(full) == 1
    assert np.array_equal(full[0][0], X) and np.array_equal(full[0][1], Y) and full[0][3] == A
    # one vertex lifted behind the near plane (the eye is at z = 1): a quad, two pieces
    assert len(oracle.setup_clipped(a, b, (0.0, 0.3, 0.99), vp, 64, 64)) == 2
    # two vertices behind: one piece
    assert len(oracle.setup_clipped((-0.3, -0.3, 0.99), b, (0.0, 0.3, 0.99), vp, 64, 64)) == 1
    # all behind: nothing
    assert len(oracle.setup_clipped((0, 0, 0.99), (0.1, 0, 0.99), (0, 0.1, 0.99), vp, 64, 64)) == 0
    # a vertex in front but outside the guard band culls the whole triangle
    assert len(oracle.setup_clipped((500.0, 0.0, 0.0), b, (0.0, 0.3, 0.99), vp, 64, 64)) == 0
    # a cut piece keeps the triangle's orientation: positive area, and its
    # cut vertices lie at depth about 0 (on the near plane)
    for X, Y, z, A in oracle.setup_clipped(a, b, (0.0, 0.3, 0.99), vp, 64, 64):
        assert A > 0
        assert np.min(z) < 1e-5


def test_ground_seen_from_just_above_is_cut_at_the_near_plane():
    W, H = 64, 48
    eye = np.array([0.0, 0.0, 0.03])
    vp32 = sg.view_proj(tuple(eye), target=(1.0, 0.2, -0.01), aspect=W / H)
    sc = tiny_scene([dict(type=0, size=0.01, pos=(5.0, 5.0, 0.01))], res=W, vp=vp32)
    sc.cam_w[:] = W
    sc.cam_h[:] = H
    sc.near_clip = True
    out = oracle.render_image(sc, sc.state(), 0, e=0, debug=True)
    cover, winner = out["cover"], out["winner"]
    vp = vp32.reshape(4, 4).astype(np.float64)
    inv = np.linalg.inv(vp)
    want = np.zeros((H, W), bool)
    margin = np.zeros((H, W), bool)  # centre rays too close to the boundary to call
    for py in range(H):
        for px in range(W):
            nx = (px + 0.5) / W * 2.0 - 1.0
            ny = 1.0 - (py + 0.5) / H * 2.0
            p0 = inv @ np.array([nx, ny, 0.0, 1.0])
            p1 = inv @ np.array([nx, ny, 1.0, 1.0])
            p0, p1 = p0[:3] / p0[3], p1[:3] / p1[3]
            d = p1 - p0
            if d[2] >= 0:
                continue
            t = -p0[2] / d[2]
            hit = p0 + t * d
            w = vp[3] @ np.append(hit, 1.0)
            inside = abs(hit[0]) <= 1.0 and abs(hit[1]) <= 1.0
            want[py, px] = inside and w >= N
            # within 1e-3 of the near plane or of the quad's sides: snapping
            # (1/256 pixel) may move the boundary across the centre
            margin[py, px] = abs(w - N) < 1e-3 or abs(abs(hit[0]) - 1.0) < 1e-2 or abs(abs(hit[1]) - 1.0) < 1e-2
    decided = ~margin
    assert want[decided].sum() > 300 and (~want[decided]).sum() > 100
    # every pixel seen is covered exactly once by the two ground triangles
    assert np.array_equal(cover[decided] == 1, want[decided])
    assert np.all(cover <= 1)
    assert np.all((winner[want & decided] == 0) | (winner[want & decided] == 1))
    # both ground triangles reach behind the camera: without the cut they
    # are culled whole and nothing is drawn
    sc.near_clip = False
    assert oracle.render_image(sc, sc.state(), 0, e=0, debug=True)["cover"].sum() == 0
    t = sg.templates()
    for f in t.ground_f:
        ok, *_ = oracle.setup_triangle(*[t.ground_v[i] for i in f], vp32, W, H)
        assert not ok
