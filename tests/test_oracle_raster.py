"""Pins of the raster oracle (no GPU): exact coverage counts, watertightness
of shared edges under the top-left rule, back-face culling of closed meshes,
closed-form depth of a view-aligned plane, and Lambert shading at n || L and
n perpendicular to L."""
import ctypes as C
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2605_01352_amd import scenegen as sg
from tests.scenes import tiny_scene


def expected_rect(x0, x1, y0, y1, W, H):
    """Pixel centres 256p+128 in the half-open box [x0,x1) x [y0,y1)."""
    cols = [p for p in range(W) if x0 <= 256 * p + 128 < x1]
    rows = [q for q in range(H) if y0 <= 256 * q + 128 < y1]
    return len(cols) * len(rows)


def coverage_grid(tris, W, H):
    cnt = np.zeros((H, W), np.int32)
    for X, Y in tris:
        for py in range(H):
            for px in range(W):
                cnt[py, px] += oracle.covers(X, Y, px, py)
    return cnt


@pytest.mark.parametrize("rect", [(128, 128 + 256 * 4, 128, 128 + 256 * 4),   # on pixel centres
                                  (0, 1024, 0, 1024),                          # on pixel corners
                                  (77, 1301, 300, 901)])                       # arbitrary
def test_rectangle_exact_count_and_single_coverage(rect):
    x0, x1, y0, y1 = rect
    W = H = 8
    t1 = (np.array([x0, x1, x1]), np.array([y0, y0, y1]))
    t2 = (np.array([x0, x1, x0]), np.array([y0, y1, y1]))
    cnt = coverage_grid([t1, t2], W, H)
    assert cnt.max() <= 1
    assert int(cnt.sum()) == expected_rect(x0, x1, y0, y1, W, H)
    if rect[0] == 128:
        assert int(cnt.sum()) == 16  # an exact 4x4 block of pixel centres


def test_watertight_random_grids():
    rng = np.random.default_rng(11)
    W = H = 6
    for trial in range(40):
        n = 4
        xs = np.linspace(0, 256 * W, n + 1)
        ys = np.linspace(0, 256 * H, n + 1)
        gx, gy = np.meshgrid(xs, ys)
        jitter = rng.integers(-100, 100, size=gx.shape)
        snap = rng.random(gx.shape) < 0.4      # many vertices exactly on pixel centres
        gx = np.where(snap, np.round((gx - 128) / 256) * 256 + 128, gx + jitter)
        gy = np.where(snap, np.round((gy - 128) / 256) * 256 + 128, gy + jitter.T)
        gx[:, 0], gx[:, -1], gy[0, :], gy[-1, :] = 0, 256 * W, 0, 256 * H
        gx, gy = gx.astype(np.int64), gy.astype(np.int64)
        tris = []
        for i in range(n):
            for j in range(n):
                a, b, c, d = (i, j), (i, j + 1), (i + 1, j + 1), (i + 1, j)
                for tri in ((a, b, c), (a, c, d)) if (i + j + trial) % 2 else ((a, b, d), (b, c, d)):
                    X = np.array([gx[v] for v in tri])
                    Y = np.array([gy[v] for v in tri])
                    A = (X[1] - X[0]) * (Y[2] - Y[0]) - (Y[1] - Y[0]) * (X[2] - X[0])
                    if A < 0:
                        X, Y = X[[0, 2, 1]], Y[[0, 2, 1]]
                    if A != 0:
                        tris.append((X, Y))
        cnt = coverage_grid(tris, W, H)
        assert cnt.min() == 1 and cnt.max() == 1, f"trial {trial}"


def _exact_inside(X, Y, px, py):
    """Independent test by exact barycentric coordinates (Cramer's rule) with
    the top-left tie rule on edges through the point."""
    P = (Fraction(256 * px + 128), Fraction(256 * py + 128))
    (x0, x1, x2), (y0, y1, y2) = [list(map(Fraction, X)), list(map(Fraction, Y))]
    det = (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0)
    l1 = ((P[0] - x0) * (y2 - y0) - (x2 - x0) * (P[1] - y0)) / det
    l2 = ((x1 - x0) * (P[1] - y0) - (P[0] - x0) * (y1 - y0)) / det
    l0 = 1 - l1 - l2
    edges = {0: ((x1, y1), (x2, y2)), 1: ((x2, y2), (x0, y0)), 2: ((x0, y0), (x1, y1))}
    for lam, k in ((l0, 0), (l1, 1), (l2, 2)):
        if lam < 0:
            return False
        if lam == 0:
            (ax, ay), (bx, by) = edges[k]
            dx, dy = bx - ax, by - ay
            if not (dy < 0 or (dy == 0 and dx > 0)):
                return False
    return True


def test_single_triangles_match_exact_barycentric():
    rng = np.random.default_rng(3)
    W = H = 8
    for _ in range(150):
        X = rng.integers(-300, 256 * W + 300, 3)
        Y = rng.integers(-300, 256 * H + 300, 3)
        if rng.random() < 0.5:  # put vertices on pixel centres to create ties
            X = (X // 256) * 256 + 128
            Y = (Y // 256) * 256 + 128
        A = (X[1] - X[0]) * (Y[2] - Y[0]) - (Y[1] - Y[0]) * (X[2] - X[0])
        if A == 0:
            continue
        if A < 0:
            X, Y = X[[0, 2, 1]], Y[[0, 2, 1]]
        for py in range(H):
            for px in range(W):
                assert oracle.covers(X, Y, px, py) == _exact_inside(X, Y, px, py)


def test_top_left_orientation():
    # triangle with a horizontal top edge through pixel-centre row 1 and a
    # horizontal bottom edge through row 5
    top = (np.array([0, 2048, 1024]), np.array([384, 384, 1408 + 1]))   # flat top at y=384 (row 1)
    assert oracle.covers(*top, 4, 1)          # on the flat top edge: covered
    bot = (np.array([1024, 2048, 0]), np.array([0, 1408, 1408]))       # flat bottom at y=1408 (row 5)
    A = (bot[0][1] - bot[0][0]) * (bot[1][2] - bot[1][0]) - (bot[1][1] - bot[1][0]) * (bot[0][2] - bot[0][0])
    assert A > 0
    assert not oracle.covers(*bot, 4, 5)      # on the flat bottom edge: not covered
    assert oracle.covers(*bot, 4, 4)


def _render(scene, light=None, debug=True):
    if light is not None:
        smooth = bool(getattr(scene, "smooth", False))
        rp = oracle._Render(light=light, smooth=smooth)
        old = dict(oracle._RENDER)
        oracle._RENDER[(False, smooth)] = rp
        try:
            return oracle.render_image(scene, scene.state(), 0, debug=debug)
        finally:
            oracle._RENDER.clear()
            oracle._RENDER.update(old)
    return oracle.render_image(scene, scene.state(), 0, debug=debug)


def _topdown(h, res=32):
    return sg.view_proj((0.0, 0.0, h), target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0))


def test_ground_depth_closed_form_and_watertight():
    h = 1.0
    sc = tiny_scene([dict(type=0, size=0.05, pos=(5.0, 5.0, 5.0))], vp=_topdown(h), res=32)
    out = _render(sc)
    n, f = sg.NEAR, sg.FAR
    D = round(f * (h - n) / (h * (f - n)) * (2 ** 24 - 1))
    assert np.abs(out["depth"].astype(np.int64) - D).max() <= 2
    assert (out["winner"] <= 1).all() and (out["winner"] >= 0).all()
    # the two ground triangles share a diagonal: every pixel exactly once
    assert (out["cover"] == 1).all()


def test_shading_parallel_and_perpendicular_light():
    sc = tiny_scene([dict(type=1, size=0.2, pos=(0.0, 0.0, 0.2))], vp=_topdown(1.5), res=32)
    out = _render(sc, light=(0.0, 0.0, 1.0))
    top = out["winner"] >= 2
    assert top.sum() > 50
    # n || L: the albedo itself
    expect = np.rint(sg.PALETTE[0] * 255).astype(int)
    assert np.abs(out["rgb"][top].astype(int) - expect).max() <= 1
    # ground, n || L
    assert np.abs(out["rgb"][~top].astype(int) - round(0.6 * 255)).max() <= 1
    # n perpendicular to L: ambient only
    out = _render(sc, light=(1.0, 0.0, 0.0))
    assert np.abs(out["rgb"][top].astype(int) - np.rint(0.2 * sg.PALETTE[0] * 255)).max() <= 1
    assert np.abs(out["rgb"][~top].astype(int) - round(0.12 * 255)).max() <= 1


def test_closed_meshes_cover_silhouette_once():
    # with back faces culled, a closed convex mesh covers each silhouette pixel
    # exactly once (plus the ground underneath)
    for t in (0, 1):
        sc = tiny_scene([dict(type=t, size=0.25, pos=(0.0, 0.0, 0.3),
                              quat=(0.9238795, 0.3826834, 0.0, 0.0))], vp=_topdown(1.5), res=48)
        out = _render(sc)
        body = out["winner"] >= 2
        assert body.sum() > 100
        assert (out["cover"][body] == 2).all()
        assert (out["cover"][~body] == 1).all()


def test_near_plane_and_guard_band_culling():
    vp = _topdown(1.0)
    ok, *_ = oracle.setup_triangle((0, 0, 0), (0.1, 0, 0), (0, 0.1, 0), vp, 64, 64)
    assert ok
    # a vertex behind the near plane culls the whole triangle
    ok, *_ = oracle.setup_triangle((0, 0, 0.99), (0.1, 0, 0), (0, 0.1, 0), vp, 64, 64)
    assert not ok
    # a vertex far outside the guard band
    ok, *_ = oracle.setup_triangle((0, 0, 0), (500.0, 0, 0), (0, 0.1, 0), vp, 64, 64)
    assert not ok
    # reversed winding (seen from below) is culled
    ok, *_ = oracle.setup_triangle((0, 0, 0), (0, 0.1, 0), (0.1, 0, 0), vp, 64, 64)
    assert not ok


def test_depth_ordering_nearer_body_wins():
    sc = tiny_scene([dict(type=0, size=0.1, pos=(0.0, 0.0, 0.1)),
                     dict(type=0, size=0.1, pos=(0.0, 0.0, 0.5))], vp=_topdown(1.5), res=32)
    out = _render(sc)
    c = out["winner"][16, 16]
    assert 2 + 80 <= c < 2 + 160  # the upper (nearer) sphere


def test_shading_of_a_rotated_cube_off_axis():
    """A cube turned 90 degrees about x, then 30 degrees about z, seen
    obliquely under an off-axis light.  Worked by hand: Rx(90) takes the body
    axes x, y, z to x, z, -y; Rz(30) then turns them about z, so the body's
    +x face looks along (cos 30, sin 30, 0), its +y face along (0, 0, 1) and
    its +z face along (sin 30, -cos 30, 0).  Each visible pixel of a face
    takes albedo * (0.2 + 0.8 max(0, n.L)) with that world normal.  A normal
    taken through the transposed rotation points elsewhere for every face
    and changes the colours."""
    c30, s30 = math.cos(math.radians(30)), math.sin(math.radians(30))
    c15, s15 = math.cos(math.radians(15)), math.sin(math.radians(15))
    c45 = s45 = math.sqrt(0.5)
    # q = qz(30) (x) qx(90), Hamilton product, w first
    quat = (c15 * c45, c15 * s45, s15 * s45, s15 * c45)
    world_n = {(0, 1): (c30, s30, 0.0), (1, 1): (0.0, 0.0, 1.0), (2, 1): (s30, -c30, 0.0)}
    for (k, s), n in list(world_n.items()):
        world_n[(k, -1)] = tuple(-x for x in n)
    light = np.array([0.5, -0.7, 0.5])
    light = light / np.linalg.norm(light)
    vp = sg.view_proj((1.1, -1.3, 1.2), target=(0.0, 0.0, 0.25))
    sc = tiny_scene([dict(type=1, size=0.2, pos=(0.0, 0.0, 0.25), quat=quat)], vp=vp, res=64)
    out = _render(sc, light=tuple(light))
    face = out["winner"] - 2
    t = sg.templates()
    alb = sg.PALETTE[0].astype(np.float64)
    seen = {}
    for f in range(12):
        px = face == f
        if not px.any():
            continue
        bn = t.cube_n[f]
        k = int(np.argmax(np.abs(bn)))
        n = np.array(world_n[(k, 1 if bn[k] > 0 else -1)])
        lam = max(0.0, float(n @ light))
        expect = np.rint(255 * alb * (0.2 + 0.8 * lam)).astype(int)
        assert np.abs(out["rgb"][px].astype(int) - expect).max() <= 1, (f, expect)
        seen[(k, int(np.sign(bn[k])))] = lam
    # three faces in view, lit differently: the body's +x, +y and +z faces,
    # whose world normals have a positive component toward the eye
    assert set(seen) == {(0, 1), (1, 1), (2, 1)}
    assert len({round(v, 3) for v in seen.values()}) == 3
