"""Pins of the oracle's smooth shading (no GPU): the perspective-correct
interpolation of vertex normals against exact ray-triangle geometry in
float64, the rendered colours of a sphere close to the camera against an
independent float64 ray cast, and flat faces (equal vertex normals) against
flat shading."""
import math

import numpy as np
import pytest

import oracle
from paper_2605_01352_amd import scenegen as sg
from tests.scenes import quat_axis_angle, tiny_scene

W = H = 64


def _ray(vp, px, py, w=W, h=H):
    """Origin and direction (float64) of the ray through the centre of
    pixel (px, py): the points of NDC depth 0 and 1 unprojected."""
    inv = np.linalg.inv(np.asarray(vp, np.float64).reshape(4, 4))
    x = 2.0 * (px + 0.5) / w - 1.0
    y = 1.0 - 2.0 * (py + 0.5) / h
    a = inv @ np.array([x, y, 0.0, 1.0])
    b = inv @ np.array([x, y, 1.0, 1.0])
    a, b = a[:3] / a[3], b[:3] / b[3]
    return a, b - a


def _bary(o, d, tri):
    """Barycentric coordinates of the ray's hit on the plane of tri
    (3 x 3, float64)."""
    p0, p1, p2 = tri
    nrm = np.cross(p1 - p0, p2 - p0)
    t = np.dot(p0 - o, nrm) / np.dot(d, nrm)
    P = o + t * d
    T = np.stack([p0 - p2, p1 - p2], 1)
    ab = np.linalg.lstsq(T, P - p2, rcond=None)[0]
    return np.array([ab[0], ab[1], 1.0 - ab[0] - ab[1]])


def _clip_w(vp, p):
    m = np.asarray(vp, np.float64).reshape(4, 4)
    return float(m[3, :3] @ np.asarray(p, np.float64) + m[3, 3])


def test_weights_are_perspective_correct():
    """A triangle receding from 0.4 m to 3 m in depth: with the unit axes as
    its vertex normals, the interpolated normal is the direction of the
    perspective-correct weights, which must be the barycentric coordinates
    of the pixel ray's hit on the triangle (float64 geometry), within the
    24.8 snapping of the vertices.  Screen-space (affine) weights differ by
    far more."""
    vp = sg.view_proj((0.0, -1.0, 0.4), target=(0.0, 1.0, 0.2))
    world = [np.array(p, np.float32) for p in ((-0.6, -0.2, 0.0), (0.6, -0.2, 0.0), (0.0, 3.0, 0.0))]
    ok, X, Y, z, A = oracle.setup_triangle(*world, vp, W, H)
    assert ok
    order = (0, 2, 1)  # setup order of the face's vertices
    iw = np.array([1.0 / _clip_w(vp, world[k]) for k in order], np.float32)
    basis = np.eye(3, dtype=np.float32)
    worst = worst_affine = 0.0
    n = 0
    for py in range(H):
        for px in range(W):
            if not oracle.covers(X, Y, px, py):
                continue
            got = oracle.smooth_normal(X, Y, iw, basis, px, py).astype(np.float64)
            o, d = _ray(vp, px, py)
            beta = _bary(o, d, np.stack([np.asarray(world[k], np.float64) for k in order]))
            want = beta / np.linalg.norm(beta)
            worst = max(worst, float(np.abs(got - want).max()))
            Px, Py = 256 * px + 128, 256 * py + 128
            E = [(X[(k + 2) % 3] - X[(k + 1) % 3]) * (Py - Y[(k + 1) % 3]) -
                 (Y[(k + 2) % 3] - Y[(k + 1) % 3]) * (Px - X[(k + 1) % 3]) for k in range(3)]
            aff = np.array(E, np.float64)
            worst_affine = max(worst_affine, float(np.abs(aff / np.linalg.norm(aff) - want).max()))
            n += 1
    assert n > 300
    assert worst < 2e-3, worst
    assert worst_affine > 0.1, worst_affine


def _smooth_scene(bodies, vp, smooth=True):
    sc = tiny_scene(bodies, res=W, vp=vp)
    sc.smooth = smooth
    return sc


def _render(sc, light=None):
    rp = oracle._Render(light=light, smooth=sc.smooth)
    old = dict(oracle._RENDER)
    oracle._RENDER[(False, bool(sc.smooth))] = rp
    try:
        return oracle.render_image(sc, sc.state(), 0, debug=True)
    finally:
        oracle._RENDER.clear()
        oracle._RENDER.update(old)


def test_sphere_close_up_matches_float64_ray_cast():
    """A sphere of radius 0.35 m seen from 0.75 m away, turned, under an
    off-axis light.  For every pixel of the sphere: its winning face (from
    the oracle), the face's world vertices and vertex normals (the unit
    template vertices turned by R) in float64, the pixel ray's barycentric
    coordinates on the face, the normalized weighted normal, then Lambert
    shading: the oracle's colour within 1.  The same computation with
    screen-space weights misses it by more on some pixels."""
    q = quat_axis_angle((0.3, 0.5, 0.8), 0.9)
    centre = np.array((0.05, -0.02, 0.4))
    vp = sg.view_proj((0.5, -0.45, 0.75), target=tuple(centre))
    light = np.array([0.5, -0.6, 0.62])
    light /= np.linalg.norm(light)
    sc = _smooth_scene([dict(type=0, size=0.35, pos=tuple(centre), quat=q)], vp)
    out = _render(sc, light=tuple(light))
    t = sg.templates()
    R = np.array(_rot(np.asarray(sc.quat[0], np.float64)))
    P = np.asarray(sc.pos[0], np.float64)
    alb = sg.PALETTE[0].astype(np.float64)
    bad = bad_affine = n = 0
    for py in range(H):
        for px in range(W):
            f = int(out["winner"][py, px]) - 2
            if f < 0:
                continue
            vi = t.sphere_f[f]
            verts = [P + R @ (0.35 * t.sphere_v[k].astype(np.float64)) for k in vi]
            nrm = [R @ t.sphere_v[k].astype(np.float64) for k in vi]
            o, d = _ray(vp, px, py)
            beta = _bary(o, d, np.stack(verts))
            m = sum(b * nk for b, nk in zip(beta, nrm))
            lam = max(0.0, float(m / np.linalg.norm(m) @ light))
            want = np.rint(255 * alb * (0.2 + 0.8 * lam))
            bad += int(np.abs(out["rgb"][py, px].astype(int) - want).max() > 1)
            # screen-space weights: barycentric coordinates of the pixel
            # centre in the projected triangle
            scr = np.array([_project(vp, v) for v in verts])
            ba = _bary2(scr, np.array([px + 0.5, py + 0.5]))
            ma = sum(b * nk for b, nk in zip(ba, nrm))
            la = max(0.0, float(ma / np.linalg.norm(ma) @ light))
            bad_affine += int(np.abs(np.rint(255 * alb * (0.2 + 0.8 * la)) - want).max() > 1)
            n += 1
    assert n > 1000
    assert bad == 0, f"{bad} of {n} pixels off by more than 1"
    assert bad_affine > 0


def _rot(q):
    w, x, y, z = q
    return [[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
            [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
            [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]]


def _project(vp, p):
    c = np.asarray(vp, np.float64).reshape(4, 4) @ np.append(p, 1.0)
    return np.array([(c[0] / c[3] * 0.5 + 0.5) * W, (0.5 - c[1] / c[3] * 0.5) * H])


def _bary2(tri, p):
    a, b, c = tri
    T = np.stack([a - c, b - c], 1)
    l = np.linalg.solve(T, p - c)
    return np.array([l[0], l[1], 1.0 - l[0] - l[1]])


@pytest.mark.parametrize("kind", [1, 2])
def test_flat_faces_shade_as_flat(kind):
    """A cube or a box (equal normals at a face's vertices) and the ground:
    smooth shading gives the flat colours within 1, with the same winners,
    depth and coverage."""
    body = dict(type=kind, size=0.2, pos=(0.0, 0.0, 0.25), quat=quat_axis_angle((1.0, 2.0, 0.5), 0.7))
    if kind == 2:
        body["ext"] = (0.2, 0.12, 0.08)
    vp = sg.view_proj((1.1, -0.9, 1.0), target=(0.0, 0.0, 0.2))
    flat = _render(_smooth_scene([body], vp, smooth=False))
    smooth = _render(_smooth_scene([body], vp, smooth=True))
    for k in ("winner", "depth", "cover"):
        assert np.array_equal(flat[k], smooth[k]), k
    assert (flat["winner"] >= 2).sum() > 100
    assert np.abs(flat["rgb"].astype(int) - smooth["rgb"].astype(int)).max() <= 1


def test_smooth_sphere_changes_colour_inside_faces():
    """On a sphere the colour now varies inside a face (flat shading is
    constant per face): some face shows several colours."""
    vp = sg.view_proj((0.6, -0.5, 0.9), target=(0.0, 0.0, 0.3))
    body = dict(type=0, size=0.3, pos=(0.0, 0.0, 0.3))
    out = _render(_smooth_scene([body], vp))
    face = out["winner"]
    varied = 0
    for f in np.unique(face[face >= 2]):
        cols = {tuple(c) for c in out["rgb"][face == f].tolist()}
        varied += len(cols) > 2
    assert varied > 10
