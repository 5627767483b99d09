"""Pins of the texture reading (no GPU).

A textured world (smooth shading plus a texture) multiplies a pixel's albedo
by the texel (nearest, repeating) at the perspective-correct texture
coordinates of the pixel centre.  The ground's coordinates are its world
(x, y) times a scale; a cube face maps its unit square over the two tangent
axes of the body frame; spheres are not textured.  The pins check the
oracle's texels against ray casts done here in float64: the ground seen
obliquely (where an affine, screen-space interpolation would pick other
texels), a cube face seen from above split into its four texels, the same
cube turned a quarter turn, and the untextured spheres.
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle
from paper_2605_01352_amd import scenegen as sg
from tests.scenes import quat_axis_angle, tiny_scene


def coord_texture(w, h):
    """Texel (i, j) has colour (16 i + 8, 24 j + 12, 77): every texel differs."""
    t = np.zeros((h, w, 3), np.uint8)
    t[..., 0] = (16 * np.arange(w) + 8)[None, :]
    t[..., 1] = (24 * np.arange(h) + 12)[:, None]
    t[..., 2] = 77
    return t


def textured(scene, tex, scale=1.0):
    return dataclasses.replace(scene, smooth=True, texture=tex, ground_uv_scale=scale)


def ray_hits(vp, W, H, plane_z):
    """Per pixel centre, the float64 point where its ray meets z = plane_z
    (NaN where it does not, in front of the camera)."""
    inv = np.linalg.inv(vp.reshape(4, 4).astype(np.float64))
    out = np.full((H, W, 3), np.nan)
    for py in range(H):
        for px in range(W):
            nx = (px + 0.5) / W * 2.0 - 1.0
            ny = 1.0 - (py + 0.5) / H * 2.0
            a = inv @ np.array([nx, ny, 0.0, 1.0])
            b = inv @ np.array([nx, ny, 1.0, 1.0])
            a, b = a[:3] / a[3], b[:3] / b[3]
            if (a[2] - plane_z) * (b[2] - plane_z) >= 0:
                continue
            t = (a[2] - plane_z) / (a[2] - b[2])
            out[py, px] = a + t * (b - a)
    return out


def shade(albedo, t, normal):
    """The colour formula in float32, in the oracle's order of operations."""
    L = np.asarray(sg.LIGHT, np.float32)
    n = np.asarray(normal, np.float32)
    lam = np.float32(max(np.float32(0.0), (n[0] * L[0] + n[1] * L[1]) + n[2] * L[2]))
    s = np.float32(0.2) + np.float32(0.8) * lam
    col = (np.asarray(albedo, np.float32) * np.asarray(t, np.float32)) * s
    return np.minimum(np.float32(255.0), np.rint(col * np.float32(255.0))).astype(np.uint8)


def texel_index(U, V, w, h):
    U, V = np.nan_to_num(U), np.nan_to_num(V)
    fu, fv = U - np.floor(U), V - np.floor(V)
    return np.minimum((fu * w).astype(np.int64), w - 1), np.minimum((fv * h).astype(np.int64), h - 1)


def test_ground_texels_match_a_ray_cast_not_an_affine_map():
    W = H = 64
    Tw, Th, scale = 16, 8, 1.5
    tex = coord_texture(Tw, Th)
    sc = textured(tiny_scene([dict(type=0, size=0.02, pos=(5.0, 5.0, 0.02))], res=W), tex, scale)
    out = oracle.render_image(sc, sc.state(), 0, e=0, debug=True)
    ground = (out["winner"] >= 0) & (out["winner"] < 2)
    p = ray_hits(sc.cam_vp[0], W, H, 0.0)
    U, V = p[..., 0] * scale, p[..., 1] * scale
    ii, jj = texel_index(U, V, Tw, Th)
    # texels per pixel, from the neighbours; the vertex snap (1/256 pixel)
    # and float32 interpolation move a pixel's coordinates by far less
    du = np.abs(np.gradient(U * Tw)[0]) + np.abs(np.gradient(U * Tw)[1])
    dv = np.abs(np.gradient(V * Th)[0]) + np.abs(np.gradient(V * Th)[1])
    fu, fv = (U * Tw) % 1.0, (V * Th) % 1.0
    safe = ground & np.isfinite(U) & (np.minimum(fu, 1 - fu) > 0.01 + du / 64) & \
        (np.minimum(fv, 1 - fv) > 0.01 + dv / 64)
    assert safe.sum() > 1500
    got = out["rgb"]
    # the texel: its red and green channels name it (albedo and shading scale them alike)
    exp = np.zeros((H, W, 3), np.uint8)
    ga = [sg.GROUND_ALBEDO] * 3
    for py, px in zip(*np.nonzero(safe)):
        t = tex[jj[py, px], ii[py, px]].astype(np.float32) / np.float32(255.0)
        exp[py, px] = shade(ga, t, (0.0, 0.0, 1.0))
    assert np.array_equal(got[safe], exp[safe])
    # The view is oblique enough that interpolating the coordinates linearly
    # in screen space picks other texels at many of these pixels.
    vp = sc.cam_vp[0].reshape(4, 4).astype(np.float64)
    gv = sg.templates().ground_v.astype(np.float64)
    wrong = 0
    for f in sg.templates().ground_f:
        c = np.array([vp @ np.append(gv[k], 1.0) for k in f])
        sx = (c[:, 0] / c[:, 3] * 0.5 + 0.5) * W
        sy = (0.5 - c[:, 1] / c[:, 3] * 0.5) * H
        T = np.array([[sx[0] - sx[2], sx[1] - sx[2]], [sy[0] - sy[2], sy[1] - sy[2]]])
        Ti = np.linalg.inv(T)
        for py, px in zip(*np.nonzero(safe)):
            l01 = Ti @ np.array([px + 0.5 - sx[2], py + 0.5 - sy[2]])
            lam = np.array([l01[0], l01[1], 1.0 - l01.sum()])
            if lam.min() < 0:
                continue
            ua = (lam * gv[f, 0]).sum() * scale
            va = (lam * gv[f, 1]).sum() * scale
            ia, ja = texel_index(np.array(ua), np.array(va), Tw, Th)
            wrong += int(ia != ii[py, px] or ja != jj[py, px])
    assert wrong > 0.1 * safe.sum()


def above(res=64):
    """Straight down onto the origin from 1.2 m, image up = world +y."""
    return sg.view_proj((0.0, 0.0, 1.2), target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0), fovy_deg=30.0)


@pytest.mark.parametrize("turn", [0, 1], ids=["unrotated", "quarter-turn"])
def test_cube_top_face_shows_its_four_texels(turn):
    """A 2 x 2 texture on a cube's +z face: each quadrant of the face takes
    one texel; u runs along the body x axis, v along the body y axis, so a
    quarter turn about z turns the quadrants with the body."""
    W = H = 64
    a = 0.1
    tex = coord_texture(2, 2)
    q = quat_axis_angle((0.0, 0.0, 1.0), turn * math.pi / 2)
    sc = textured(tiny_scene([dict(type=1, size=a, pos=(0.0, 0.0, a), quat=q)], res=W, vp=above()), tex)
    out = oracle.render_image(sc, sc.state(), 0, e=0, debug=True)
    top = (out["winner"] >= 2 + 10) & (out["winner"] < 2 + 12)  # faces 10, 11: the +z face
    p = ray_hits(sc.cam_vp[0], W, H, 2 * a)
    # body coordinates of the hit: undo the turn about z
    c, s = math.cos(turn * math.pi / 2), math.sin(turn * math.pi / 2)
    bx = (c * p[..., 0] + s * p[..., 1]) / a
    by = (-s * p[..., 0] + c * p[..., 1]) / a
    safe = top & (np.abs(bx) > 0.08) & (np.abs(by) > 0.08) & (np.abs(bx) < 0.92) & (np.abs(by) < 0.92)
    assert safe.sum() > 300
    albedo = sg.PALETTE[0]
    for py, px in zip(*np.nonzero(safe)):
        i, j = int(bx[py, px] > 0), int(by[py, px] > 0)
        t = tex[j, i].astype(np.float32) / np.float32(255.0)
        assert np.array_equal(out["rgb"][py, px], shade(albedo, t, (0.0, 0.0, 1.0))), (py, px, i, j)
    # all four texels appear
    seen = {(int(bx[py, px] > 0), int(by[py, px] > 0)) for py, px in zip(*np.nonzero(safe))}
    assert seen == {(0, 0), (1, 0), (0, 1), (1, 1)}


def test_face_coordinates_of_the_cube_template():
    """Each face's corners take the unit square over the face's tangent axes:
    the two triangles of a face cover it, with corners at 0 and 1."""
    t = sg.templates()
    for f in range(len(t.cube_f)):
        uv = oracle.cube_face_uv(f)
        n = t.cube_n[f]
        ax = int(np.argmax(np.abs(n)))
        tang = [k for k in range(3) if k != ax]
        for k in range(3):
            v = t.cube_v[t.cube_f[f][k]]
            assert uv[k].tolist() == [(v[tang[0]] + 1) / 2, (v[tang[1]] + 1) / 2]


def test_uv_interpolation_by_hand():
    """A right triangle with 1/w = 1 at every corner: the coordinates are the
    screen-space barycentric mix; with 1/w doubled at one corner the weights
    tilt towards it exactly as E_k / w_k says."""
    X = np.array([0, 256 * 8, 0], np.int32)
    Y = np.array([0, 0, 256 * 8], np.int32)
    uv = np.array([[0, 0], [1, 0], [0, 1]], np.float32)
    got = oracle.smooth_uv(X, Y, np.ones(3, np.float32), uv, 2, 1)
    # pixel centre (2.5, 1.5) px: weights E_k are the opposite sub-areas
    P = (2.5 * 256, 1.5 * 256)
    E = [(X[2] - X[1]) * (P[1] - Y[1]) - (Y[2] - Y[1]) * (P[0] - X[1]),
         (X[0] - X[2]) * (P[1] - Y[2]) - (Y[0] - Y[2]) * (P[0] - X[2]),
         (X[1] - X[0]) * (P[1] - Y[0]) - (Y[1] - Y[0]) * (P[0] - X[0])]
    E = np.array(E, np.float64)
    exp = (E[:, None] * uv).sum(0) / E.sum()
    assert np.allclose(got, exp, atol=1e-6)
    iw = np.array([1.0, 2.0, 1.0], np.float32)
    got2 = oracle.smooth_uv(X, Y, iw, uv, 2, 1)
    w = E * iw
    assert np.allclose(got2, (w[:, None] * uv).sum(0) / w.sum(), atol=1e-6)
    assert got2[0] > got[0]
    # the opposite winding has no positive weights: (0, 0)
    assert oracle.smooth_uv(X[[0, 2, 1]], Y[[0, 2, 1]], np.ones(3, np.float32), uv, 2, 1).tolist() == [0.0, 0.0]


def test_spheres_stay_untextured():
    W = 64
    sc = tiny_scene([dict(type=0, size=0.1, pos=(0.0, 0.0, 0.1))], res=W, vp=above())
    plain = oracle.render_image(dataclasses.replace(sc, smooth=True), sc.state(), 0, e=0, debug=True)
    tex = textured(sc, coord_texture(4, 4), 3.0)
    out = oracle.render_image(tex, sc.state(), 0, e=0, debug=True)
    sphere = out["winner"] >= 2
    assert sphere.sum() > 300
    assert np.array_equal(out["rgb"][sphere], plain["rgb"][sphere])
    assert np.array_equal(out["depth"], plain["depth"])
    ground = (out["winner"] >= 0) & (out["winner"] < 2)
    assert np.any(out["rgb"][ground] != plain["rgb"][ground])


def test_texture_needs_smooth_shading():
    sc = tiny_scene([dict(type=0, size=0.1, pos=(0.0, 0.0, 0.1))], res=16)
    bad = dataclasses.replace(sc, smooth=False, texture=coord_texture(2, 2))
    with pytest.raises(ValueError):
        oracle.render_image(bad, sc.state(), 0, e=0)
