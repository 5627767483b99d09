"""Pins of the oracle's separating-axis edge-edge contact of two boxes.

Checked against geometry fixed independently of the oracle's code: the
closed form of two crossed ridges, the penetration depth of two convex
boxes as the least overlap over all directions (sampled here in float64),
the containment of the contact point, face contacts left to the vertex
points, and a drop onto a ridge that the vertex tests alone let pass."""
import dataclasses
import math

import numpy as np

import oracle
from tests.scenes import quat_axis_angle, tiny_scene


def pair_scene(bodies, edge=True):
    s = tiny_scene(bodies)
    return dataclasses.replace(s, edge_contacts=edge)


def points(sc, i=0, j=1):
    return oracle.narrowphase(sc, sc.state(), i, j)


def rot(q):
    w, x, y, z = (float(v) for v in q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def overlap(L, boxes):
    """Overlap of two boxes along unit direction L (float64)."""
    (pa, Ra, ea), (pb, Rb, eb) = boxes
    r = lambda R, e: float(np.sum(e * np.abs(R.T @ L)))
    return r(Ra, ea) + r(Rb, eb) - abs(float((pa - pb) @ L))


def ridge_pair(delta, a=0.05):
    """Box j: a cube turned 45 deg about x (a ridge along x on top); box i:
    a cube turned 45 deg about y above it (a ridge along y below), the
    ridges crossing by delta."""
    h = a * math.sqrt(2.0)
    return [dict(type=1, size=a, pos=(0.0, 0.0, 2 * h - delta + 1.0), quat=quat_axis_angle((0, 1, 0), math.pi / 4)),
            dict(type=1, size=a, pos=(0.0, 0.0, 1.0), quat=quat_axis_angle((1, 0, 0), math.pi / 4))]


def test_crossed_ridges_closed_form():
    a, delta = 0.05, 0.004
    h = a * math.sqrt(2.0)
    pts = points(pair_scene(ridge_pair(delta, a)))
    assert len(pts) == 1
    p = pts[0]
    assert p.a_is_first == 1
    assert np.allclose(list(p.n), [0.0, 0.0, 1.0], atol=1e-6)
    assert abs(p.delta - delta) < 2e-6
    # midway between the ridges' closest points, above the crossing
    assert np.allclose(list(p.xc), [0.0, 0.0, 1.0 + h - delta / 2], atol=2e-6)
    # the vertex tests alone see no contact at all
    assert len(points(pair_scene(ridge_pair(delta, a), edge=False))) == 0


def test_face_contacts_are_left_to_the_vertex_points():
    a = 0.05
    for ang in (0.0, 0.3, 0.7):
        bodies = [dict(type=1, size=a, pos=(0.01, -0.005, 1.0 + 2 * a - 0.003), quat=quat_axis_angle((0, 0, 1), ang)),
                  dict(type=2, ext=(0.1, 0.09, a), pos=(0.0, 0.0, 1.0))]
        on = points(pair_scene(bodies, edge=True))
        off = points(pair_scene(bodies, edge=False))
        assert len(off) == 4 and len(on) == len(off)
        for u, v in zip(on, off):
            assert list(u.n) == list(v.n) and u.delta == v.delta and list(u.xc) == list(v.xc)


def test_edge_point_is_the_penetration_depth_and_inside_both():
    rng = np.random.default_rng(7)
    dirs = rng.normal(size=(20000, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    found = 0
    for trial in range(300):
        ea = rng.uniform(0.03, 0.1, 3)
        eb = rng.uniform(0.03, 0.1, 3)
        qa = quat_axis_angle(rng.normal(size=3), rng.uniform(0, math.pi))
        qb = quat_axis_angle(rng.normal(size=3), rng.uniform(0, math.pi))
        d = rng.normal(size=3)
        d *= rng.uniform(0.6, 1.0) * (np.linalg.norm(ea) + np.linalg.norm(eb)) / np.linalg.norm(d)
        bodies = [dict(type=2, ext=tuple(ea), pos=tuple(np.array([0.0, 0.0, 1.0]) + d), quat=qa),
                  dict(type=2, ext=tuple(eb), pos=(0.0, 0.0, 1.0), quat=qb)]
        sc = pair_scene(bodies)
        st = sc.state()
        pts = oracle.narrowphase(sc, st, 0, 1)
        boxes = [(st["pos"][k].astype(np.float64), rot(st["quat"][k]), sc.ext[k].astype(np.float64)) for k in (0, 1)]
        if not pts:
            continue
        n_vert = len(points(dataclasses.replace(sc, edge_contacts=False)))
        if len(pts) == n_vert:
            continue  # no edge point
        found += 1
        e = pts[-1]
        n = np.array(list(e.n), np.float64)
        # depth: the overlap along n, and no sampled direction overlaps less
        assert abs(overlap(n, boxes) - e.delta) < 1e-5
        sampled = min(overlap(L, boxes) for L in dirs)
        assert sampled >= e.delta - 1e-5
        # n points from j to i
        assert float((boxes[0][0] - boxes[1][0]) @ n) >= 0.0
        # the point lies in both boxes grown by the depth
        xc = np.array(list(e.xc), np.float64)
        for p, R, ext in boxes:
            assert np.all(np.abs(R.T @ (xc - p)) <= ext + e.delta + 1e-5)
    assert found >= 20


def test_separated_boxes_have_no_points():
    a = 0.05
    bodies = ridge_pair(-0.001, a)  # ridges 1 mm apart
    assert points(pair_scene(bodies)) == []


def test_drop_onto_a_ridge_is_caught():
    """A cube turned 45 deg about y falls 2 cm onto a ridge along x: with
    edge points the ridge stops it like a spring; with the vertex tests
    alone it sinks until its faces meet the ridge's vertices."""
    a = 0.05
    h = a * math.sqrt(2.0)

    def max_pen(edge):
        bodies = [dict(type=1, size=a, pos=(0.0, 0.0, 2 * h + 0.02), quat=quat_axis_angle((0, 1, 0), math.pi / 4)),
                  dict(type=1, size=a, pos=(0.0, 0.0, 0.0), quat=quat_axis_angle((1, 0, 0), math.pi / 4),
                       mass=1.0e6)]
        sc = dataclasses.replace(tiny_scene(bodies), edge_contacts=edge)
        st = sc.state()
        worst = 0.0
        for _ in range(120):
            oracle.step_scene(sc, st)
            st["pos"][1] = 0.0  # the lower cube held in place
            st["vel"][1] = 0.0
            st["omega"][1] = 0.0
            st["quat"][1] = sc.quat[1]
            worst = max(worst, 2 * h - float(st["pos"][0][2]))
        return worst

    # an undamped spring of stiffness k met at the impact speed v0 of the
    # 2 cm fall compresses by v0 sqrt(m / k), plus at most 2 m g / k
    v0 = math.sqrt(2 * 9.81 * 0.02)
    assert max_pen(True) < v0 * math.sqrt(1.0 / 1.0e4) + 2 * 9.81 / 1.0e4
    assert max_pen(False) > 0.02
