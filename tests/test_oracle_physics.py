"""Pins of the physics oracle against closed forms, invariants and hand-worked
contact geometry (no GPU).

Each test fixes a quantity the mathematics determines independently of the
oracle's code: the discrete solution of semi-implicit Euler under constant
acceleration, its exact energy drift, conservation of linear and angular
momentum under pairwise contact forces, the spring-dashpot equilibrium and
restitution, and contact geometry worked out by hand.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2605_01352_amd import scenegen as sg
from tests.scenes import quat_axis_angle, tiny_scene

H = (1.0 / 240.0) / 4.0
G = 9.81


def run(scene, steps, record=False):
    st = scene.state()
    pairs = []
    for _ in range(steps):
        sts, prs = oracle.step_scene(scene, st, record_pairs=record)
        assert all(v == 0 for v in sts.values())
        pairs.append(prs)
    return st, pairs


# P1: free fall follows the discrete closed form of semi-implicit Euler:
# v_n = v0 + n h g,  x_n = x0 + n h v0 + h^2 g n(n+1)/2.
def test_free_fall_discrete_closed_form():
    sc = tiny_scene([dict(type=0, size=0.1, pos=(0.0, 0.0, 50.0))])
    steps = 100
    st, _ = run(sc, steps)
    n = 4 * steps
    v = -G * n * H
    z = 50.0 - G * H * H * n * (n + 1) / 2.0
    assert abs(st["vel"][0, 2] - v) <= 1e-5 * max(1.0, abs(v))
    assert abs(st["pos"][0, 2] - z) <= 2e-5 * max(1.0, abs(z))
    # the continuous-time answer differs by exactly g h t / 2, i.e. h = dt/4
    t = n * H
    assert abs((50.0 - 0.5 * G * t * t) - z - 0.5 * G * H * t) < 1e-9


# P2: ballistic flight with spin.  Position per axis follows P1's form; each
# substep's q <- normalize(q + h/2 (0,w) q) is an exact rotation by
# 2 atan(|w| h / 2) about w (applied on the left), so q_n is known in closed
# form; |q| stays 1.
def test_ballistic_with_spin_closed_form():
    q0 = quat_axis_angle((1.0, 2.0, 0.5), 0.7)
    w = np.array([3.0, -1.5, 2.0])
    v0 = np.array([0.5, -0.25, 3.0])
    sc = tiny_scene([dict(type=1, size=0.05, pos=(0.0, 0.0, 20.0), quat=q0, vel=v0, omega=w)])
    steps = 50
    st, _ = run(sc, steps)
    n = 4 * steps
    g = np.array([0.0, 0.0, -G])
    x = np.array([0.0, 0.0, 20.0]) + n * H * v0 + H * H * g * n * (n + 1) / 2.0
    np.testing.assert_allclose(st["pos"][0], x, rtol=0, atol=2e-5)
    np.testing.assert_allclose(st["omega"][0], w, rtol=0, atol=1e-6)
    wn = np.linalg.norm(w)
    ang = n * 2.0 * math.atan(wn * H / 2.0)
    r = np.array(quat_axis_angle(w, ang))

    def qmul(a, b):
        aw, ax, ay, az = a
        bw, bx, by, bz = b
        return np.array([aw * bw - ax * bx - ay * by - az * bz, aw * bx + ax * bw + ay * bz - az * by,
                         aw * by - ax * bz + ay * bw + az * bx, aw * bz + ax * by - ay * bx + az * bw])

    expect = qmul(r, np.array(q0))
    got = st["quat"][0].astype(np.float64)
    assert abs(np.linalg.norm(got) - 1.0) < 1e-6
    assert min(np.abs(got - expect).max(), np.abs(got + expect).max()) < 2e-5
    # the right-multiplied (body-frame) update would be far off
    wrong = qmul(np.array(q0), r)
    assert min(np.abs(got - wrong).max(), np.abs(got + wrong).max()) > 1e-2


# P3: contact-free energy drifts by exactly -1/2 m g^2 h^2 per substep.
def test_energy_drift_exact():
    sc = tiny_scene([dict(type=0, size=0.1, pos=(0.0, 0.0, 30.0), vel=(1.0, 0.0, 2.0))])
    st0 = sc.state()
    steps = 100
    st, _ = run(sc, steps)

    def energy(s):
        v = s["vel"][0].astype(np.float64)
        return 0.5 * v @ v + G * float(s["pos"][0, 2])

    n = 4 * steps
    drift = energy(st) - energy(st0)
    assert abs(drift - (-0.5 * G * G * H * H * n)) < 2e-4
    assert abs(0.5 * G * G * H * H * n - 0.020885) < 1e-5


# P4a: contact-free momentum P_n = P_0 + n h M g.
def test_momentum_contact_free():
    bodies = [dict(type=i % 2, size=0.05, pos=(i * 1.0, 0.0, 40.0), vel=(0.1 * i, 0.2, -0.3)) for i in range(4)]
    sc = tiny_scene(bodies)
    st0 = sc.state()
    st, _ = run(sc, 25)
    P0 = st0["vel"].astype(np.float64).sum(0)
    P = st["vel"].astype(np.float64).sum(0)
    np.testing.assert_allclose(P, P0 + np.array([0, 0, -G]) * 100 * H * 4, atol=1e-5)


# P4b: with g = 0 and no ground, pairwise contact forces conserve total linear
# momentum and total angular momentum sum(m x cross v + I w) exactly in exact
# arithmetic (x_{n+1} x v_{n+1} = x_n x v_{n+1}; both bodies' torque arms
# share the contact point), so only rounding remains.
def test_momentum_and_angular_momentum_with_contacts():
    rng = np.random.default_rng(5)
    bodies = []
    for i in range(10):
        t = i % 2
        bodies.append(dict(type=t, size=0.08, pos=(0.13 * (i % 4) - 0.2, 0.13 * (i // 4) - 0.13, 1.5 + 0.02 * i),
                           quat=quat_axis_angle(rng.normal(size=3), rng.uniform(0, 3)),
                           vel=rng.normal(size=3) * 0.5, omega=rng.normal(size=3) * 2.0,
                           mass=1.0))
    sc = tiny_scene(bodies, gravity=(0.0, 0.0, 0.0))

    def moments(s):
        x = s["pos"].astype(np.float64)
        v = s["vel"].astype(np.float64)
        w = s["omega"].astype(np.float64)
        I = 1.0 / sc.inv_I.astype(np.float64)
        return v.sum(0), (np.cross(x, v) + I[:, None] * w).sum(0)

    P0, L0 = moments(sc.state())
    st, pairs = run(sc, 40, record=True)
    ncontacts = sum(len(p) for step in pairs for e in step.values() for p in e)
    assert ncontacts > 20  # bodies really collide
    P, L = moments(st)
    np.testing.assert_allclose(P, P0, atol=5e-6)
    np.testing.assert_allclose(L, L0, atol=5e-5)
    assert np.abs(st["vel"] - sc.vel).max() > 0.05  # momentum really moved between bodies


# P5: resting contact converges to the spring-dashpot equilibrium.
def test_resting_sphere_equilibrium():
    r = 0.1
    sc = tiny_scene([dict(type=0, size=r, pos=(0.0, 0.0, r - 5e-4))])
    st, _ = run(sc, 2400)
    assert abs(st["pos"][0, 2] - (r - G / 1.0e4)) < 2e-6
    assert abs(st["vel"][0, 2]) < 1e-5


def test_resting_cube_equilibrium():
    a = 0.08
    sc = tiny_scene([dict(type=1, size=a, pos=(0.0, 0.0, a - 1e-4))])
    st, _ = run(sc, 2400)
    assert abs(st["pos"][0, 2] - (a - G / (4 * 1.0e4))) < 2e-6
    assert np.abs(st["omega"][0]).max() < 1e-6


# P6: a vertical drop onto the ground equals the 1-D spring-dashpot recurrence
# iterated independently in double; the restitution coefficient is near
# exp(-zeta pi / sqrt(1 - zeta^2)).
def test_drop_matches_1d_recurrence_and_restitution():
    r, z0, v0 = 0.1, 0.3, 0.0
    sc = tiny_scene([dict(type=0, size=r, pos=(0.0, 0.0, z0))])
    steps = 150
    st = sc.state()
    zs, vs = [], []
    for _ in range(steps):
        oracle.step_scene(sc, st)
        zs.append(float(st["pos"][0, 2]))
        vs.append(float(st["vel"][0, 2]))
    z, v = z0, v0
    zr, vr = [], []
    for _ in range(steps):
        for _ in range(4):
            d = r - z
            f = 0.0
            if d > 0:
                f = max(0.0, 1.0e4 * d - 10.0 * v)
            v = v + H * (f - G)
            z = z + H * v
        zr.append(z)
        vr.append(v)
    np.testing.assert_allclose(zs, zr, atol=5e-5)
    np.testing.assert_allclose(vs, vr, atol=5e-3)
    # restitution: ratio of the rebound speed to the impact speed
    vin = -min(vs)
    vout = max(vs[int(np.argmin(vs)):])
    zeta = 10.0 / (2.0 * math.sqrt(1.0e4))
    e = math.exp(-zeta * math.pi / math.sqrt(1 - zeta * zeta))
    assert abs(vout / vin - e) < 0.05 * e


def test_head_on_spheres_restitution():
    r = 0.1
    sc = tiny_scene([dict(type=0, size=r, pos=(-0.3, 0.0, 5.0), vel=(1.0, 0.0, 0.0)),
                     dict(type=0, size=r, pos=(0.3, 0.0, 5.0), vel=(-1.0, 0.0, 0.0))],
                    gravity=(0.0, 0.0, 0.0))
    st, _ = run(sc, 240)
    rel_out = st["vel"][1, 0] - st["vel"][0, 0]
    zeta = 10.0 / (2.0 * math.sqrt(1.0e4 * 0.5))
    e = math.exp(-zeta * math.pi / math.sqrt(1 - zeta * zeta))
    assert abs(rel_out / 2.0 - e) < 0.05 * e
    assert abs(st["vel"][:, 0].sum()) < 1e-5


# P7: contact geometry worked out by hand.
def _np(bodies, i, j):
    sc = tiny_scene(bodies)
    return oracle.narrowphase(sc, sc.state(), i, j)


def test_sphere_sphere_geometry():
    b = [dict(type=0, size=0.1, pos=(0.0, 0.0, 1.0)), dict(type=0, size=0.1, pos=(0.19, 0.0, 1.0))]
    pts = _np(b, 0, 1)
    assert len(pts) == 1
    p = pts[0]
    assert abs(p.delta - 0.01) < 1e-6
    np.testing.assert_allclose(list(p.n), [-1, 0, 0], atol=1e-7)
    np.testing.assert_allclose(list(p.xc), [0.095, 0, 1.0], atol=1e-6)
    b[1]["pos"] = (0.21, 0.0, 1.0)
    assert _np(b, 0, 1) == []
    # coincident centres: normal defaults to +z
    b[1]["pos"] = (0.0, 0.0, 1.0)
    pts = _np(b, 0, 1)
    assert list(pts[0].n) == [0.0, 0.0, 1.0] and abs(pts[0].delta - 0.2) < 1e-7


def test_sphere_cube_geometry():
    cube = dict(type=1, size=0.1, pos=(0.0, 0.0, 1.0))
    # sphere above the top face
    pts = _np([dict(type=0, size=0.1, pos=(0.0, 0.0, 1.18)), cube], 0, 1)
    assert len(pts) == 1 and pts[0].a_is_first == 1
    assert abs(pts[0].delta - 0.02) < 1e-6
    np.testing.assert_allclose(list(pts[0].n), [0, 0, 1], atol=1e-6)
    np.testing.assert_allclose(list(pts[0].xc), [0, 0, 1.1], atol=1e-6)
    # sphere near an edge, cube first in the pair: normal still cube -> sphere
    pts = _np([cube, dict(type=0, size=0.1, pos=(0.15, 0.15, 1.0))], 0, 1)
    assert len(pts) == 1 and pts[0].a_is_first == 0
    assert abs(pts[0].delta - (0.1 - math.sqrt(0.005))) < 1e-6
    np.testing.assert_allclose(list(pts[0].n), [math.sqrt(0.5), math.sqrt(0.5), 0], atol=1e-6)
    # centre inside the cube: nearest face (x at 0.05 from it)
    pts = _np([dict(type=0, size=0.1, pos=(0.05, 0.0, 1.02)), cube], 0, 1)
    assert abs(pts[0].delta - 0.15) < 1e-6
    np.testing.assert_allclose(list(pts[0].n), [1, 0, 0], atol=1e-6)
    # rotating the cube by 90 degrees about z changes nothing for a top contact
    cube_r = dict(cube, quat=quat_axis_angle((0, 0, 1), math.pi / 2))
    pts = _np([dict(type=0, size=0.1, pos=(0.0, 0.0, 1.18)), cube_r], 0, 1)
    np.testing.assert_allclose(list(pts[0].n), [0, 0, 1], atol=1e-6)


def test_cube_cube_geometry():
    big = dict(type=1, size=0.1, pos=(0.0, 0.0, 1.0))
    small = dict(type=1, size=0.05, pos=(0.0, 0.0, 1.14))
    pts = _np([small, big], 0, 1)
    assert len(pts) == 4
    for p in pts:
        assert p.a_is_first == 1
        assert abs(p.delta - 0.01) < 1e-6
        np.testing.assert_allclose(list(p.n), [0, 0, 1], atol=1e-6)
        assert abs(p.xc[2] - 1.09) < 1e-6
    # pair order reversed: the small cube's vertices come second, A = second body
    pts = _np([big, small], 0, 1)
    assert len(pts) == 4 and all(p.a_is_first == 0 for p in pts)
    # a vertex exactly on the face plane is not inside (strict test)
    touching = dict(type=1, size=0.05, pos=(0.0, 0.0, 1.15))
    assert _np([touching, big], 0, 1) == []


def test_ground_geometry():
    pts = _np([dict(type=0, size=0.1, pos=(0.3, 0.2, 0.09))], 0, oracle.GROUND)
    assert len(pts) == 1 and abs(pts[0].delta - 0.01) < 1e-7
    np.testing.assert_allclose(list(pts[0].xc), [0.3, 0.2, -0.01], atol=1e-7)
    pts = _np([dict(type=1, size=0.1, pos=(0.0, 0.0, 0.09))], 0, oracle.GROUND)
    assert len(pts) == 4
    assert all(abs(p.delta - 0.01) < 1e-6 for p in pts)
    # tilted 45 degrees about x: one edge (2 vertices) dips below
    q = quat_axis_angle((1, 0, 0), math.pi / 4)
    pts = _np([dict(type=1, size=0.1, pos=(0.0, 0.0, 0.1 * math.sqrt(2) - 0.01), quat=q)], 0, oracle.GROUND)
    assert len(pts) == 2
    assert all(abs(p.delta - 0.01) < 1e-6 for p in pts)


def test_contact_pair_set_of_a_sphere_chain():
    # five touching spheres in a row (gap 0.19 < 0.2) sunk 5 mm into the
    # ground, and one isolated sphere in the air
    bodies = [dict(type=0, size=0.1, pos=(0.19 * i, 0.0, 0.095)) for i in range(5)]
    bodies.append(dict(type=0, size=0.1, pos=(3.0, 0.0, 0.5)))
    sc = tiny_scene(bodies)
    st = sc.state()
    _, prs = oracle.step_scene(sc, st, record_pairs=True)
    got = [tuple(p) for p in prs[0][0]]
    G_ = oracle.GROUND
    assert got == [(0, 1), (0, G_), (1, 2), (1, G_), (2, 3), (2, G_), (3, 4), (3, G_), (4, G_)]


# P11: determinism; an env's result does not depend on the batch around it.
def test_determinism_and_batch_independence():
    sc = sg.config_scene(2, n_envs=6)
    a = sc.state()
    b = sc.state()
    for _ in range(20):
        oracle.step_scene(sc, a)
        oracle.step_scene(sc, b)
    for k in a:
        assert np.array_equal(a[k], b[k])
    sub = sc.subset([4])
    c = sub.state()
    for _ in range(20):
        oracle.step_scene(sub, c)
    b0, b1 = sc.body_off[4], sc.body_off[5]
    for k in a:
        assert np.array_equal(a[k][b0:b1], c[k])


def test_batch_driver_matches_per_env_calls():
    sc = sg.config_scene(1)
    a = sc.state()
    for _ in range(5):
        oracle.step_scene(sc, a)
    b = sc.state()
    st, rgb, depth = oracle.run_batch(sc, b, 5, nthreads=4, do_render=True)
    assert st == 0
    for k in a:
        assert np.array_equal(a[k], b[k])
    img = oracle.render_image(sc, a, 3)
    off = oracle.image_offsets(sc)[3]
    assert np.array_equal(depth[off:off + 64 * 64].reshape(64, 64), img["depth"])
    assert np.array_equal(rgb[3 * off:3 * (off + 64 * 64)].reshape(64, 64, 3), img["rgb"])
