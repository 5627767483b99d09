"""Pins of the friction reading in the oracle (no GPU).

Regularized Coulomb friction: at each contact point the slip v_t (the
tangential part of the relative velocity) adds -mu f v_t / max(|v_t|, v_eps)
to the normal force f n.  Checked against closed forms of rigid-body
mechanics that do not depend on the contact model's details:

  * a block sliding down a slope accelerates at g (sin t - mu cos t);
  * a block on a slope below the friction angle creeps at the speed where
    the linear (regularized) friction balances gravity, v_eps tan t / mu;
  * a sliding sphere ends up rolling at 5/7 of its initial speed (angular
    momentum about the contact point is conserved, I = 2/5 m r^2);
  * a purely normal approach has no slip, so friction changes nothing, and
    with mu = 0 a sliding block keeps its speed exactly.

The slope is modelled by tilting gravity (the ground stays z = 0).
"""
import math

import numpy as np

import oracle
from tests.scenes import tiny_scene

G = 9.81


def run(sc, steps, st=None):
    st = sc.state() if st is None else st
    for _ in range(steps):
        status, _ = oracle.step_env(sc, 0, st)
        assert status == 0
    return st


def slope_block(theta_deg, mu, v_eps=0.05, a=0.05):
    th = math.radians(theta_deg)
    return tiny_scene([dict(type=1, size=a, pos=(0.0, 0.0, a))],
                      gravity=(G * math.sin(th), 0.0, -G * math.cos(th)), mu=mu, v_eps=v_eps)


def test_block_slides_at_the_coulomb_acceleration():
    # 30 degrees, mu = 0.3 < tan 30: once the slip exceeds v_eps the friction
    # is mu times the normal force, whose mean is m g cos t
    th = math.radians(30.0)
    sc = slope_block(30.0, 0.3)
    st = run(sc, 120)
    v1 = float(st["vel"][0][0])
    st = run(sc, 120, st)
    v2 = float(st["vel"][0][0])
    expect = 0.5 * G * (math.sin(th) - 0.3 * math.cos(th))
    assert v1 > 0.05
    assert abs((v2 - v1) - expect) <= 1e-4 * expect
    # it slides without tipping or turning
    assert np.all(np.abs(st["omega"][0]) < 1e-4)
    assert abs(float(st["vel"][0][1])) < 1e-6


def test_block_below_the_friction_angle_creeps_at_the_regularized_speed():
    # 10 degrees, mu = 0.3 > tan 10: the slip settles where mu m g cos t
    # |v| / v_eps = m g sin t
    for mu, v_eps in ((0.3, 0.05), (0.6, 0.1)):
        sc = slope_block(10.0, mu, v_eps)
        st = run(sc, 240)
        creep = v_eps * math.tan(math.radians(10.0)) / mu
        assert abs(float(st["vel"][0][0]) - creep) <= 1e-3 * creep
        assert abs(float(st["vel"][0][1])) < 1e-6


def test_sliding_sphere_ends_up_rolling_at_five_sevenths():
    r, v0 = 0.1, 2.0
    for mu in (0.2, 0.5):
        sc = tiny_scene([dict(type=0, size=r, pos=(0.0, 0.0, r), vel=(v0, 0.0, 0.0))], mu=mu)
        st = run(sc, 480)
        v = float(st["vel"][0][0])
        w = float(st["omega"][0][1])
        assert abs(v - 5.0 / 7.0 * v0) <= 2e-4 * v0
        # rolling: the contact point is at rest (omega about +y for motion +x)
        assert abs(v - w * r) <= 1e-3 * v0
        assert abs(float(st["vel"][0][1])) == 0.0


def test_normal_approach_is_unchanged_by_friction():
    bodies = [dict(type=0, size=0.1, pos=(0.0, 0.0, 0.3)), dict(type=1, size=0.08, pos=(0.0, 0.0, 0.6))]
    plain = run(tiny_scene(bodies), 200)
    rough = run(tiny_scene(bodies, mu=0.8), 200)
    for k in ("pos", "vel", "quat", "omega"):
        assert np.array_equal(plain[k], rough[k]), k


def test_frictionless_block_keeps_its_speed():
    a = 0.05
    sc = tiny_scene([dict(type=1, size=a, pos=(0.0, 0.0, a), vel=(1.5, -0.5, 0.0))], mu=0.0)
    st = run(sc, 240)
    assert float(st["vel"][0][0]) == np.float32(1.5)
    assert float(st["vel"][0][1]) == np.float32(-0.5)
    # with friction the same block stops: mu g = 3.9 m/s^2 brakes 1.6 m/s
    # within half a second, after which it stays at rest
    sc = tiny_scene([dict(type=1, size=a, pos=(0.0, 0.0, a), vel=(1.5, -0.5, 0.0))], mu=0.4)
    st = run(sc, 240)
    assert np.all(np.abs(st["vel"][0][:2]) < 1e-4)
