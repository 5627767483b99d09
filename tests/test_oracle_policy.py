"""Pins of the policy oracle and of the external-force step (no GPU).

The MLP reading (observation layout, layers, clamp) is checked against
values worked out by hand, against IEEE bfloat16 definitions, and against a
float32 evaluation that must stay within the oracle's own error bound; the
force path against the discrete closed form of semi-implicit Euler under a
constant force.
"""
import numpy as np
import pytest

import oracle
from oracle import policy as op
from tests.scenes import tiny_scene

H = (1.0 / 240.0) / 4.0
G = 9.81


def bf(x):
    return op.f32_to_bf16_rne(np.asarray(x, np.float32))


def test_bfloat16_patterns():
    # IEEE binary32 with its low 16 bits dropped: sign, 8 exponent bits, 7
    # fraction bits
    assert list(op.bf16_to_f64(np.array([0x3F80, 0xC000, 0x3F81, 0x0000, 0x4300], np.uint16))) == \
        [1.0, -2.0, 1.0 + 2.0 ** -7, 0.0, 128.0]
    # round to nearest even: 1 + 2^-8 is a tie between 1 and 1 + 2^-7
    assert bf([1.0 + 2.0 ** -8])[0] == 0x3F80
    assert bf([1.0 + 3 * 2.0 ** -8])[0] == 0x3F82
    assert bf([1.0 + 2.0 ** -8 + 2.0 ** -20])[0] == 0x3F81
    # every 8-bit integer is exact, so the observation needs no rounding
    ints = np.arange(256, dtype=np.float32)
    assert np.array_equal(op.bf16_to_f64(bf(ints)), ints.astype(np.float64))


def test_observation_layout():
    Wd, Ht = 5, 3
    rgb = np.zeros((Ht, Wd, 3), np.uint8)
    depth = np.full((Ht, Wd), 0xFFFFFFFF, np.uint32)
    rgb[1, 2] = (10, 20, 30)
    depth[1, 2] = 0xABCDEF
    x = op.observation(rgb, depth)
    p = 1 * Wd + 2
    assert x.shape == (4 * Wd * Ht,)
    nz = np.nonzero(x[:3 * Wd * Ht])[0]
    assert list(nz) == [3 * p, 3 * p + 1, 3 * p + 2]
    assert list(x[3 * p:3 * p + 3]) == [10.0, 20.0, 30.0]
    dep = x[3 * Wd * Ht:]
    assert dep[p] == 0xAB and np.all(np.delete(dep, p) == 255.0)


def tiny_policy(K=4, Hd=2, A=3):
    # W1 picks x0 and x1 (times 1 and 0.5), W2 = identity, W3 by hand
    w1 = np.zeros((K, Hd), np.float32)
    w1[0, 0], w1[1, 1] = 1.0, 0.5
    return dict(w1_bf16=bf(w1), b1=np.array([0.25, -1.0], np.float32),
                w2=np.eye(Hd, dtype=np.float32), b2=np.zeros(Hd, np.float32),
                w3=np.array([[0.125, -0.5, 0.0], [0.25, 0.0, 1.0]], np.float32),
                b3=np.array([0.0, 0.5, -0.25], np.float32), a_max=np.float32(4.0))


def test_forward_by_hand():
    P = tiny_policy()
    x = np.array([3.0, 6.0, 7.0, 9.0])
    a, inner = op.forward(x, P)
    # s1 = (3 + 0.25, 3 - 1) = (3.25, 2); h2 = h1; y = (3.25/8 + 2/4, -3.25/2 + 0.5, 2 - 0.25)
    assert np.allclose(inner["s1"], [3.25, 2.0], rtol=0, atol=0)
    assert np.allclose(inner["y"], [0.90625, -1.125, 1.75], rtol=0, atol=0)
    assert np.allclose(a, [4.0 * 0.90625, -4.0, 4.0], rtol=0, atol=0)


def test_relu_and_clamp():
    P = tiny_policy()
    # x0 = 0 and x1 = 0: s1 = (0.25, -1), the second unit is cut
    a, inner = op.forward(np.zeros(4), P)
    assert list(inner["h1"]) == [0.25, 0.0]
    # all weights zero: y = b3 exactly; |b3| >= 1 saturates to +-a_max
    Z = dict(P, w1_bf16=bf(np.zeros((4, 2))), w2=np.zeros((2, 2), np.float32),
             w3=np.zeros((2, 3), np.float32), b3=np.array([2.0, -3.0, 0.5], np.float32))
    a, _ = op.forward(np.full(4, 200.0), Z)
    assert list(a) == [4.0, -4.0, 2.0]


def test_float32_evaluation_within_the_bound():
    rng = np.random.default_rng(7)
    K, Hd, A = 4096, 64, 9
    # layer 1 scaled to values of order one; layers 2 and 3 with absolute
    # row sums below one, so that they do not amplify errors
    P = dict(w1_bf16=bf(rng.normal(0, 1.0 / (np.sqrt(K) * 128), (K, Hd))),
             b1=rng.normal(0, 0.1, Hd).astype(np.float32),
             w2=rng.normal(0, 1.0 / Hd, (Hd, Hd)).astype(np.float32), b2=rng.normal(0, 0.5, Hd).astype(np.float32),
             w3=rng.normal(0, 1.0 / Hd, (Hd, A)).astype(np.float32), b3=rng.normal(0, 0.3, A).astype(np.float32),
             a_max=np.float32(2.0))
    for _ in range(3):
        x = rng.integers(0, 256, K).astype(np.float64)
        a, inner = op.forward(x, P)
        bound = op.error_bound(x, P, inner)
        # a float32 evaluation in a different order: blocks of 128 terms
        W1 = op.bf16_to_f64(P["w1_bf16"]).astype(np.float32)
        x32 = x.astype(np.float32)
        s = np.zeros(Hd, np.float32)
        for k0 in range(K - 128, -1, -128):
            s = (s + (x32[k0:k0 + 128] @ W1[k0:k0 + 128]).astype(np.float32)).astype(np.float32)
        h1 = np.maximum(s + P["b1"], 0).astype(np.float32)
        h2 = np.maximum((h1 @ P["w2"]).astype(np.float32) + P["b2"], 0).astype(np.float32)
        y = ((h2 @ P["w3"]).astype(np.float32) + P["b3"]).astype(np.float32)
        a32 = (np.float32(P["a_max"]) * np.clip(y, -1, 1)).astype(np.float32)
        assert np.all(np.abs(a32 - a) <= bound)
        # and the bound is not vacuous: the actions are unsaturated and the
        # bound is below a percent of their range
        assert np.all(np.abs(inner["y"]) < 1.0)
        assert np.all(bound < 1e-2 * float(P["a_max"]))


def test_forces_of_actions():
    a = np.arange(9, dtype=np.float32)
    f = op.forces(a, n_bodies=2, act_bodies=3)
    assert f.tolist() == [[0, 1, 2], [3, 4, 5]]
    f = op.forces(a, n_bodies=4, act_bodies=3)
    assert f[3].tolist() == [0, 0, 0] and f[2].tolist() == [6, 7, 8]


# A constant external force F on a free body adds F/m to gravity: the
# discrete closed form of semi-implicit Euler, v_n = v0 + n h a and
# x_n = x0 + h^2 a n(n+1)/2, with a = F/m + g.
def test_constant_external_force_closed_form():
    sc = tiny_scene([dict(type=1, size=0.05, pos=(0.0, 0.0, 50.0))])
    st = sc.state()
    F = np.array([[1.5, -0.75, 20.0]], np.float32)
    m = 1.0 / float(sc.inv_m[0])
    steps = 25
    for _ in range(steps):
        s, _ = oracle.step_env(sc, 0, st, fext=F)
        assert s == 0
    n = 4 * steps
    acc = F[0] / m + np.array([0.0, 0.0, -G])
    v = n * H * acc
    x = np.array([0.0, 0.0, 50.0]) + H * H * acc * n * (n + 1) / 2.0
    assert np.allclose(st["vel"][0], v, rtol=2e-5, atol=1e-6)
    assert np.allclose(st["pos"][0], x, rtol=2e-6, atol=2e-6)
    # no torque: the orientation stays the identity exactly
    assert st["quat"][0].tolist() == [1.0, 0.0, 0.0, 0.0]


def test_zero_force_is_the_plain_step():
    sc = tiny_scene([dict(type=0, size=0.1, pos=(0.0, 0.0, 0.09)),
                     dict(type=1, size=0.08, pos=(0.05, 0.0, 0.25))])
    a, b = sc.state(), sc.state()
    for _ in range(30):
        oracle.step_env(sc, 0, a)
        oracle.step_env(sc, 0, b, fext=np.zeros((2, 3), np.float32))
    for k in ("pos", "vel", "quat", "omega"):
        assert np.allclose(a[k], b[k], rtol=0, atol=0)
