"""GPU parity of the MLP policy phase and of the forces it applies, through
the C ABI.

Gates: actions within the oracle's float32 error bound (oracle.policy.error_bound,
Higham-Mary probabilistic bound at lambda = 8) of the float64 evaluation on
the oracle's own rendering of the same state, after checking that the two
frames are identical; a step under saturated actions (exactly +-a_max or
a_max/4, known from the policy alone) against the oracle's step with those
forces at the usual physics gates (contact sets bit-exact, state 1e-5).
"""
import numpy as np
import pytest

import oracle
from oracle import policy as op
from paper_2605_01352_amd import scenegen as sg
from paper_2605_01352_amd import vuda
from tests.gpu_util import STATE_KEYS, say, state_close

pytestmark = pytest.mark.gpu


def oracle_actions(scene, st, P, envs):
    """Per env: (actions, bound, rgb, depth) from the oracle's rendering."""
    out = {}
    for e in envs:
        c = int(scene.cam_off[e])
        ref = oracle.render_image(scene, st, c, e=e)
        x = op.observation(ref["rgb"], ref["depth"])
        a, inner = op.forward(x, P)
        out[e] = (a, op.error_bound(x, P, inner), ref["rgb"], ref["depth"])
    return out


def check_actions(w, scene, P, envs, label):
    st = w.state()
    w.render()
    w.act()
    w.wait()
    A = 3 * int(P["act_bodies"])
    got = w.fetch(vuda.FETCH_ACTIONS).reshape(scene.n_envs, A)
    rgb = w.images(vuda.FETCH_RGB)
    dep = w.images(vuda.FETCH_DEPTH)
    ref = oracle_actions(scene, st, op.prepare(P), envs)
    worst = 0.0
    for e in envs:
        a, bound, r_rgb, r_dep = ref[e]
        c = int(scene.cam_off[e])
        assert np.array_equal(rgb[c], r_rgb) and np.array_equal(dep[c], r_dep), f"env {e}: frames differ"
        err = np.abs(got[e].astype(np.float64) - a)
        assert np.all(err <= bound), f"env {e}: action error {err.max():.3g} > bound {bound[np.argmax(err)]:.3g}"
        worst = max(worst, float((err / bound).max()))
    say(f"{label}: {len(envs)} envs, worst error / bound {worst:.3g}")
    return got


def test_policy_actions_parity():
    """64 envs of the 1024-env config at 128x128, hidden 256, after a few
    steps (bodies in flight): layer 1 split over 256 chunks of K."""
    s = sg.config_scene(2, n_envs=64)
    P = sg.policy_weights(11, 128, 128, 256, 32)
    with vuda.World(s) as w:
        w.step(nsteps=30)
        w.set_policy(P)
        check_actions(w, s, P, range(s.n_envs), "policy c2[0:64] H256")


def test_policy_ragged_shapes():
    """50 envs (not a multiple of the 64-row tile) of 12 bodies and hidden
    96 (not a multiple of the 256-unit tile), 64x64 frames."""
    s = sg.make_scene(1004, [12] * 50, 64, mixed=True)
    P = sg.policy_weights(12, 64, 64, 96, 12)
    with vuda.World(s) as w:
        w.step(nsteps=5)
        w.set_policy(P)
        check_actions(w, s, P, range(s.n_envs), "policy 50 envs 64x64 H96")


def test_policy_layered_head_parity():
    """Layers 2 and 3 as batched float32 MFMA products, forced at hidden 256
    on 64 envs of the 1024-env config: within the oracle's bound, like the
    per-env head on the same frames."""
    s = sg.config_scene(2, n_envs=64)
    P = sg.policy_weights(11, 128, 128, 256, 32)
    with vuda.World(s) as w:
        w.step(nsteps=30)
        w.set_policy(P)
        check_actions(w, s, P, range(s.n_envs), "policy c2[0:64] H256 per-env head")
        w.set_tuning(vuda.TUNE_POLICY_LAYERED, 1)
        assert w.get_tuning(vuda.TUNE_POLICY_LAYERED) == 1
        check_actions(w, s, P, range(s.n_envs), "policy c2[0:64] H256 layered")


def test_policy_wide_hidden():
    """Hidden 2048 and 4096 (above the per-env head, so layers 2 and 3 run
    as batched products) over 100 envs (a 64-row tile and a ragged 36) of
    32x32 frames: K = 4096, split 16 ways in layer 1, 4 in layer 2 and 32 in
    layer 3 at hidden 4096."""
    s = sg.make_scene(1006, [16] * 100, 32, mixed=True)
    for H, seed in ((2048, 15), (4096, 16)):
        P = sg.policy_weights(seed, 32, 32, H, 16)
        with vuda.World(s) as w:
            w.step(nsteps=10)
            w.set_policy(P)
            check_actions(w, s, P, range(s.n_envs), f"policy 100 envs 32x32 H{H}")


def test_saturated_actions_drive_the_step():
    """A policy with zero weights acts exactly a_max clamp(b3): the step that
    follows matches the oracle's step with those forces."""
    s = sg.config_scene(2, n_envs=32)
    P = sg.policy_weights(13, 128, 128, 64, 16, a_max=4.0, zero=True)
    with vuda.World(s, debug=True) as w:
        w.step(nsteps=20)
        w.set_policy(P)
        for t in range(3):
            st_in = w.state()
            w.render()
            w.act()
            w.step()
            w.wait()
            a_known = np.float32(P["a_max"]) * np.clip(P["b3"], -1, 1)
            got = w.fetch(vuda.FETCH_ACTIONS).reshape(s.n_envs, -1)
            assert np.array_equal(got, np.broadcast_to(a_known, got.shape))
            st_g = w.state()
            cts = w.contacts()
            st_o = {k: v.copy() for k, v in st_in.items()}
            worst = 0.0
            for e in range(s.n_envs):
                b0, b1 = int(s.body_off[e]), int(s.body_off[e + 1])
                f = op.forces(a_known, b1 - b0, int(P["act_bodies"]))
                status, pairs = oracle.step_env(s, e, st_o, record_pairs=True, fext=f)
                assert status == 0
                for sub in range(s.substeps):
                    assert np.array_equal(cts[e][sub], pairs[sub]), f"env {e} substep {sub}: contact sets differ"
                g = {k: st_g[k][b0:b1] for k in STATE_KEYS}
                o = {k: st_o[k][b0:b1] for k in STATE_KEYS}
                worst = max(worst, state_close(g, o))
            assert worst <= 1e-5, f"state error {worst:.3g}"
        say(f"saturated policy: 3 steps, max state err {worst:.3g}")
        # without the policy the forces are gone: the plain step again
        w.set_policy(None)
        st_in = w.state()
        w.step()
        st_g = w.state()
        st_o = {k: v.copy() for k, v in st_in.items()}
        for e in range(s.n_envs):
            oracle.step_env(s, e, st_o)
        assert max(state_close({k: st_g[k] for k in STATE_KEYS}, {k: st_o[k] for k in STATE_KEYS}), 0) <= 1e-5


def test_policy_loop_same_in_every_schedule():
    """render -> act -> step in serialized and co-scheduled modes: the same
    bits (the events order the frames, the actions and the state)."""
    s = sg.config_scene(2, n_envs=48)
    P = sg.policy_weights(14, 128, 128, 128, 32)
    res = []
    for split in (0.0, 2.0, 0.5):
        with vuda.World(s) as w:
            w.set_policy(P)
            w.cosched(split)
            for _ in range(6):
                w.render()
                w.act()
                w.step()
            w.wait()
            res.append((w.state(), w.fetch(vuda.FETCH_ACTIONS)))
    for st, a in res[1:]:
        assert np.array_equal(a, res[0][1])
        for k in STATE_KEYS:
            assert np.array_equal(st[k], res[0][0][k]), k


def test_policy_errors():
    s = sg.config_scene(2, n_envs=4)
    with vuda.World(s) as w:
        with pytest.raises(vuda.VudaError):
            w.act()  # no policy
        bad = sg.policy_weights(1, 100, 61, 16, 4)  # 6100 pixels: not a multiple of 32
        with pytest.raises(vuda.VudaError):
            w.set_policy(bad)
        other = sg.policy_weights(1, 64, 64, 16, 4)  # the cameras are 128x128
        w.set_policy(other)
        with pytest.raises(vuda.VudaError):
            w.act()
        with pytest.raises(vuda.VudaError):
            w.set_policy(sg.policy_weights(1, 8, 8, 1100, 4))  # above 1024, not a multiple of 64
        with pytest.raises(vuda.VudaError):
            w.set_policy(sg.policy_weights(1, 8, 8, 8256, 4))  # above 8192
        # the batched layers 2-3 need a multiple of 64: refused at act time
        w.set_policy(sg.policy_weights(1, 128, 128, 96, 4))
        w.set_tuning(vuda.TUNE_POLICY_LAYERED, 1)
        with pytest.raises(vuda.VudaError):
            w.act()
        w.set_tuning(vuda.TUNE_POLICY_LAYERED, 0)
        w.act()
        w.wait()
