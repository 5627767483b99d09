"""GPU parity of the physics step with regularized Coulomb friction, through
the C ABI, at the usual gates: contact-pair sets bit-exact every substep,
state within 1e-5 relative per step from identical input state."""
import dataclasses
import math

import numpy as np
import pytest

import oracle
from paper_2605_01352_amd import scenegen as sg
from paper_2605_01352_amd import vuda
from tests.gpu_util import compare_step, say
from tests.scenes import tiny_scene

pytestmark = pytest.mark.gpu


def run_steps(scene, steps, label):
    with vuda.World(scene, debug=True) as w:
        exact, worst = 0, 0.0
        for _ in range(steps):
            r = compare_step(w, scene)
            exact += r["bitexact"]
            worst = max(worst, r["max_err"])
        say(f"{label}: {steps} steps, bit-exact steps {exact}/{steps}, max state err {worst:.3g}")


def test_friction_c2_subset_parity():
    """32 envs of the 1024-env config with mu = 0.5: drops, impacts, sliding."""
    s = dataclasses.replace(sg.config_scene(2, n_envs=32), mu=0.5)
    run_steps(s, 40, "friction c2[0:32] mu 0.5")


def test_friction_settled_pile_parity():
    """Two c2 envs after 300 oracle steps with mu = 0.8 (resting contacts,
    slow slips below v_eps), then 10 steps on both sides."""
    s = dataclasses.replace(sg.config_scene(2, n_envs=2), mu=0.8)
    st = s.state()
    for _ in range(300):
        oracle.step_scene(s, st)
    for k, v in st.items():
        getattr(s, k)[:] = v
    run_steps(s, 10, "friction settled mu 0.8")


def test_friction_slope_closed_form_on_gpu():
    """A block on a 30 degree slope (tilted gravity) with mu = 0.3: from 0.5
    to 1 s its speed grows by g (sin t - mu cos t) 0.5 s."""
    th = math.radians(30.0)
    a = 0.05
    s = tiny_scene([dict(type=1, size=a, pos=(0.0, 0.0, a))], gravity=(9.81 * math.sin(th), 0.0, -9.81 * math.cos(th)),
                   mu=0.3, envs=4)
    with vuda.World(s) as w:
        w.step(nsteps=120)
        v1 = w.state()["vel"][:, 0].astype(np.float64)
        w.step(nsteps=120)
        v2 = w.state()["vel"][:, 0].astype(np.float64)
    expect = 0.5 * 9.81 * (math.sin(th) - 0.3 * math.cos(th))
    assert np.all(np.abs((v2 - v1) - expect) <= 1e-4 * expect)


def test_friction_parameter_errors():
    s = sg.config_scene(1, n_envs=2)
    for mu, v_eps in ((-0.1, 0.05), (float("nan"), 0.05), (0.5, 0.0), (0.5, float("inf"))):
        with pytest.raises(vuda.VudaError):
            vuda.World(dataclasses.replace(s, mu=mu, v_eps=v_eps))
    # without friction v_eps is not read
    with vuda.World(dataclasses.replace(s, mu=0.0, v_eps=0.0)) as w:
        w.step()
