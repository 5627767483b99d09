"""GPU parity of the separating-axis edge-edge contacts of boxes and cubes
(edge_contacts = 1) through the C ABI, at the usual gates: contact-pair
sets bit-exact every substep, state within 1e-5 relative per step from
identical input state."""
import dataclasses
import math

import numpy as np
import pytest

import oracle
from paper_2605_01352_amd import scenegen as sg
from paper_2605_01352_amd import vuda
from tests.gpu_util import compare_render, compare_step, say
from tests.scenes import quat_axis_angle, tiny_scene

pytestmark = pytest.mark.gpu


def run_steps(scene, steps, label):
    with vuda.World(scene, debug=True) as w:
        worst = 0.0
        for _ in range(steps):
            worst = max(worst, compare_step(w, scene)["max_err"])
        compare_render(w, scene)
        say(f"{label}: {steps} steps, max state err {worst:.3g}")


def ridges(envs=2):
    """Cubes dropped crosswise onto ridges (cubes and a box turned 45 deg)."""
    a = 0.05
    h = a * math.sqrt(2.0)
    bodies = [dict(type=1, size=a, pos=(0.0, 0.0, h), quat=quat_axis_angle((1, 0, 0), math.pi / 4)),
              dict(type=1, size=a, pos=(0.0, 0.0, 3 * h + 0.01), quat=quat_axis_angle((0, 1, 0), math.pi / 4)),
              dict(type=2, ext=(0.09, 0.04, 0.03), pos=(0.4, 0.0, 0.06), quat=quat_axis_angle((1, 0, 0), 0.9)),
              dict(type=2, ext=(0.06, 0.05, 0.02), pos=(0.4, 0.01, 0.2), quat=quat_axis_angle((0, 1, 1), 0.8))]
    return dataclasses.replace(tiny_scene(bodies, envs=envs), edge_contacts=True)


def test_edge_ridges_parity():
    s = ridges()
    # the ridges do cross edge to edge during the run
    st = s.state()
    crossed = False
    for _ in range(40):
        oracle.step_scene(s, st)
        pts = oracle.narrowphase(s, st, 0, 1)
        off = oracle.narrowphase(dataclasses.replace(s, edge_contacts=False), st, 0, 1)
        crossed = crossed or len(pts) > len(off)
    assert crossed
    run_steps(s, 60, "edge ridges")


def test_edge_c2_boxes_parity():
    s = dataclasses.replace(sg.with_boxes(sg.config_scene(2, n_envs=16)), edge_contacts=True)
    run_steps(s, 40, "edge c2[0:16] boxes")


def test_edge_settled_pile_with_friction_parity():
    s = dataclasses.replace(sg.with_boxes(sg.config_scene(2, n_envs=2), every=1), edge_contacts=True, mu=0.5)
    st = s.state()
    for _ in range(300):
        oracle.step_scene(s, st)
    for k, v in st.items():
        getattr(s, k)[:] = v
    run_steps(s, 10, "edge settled mu 0.5")


def test_edge_flag_errors():
    s = sg.config_scene(1, n_envs=2)
    with pytest.raises(vuda.VudaError):
        vuda.World(s, phys={"edge_contacts": 2})


def test_edge_boxes_two_wave_envs_parity():
    """Envs of 100 bodies (the two-wave physics kernel) with boxes and edge
    points, 20 steps."""
    s = sg.make_scene(4242, np.full(6, 100), 128, mixed=True, name="b100")
    s = dataclasses.replace(sg.with_boxes(s), edge_contacts=True)
    run_steps(s, 20, "edge boxes 100 bodies")
