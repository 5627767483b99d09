"""Trajectory divergence between the GPU and the oracle, each running free.

The per-step gate compares one step from identical input.  Here both sides
start from the spawn and run 100 steps on their own, and the largest
position difference max_b |p_gpu - p_oracle| is reported at every step.  It
is reported, not gated: a contact-rich scene is chaotic, so one rounding
difference can grow.  The test only requires that the report exists and is
finite.  Printed lines: `divergence <config> step <t> max_dp <m> bit_equal
<0|1>`, then a summary.
"""
import numpy as np
import pytest

import oracle
from paper_2605_01352_amd import scenegen as sg
from paper_2605_01352_amd import vuda
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def free_run_divergence(scene, steps):
    st_o = scene.state()
    out = []
    with vuda.World(scene) as w:
        for t in range(1, steps + 1):
            w.step()
            oracle.step_scene(scene, st_o)
            g = w.state()
            dp = np.linalg.norm(g["pos"].astype(np.float64) - st_o["pos"].astype(np.float64), axis=1)
            same = all(np.array_equal(g[k], st_o[k]) for k in ("pos", "vel", "quat", "omega"))
            out.append((float(dp.max()) if dp.size else 0.0, same))
    return out


@pytest.mark.parametrize("cfg,n_envs", [(1, 16), (2, 32)])
def test_free_running_divergence_report(cfg, n_envs):
    scene = sg.config_scene(cfg, n_envs=n_envs)
    rep = free_run_divergence(scene, 100)
    for t, (m, same) in enumerate(rep, 1):
        if t in (1, 2, 5, 10, 20, 50, 100) or t % 25 == 0:
            say(f"divergence c{cfg}[0:{n_envs}] step {t} max_dp {m:.3e} bit_equal {int(same)}")
    worst = max(m for m, _ in rep)
    n_same = sum(s for _, s in rep)
    first = next((t for t, (m, s) in enumerate(rep, 1) if not s), None)
    say(f"divergence c{cfg}[0:{n_envs}] summary: max_dp over 100 steps {worst:.3e} m, "
        f"bit-equal states in {n_same}/100 steps, first difference at step {first}")
    assert all(np.isfinite(m) for m, _ in rep)
