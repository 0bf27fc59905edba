"""LOPE_LOG=1: every compute call names the kernel it chose on stderr; without
it the library writes nothing."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROGRAM = """
import numpy as np, torch
import paper_1502_03504_amd as L, synth
case = synth.case_heat3d(n=40, dtype=np.float32, steps=3)
a = L.Grid.from_array(case.field[:, :33, :], 1)
b = a.empty_like()
L.lope_iterate(a, b, case.stencil, case.bc, 3)
c = synth.case_diffusion(n=20, steps=1)
u, k = L.Grid.from_array(c.u0, 1), L.Grid.from_array(c.kappa, 1)
L.lope_apply_var(u, u.empty_like(), k, c.dt, (("periodic",) * 3, 0.0))
g = L.Grid.allocate(c.u0.shape, 1, torch.float64, "cuda")
L.lope_apply_var_adjoint2(u, u.empty_like(), u, u, k, c.dt, (("periodic",) * 3, 0.0), g)
k2 = L.Grid.from_array(c.kappa, 2)
L.lope_apply_var_adjoint2(u, u.empty_like(), u, u, k2, c.dt, (("periodic",) * 3, 0.0), g)
torch.cuda.synchronize()
"""


def _run(env_extra):
    env = dict(os.environ)
    env.pop("LOPE_LOG", None)
    env.update(env_extra)
    r = subprocess.run([sys.executable, "-c", PROGRAM], cwd=ROOT, env=env, capture_output=True, text=True, timeout=180)
    assert r.returncode == 0, r.stderr[-2000:]
    return [line for line in r.stderr.splitlines() if line.startswith("lope: ")]


def test_log_names_each_kernel():
    lines = _run({"LOPE_LOG": "1"})
    assert any(line.startswith("lope: iterate 3 sweeps on 40x33x40 f32 radius 1: ") for line in lines), lines
    assert "lope: diffusion step on 20x20x20: k_varw_forward" in lines, lines
    # the wave pair needs its four inputs laid out alike; else the LDS pair runs
    assert "lope: diffusion reverse pair on 20x20x20: k_varw_adjoint2" in lines, lines
    assert "lope: diffusion reverse pair on 20x20x20: k_var_adjoint2" in lines, lines


def test_no_log_by_default():
    assert _run({}) == []
