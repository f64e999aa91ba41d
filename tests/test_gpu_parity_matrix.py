"""Parity matrix at 256^2 and the bench workloads, FP64 against the oracle.

256^2 (several column and row tiles), rho in {0, 1} x gdot in {0, 0.01, 0.1},
100 steps, each sheared case started 50 steps before a strain wrap (the state
set at that step by le_set_fields, psi re-solved by both sides from the flow
constraint at the step's strain offset); the 1024^2 bench-size inertial
workload over 100 steps.  Bar: 1e-10 relative, max norm, for every field.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import pytest

from oracle import model_h as mh
from paper_0710_5912_amd import configs, inputs

pytestmark = pytest.mark.gpu

le = pytest.importorskip("paper_0710_5912_amd.le")


def rel(a, b):
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


def oracle_state_at(op, phi, omega, n):
    """The oracle's state at step n from phi, omega: psi from the flow
    constraint at s(t_n) (Poisson from omega, or the Stokes solve from phi)."""
    s = mh.strain_offset(op, n)
    if op.rho > 0:
        w = omega - omega.mean()
        _, psi = mh.stage_flow(dataclasses.replace(op, dt=0.0), w, np.zeros_like(w), s)
    else:
        w = np.zeros_like(phi)
        _, psi = mh.stage_flow(op, w, mh.vorticity_source(op, phi, s), s)
    return mh.State(phi=phi.copy(), omega=w, psi=psi, step=n, wraps=mh.wrap_count(op, n))


@pytest.mark.parametrize("gdot", [0.0, 0.01, 0.1])
@pytest.mark.parametrize("rho", [1.0, 0.0])
def test_matrix_256_fp64_100_steps(rho, gdot):
    p = configs.model_h(256, 256, gdot=gdot, rho=rho)
    op = mh.Params(**p)
    # 50 steps before the first wrap (strain 1/2 at c = 1), or from 0 unsheared
    n0 = 0 if gdot == 0 else int(round(0.5 / (gdot * p["dt"]))) - 50
    seed = 500 + int(100 * gdot) + int(rho)
    phi = inputs.noise_phi0(256, 256, seed, amp=0.5)
    om = inputs.noise_omega0(256, 256, seed) if rho > 0 else np.zeros_like(phi)
    om = om - om.mean()
    print(f"matrix case rho={rho} gdot={gdot} from step {n0}", flush=True)
    st = mh.run(op, oracle_state_at(op, phi, om, n0), 100)
    with le.Context(p, np.zeros_like(phi)) as c:
        c.set_fields(phi, om if rho > 0 else None, n0)
        c.step(100)
        g = c.get_state()
    assert g["step"] == st.step == n0 + 100 and g["wraps"] == st.wraps
    if gdot > 0:
        assert st.wraps == 1
    for k in ("phi", "psi") + (("omega",) if rho > 0 else ()):
        assert rel(g[k], getattr(st, k)) <= 1e-10, k


def test_bench_size_1024_fp64_100_steps():
    """The 1024^2 inertial workload (gdot = 0.01), 100 steps, whole fields."""
    p = configs.single_1024(rho=1.0, gdot=0.01)["params"]
    phi0 = inputs.noise_phi0(1024, 1024, 0, amp=0.05)
    print("1024^2 fp64 100 steps", flush=True)
    with le.Context(p, phi0) as c:
        c.step(100)
        g = c.get_state()
    op = mh.Params(**p)
    st = mh.run(op, mh.initial_state(op, phi0), 100)
    for k in ("phi", "omega", "psi"):
        assert rel(g[k], getattr(st, k)) <= 1e-10, k
