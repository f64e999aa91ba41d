"""Parity at the full workload sizes, in the configuration the bench runs.

The bench's grids (1024^2 and 4096^2, FP64 and FP32 bulk, autotuned kernel
variants as the bench gets them) against the FP64 oracle on the same seeded
input: whole fields after a few steps (the oracle takes ~1 s per 1024^2 step
and ~25 s per 4096^2 step on one core), and mean-phi conservation over many
steps (a property that holds at any size).
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import model_h as mh
from paper_0710_5912_amd import configs, inputs

pytestmark = pytest.mark.gpu

le = pytest.importorskip("paper_0710_5912_amd.le")


def rel(a, b):
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


_ORACLE = {}


def pair(p, steps, precision, seed=0, amp=0.05):
    n = p["nx"]
    phi0 = inputs.noise_phi0(p["ny"], n, seed, amp=amp)
    om0 = inputs.noise_omega0(p["ny"], n, seed) if p["rho"] > 0 else None
    print(f"case {n}^2 rho={p['rho']} {precision} steps={steps} seed={seed}", flush=True)
    with le.Context(p, phi0, om0, precision=precision) as c:
        t = c.tuning()[0]
        c.step(steps)
        g = c.get_state()
    key = (tuple(sorted(p.items())), steps, seed, amp)
    if key not in _ORACLE:
        op = mh.Params(**p)
        _ORACLE.clear()
        _ORACLE[key] = mh.run(op, mh.initial_state(op, phi0, om0), steps)
    return g, _ORACLE[key], t


@pytest.mark.parametrize("rho", [1.0, 0.0])
def test_bench_workload_1024_fp64(rho):
    """The bench's 1024^2 workload (gdot = 0.01), 3 steps, whole fields."""
    p = configs.single_1024(rho=rho, gdot=0.01)["params"]
    g, st, t = pair(p, 3, "fp64", amp=0.5)
    print("variants", t, flush=True)
    for k in ("phi", "psi") + (("omega",) if rho > 0 else ()):
        assert rel(g[k], getattr(st, k)) <= 1e-10, k


def test_bench_workload_1024_fp32():
    p = configs.single_1024(rho=1.0, gdot=0.01)["params"]
    g, st, _ = pair(p, 3, "fp32", amp=0.5)
    assert rel(g["phi"], st.phi) <= 2e-5
    assert rel(g["psi"], st.psi) <= 2e-4


@pytest.mark.parametrize("precision,tol,tol_flow", [("fp64", 1e-10, 1e-10), ("fp32", 2e-5, 2e-4)])
def test_large_workload_4096_two_steps(precision, tol, tol_flow):
    """The bench's 4096^2 headline workload (inertial, gdot = 0.001), two steps
    against the oracle, every field (FP32 bulk: omega and psi within the FP32
    bound of the flow fields)."""
    p = configs.LARGE_4096["params"]
    g, st, t = pair(p, 2, precision, amp=0.5)
    print("variants", t, {k: rel(g[k], getattr(st, k)) for k in ("phi", "omega", "psi")},
          flush=True)
    assert rel(g["phi"], st.phi) <= tol
    assert rel(g["omega"], st.omega) <= tol_flow
    assert rel(g["psi"], st.psi) <= tol_flow


def test_large_workload_4096_graph_replayed_steps():
    """The headline workload in the bench's launch configuration: eight FP64
    steps as one graph piece (captured, then replayed by a second call), every
    field against the oracle at 1e-10, with the autotuned kernel variants."""
    p = configs.LARGE_4096["params"]
    phi0 = inputs.noise_phi0(4096, 4096, 4, amp=0.5)
    print("case 4096^2 fp64 two graph-replayed calls of 8 steps, seed 4", flush=True)
    with le.Context(p, phi0) as c:
        c.step(8)          # captures the 8-step graph and launches it
        c.step(8)          # replays it
        g = c.get_state()
        print("variants", c.tuning()[0], flush=True)
    op = mh.Params(**p)
    st = mh.initial_state(op, phi0, None)
    for k in range(16):
        st = mh.step(op, st)
        print(f"oracle step {k + 1}/16", flush=True)
    for k in ("phi", "omega", "psi"):
        r = rel(g[k], getattr(st, k))
        print(k, r, flush=True)
        assert r <= 1e-10, k


def test_large_workload_4096_mean_phi_and_finiteness():
    """200 steps at 4096^2: mean phi conserved to 1e-13, state finite."""
    p = configs.LARGE_4096["params"]
    phi0 = inputs.noise_phi0(4096, 4096, 3, amp=0.05, mean=0.02)
    with le.Context(p, phi0) as c:
        c.step(200)
        o, _ = c.observables(sk=False)
    assert o["finite"] == 1
    assert abs(o["mean_phi"] - float(np.mean(phi0))) <= 1e-13
