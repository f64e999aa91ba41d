"""The inertialess sheared series of Table I (sets DV1s .. DV6s) in paper
units: the step against the oracle at those parameters, and a short series
through the runner."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import model_h as mh
from paper_0710_5912_amd import configs, inputs

pytestmark = pytest.mark.gpu

le = pytest.importorskip("paper_0710_5912_amd.le")
series = pytest.importorskip("paper_0710_5912_amd.series")


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("name", ["DV1s", "DV4s", "DV6s"])
def test_dv_step_matches_oracle(name):
    """1024 x 512, box 2 x 1, kappa = M = l^2, rho = 0: 20 steps, FP64."""
    p = configs.dv_sheared(name)
    phi0 = inputs.noise_phi0(512, 1024, 41, amp=configs.DV_AMP)
    print(f"case {name} 1024x512 20 steps", flush=True)
    with le.Context(p, phi0) as c:
        c.step(20)
        g = c.get_state()
    op = mh.Params(**p)
    st = mh.run(op, mh.initial_state(op, phi0, None), 20)
    assert rel(g["phi"], st.phi) <= 1e-10
    assert rel(g["psi"], st.psi) <= 1e-10


def test_dv_refined_step_matches_oracle():
    """DV6s on the refined grid (2048 x 1024, half the mesh interval at the same
    l, dt = 0.004): 10 steps, FP64."""
    p = configs.dv_sheared("DV6s", 2)
    phi0 = inputs.noise_phi0(1024, 2048, 45, amp=configs.DV_AMP)
    print("case DV6s 2048x1024 10 steps", flush=True)
    with le.Context(p, phi0) as c:
        c.step(10)
        g = c.get_state()
    op = mh.Params(**p)
    st = mh.run(op, mh.initial_state(op, phi0, None), 10)
    assert rel(g["phi"], st.phi) <= 1e-10
    assert rel(g["psi"], st.psi) <= 1e-10


def test_dv_series_runner():
    """DV4s for 3000 steps sampled every 500: strain = gdot t, mean phi kept,
    every sample finite, the domains coarsen."""
    p = configs.dv_sheared("DV4s")
    phi0 = inputs.noise_phi0(512, 1024, 42, amp=configs.DV_AMP)
    r = series.run_series(p, phi0, 3000, 500)
    assert len(r["t"]) == 6
    assert np.allclose(r["t"], p["dt"] * np.arange(500, 3001, 500), rtol=1e-12)
    assert np.allclose(r["strain"], p["gdot"] * r["t"], rtol=1e-12)
    assert np.max(np.abs(r["mean_phi"] - phi0.mean())) <= 1e-13
    assert r["Ls"][-1] > r["Ls"][0] > 0.0
    assert r["site_updates_per_s"] > 0.0


@pytest.mark.parametrize("name", ["DV2u", "DV5u"])
def test_dv_unsheared_step_matches_oracle(name):
    """Zero-shear sets on 512^2 (box 1): 20 steps against the oracle, FP64."""
    p = configs.dv_unsheared(name)
    phi0 = inputs.noise_phi0(512, 512, 43, amp=configs.DV_AMP)
    print(f"case {name} 512x512 20 steps", flush=True)
    with le.Context(p, phi0) as c:
        c.step(20)
        g = c.get_state()
    op = mh.Params(**p)
    st = mh.run(op, mh.initial_state(op, phi0, None), 20)
    assert rel(g["phi"], st.phi) <= 1e-10
    assert rel(g["psi"], st.psi) <= 1e-10


@pytest.mark.parametrize("name", ["R029bs", "R028s"])
def test_inertial_sheared_step_matches_oracle(name):
    """Table I sets R029bs and R028s (inertial, sheared, 1024 x 512; R028s has
    the lowest density of the table): 20 steps, FP64."""
    p = configs.r_sheared(name)
    phi0 = inputs.noise_phi0(512, 1024, 44, amp=configs.DV_AMP)
    print(f"case {name} 1024x512 20 steps", flush=True)
    with le.Context(p, phi0) as c:
        c.step(20)
        g = c.get_state()
    op = mh.Params(**p)
    st = mh.run(op, mh.initial_state(op, phi0, None), 20)
    for k in ("phi", "omega", "psi"):
        assert rel(g[k], getattr(st, k)) <= 1e-10, k
