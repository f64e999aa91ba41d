"""Scheme variants (le_set_scheme) against the oracle's matching switches:
f of the advected phi through every advection variant, the midpoint sawtooth,
both together across a strain wrap, and switching back to the default."""
from __future__ import annotations

import dataclasses

import numpy as np
import pytest

from oracle import model_h as mh
from paper_0710_5912_amd import inputs

pytestmark = pytest.mark.gpu

le = pytest.importorskip("paper_0710_5912_amd.le")

KEYS = ("LE_TUNE_ADV", "LE_TUNE_MU", "LE_TUNE_COL_CH", "LE_TUNE_COL_FLOW", "LE_TUNE_ROW",
        "LE_TUNE_ROW_FWD")


def params(nx, ny, **kw):
    base = dict(nx=nx, ny=ny, lx=float(nx), ly=float(ny), gdot=0.3, A=1.0, B=1.0,
                kappa=1.0, M=1.0, eta=1.0, rho=1.0, dt=0.005)
    base.update(kw)
    return base


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def run_both(monkeypatch, p, steps, seed, f_half, midpoint_s, adv=None, upwind3=False,
             banded=False):
    if adv is not None:
        for k, v in zip(KEYS, (adv, 0, 0, 0, 0, 0)):
            monkeypatch.setenv(k, str(v))
    phi0 = inputs.noise_phi0(p["ny"], p["nx"], seed, amp=0.5)
    om0 = inputs.noise_omega0(p["ny"], p["nx"], seed) if p["rho"] > 0 else None
    print(f"case {p['nx']}x{p['ny']} rho={p['rho']} adv={adv} f_half={f_half} "
          f"midpoint_s={midpoint_s} upwind3={upwind3} steps={steps}", flush=True)
    with le.Context(p, phi0, om0) as c:
        c.set_scheme(f_half=f_half, midpoint_s=midpoint_s, upwind3=upwind3, banded=banded)
        c.step(steps)
        g = c.get_state()
    op = dataclasses.replace(mh.Params(**p), f_half=f_half, midpoint_s=midpoint_s,
                             upwind3=upwind3, banded=banded)
    st = mh.run(op, mh.initial_state(op, phi0, om0), steps)
    return g, st


@pytest.mark.parametrize("adv", [0, 4, 66, 100])
@pytest.mark.parametrize("rho", [1.0, 0.0])
def test_f_half_every_advection_variant(monkeypatch, adv, rho):
    p = params(256, 256, rho=rho)
    g, st = run_both(monkeypatch, p, 5, 31, True, False, adv)
    for k in ("phi", "psi") + (("omega",) if rho > 0 else ()):
        assert rel(g[k], getattr(st, k)) <= 1e-10, k


def test_both_variants_across_a_wrap(monkeypatch):
    """64^2, gdot = 0.5: the strain wraps at step 200; 220 steps."""
    p = params(64, 64, gdot=0.5)
    g, st = run_both(monkeypatch, p, 220, 32, True, True)
    assert g["wraps"] == st.wraps == 1
    for k in ("phi", "omega", "psi"):
        assert rel(g[k], getattr(st, k)) <= 1e-10, k


def test_midpoint_stokes_sheared_box(monkeypatch):
    p = params(128, 64, lx=128.0, ly=64.0, gdot=0.4, rho=0.0)
    g, st = run_both(monkeypatch, p, 60, 33, False, True)
    for k in ("phi", "psi"):
        assert rel(g[k], getattr(st, k)) <= 1e-10, k


def test_scheme_switches_back_and_rejects_unknown_flags():
    p = params(64, 64)
    phi0 = inputs.noise_phi0(64, 64, 34, amp=0.5)
    with le.Context(p, phi0) as c:
        c.set_scheme(f_half=True, midpoint_s=True)
        c.step(10)
        c.set_scheme()
        c.step(10)
        g = c.get_state()
        rc = le.lib().le_set_scheme(c._h, 16)
        assert rc == le.LE_EINVAL
    a = mh.Params(**p)
    b = dataclasses.replace(a, f_half=True, midpoint_s=True)
    st = mh.run(a, mh.run(b, mh.initial_state(b, phi0), 10), 10)
    assert rel(g["phi"], st.phi) <= 1e-10


def test_batch_scheme_equals_single_runs(fixed_variants):
    """le_batch_set_scheme: a batch of two grid classes with both variants on
    equals each run stepped alone with the same switches, bit for bit."""
    runs = [(params(64, 64, gdot=0.5), inputs.noise_phi0(64, 64, 35, amp=0.5)),
            (params(128, 64, lx=128.0, ly=64.0, gdot=0.2, rho=0.0),
             inputs.noise_phi0(64, 128, 36, amp=0.5))]
    b = le.Batch([r[0] for r in runs], [r[1] for r in runs])
    try:
        b.set_scheme(f_half=True, midpoint_s=True)
        b.step(30)
        for i, (p, phi0) in enumerate(runs):
            gb = b.get_state(i)
            with le.Context(p, phi0) as c:
                c.set_scheme(f_half=True, midpoint_s=True)
                c.step(30)
                gc = c.get_state()
            for k in ("phi", "psi"):
                assert np.array_equal(gb[k], gc[k]), (i, k)
    finally:
        b.close()


@pytest.mark.parametrize("adv", [136, 196])
@pytest.mark.parametrize("rho", [1.0, 0.0])
def test_f_half_batched_advection(monkeypatch, rho, adv):
    """f of the advected phi through the batched one-kernel advection (512^2)."""
    p = params(512, 512, rho=rho)
    g, st = run_both(monkeypatch, p, 3, 32, True, False, adv)
    for k in ("phi", "psi") + (("omega",) if rho > 0 else ()):
        assert rel(g[k], getattr(st, k)) <= 1e-10, k


@pytest.mark.parametrize("geom", [dict(nx=128, ny=128), dict(nx=256, ny=64, lx=256.0, ly=64.0)])
@pytest.mark.parametrize("rho", [1.0, 0.0])
def test_upwind3_matches_the_oracle(monkeypatch, geom, rho):
    """Third-order upwind advection (square cells, and r = 4 with the sheared
    samples four columns per row apart), 100 steps across a strain wrap."""
    p = params(gdot=0.5, rho=rho, **geom)
    steps = 220 if geom["nx"] == geom["ny"] else 100
    g, st = run_both(monkeypatch, p, steps, 33, False, False, upwind3=True)
    if geom["nx"] == geom["ny"]:
        assert g["wraps"] == st.wraps == 1
    for k in ("phi", "psi") + (("omega",) if rho > 0 else ()):
        assert rel(g[k], getattr(st, k)) <= 1e-10, k


def test_upwind3_with_the_other_switches_and_back(monkeypatch):
    """All three switches together, then back to the default scheme on the
    same context (the captured graphs of the other advection are dropped)."""
    p = params(128, 128, gdot=0.3)
    phi0 = inputs.noise_phi0(128, 128, 34, amp=0.5)
    om0 = inputs.noise_omega0(128, 128, 34)
    with le.Context(p, phi0, om0) as c:
        c.set_scheme(f_half=True, midpoint_s=True, upwind3=True)
        c.step(40)
        c.set_scheme()
        c.step(40)
        g = c.get_state()
    op = dataclasses.replace(mh.Params(**p), f_half=True, midpoint_s=True, upwind3=True)
    st = mh.run(op, mh.initial_state(op, phi0, om0), 40)
    st = mh.run(mh.Params(**p), st, 40)
    for k in ("phi", "omega", "psi"):
        assert rel(g[k], getattr(st, k)) <= 1e-10, k


@pytest.mark.parametrize("geom", [dict(nx=64, ny=64), dict(nx=128, ny=32, lx=128.0, ly=32.0)])
@pytest.mark.parametrize("rho", [1.0, 0.0])
def test_banded_matches_the_oracle(monkeypatch, geom, rho):
    """The banded scheme (cyclic banded y systems per x wavenumber, solved
    densely by the oracle) against the GPU's per-mode division by the banded
    operators' eigenvalues, 100 steps; the square case crosses a wrap."""
    p = params(gdot=0.5 if geom["nx"] == geom["ny"] else 0.2, rho=rho, **geom)
    steps = 220 if geom["nx"] == geom["ny"] else 100
    g, st = run_both(monkeypatch, p, steps, 35, False, False, banded=True)
    if geom["nx"] == geom["ny"]:
        assert g["wraps"] == st.wraps == 1
    for k in ("phi", "psi") + (("omega",) if rho > 0 else ()):
        assert rel(g[k], getattr(st, k)) <= 1e-10, k


def test_all_four_switches_together(monkeypatch):
    p = params(64, 64, gdot=0.3)
    g, st = run_both(monkeypatch, p, 60, 36, True, True, upwind3=True, banded=True)
    for k in ("phi", "omega", "psi"):
        assert rel(g[k], getattr(st, k)) <= 1e-10, k
