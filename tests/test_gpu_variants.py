"""Every kernel variant the autotuner may pick computes the same step.

The variants of a stage (fused stencil-and-transform kernel or strip stencil
plus in-place row transforms; column block shapes) are forced one by one
through LE_TUNE_* at creation and each run is checked against the FP64 oracle
(1e-10 relative, max norm) at sizes where the column shapes differ (512^2)
and across a strain wrap.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import model_h as mh
from paper_0710_5912_amd import inputs

pytestmark = pytest.mark.gpu

le = pytest.importorskip("paper_0710_5912_amd.le")

KEYS = ("LE_TUNE_ADV", "LE_TUNE_MU", "LE_TUNE_COL_CH", "LE_TUNE_COL_FLOW", "LE_TUNE_ROW")
# the row shape of a combination is forced for the forward and the inverse row
# transforms alike
# (advect, mu_source, column_ch, column_flow, row)
# advect 64 + k / 96 + k, mu_source 64 + k: strip stencil and row transforms
# in one kernel (k-row strips; advect with two / one x pairs per thread);
# advect and mu_source 128 + k / 192 + k / 256 + k: the batched one-kernel
# forms (k-row strips in batches of four / two / two rows; at 512 the two-row
# 16-value form falls back to the strips); strips shorter than a batch (130,
# 129, 193) leave the batch's last rows unstored
COMBOS = [(0, 0, 0, 0, 0), (4, 4, 1, 1, 1), (32, 32, 2, 2, 2), (8, 16, 3, 3, 3),
          (2, 2, 0, 0, 1), (66, 4, 0, 1, 2), (72, 8, 2, 0, 0), (100, 2, 1, 3, 0),
          (98, 66, 0, 0, 3), (4, 68, 1, 1, 0), (100, 72, 3, 2, 1), (8, 8, 4, 4, 4),
          (68, 68, 4, 3, 5), (4, 4, 2, 4, 5), (132, 4, 0, 3, 5), (136, 68, 4, 4, 4),
          (160, 8, 3, 0, 0), (194, 4, 4, 3, 5), (200, 68, 0, 1, 2),
          (132, 132, 0, 0, 0), (196, 196, 3, 3, 5), (136, 144, 1, 2, 4), (4, 194, 4, 4, 1),
          (68, 200, 2, 1, 3), (258, 260, 0, 3, 5), (264, 258, 1, 1, 2),
          (130, 129, 0, 0, 0), (193, 193, 1, 1, 1), (257, 130, 2, 2, 2)]


def params(nx, ny, **kw):
    base = dict(nx=nx, ny=ny, lx=float(nx), ly=float(ny), gdot=0.3, A=1.0, B=1.0,
                kappa=1.0, M=1.0, eta=1.0, rho=1.0, dt=0.005)
    base.update(kw)
    return base


def rel(a, b):
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


_ORACLE = {}


def oracle(p, steps, seed):
    key = (tuple(sorted(p.items())), steps, seed)
    if key not in _ORACLE:
        phi0 = inputs.noise_phi0(p["ny"], p["nx"], seed, amp=0.5)
        om0 = inputs.noise_omega0(p["ny"], p["nx"], seed) if p["rho"] > 0 else None
        op = mh.Params(**p)
        _ORACLE[key] = (phi0, om0, mh.run(op, mh.initial_state(op, phi0, om0), steps))
    return _ORACLE[key]


def run_forced(monkeypatch, p, steps, seed, combo, precision="fp64"):
    for k, v in zip(KEYS, combo):
        monkeypatch.setenv(k, str(v))
    monkeypatch.setenv("LE_TUNE_ROW_FWD", str(combo[4]))
    phi0, om0, st = oracle(p, steps, seed)
    print(f"case nx={p['nx']} ny={p['ny']} rho={p['rho']} steps={steps} combo={combo} "
          f"{precision}", flush=True)
    with le.Context(p, phi0, om0, precision=precision) as c:
        t = c.tuning()[0]
        c.step(steps)
        g = c.get_state()
    assert (t["advect"], t["mu_source"], t["column_ch"], t["column_flow"], t["row"]) == combo
    assert t["row_fwd"] == combo[4]
    return g, st


@pytest.mark.parametrize("combo", COMBOS)
@pytest.mark.parametrize("rho", [1.0, 0.0])
def test_variants_512_fp64(monkeypatch, combo, rho):
    p = params(512, 512, rho=rho)
    g, st = run_forced(monkeypatch, p, 3, 21, combo)
    for k in ("phi", "psi") + (("omega",) if rho > 0 else ()):
        assert rel(g[k], getattr(st, k)) <= 1e-10, k


@pytest.mark.parametrize("combo", [(4, 4, 1, 3, 1), (32, 8, 3, 2, 3), (68, 4, 0, 0, 1),
                                   (98, 8, 2, 1, 2), (66, 68, 1, 1, 2), (8, 4, 4, 4, 4), (16, 8, 3, 4, 5),
                                   (144, 8, 0, 2, 4), (132, 136, 0, 2, 4), (194, 196, 3, 3, 3)])
def test_variants_512_fp32(monkeypatch, combo):
    """FP32 shapes (16 values per thread in shapes 2 and 3) within the FP32 bound."""
    p = params(512, 512)
    g, st = run_forced(monkeypatch, p, 3, 22, combo, precision="fp32")
    assert rel(g["phi"], st.phi) <= 2e-5
    assert rel(g["psi"], st.psi) <= 2e-4


@pytest.mark.parametrize("combo", [(4, 4, 0, 2, 1), (16, 32, 3, 0, 2), (2, 2, 2, 1, 3),
                                   (68, 68, 0, 0, 0)])
def test_strip_variants_across_a_wrap(monkeypatch, combo):
    """64^2, gdot = 0.5: the strain wraps at step 200; 220 steps."""
    p = params(64, 64, gdot=0.5)
    g, st = run_forced(monkeypatch, p, 220, 23, combo)
    assert g["wraps"] == st.wraps == 1
    for k in ("phi", "omega", "psi"):
        assert rel(g[k], getattr(st, k)) <= 1e-10, k


@pytest.mark.parametrize("combo", [(8, 8, 2, 3, 3), (66, 8, 0, 1, 0), (104, 4, 1, 0, 1)])
def test_strip_variants_non_square_cells(monkeypatch, combo):
    """nx = 4 ny (r = 4): the strip advect reads the diagonal pairs; the mu
    strip applies to square cells only and falls back."""
    p = params(256, 64, gdot=0.2, lx=256.0, ly=64.0)
    g, st = run_forced(monkeypatch, p, 20, 24, combo)
    for k in ("phi", "omega", "psi"):
        assert rel(g[k], getattr(st, k)) <= 1e-10, k


@pytest.mark.parametrize("combo", [(68, 4, 0, 0, 0), (100, 8, 1, 1, 3), (66, 2, 2, 3, 1)])
def test_one_kernel_strips_flat_grid(monkeypatch, combo):
    """nx = 64 ny (512 x 8, r = 64): strips longer than the grid, every row a
    halo row of the next, the diagonal pairs read r = 64 columns away."""
    p = params(512, 8, gdot=0.05, lx=512.0, ly=8.0)
    g, st = run_forced(monkeypatch, p, 30, 26, combo)
    for k in ("phi", "omega", "psi"):
        assert rel(g[k], getattr(st, k)) <= 1e-10, k


def test_autotuner_reports_valid_choices():
    p = params(256, 256)
    with le.Context(p, inputs.noise_phi0(256, 256, 0)) as c:
        t = c.tuning()
    assert len(t) == 1
    t = t[0]
    assert (t["nx"], t["ny"], t["precision"], t["inertial"]) == (256, 256, 0, 1)
    batched = (132, 136, 144, 194, 196, 200, 258, 260, 264)
    assert t["advect"] in (0, 2, 4, 8, 16, 32, 66, 68, 72, 98, 100, 104) + batched
    assert t["mu_source"] in (0, 2, 4, 8, 16, 32, 66, 68, 72) + batched
    assert t["column_ch"] in range(5) and t["column_flow"] in range(5) and t["row"] in range(6)
    assert t["row_fwd"] in range(6)


@pytest.mark.parametrize("rho", [1.0, 0.0])
def test_stage_timer_leaves_the_state(monkeypatch, rho):
    """le_time_stage launches each stage back to back without touching the
    state: the run continues bit for bit as its untimed twin (both with the
    same variants, fixed here)."""
    for k, v in zip(KEYS, (4, 4, 0, 0, 1)):
        monkeypatch.setenv(k, str(v))
    monkeypatch.setenv("LE_TUNE_ROW_FWD", "1")
    p = params(128, 128, rho=rho)
    phi0 = inputs.noise_phi0(128, 128, 31, amp=0.5)
    with le.Context(p, phi0) as a, le.Context(p, phi0) as b:
        for ctx in (a, b):
            ctx.step(5)
        before = a.get_state()
        for s in le.STAGES:
            assert a.time_stage(s, 3) > 0.0
        after = a.get_state()
        for k in ("phi", "omega", "psi"):
            assert np.array_equal(before[k], after[k]), k
        a.step(7)
        b.step(7)
        ga, gb = a.get_state(), b.get_state()
        for k in ("phi", "omega", "psi"):
            assert np.array_equal(ga[k], gb[k]), k


@pytest.mark.parametrize("col", range(5))
@pytest.mark.parametrize("rho", [1.0, 0.0])
def test_column_shapes_at_4096_point_columns(monkeypatch, col, rho):
    """16 x 4096 (gdot = 0): the column passes transform 4096-point columns,
    the length of the largest grid, in every block shape."""
    p = params(16, 4096, gdot=0.0, rho=rho)
    g, st = run_forced(monkeypatch, p, 3, 27, (0, 0, col, col, 0))
    for k in ("phi", "psi") + (("omega",) if rho > 0 else ()):
        assert rel(g[k], getattr(st, k)) <= 1e-10, k


@pytest.mark.parametrize("adv", [4, 136, 196])
@pytest.mark.parametrize("row", range(6))
def test_row_shapes_at_4096_point_rows(monkeypatch, row, adv):
    """4096 x 16 (gdot = 0.05, r = 256): 4096-point rows in every row shape,
    with the two-kernel strip stages (real rows through the real scratch) and
    the batched one-kernel advection."""
    p = params(4096, 16, gdot=0.05)
    g, st = run_forced(monkeypatch, p, 3, 28, (adv, 8, 0, 0, row))
    for k in ("phi", "omega", "psi"):
        assert rel(g[k], getattr(st, k)) <= 1e-10, k


@pytest.mark.parametrize("n,combo", [(1024, (132, 132, 3, 3, 5)), (1024, (196, 200, 2, 2, 4)),
                                     (1024, (258, 260, 0, 0, 0)), (2048, (136, 136, 3, 3, 5)),
                                     (2048, (260, 258, 0, 3, 5))])
def test_batched_mu_source_long_rows(monkeypatch, n, combo):
    """The batched one-kernel advect and mu_source forms at 1024^2 and 2048^2
    (FP64, two steps) against the oracle, every field."""
    p = params(n, n, gdot=0.01)
    g, st = run_forced(monkeypatch, p, 2, 30, combo)
    for k in ("phi", "omega", "psi"):
        assert rel(g[k], getattr(st, k)) <= 1e-10, k


@pytest.mark.parametrize("combo", [(132, 4, 0, 0, 0), (144, 8, 1, 1, 1), (194, 2, 3, 3, 3)])
def test_batched_advection_non_square_cells(monkeypatch, combo):
    """512 x 128 (r = 4, gdot = 0.2, strain wrap inside): the batched
    one-kernel advection reads the diagonal pairs r = 4 columns away."""
    p = params(512, 128, gdot=0.2, lx=512.0, ly=128.0)
    g, st = run_forced(monkeypatch, p, 20, 29, combo)
    for k in ("phi", "omega", "psi"):
        assert rel(g[k], getattr(st, k)) <= 1e-10, k


def test_tuning_cache_gives_equal_kernels_and_results(tmp_path, monkeypatch):
    """Contexts of one shape created in one process take the cached choices of
    the first (equal results bit for bit); LE_TUNE_CACHE writes them to a file
    that a later process would read."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("LE_TUNE_CACHE", str(cache))
    p = params(128, 16, gdot=0.2, lx=128.0, ly=16.0)   # a shape no other test tunes (FP32)
    phi0 = inputs.noise_phi0(16, 128, 41, amp=0.5)
    with le.Context(p, phi0, precision="fp32") as a, le.Context(p, phi0, precision="fp32") as b:
        assert a.tuning() == b.tuning()
        a.step(30)
        b.step(30)
        ga, gb = a.get_state(), b.get_state()
    for k in ("phi", "omega", "psi"):
        assert np.array_equal(ga[k], gb[k]), k
    lines = cache.read_text().split("\n")
    rec = [list(map(int, l.split())) for l in lines if l.strip()]
    with le.Context(p, phi0, precision="fp32") as c:
        t = c.tuning()[0]
    assert any(r[1:6] == [128, 16, 1, 1, 1] and
               r[6:] == [t["advect"], t["mu_source"], t["column_ch"], t["column_flow"],
                         t["row"], t["row_fwd"]] for r in rec), rec
