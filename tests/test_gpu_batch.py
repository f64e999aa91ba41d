"""Batched runs: each run of a heterogeneous batch equals the same run alone.

Runs of different grids, shear rates (wrapping at different steps), inertia
and precision advance in one engine; every run must reproduce its single-run
result bit for bit (the kernels are the same, only the launch covers more
runs), and FP64 runs must match the oracle to 1e-10.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import model_h as mh
from paper_0710_5912_amd import configs, inputs

pytestmark = pytest.mark.gpu

le = pytest.importorskip("paper_0710_5912_amd.le")


def mixed_runs():
    runs = []
    for k, (n, nyy, rho, gdot, prec) in enumerate([
            (64, 64, 1.0, 0.4, "fp64"),
            (64, 64, 0.0, -0.3, "fp64"),
            (32, 32, 1.0, 2.0, "fp64"),      # wraps every 50 steps (c = 1)
            (128, 64, 1.0, 0.0, "fp64"),
            (64, 64, 1.0, 0.25, "fp32"),
            (32, 32, 0.0, 1.5, "fp32"),
            (64, 64, 1.0, 0.4, "fp64"),      # same class as run 0, other seed
    ]):
        p = configs.model_h(n, nyy, gdot=gdot, rho=rho)
        runs.append((p, prec, inputs.noise_phi0(nyy, n, 100 + k, amp=0.4)))
    return runs


def test_batch_equals_single_runs_bitwise(fixed_variants):
    runs = mixed_runs()
    print(f"batch of {len(runs)} runs, 130 steps", flush=True)
    b = le.Batch([r[0] for r in runs], [r[2] for r in runs],
                 precisions=[r[1] for r in runs])
    b.step(60)
    b.step(70)
    for i, (p, prec, phi0) in enumerate(runs):
        with le.Context(p, phi0, precision=prec) as c:
            c.step(60)
            c.step(70)
            ref = c.get_state()
            ro, rsk = c.observables()
        got = b.get_state(i)
        assert got["step"] == 130 and got["wraps"] == ref["wraps"], i
        for k in ("phi", "omega", "psi"):
            assert np.array_equal(got[k], ref[k]), (i, k)
        o, sk = b.observables(i)
        assert o["Ls"] == ro["Ls"] and o["sigma_xy"] == ro["sigma_xy"], i
        assert np.array_equal(sk, rsk), i
    b.close()


@pytest.mark.parametrize("adv,mu", [(98, 66), (68, 72)])
def test_batch_one_kernel_strips_equal_single_runs(monkeypatch, adv, mu):
    """The one-kernel strip stages (whole rows per block, grid z = run) over a
    batch of 256^2 and 512^2 runs (two runs per class, inertial and Stokes)
    reproduce each run alone with the same variants bit for bit."""
    for k, v in (("LE_TUNE_ADV", adv), ("LE_TUNE_MU", mu), ("LE_TUNE_COL_CH", 0),
                 ("LE_TUNE_COL_FLOW", 0), ("LE_TUNE_ROW", 0),
                 ("LE_TUNE_ROW_FWD", 0)):
        monkeypatch.setenv(k, str(v))
    runs = []
    for k, (n, rho, gdot) in enumerate([(256, 1.0, 0.3), (256, 1.0, -0.2), (512, 0.0, 0.1),
                                        (512, 0.0, 0.05)]):
        runs.append((configs.model_h(n, n, gdot=gdot, rho=rho),
                     inputs.noise_phi0(n, n, 300 + k, amp=0.4)))
    print(f"batch of {len(runs)} runs, advect {adv}, mu {mu}, 30 steps", flush=True)
    b = le.Batch([r[0] for r in runs], [r[1] for r in runs])
    assert all(t["advect"] == adv and t["mu_source"] == mu for t in b.tuning())
    b.step(30)
    for i, (p, phi0) in enumerate(runs):
        with le.Context(p, phi0) as c:
            c.step(30)
            ref = c.get_state()
        got = b.get_state(i)
        for k in ("phi", "omega", "psi"):
            assert np.array_equal(got[k], ref[k]), (i, k)
    b.close()


def test_batch_fp64_runs_match_oracle():
    runs = [r for r in mixed_runs() if r[1] == "fp64"][:4]
    b = le.Batch([r[0] for r in runs], [r[2] for r in runs])
    b.step(100)
    for i, (p, _, phi0) in enumerate(runs):
        op = mh.Params(**p)
        st = mh.run(op, mh.initial_state(op, phi0), 100)
        got = b.get_state(i)
        assert got["wraps"] == st.wraps
        for k in ("phi", "psi"):
            ref = getattr(st, k)
            err = np.max(np.abs(got[k] - ref)) / np.max(np.abs(ref))
            assert err <= 1e-10, (i, k, err)
    b.close()


def test_batch_rejects_bad_run_index_and_params():
    p = configs.model_h(32, 32)
    phi0 = inputs.noise_phi0(32, 32, 0)
    b = le.Batch([p], [phi0])
    with pytest.raises(le.LeError):
        b.get_state(1)
    b.close()
    with pytest.raises(le.LeError) as ei:
        le.Batch([p, dict(p, nx=48)], [phi0, np.zeros((32, 48))])
    assert ei.value.code == le.LE_EINVAL
