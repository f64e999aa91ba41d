"""Workload presets against the paper's parameter tables, and the growth-law
fit of the coarsening series."""
import numpy as np
import pytest

from oracle import model_h as mh

from paper_0710_5912_amd import configs, series


def test_dv_sheared_presets_follow_table_one():
    """Sets DV1s .. DV6s of Table I: (eta, gdot) per set, l = 0.00156 giving
    kappa = M = l^2, rho = 0, box 2 x 1 on 1024 x 512, dt = 0.016."""
    table = {"DV1s": (1000.0, 0.01), "DV2s": (100.0, 0.01), "DV3s": (10.0, 0.01),
             "DV4s": (1.0, 0.01), "DV5s": (0.3, 0.01), "DV6s": (0.1, 0.03)}
    for name, (eta, gdot) in table.items():
        p = configs.dv_sheared(name)
        assert (p["eta"], p["gdot"], p["rho"]) == (eta, gdot, 0.0)
        assert p["kappa"] == p["M"] == 0.00156 ** 2
        assert (p["nx"], p["ny"], p["lx"], p["ly"], p["dt"]) == (1024, 512, 2.0, 1.0, 0.016)
        assert p["A"] == p["B"] == 1.0


def test_dv_unsheared_presets_follow_table_one():
    """Sets DV1u .. DV6u of Table I: eta per set, zero shear, 512^2, box 1."""
    table = {"DV1u": 1000.0, "DV2u": 100.0, "DV3u": 10.0, "DV4u": 1.0, "DV5u": 0.3,
             "DV6u": 0.1}
    for name, eta in table.items():
        p = configs.dv_unsheared(name)
        assert (p["eta"], p["gdot"], p["rho"]) == (eta, 0.0, 0.0)
        assert p["kappa"] == p["M"] == 0.00156 ** 2
        assert (p["nx"], p["ny"], p["lx"], p["ly"], p["dt"]) == (512, 512, 1.0, 1.0, 0.016)


def test_fit_power_recovers_a_known_law():
    """L = a (t - t0)^p sampled on a grid: the fit returns p and t0 (close to
    the grid of offsets), after dropping t < t_min and cutting at L_max."""
    t = np.arange(20.0, 3000.0, 10.0)
    for p, t0, a in ((1.0 / 3.0, 15.0, 1e-3), (2.0 / 3.0, -30.0, 1e-4)):
        L = a * (t - t0) ** p
        e, ti, n = series.fit_power(t, L, t_min=40.0, L_max=0.02)
        assert abs(e - p) < 0.01, (p, e)
        assert abs(ti - t0) < 2.0, (t0, ti)
        assert n >= 4 and n < t.size


def test_inertial_sheared_presets_and_crossover_scales():
    """Table I inertial sheared sets: (eta, rho, gdot, dt) per set, and the
    crossover length L_VI = eta^2 / (rho sigma) reproduces the table's column
    (sigma = 2 sqrt(2) l / 3) to 1% (R022bs differs by 0.9%, the other sets
    by at most 0.2%)."""
    table = {"R028bs": (0.444, 8704.0, 0.0765, 0.008, 0.0154),
             "R022bs": (0.339, 22590.0, 0.0355, 0.008, 0.00349),
             "R029bs": (0.0809, 8037.0, 0.0591, 0.008, 0.000554),
             "R020s": (0.0785, 16180.0, 0.0256, 0.008, 0.000259),
             "R030s": (0.0122, 6250.0, 0.0410, 0.004, 0.0000162),
             "R019s": (0.00876, 32814.0, 0.0251, 0.004, 0.00000159),
             "R032s": (0.00391, 20067.0, 0.051, 0.004, 0.000000518),
             "R028s": (0.111, 136.0, 0.0765, 0.008, 0.0616),
             "R022s": (0.196, 2510.0, 0.0205, 0.008, 0.0104),
             "R029s": (0.0467, 893.0, 0.0341, 0.008, 0.00166)}
    assert set(table) == set(configs.R_SHEARED) | set(configs.R_SHEARED_LB)
    for name, (eta, rho, gdot, dt, lvi) in table.items():
        p = configs.r_sheared(name)
        assert (p["eta"], p["rho"], p["gdot"], p["dt"]) == (eta, rho, gdot, dt)
        assert (p["nx"], p["ny"], p["lx"], p["ly"]) == (1024, 512, 2.0, 1.0)
        L_VI, t_VI = series.visco_inertial_scales(p)
        assert abs(L_VI - lvi) <= 0.01 * lvi, (name, L_VI, lvi)
        assert abs(t_VI - L_VI * eta / series.interfacial_tension(p)) <= 1e-12 * t_VI
    assert abs(series.interfacial_tension(configs.r_sheared("R020s"))
               - 2.0 * np.sqrt(2.0) * 0.00156 / 3.0) <= 1e-15


def test_power_fit_slope_and_error():
    """An exact power law gives its exponent with zero error; scatter of known
    size gives the textbook standard error of a regression slope."""
    x = np.logspace(-7, -0.5, 7)
    e, se = series.power_fit(x, 3.0 * x ** -0.62)
    assert abs(e + 0.62) < 1e-12 and se < 1e-12
    rng = np.random.default_rng(5)
    noise = rng.normal(0.0, 0.05, x.size)
    e, se = series.power_fit(x, 3.0 * x ** -0.62 * np.exp(noise))
    lx = np.log(x)
    ly = np.log(3.0 * x ** -0.62 * np.exp(noise))
    # textbook simple regression: slope from centred sums, intercept from the
    # means, standard error from the residual variance over n - 2
    sxx = np.sum((lx - lx.mean()) ** 2)
    slope = np.sum((lx - lx.mean()) * (ly - ly.mean())) / sxx
    resid = ly - (ly.mean() + slope * (lx - lx.mean()))
    expect = np.sqrt((resid @ resid) / (x.size - 2) / sxx)
    assert abs(e - slope) <= 1e-12
    assert abs(se - expect) <= 1e-10 * expect


def test_inertial_unsheared_presets_follow_table_one():
    """Sets R028u .. R032u of Table I: (eta, rho), zero shear, 512^2, box 1,
    dt = 0.008."""
    table = {"R028u": (0.111, 136.0), "R022u": (0.196, 2510.0), "R029u": (0.0467, 893.0),
             "R020u": (0.0785, 16180.0), "R030u": (0.0122, 6250.0),
             "R019u": (0.00876, 32814.0), "R032u": (0.00391, 20067.0)}
    for name, (eta, rho) in table.items():
        p = configs.r_unsheared(name)
        assert (p["eta"], p["rho"], p["gdot"], p["dt"]) == (eta, rho, 0.0, 0.008)
        assert (p["nx"], p["ny"], p["lx"], p["ly"]) == (512, 512, 1.0, 1.0)


def test_explicit_ch_number_is_the_oracle_stability_edge():
    """A Nyquist-corner perturbation of phi = 1 under the oracle's Cahn-Hilliard
    stage (Appendix B, stage 1b; no flow) decays at explicit_ch_number 0.98 and
    grows at 1.02: the number is the edge of the linearised scheme (the nabla^4
    Crank-Nicolson part cancels from the edge; kappa is small here so that it
    does not also pull the growth factor towards -1 on both sides).  Under shear the bound's lab
    wavenumber 5 (pi/delta)^2 caps the oracle's |lambda| at s = -1 and is
    reached to within the grid's last modes."""
    base = dict(nx=32, ny=32, lx=1.0, ly=1.0, gdot=0.0, A=1.0, B=1.0, kappa=1e-6,
                M=0.7e-3, eta=1.0, rho=0.0, dt=1.0)
    unit = series.explicit_ch_number(base)
    j, i = np.mgrid[0:32, 0:32]
    mode = np.where((i + j) % 2 == 0, 1.0, -1.0)
    growth = {}
    for target in (0.98, 1.02):
        p = dict(base, dt=target / unit)
        assert abs(series.explicit_ch_number(p) - target) < 1e-12
        op = mh.Params(**p)
        phi = 1.0 + 1e-8 * mode
        for _ in range(200):
            phi = mh.stage_cahn_hilliard(op, phi, phi ** 3, 0.0)
        growth[target] = float(np.max(np.abs(phi - 1.0)) / 1e-8)
    assert growth[0.98] < 1e-2 and growth[1.02] > 1e2, growth
    sh = mh.Params(nx=128, ny=64, lx=2.0, ly=1.0, gdot=0.01)
    lam_max = float(np.max(-mh.symbol_laplacian(sh, -1.0)))
    bound = 5.0 * (np.pi * 64) ** 2
    assert 0.9 * bound < lam_max <= bound


def test_presets_within_the_explicit_bound():
    """Every Table I preset (and the refined DV grids) keeps the explicit
    Cahn-Hilliard terms stable; the refined sheared grid at the table's dt
    would not (2.0), hence its dt = 0.004."""
    ps = [configs.dv_sheared(n, r) for n in configs.DV_SHEARED for r in (1, 2)]
    ps += [configs.dv_unsheared(n, r) for n in configs.DV_UNSHEARED for r in (1, 2)]
    ps += [configs.r_sheared(n, r) for n in list(configs.R_SHEARED) + list(configs.R_SHEARED_LB)
           for r in (1, 2)]
    ps += [configs.r_unsheared(n, r) for n in configs.R_UNSHEARED for r in (1, 2)]
    assert all(series.explicit_ch_number(p) <= 0.81 for p in ps)
    p = configs.dv_sheared("DV6s", 2)
    assert (p["nx"], p["ny"], p["dt"]) == (2048, 1024, 0.004)
    assert configs.dv_unsheared("DV6u", 2)["nx"] == 1024
    assert abs(series.explicit_ch_number(dict(p, dt=0.016)) - 2.0148) < 1e-3
    with pytest.raises(ValueError):
        configs.dv_sheared("DV1s", 3)


def test_campaign_set_selection():
    """The campaigns' --sets subset keeps the table's index (the seed offset)
    and rejects unknown names."""
    from paper_0710_5912_amd import campaigns
    assert campaigns._pick(configs.DV_SHEARED, "DV5s,DV6s") == [(4, "DV5s"), (5, "DV6s")]
    assert [n for _, n in campaigns._pick(configs.R_SHEARED, "")] == list(configs.R_SHEARED)
    with pytest.raises(SystemExit):
        campaigns._pick(configs.DV_SHEARED, "DV7s")
    p = configs.r_sheared("R028bs", 2)
    assert (p["nx"], p["ny"], p["dt"]) == (2048, 1024, 0.004)
    assert configs.r_sheared("R032s", 2)["dt"] == 0.004
