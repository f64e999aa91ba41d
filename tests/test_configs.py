"""Workload presets against the paper's parameter tables, and the growth-law
fit of the coarsening series."""
import numpy as np

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
