"""Workload presets against the paper's parameter tables."""
from paper_0710_5912_amd import configs


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
