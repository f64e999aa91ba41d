"""Named workloads (parameter sets only; no arithmetic of the method).

Common setting: A = B = kappa = M = 1, grid spacing 1 (box = grid), eta = 1,
dt = 0.005, phi0 = U(-0.05, 0.05) per site, omega0 = 0.
"""
from __future__ import annotations


def model_h(nx, ny, gdot=0.01, rho=1.0, eta=1.0, dt=0.005, lx=None, ly=None,
            A=1.0, B=1.0, kappa=1.0, M=1.0):
    return dict(nx=nx, ny=ny, lx=float(nx if lx is None else lx),
                ly=float(ny if ly is None else ly), gdot=gdot, A=A, B=B,
                kappa=kappa, M=M, eta=eta, rho=rho, dt=dt)


# 64x64 inertial, gdot = 0.01, 200 steps: the case the oracle finishes in seconds.
SMALL_64 = dict(params=model_h(64, 64, gdot=0.01, rho=1.0), steps=200, amp=0.05)

# 1024x1024 single run, inertial and Stokes, gdot in {0.001, 0.01}: the
# throughput workload (10^4 steps in the full protocol).
def single_1024(rho=1.0, gdot=0.01):
    return dict(params=model_h(1024, 1024, gdot=gdot, rho=rho), steps=10000, amp=0.05)


# 4096x4096 inertial, gdot = 0.001: the large single-GPU case.
LARGE_4096 = dict(params=model_h(4096, 4096, gdot=0.001, rho=1.0), steps=50000, amp=0.05)


def paper_units(l, eta, rho, gdot, lx, nx, ny, dt):
    """Table I parameters mapped to A = B = 1, kappa = M = l^2, Ly = 1."""
    return dict(nx=nx, ny=ny, lx=float(lx), ly=1.0, gdot=gdot, A=1.0, B=1.0,
                kappa=l * l, M=l * l, eta=eta, rho=rho, dt=dt)


def _refine(refine):
    if refine not in (1, 2):
        raise ValueError("refine must be 1 (the grid of Table I) or 2 (half its mesh interval)")
    return refine


# Inertialess sheared series of Table I (sets DV1s .. DV6s): l = 0.00156,
# rho = 0, box 2 x 1, 1024 x 512, dt = 0.016; the sets differ in eta and
# the shear rate.  phi0 uniform in [-0.01, 0.01] (the initial condition of
# Section VIII).
DV_SHEARED = {
    "DV1s": (1000.0, 0.01),
    "DV2s": (100.0, 0.01),
    "DV3s": (10.0, 0.01),
    "DV4s": (1.0, 0.01),
    "DV5s": (0.3, 0.01),
    "DV6s": (0.1, 0.03),
}
DV_AMP = 0.01


def dv_sheared(name, refine=1):
    """refine = 2: half the mesh interval at the same l (2048 x 1024).  The
    explicit Cahn-Hilliard terms then need dt = 0.004: with |s| up to 1 the
    lab wavenumber reaches |q|^2 = 5 (pi / delta)^2 (series.explicit_ch_number)."""
    eta, gdot = DV_SHEARED[name]
    r = _refine(refine)
    return paper_units(0.00156, eta, 0.0, gdot, 2.0, 1024 * r, 512 * r, 0.016 / (r * r))


# Zero-shear diffusive-to-viscous series of Table I (sets DV1u .. DV6u):
# l = 0.00156, rho = 0, box 1 x 1 on 512 x 512, dt = 0.016.
DV_UNSHEARED = {
    "DV1u": 1000.0,
    "DV2u": 100.0,
    "DV3u": 10.0,
    "DV4u": 1.0,
    "DV5u": 0.3,
    "DV6u": 0.1,
}


def dv_unsheared(name, refine=1):
    """refine = 2: 1024^2 at the same l and dt (still within the explicit bound)."""
    r = _refine(refine)
    return paper_units(0.00156, DV_UNSHEARED[name], 0.0, 0.0, 1.0, 512 * r, 512 * r, 0.016)


# Inertial sheared sets of Table I used for the steady-state scaling plot
# (R028bs, R022bs, R029bs, R020s, R030s, R019s, R032s): (eta, rho, gdot, dt);
# l = 0.00156, box 2 x 1 on 1024 x 512.
R_SHEARED = {
    "R028bs": (0.444, 8704.0, 0.0765, 0.008),
    "R022bs": (0.339, 22590.0, 0.0355, 0.008),
    "R029bs": (0.0809, 8037.0, 0.0591, 0.008),
    "R020s": (0.0785, 16180.0, 0.0256, 0.008),
    "R030s": (0.0122, 6250.0, 0.0410, 0.004),
    "R019s": (0.00876, 32814.0, 0.0251, 0.004),
    "R032s": (0.00391, 20067.0, 0.051, 0.004),
}


# The three remaining inertial sheared sets of Table I (the lattice Boltzmann
# parameters as first converted; the scaling plot of Section VIII B uses their
# revised counterparts R028bs, R022bs, R029bs above): (eta, rho, gdot, dt).
R_SHEARED_LB = {
    "R028s": (0.111, 136.0, 0.0765, 0.008),
    "R022s": (0.196, 2510.0, 0.0205, 0.008),
    "R029s": (0.0467, 893.0, 0.0341, 0.008),
}


def r_sheared(name, refine=1):
    """refine = 2: half the mesh interval at the same l (2048 x 1024), with dt
    capped at 0.004 for the explicit Cahn-Hilliard terms."""
    eta, rho, gdot, dt = R_SHEARED[name] if name in R_SHEARED else R_SHEARED_LB[name]
    r = _refine(refine)
    return paper_units(0.00156, eta, rho, gdot, 2.0, 1024 * r, 512 * r,
                       min(dt, 0.016 / (r * r)))


# Zero-shear viscous-to-inertial series of Table I (sets R028u .. R032u):
# (eta, rho); l = 0.00156, box 1 x 1 on 512 x 512, dt = 0.008.
R_UNSHEARED = {
    "R028u": (0.111, 136.0),
    "R022u": (0.196, 2510.0),
    "R029u": (0.0467, 893.0),
    "R020u": (0.0785, 16180.0),
    "R030u": (0.0122, 6250.0),
    "R019u": (0.00876, 32814.0),
    "R032u": (0.00391, 20067.0),
}


def r_unsheared(name, refine=1):
    """refine = 2: 1024^2 at the same l and dt (within the explicit bound)."""
    eta, rho = R_UNSHEARED[name]
    r = _refine(refine)
    return paper_units(0.00156, eta, rho, 0.0, 1.0, 512 * r, 512 * r, 0.008)
