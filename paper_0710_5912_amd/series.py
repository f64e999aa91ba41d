"""Time series of one run: the characteristic lengths against strain.

Drives a Context through `steps` steps and samples the observables every
`every` steps (Section VI: L_s from the structure factor, L_par and L_perp
from the principal axes of the second-moment tensor of S(q), the excess
shear stress).  Every step and observable runs in the library; this module
only loops and collects.
"""
from __future__ import annotations

import time

import numpy as np

from . import le


def run_series(params, phi0, steps: int, every: int, precision: str = "fp64", stream=None,
               on_sample=None):
    """Advance a run from phi0 (omega0 = 0) and return the sampled series:
    dict of arrays t, strain, Ls, L_par, L_perp, sigma_xy, mean_phi, plus the
    GPU-side wall time of the stepping (seconds) and the site-updates/s.
    on_sample(steps_done, observables) is called after each sample."""
    keys = ("t", "strain", "Ls", "L_par", "L_perp", "sigma_xy", "mean_phi")
    out = {k: [] for k in keys}
    wall = 0.0
    with le.Context(params, phi0, precision=precision, stream=stream) as c:
        done = 0
        while done < steps:
            n = min(every, steps - done)
            t0 = time.perf_counter()
            c.step(n)
            o, _ = c.observables(sk=False)   # synchronises
            wall += time.perf_counter() - t0
            done += n
            if not o["finite"]:
                raise FloatingPointError(f"state not finite at step {done}")
            for k in keys:
                out[k].append(o[k])
            if on_sample is not None:
                on_sample(done, o)
    res = {k: np.asarray(v) for k, v in out.items()}
    res["wall_s"] = wall
    res["site_updates_per_s"] = params["nx"] * params["ny"] * steps / wall
    return res


def explicit_ch_number(params):
    """dt M max|q_lab|^2 (3B - A) / 2 for a run: the Cahn-Hilliard terms taken
    explicitly (the A and f terms of Appendix B) stay stable while it is <= 1
    (linearised about phi = +-1).  In the cosheared frame the lab wave vector
    is (q_x, q_y - s q_x) with |s| <= Lx / (2 Ly) under shear, so the largest
    |q_lab|^2 is reached at the corner mode with the largest |s|."""
    qx = np.pi * params["nx"] / params["lx"]
    qy = np.pi * params["ny"] / params["ly"]
    smax = params["lx"] / (2.0 * params["ly"]) if params["gdot"] != 0.0 else 0.0
    q2 = qx * qx + (qy + smax * qx) ** 2
    return params["dt"] * params["M"] * q2 * (3.0 * params["B"] - params["A"]) / 2.0


def fit_power(t, L, t_min: float = 40.0, L_max: float = 0.02, n_int: int = 400):
    """Growth exponent of a coarsening segment (the protocol of Section VIII A): samples
    with t < t_min are discarded as the initial transient, the segment is cut
    once L reaches L_max, and an offset t_int is subtracted from t.  t_int is
    chosen (on a grid in [-4 t_first, t_first)) as the one whose straight-line
    fit of log L against log(t - t_int) leaves the smallest residual; returns
    (exponent, t_int, number of samples)."""
    t = np.asarray(t, dtype=float)
    L = np.asarray(L, dtype=float)
    keep = t >= t_min
    t, L = t[keep], L[keep]
    if L.size and np.any(L >= L_max):
        stop = int(np.argmax(L >= L_max))
        t, L = t[:stop], L[:stop]
    if t.size < 4:
        raise ValueError("too few samples in the segment")
    y = np.log(L)
    best = None
    for ti in np.linspace(-4.0 * t[0], t[0], n_int, endpoint=False):
        x = np.log(t - ti)
        a = np.vstack([x, np.ones_like(x)]).T
        coef, res, _, _ = np.linalg.lstsq(a, y, rcond=None)
        r = float(np.sum((a @ coef - y) ** 2))
        if best is None or r < best[0]:
            best = (r, float(coef[0]), float(ti))
    return best[1], best[2], int(t.size)


def interfacial_tension(params) -> float:
    """sigma = sqrt(8 kappa A^3 / (9 B^2)) of the flat interface of the
    phi^4 free energy; with A = B = G and kappa = l^2 G this is the paper's
    2 sqrt(2) l G / 3 (Section II)."""
    return float(np.sqrt(8.0 * params["kappa"] * params["A"] ** 3 / (9.0 * params["B"] ** 2)))


def visco_inertial_scales(params):
    """(L_VI, t_VI) = (eta^2 / (rho sigma), eta^3 / (rho sigma^2)), the
    viscous-to-inertial crossover length and time (Section VI)."""
    s = interfacial_tension(params)
    eta, rho = params["eta"], params["rho"]
    return eta * eta / (rho * s), eta ** 3 / (rho * s * s)


def steady_average(res, strain_min: float = 100.0):
    """Mean and standard deviation of L_par and L_perp over the samples with
    strain >= strain_min (the steady-state averages of the scaling plot)."""
    keep = res["strain"] >= strain_min
    if not np.any(keep):
        raise ValueError("no samples past the strain cut")
    lp, lq = res["L_par"][keep], res["L_perp"][keep]
    return dict(L_par=float(lp.mean()), L_par_sd=float(lp.std()), L_perp=float(lq.mean()),
                L_perp_sd=float(lq.std()), samples=int(keep.sum()))


def power_fit(x, y):
    """Least-squares slope of log y against log x and its standard error
    (the power-law fits of the steady-state scaling plot, Section VIII B)."""
    lx = np.log(np.asarray(x, dtype=float))
    ly = np.log(np.asarray(y, dtype=float))
    a = np.vstack([lx, np.ones_like(lx)]).T
    coef, _, _, _ = np.linalg.lstsq(a, ly, rcond=None)
    r = ly - a @ coef
    s2 = float(r @ r) / max(1, lx.size - 2)
    cov = s2 * np.linalg.inv(a.T @ a)
    return float(coef[0]), float(np.sqrt(cov[0, 0]))
