"""Time series of one run: the characteristic lengths against strain.

Drives a Context through `steps` steps and samples the observables every
`every` steps (Section IV: L_s from the structure factor, L_par and L_perp
from the principal axes of the second-moment tensor of S(q), the excess
shear stress).  Every step and observable runs in the library; this module
only loops and collects.
"""
from __future__ import annotations

import time

import numpy as np

from . import le


def run_series(params, phi0, steps: int, every: int, precision: str = "fp64", stream=None):
    """Advance a run from phi0 (omega0 = 0) and return the sampled series:
    dict of arrays t, strain, Ls, L_par, L_perp, sigma_xy, mean_phi, plus the
    GPU-side wall time of the stepping (seconds) and the site-updates/s."""
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
    res = {k: np.asarray(v) for k, v in out.items()}
    res["wall_s"] = wall
    res["site_updates_per_s"] = params["nx"] * params["ny"] * steps / wall
    return res


def fit_power(t, L, t_min: float = 40.0, L_max: float = 0.02, n_int: int = 400):
    """Growth exponent of a coarsening segment (Section V A protocol): samples
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
