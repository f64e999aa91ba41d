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
