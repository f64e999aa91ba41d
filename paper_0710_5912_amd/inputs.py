"""Seeded synthetic inputs shared by the GPU path's tests and the oracle's.

Holds none of the method's arithmetic: only the random initial conditions of
the paper's quench protocol (section "Numerical results": phi drawn i.i.d.
from a flat distribution per grid point, omega = 0), generated with NumPy's
PCG64 so that both sides receive bit-identical arrays.
"""
from __future__ import annotations

import numpy as np


def noise_phi0(ny: int, nx: int, seed: int, amp: float = 0.05,
               mean: float = 0.0) -> np.ndarray:
    """phi0[j, i] ~ mean + U(-amp, amp), shape (ny, nx), float64, C order."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(mean + rng.uniform(-amp, amp, (ny, nx)))


def noise_omega0(ny: int, nx: int, seed: int, amp: float = 0.05) -> np.ndarray:
    """A nonzero vorticity field for tests that start with flow (omega0 = 0 in the paper)."""
    rng = np.random.default_rng(seed + 7919)
    return np.ascontiguousarray(rng.uniform(-amp, amp, (ny, nx)))


def zeros(ny: int, nx: int) -> np.ndarray:
    return np.zeros((ny, nx), dtype=np.float64)


def batch_draws(nruns: int, seed: int = 1000):
    """Per-run shear rates log-uniform in [1e-3, 1e-1] for the batched workload."""
    rng = np.random.default_rng(seed)
    return 10.0 ** rng.uniform(-3.0, -1.0, nruns)


CNN_LAYERS = ((2, 32), (32, 32), (32, 32), (32, 2))


def cnn_init_params(seed: int = 0) -> np.ndarray:
    """Seeded initial weights of the corrector network (float64 vector).

    Layout per layer: W[co][ci][ky][kx] then b[co]; W uniform in
    +-0.5 sqrt(6 / (9 ci)), b = 0.
    """
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in CNN_LAYERS:
        bound = np.sqrt(6.0 / (9 * ci)) * 0.5
        parts.append(rng.uniform(-bound, bound, co * ci * 9))
        parts.append(np.zeros(co))
    return np.concatenate(parts)
