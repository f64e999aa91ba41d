"""Characteristic length and time scales in the paper's units (G = Ly = tau_0 = 1).

TEST INFRASTRUCTURE ONLY (see the header of oracle.model_h).

From section "Lengthscales and timescales": the interfacial tension is
sigma = 2 sqrt(2) l G / 3 and, in the paper's units, M = kappa = l^2.  The
crossover scales follow by equating the diffusive, viscous and inertial growth
laws.  Table I prints L_DV and L_VI for every run and a figure comment prints
T_DV and 1/(gdot T_DV) for the DV series: tests/golden holds those values.
"""
from __future__ import annotations

import math

ALPHA = (2.0 * math.sqrt(2.0) / 3.0) ** (1.0 / 3.0)


def sigma(l: float) -> float:
    """Surface tension with G = 1."""
    return 2.0 * math.sqrt(2.0) * l / 3.0


def L_D(l: float, t: float) -> float:
    """Diffusive growth law (M sigma t)^(1/3) with M = l^2."""
    return (l * l * sigma(l) * t) ** (1.0 / 3.0)


def L_V(l: float, eta: float, t: float) -> float:
    """Viscous growth law sigma t / eta."""
    return sigma(l) * t / eta


def L_I(l: float, rho: float, t: float) -> float:
    """Inertial growth law (sigma t^2 / rho)^(1/3)."""
    return (sigma(l) * t * t / rho) ** (1.0 / 3.0)


def L_DV(l: float, eta: float) -> float:
    """Diffusive-to-viscous crossover length sqrt(M eta)."""
    return math.sqrt(l * l * eta)


def L_VI(l: float, eta: float, rho: float) -> float:
    """Viscous-to-inertial crossover length eta^2 / (rho sigma); inf at rho = 0."""
    if rho == 0.0:
        return math.inf
    return eta * eta / (rho * sigma(l))


def T_DV(l: float, eta: float) -> float:
    """Diffusive-to-viscous crossover time sqrt(M eta^3) / sigma."""
    return math.sqrt(l * l * eta ** 3) / sigma(l)


def T_VI(l: float, eta: float, rho: float) -> float:
    """Viscous-to-inertial crossover time eta^3 / (rho sigma^2)."""
    if rho == 0.0:
        return math.inf
    return eta ** 3 / (rho * sigma(l) ** 2)


def tau0(l: float) -> float:
    """Microscopic interfacial diffusion time (sqrt(2) l)^3 / (3 M sigma); 1 in these units."""
    return (math.sqrt(2.0) * l) ** 3 / (3.0 * l * l * sigma(l))
