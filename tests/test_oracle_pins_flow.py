"""Pins of the oracle's flow coupling against continuum identities.

These cover the parts of the step that the single-mode and energy pins leave
open: the scale of the vorticity source g (1/eta on the Stokes branch, 1/rho
on the inertial one), the start of the omega Crank-Nicolson update from the
advected omega (reading Q6), and the midpoint sawtooth of the scheme switch.
Each pin compares the oracle with something computed independently of it
(spectral derivatives, a pseudo-spectral RK4 integration of the vorticity
equation, a closed-form product), and each has a companion test that plants
the plausible slip in the oracle (on the CPU, by monkeypatching) and checks
that the pin then fails.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import model_h as mh


# ------------------------------------------------------------ helpers

def _spec(p, a):
    """Independent spectral d_x a, d_y a and Laplacian (odd derivatives zero at Nyquist)."""
    kx = 2 * math.pi * np.fft.fftfreq(p.nx, d=p.dx)
    ky = 2 * math.pi * np.fft.fftfreq(p.ny, d=p.dy)
    kxo, kyo = kx.copy(), ky.copy()
    kxo[p.nx // 2] = 0.0
    kyo[p.ny // 2] = 0.0
    A = np.fft.fft2(a)
    ax = np.real(np.fft.ifft2(1j * kxo[None, :] * A))
    ay = np.real(np.fft.ifft2(1j * kyo[:, None] * A))
    lap = np.real(np.fft.ifft2(-(kx[None, :] ** 2 + ky[:, None] ** 2) * A))
    return ax, ay, lap


def _two_scale_phi(p):
    """Smooth phi made of modes of different |q| (so grad mu is not parallel to grad phi)."""
    j, i = np.meshgrid(np.arange(p.ny), np.arange(p.nx), indexing="ij")
    x, y = 2 * math.pi * i / p.nx, 2 * math.pi * j / p.ny
    return 0.5 * np.cos(x) * np.sin(2 * y) + 0.3 * np.sin(3 * x + y) + 0.05


def _mu_and_K(p, phi):
    """Continuum mu = B phi^3 - A phi - kappa lap phi and K = d_x phi d_y mu - d_y phi d_x mu."""
    px, py, plap = _spec(p, phi)
    mu = p.B * phi ** 3 - p.A * phi - p.kappa * plap
    mx, my, _ = _spec(p, mu)
    return mu, mx, my, px * my - py * mx


def _orders(d):
    return [math.log2(d[k] / d[k + 1]) for k in range(len(d) - 1)]


def _scaled_source(scale):
    """A vorticity source with the bracket scaled by scale(p) instead of -1/rho or -1/eta."""
    def vs(p, phi, s):
        mu = mh.chemical_potential(p, phi, s)
        return scale(p) * mh.korteweg_bracket(p, phi, mu, s)
    return vs


# -------------------------------------- Stokes branch: power balance

def stokes_power_defect(N, eta):
    """|P_in - D| / D for the oracle's Stokes solve at gamma-dot = 0.

    Force balance eta lap v = grad p + phi grad mu with div v = 0 gives, on a
    torus, the power balance  int v . (-phi grad mu) = eta int omega^2.  psi is
    the oracle's (stage 2a source, zero-Reynolds solve); v = (d_y psi, -d_x psi),
    omega = -lap psi, mu and its gradient are formed spectrally.  The discrete
    scheme meets it up to its O(delta^2) truncation error.
    """
    p = mh.Params(nx=N, ny=N, lx=32.0, ly=32.0, rho=0.0, eta=eta, kappa=1.5, A=1.0, B=1.0)
    phi = _two_scale_phi(p)
    g = mh.vorticity_source(p, phi, 0.0)
    _, psi = mh.stage_flow(p, np.zeros_like(phi), g, 0.0)
    _, mx, my, _ = _mu_and_K(p, phi)
    sx, sy, slap = _spec(p, psi)
    p_in = np.sum(sy * (-phi * mx) + (-sx) * (-phi * my))
    diss = eta * np.sum(slap ** 2)
    return abs(p_in - diss) / diss


@pytest.mark.parametrize("eta", [0.5, 2.0])
def test_stokes_power_balance(eta):
    d = [stokes_power_defect(N, eta) for N in (32, 64, 128)]
    assert all(abs(o - 2.0) < 0.3 for o in _orders(d)), d
    assert d[-1] < 0.015, d


def test_stokes_power_balance_catches_a_dropped_viscosity(monkeypatch):
    """g = -K (the 1/eta dropped) or -K eta: the balance misses by a factor of eta."""
    for scale in (lambda p: -1.0, lambda p: -p.eta):
        monkeypatch.setattr(mh, "vorticity_source", _scaled_source(scale))
        assert stokes_power_defect(128, 2.0) > 0.3


# -------------------------------------- inertial branch: impulse from rest

def impulse_defect(N, rho, dt=1e-4):
    """From rest (omega = psi = 0) one step gives omega^1 / dt -> -K / rho.

    The advection of omega vanishes, Crank-Nicolson multiplies dt G by
    1 / (1 - dt nu lambda / 2) = 1 + O(dt), and K at phi^1 differs from K at
    phi^0 by O(dt): the defect is O(dt + delta^2) against K formed spectrally.
    """
    p = mh.Params(nx=N, ny=N, lx=32.0, ly=32.0, rho=rho, eta=1.0, kappa=1.5, dt=dt)
    phi = _two_scale_phi(p)
    st = mh.step(p, mh.initial_state(p, phi))
    _, _, _, K = _mu_and_K(p, phi)
    ref = -K / rho
    return float(np.max(np.abs(st.omega / dt - ref)) / np.max(np.abs(ref)))


@pytest.mark.parametrize("rho", [0.5, 2.0])
def test_inertial_impulse_from_rest(rho):
    d = [impulse_defect(N, rho) for N in (32, 64, 128)]
    assert all(abs(o - 2.0) < 0.3 for o in _orders(d)), d
    assert d[-1] < 0.03, d


def test_inertial_impulse_catches_a_density_slip(monkeypatch):
    """g = -K rho (rho and 1/rho swapped) misses by rho^2."""
    monkeypatch.setattr(mh, "vorticity_source", _scaled_source(lambda p: -p.rho))
    for rho in (0.5, 2.0):
        assert impulse_defect(128, rho) > 0.5


# ------------------------------- omega advection (reading Q6) vs the continuum

def _rk4_vorticity(N, L, om0, nu, T, dt):
    """Pseudo-spectral RK4 (2/3-rule dealiased) of d_t w + v . grad w = nu lap w
    with v = (d_y psi, -d_x psi), lap psi = -w: the 2D Navier-Stokes vorticity
    equation of the paper's Appendix A at uniform phi, written independently."""
    k = 2 * math.pi * np.fft.fftfreq(N, d=L / N)
    KX, KY = k[None, :], k[:, None]
    K2 = KX ** 2 + KY ** 2
    K2s = K2.copy()
    K2s[0, 0] = 1.0
    kmax = np.max(np.abs(k))
    keep = (np.abs(KX) < 2 * kmax / 3) & (np.abs(KY) < 2 * kmax / 3)

    def rhs(W):
        Psi = W / K2s
        Psi[0, 0] = 0.0
        vx = np.real(np.fft.ifft2(1j * KY * Psi))
        vy = np.real(np.fft.ifft2(-1j * KX * Psi))
        wx = np.real(np.fft.ifft2(1j * KX * W))
        wy = np.real(np.fft.ifft2(1j * KY * W))
        return -np.fft.fft2(vx * wx + vy * wy) * keep - nu * K2 * W

    W = np.fft.fft2(om0)
    for _ in range(int(round(T / dt))):
        k1 = rhs(W)
        k2 = rhs(W + 0.5 * dt * k1)
        k3 = rhs(W + 0.5 * dt * k2)
        k4 = rhs(W + dt * k3)
        W = W + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
    return np.real(np.fft.ifft2(W))


_N, _L, _NU, _T = 128, 2 * math.pi, 0.05, 1.0


@pytest.fixture(scope="module")
def vorticity_reference():
    j, i = np.meshgrid(np.arange(_N), np.arange(_N), indexing="ij")
    x, y = _L * i / _N, _L * j / _N
    om0 = np.cos(x) + np.cos(2 * y)        # |q| = 1 and 2: v . grad omega != 0
    return om0, _rk4_vorticity(_N, _L, om0, _NU, _T, 0.005)


def _vorticity_error(om0, ref, dt):
    p = mh.Params(nx=_N, ny=_N, lx=_L, ly=_L, rho=1.0, eta=_NU, dt=dt)
    st = mh.run(p, mh.initial_state(p, np.full((_N, _N), 0.3), om0), int(round(_T / dt)))
    return float(np.max(np.abs(st.omega - ref)) / np.max(np.abs(ref)))


def test_vorticity_advection_converges_to_continuum(vorticity_reference):
    """Uniform phi (K = 0), two vorticity modes of different |q| at nu = 0.05
    to t = 1: the oracle converges at order 1 in dt to the continuum solution
    (the O(delta^2) floor of the stencils at 128^2 is below 1e-3)."""
    om0, ref = vorticity_reference
    e = [_vorticity_error(om0, ref, dt) for dt in (0.04, 0.02, 0.01)]
    assert all(abs(o - 1.0) < 0.2 for o in _orders(e)), e
    assert e[-1] < 0.01, e


def test_vorticity_pin_catches_unadvected_crank_nicolson_start(monkeypatch, vorticity_reference):
    """Starting the Crank-Nicolson update from omega^n instead of the advected
    omega^{n+1/2} discards the advection: the error stays O(1) as dt -> 0."""
    om0, ref = vorticity_reference
    orig = mh.stage_advect

    def slip(p, st, s):
        ph, _, f = orig(p, st, s)
        return ph, st.omega, f

    monkeypatch.setattr(mh, "stage_advect", slip)
    assert _vorticity_error(om0, ref, 0.01) > 0.1


# ------------------------------------------- midpoint sawtooth (scheme switch)

def midpoint_kelvin_defect(frac):
    """Kelvin mode under the midpoint switch against the closed-form product of
    Crank-Nicolson factors with lambda at the lab wavevector of t_k + frac dt.

    omega0 = eps cos(q . x), phi = 0: psi is proportional to omega, so the
    advection and K vanish and each step multiplies the mode by
    (1 + dt nu lambda_k / 2) / (1 - dt nu lambda_k / 2),
    lambda_k = -(kx^2 + (ky - gdot (k + frac) dt kx)^2); one wrap is crossed.
    """
    p = mh.Params(nx=32, ny=32, lx=32.0, ly=32.0, gdot=0.2, dt=0.02, eta=1.5, rho=2.0,
                  midpoint_s=True)
    m, n = 1, 2
    kx, ky = 2 * math.pi * m / p.lx, 2 * math.pi * n / p.ly
    j, i = np.meshgrid(np.arange(p.ny), np.arange(p.nx), indexing="ij")
    eps = 1e-3
    w0 = eps * np.cos(kx * i * p.dx + ky * j * p.dy)
    st = mh.initial_state(p, np.zeros_like(w0), w0)
    nu = p.eta / p.rho
    amp = eps
    for k in range(200):
        X = p.gdot * ((k + frac) * p.dt)
        lam = -(kx ** 2 + (ky - X * kx) ** 2)
        amp *= (1 + 0.5 * p.dt * nu * lam) / (1 - 0.5 * p.dt * nu * lam)
        st = mh.step(p, st)
    assert st.wraps == 1
    W = mh.fft2(st.omega)
    got = 2 * abs(W[(n - st.wraps * m) % p.ny, m]) / (p.nx * p.ny)
    return abs(got - amp) / amp


def test_midpoint_sawtooth_kelvin_mode():
    assert midpoint_kelvin_defect(0.5) <= 1e-12
    # the closed form tells the midpoint from either end of the step
    assert midpoint_kelvin_defect(0.0) > 1e-5 and midpoint_kelvin_defect(1.0) > 1e-5


def test_midpoint_pin_catches_an_end_of_step_sawtooth(monkeypatch):
    monkeypatch.setattr(mh, "strain_offset_mid",
                        lambda p, n: p.gdot * ((float(n) + 1.0) * p.dt) - p.c * mh.wrap_count(p, n))
    assert midpoint_kelvin_defect(0.5) > 1e-5
