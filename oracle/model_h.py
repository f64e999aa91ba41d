"""Plain FP64 CPU oracle for the sheared model-H time step.

TEST INFRASTRUCTURE ONLY.  This module is the independent reference that the
GPU library is checked against.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never does.
It shares no code, tables or helpers with the HIP implementation.

What it computes (Fielding, "The need for inertia in nonequilibrium steady
states of sheared binary fluids"):

* the 2D model-H equations posed in the cosheared frame (section "Numerical
  method", Eqs. equation1-equation4, with the sawtooth strain s(t) of Eq.
  coshearedNabluFinal);
* advanced by the three-stage split step of Appendix B: explicit-Euler
  advection with the shear-interpolated y stencil (Eqs. advective, p1y),
  the Cahn-Hilliard diffusive update in Fourier space with explicit Euler for
  the nabla^2 terms and Crank-Nicolson for nabla^4, mu and the vorticity
  source g by finite differences, Crank-Nicolson for omega, and the
  per-wavenumber solve for psi (or the biharmonic solve at rho = 0, Appendix B
  "Algorithm at zero Reynolds number").

Readings taken where the paper is silent (each is listed in the design notes):

* general free energy mu = B phi^3 - A phi - kappa nabla_c^2 phi and
  d_t phi = M nabla_c^2 mu (the paper's units are A = B = 1, kappa = M = l^2);
* the paper's per-mode 4x4 real blocks act on one complex Fourier coefficient
  per mode as the scalar lambda = D + Delta = -|q_lab|^2; the odd cross term
  q_x q_y is set to zero on the Nyquist row and column so every multiplier is
  Hermitian;
* every operator of step n uses s_n; f = (phi^n)^3; the omega Crank-Nicolson
  update starts from the advected omega^{n+1/2} (Params.f_half and
  Params.midpoint_s switch to the other readings of the first two: f of the
  advected phi, and s at the step's midpoint; Params.upwind3 takes the
  advected field's derivatives by the third-order upwind differences that
  Appendix B keeps as a commented-out alternative, sheared like Eq. p1y;
  Params.banded replaces the y part of the per-mode operators by the central
  differences of the stencils: Fourier in x only, a cyclic banded system in
  y per x wavenumber, solved here as such);
* the q = 0 mode: phi untouched, omega and psi set to zero;
* at a strain wrap s -> s - c (c = Lx/Ly) the fields are remapped row by row,
  new[j][i] = old[j][(i - r j) mod Nx] with r = Nx/Ny, so the lab-frame field
  is continuous;
* the sheared y stencil uses offsets +-r cells in x with weight |s|/c, which is
  the paper's "i -+ 2, weight s/2" at its own geometry (Lx = 2 Ly, Nx = 2 Ny).

Arrays are indexed a[j, i]: j along y (gradient direction), i along x (flow
direction), x fastest.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Params:
    """Problem statement of section "Choice of units" plus the grid.

    f(phi) = -A/2 phi^2 + B/4 phi^4 + kappa/2 |grad phi|^2; mobility M;
    viscosity eta; density rho (rho == 0 selects the Stokes branch); shear
    rate gdot; box lx x ly on an nx x ny grid; time step dt.
    """

    nx: int
    ny: int
    lx: float
    ly: float
    gdot: float = 0.0
    A: float = 1.0
    B: float = 1.0
    kappa: float = 1.0
    M: float = 1.0
    eta: float = 1.0
    rho: float = 1.0
    dt: float = 0.005
    # scheme variants either side of the default reading (all off: the scheme
    # as read): f from the advected phi; the sawtooth at the step's midpoint;
    # third-order upwinding of the advected field's derivatives
    f_half: bool = False
    midpoint_s: bool = False
    upwind3: bool = False
    # x spectral, y by finite differences in the per-mode operators: cyclic
    # banded (tri-/penta-diagonal) systems per x wavenumber
    banded: bool = False

    @property
    def dx(self) -> float:
        return self.lx / self.nx

    @property
    def dy(self) -> float:
        return self.ly / self.ny

    @property
    def c(self) -> float:
        """Box aspect ratio Lx/Ly: the height of the sawtooth's jumps."""
        return self.lx / self.ly

    @property
    def r(self) -> int:
        """Grid ratio Nx/Ny: the x offset (in cells) of the sheared stencil."""
        return self.nx // self.ny


@dataclasses.dataclass
class State:
    phi: np.ndarray
    omega: np.ndarray  # zeros (and unused) when rho == 0
    psi: np.ndarray
    step: int = 0
    wraps: int = 0


# ---------------------------------------------------------------------------
# Shear clock (section "Numerical method", sawtooth s(t))
# ---------------------------------------------------------------------------

def strain_total(p: Params, n: int) -> float:
    """Accumulated strain gdot * t at step n, formed as gdot * (n * dt)."""
    return p.gdot * (float(n) * p.dt)


def wrap_count(p: Params, n: int) -> int:
    """Number of jumps of height c taken by step n (s kept in [-c/2, c/2))."""
    X = strain_total(p, n)
    return int(math.floor((X + 0.5 * p.c) / p.c))


def strain_offset(p: Params, n: int) -> float:
    """The sawtooth s(t_n) of the cosheared gradient operator."""
    return strain_total(p, n) - p.c * wrap_count(p, n)


def strain_offset_mid(p: Params, n: int) -> float:
    """The sawtooth at t_n + dt/2, in the frame of step n (wrap count k_n)."""
    return p.gdot * ((float(n) + 0.5) * p.dt) - p.c * wrap_count(p, n)


def remap(p: Params, a: np.ndarray, dk: int) -> np.ndarray:
    """Re-express a cosheared-frame field after s -> s - dk*c.

    Keeps the lab-frame field unchanged: new[j, i] = old[j, (i - dk*r*j) mod Nx].
    """
    out = np.empty_like(a)
    for j in range(p.ny):
        shift = (dk * p.r * j) % p.nx
        out[j] = np.roll(a[j], shift)  # out[j, i] = a[j, i - shift]
    return out


# ---------------------------------------------------------------------------
# Finite-difference stencils (Appendix B, Eq. p1y and the mu stencils)
# ---------------------------------------------------------------------------

def at(a: np.ndarray, dj: int, di: int) -> np.ndarray:
    """Periodic neighbour: at(a, dj, di)[j, i] = a[j + dj, i + di]."""
    return np.roll(a, (-dj, -di), axis=(0, 1))


def d_x(p: Params, a: np.ndarray) -> np.ndarray:
    """Central first difference in x."""
    return (at(a, 0, 1) - at(a, 0, -1)) / (2.0 * p.dx)


def d_y_sheared(p: Params, a: np.ndarray, s: float) -> np.ndarray:
    """Shear-interpolated central y difference of Eq. p1y.

    Blends the plain central difference with one taken along the grid
    diagonal (j+1, i - sign(s) r) / (j-1, i + sign(s) r), weight |s|/c.
    It approximates the lab-frame derivative d_y - s d_x to second order.
    """
    w = abs(s) / p.c
    sg = 1 if s >= 0 else -1
    plain = at(a, 1, 0) - at(a, -1, 0)
    diag = at(a, 1, -sg * p.r) - at(a, -1, sg * p.r)
    return ((1.0 - w) * plain + w * diag) / (2.0 * p.dy)


def d_xx(p: Params, a: np.ndarray) -> np.ndarray:
    return (at(a, 0, 1) - 2.0 * a + at(a, 0, -1)) / (p.dx * p.dx)


def d_yy(p: Params, a: np.ndarray) -> np.ndarray:
    return (at(a, 1, 0) - 2.0 * a + at(a, -1, 0)) / (p.dy * p.dy)


def d_xy(p: Params, a: np.ndarray) -> np.ndarray:
    """Four-point mixed derivative."""
    return (at(a, 1, 1) - at(a, -1, 1) - at(a, 1, -1) + at(a, -1, -1)) / (
        4.0 * p.dx * p.dy)


def advection(p: Params, psi: np.ndarray, a: np.ndarray, s: float) -> np.ndarray:
    """The bracket d_y psi d_x a - d_x psi d_y a of Eq. advective.

    With p.upwind3 the derivatives of the advected field a are the
    third-order upwind ones (the alternative Appendix B keeps in a comment),
    upwind with respect to the velocity v = (d_y psi, -d_x psi) at each point;
    the derivatives of psi stay central.
    """
    if p.upwind3:
        vx = d_y_sheared(p, psi, s)
        vy = -d_x(p, psi)
        return vx * d_x_upwind(p, a, vx) + vy * d_y_sheared_upwind(p, a, vy, s)
    return d_y_sheared(p, psi, s) * d_x(p, a) - d_x(p, psi) * d_y_sheared(p, a, s)


# Third-order upwind first difference: offsets -2 .. 1 with weights
# (1, -6, 3, 2)/6 where the velocity is positive, the mirror image
# (offsets 2 .. -1, weights (-1, 6, -3, -2)/6) where it is not.
_UPWIND_POS = ((-2, 1.0), (-1, -6.0), (0, 3.0), (1, 2.0))
_UPWIND_NEG = ((2, -1.0), (1, 6.0), (0, -3.0), (-1, -2.0))


def d_x_upwind(p: Params, a: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Third-order upwind x difference, upwind for the velocity field v."""
    pos = sum(c * at(a, 0, k) for k, c in _UPWIND_POS) / (6.0 * p.dx)
    neg = sum(c * at(a, 0, k) for k, c in _UPWIND_NEG) / (6.0 * p.dx)
    return np.where(v > 0.0, pos, neg)


def d_y_sheared_upwind(p: Params, a: np.ndarray, v: np.ndarray, s: float) -> np.ndarray:
    """Third-order upwind y difference in the sheared frame.

    The sample of row j + k is taken, as in Eq. p1y, between the column
    straight above (weight 1 - |s|/c) and the column k r cells along the
    grid diagonal (weight |s|/c, offset -sign(s) r k), i.e. on the line of
    constant lab x; the upwind weights then act on these samples.  It
    approximates the lab derivative d_y - s d_x to third order.
    """
    w = abs(s) / p.c
    sg = 1 if s >= 0 else -1

    def sample(k):
        return (1.0 - w) * at(a, k, 0) + w * at(a, k, -sg * p.r * k)

    pos = sum(c * sample(k) for k, c in _UPWIND_POS) / (6.0 * p.dy)
    neg = sum(c * sample(k) for k, c in _UPWIND_NEG) / (6.0 * p.dy)
    return np.where(v > 0.0, pos, neg)


def chemical_potential(p: Params, phi: np.ndarray, s: float) -> np.ndarray:
    """mu = B phi^3 - A phi - kappa[(1+s^2) d_xx + d_yy - 2 s d_xy] phi."""
    lap_c = (1.0 + s * s) * d_xx(p, phi) + d_yy(p, phi) - 2.0 * s * d_xy(p, phi)
    return p.B * phi ** 3 - p.A * phi - p.kappa * lap_c


def korteweg_bracket(p: Params, phi: np.ndarray, mu: np.ndarray, s: float) -> np.ndarray:
    """K = d_x phi d_y mu - d_y phi d_x mu (Eq. G without the -1/rho)."""
    return d_x(p, phi) * d_y_sheared(p, mu, s) - d_y_sheared(p, phi, s) * d_x(p, mu)


# ---------------------------------------------------------------------------
# Fourier space (Appendix B: D, Delta, a = 1 + s^2, b = 2s)
# ---------------------------------------------------------------------------

def wavenumbers(p: Params):
    """Signed wavenumbers qx[m], qy[n] and the Nyquist masks."""
    m = np.arange(p.nx)
    n = np.arange(p.ny)
    ms = np.where(m >= p.nx // 2, m - p.nx, m)
    ns = np.where(n >= p.ny // 2, n - p.ny, n)
    qx = 2.0 * math.pi * ms / p.lx
    qy = 2.0 * math.pi * ns / p.ly
    return qx, qy, (m == p.nx // 2), (n == p.ny // 2)


def symbol_laplacian(p: Params, s: float) -> np.ndarray:
    """lambda(q; s), the eigenvalue D + Delta of the cosheared Laplacian block.

    D = -(a qx^2 + qy^2), Delta = b qx qy with a = 1 + s^2, b = 2s; the cross
    term is dropped on the Nyquist row/column.  Shape (ny, nx).
    """
    qx, qy, nyq_x, nyq_y = wavenumbers(p)
    QX = qx[None, :]
    QY = qy[:, None]
    P = QX * QY
    P = np.where(nyq_x[None, :] | nyq_y[:, None], 0.0, P)
    D = -((1.0 + s * s) * QX * QX + QY * QY)
    Delta = 2.0 * s * P
    return D + Delta


def fft2(a: np.ndarray) -> np.ndarray:
    """Unnormalised forward DFT F[a](m, n) = sum a_ij exp(-2 pi i (mi/Nx + nj/Ny))."""
    return np.fft.fft2(a)


def ifft2_real(A: np.ndarray) -> np.ndarray:
    """Inverse DFT with 1/N, real part (the imaginary part is rounding only)."""
    return np.real(np.fft.ifft2(A))


# ---------------------------------------------------------------------------
# The split step (Appendix B, stages 1-3, and the zero-Reynolds variant)
# ---------------------------------------------------------------------------

def stage_advect(p: Params, st: State, s: float):
    """Stage 1a: explicit-Euler advection of phi (and omega when rho > 0), and f."""
    phi_h = st.phi - p.dt * advection(p, st.psi, st.phi, s)
    if p.rho > 0.0:
        omega_h = st.omega - p.dt * advection(p, st.psi, st.omega, s)
    else:
        omega_h = st.omega
    f = (phi_h if p.f_half else st.phi) ** 3
    return phi_h, omega_h, f


# ---------------------------------------------------------------------------
# The banded variant: Fourier in x only, y derivatives of the per-mode
# operators by the central differences of the stencils (periodic), so each x
# wavenumber carries a cyclic banded system in y
# ---------------------------------------------------------------------------

def banded_laplacian(p: Params, m: int, s: float) -> np.ndarray:
    """The cosheared Laplacian on column m of the x transform, (ny, ny) complex:

        L = -(1 + s^2) qx^2 I + D2 - 2 s (i qx) D1,

    D2 = [1, -2, 1] / dy^2 and D1 = [-1, 0, 1] / (2 dy), cyclic in y (a cyclic
    tridiagonal matrix); the cross term is dropped on the x Nyquist column, as
    in the spectral symbol.
    """
    qx_all, _, nyq_x, _ = wavenumbers(p)
    qx = qx_all[m]
    n = p.ny
    I = np.eye(n)
    up = np.roll(I, 1, axis=1)     # (up a)[j] = a[j + 1]
    dn = np.roll(I, -1, axis=1)    # (dn a)[j] = a[j - 1]
    D2 = (up - 2.0 * I + dn) / (p.dy * p.dy)
    D1 = (up - dn) / (2.0 * p.dy)
    cross = 0.0 if nyq_x[m] else 1.0
    return -(1.0 + s * s) * qx * qx * I + D2 - cross * 2.0 * s * 1j * qx * D1


def _gauged_solve(Lop: np.ndarray, rhs: np.ndarray, m: int) -> np.ndarray:
    """Solve Lop x = rhs; on column 0 (Lop singular on the constants) the
    constant part of rhs is dropped and the solution taken with zero mean."""
    if m != 0:
        return np.linalg.solve(Lop, rhs)
    n = len(rhs)
    J = np.ones((n, n)) / n
    r = rhs - rhs.mean()
    return np.linalg.solve(Lop + J, r)


def stage_cahn_hilliard_banded(p, phi_h, f, s):
    """Stage 1b with the banded operators: per column m,
    (I + dt kM L^2/2) Phi' = (I - dt A M L - dt kM L^2/2) Phi_h + dt B M L F."""
    Ph = np.fft.fft(phi_h, axis=1)
    F = np.fft.fft(f, axis=1)
    out = np.empty_like(Ph)
    I = np.eye(p.ny)
    for m in range(p.nx):
        L = banded_laplacian(p, m, s)
        L2 = L @ L
        lhs = I + 0.5 * p.dt * p.kappa * p.M * L2
        rhs = (I - p.dt * p.A * p.M * L - 0.5 * p.dt * p.kappa * p.M * L2) @ Ph[:, m] \
            + p.dt * p.B * p.M * (L @ F[:, m])
        out[:, m] = np.linalg.solve(lhs, rhs)
    return np.real(np.fft.ifft(out, axis=1))


def stage_flow_banded(p, omega_h, g, s):
    """Stages 2b and 3 with the banded operators: per column m,
    (I - dt nu L/2) Om' = (I + dt nu L/2) Om_h + dt G,  -L Psi' = Om';
    rho == 0: L^2 Psi' = G.  The q = 0 mode (column 0's mean) of Om' and Psi'
    is zero."""
    G = np.fft.fft(g, axis=1)
    I = np.eye(p.ny)
    Psi = np.empty_like(G)
    if p.rho > 0.0:
        nu = p.eta / p.rho
        Om = np.fft.fft(omega_h, axis=1)
        Om_new = np.empty_like(Om)
        for m in range(p.nx):
            L = banded_laplacian(p, m, s)
            rhs = (I + 0.5 * p.dt * nu * L) @ Om[:, m] + p.dt * G[:, m]
            o = np.linalg.solve(I - 0.5 * p.dt * nu * L, rhs)
            if m == 0:
                o = o - o.mean()
            Om_new[:, m] = o
            Psi[:, m] = _gauged_solve(-L, o, m)
        return np.real(np.fft.ifft(Om_new, axis=1)), np.real(np.fft.ifft(Psi, axis=1))
    for m in range(p.nx):
        L = banded_laplacian(p, m, s)
        Psi[:, m] = _gauged_solve(L @ L, G[:, m], m)
    return np.zeros_like(omega_h), np.real(np.fft.ifft(Psi, axis=1))


def stage_cahn_hilliard(p: Params, phi_h: np.ndarray, f: np.ndarray, s: float) -> np.ndarray:
    """Stage 1b: per-mode update, explicit in nabla^2 and f, Crank-Nicolson in nabla^4.

    phi' = phi_h + (1 + dt kM lam^2/2)^-1 (-dt A M lam phi_h - dt kM lam^2 phi_h
                                           + dt B M lam F)
    """
    if p.banded:
        return stage_cahn_hilliard_banded(p, phi_h, f, s)
    lam = symbol_laplacian(p, s)
    Ph = fft2(phi_h)
    F = fft2(f)
    d2 = p.dt * p.M * lam          # tilde D_2 acting on phi (times A) and f (times B)
    d4 = p.dt * p.kappa * p.M * lam * lam   # tilde D_4
    incr = (-p.A * d2 * Ph - d4 * Ph + p.B * d2 * F) / (1.0 + 0.5 * d4)
    return ifft2_real(Ph + incr)


def vorticity_source(p: Params, phi_new: np.ndarray, s: float) -> np.ndarray:
    """Stage 2a: the bracket K at phi^{n+1}; g = -K/rho, or -K/eta when rho == 0."""
    mu = chemical_potential(p, phi_new, s)
    K = korteweg_bracket(p, phi_new, mu, s)
    return -K / (p.rho if p.rho > 0.0 else p.eta)


def stage_flow(p: Params, omega_h: np.ndarray, g: np.ndarray, s: float):
    """Stages 2b and 3: Crank-Nicolson for omega, then psi per wavenumber.

    rho > 0:  Om' = Om_h + (1 - dt nu lam/2)^-1 (dt nu lam Om_h + dt G),
              Psi' = -Om' / lam.
    rho == 0: Psi' = G / lam^2 (biharmonic solve).  q = 0: Om' = Psi' = 0.
    """
    if p.banded:
        return stage_flow_banded(p, omega_h, g, s)
    lam = symbol_laplacian(p, s)
    G = fft2(g)
    zero = np.zeros_like(lam, dtype=bool)
    zero[0, 0] = True
    safe = np.where(zero, 1.0, lam)
    if p.rho > 0.0:
        nu = p.eta / p.rho
        Om = fft2(omega_h)
        c_t = p.dt * nu * lam      # tilde C = dt nu lambda
        Om_new = Om + (c_t * Om + p.dt * G) / (1.0 - 0.5 * c_t)
        Om_new[0, 0] = 0.0
        Psi = -Om_new / safe
        Psi[0, 0] = 0.0
        return ifft2_real(Om_new), ifft2_real(Psi)
    Psi = G / (safe * safe)
    Psi[0, 0] = 0.0
    return np.zeros_like(omega_h), ifft2_real(Psi)


def initial_state(p: Params, phi0: np.ndarray, omega0: np.ndarray | None = None) -> State:
    """State at n = 0 (s = 0) with psi consistent with the flow constraint.

    rho > 0: Poisson solve from omega0; rho == 0: Stokes solve from phi0.
    """
    phi = np.array(phi0, dtype=np.float64, copy=True)
    if omega0 is None or p.rho == 0.0:
        omega = np.zeros_like(phi)
    else:
        omega = np.array(omega0, dtype=np.float64, copy=True)
    s0 = strain_offset(p, 0)
    lam = symbol_laplacian(p, s0)
    safe = lam.copy()
    safe[0, 0] = 1.0
    if p.rho > 0.0:
        Psi = -fft2(omega) / safe
    else:
        Psi = fft2(vorticity_source(p, phi, s0)) / (safe * safe)
    Psi[0, 0] = 0.0
    return State(phi=phi, omega=omega, psi=ifft2_real(Psi), step=0,
                 wraps=wrap_count(p, 0))


def step(p: Params, st: State) -> State:
    """One full time step n -> n+1, then the sawtooth shift and remap if due."""
    n = st.step
    s = strain_offset_mid(p, n) if p.midpoint_s else strain_offset(p, n)
    phi_h, omega_h, f = stage_advect(p, st, s)
    phi_new = stage_cahn_hilliard(p, phi_h, f, s)
    g = vorticity_source(p, phi_new, s)
    omega_new, psi_new = stage_flow(p, omega_h, g, s)
    k_old = wrap_count(p, n)
    k_new = wrap_count(p, n + 1)
    if k_new != k_old:
        dk = k_new - k_old
        phi_new = remap(p, phi_new, dk)
        omega_new = remap(p, omega_new, dk)
        psi_new = remap(p, psi_new, dk)
    return State(phi=phi_new, omega=omega_new, psi=psi_new, step=n + 1, wraps=k_new)


def run(p: Params, st: State, nsteps: int) -> State:
    for _ in range(nsteps):
        st = step(p, st)
    return st
