"""FP64 CPU oracle for the observables of section "Lengthscales and timescales".

TEST INFRASTRUCTURE ONLY (see the header of oracle.model_h).

* mean phi and <phi^2> in real space;
* the structure factor S(q) = |F[phi](q)|^2 / N (read of the "2D Fourier
  transform of phi");
* L_s of Eq. L_structure, with the lab-frame |q| = sqrt(-lambda) under shear;
* the tensor D_ab of Eq. L_matrix, with the lab-frame derivatives taken in
  Fourier space, and its reciprocal eigenvalues L_par (long axis), L_perp;
* the interfacial (Korteweg) excess shear stress sigma_xy = -kappa <d_x phi d_y phi>
  and the Reynolds part rho <...> of the velocity fluctuations (the paper
  names neither formula; the design notes give the reading);
* S(k) averaged over shells of width 2 pi / Ly.
"""
from __future__ import annotations

import math

import numpy as np

from .model_h import Params, State, fft2, strain_offset, wavenumbers


def lab_products(p: Params, s: float):
    """qx^2, qx q_lab_y and q_lab_y^2 on the full (ny, nx) mode grid.

    q_lab = (qx, qy - s qx); the odd product qx qy is zero on the Nyquist
    row and column, as in the step's Laplacian symbol.
    """
    qx, qy, nyq_x, nyq_y = wavenumbers(p)
    QX = np.broadcast_to(qx[None, :], (p.ny, p.nx))
    QY = np.broadcast_to(qy[:, None], (p.ny, p.nx))
    P = np.where(nyq_x[None, :] | nyq_y[:, None], 0.0, QX * QY)
    xx = QX * QX
    xy = P - s * xx
    yy = QY * QY - 2.0 * s * P + s * s * xx
    return xx, xy, yy


def observables(p: Params, st: State, nbins: int | None = None):
    """All observables of one state; returns a dict (and S(k) shell means)."""
    N = p.nx * p.ny
    s = strain_offset(p, st.step)
    phi = st.phi
    out = {
        "step": st.step,
        "wraps": st.wraps,
        "t": st.step * p.dt,
        "strain": p.gdot * (st.step * p.dt),
        "s": s,
        "mean_phi": float(np.sum(phi) / N),
        "phi2": float(np.sum(phi * phi) / N),
        "finite": int(np.all(np.isfinite(phi))),
    }
    Phi = fft2(phi)
    S = (Phi.real ** 2 + Phi.imag ** 2) / N
    xx, xy, yy = lab_products(p, s)
    q2 = xx + yy                       # |q_lab|^2 = -lambda
    qmod = np.sqrt(q2)
    nz = np.ones_like(S, dtype=bool)
    nz[0, 0] = False
    sum_S_nz = float(np.sum(S[nz]))
    sum_S_over_q = float(np.sum(S[nz] / qmod[nz]))
    out["Ls"] = sum_S_over_q / sum_S_nz if sum_S_nz > 0 else 0.0
    l_int = math.sqrt(p.kappa / p.A)
    sum_S = float(np.sum(S))
    Dxx = l_int * float(np.sum(xx * S)) / sum_S
    Dxy = l_int * float(np.sum(xy * S)) / sum_S
    Dyy = l_int * float(np.sum(yy * S)) / sum_S
    out.update(Dxx=Dxx, Dxy=Dxy, Dyy=Dyy)
    ev = np.linalg.eigvalsh(np.array([[Dxx, Dxy], [Dxy, Dyy]]))
    lo, hi = float(ev[0]), float(ev[1])
    out["L_perp"] = 1.0 / hi if hi > 0 else math.inf
    out["L_par"] = 1.0 / lo if lo > 0 else math.inf
    out["sigma_xy"] = -p.kappa * float(np.sum(xy * S)) / N
    if p.rho > 0.0:
        Psi = fft2(st.psi)
        P2 = Psi.real ** 2 + Psi.imag ** 2
        out["sigma_xy_re"] = p.rho * float(np.sum(xy * P2)) / (N * N)
    else:
        out["sigma_xy_re"] = 0.0
    # S(k) shells of width dk = 2 pi / Ly, bins 1 .. Ny/2.
    if nbins is None:
        nbins = p.ny // 2
    dk = 2.0 * math.pi / p.ly
    b = np.floor(qmod / dk + 0.5).astype(np.int64)
    sums = np.zeros(nbins + 1)
    counts = np.zeros(nbins + 1, dtype=np.int64)
    sel = (b >= 1) & (b <= nbins)
    np.add.at(sums, b[sel], S[sel])
    np.add.at(counts, b[sel], 1)
    Sk = np.where(counts[1:] > 0, sums[1:] / np.maximum(counts[1:], 1), 0.0)
    out["nbins"] = nbins
    out["dk"] = dk
    return out, Sk, counts[1:]
