"""Turbulence diagnostics of Sec. 4.1 for one conservative field (test infrastructure only: the
oracle of the library's at_field_diagnostics; the product path never imports it).

The per-point fields come from the C oracle (ora_diag_fields): u, v, w, p = rho R T, the
longitudinal gradient du/dx, the dissipation sigma_ij du_i/dx_j and the enstrophy density
|curl u|^2, all with the synchronous central derivatives of the run's order on the periodic grid
(the derivatives of the oracle's statistics).  From them, in the plainest form:

* energy spectrum (Sec. 4.1.2, Eq. ener): E(kappa) = sum over the integer wavevectors k whose shell
  round(|k|) is kappa of (|u_k|^2 + |v_k|^2 + |w_k|^2) / 2, with u_k the discrete Fourier
  coefficient (numpy's forward FFT divided by the number of points), so that the shells add up to
  <u.u> / 2 (Parseval);
* pressure spectrum (Eq. pres): E_p(kappa) = the same shell sum of |p_k|^2 (E_p(0) = <p>^2);
* skewness S = <g^3> / <g^2>^(3/2) and flatness F = <g^4> / <g^2>^2 of g = du/dx (Sec. 4.1.3),
  both 0 when <g^2> = 0;
* the PDFs of eps / <eps> and Omega / <Omega> (Sec. 4.1.3, Fig. enst_pdf) as counts in nbins equal
  bins of [0, x_max) plus one last bin for x >= x_max: bin = floor(x * (nbins / x_max)), taken in
  FP64, clamped to 0 below (rounding can make eps slightly negative) and to nbins above; a PDF
  whose mean is not positive (a field without strain or without vorticity) has all counts 0.

Shells: round(|k|) for an integer |k|^2 = k2 is s = floor(sqrt(k2)) plus one when k2 > s^2 + s
(no integer k2 lies on a tie, (s + 1/2)^2 = s^2 + s + 1/4).  Wavenumbers follow the FFT index
convention: index j of an axis of n points is wavenumber j for j <= n/2 and j - n above.
"""
from __future__ import annotations

import math

import numpy as np

from .oracle import Oracle, OracleConfig

N_SCALARS = 8  # S, F, <g^2>, <g^3>, <g^4>, <eps>, <Omega>, <p>


def wavenumbers(n: int) -> np.ndarray:
    """Integer wavenumber of each FFT index of an axis of n points (n/2 counts as +n/2)."""
    j = np.arange(n, dtype=np.int64)
    return np.where(j <= n // 2, j, j - n)


def shell_of_k2(k2: np.ndarray) -> np.ndarray:
    """round(sqrt(k2)) for non-negative integers k2, in integer arithmetic."""
    k2 = np.asarray(k2, dtype=np.int64)
    s = np.array([math.isqrt(int(v)) for v in k2.ravel()], dtype=np.int64).reshape(k2.shape)
    return s + (k2 > s * s + s)


def shell_index(shape_zyx) -> np.ndarray:
    """Shell of every wavevector of a grid of shape (nz, ny, nx)."""
    nz, ny, nx = shape_zyx
    kz, ky, kx = wavenumbers(nz), wavenumbers(ny), wavenumbers(nx)
    k2 = kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2
    lut = shell_of_k2(np.arange(int(k2.max()) + 1))
    return lut[k2]


def pdf_counts(x: np.ndarray, nbins: int, x_max: float) -> np.ndarray:
    if not np.all(np.isfinite(x)):
        return np.zeros(nbins + 1, dtype=np.int64)
    b = np.floor(x * (nbins / x_max))
    b = np.clip(b, 0, nbins).astype(np.int64)
    return np.bincount(b.ravel(), minlength=nbins + 1)


def diagnostics(cfg: OracleConfig, q: np.ndarray, nshell: int, nbins: int, eps_max: float, ens_max: float):
    """Diagnostics of the conservative field q [5][nz][ny][nx] (see the module text)."""
    u, v, w, p, g, eps, om = Oracle.diag_fields(cfg, q)
    npts = float(u.size)
    shell = shell_index(u.shape).ravel()

    def shells(weights):
        full = np.bincount(shell, weights=weights, minlength=nshell)
        return full[:nshell]

    E = np.zeros(nshell)
    for c in (u, v, w):
        ck = np.fft.fftn(c) / npts
        E += shells(0.5 * np.abs(ck.ravel()) ** 2)
    pk = np.fft.fftn(p) / npts
    Ep = shells(np.abs(pk.ravel()) ** 2)
    m2, m3, m4 = (float(np.mean(g ** k)) for k in (2, 3, 4))
    eps_mean, om_mean = float(eps.mean()), float(om.mean())
    with np.errstate(divide="ignore", invalid="ignore"):
        eps_x = eps / eps_mean if eps_mean > 0 else np.full_like(eps, np.nan)
        ens_x = om / om_mean if om_mean > 0 else np.full_like(om, np.nan)
    return {
        "E": E, "Ep": Ep,
        "S": m3 / m2 ** 1.5 if m2 > 0 else 0.0, "F": m4 / m2 ** 2 if m2 > 0 else 0.0, "g2": m2, "g3": m3, "g4": m4,
        "eps_mean": eps_mean, "ens_mean": om_mean, "p_mean": float(p.mean()),
        "eps_pdf": pdf_counts(eps_x, nbins, eps_max),
        "ens_pdf": pdf_counts(ens_x, nbins, ens_max),
        # the normalised point values, for tests that need to know which points lie near a bin edge
        "eps_x": eps_x, "ens_x": ens_x,
    }
