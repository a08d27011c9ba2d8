"""Seeded synthetic inputs shared by the HIP path, its tests, the bench and the CPU oracle.

This module produces *inputs* only: initial conservative fields, explicit delay tables,
stochastic forcing amplitudes and the two run parameters the paper fixes by rule
(time step and viscosity).  It holds none of the right-hand-side, stencil or time-stepping
arithmetic of the method, so neither the oracle nor the GPU library depends on the other
through it.

Paper context (Kumari & Donzis, "DNS of turbulent flows using high-order Asynchrony-Tolerant
schemes"):
  * the DNS fields of the paper are stationary states of earlier runs (Sec. 4, set-up) and are
    not available; a seeded solenoidal field with E(k) ~ k^4 exp(-2 (k/k0)^2) stands in;
  * resolution rule kappa_max * eta ~= 1.5 with kappa_max = sqrt(2) N / 3 (Sec. 4, set-up);
  * fixed time step giving an initial CFL of O(0.1) (Sec. 2.2 and Sec. 4, set-up);
  * turbulent Mach number M_t = <u_i u_i>^{1/2} / c (Sec. 4, set-up);
  * stochastic large-scale forcing of the Eswaran-Pope kind (Sec. 4.2, forced turbulence).
"""
from __future__ import annotations

import math
import os

import numpy as np
import scipy.fft as sfft

GAMMA = 1.4
GAS_R = 1.0

# Forcing wavevectors: all integer k with 0 < |k|^2 <= 6 (|k| <= 2.5), 80 vectors, kept as the
# 40 members of the half space (kz > 0) or (kz == 0 and ky > 0) or (kz == ky == 0 and kx > 0).
# Order: ascending kz, then ky, then kx, each scanned over -2..2.  The forcing field is
# f(x) = sum_k 2 Re(fhat_k exp(i k.x)) over these 40 vectors.
FORCE_KMAX2 = 6


def forcing_wavevectors() -> np.ndarray:
    ks = []
    for kz in range(-2, 3):
        for ky in range(-2, 3):
            for kx in range(-2, 3):
                k2 = kx * kx + ky * ky + kz * kz
                if k2 == 0 or k2 > FORCE_KMAX2:
                    continue
                half = kz > 0 or (kz == 0 and ky > 0) or (kz == 0 and ky == 0 and kx > 0)
                if half:
                    ks.append((kx, ky, kz))
    return np.array(ks, dtype=np.int64)


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def make_velocity(n: int, seed: int, urms2: float, k0: float = 4.0, log=None) -> np.ndarray:
    """Seeded solenoidal velocity [3][n][n][n] (index order [comp][z][y][x]) on [0, 2pi)^3.

    Half-spectrum modes (kx >= 0) with 0 < |k| < n/2 get complex Gaussian amplitudes and are
    projected onto the plane normal to k; the inverse real FFT gives a real field (Hermitian
    symmetry is implied).  Its true spectrum is then scaled per integer shell round(|k|) to the
    shell energy E(k) ~ k^4 exp(-2 (k/k0)^2), and the field is rescaled to <|u|^2> = urms2.
    """
    rng = np.random.default_rng(seed)
    kf = np.fft.fftfreq(n, d=1.0 / n)
    kr = np.arange(n // 2 + 1, dtype=np.float64)
    kz = kf[:, None, None]
    ky = kf[None, :, None]
    kx = kr[None, None, :]
    shp = (n, n, n // 2 + 1)
    k2 = np.empty(shp)
    np.add(kx * kx, ky * ky, out=k2)
    k2 += kz * kz
    kmag = np.sqrt(k2)
    active = (k2 > 0) & (kmag < n / 2)
    uh = np.empty((3,) + shp, dtype=np.complex128)
    for c in range(3):
        uh[c].real = rng.standard_normal(shp)
        uh[c].imag = rng.standard_normal(shp)
        uh[c] *= active
    # solenoidal projection (I - k k^T / |k|^2), in place
    k2[k2 == 0] = 1.0
    kd = np.empty(shp, dtype=np.complex128)
    tmp = np.empty(shp, dtype=np.complex128)
    np.multiply(uh[0], kx, out=kd)
    np.multiply(uh[1], ky, out=tmp)
    kd += tmp
    np.multiply(uh[2], kz, out=tmp)
    kd += tmp
    kd /= k2
    for c, kc in enumerate((kx, ky, kz)):
        np.multiply(kd, kc, out=tmp)
        uh[c] -= tmp
    del kd, tmp
    if log:
        log(f"field {n}^3: random projected modes ready")
    u = sfft.irfftn(uh, s=(n, n, n), axes=(1, 2, 3), workers=_workers())
    if log:
        log(f"field {n}^3: first inverse FFT done")
    # true (Hermitian) spectrum of the real field, then per-shell scaling
    uh = sfft.rfftn(u, axes=(1, 2, 3), workers=_workers())
    del u
    shell = np.rint(kmag).astype(np.int64)
    del kmag
    e_mode = np.zeros(shp)
    for c in range(3):
        e_mode += uh[c].real ** 2
        e_mode += uh[c].imag ** 2
    e_mode *= 0.5
    e_mode[..., 1:(n + 1) // 2] *= 2.0  # modes kx and -kx are both represented by kx > 0
    e_mode *= active
    nshell = int(shell.max()) + 1
    e_shell = np.bincount(shell.ravel(), weights=e_mode.ravel(), minlength=nshell)
    del e_mode
    ks = np.arange(nshell, dtype=np.float64)
    target = ks ** 4 * np.exp(-2.0 * (ks / k0) ** 2)
    fac = np.zeros(nshell)
    np.divide(target, e_shell, out=fac, where=e_shell > 0)
    fac = np.sqrt(fac)
    scale = fac[shell]
    scale *= active
    del shell
    for c in range(3):
        uh[c] *= scale
    del scale
    if log:
        log(f"field {n}^3: shells scaled")
    u = sfft.irfftn(uh, s=(n, n, n), axes=(1, 2, 3), workers=_workers())
    del uh
    u -= u.mean(axis=(1, 2, 3), keepdims=True)
    cur = float(np.einsum("cijk,cijk->", u, u)) / (n ** 3)
    u *= math.sqrt(urms2 / cur)
    return u


def sound_speed(t0: float = 1.0, gamma: float = GAMMA, gas_r: float = GAS_R) -> float:
    return math.sqrt(gamma * gas_r * t0)


def make_field(n: int, seed: int, mt: float = 0.3, k0: float = 4.0, rho0: float = 1.0,
               t0: float = 1.0, gamma: float = GAMMA, gas_r: float = GAS_R, log=None) -> np.ndarray:
    """Initial conservative state Q = (rho, rho u, rho v, rho w, E) as float64 [5][n][n][n].

    Uniform density and temperature, velocity from `make_velocity` with
    <|u|^2> = (mt * c0)^2, c0 = sqrt(gamma R T0); E = rho (c_v T + |u|^2 / 2) for an ideal gas
    with c_v = R / (gamma - 1).
    """
    c0 = sound_speed(t0, gamma, gas_r)
    u = make_velocity(n, seed, (mt * c0) ** 2, k0, log=log)
    cv = gas_r / (gamma - 1.0)
    q = np.empty((5, n, n, n), dtype=np.float64)
    q[0] = rho0
    np.multiply(u, rho0, out=q[1:4])
    e = q[4]
    np.multiply(u[0], u[0], out=e)
    for c in (1, 2):
        e += u[c] * u[c]
    e *= 0.5 * rho0
    e += rho0 * cv * t0
    return q


def default_dt(q: np.ndarray, cfl: float = 0.1, gamma: float = GAMMA, gas_r: float = GAS_R) -> float:
    """Fixed time step from an initial convective CFL: dt = cfl * h / (max_{x,d} |u_d| + max c)."""
    n = q.shape[-1]
    h = 2.0 * math.pi / n
    rho = q[0]
    u = q[1:4] / rho
    cv = gas_r / (gamma - 1.0)
    temp = (q[4] / rho - 0.5 * (u * u).sum(axis=0)) / cv
    c = np.sqrt(gamma * gas_r * temp)
    return cfl * h / (float(np.abs(u).max()) + float(c.max()))


def default_mu(n: int, mt: float = 0.3, k0: float = 4.0, rho0: float = 1.0, t0: float = 1.0,
               gamma: float = GAMMA, gas_r: float = GAS_R) -> float:
    """Viscosity from kappa_max * eta = 1.5, kappa_max = sqrt(2) n / 3, on the initial spectrum.

    For E(k) ~ k^4 exp(-2 (k/k0)^2) the dissipation is eps = 2 nu int k^2 E = (5/2) k0^2 nu K
    (= 40 nu K at k0 = 4), and eta^4 = nu^3 / eps gives nu = eta^2 sqrt((5/2) k0^2 K).
    """
    c0 = sound_speed(t0, gamma, gas_r)
    kin = 0.5 * (mt * c0) ** 2
    kmax = math.sqrt(2.0) * n / 3.0
    eta = 1.5 / kmax
    nu = eta * eta * math.sqrt(2.5 * k0 * k0 * kin)
    return nu * rho0


def random_schedule(seed: int, n_steps: int, ntiles: int, max_k: int, warmup: int) -> np.ndarray:
    """Explicit delay table int8 [n_steps][ntiles][6]: zeros for steps < warmup, then iid U{0..max_k}.

    Uses NumPy's PCG64 stream, so it is a different generator from the counter-based draws the
    library and the oracle make for the random (SAA) mode.
    """
    rng = np.random.default_rng(seed)
    tab = rng.integers(0, max_k + 1, size=(n_steps, ntiles, 6), dtype=np.int64)
    tab[:warmup] = 0
    return tab.astype(np.int8)


def make_forcing(seed: int, n_steps: int, dt: float, t_l: float = 1.0, sigma: float = 0.1) -> np.ndarray:
    """Forcing amplitudes fhat [n_steps][40][3][2] (re, im) from a seeded Ornstein-Uhlenbeck process.

    b^{n+1} = alpha b^n + sigma sqrt(1 - alpha^2) xi, alpha = exp(-dt / T_L), xi complex Gaussian
    with unit variance per real part, started from the stationary distribution; the amplitude is
    the solenoidal projection fhat_k = (I - k k^T / |k|^2) b_k, so the forcing is divergence free.
    """
    ks = forcing_wavevectors().astype(np.float64)
    nk = ks.shape[0]
    rng = np.random.default_rng(seed)
    alpha = math.exp(-dt / t_l)
    beta = sigma * math.sqrt(1.0 - alpha * alpha)

    def cgauss():
        return rng.standard_normal((nk, 3)) + 1j * rng.standard_normal((nk, 3))

    b = sigma * cgauss()
    proj = np.eye(3)[None] - ks[:, :, None] * ks[:, None, :] / (ks * ks).sum(axis=1)[:, None, None]
    out = np.empty((n_steps, nk, 3, 2), dtype=np.float64)
    for n in range(n_steps):
        fh = np.einsum("kij,kj->ki", proj, b)
        out[n, :, :, 0] = fh.real
        out[n, :, :, 1] = fh.imag
        b = alpha * b + beta * cgauss()
    return out


def urms_of(q: np.ndarray) -> float:
    """Per-component rms velocity ((1/3) <|u|^2>)^{1/2} of a conservative field."""
    u = q[1:4] / q[0]
    return math.sqrt(float((u * u).sum(axis=0).mean()) / 3.0)
