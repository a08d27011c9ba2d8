"""Pins of the oracle's turbulence diagnostics (Sec. 4.1: E(kappa), E_p(kappa), S and F of du/dx,
PDFs of eps / <eps> and Omega / <Omega>) against closed forms and identities (CPU only).

* shells: the integer rule against the correctly rounded sqrt (no integer lies on a tie);
* single Fourier modes of known |k| (including (1,1,1), where rounding and truncation of |k|
  differ) put exactly the closed-form energy in exactly one shell;
* Parseval on a seeded random field: the shells add up to <u.u>/2 and <p^2>, E_p(0) = <p>^2, with
  the velocity and pressure formed in the test from the conservative field;
* S and F of u = sin x + c sin 2x + d sin y against the closed forms of the moments of
  a cos x + b cos 2x, with a, b the modified wavenumbers of the 4th- and 6th-order central stencils
  (the d sin y term catches a gradient taken along the wrong axis);
* the dissipation and enstrophy of u = sin y, v = sin x (eps = mu (cos x + cos y)^2 k'^2,
  Omega = (cos x - cos y)^2 k'^2) and of u = sin x (eps = 4/3 mu k'^2 cos^2 x, the dilatational
  term), and their PDF counts against the closed forms binned in the test.
"""
import math

import numpy as np
import pytest

from oracle import OracleConfig
from oracle.diagnostics import diagnostics, shell_index, shell_of_k2, wavenumbers
from paper_2003_10561_amd import workload as W
from tests import fields as F

GAMMA, R = 1.4, 1.0


def kprime(m, h, order):
    """Modified wavenumber of the central first-derivative stencil: D sin(m x) = k' cos(m x)."""
    t = m * h
    if order == 4:  # (-1, 8, -8, 1) / 12h
        return (8.0 * math.sin(t) - math.sin(2 * t)) / (6.0 * h)
    return (45.0 * math.sin(t) - 9.0 * math.sin(2 * t) + math.sin(3 * t)) / (30.0 * h)  # (1,6) row, k = 0


def cfg_n(n, order=4, mu=0.01):
    return OracleConfig(n=(n,) * 3, p=(1, 1, 1), dt=1e-3, mu_ref=mu, max_delay=0, order=order,
                        gamma=GAMMA, gas_r=R, mu_exp=0.76)


def state(n, u, v, w, T, rho=None):
    X, _, _ = F.grid((n,) * 3)
    rho = np.ones_like(X) if rho is None else rho
    return F.conservative(rho, u, v, w, T, GAMMA, R)


def test_shell_rule_is_rounded_sqrt():
    k2 = np.arange(0, 1_000_001, dtype=np.int64)
    got = shell_of_k2(k2)
    ref = np.rint(np.sqrt(k2.astype(np.float64))).astype(np.int64)
    assert np.array_equal(got, ref)
    assert [int(shell_of_k2(np.array([v]))[0]) for v in (2, 3, 6, 7, 12, 13, 25)] == [1, 2, 2, 3, 3, 4, 5]
    assert list(wavenumbers(8)) == [0, 1, 2, 3, 4, -3, -2, -1]
    sh = shell_index((4, 8, 6))
    assert sh.shape == (4, 8, 6) and sh[0, 0, 0] == 0 and sh[2, 4, 3] == round(math.sqrt(4 + 16 + 9))


@pytest.mark.parametrize("order", [4, 6])
def test_single_modes_fill_their_shells(order):
    n = 16
    X, Y, Z = F.grid((n,) * 3)
    A, B, C, T0, a = 0.3, 0.2, 0.15, 1.1, 0.05
    u = A * np.cos(X + Y + Z)          # |k| = sqrt 3 -> shell 2 (truncation would give 1)
    v = B * np.sin(3 * X + 4 * Y)      # |k| = 5
    w = C * np.cos(X + Y)              # |k| = sqrt 2 -> shell 1
    T = T0 + a * np.cos(6 * X)         # p = R T: shells 0 and 6
    d = diagnostics(cfg_n(n, order), state(n, u, v, w, T), 16, 8, 4.0, 4.0)
    E, Ep = d["E"], d["Ep"]
    want_E = np.zeros(16)
    want_E[2], want_E[5], want_E[1] = A * A / 4, B * B / 4, C * C / 4
    want_Ep = np.zeros(16)
    want_Ep[0], want_Ep[6] = (R * T0) ** 2, R * R * a * a / 2
    assert np.allclose(E, want_E, rtol=0, atol=1e-15)
    assert np.allclose(Ep, want_Ep, rtol=0, atol=1e-14)
    assert d["p_mean"] == pytest.approx(R * T0, rel=1e-14)


def test_parseval_on_random_field():
    n = 32
    q = W.make_field(n, seed=7, mt=0.3)
    rho = q[0]
    u, v, w = q[1] / rho, q[2] / rho, q[3] / rho
    T = (q[4] / rho - 0.5 * (u * u + v * v + w * w)) / (R / (GAMMA - 1.0))
    p = rho * R * T
    nshell = int(math.isqrt(3 * (n // 2) ** 2)) + 2
    d = diagnostics(cfg_n(n), q, nshell, 16, 8.0, 16.0)
    assert d["E"].sum() == pytest.approx(0.5 * np.mean(u * u + v * v + w * w), rel=1e-13)
    assert d["Ep"].sum() == pytest.approx(np.mean(p * p), rel=1e-13)
    assert d["Ep"][0] == pytest.approx(np.mean(p) ** 2, rel=1e-13)
    assert d["E"][0] == pytest.approx(0.5 * (np.mean(u) ** 2 + np.mean(v) ** 2 + np.mean(w) ** 2),
                                      rel=1e-10, abs=1e-18)
    # truncating the shell list drops exactly the energy of the shells left out
    d8 = diagnostics(cfg_n(n), q, 8, 16, 8.0, 16.0)
    assert np.allclose(d8["E"], d["E"][:8], rtol=1e-14, atol=0)
    assert d["eps_pdf"].sum() == n ** 3 and d["ens_pdf"].sum() == n ** 3


@pytest.mark.parametrize("order", [4, 6])
def test_skewness_flatness_closed_form(order):
    n = 32
    h = 2 * math.pi / n
    X, Y, Z = F.grid((n,) * 3)
    c, dd = 0.4, 0.7
    u = np.sin(X) + c * np.sin(2 * X) + dd * np.sin(Y)
    zero = np.zeros_like(X)
    d = diagnostics(cfg_n(n, order), state(n, u, zero, zero, np.ones_like(X)), 4, 4, 4.0, 4.0)
    a, b = kprime(1, h, order), c * kprime(2, h, order)
    g2 = (a * a + b * b) / 2
    g3 = 3 * a * a * b / 4
    g4 = 3 * (a ** 4 + b ** 4) / 8 + 3 * a * a * b * b / 2
    assert d["g2"] == pytest.approx(g2, rel=1e-13)
    assert d["g3"] == pytest.approx(g3, rel=1e-12)
    assert d["g4"] == pytest.approx(g4, rel=1e-13)
    assert d["S"] == pytest.approx(g3 / g2 ** 1.5, rel=1e-12)
    assert d["F"] == pytest.approx(g4 / g2 ** 2, rel=1e-13)


def _binned(x, nbins, xmax):
    b = np.clip(np.floor(x * (nbins / xmax)), 0, nbins).astype(np.int64)
    return np.bincount(b.ravel(), minlength=nbins + 1)


@pytest.mark.parametrize("order", [4, 6])
def test_shear_dissipation_enstrophy_and_pdfs(order):
    n, mu = 32, 0.02
    h = 2 * math.pi / n
    X, Y, Z = F.grid((n,) * 3)
    zero = np.zeros_like(X)
    q = state(n, np.sin(Y), np.sin(X), zero, np.ones_like(X))
    kp = kprime(1, h, order)
    xe = (np.cos(X) + np.cos(Y)) ** 2          # eps / <eps>, <(cos x + cos y)^2> = 1
    xo = (np.cos(X) - np.cos(Y)) ** 2          # Omega / <Omega>
    for nbins, xmax in ((37, 4.1), (23, 2.05)):
        edges = np.arange(1, nbins + 1) * (xmax / nbins)
        for x in (xe, xo):  # no closed-form value within 1e-9 of an inner edge
            assert np.abs(x.ravel()[:, None] - edges[None, :]).min() > 1e-9
        d = diagnostics(cfg_n(n, order, mu), q, 4, nbins, xmax, xmax)
        assert d["eps_mean"] == pytest.approx(mu * kp * kp, rel=1e-13)
        assert d["ens_mean"] == pytest.approx(kp * kp, rel=1e-13)
        assert np.array_equal(d["eps_pdf"], _binned(xe, nbins, xmax))
        assert np.array_equal(d["ens_pdf"], _binned(xo, nbins, xmax))
        assert d["eps_pdf"].sum() == n ** 3
    assert d["ens_pdf"][-1] > 0  # the second case sends the values above 2.05 to the last bin


def test_dilatation():
    n, mu = 32, 0.02
    h = 2 * math.pi / n
    X, Y, Z = F.grid((n,) * 3)
    zero = np.zeros_like(X)
    d = diagnostics(cfg_n(n, 4, mu), state(n, np.sin(X), zero, zero, np.ones_like(X)), 4, 10, 3.0, 3.0)
    kp = kprime(1, h, 4)
    # sigma_xx = 2 mu G - 2/3 mu G: eps = 4/3 mu k'^2 cos^2 x, mean 2/3 mu k'^2
    assert d["eps_mean"] == pytest.approx(2.0 / 3.0 * mu * kp * kp, rel=1e-13)
    assert d["ens_mean"] < 1e-28  # no vorticity beyond the rounding of the stencil sums
    assert d["eps_pdf"].sum() == n ** 3


def test_fluid_at_rest_has_empty_pdfs():
    """No strain and no vorticity: <eps> = <Omega> = 0, both PDFs empty, E = 0, E_p only at 0."""
    n = 16
    X, Y, Z = F.grid((n,) * 3)
    zero = np.zeros_like(X)
    d = diagnostics(cfg_n(n), state(n, zero, zero, zero, np.full_like(X, 1.25)), 6, 10, 3.0, 3.0)
    assert d["eps_mean"] == 0.0 and d["ens_mean"] == 0.0
    assert d["eps_pdf"].sum() == 0 and d["ens_pdf"].sum() == 0
    assert not d["E"].any() and d["S"] == 0.0 and d["F"] == 0.0
    assert d["Ep"][0] == pytest.approx(1.25 ** 2, rel=1e-15) and not d["Ep"][1:].any()
