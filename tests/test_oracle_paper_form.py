"""Pins of the oracle's paper form (form 1: Sec. 2, Eqs. cont, mome, ie in the variables
(rho, rho u_i, rho e); (2,4) AT second derivatives, 3-step mixed derivatives, Sutherland's law)
against what the paper and the mathematics fix (CPU only).

* the (2,4) rows of Appendix B as printed (tests/golden/appb_at24.txt), evaluated line by line on
  arbitrary history levels with per-face delays, against the energy RHS of pure heat conduction
  (u = 0, constant mu: kappa d2T/dx2), and the printed (1,4) rows against the pressure gradient of
  the same data;
* the PE-local derivative of the mixed-derivative step: exact for polynomials up to degree 4 at
  every point of a PE, and not for degree 5 (a negative control);
* fourth-order convergence of the whole RHS, with delays, to the exact RHS of the internal-energy
  equations derived with sympy, for the power law and for Sutherland's law (this pins the
  expanded viscous and conduction terms, mu'(T), the mixed derivatives and every ghost);
* AT exactness: history levels quadratic in time make the delayed RHS equal the synchronous one;
* a uniform state at rest has a zero RHS under any schedule; the synchronous continuity RHS sums
  to zero (mass is conserved);
* Sutherland's law at T_ref and its derivative against a centred difference.
"""
import math
import os

import numpy as np
import pytest

from oracle import Oracle, OracleConfig
from oracle.oracle import EXPLICIT, SAA, SYNC
from tests import fields as F
from tests.test_oracle_pins import _appb_derivative_1d

GOLD = os.path.join(os.path.dirname(__file__), "golden")
GAMMA, R, PR = 1.4, 1.0, 0.7
CV = R / (GAMMA - 1.0)
CP = GAMMA * R / (GAMMA - 1.0)


def pcfg(n, p, dt=0.01, mu=0.05, L=3, visc=0, suth_s=0.0, mu_exp=0.76, **kw):
    return OracleConfig(n=tuple(n), p=tuple(p), dt=dt, mu_ref=mu, max_delay=L, form=1, visc=visc,
                        suth_s=suth_s, mu_exp=mu_exp, gamma=GAMMA, gas_r=R, prandtl=PR, **kw)


def paper_state(rho, u, v, w, T):
    return np.stack([rho, rho * u, rho * v, rho * w, rho * CV * T])


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_appb_24_rows_heat_conduction_and_pressure(axis):
    rng = np.random.default_rng(31 + axis)
    N, e = 20, 5
    n = [5, 5, 5]
    n[axis] = N
    p = [1, 1, 1]
    p[axis] = N // e
    nlev, cur = 6, 5
    mu = 0.2
    kap = mu * CP / PR
    h = 2 * math.pi / N
    shape = (n[2], n[1], n[0])
    lines = [1.0 + 0.1 * rng.standard_normal(N) for _ in range(nlev)]
    qs = []
    for m in range(nlev):
        ls = [1, 1, 1]
        ls[2 - axis] = N
        T = np.broadcast_to(lines[m].reshape(ls), shape).copy()
        z = np.zeros(shape)
        qs.append(paper_state(np.ones(shape), z, z, z, T))
    cfg = pcfg(n, p, mu=mu, mu_exp=0.0)
    nt = cfg.ntiles
    tab = np.zeros((nlev + 1, nt, 6), dtype=np.int8)
    # delays on the faces normal to the axis only: across the other faces T does not vary in space,
    # but its older levels differ, so their ghosts would add transverse terms
    tab[cur, :, 2 * axis:2 * axis + 2] = rng.integers(0, 4, size=(nt, 2))
    o = Oracle(cfg)
    o.init_field(np.ascontiguousarray(np.stack(qs)), nlev)
    o.set_schedule(EXPLICIT, table=tab)
    r = o.rhs()
    kl = [int(tab[cur, t, 2 * axis]) for t in range(nt)]
    kr = [int(tab[cur, t, 2 * axis + 1]) for t in range(nt)]
    assert any(k > 0 for k in kl + kr)
    rows24 = F.read_appb(os.path.join(GOLD, "appb_at24.txt"))
    rows14 = F.read_appb(os.path.join(GOLD, "appb_at14.txt"))
    want_e = kap * _appb_derivative_1d(lines, cur, e, kl, kr, h * h, rows24)
    want_m = -_appb_derivative_1d([R * l for l in lines], cur, e, kl, kr, h, rows14)
    got_e = np.moveaxis(r[4], 2 - axis, 0).reshape(N, -1)
    got_m = np.moveaxis(r[1 + axis], 2 - axis, 0).reshape(N, -1)
    for col in range(got_e.shape[1]):
        np.testing.assert_allclose(got_e[:, col], want_e, rtol=0, atol=1e-11 * np.abs(want_e).max())
        np.testing.assert_allclose(got_m[:, col], want_m, rtol=0, atol=1e-12 * np.abs(want_m).max())
    assert np.abs(r[0]).max() == 0.0
    for a in range(3):
        if a != axis:  # the central stencil of a uniform pressure: zero up to its rounding
            assert np.abs(r[1 + a]).max() < 1e-14 * np.abs(want_m).max()


def test_pe_derivative_exact_to_degree_four():
    h = 0.3
    for e in (5, 6, 9):
        x = np.arange(e) * h
        for deg in range(5):
            c = np.arange(1, deg + 2, dtype=float)
            g = sum(ci * x ** k for k, ci in enumerate(c))
            dg = sum(k * ci * x ** (k - 1) for k, ci in enumerate(c) if k > 0) if deg > 0 else np.zeros(e)
            np.testing.assert_allclose(Oracle.pe_derivative(g, h), dg, rtol=0, atol=1e-11)
        g5 = x ** 5
        err = np.abs(Oracle.pe_derivative(g5, h) - 5 * x ** 4)
        assert err[0] > 1e-6 and err[-1] > 1e-6  # the one-sided ends are fourth order, not fifth


@pytest.mark.slow
@pytest.mark.parametrize("law", ["power", "sutherland"])
def test_paper_form_converges_fourth_order_under_delays(law):
    errs = []
    visc, suth = (0, 0.0) if law == "power" else (1, 0.4)
    param = (19, 25) if law == "power" else (2, 5)
    for N in (16, 32, 64):
        h = 2 * math.pi / N
        dt = 0.5 * h * h
        nlev = 6
        cfg = pcfg((N, N, N), (2, 2, 2), dt=dt, mu=0.05, visc=visc, suth_s=suth, mu_exp=19 / 25)
        hist = np.ascontiguousarray(np.stack([F.analytic_paper((N, N, N), (m - (nlev - 1)) * dt, law, param)[0]
                                              for m in range(nlev)]))
        tab = np.zeros((nlev + 1, 8, 6), dtype=np.int8)
        tab[nlev - 1] = np.random.default_rng(N).integers(0, 4, size=(8, 6))
        o = Oracle(cfg)
        o.init_field(hist, nlev)
        o.set_schedule(EXPLICIT, table=tab)
        exact = F.analytic_paper((N, N, N), 0.0, law, param)[1]
        errs.append([float(np.abs(o.rhs()[c] - exact[c]).max()) for c in range(5)])
    errs = np.array(errs)
    orders = np.log2(errs[1] / errs[2])
    assert (orders >= 3.6).all(), (errs, orders)


def test_quadratic_time_levels_are_extrapolated_exactly():
    """rho = 1, u = 0, rho e quadratic in time: T and p (the only functions differentiated that vary)
    are quadratic in time, so every AT ghost equals the current value and the delayed RHS equals the
    synchronous RHS of the current level."""
    rng = np.random.default_rng(9)
    N, nlev = 10, 6
    a, b, c = (rng.standard_normal((N, N, N)) * s for s in (0.1, 0.03, 0.01))
    qs = []
    for m in range(nlev):
        z = np.zeros((N, N, N))
        qs.append(paper_state(np.ones_like(z), z, z, z, 1.0 + a + b * m + c * m * m))
    cfg = pcfg((N, N, N), (2, 2, 2), mu=0.05)
    tab = np.zeros((nlev + 1, 8, 6), dtype=np.int8)
    tab[nlev - 1] = rng.integers(1, 4, size=(8, 6))
    o = Oracle(cfg)
    o.init_field(np.ascontiguousarray(np.stack(qs)), nlev)
    o.set_schedule(EXPLICIT, table=tab)
    r = o.rhs()
    s = Oracle(cfg)
    s.init_field(qs[-1])
    s.set_schedule(SYNC, n_steps=1)
    ref = s.rhs()
    for comp in range(5):
        np.testing.assert_allclose(r[comp], ref[comp], rtol=0, atol=1e-10 * max(1.0, np.abs(ref[comp]).max()))


def test_uniform_state_and_mass_conservation():
    N = 10
    z = np.zeros((N, N, N))
    q = paper_state(np.full_like(z, 1.3), z + 0.2, z - 0.1, z + 0.05, np.full_like(z, 0.9))
    cfg = pcfg((N, N, N), (2, 2, 2), mu=0.05, visc=1, suth_s=0.4)
    o = Oracle(cfg)
    o.init_field(q)
    o.set_schedule(SAA, L=3, seed=5, n_steps=12)
    o.rk_step(8)
    o.set_schedule(SAA, L=3, seed=5, n_steps=12)
    assert np.abs(o.field() - q).max() < 1e-13
    qs, _ = F.analytic_paper((16, 16, 16), 0.0)
    s = Oracle(pcfg((16, 16, 16), (2, 2, 2), mu=0.05))
    s.init_field(qs)
    s.set_schedule(SYNC, n_steps=1)
    assert abs(s.rhs()[0].sum()) < 1e-12 * np.abs(s.rhs()[0]).sum()


def test_sutherland_law():
    cfg = pcfg((10, 10, 10), (2, 2, 2), mu=0.05, visc=1, suth_s=0.4, t_ref=1.0)
    mu, _ = Oracle.viscosity(cfg, 1.0)
    assert mu == pytest.approx(0.05, rel=1e-15)
    for T in (0.6, 1.0, 1.7):
        mu, dmu = Oracle.viscosity(cfg, T)
        eps = 1e-5
        fd = (Oracle.viscosity(cfg, T + eps)[0] - Oracle.viscosity(cfg, T - eps)[0]) / (2 * eps)
        assert dmu == pytest.approx(fd, rel=1e-8)
        # Sutherland's law grows like T^(1/2) at large T: mu(4T) / mu(T) -> 2 (T + S) / (4T + S) * 8
        mu4 = Oracle.viscosity(cfg, 4 * T)[0]
        assert mu4 / mu == pytest.approx(8 * (T + 0.4) / (4 * T + 0.4), rel=1e-14)


def test_mixed_derivative_is_the_average_of_two_pe_local_derivatives():
    """u = w = 0, v = sin x sin y, rho = 1, T and mu uniform: the x-momentum RHS is mu/3 times the
    mixed derivative d2 v / dx dy alone, which the paper forms at PE boundaries in three steps (AT
    first derivatives along y and along x, then a derivative of each along the other direction
    with the PE's own points, then the average).  With synchronous gradients (k' = modified
    wavenumber), that is 1/2 k' (cos y D_x^PE[sin x] + cos x D_y^PE[sin y]); PE edges 5 along x and
    10 along y make the two halves differ."""
    N, mu = 20, 0.3
    h = 2 * math.pi / N
    p = (4, 2, 1)
    X, Y, Z = F.grid((N, N, N))
    z = np.zeros_like(X)
    q = paper_state(np.ones_like(X), z, np.sin(X) * np.sin(Y), z, np.full_like(X, 1.2))
    o = Oracle(pcfg((N, N, N), p, mu=mu, mu_exp=0.0))
    o.init_field(q)
    o.set_schedule(SYNC, n_steps=1)
    r = o.rhs()
    kp = (8 * math.sin(h) - math.sin(2 * h)) / (6 * h)
    x = np.arange(N) * h
    dx_pe = np.concatenate([Oracle.pe_derivative(np.sin(x[t * 5:(t + 1) * 5]), h) for t in range(4)])
    dy_pe = np.concatenate([Oracle.pe_derivative(np.sin(x[t * 10:(t + 1) * 10]), h) for t in range(2)])
    want = mu / 3 * 0.5 * kp * (np.cos(Y) * dx_pe[None, None, :] + np.cos(X) * dy_pe[None, :, None])
    np.testing.assert_allclose(r[1], want, rtol=0, atol=1e-13)
    one_sided_only = mu / 3 * kp * np.cos(Y) * dx_pe[None, None, :]
    assert np.abs(r[1] - one_sided_only).max() > 1e-5  # not a single one of the two halves
