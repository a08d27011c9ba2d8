"""Pins of the CPU oracle against what the paper and the mathematics fix (CPU only).

Each test names the passage or the closed form it checks.  None of them re-types the oracle's own
formulas as the only check: they compare against printed tables (tests/golden), closed forms,
library routines (FFT), or properties a mistake would break.
"""
import math
import os

import numpy as np
import pytest

from oracle import Oracle, OracleConfig
from oracle.oracle import CAA, EXPLICIT, SAA, SYNC, OracleError
from paper_2003_10561_amd import workload as W
from tests import fields as F

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def cfg_for(n, p, dt=0.01, mu=0.0, L=3, **kw):
    return OracleConfig(n=tuple(n), p=tuple(p), dt=dt, mu_ref=mu, max_delay=L, **kw)


# ------------------------------------------------------------------ Appendix B weights
def test_appb_weights_at_integer_delay():
    """w_l(k) of the oracle equal the Appendix B polynomials at integer k and sum to one."""
    rows = F.read_appb(os.path.join(GOLD, "appb_at14.txt"))
    for k in range(0, 6):
        for r in rows:
            w2, w1, w0 = r["w"]
            assert Oracle.at_weight(r["l"], float(k)) == w2 * k * k + w1 * k + w0
        assert sum(Oracle.at_weight(l, float(k)) for l in range(3)) == 1.0
    # reduces to the standard scheme without delay (Sec. 2.1)
    assert [Oracle.at_weight(l, 0.0) for l in range(3)] == [1.0, 0.0, 0.0]
    assert [Oracle.at_weight(l, 3.0) for l in range(3)] == [10.0, -15.0, 6.0]


def _appb_derivative_1d(levels, n, e, kl, kr, h, rows, current_override=None):
    """Evaluate the printed (1,4) AT rows along one periodic line.

    levels[m] is the line at level m (n = current).  kl[t], kr[t] are the delays on the left and
    right faces of PE t.  Points outside the PE take level n-k-l in row l, with k the delay of
    that face; the row weights are w_l(k).  At the first boundary point (both buffer points
    outside) this is the printed table; deeper points have fewer buffer points.
    """
    N = levels[n].shape[0]
    cur = levels[n] if current_override is None else current_override
    rows = [r for r in rows if r["side"] == "left"]  # identical weights and stencil on both sides
    offs = [-2, -1, 0, 1, 2]
    out = np.zeros(N)
    for i in range(N):
        t, loc = divmod(i, e)
        k = 0
        if loc < 2:
            k = kl[t]
        elif loc >= e - 2:
            k = kr[t]
        acc = 0.0
        for r in rows:
            w2, w1, w0 = r["w"]
            s = 0.0
            for a, m in zip(r["a"], offs):
                outside = not (0 <= loc + m < e)
                j = (i + m) % N
                s += a * (levels[n - k - r["l"]][j] if (outside and k > 0) else cur[j])
            acc += (w2 * k * k + w1 * k + w0) * s
        out[i] = acc / (rows[0]["div"] * h)
    return out


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_appb_stencil_mass_flux(axis):
    """Continuity RHS at every point equals -(1,4) AT derivative of the mass flux as printed in
    Appendix B, with per-face delays, for data that vary only along one axis (mu = 0, u = U e_axis,
    p uniform).  History levels are arbitrary, so the check covers each weight and level index."""
    rng = np.random.default_rng(7 + axis)
    N, e = 16, 4
    n = [4, 4, 4]
    n[axis] = N
    p = [1, 1, 1]
    p[axis] = N // e
    nlev = 6
    cur = nlev - 1
    U = 0.7
    lines = [1.0 + 0.2 * rng.standard_normal(N) for _ in range(nlev)]
    qs = []
    shape = (n[2], n[1], n[0])
    for m in range(nlev):
        line_shape = [1, 1, 1]
        line_shape[2 - axis] = N
        rho = np.broadcast_to(lines[m].reshape(line_shape), shape).copy()
        vel = [np.zeros(shape) for _ in range(3)]
        vel[axis][:] = U
        T = 1.0 / rho  # p = rho R T = 1
        qs.append(F.conservative(rho, vel[0], vel[1], vel[2], T))
    q = np.ascontiguousarray(np.stack(qs))
    cfg = cfg_for(n, p, mu=0.0, L=3)
    ntiles = cfg.ntiles
    tab = np.zeros((nlev + 1, ntiles, 6), dtype=np.int8)
    tab[cur] = rng.integers(0, 4, size=(ntiles, 6))
    o = Oracle(cfg)
    o.init_field(q, nlev)
    o.set_schedule(EXPLICIT, table=tab)
    r = o.rhs()
    kl = [int(tab[cur, t, 2 * axis]) for t in range(ntiles)]
    kr = [int(tab[cur, t, 2 * axis + 1]) for t in range(ntiles)]
    rows = F.read_appb(os.path.join(GOLD, "appb_at14.txt"))
    flux_levels = [U * l for l in lines]
    expect = -_appb_derivative_1d(flux_levels, cur, e, kl, kr, 2 * math.pi / N, rows)
    got = np.moveaxis(r[0], 2 - axis, 0).reshape(N, -1)
    for col in range(got.shape[1]):
        np.testing.assert_allclose(got[:, col], expect, rtol=0, atol=1e-12)
    assert any(k > 0 for k in kl + kr)


@pytest.mark.parametrize("axis", [0, 2])
def test_appb_nested_heat_conduction(axis):
    """Energy RHS for pure heat conduction (u = 0, constant mu) = D^{AT}(kappa D^{AT} T): the
    inner derivative uses the published temperatures, the outer one the published heat fluxes of
    history levels (synchronous gradients) or the owner's current AT gradient at k = 0."""
    rng = np.random.default_rng(11 + axis)
    N, e = 16, 4
    n = [4, 4, 4]
    n[axis] = N
    p = [1, 1, 1]
    p[axis] = N // e
    nlev, cur = 6, 5
    gamma, R, Pr, mu = 1.4, 1.0, 0.7, 0.3
    cp = gamma * R / (gamma - 1)
    kap = mu * cp / Pr
    h = 2 * math.pi / N
    shape = (n[2], n[1], n[0])
    lines = [1.0 + 0.1 * rng.standard_normal(N) for _ in range(nlev)]
    qs = []
    for m in range(nlev):
        ls = [1, 1, 1]
        ls[2 - axis] = N
        T = np.broadcast_to(lines[m].reshape(ls), shape).copy()
        z = np.zeros(shape)
        qs.append(F.conservative(np.ones(shape), z, z, z, T))
    cfg = cfg_for(n, p, mu=mu, L=3, mu_exp=0.0)
    tab = np.zeros((nlev + 1, cfg.ntiles, 6), dtype=np.int8)
    # delays on this axis only: the history is random in time, so a delayed transverse face would
    # see an older temperature and produce a transverse gradient
    tab[cur, :, 2 * axis:2 * axis + 2] = rng.integers(0, 4, size=(cfg.ntiles, 2))
    o = Oracle(cfg)
    o.init_field(np.ascontiguousarray(np.stack(qs)), nlev)
    o.set_schedule(EXPLICIT, table=tab)
    r = o.rhs()
    kl = [int(tab[cur, t, 2 * axis]) for t in range(cfg.ntiles)]
    kr = [int(tab[cur, t, 2 * axis + 1]) for t in range(cfg.ntiles)]
    rows = F.read_appb(os.path.join(GOLD, "appb_at14.txt"))
    # history heat fluxes from synchronous derivatives, current one from the AT derivative
    hist_flux = [-kap * _appb_derivative_1d({0: l}, 0, N, [0], [0], h, rows) for l in lines]
    g_cur = _appb_derivative_1d(lines, cur, e, kl, kr, h, rows)
    flux_levels = list(hist_flux)
    expect = -_appb_derivative_1d(flux_levels, cur, e, kl, kr, h, rows, current_override=-kap * g_cur)
    got = np.moveaxis(r[4], 2 - axis, 0).reshape(N, -1)
    for col in range(got.shape[1]):
        np.testing.assert_allclose(got[:, col], expect, rtol=0, atol=1e-11)


# ------------------------------------------------------------------ zero delay = standard (Sec. 2.1)
@pytest.mark.parametrize("p", [(2, 2, 1), (1, 1, 1), (4, 2, 2), (2, 4, 4)])
def test_zero_delay_is_standard_bitwise(p):
    q = W.make_field(16, 3)
    cfg = cfg_for((16, 16, 16), p, mu=0.02)
    o = Oracle(cfg)
    o.init_field(q)
    o.set_schedule(SYNC, n_steps=4)
    np.testing.assert_array_equal(o.rhs(), Oracle.rhs_periodic_standard(cfg, q))


# ------------------------------------------------------------------ conservation (Sec. 2.1, Eqs. tsf-ts4)
def test_conservation_synchronous():
    q = W.make_field(16, 4)
    cfg = cfg_for((16, 16, 16), (2, 2, 2), dt=W.default_dt(q), mu=W.default_mu(16))
    o = Oracle(cfg)
    o.init_field(q)
    o.set_schedule(SYNC, n_steps=10)
    r = o.rhs()
    for c in range(5):
        assert abs(r[c].sum()) <= 1e-13 * np.abs(r[c]).sum()
    s0 = o.stats()
    o.rk_step(6)
    s1 = o.stats()
    for k in ("mass", "energy"):
        assert abs(s1[k] - s0[k]) <= 1e-13 * abs(s0[k])
        assert abs(s1[k + "_rk"] - s1[k]) <= 1e-13 * abs(s0[k])
    for k in ("momx", "momy", "momz"):
        assert abs(s1[k] - s0[k]) <= 1e-13 * s0["mass"]


def _analytic_history(n, nlev, dt, mu=0.05):
    return np.ascontiguousarray(np.stack([F.analytic_state(n, (m - (nlev - 1)) * dt, mu_ref=mu)
                                          for m in range(nlev)]))


@pytest.mark.slow
def test_conservation_residual_high_order_with_delays():
    """With delays the discrete integral of the divergence is no longer zero, but its residual
    vanishes at high order (Eq. ts4: O(dx^{a+1}) for dt ~ dx^2)."""
    res = []
    for N in (16, 32, 64):
        h = 2 * math.pi / N
        dt = 0.5 * h * h
        nlev = 6
        cfg = cfg_for((N, N, N), (2, 2, 2), dt=dt, mu=0.05)
        tab = np.zeros((nlev + 1, 8, 6), dtype=np.int8)
        tab[nlev - 1] = 3
        o = Oracle(cfg)
        o.init_field(_analytic_history((N, N, N), nlev, dt), nlev)
        o.set_schedule(EXPLICIT, table=tab)
        r = o.rhs()
        res.append(max(abs(r[c].sum()) * h ** 3 for c in range(5)))
    order = math.log2(res[1] / res[2])
    assert order >= 4.5, res


# ------------------------------------------------------------------ design order under delays
@pytest.mark.slow
@pytest.mark.parametrize("k", [1, 3])
def test_rhs_fourth_order_under_delays(k):
    """Full NS RHS with AT ghosts at every PE face converges at 4th order to the exact RHS when
    dt ~ dx^2 (Sec. 2.1: the AT orders assume a diffusive relation between dt and dx)."""
    errs = []
    for N in (16, 32, 64):
        h = 2 * math.pi / N
        dt = 0.5 * h * h
        nlev = 6
        cfg = cfg_for((N, N, N), (2, 2, 2), dt=dt, mu=0.05)
        tab = np.zeros((nlev + 1, 8, 6), dtype=np.int8)
        tab[nlev - 1] = k
        o = Oracle(cfg)
        o.init_field(_analytic_history((N, N, N), nlev, dt), nlev)
        o.set_schedule(EXPLICIT, table=tab)
        err = np.abs(o.rhs() - F.analytic_rhs((N, N, N), 0.0)).max()
        errs.append(err)
    order = math.log2(errs[1] / errs[2])
    assert order >= 3.7, errs


def test_rhs_synchronous_matches_exact_rhs():
    N = 32
    cfg = cfg_for((N, N, N), (2, 2, 2), dt=0.01, mu=0.05)
    o = Oracle(cfg)
    o.init_field(F.analytic_state((N, N, N), 0.0))
    o.set_schedule(SYNC, n_steps=1)
    ex = F.analytic_rhs((N, N, N), 0.0)
    err = np.abs(o.rhs() - ex).max()
    assert err < 2e-3 * np.abs(ex).max()


def test_quadratic_time_levels_are_extrapolated_exactly():
    """Fluxes varying quadratically in time: the AT ghost equals the current value, so the AT RHS
    equals the synchronous one to rounding, for every delay (3-level Lagrange extrapolation)."""
    rng = np.random.default_rng(5)
    N, nlev = 16, 6
    a, b, c = (rng.standard_normal((N, N, N)) * s for s in (0.2, 0.05, 0.01))
    U = 0.5
    qs = []
    for m in range(nlev):
        rho = 1.0 + a + b * m + c * m * m
        z = np.zeros_like(rho)
        qs.append(F.conservative(rho, U + z, z, z, 1.0 / rho))
    cfg = cfg_for((N, N, N), (2, 2, 2), mu=0.0)
    tab = np.zeros((nlev + 1, 8, 6), dtype=np.int8)
    tab[nlev - 1] = rng.integers(1, 4, size=(8, 6))
    o = Oracle(cfg)
    o.init_field(np.ascontiguousarray(np.stack(qs)), nlev)
    o.set_schedule(EXPLICIT, table=tab)
    r = o.rhs()
    std = Oracle.rhs_periodic_standard(cfg, qs[-1])
    np.testing.assert_allclose(r[0], std[0], rtol=0, atol=1e-11 * np.abs(std[0]).max())


# ------------------------------------------------------------------ closed forms
def test_modified_wavenumber_advection():
    """rho = 1 + eps sin(m x_d), u = U e_d, p uniform, mu = 0: continuity RHS is exactly
    -U eps k'_m cos(m x_d) with k'_m = (8 sin mh - sin 2mh) / (6h) (4th-order central stencil)."""
    N = 16
    for d in range(3):
        for m in (1, 3):
            X = F.grid((N, N, N))
            eps, U = 0.1, 0.4
            rho = 1.0 + eps * np.sin(m * X[d])
            vel = [np.zeros_like(rho) for _ in range(3)]
            vel[d][:] = U
            q = F.conservative(rho, *vel, 1.0 / rho)
            cfg = cfg_for((N, N, N), (2, 2, 2), mu=0.0)
            o = Oracle(cfg)
            o.init_field(q)
            o.set_schedule(SYNC, n_steps=1)
            kp = F.modified_wavenumber(m, 2 * math.pi / N)
            np.testing.assert_allclose(o.rhs()[0], -U * eps * kp * np.cos(m * X[d]), rtol=0, atol=1e-13)


def test_stats_closed_forms():
    """u = (A sin y, 0, 0), rho = T = 1: K = A^2/4, Omega = A^2 k'^2 / 2, <eps> = mu A^2 k'^2 / 2,
    M_t = (A^2/2)^{1/2} / (gamma R)^{1/2}, totals over [0, 2pi)^3."""
    N, A, mu = 16, 0.3, 0.02
    X, Y, Z = F.grid((N, N, N))
    z = np.zeros_like(X)
    q = F.conservative(1.0 + z, A * np.sin(Y), z, z, 1.0 + z)
    cfg = cfg_for((N, N, N), (2, 2, 2), mu=mu)
    o = Oracle(cfg)
    o.init_field(q)
    o.set_schedule(SYNC, n_steps=1)
    s = o.stats()
    kp = F.modified_wavenumber(1, 2 * math.pi / N)
    vol = (2 * math.pi) ** 3
    assert s["K"] == pytest.approx(A * A / 4, rel=1e-13)
    assert s["enstrophy"] == pytest.approx(A * A * kp * kp / 2, rel=1e-13)
    assert s["eps"] == pytest.approx(mu * A * A * kp * kp / 2, rel=1e-12)
    assert s["Mt"] == pytest.approx(math.sqrt(A * A / 2) / math.sqrt(1.4), rel=1e-13)
    assert s["mass"] == pytest.approx(vol, rel=1e-14)
    assert s["energy"] == pytest.approx(vol * (2.5 + A * A / 4), rel=1e-13)
    assert abs(s["momx"]) < 1e-13 and s["umax"] == pytest.approx(A, rel=1e-15)
    assert s["nonfinite"] == 0


@pytest.mark.parametrize("p", [(1, 1, 1), (2, 2, 2)])
def test_rk3_entropy_wave_one_step(p):
    """Inviscid entropy wave rho = 1 + 0.2 sin(x+y+z), u = (U,U,U), p uniform: each Fourier mode
    evolves as y' = lambda y with lambda = -3 i U k'_1, so one LS-RK3 step multiplies it exactly by
    1 + z + z^2/2 + z^3/6, z = lambda dt (third-order Runge-Kutta)."""
    N, U, amp = 16, 0.3, 0.2
    X, Y, Z = F.grid((N, N, N))
    th = X + Y + Z
    rho = 1.0 + amp * np.sin(th)
    vel = [U + 0 * rho] * 3
    q = F.conservative(rho, *vel, 1.0 / rho)
    dt = 0.05
    cfg = cfg_for((N, N, N), p, dt=dt, mu=0.0)
    o = Oracle(cfg)
    o.init_field(q)
    o.set_schedule(SYNC, n_steps=2)
    o.rk_step(1)
    kp = F.modified_wavenumber(1, 2 * math.pi / N)
    g = F.rk3_amplification(-3j * U * kp * dt)
    rho1 = 1.0 + amp * np.imag(g * np.exp(1j * th))
    out = o.field()
    np.testing.assert_allclose(out[0], rho1, rtol=0, atol=1e-13)
    for c in range(1, 4):
        np.testing.assert_allclose(out[c], U * rho1, rtol=0, atol=1e-13)
    np.testing.assert_allclose(out[4], 1.0 / 0.4 + 1.5 * U * U * rho1, rtol=0, atol=1e-12)


@pytest.mark.parametrize("p", [(1, 1, 1), (2, 2, 2)])
def test_ab2_entropy_wave_closed_form(p):
    """Second-order Adams-Bashforth (Sec. 2.2, Eq. time_ab, beta = (3/2, -1/2)) on the inviscid
    entropy wave of test_rk3_entropy_wave_one_step: each Fourier mode is y' = lambda y, so after a
    forward-Euler start y_n = A r1^n + B r2^n, with r1, r2 the roots of the method's characteristic
    polynomial r^2 - (1 + 3z/2) r + z/2 = 0 (z = lambda dt), A + B = 1 and A r1 + B r2 = 1 + z."""
    N, U, amp = 16, 0.3, 0.2
    X, Y, Z = F.grid((N, N, N))
    th = X + Y + Z
    rho = 1.0 + amp * np.sin(th)
    q = F.conservative(rho, *([U + 0 * rho] * 3), 1.0 / rho)
    dt, nsteps = 0.05, 5
    o = Oracle(cfg_for((N, N, N), p, dt=dt, mu=0.0))
    o.init_field(q)
    o.set_schedule(SYNC, n_steps=nsteps + 1)
    o.ab2_step(nsteps)
    z = -3j * U * F.modified_wavenumber(1, 2 * math.pi / N) * dt
    b = 1 + 1.5 * z
    disc = np.sqrt(b * b - 2 * z + 0j)
    r1, r2 = (b + disc) / 2, (b - disc) / 2
    B = (1 + z - r1) / (r2 - r1)
    A = 1 - B
    g = A * r1 ** nsteps + B * r2 ** nsteps
    rho_n = 1.0 + amp * np.imag(g * np.exp(1j * th))
    out = o.field()
    np.testing.assert_allclose(out[0], rho_n, rtol=0, atol=1e-13)
    for c in range(1, 4):
        np.testing.assert_allclose(out[c], U * rho_n, rtol=0, atol=1e-13)
    assert o.step == nsteps


def test_ab2_second_order_in_time():
    """Sec. 2.2: the AB scheme of order 2.  On a smooth viscous field (synchronous derivatives),
    the state at a fixed time from dt, dt/2, dt/4 differs from a Runge-Kutta reference at dt/32 by
    errors whose ratios are ~4 (forward Euler would give ~2)."""
    n = 16
    q = W.make_field(n, 11, 0.3)
    dt0 = W.default_dt(q)
    mu = W.default_mu(n)

    def run(dt, steps, ab2):
        o = Oracle(cfg_for((n, n, n), (2, 2, 2), dt=dt, mu=mu))
        o.init_field(q)
        o.set_schedule(SYNC, n_steps=steps + 1)
        (o.ab2_step if ab2 else o.rk_step)(steps)
        return o.field()

    ref = run(dt0 / 32, 256, False)
    errs = [np.linalg.norm(run(dt0 / m, 8 * m, True) - ref) for m in (1, 2, 4)]
    ratios = [errs[0] / errs[1], errs[1] / errs[2]]
    assert all(3.4 < r < 4.6 for r in ratios), (errs, ratios)


def test_uniform_state_any_schedule():
    """Constant state: every flux is uniform and the extrapolation weights sum to one, so the RHS
    vanishes whatever the delays."""
    N = 16
    q = np.empty((5, N, N, N))
    vals = [1.2, 0.3, -0.1, 0.2, 3.0]
    for c in range(5):
        q[c] = vals[c]
    cfg = cfg_for((N, N, N), (2, 2, 2), dt=0.01, mu=0.05, L=3)
    o = Oracle(cfg)
    o.init_field(q)
    o.set_schedule(SAA, L=3, seed=9, n_steps=12)
    o.rk_step(10)
    out = o.field()
    for c in range(5):
        np.testing.assert_allclose(out[c], vals[c], rtol=2e-14, atol=2e-14)


def test_axis_permutation_symmetry():
    """Swapping x and y in the field, the PE grid and the per-face delays swaps the RHS."""
    rng = np.random.default_rng(3)
    N = 16
    nlev = 6
    qs = [W.make_field(N, 20 + m, 0.3) for m in range(nlev)]
    q = np.ascontiguousarray(np.stack(qs))
    p = (2, 4, 1)
    cfg = cfg_for((N, N, N), p, mu=0.03, L=3)
    nt = cfg.ntiles
    tab = np.zeros((nlev + 1, nt, 6), dtype=np.int8)
    tab[nlev - 1] = rng.integers(0, 4, size=(nt, 6))
    o = Oracle(cfg)
    o.init_field(q, nlev)
    o.set_schedule(EXPLICIT, table=tab)
    r = o.rhs()
    # permuted problem
    qp = q.transpose(0, 1, 2, 4, 3)[:, [0, 2, 1, 3, 4]].copy()
    pp = (p[1], p[0], p[2])
    cfgp = cfg_for((N, N, N), pp, mu=0.03, L=3)
    tabp = np.zeros_like(tab)
    for tz in range(p[2]):
        for ty in range(p[1]):
            for tx in range(p[0]):
                t = (tz * p[1] + ty) * p[0] + tx
                tp = (tz * pp[1] + tx) * pp[0] + ty
                tabp[:, tp] = tab[:, t][:, [2, 3, 0, 1, 4, 5]]
    op = Oracle(cfgp)
    op.init_field(np.ascontiguousarray(qp), nlev)
    op.set_schedule(EXPLICIT, table=tabp)
    rp = op.rhs()
    back = rp.transpose(0, 1, 3, 2)[[0, 2, 1, 3, 4]]
    np.testing.assert_allclose(back, r, rtol=0, atol=1e-12 * np.abs(r).max())


# ------------------------------------------------------------------ schedules (Sec. 3.1)
def test_caa_schedule_pattern_and_uniform_pdf():
    cfg = cfg_for((16, 16, 16), (2, 2, 2), L=3)
    o = Oracle(cfg)
    o.init_field(W.make_field(16, 1))
    o.set_schedule(CAA, L=3, c_r=4, n_steps=44)
    t = o.get_schedule(44)
    assert (t[:4] == 0).all()
    for n in range(4, 44):
        assert (t[n] == n % 4).all()
    hist = np.bincount(t[4:].ravel(), minlength=4)
    assert (hist == hist[0]).all()  # uniform PDF over whole periods (Fig. del_pdf(d))


def test_saa_schedule_statistics():
    cfg = cfg_for((32, 32, 32), (4, 4, 4), L=3)
    o = Oracle(cfg)
    o.init_field(W.make_field(32, 1))
    L, nst = 2, 200
    o.set_schedule(SAA, L=L, seed=102, n_steps=nst)
    t = o.get_schedule(nst)
    assert (t[:L + 3] == 0).all()
    body = t[L + 3:].ravel()
    assert body.min() == 0 and body.max() == L
    cnt = np.bincount(body, minlength=L + 1)
    nexp = body.size / (L + 1)
    sd = math.sqrt(body.size * (1 / (L + 1)) * (1 - 1 / (L + 1)))
    assert np.all(np.abs(cnt - nexp) < 5 * sd)


def test_splitmix64_known_answers():
    """Published SplitMix64 outputs for seed 0 (Steele, Lea & Flood 2014; reference splitmix64.c)."""
    assert Oracle.splitmix64(0, 0) == 0xE220A8397B1DCDAF
    assert Oracle.splitmix64(0, 1) == 0x6E789E6AA1B965F4
    assert Oracle.splitmix64(0, 2) == 0x06C45D188009454F


def test_schedule_validation():
    cfg = cfg_for((16, 16, 16), (2, 2, 2), L=2)
    o = Oracle(cfg)
    o.init_field(W.make_field(16, 1))
    bad = np.zeros((8, 8, 6), dtype=np.int8)
    bad[6, 0, 0] = 3  # beyond max_delay
    with pytest.raises(OracleError):
        o.set_schedule(EXPLICIT, table=bad)
    bad[6, 0, 0] = 0
    bad[2, 0, 0] = 1  # needs level -1
    with pytest.raises(OracleError):
        o.set_schedule(EXPLICIT, table=bad)
    with pytest.raises(OracleError):
        o.set_schedule(CAA, L=3, c_r=4, n_steps=8)  # L = 3 > max_delay = 2


# ------------------------------------------------------------------ Eq. NB and Table DNS
def test_boundary_point_fraction_table_dns():
    for line in open(os.path.join(GOLD, "table_dns_nb.txt")):
        if line.startswith("#") or not line.strip():
            continue
        n, ex, ey, ez, pct = line.split()
        n, ex, ey, ez, pct = int(n), int(ex), int(ey), int(ez), float(pct)
        m = 64  # a smaller grid with the same per-PE block gives the same percentage
        cfg = cfg_for((max(m, ex), max(m, ey), max(m, ez)),
                      (max(m, ex) // ex, max(m, ey) // ey, max(m, ez) // ez))
        cnt = Oracle.count_at_points(cfg)
        frac = 100.0 * cnt / (max(m, ex) * max(m, ey) * max(m, ez))
        assert round(frac, 1) == pct
        nt = ex * ey * ez
        ni = (ex - 4) * (ey - 4) * (ez - 4)
        assert frac == pytest.approx(100.0 * (nt - ni) / nt, rel=1e-15)  # Eq. NB


# ------------------------------------------------------------------ inputs: field and forcing
def test_initial_field_generator():
    N, mt = 32, 0.3
    q = W.make_field(N, 1, mt)
    u = q[1:4] / q[0]
    c0 = math.sqrt(1.4)
    assert float((u * u).sum(axis=0).mean()) == pytest.approx((mt * c0) ** 2, rel=1e-12)
    uh = np.fft.fftn(u, axes=(1, 2, 3))
    k = np.fft.fftfreq(N, 1.0 / N)
    KZ, KY, KX = np.meshgrid(k, k, k, indexing="ij")
    div = KX * uh[0] + KY * uh[1] + KZ * uh[2]
    assert np.abs(div).max() < 1e-10 * np.abs(uh).max()
    km = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    sh = np.rint(km).astype(int)
    e = np.bincount(sh.ravel(), weights=(0.5 * (np.abs(uh) ** 2).sum(axis=0)).ravel())
    ks = np.arange(1, N // 2 - 1)
    target = ks ** 4.0 * np.exp(-2 * (ks / 4.0) ** 2)
    ratio = e[ks] / target
    np.testing.assert_allclose(ratio, ratio[0], rtol=1e-9)


def test_forcing_field_matches_fft_of_amplitudes():
    """The oracle's forcing field has FFT coefficient N^3 fhat_k at k and its conjugate at -k."""
    N = 8
    fh = W.make_forcing(303, 2, 0.01)[1]
    cfg = cfg_for((N, N, N), (2, 2, 2))
    f = Oracle.forcing_field(cfg, fh)
    ks = W.forcing_wavevectors()
    assert ks.shape == (40, 3)
    fft = np.fft.fftn(f, axes=(1, 2, 3)) / N ** 3
    expect = np.zeros_like(fft)
    for i, (kx, ky, kz) in enumerate(ks):
        c = fh[i, :, 0] + 1j * fh[i, :, 1]
        expect[:, kz % N, ky % N, kx % N] += c
        expect[:, (-kz) % N, (-ky) % N, (-kx) % N] += np.conj(c)
    np.testing.assert_allclose(fft, expect, atol=1e-14)


def test_forcing_amplitudes_ou_statistics():
    dt, tl, sig = 0.05, 1.0, 0.1
    fh = W.make_forcing(5, 4000, dt, tl, sig)
    ks = W.forcing_wavevectors().astype(float)
    c = fh[..., 0] + 1j * fh[..., 1]
    # solenoidal
    assert np.abs(np.einsum("nki,ki->nk", c, ks)).max() < 1e-14
    # stationary variance: projection keeps 2 of 3 complex components -> E|fhat|^2 = 4 sigma^2
    m = float((np.abs(c) ** 2).sum(axis=2).mean())
    assert m == pytest.approx(4 * sig * sig, rel=0.08)
    # lag-1 correlation alpha = exp(-dt/T_L)
    b = c[:, :, 0].real
    r1 = float((b[1:] * b[:-1]).mean() / (b * b).mean())
    assert r1 == pytest.approx(math.exp(-dt / tl), abs=0.02)


def test_default_mu_resolution_rule():
    # kappa_max eta = 1.5 with kappa_max = sqrt(2) N / 3 (Sec. 4 set-up); values for M_t = 0.3
    assert W.default_mu(32) == pytest.approx(1.57e-2, rel=5e-3)
    assert W.default_mu(256) == pytest.approx(2.45e-4, rel=5e-3)
    assert W.default_mu(512) == pytest.approx(6.13e-5, rel=5e-3)


@pytest.mark.slow
def test_dt_proportional_to_h_loses_order():
    """Negative control: the AT orders assume dt ~ dx^2 (Sec. 2.1); with dt ~ dx the time
    extrapolation error O(dt^3 / dx) caps the face error at second order."""
    errs = []
    for N in (16, 32, 64):
        h = 2 * math.pi / N
        dt = 0.2 * h
        nlev = 6
        cfg = cfg_for((N, N, N), (2, 2, 2), dt=dt, mu=0.05)
        tab = np.zeros((nlev + 1, 8, 6), dtype=np.int8)
        tab[nlev - 1] = 3
        o = Oracle(cfg)
        o.init_field(_analytic_history((N, N, N), nlev, dt), nlev)
        o.set_schedule(EXPLICIT, table=tab)
        errs.append(np.abs(o.rhs() - F.analytic_rhs((N, N, N), 0.0)).max())
    order = math.log2(errs[1] / errs[2])
    assert 1.5 < order < 2.7, errs


@pytest.mark.slow
def test_stage_time_extrapolation_order():
    """Delayed ghosts at RK stage s are extrapolated to t_n + c_s dt (kappa = k + c_s).  Then the
    difference between a CAA run and the synchronous run over a fixed time falls as dt^3 at fixed
    dx; extrapolating every stage to t_n instead would leave an O(dt) error."""
    N = 16
    q = F.analytic_state((N, N, N), 0.0)
    T = 0.4
    diffs = []
    for dt in (0.01, 0.005):
        ns = int(round(T / dt))
        runs = []
        for mode in (CAA, SYNC):
            o = Oracle(cfg_for((N, N, N), (2, 2, 2), dt=dt, mu=0.05))
            o.init_field(q)
            if mode == CAA:
                o.set_schedule(CAA, L=3, c_r=4, n_steps=ns + 1)
            else:
                o.set_schedule(SYNC, n_steps=ns + 1)
            o.rk_step(ns)
            runs.append(o.field())
        diffs.append(np.abs(runs[0] - runs[1]).max())
    assert math.log2(diffs[0] / diffs[1]) > 2.5, diffs


# ------------------------------------------------------------------ forcing source (Sec. 4.2)
def _single_mode_forcing(n_steps):
    """Forcing tables whose rows hold one or two wavevectors each, so that every row's field is a
    known closed form: a real amplitude a at k gives 2 a cos(k.x), an imaginary one b gives
    -2 b sin(k.x).  Row 0: f_y = cos(x), f_x = -0.5 sin(z).  Row 1: f_z = cos(y) + 0.25 cos(x + y).
    Row 2 (and later): f_x = 0.75 cos(2 y).  Each amplitude is normal to its k (solenoidal)."""
    ks = [tuple(k) for k in W.forcing_wavevectors().tolist()]
    fh = np.zeros((n_steps, 40, 3, 2))
    fh[0, ks.index((1, 0, 0)), 1, 0] = 0.5
    fh[0, ks.index((0, 0, 1)), 0, 1] = 0.25
    fh[1, ks.index((0, 1, 0)), 2, 0] = 0.5
    fh[1, ks.index((1, 1, 0)), 2, 0] = 0.125
    fh[2:, ks.index((0, 2, 0)), 0, 0] = 0.375
    return fh


def _closed_form_force(row, n):
    X, Y, Z = F.grid(n)
    z = np.zeros_like(X)
    if row == 0:
        return np.stack([-0.5 * np.sin(Z), np.cos(X), z])
    if row == 1:
        return np.stack([z, z, np.cos(Y) + 0.25 * np.cos(X + Y)])
    return np.stack([0.75 * np.cos(2 * Y), z, z])


def _uniform_forced_state(n, rho=2.0, vel=(0.25, -0.5, 0.125), T=1.5, gamma=1.5):
    """rho, u, T constant: every flux is the same number at every point, so the flux divergence
    vanishes and the RHS is the forcing source alone.  gamma = 1.5 makes c_v = 2 exact."""
    cv = 1.0 / (gamma - 1.0)
    ke = 0.5 * sum(v * v for v in vel)
    q = np.empty((5,) + (n[2], n[1], n[0]))
    q[0] = rho
    for a in range(3):
        q[1 + a] = rho * vel[a]
    q[4] = rho * (cv * T + ke)
    return q


def test_forcing_source_on_uniform_state_two_steps():
    """Eq. mome carries rho f_i (Sec. 4.2); in total-energy form the energy equation gains its work
    rho f.u.  On a uniform state with constant velocity the RHS is therefore exactly
    (0, rho f, rho f.u) with f the closed form of the current step's forcing row.  Checked at step
    0 (one supplied level) and step 1 (two supplied levels), whose rows differ: a wrong sign, a
    missing or wrong energy term, a permuted component or the wrong row fails."""
    n = (16, 12, 8)
    q = _uniform_forced_state(n)
    rho, m = 2.0, (0.5, -1.0, 0.25)
    fh = _single_mode_forcing(4)
    for nlev, row in ((1, 0), (2, 1)):
        o = Oracle(cfg_for(n, (2, 3, 1), dt=1e-3, mu=0.01, gamma=1.5, forcing=True))
        o.init_field(np.stack([q] * nlev) if nlev > 1 else q, nlev)
        o.set_schedule(SYNC, n_steps=4)
        o.set_forcing(fh)
        r = o.rhs()
        f = _closed_form_force(row, n)
        assert np.abs(r[0]).max() == 0.0
        for a in range(3):
            np.testing.assert_allclose(r[1 + a], rho * f[a], rtol=0, atol=1e-14)
        np.testing.assert_allclose(r[4], m[0] * f[0] + m[1] * f[1] + m[2] * f[2], rtol=0, atol=1e-14)
        # the other rows' fields really differ from this one (so the row choice is tested)
        for other in (0, 1, 2):
            if other != row:
                assert np.abs(_closed_form_force(other, n) - f).max() > 0.5


def test_forcing_held_fixed_within_step():
    """The force is held fixed over the three stages of a step (reading A16).  From a uniform state
    one RK3 step gives Q + dt (0, rho f_n, rho f_n.u) + O(dt^2): the error against that falls four
    times when dt halves.  Evaluating a later stage with the next row (which differs here) would
    leave an O(dt) error, a ratio near 2."""
    n = (16, 16, 8)
    q = _uniform_forced_state(n)
    fh = _single_mode_forcing(4)
    f1 = _closed_form_force(1, n)
    src = np.stack([np.zeros_like(f1[0]), 2.0 * f1[0], 2.0 * f1[1], 2.0 * f1[2],
                    0.5 * f1[0] - 1.0 * f1[1] + 0.25 * f1[2]])
    errs = []
    for dt in (2e-3, 1e-3):
        o = Oracle(cfg_for(n, (2, 2, 1), dt=dt, mu=0.01, gamma=1.5, forcing=True))
        o.init_field(np.stack([q, q]), 2)  # current step 1: row 1
        o.set_schedule(SYNC, n_steps=4)
        o.set_forcing(fh)
        o.rk_step(1)
        errs.append(np.abs(o.field() - (q + dt * src)).max())
    ratio = errs[0] / errs[1]
    assert 3.6 < ratio < 4.4, errs
    # and the step moved the state by dt * source to leading order
    assert errs[1] < 1e-3 * 1e-3 * np.abs(src).max(), errs


# ------------------------------------------------------------------ sixth-order AT (Sec. 4.1.2; Appendix B, (1,6) rows)
def cfg6(n, p, dt=0.01, mu=0.0, L=3, **kw):
    return cfg_for(n, p, dt=dt, mu=mu, L=L, order=6, **kw)


def _poly(w, k):
    return sum(c * k ** (len(w) - 1 - i) for i, c in enumerate(w))


def test_appb6_weights_at_integer_delay_and_stage_times():
    """w_l(k) of the cubic extrapolation equal the (1,6) Appendix B polynomials at integer k and sum
    to one; at k = 0 the scheme is the standard one (Sec. 2.1).  At non-integer kappa = k + c_s (RK
    stage times) they are the weights that extrapolate every cubic in time exactly: the solution of
    the Vandermonde system on the level times -(kappa + l), solved here with numpy."""
    rows = F.read_appb(os.path.join(GOLD, "appb_at16.txt"))
    assert len(rows) == 8 and all(len(r["w"]) == 4 and len(r["a"]) == 7 for r in rows)
    for k in range(0, 6):
        for r in rows:
            assert Oracle.at_weight6(r["l"], float(k)) == pytest.approx(_poly(r["w"], k), rel=1e-15, abs=1e-13)
        assert sum(Oracle.at_weight6(l, float(k)) for l in range(4)) == pytest.approx(1.0, abs=1e-13)
    assert [Oracle.at_weight6(l, 0.0) for l in range(4)] == [1.0, 0.0, 0.0, 0.0]
    assert [Oracle.at_weight6(l, 3.0) for l in range(4)] == [20.0, -45.0, 36.0, -10.0]
    for kap in (0.25, 1.0 / 3.0, 1.75, 3.75):
        tau = -(kap + np.arange(4.0))
        V = np.vander(tau, 4, increasing=True).T  # rows: sum_l w_l tau_l^j = delta_j0
        w = np.linalg.solve(V, np.array([1.0, 0.0, 0.0, 0.0]))
        got = [Oracle.at_weight6(l, kap) for l in range(4)]
        np.testing.assert_allclose(got, w, rtol=1e-12, atol=1e-12)


def _appb_line(levels, n, e, kl, kr, h, rows, current_override=None):
    """The printed AT rows (either order) along one periodic line; as _appb_derivative_1d."""
    N = levels[n].shape[0]
    cur = levels[n] if current_override is None else current_override
    rows = [r for r in rows if r["side"] == "left"]
    M = (len(rows[0]["a"]) - 1) // 2
    offs = list(range(-M, M + 1))
    out = np.zeros(N)
    for i in range(N):
        t, loc = divmod(i, e)
        k = kl[t] if loc < M else (kr[t] if loc >= e - M else 0)
        acc = 0.0
        for r in rows:
            s = 0.0
            for a, m in zip(r["a"], offs):
                outside = not (0 <= loc + m < e)
                j = (i + m) % N
                s += a * (levels[n - k - r["l"]][j] if (outside and k > 0) else cur[j])
            acc += _poly(r["w"], k) * s
        out[i] = acc / (rows[0]["div"] * h)
    return out


@pytest.mark.parametrize("axis", [0, 2])
def test_appb6_stencil_mass_flux(axis):
    """Continuity RHS with the sixth-order scheme equals -(1,6) AT derivative of the mass flux as
    printed in Appendix B (misprints corrected, see the golden file), per-face delays 0..3 and
    arbitrary history levels: checks each cubic weight, each level index and the 3-point ghosts."""
    rng = np.random.default_rng(17 + axis)
    N, e = 24, 6
    n = [6, 6, 6]
    n[axis] = N
    p = [1, 1, 1]
    p[axis] = N // e
    nlev = 7
    cur = nlev - 1
    U = 0.7
    lines = [1.0 + 0.2 * rng.standard_normal(N) for _ in range(nlev)]
    shape = (n[2], n[1], n[0])
    qs = []
    for m in range(nlev):
        ls = [1, 1, 1]
        ls[2 - axis] = N
        rho = np.broadcast_to(lines[m].reshape(ls), shape).copy()
        vel = [np.zeros(shape) for _ in range(3)]
        vel[axis][:] = U
        qs.append(F.conservative(rho, vel[0], vel[1], vel[2], 1.0 / rho))
    cfg = cfg6(n, p, L=3)
    tab = np.zeros((nlev + 1, cfg.ntiles, 6), dtype=np.int8)
    tab[cur] = rng.integers(0, 4, size=(cfg.ntiles, 6))  # transverse fluxes vanish at every level
    tab[cur, :, 2 * axis] = [0, 1, 2, 3]  # every delay on the faces along the axis
    tab[cur, :, 2 * axis + 1] = [3, 1, 0, 2]
    o = Oracle(cfg)
    o.init_field(np.ascontiguousarray(np.stack(qs)), nlev)
    o.set_schedule(EXPLICIT, table=tab)
    r = o.rhs()
    kl = [int(tab[cur, t, 2 * axis]) for t in range(cfg.ntiles)]
    kr = [int(tab[cur, t, 2 * axis + 1]) for t in range(cfg.ntiles)]
    rows = F.read_appb(os.path.join(GOLD, "appb_at16.txt"))
    expect = -_appb_line([U * l for l in lines], cur, e, kl, kr, 2 * math.pi / N, rows)
    got = np.moveaxis(r[0], 2 - axis, 0).reshape(N, -1)
    for col in range(got.shape[1]):
        np.testing.assert_allclose(got[:, col], expect, rtol=0, atol=1e-12)
    assert 3 in kl + kr


@pytest.mark.parametrize("p", [(2, 2, 1), (1, 1, 1), (3, 2, 2)])
def test_order6_zero_delay_is_standard_bitwise(p):
    q = W.make_field(24, 3)
    cfg = cfg6((24, 24, 24), p, mu=0.02)
    o = Oracle(cfg)
    o.init_field(q)
    o.set_schedule(SYNC, n_steps=4)
    np.testing.assert_array_equal(o.rhs(), Oracle.rhs_periodic_standard(cfg, q))


def test_order6_conservation_synchronous():
    q = W.make_field(24, 4)
    cfg = cfg6((24, 24, 24), (2, 2, 2), dt=W.default_dt(q), mu=W.default_mu(24))
    o = Oracle(cfg)
    o.init_field(q)
    o.set_schedule(SYNC, n_steps=4)
    r = o.rhs()
    for c in range(5):
        assert abs(r[c].sum()) <= 1e-13 * np.abs(r[c]).sum()


def test_order6_modified_wavenumber():
    """rho = 1 + eps sin(m x), u = U e_x, p uniform, mu = 0: continuity RHS = -U eps k'_m cos(m x)
    with the 6th-order modified wavenumber k'_m = (45 sin mh - 9 sin 2mh + sin 3mh) / (30 h)."""
    N = 24
    h = 2 * math.pi / N
    X = F.grid((N, N, N))
    for m in (1, 4):
        eps, U = 0.1, 0.4
        rho = 1.0 + eps * np.sin(m * X[0])
        z = np.zeros_like(rho)
        o = Oracle(cfg6((N, N, N), (2, 2, 2)))
        o.init_field(F.conservative(rho, U + z, z, z, 1.0 / rho))
        o.set_schedule(SYNC, n_steps=1)
        kp = (45 * math.sin(m * h) - 9 * math.sin(2 * m * h) + math.sin(3 * m * h)) / (30 * h)
        np.testing.assert_allclose(o.rhs()[0], -U * eps * kp * np.cos(m * X[0]), rtol=0, atol=1e-13)


def test_cubic_time_levels_are_extrapolated_exactly():
    """Fluxes varying cubically in time: the 4-level AT ghost equals the current value, so the AT
    RHS equals the synchronous one to rounding for every delay; the 4th-order scheme (3 levels) is
    not exact on the same data."""
    rng = np.random.default_rng(6)
    N, nlev = 24, 7
    a, b, c, d = (rng.standard_normal((N, N, N)) * s for s in (0.2, 0.05, 0.01, 0.003))
    qs = []
    for m in range(nlev):
        rho = 1.0 + a + b * m + c * m * m + d * m ** 3
        z = np.zeros_like(rho)
        qs.append(F.conservative(rho, 0.5 + z, z, z, 1.0 / rho))
    q = np.ascontiguousarray(np.stack(qs))
    tab = np.zeros((nlev + 1, 8, 6), dtype=np.int8)
    tab[nlev - 1] = rng.integers(1, 4, size=(8, 6))
    out = {}
    for order in (6, 4):
        cfg = cfg_for((N, N, N), (2, 2, 2), mu=0.0, L=3, order=order)
        o = Oracle(cfg)
        nl = nlev if order == 6 else 6
        o.init_field(np.ascontiguousarray(q[nlev - nl:]), nl)
        o.set_schedule(EXPLICIT, table=tab[nlev - nl:])
        out[order] = (o.rhs()[0], Oracle.rhs_periodic_standard(cfg, qs[-1])[0])
    r, std = out[6]
    np.testing.assert_allclose(r, std, rtol=0, atol=1e-11 * np.abs(std).max())
    r4, std4 = out[4]
    assert np.abs(r4 - std4).max() > 1e-6 * np.abs(std4).max()


@pytest.mark.slow
@pytest.mark.parametrize("k", [1, 3])
def test_rhs_sixth_order_under_delays(k):
    """Full NS RHS with (1,6) AT ghosts at every PE face converges at 6th order to the exact RHS
    when dt ~ dx^2 (the cubic extrapolation error O(dt^4 / dx) is then O(dx^7))."""
    errs = []
    for N in (16, 32, 64):
        h = 2 * math.pi / N
        dt = 0.5 * h * h
        nlev = 7
        cfg = cfg6((N, N, N), (2, 2, 2), dt=dt, mu=0.05)
        tab = np.zeros((nlev + 1, 8, 6), dtype=np.int8)
        tab[nlev - 1] = k
        o = Oracle(cfg)
        o.init_field(_analytic_history((N, N, N), nlev, dt), nlev)
        o.set_schedule(EXPLICIT, table=tab)
        errs.append(np.abs(o.rhs() - F.analytic_rhs((N, N, N), 0.0)).max())
    order = math.log2(errs[1] / errs[2])
    assert order >= 5.5, errs


def test_order6_schedules_and_validation():
    """t_l = 4 levels: SAA runs synchronously for L + 4 steps, CAA for max(c_r, 4); a delay k at
    step n needs n - k - 3 >= 0; the ring keeps L + 4 levels."""
    cfg = cfg6((24, 24, 24), (2, 2, 2), L=2)
    o = Oracle(cfg)
    o.init_field(W.make_field(24, 1))
    o.set_schedule(SAA, L=2, seed=102, n_steps=40)
    t = o.get_schedule(40)
    assert (t[:6] == 0).all() and (t[6:] > 0).any() and t.max() == 2
    o.set_schedule(CAA, L=1, c_r=2, n_steps=12)
    t = o.get_schedule(12)
    assert (t[:4] == 0).all() and all((t[n] == n % 2).all() for n in range(4, 12))
    bad = np.zeros((8, 8, 6), dtype=np.int8)
    bad[4, 0, 0] = 2  # needs level 4 - 2 - 3 = -1
    with pytest.raises(OracleError):
        o.set_schedule(EXPLICIT, table=bad)
    bad[4, 0, 0] = 1  # levels 3 .. 0: fine
    o.set_schedule(EXPLICIT, table=bad)
    with pytest.raises(OracleError):
        o.init_field(np.stack([W.make_field(24, 1)] * 7), 7)  # more levels than L + 4 = 6


def test_order6_boundary_point_fraction():
    """Eq. NB with M = 3 boundary layers: N_B = N_T - (ex - 6)(ey - 6)(ez - 6) per PE."""
    for ex, ey, ez in ((16, 16, 16), (32, 16, 16), (12, 8, 24)):
        cfg = cfg6((2 * ex, 2 * ey, 2 * ez), (2, 2, 2))
        nt = ex * ey * ez
        assert Oracle.count_at_points(cfg) == 8 * (nt - (ex - 6) * (ey - 6) * (ez - 6))
