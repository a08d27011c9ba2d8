"""The sixth-order AT scheme on the GPU (the (1,6) rows of Appendix B, Sec. 4.1.2) against the CPU
FP64 oracle, through the C ABI.  FP64 bar: relative L2 <= 1e-12 per conserved component and per
statistic; FP32 bound 2e-6 per component (as for the fourth-order scheme: ~6e-8 relative rounding
per operation, mildly amplified over the steps)."""
import sys

import numpy as np
import pytest

from oracle import Oracle, OracleConfig
from paper_2003_10561_amd import workload as W
from tests import fields as F

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2003_10561_amd import atns  # noqa: E402

TOL64 = 1e-12
STAT_KEYS = ["mass", "energy", "mass_rk", "energy_rk", "K", "eps", "enstrophy", "Mt", "umax"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def compare_fields(got, ref, tol, what):
    errs = [rel_l2(got[c], ref[c]) for c in range(5)]
    say(f"  {what} rel-L2 per component: " + " ".join(f"{e:.2e}" for e in errs))
    assert max(errs) <= tol, errs
    return errs


def compare_stats(gs, os_, tol):
    for k in STAT_KEYS:
        err = abs(gs[k] - os_[k]) / max(abs(os_[k]), 1e-300)
        assert err <= tol, (k, gs[k], os_[k], err)
    assert gs["step"] == os_["step"] and gs["nonfinite"] == 0


def pair(n, p, q, nlev=1, dt=None, mu=None, L=3, precision="fp64"):
    qcur = q[-1] if nlev > 1 else q
    dt = dt if dt is not None else W.default_dt(qcur)
    mu = mu if mu is not None else W.default_mu(n[0])
    g = atns.Sim(atns.Config(n=n, p=p, dt=dt, mu_ref=mu, max_delay=L, precision=precision, order=6))
    o = Oracle(OracleConfig(n=n, p=p, dt=dt, mu_ref=mu, max_delay=L, order=6))
    g.init_field(q, nlev)
    o.init_field(q, nlev)
    return g, o


def history_levels(n, nlev, seed):
    """Levels that vary smoothly in time (a drift plus a small per-level perturbation)."""
    rng = np.random.default_rng(seed)
    shp = (n[2], n[1], n[0])
    base_u = W.make_velocity(max(n), seed, 0.1)[:, :n[2], :n[1], :n[0]]
    drift_u = W.make_velocity(max(n), seed + 1, 0.1)[:, :n[2], :n[1], :n[0]]
    rho0, rho1 = 1.0 + 0.05 * rng.standard_normal(shp), 0.01 * rng.standard_normal(shp)
    t0, t1 = 1.0 + 0.05 * rng.standard_normal(shp), 0.01 * rng.standard_normal(shp)
    out = []
    for m in range(nlev):
        s = m / nlev
        jit = 1e-3 * rng.standard_normal((5,) + shp)
        u = base_u + s * drift_u + jit[:3]
        out.append(F.conservative(rho0 + s * rho1 + jit[3], *u, t0 + s * t1 + jit[4]))
    return np.ascontiguousarray(np.stack(out))


@pytest.mark.parametrize("n,p", [((36, 24, 48), (3, 2, 4)), ((48, 24, 24), (2, 2, 2)), ((24, 12, 18), (4, 2, 3)),
                                 ((64, 16, 12), (2, 1, 2))])
def test_order6_rhs_random_delays_history_levels(n, p):
    """RHS with seven supplied levels and random per-face delays 0..3 on ragged grids (PE edges 6 to
    32, tiles of 2x2 to 32x8 columns), one RK step, and the RHS at the next step, which reads the
    level the GPU published itself."""
    say(f"case order-6 rhs n={n} p={p}")
    nlev = 7
    q = history_levels(n, nlev, sum(n) + 3 * sum(p))
    rng = np.random.default_rng(sum(n) + sum(p))
    g, o = pair(n, p, q, nlev=nlev, dt=0.01, mu=0.02)
    nt = p[0] * p[1] * p[2]
    tab = np.zeros((nlev + 2, nt, 6), dtype=np.int8)
    tab[nlev - 1] = rng.integers(0, 4, size=(nt, 6))
    tab[nlev] = rng.integers(0, 4, size=(nt, 6))
    g.set_delay_schedule(atns.EXPLICIT, table=tab)
    o.set_schedule(atns.EXPLICIT, table=tab)
    compare_fields(g.rhs().cpu().numpy(), o.rhs(), TOL64, "rhs")
    g.rk_step(1)
    o.rk_step(1)
    compare_fields(g.get_field(), o.field(), TOL64, "after 1 step")
    compare_stats(g.stats(), o.stats(), TOL64)
    compare_fields(g.rhs().cpu().numpy(), o.rhs(), TOL64, "rhs at next step")


def test_order6_caa_10_steps_fp64_and_fp32():
    """32^3 on 2x2x2 PEs, CAA c_r = 4 (L = 3), 10 RK steps: FP64 statistics after every step and the
    fields within 1e-12 of the oracle; FP32 fields within 2e-6."""
    n, p = (32, 32, 32), (2, 2, 2)
    say("case order-6 32^3 CAA L=3 10 steps")
    q = W.make_field(32, 1, 0.3)
    g, o = pair(n, p, q)
    h = atns.Sim(atns.Config(n=n, p=p, dt=W.default_dt(q), mu_ref=W.default_mu(32), max_delay=3, precision="fp32",
                             order=6))
    h.init_field(q)
    for s in (g, h):
        s.set_delay_schedule(atns.CAA, L=3, c_r=4, n_steps=12)
    o.set_schedule(atns.CAA, L=3, c_r=4, n_steps=12)
    for _ in range(10):
        g.rk_step(1)
        h.rk_step(1)
        o.rk_step(1)
        compare_stats(g.stats(), o.stats(), TOL64)
    ref = o.field()
    compare_fields(g.get_field(), ref, TOL64, "fp64 after 10 steps")
    compare_fields(h.get_field(), ref, 2e-6, "fp32 after 10 steps")


def test_order6_saa_seeded_schedule():
    """Random delays from the library's SplitMix64 draws and the oracle's own, 48^3 on 4x4x4 PEs of
    12^3, L = 2, past the L + 4 synchronous warm-up steps."""
    n, p = (48, 48, 48), (4, 4, 4)
    say("case order-6 SAA L=2 seed 102 48^3 4x4x4")
    q = W.make_field(48, 2, 0.3)
    g, o = pair(n, p, q, L=2)
    g.set_delay_schedule(atns.SAA, L=2, seed=102, n_steps=12)
    o.set_schedule(atns.SAA, L=2, seed=102, n_steps=12)
    tab = o.get_schedule(12)
    assert (tab[:6] == 0).all() and (tab[6:10] == 2).any()
    g.rk_step(10)
    o.rk_step(10)
    compare_fields(g.get_field(), o.field(), TOL64, "SAA after 10 steps")
    compare_stats(g.stats(), o.stats(), TOL64)


def test_order6_ab2_matches_oracle():
    """Adams-Bashforth steps (Sec. 2.2, Eq. time_ab) with the sixth-order scheme under CAA delays,
    interleaved with RK3 steps (each AB2 run restarts with forward Euler)."""
    n, p = (32, 24, 24), (2, 2, 2)
    say("case order-6 ab2 32x24x24")
    q = history_levels(n, 1, 99)[0]
    g, o = pair(n, p, q)
    g.set_delay_schedule(atns.CAA, L=3, c_r=4, n_steps=14)
    o.set_schedule(atns.CAA, L=3, c_r=4, n_steps=14)
    for kind, k in (("rk", 2), ("ab2", 5), ("rk", 1), ("ab2", 3)):
        for s in (g, o):
            (s.rk_step if kind == "rk" else s.ab2_step)(k)
        compare_stats(g.stats(), o.stats(), TOL64)
        compare_fields(g.get_field(), o.field(), TOL64, f"after {kind} x{k}")


def test_order6_error_paths():
    q = W.make_field(24, 1)
    with pytest.raises(atns.AtError) as e:  # PE edge below 6
        atns.Sim(atns.Config(n=(24, 24, 24), p=(6, 2, 2), dt=0.01, mu_ref=0.01, order=6))
    assert e.value.rc == atns.AT_E_INVAL
    with pytest.raises(atns.AtError) as e:  # forcing is fourth order only
        atns.Sim(atns.Config(n=(24, 24, 24), p=(2, 2, 2), dt=0.01, mu_ref=0.01, order=6, forcing=True))
    assert e.value.rc == atns.AT_E_INVAL
    s = atns.Sim(atns.Config(n=(24, 24, 24), p=(2, 2, 2), dt=0.01, mu_ref=0.01, max_delay=2, order=6, precision="fp32"))
    s.init_field(q)
    bad = np.zeros((6, 8, 6), dtype=np.int8)
    bad[4, 0, 0] = 2  # needs level 4 - 2 - 3 = -1
    with pytest.raises(atns.AtError) as e:
        s.set_delay_schedule(atns.EXPLICIT, table=bad)
    assert e.value.rc == atns.AT_E_SCHEDULE
    b = atns.Batch("fp32")
    with pytest.raises(atns.AtError) as e:  # batches are fourth order only
        b.add(s)
    assert e.value.rc == atns.AT_E_INVAL
    b.close()
