"""The paper's own discretisation (form 1) on the GPU against the oracle, through the C ABI.

Form 1 evolves (rho, rho u_i, rho e) with the internal-energy equation (Sec. 2, Eq. ie), (2,4) AT
second derivatives and the three-step mixed derivatives (Sec. 2.1), the power law or Sutherland's
law.  FP64 bar: relative L2 <= 1e-12 per component (RHS and fields) and statistics within 1e-12;
FP32: fields within 2e-6 relative L2 after the steps (the rounding of FP32 operands, about 6e-8,
enters the second derivatives through 30 / (12 h^2) and the fields through dt times that).
"""
import sys

import numpy as np
import pytest

from oracle import Oracle, OracleConfig
from oracle.oracle import CAA, EXPLICIT, SAA
from paper_2003_10561_amd import workload as W
from tests import fields as F

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2003_10561_amd import atns  # noqa: E402

GAMMA, R = 1.4, 1.0
CV = R / (GAMMA - 1.0)
STAT_KEYS = ["mass", "momx", "energy", "mass_rk", "energy_rk", "K", "eps", "enstrophy", "Mt", "umax"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def history(n, nlev, dt, law="power", param=(19, 25)):
    """Levels of the analytic paper-form state at times (m - nlev + 1) dt, oldest first."""
    return np.ascontiguousarray(np.stack([F.analytic_paper(n, (m - (nlev - 1)) * dt, law, param)[0]
                                          for m in range(nlev)]))


def turbulent_paper_state(n, seed):
    """The seeded isotropic field of the benchmark (M_t = 0.3) in the paper's variables, with smooth
    density and temperature fluctuations (so every term of the form is exercised)."""
    q = W.make_field(n, seed, mt=0.3)
    X, Y, Z = F.grid((n,) * 3)
    rho = 1.0 + 0.03 * np.sin(X + 2 * Y) * np.cos(Z)
    T = 1.0 + 0.03 * np.cos(2 * X - Z) * np.sin(Y + 1.0)
    u, v, w = q[1] / q[0], q[2] / q[0], q[3] / q[0]
    return np.stack([rho, rho * u, rho * v, rho * w, rho * CV * T])


def pair(n, p, dt, mu, L=3, precision="fp64", visc=0, suth=0.0):
    g = atns.Sim(atns.Config(n=n, p=p, dt=dt, mu_ref=mu, max_delay=L, precision=precision, form=1,
                             visc_law=visc, sutherland_s=suth))
    o = Oracle(OracleConfig(n=n, p=p, dt=dt, mu_ref=mu, max_delay=L, form=1, visc=visc, suth_s=suth))
    return g, o


def compare_stats(gs, os_, tol):
    for k in STAT_KEYS:
        err = abs(gs[k] - os_[k]) / max(abs(os_[k]), 1e-300)
        assert err <= tol, (k, gs[k], os_[k], err)
    assert gs["step"] == os_["step"] and gs["nonfinite"] == 0


@pytest.mark.parametrize("visc,n,p,seed", [(0, (40, 20, 10), (4, 2, 2), 3), (1, (40, 20, 10), (4, 2, 2), 4),
                                            (0, (32, 48, 20), (2, 3, 2), 31), (1, (32, 48, 20), (2, 3, 2), 32),
                                            (1, (32, 16, 80), (2, 1, 8), 33)])
def test_paper_rhs_random_delays_history_levels(visc, n, p, seed):
    """RHS with six supplied levels and random delays 0..3 on every face at the current step: every
    ghost level, both viscosity laws.  A ragged grid (40 x 20 x 10 on 4 x 2 x 2 PEs of 10 x 10 x 5)
    runs the point-per-thread kernels; PEs of 16 x 16 x 10 run the LDS tiles, whose halos then
    hold the extrapolated values of delayed x and y faces; at 80 planes the tiles' second z chunk
    (64 planes each) starts inside a PE, with six z-PEs in the first."""
    nlev = 6
    say(f"case paper-form rhs {n} on {p}, visc {visc}")
    dt = 2e-3
    law, param = ("power", (19, 25)) if visc == 0 else ("sutherland", (2, 5))
    q = history(n, nlev, dt, law, param)
    g, o = pair(n, p, dt, 0.05, visc=visc, suth=0.4)
    npe = p[0] * p[1] * p[2]
    tab = np.zeros((nlev + 1, npe, 6), dtype=np.int8)
    tab[nlev - 1] = np.random.default_rng(seed).integers(0, 4, size=(npe, 6))
    for s in (g, o):
        s.init_field(q, nlev)
    g.set_delay_schedule(atns.EXPLICIT, table=tab)
    o.set_schedule(EXPLICIT, table=tab)
    got = g.rhs().cpu().numpy()
    ref = o.rhs()
    errs = [rel_l2(got[c], ref[c]) for c in range(5)]
    say("  rhs rel-L2: " + " ".join(f"{e:.2e}" for e in errs))
    assert max(errs) <= 1e-12
    g.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_paper_caa_10_steps(precision):
    n, p = (32, 32, 32), (2, 2, 2)
    say(f"case paper-form 10 CAA steps {precision}")
    q = turbulent_paper_state(32, 5)
    dt, mu = W.default_dt(q) * 0.5, W.default_mu(32)
    g, o = pair(n, p, dt, mu, precision=precision, visc=1, suth=0.4)
    for s in (g, o):
        s.init_field(q)
    g.set_delay_schedule(atns.CAA, L=3, c_r=4, n_steps=12)
    o.set_schedule(CAA, L=3, c_r=4, n_steps=12)
    g.rk_step(10)
    o.rk_step(10)
    got, ref = g.get_field(), o.field()
    errs = [rel_l2(got[c], ref[c]) for c in range(5)]
    say("  field rel-L2: " + " ".join(f"{e:.2e}" for e in errs))
    if precision == "fp64":
        assert max(errs) <= 1e-12
        compare_stats(g.stats(), o.stats(), 1e-12)
    else:
        assert max(errs) <= 2e-6
        compare_stats(g.stats(), o.stats(), 2e-5)
    g.close()


def test_paper_ab2_and_saa():
    """Adams-Bashforth steps (the paper's integrator) under SAA delays, then RK3 steps, FP64."""
    n, p = (24, 24, 24), (2, 2, 2)
    say("case paper-form AB2 + SAA")
    q = turbulent_paper_state(24, 9)
    dt, mu = W.default_dt(q) * 0.5, W.default_mu(24)
    g, o = pair(n, p, dt, mu)
    for s in (g, o):
        s.init_field(q)
    g.set_delay_schedule(atns.SAA, L=3, seed=77, n_steps=16)
    o.set_schedule(SAA, L=3, seed=77, n_steps=16)
    g.ab2_step(8)
    o.ab2_step(8)
    g.rk_step(2)
    o.rk_step(2)
    g.ab2_step(3)
    o.ab2_step(3)
    got, ref = g.get_field(), o.field()
    errs = [rel_l2(got[c], ref[c]) for c in range(5)]
    say("  field rel-L2: " + " ".join(f"{e:.2e}" for e in errs))
    assert max(errs) <= 1e-12
    compare_stats(g.stats(), o.stats(), 1e-12)
    g.close()


def test_paper_form_error_paths():
    cfg = atns.Config(n=(32,) * 3, p=(2, 2, 2), dt=1e-3, mu_ref=0.01, form=1, precision="fp32")
    g = atns.Sim(cfg)
    g.init_field(turbulent_paper_state(32, 1))
    b = atns.Batch("fp32")
    with pytest.raises(atns.AtError):
        b.add(g)
    b.close()
    with pytest.raises(atns.AtError):
        atns.Sim(atns.Config(n=(32,) * 3, p=(8, 2, 2), dt=1e-3, mu_ref=0.01, form=1))  # PE edge 4
    with pytest.raises(atns.AtError):
        g.rk_step(1)  # no schedule yet
    g.close()


@pytest.mark.slow
def test_paper_bench_pe_shape_fp32():
    """The benchmark's PE shape (64^3 PEs; here 128^3 on 2 x 2 x 2), FP32, Sutherland's law, CAA
    c_r = 4 past the ring wrap (8 steps), against the FP64 oracle: fields within 2e-6."""
    n, p = (128, 128, 128), (2, 2, 2)
    say("case paper-form 128^3 on 64^3 PEs fp32, 8 CAA steps")
    q = turbulent_paper_state(128, 13)
    dt, mu = W.default_dt(q), W.default_mu(128)
    g, o = pair(n, p, dt, mu, precision="fp32", visc=1, suth=0.4)
    for s in (g, o):
        s.init_field(q)
    g.set_delay_schedule(atns.CAA, L=3, c_r=4, n_steps=10)
    o.set_schedule(CAA, L=3, c_r=4, n_steps=10)
    g.rk_step(8)
    o.rk_step(8)
    got, ref = g.get_field(), o.field()
    errs = [rel_l2(got[c], ref[c]) for c in range(5)]
    say("  field rel-L2: " + " ".join(f"{e:.2e}" for e in errs))
    assert max(errs) <= 2e-6
    compare_stats(g.stats(), o.stats(), 2e-5)
    g.close()
