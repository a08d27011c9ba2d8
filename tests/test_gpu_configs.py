"""Parity of whole configurations against the CPU FP64 oracle, through the C ABI.

* The headline path's exact shape at 256^3: FP32 fields, the 64x8 workgroup tile with one z chunk
  per column (the shape the 512^3 bench runs), OU forcing, periodic (CAA) delays with c_r = 4 on
  4x4x4 PEs of 64^3, nine steps, so that delays 1, 2, 3 (and both later RK stages' extrapolation
  times) and the wrap of the six-slot ring are all reached.
* The decaying-turbulence configuration: FP64, 256^3 on 4x4x4 PEs, random (SAA) delays uniform in
  {0, 1, 2} from seed 102, past the five synchronous warm-up steps, statistics after every step.

FP64 bar: relative L2 <= 1e-12 per conserved component and per statistic.  FP32 bound: 2e-6 per
component (the FP32 state carries ~6e-8 relative rounding per operation; the steps amplify it
mildly; the 32^3 test of the same bound observes ~1e-7), statistics 1e-5.
"""
import sys
import time

import numpy as np
import pytest

from oracle import Oracle, OracleConfig
from paper_2003_10561_amd import workload as W

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2003_10561_amd import atns  # noqa: E402

STATS = ["mass", "energy", "mass_rk", "energy_rk", "K", "eps", "enstrophy", "Mt", "umax"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def check_fields(got, ref, tol, what):
    errs = [rel_l2(got[c], ref[c]) for c in range(5)]
    say(f"  {what}: rel-L2 per component " + " ".join(f"{e:.2e}" for e in errs))
    assert max(errs) <= tol, errs
    return errs


def check_stats(gs, os_, tol, keys=STATS):
    for k in keys:
        err = abs(gs[k] - os_[k]) / max(abs(os_[k]), 1e-300)
        assert err <= tol, (k, gs[k], os_[k], err)
    assert gs["step"] == os_["step"] and gs["nonfinite"] == 0


def test_headline_shape_fp32_256_forced_caa():
    n, pe, steps = 256, 4, 9
    say(f"case headline shape: {n}^3 fp32 on {pe}^3 PEs, tile 64x8, z chunk {n}, forced, CAA c_r=4, {steps} steps")
    t0 = time.perf_counter()
    q = W.make_field(n, 3, 0.3)
    dt, mu = W.default_dt(q), W.default_mu(n)
    fh = W.make_forcing(303, steps + 1, dt, 1.0, 0.1 * W.urms_of(q))
    g = atns.Sim(atns.Config(n=(n,) * 3, p=(pe,) * 3, dt=dt, mu_ref=mu, max_delay=3, precision="fp32",
                             forcing=True))
    g.set_stage_tuning(0, n, 0, n)  # 64x8 columns, one z chunk per column, both stage kinds
    g.init_field(q)
    g.set_delay_schedule(atns.CAA, L=3, c_r=4, n_steps=steps + 1)
    g.set_forcing(fh)
    g.rk_step(steps)
    got, gs = g.get_field(), g.stats()
    g.close()
    torch.cuda.empty_cache()
    say(f"  gpu done in {time.perf_counter() - t0:.1f} s; oracle ...")
    o = Oracle(OracleConfig(n=(n,) * 3, p=(pe,) * 3, dt=dt, mu_ref=mu, max_delay=3, forcing=True))
    o.init_field(q)
    o.set_schedule(atns.CAA, L=3, c_r=4, n_steps=steps + 1)
    o.set_forcing(fh)
    for s in range(steps):
        o.rk_step(1)
        say(f"  oracle step {s + 1}/{steps}")
    errs = check_fields(got, o.field(), 2e-6, f"fp32 after {steps} steps")
    check_stats(gs, o.stats(), 1e-5, ["mass", "energy", "K", "eps", "enstrophy", "Mt", "umax"])
    say(f"  fp32 max rel-L2 {max(errs):.3e}")


def test_decaying_fp64_256_saa_stats_every_step():
    n, pe, L, steps = 256, 4, 2, 9
    say(f"case decaying: {n}^3 fp64 on {pe}^3 PEs, SAA L={L} seed 102, {steps} steps, stats every step")
    q = W.make_field(n, 2, 0.3)
    dt, mu = W.default_dt(q), W.default_mu(n)
    g = atns.Sim(atns.Config(n=(n,) * 3, p=(pe,) * 3, dt=dt, mu_ref=mu, max_delay=L, precision="fp64"))
    g.init_field(q)
    g.set_delay_schedule(atns.SAA, L=L, seed=102, n_steps=steps + 1)
    o = Oracle(OracleConfig(n=(n,) * 3, p=(pe,) * 3, dt=dt, mu_ref=mu, max_delay=L))
    o.init_field(q)
    o.set_schedule(atns.SAA, L=L, seed=102, n_steps=steps + 1)
    tab = o.get_schedule(steps + 1)
    assert (tab[:L + 3] == 0).all() and (tab[L + 3:steps] > 0).any() and (tab[L + 3:steps] == L).any()
    for s in range(steps):
        g.rk_step(1)
        o.rk_step(1)
        check_stats(g.stats(), o.stats(), 1e-12)
        say(f"  step {s + 1}: statistics match")
    check_fields(g.get_field(), o.field(), 1e-12, f"fp64 after {steps} steps")
    g.close()
    torch.cuda.empty_cache()


def test_order6_bench_pe_shape_fp64_fp32_caa():
    """The sixth-order scheme in the PE shape of the 512^3 benchmark leg: 128^3 on 2x2x2 PEs of 64^3
    (32x8-column tiles), unforced, CAA c_r = 4, eight steps (delays 1, 2, 3 reached, the seven-slot
    ring wrapping): FP64 fields and statistics within 1e-12 of the oracle, FP32 fields within 2e-6."""
    n, pe, steps = 128, 2, 8
    say(f"case order-6 {n}^3 on {pe}^3 PEs of 64^3, CAA c_r=4, {steps} steps, fp64 and fp32")
    q = W.make_field(n, 3, 0.3)
    dt, mu = W.default_dt(q), W.default_mu(n)
    got = {}
    for prec in ("fp64", "fp32"):
        g = atns.Sim(atns.Config(n=(n,) * 3, p=(pe,) * 3, dt=dt, mu_ref=mu, max_delay=3, precision=prec, order=6))
        g.init_field(q)
        g.set_delay_schedule(atns.CAA, L=3, c_r=4, n_steps=steps + 1)
        g.rk_step(steps)
        got[prec] = (g.get_field(), g.stats())
        g.close()
    o = Oracle(OracleConfig(n=(n,) * 3, p=(pe,) * 3, dt=dt, mu_ref=mu, max_delay=3, order=6))
    o.init_field(q)
    o.set_schedule(atns.CAA, L=3, c_r=4, n_steps=steps + 1)
    for s in range(steps):
        o.rk_step(1)
        say(f"  oracle step {s + 1}/{steps}")
    ref = o.field()
    check_fields(got["fp64"][0], ref, 1e-12, f"fp64 after {steps} steps")
    check_stats(got["fp64"][1], o.stats(), 1e-12)
    check_fields(got["fp32"][0], ref, 2e-6, f"fp32 after {steps} steps")
