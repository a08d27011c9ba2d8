"""Served runs through the C ABI (at_serve): continuous batching returns, for every request, the
state and statistics of the same run stepped alone and, in FP64, those of the CPU oracle run on
the same inputs; admission respects the limits."""
import sys

import numpy as np
import pytest

from oracle import Oracle, OracleConfig
from paper_2003_10561_amd import workload as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2003_10561_amd import atns  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def trace(seed, count, spread_s):
    """Small requests with staggered arrivals, mixed sizes, lengths and delay modes."""
    rng = np.random.default_rng(seed)
    reqs = []
    t = 0.0
    for j in range(count):
        n = int(rng.choice([16, 24, 32]))
        p = {16: 2, 24: 3, 32: 2}[n]
        mode = int(rng.choice([atns.SYNC, atns.CAA, atns.SAA]))
        L = 0 if mode == atns.SYNC else int(rng.integers(1, 4))
        q0 = W.make_field(n, 5000 + j, 0.3)
        reqs.append(dict(arrival_s=t, n=n, p=p, steps=int(rng.integers(4, 13)), mode=mode, L=L, seed=5000 + j,
                         dt=W.default_dt(q0), mu_ref=W.default_mu(n), q0=q0,
                         q_final=np.empty_like(q0)))
        t += float(rng.exponential(spread_s / count))
    return reqs


def run_alone(r, tile, zchunk):
    cfg = atns.Config(n=(r["n"],) * 3, p=(r["p"],) * 3, dt=r["dt"], mu_ref=r["mu_ref"], max_delay=r["L"],
                      precision="fp32")
    s = atns.Sim(cfg)
    s.set_tuning(tile, zchunk)
    s.init_field(r["q0"])
    if r["mode"] == atns.CAA:
        s.set_delay_schedule(atns.CAA, L=r["L"], c_r=r["L"] + 1, n_steps=r["steps"] + 1)
    elif r["mode"] == atns.SAA:
        s.set_delay_schedule(atns.SAA, L=r["L"], seed=r["seed"], n_steps=r["steps"] + 1)
    else:
        s.set_delay_schedule(atns.SYNC, n_steps=r["steps"] + 1)
    s.rk_step(r["steps"])
    return s.get_field(), s.stats()


def test_served_equals_alone():
    """Ten requests through four slots (so some queue and join late): every final state and
    statistic equals the request run alone at the server's launch shape, bit for bit."""
    say("case serve 10 requests, 4 slots")
    reqs = trace(5, 10, 0.3)
    res, makespan = atns.serve(reqs, max_active=4, tile=1, zchunk=64)
    say(f"  makespan {makespan:.3f} s")
    for j, (r, o) in enumerate(zip(reqs, res)):
        assert o["status"] == 0, (j, o["status"])
        assert r["arrival_s"] <= o["admit_s"] + 1e-3 and o["admit_s"] <= o["done_s"] <= makespan
        f, st = run_alone(r, 1, 64)
        assert np.array_equal(r["q_final"], f), (j, np.abs(r["q_final"] - f).max())
        for k in ("mass_rk", "energy_rk", "K", "eps", "enstrophy", "step"):
            assert o["stats"][k] == st[k], (j, k)
        assert o["stats"]["step"] == r["steps"]


def test_served_fp64_matches_oracle():
    """Eight FP64 requests (16^3 - 32^3, synchronous, periodic and random delays) through three slots,
    so that runs join and leave while others are on the GPU: each final state matches the CPU FP64
    oracle run of that request within relative L2 1e-12 per component, and its statistics (including
    the RK-accumulated totals) within 1e-12."""
    say("case serve fp64 8 requests, 3 slots, vs oracle")
    reqs = trace(17, 8, 0.2)
    res, makespan = atns.serve(reqs, precision="fp64", max_active=3, tile=5, zchunk=16)
    say(f"  makespan {makespan:.3f} s")
    for j, (r, o) in enumerate(zip(reqs, res)):
        assert o["status"] == 0, (j, o["status"])
        n, p, L = r["n"], r["p"], r["L"]
        orc = Oracle(OracleConfig(n=(n,) * 3, p=(p,) * 3, dt=r["dt"], mu_ref=r["mu_ref"], max_delay=L))
        orc.init_field(r["q0"])
        if r["mode"] == atns.CAA:
            orc.set_schedule(atns.CAA, L=L, c_r=L + 1, n_steps=r["steps"] + 1)
        elif r["mode"] == atns.SAA:
            orc.set_schedule(atns.SAA, L=L, seed=r["seed"], n_steps=r["steps"] + 1)
        else:
            orc.set_schedule(atns.SYNC, n_steps=r["steps"] + 1)
        orc.rk_step(r["steps"])
        ref, ost = orc.field(), orc.stats()
        got = r["q_final"]
        errs = [float(np.linalg.norm(got[c] - ref[c]) / np.linalg.norm(ref[c])) for c in range(5)]
        say(f"  request {j}: n={n} mode={r['mode']} L={L} steps={r['steps']} rel-L2 max {max(errs):.2e}")
        assert max(errs) <= 1e-12, (j, errs)
        for k in ("mass", "energy", "mass_rk", "energy_rk", "K", "eps", "enstrophy", "Mt", "umax"):
            assert abs(o["stats"][k] - ost[k]) <= 1e-12 * abs(ost[k]), (j, k, o["stats"][k], ost[k])
        assert o["stats"]["step"] == ost["step"] == r["steps"]


def test_admission_limits():
    """A request larger than the HBM budget is refused with AT_E_WORKSPACE; the others are served."""
    reqs = trace(6, 4, 0.05)
    big = W.make_field(48, 1, 0.3)
    reqs.insert(2, dict(arrival_s=reqs[1]["arrival_s"], n=48, p=3, steps=3, mode=atns.SYNC, L=0, seed=0,
                        dt=W.default_dt(big), mu_ref=W.default_mu(48), q0=big, q_final=None))
    budget = 0
    for r in reqs:
        if r["n"] < 48:
            cfg = atns.Config(n=(r["n"],) * 3, p=(r["p"],) * 3, dt=r["dt"], mu_ref=r["mu_ref"], max_delay=r["L"],
                              precision="fp32")
            budget = max(budget, 3 * atns.workspace_bytes(cfg))
    res, _ = atns.serve(reqs, max_active=2, hbm_budget_bytes=budget)
    assert res[2]["status"] == atns.AT_E_WORKSPACE
    assert all(o["status"] == 0 for j, o in enumerate(res) if j != 2)


def test_empty_trace():
    res, makespan = atns.serve([], max_active=4)
    assert res == [] and makespan >= 0.0
