"""Batched runs through the C ABI (at_batch_*): bitwise equality with the same runs stepped alone,
graph replays against eager launches, launch-shape independence of the fields, the autotuner, and
one FP64 batch against the CPU oracle."""
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


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# (n, p, delay mode, L, forced): mixed grids, PE shapes and schedules, ragged blocks
RUNS = [
    ((32, 32, 32), (2, 2, 2), atns.CAA, 3, False),
    ((24, 40, 16), (2, 4, 2), atns.SAA, 2, False),
    ((48, 48, 48), (3, 3, 3), atns.SAA, 3, True),
    ((16, 16, 16), (1, 1, 1), atns.SYNC, 0, False),
    ((36, 20, 28), (3, 1, 7), atns.CAA, 1, True),
]
STEPS = 24


def smooth_state(n, seed):
    """A periodic state on any grid: low-mode shear waves with random phases, density and
    temperature waves, and a small random perturbation."""
    rng = np.random.default_rng(seed)
    X, Y, Z = F.grid(n)
    ph = rng.uniform(0.0, 2 * np.pi, 8)
    noise = 1e-3 * rng.standard_normal((3,) + X.shape)
    u = 0.3 * np.sin(Y + ph[0]) * np.cos(2 * Z + ph[1]) + noise[0]
    v = 0.3 * np.sin(Z + ph[2]) * np.cos(X + ph[3]) + noise[1]
    w = 0.3 * np.sin(X + ph[4]) * np.cos(Y + ph[5]) + noise[2]
    rho = 1.0 + 0.05 * np.cos(X + Y + ph[6])
    T = 1.0 + 0.05 * np.sin(Z + ph[7])
    return np.ascontiguousarray(F.conservative(rho, u, v, w, T))


def make_run(i, spec, precision, tuning=None):
    n, p, mode, L, forced = spec
    q = smooth_state(n, 100 + i)
    dt = 0.5 * W.default_dt(q)
    mu = W.default_mu(max(n))
    cfg = atns.Config(n=n, p=p, dt=dt, mu_ref=mu, max_delay=max(L, 1), precision=precision, forcing=forced)
    s = atns.Sim(cfg)
    if tuning is not None:
        s.set_tuning(*tuning)
    s.init_field(q)
    if mode == atns.CAA:
        s.set_delay_schedule(atns.CAA, L=L, c_r=L + 1, n_steps=STEPS + 1)
    elif mode == atns.SAA:
        s.set_delay_schedule(atns.SAA, L=L, seed=700 + i, n_steps=STEPS + 1)
    else:
        s.set_delay_schedule(atns.SYNC, n_steps=STEPS + 1)
    fh = None
    if forced:
        fh = W.make_forcing(900 + i, STEPS + 1, dt, 1.0, 0.1 * W.urms_of(q))
        s.set_forcing(fh)
    return s, q, cfg, fh


def assert_same(a, b, what):
    fa, fb = a.get_field(), b.get_field()
    assert np.array_equal(fa, fb), f"{what}: max |diff| {np.abs(fa - fb).max()}"
    sa, sb = a.stats(), b.stats()
    for k in ("mass_rk", "momx_rk", "energy_rk", "K", "eps", "enstrophy"):
        assert sa[k] == sb[k], (what, k, sa[k], sb[k])
    assert sa["step"] == sb["step"]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batched_equals_solo_bitwise(precision):
    """Five mixed runs, one joining two steps late: after chunks of 3, 4 and 4 steps each member
    equals the same run stepped alone (same launch shape) bit for bit, fields and statistics."""
    say(f"case batch vs solo {precision}")
    b = atns.Batch(precision)
    tile, zc = b.get_tuning()
    batched = [make_run(i, r, precision)[0] for i, r in enumerate(RUNS)]
    solo = [make_run(i, r, precision, (tile, zc))[0] for i, r in enumerate(RUNS)]
    for s in batched[:-1]:
        b.add(s)
    b.step(2)
    for s in solo[:-1]:
        s.rk_step(2)
    b.add(batched[-1])  # joins at its step 0 while the others are at step 2
    for chunk in (3, 4, 4):
        b.step(chunk)
        for s in solo:
            s.rk_step(chunk)
        for i, (x, y) in enumerate(zip(batched, solo)):
            assert_same(x, y, f"run {i} after chunk {chunk}")
    caps, reps = b.graph_stats()
    say(f"  graph captures {caps} replays {reps}")
    assert reps == 4 and caps >= 2


def test_graph_replays_match_eager_launches():
    """The same batch stepped through graph replays and through direct launches, with eager work
    (statistics, a solo RHS) between replays: identical after every chunk."""
    say("case graph vs eager")
    g_b, e_b = atns.Batch("fp32"), atns.Batch("fp32")
    e_b.set_graph(False)
    gr = [make_run(i, r, "fp32")[0] for i, r in enumerate(RUNS[:3])]
    er = [make_run(i, r, "fp32")[0] for i, r in enumerate(RUNS[:3])]
    for s in gr:
        g_b.add(s)
    for s in er:
        e_b.add(s)
    for it in range(5):
        g_b.step(4)
        e_b.step(4)
        for i, (x, y) in enumerate(zip(gr, er)):
            assert_same(x, y, f"replay {it} run {i}")
        gr[0].rhs()  # eager work on the same stream between replays
    caps, reps = g_b.graph_stats()
    say(f"  captures {caps} replays {reps}")
    assert reps == 5 and caps < reps


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_launch_shape_does_not_change_fields(precision):
    """Every feasible tile shape and several z chunks give bitwise identical fields; the FP64 RK
    totals differ only by the order of their per-workgroup partial sums."""
    say(f"case tiles {precision}")
    spec = RUNS[2]
    ref = None
    for tile in range(atns.N_TILES):
        for zc in (4, 16, 64):
            s = make_run(2, spec, precision)[0]
            try:
                s.set_tuning(tile, zc)
            except atns.AtError:
                continue  # shape does not fit the LDS at this precision
            s.rk_step(9)
            f, st = s.get_field(), s.stats()
            if ref is None:
                ref = (f, st)
                continue
            assert np.array_equal(f, ref[0]), (tile, zc, np.abs(f - ref[0]).max())
            assert st["mass_rk"] == pytest.approx(ref[1]["mass_rk"], rel=1e-13)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_separate_stage_shapes(precision):
    """Synchronous and delayed stages in different launch shapes: a batch equals its members
    stepped alone with the same two shapes bit for bit (fields and statistics), and the fields
    equal those of a single shape for every stage."""
    say(f"case stage shapes {precision}")
    shapes = (3, 16, 5, 8) if precision == "fp64" else (0, 16, 5, 8)  # z chunks within every grid
    b = atns.Batch(precision)
    b.set_stage_tuning(*shapes)
    assert b.get_stage_tuning() == shapes
    assert b.get_tuning() == shapes[:2]
    batched = [make_run(i, r, precision)[0] for i, r in enumerate(RUNS[:3])]
    solo = [make_run(i, r, precision)[0] for i, r in enumerate(RUNS[:3])]
    single = [make_run(i, r, precision, (5, 64))[0] for i, r in enumerate(RUNS[:3])]
    for s in solo:
        s.set_stage_tuning(*shapes)
        assert s.get_stage_tuning() == shapes
    for s in batched:
        b.add(s)
    for chunk in (3, 5):
        b.step(chunk)
        for s in solo + single:
            s.rk_step(chunk)
        for i in range(3):
            assert_same(batched[i], solo[i], f"run {i} after chunk {chunk}")
            assert np.array_equal(batched[i].get_field(), single[i].get_field()), i
    b.close()


def test_autotune_keeps_state_and_uses_cache(tmp_path):
    say("case autotune")
    cache = tmp_path / "tune.jsonl"
    b = atns.Batch("fp32")
    runs = [make_run(i, r, "fp32")[0] for i, r in enumerate(RUNS)]
    for s in runs:
        b.add(s)
    ms = b.autotune(cache, reps=2)  # at step 0, like the second batch below (same cache key)
    tile, zc = b.get_tuning()
    shapes = b.get_stage_tuning()
    say(f"  chose shapes {shapes}: {ms:.3f} ms per stage")
    assert ms > 0 and cache.exists() and cache.read_text().count("\n") == 1
    b.step(3)
    b.autotune(None, reps=1)  # trial stages between steps leave every member's state untouched
    b.set_tuning(tile, zc)
    b.step(5)
    solo = [make_run(i, r, "fp32", (tile, zc))[0] for i, r in enumerate(RUNS)]
    for s in solo:
        s.rk_step(8)
    for i, (x, y) in enumerate(zip(runs, solo)):
        assert np.array_equal(x.get_field(), y.get_field()), i
    # a second batch of the same shapes takes the cached choice without timing
    b2 = atns.Batch("fp32")
    for i, r in enumerate(RUNS):
        b2.add(make_run(i, r, "fp32")[0])
    b2.set_tuning(5, 8)
    assert b2.autotune(cache, reps=2) == pytest.approx(ms)
    assert b2.get_tuning() == (tile, zc)
    assert b2.get_stage_tuning() == shapes
    assert cache.read_text().count("\n") == 1


def test_autotune_keeps_adams_bashforth_register():
    """Adams-Bashforth steps keep dt f^{n-1} in the RK register (Sec. 2.2, Eq. time_ab).  Autotuning
    a batch that holds such a run (trial stages between steps) must leave that register alone, so
    that the run's next Adams-Bashforth step is still second order: FP64 fields and statistics of
    ab2 x3 -> add to a batch -> autotune -> remove -> ab2 x3 match the oracle's six AB2 steps."""
    say("case ab2 register kept by the autotuner")
    n, p = (32, 32, 32), (2, 2, 2)
    q = smooth_state(n, 31)
    dt, mu = 0.5 * W.default_dt(q), W.default_mu(32)
    s = atns.Sim(atns.Config(n=n, p=p, dt=dt, mu_ref=mu, max_delay=3, precision="fp64"))
    s.init_field(q)
    s.set_delay_schedule(atns.CAA, L=3, c_r=4, n_steps=10)
    o = Oracle(OracleConfig(n=n, p=p, dt=dt, mu_ref=mu, max_delay=3))
    o.init_field(q)
    o.set_schedule(atns.CAA, L=3, c_r=4, n_steps=10)
    s.ab2_step(3)
    b = atns.Batch("fp64")
    b.add(s)
    b.autotune(None, reps=1)
    b.remove(s)
    b.close()
    s.ab2_step(3)
    o.ab2_step(6)
    ref = o.field()
    got = s.get_field()
    errs = [float(np.linalg.norm(got[c] - ref[c]) / np.linalg.norm(ref[c])) for c in range(5)]
    say("  rel-L2 per component: " + " ".join(f"{e:.2e}" for e in errs))
    assert max(errs) <= 1e-12, errs
    gs, os_ = s.stats(), o.stats()
    for k in ("mass_rk", "energy_rk", "K", "eps", "enstrophy"):
        assert abs(gs[k] - os_[k]) <= 1e-12 * abs(os_[k]), k
    s.close()


def test_fp64_batch_matches_oracle():
    """The parity chain's last link for batches: an FP64 batch against the CPU oracle."""
    say("case fp64 batch vs oracle")
    b = atns.Batch("fp64")
    members = []
    for i in (0, 2, 4):
        s, q, cfg, fh = make_run(i, RUNS[i], "fp64")
        b.add(s)
        o = Oracle(OracleConfig(n=cfg.n, p=cfg.p, dt=cfg.dt, mu_ref=cfg.mu_ref, max_delay=cfg.max_delay,
                                forcing=cfg.forcing))
        o.init_field(q)
        sa, skw = schedule_args(i)
        o.set_schedule(*sa, **skw)
        if fh is not None:
            o.set_forcing(fh)
        members.append((s, o))
    b.step(7)
    for i, (s, o) in enumerate(members):
        o.rk_step(7)
        ref = o.field()
        got = s.get_field()
        err = max(np.linalg.norm(got[c] - ref[c]) / np.linalg.norm(ref[c]) for c in range(5))
        say(f"  member {i}: max rel-L2 {err:.2e}")
        assert err <= 1e-12


def schedule_args(i):
    n, p, mode, L, forced = RUNS[i]
    if mode == atns.CAA:
        return (atns.CAA,), {"L": L, "c_r": L + 1, "n_steps": STEPS + 1}
    if mode == atns.SAA:
        return (atns.SAA,), {"L": L, "seed": 700 + i, "n_steps": STEPS + 1}
    return (atns.SYNC,), {"n_steps": STEPS + 1}


def test_batch_error_paths():
    b = atns.Batch("fp32")
    s64 = make_run(0, RUNS[0], "fp64")[0]
    with pytest.raises(atns.AtError) as e:
        b.add(s64)
    assert e.value.rc == atns.AT_E_INVAL
    s = make_run(0, RUNS[0], "fp32")[0]
    b.add(s)
    with pytest.raises(atns.AtError) as e:
        b.add(s)
    assert e.value.rc == atns.AT_E_STATE
    with pytest.raises(atns.AtError) as e:
        b.step(STEPS + 5)  # beyond the member's schedule
    assert e.value.rc == atns.AT_E_SCHEDULE
    b.remove(s)
    assert len(b) == 0
    s.rk_step(1)  # still usable alone


def test_empty_and_zero_step_edge_cases():
    """Zero steps change nothing; an empty batch steps and tunes as a no-op / clear error."""
    s = make_run(0, RUNS[0], "fp32")[0]
    f0 = s.get_field()
    s.rk_step(0)
    assert np.array_equal(s.get_field(), f0) and s.stats()["step"] == 0
    b = atns.Batch("fp32")
    b.step(3)  # no members: nothing to do
    with pytest.raises(atns.AtError) as e:
        b.autotune(None, reps=1)
    assert e.value.rc == atns.AT_E_STATE
    b.add(s)
    b.step(0)
    assert np.array_equal(s.get_field(), f0)
