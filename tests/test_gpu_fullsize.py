"""Parity at the full benchmark size: 512^3 on 8 x 8 x 8 PEs of 64^3 in the launch shape the bench
times (the autotuner's choice), FP64, with delayed faces.  The HIP RHS is compared with the CPU
oracle's on sampled points: random points everywhere plus whole face layers, where the AT stencils
act.  The oracle evaluates the full 512^3 RHS (about 10-20 s on the host threads)."""
import sys
import time

import numpy as np
import pytest

from oracle import Oracle, OracleConfig

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2003_10561_amd import atns  # noqa: E402

N, P = 512, 8
NLEV = 4  # levels 0 .. 3; the current level is 3, so a delay of 1 reads levels 2, 1, 0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def analytic_levels(n, nlev):
    """Smooth periodic states whose phases drift with the level (a time-resolved history)."""
    x = np.arange(n) * (2 * np.pi / n)
    out = np.empty((nlev, 5, n, n, n))
    for m in range(nlev):
        s = 0.01 * m
        sx, cx = np.sin(x + s), np.cos(x + 2 * s)
        sy, cy = np.sin(x + 3 * s), np.cos(2 * x + s)
        sz, cz = np.sin(x - s), np.cos(x + 0.5 * s)
        Z, Y, X = np.ix_(np.arange(n), np.arange(n), np.arange(n))
        u = 0.3 * sy[None, :, None] * cz[:, None, None]
        v = 0.3 * sz[:, None, None] * cx[None, None, :]
        w = 0.3 * sx[None, None, :] * cy[None, :, None]
        rho = 1.0 + 0.05 * cx[None, None, :] * sy[None, :, None]
        T = 1.0 + 0.05 * sz[:, None, None] + 0.0 * X
        cv = 1.0 / 0.4
        out[m, 0] = rho
        out[m, 1] = rho * u
        out[m, 2] = rho * v
        out[m, 3] = rho * w
        out[m, 4] = rho * (cv * T + 0.5 * (u * u + v * v + w * w))
        del Z, Y, X
    return out


def test_rhs_512_fp64_with_delays_matches_oracle_on_samples():
    t0 = time.perf_counter()
    q = analytic_levels(N, NLEV)
    say(f"case 512^3 fp64 rhs: levels ready in {time.perf_counter() - t0:.1f} s")
    dt, mu = 2e-4, 1e-3
    rng = np.random.default_rng(512)
    tab = np.zeros((NLEV + 1, P ** 3, 6), dtype=np.int8)
    tab[NLEV - 1] = rng.integers(0, 2, size=(P ** 3, 6))  # k in {0, 1} at the current step
    cfg = atns.Config(n=(N,) * 3, p=(P,) * 3, dt=dt, mu_ref=mu, max_delay=1, precision="fp64")
    g = atns.Sim(cfg)
    g.init_field(q, NLEV)
    g.set_delay_schedule(atns.EXPLICIT, table=tab)
    # the launch shape the bench times: the library's autotuner through a batch of this run
    b = atns.Batch("fp64")
    b.add(g)
    b.autotune(None, reps=1)
    tile, zc = b.get_tuning()
    b.remove(g)
    b.close()
    g.set_tuning(tile, zc)
    say(f"  launch shape tile {tile} zchunk {zc}")
    rhs = g.rhs()
    torch.cuda.synchronize()
    # sample: random points, the first two and last two layers of one PE along each direction
    idx = rng.integers(0, N, size=(200_000, 3))
    layers = [0, 1, 62, 63, 64, 65]
    ii = np.arange(N)
    pts = [idx]
    for d in range(3):
        for l in layers:
            a1, a2 = np.meshgrid(ii[::7], ii[::5], indexing="ij")
            c = np.stack([np.full(a1.size, l), a1.ravel(), a2.ravel()], axis=1)
            pts.append(np.roll(c, d, axis=1))
    pts = np.concatenate(pts)
    zi, yi, xi = (torch.as_tensor(pts[:, k], device=rhs.device) for k in (2, 1, 0))
    got = rhs[:, zi, yi, xi].cpu().numpy()
    del rhs
    g.close()
    torch.cuda.empty_cache()
    say(f"  gpu done; oracle ... ({len(pts)} sampled points)")
    o = Oracle(OracleConfig(n=(N,) * 3, p=(P,) * 3, dt=dt, mu_ref=mu, max_delay=1))
    o.init_field(q, NLEV)
    del q
    o.set_schedule(atns.EXPLICIT, table=tab)
    t1 = time.perf_counter()
    ref_full = o.rhs()
    say(f"  oracle rhs in {time.perf_counter() - t1:.1f} s")
    ref = ref_full[:, pts[:, 2], pts[:, 1], pts[:, 0]]
    scale = np.sqrt(np.mean(ref_full.reshape(5, -1) ** 2, axis=1))
    del ref_full
    err = np.abs(got - ref).max(axis=1) / scale
    say("  max |err| / rms per component: " + " ".join(f"{e:.2e}" for e in err))
    assert np.isfinite(got).all()
    assert err.max() <= 1e-11
