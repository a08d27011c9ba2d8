#!/usr/bin/env python3
"""Benchmark of the AT compressible-NS step on one MI355X.

Workload (the configuration the headline metric is quoted on): forced decaying-to-stationary
turbulence at 512^3 on [0, 2pi)^3, 8 x 8 x 8 virtual PEs of 64^3, periodic (CAA) delays with
c_r = 4 (L = 3), solenoidal OU forcing on |k| <= 2.5, FP32 fields with FP64 reductions.  A step is
one full low-storage RK3 step (3 stages) over the whole grid; inputs are resident in HBM before
the timed region.  Prints ONE JSON line (rank 0) with the throughput, the roofline of the
dominant kernel measured with HIP events on the launch stream, the same workload in FP64, and the
CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import os

os.environ.setdefault("NUMPY_MADVISE_HUGEPAGE", "0")

import argparse  # noqa: E402
import json  # noqa: E402
import math  # noqa: E402
import re  # noqa: E402
import sys  # noqa: E402
import time  # noqa: E402

import numpy as np  # noqa: E402

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "grid-pt-steps/s + HBM GB/s at 512³ FP32 vs FP64; served p50/p99 latency"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--pe", type=int, default=8, help="virtual PEs per direction")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 run of the same workload")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-n", type=int, default=128)
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--no-cfg2", action="store_true", help="skip the decaying 256^3 FP64 configuration")
    ap.add_argument("--no-order6", action="store_true", help="skip the sixth-order scheme")
    ap.add_argument("--no-diag", action="store_true", help="skip the turbulence diagnostics of the final state")
    ap.add_argument("--no-paper", action="store_true", help="skip the paper's own discretisation (form 1)")
    ap.add_argument("--no-paper-ab2", action="store_true", help="the paper's form: RK3 steps only (profiling)")
    ap.add_argument("--cfg2-steps", type=int, default=100)
    ap.add_argument("--tile", type=int, default=None, help="fused-stage tile shape (default: library)")
    ap.add_argument("--zchunk", type=int, default=None)
    ap.add_argument("--no-autotune", action="store_true", help="library default launch shape for the 512^3 runs")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 64-run workload")
    ap.add_argument("--batch-steps", type=int, default=20)
    ap.add_argument("--no-serve", action="store_true", help="skip the served request trace")
    ap.add_argument("--no-ab2", action="store_true", help="skip the Adams-Bashforth steps after the timed RK3 steps")
    ap.add_argument("--serve-seconds", type=float, default=100.0, help="length of the Poisson arrival window")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file (JSON lines)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration) and exit")
    return ap.parse_args()


def build_sim(atns, W, n, pe, precision, n_steps_total, q, dt, mu, fh, tile=None, zchunk=None, autotune=True):
    cfg = atns.Config(n=(n, n, n), p=(pe, pe, pe), dt=dt, mu_ref=mu, max_delay=3,
                      precision=precision, forcing=True)
    sim = atns.Sim(cfg)
    sim.init_field(q)
    sim.set_delay_schedule(atns.CAA, L=3, c_r=4, n_steps=n_steps_total)
    sim.set_forcing(fh)
    tuned = False
    if tile is not None or zchunk is not None:
        t0, z0 = sim.get_tuning()
        sim.set_tuning(t0 if tile is None else tile, z0 if zchunk is None else zchunk)
    elif autotune:
        # the library's autotuner, through a batch of this one run (trial stages leave the state)
        b = atns.Batch(precision)
        b.add(sim)
        b.autotune(None, reps=2)
        shapes = b.get_stage_tuning()  # synchronous and delayed stages
        b.remove(sim)
        b.close()
        sim.set_stage_tuning(*shapes)
        tuned = True
    return sim, tuned


def time_window(torch, sim, steps, warmup=0):
    """`warmup` untimed steps, then `steps` RK3 steps between two HIP events on the launch stream
    (torch's current stream, which the library enqueues on); no per-kernel events inside."""
    if warmup:
        sim.rk_step(warmup)
    stream = torch.cuda.current_stream()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    sim.rk_step(steps)
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1)


def kernel_window(torch, sim, steps, step_fn=None):
    """The next `steps` steps with every kernel bracketed by HIP events on the launch stream: the
    per-kernel durations the roofline divides by.  Returns (window ms, {kernel: (ms, launches)})."""
    sim.set_kernel_timing(True)
    stream = torch.cuda.current_stream()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    (step_fn or sim.rk_step)(steps)
    t1.record(stream)
    torch.cuda.synchronize()
    kt = sim.kernel_timing()
    sim.set_kernel_timing(False)
    return t0.elapsed_time(t1), kt


STAGE_KERNELS = ("k_stage", "k_at_sums")


def roofline(kt, n, pe, word, pd, steps, kernels=STAGE_KERNELS, order=4):
    """Dominant launch = one RK stage: the fused stage kernel plus, at delayed steps, the AT sums it
    reads (the method's delayed-level reads); for the sixth-order scheme the gradient / flux and the
    divergence / update launches of a stage.  Algorithmic bytes per stage launch (the minimal count
    of traffic.words_per_point_step, a third of a step's) over the average event-timed duration of
    those kernels per stage."""
    from paper_2003_10561_amd import traffic
    stage_kernels = [k for k in kt if k in kernels]
    launches = steps * 3
    stage_ms = sum(kt[k][0] for k in stage_kernels) / launches
    words = traffic.words_per_point_step((n,) * 3, (pe,) * 3, pd, order) / 3.0
    bytes_per_launch = words * word * n ** 3
    achieved = bytes_per_launch / (stage_ms * 1e-3) / 1e9
    name = "+".join(stage_kernels)
    loose = (traffic.words_per_point_step_stage_reads((n,) * 3, (pe,) * 3, pd) * word if order == 4
             else words * 3 * word)
    return {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "bytes_per_launch": bytes_per_launch, "avg_launch_ms": stage_ms,
            "algorithmic_bytes_per_point_step": words * 3 * word,
            "bytes_per_point_step_stage_reads": loose,
            "frac_stage_reads": loose / 3.0 * n ** 3 / (stage_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}


def stage_source_sha(source="stage_fused.hip"):
    import hashlib
    src = os.path.join(ROOT, "paper_2003_10561_amd", "csrc", source)
    with open(src, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(name, source="stage_fused.hip"):
    """HBM bytes per stage from the committed counter summary profiles/<name>_traffic.md, if it was
    taken on the current source of the kernels it covers; otherwise None."""
    path = os.path.join(ROOT, "profiles", f"{name}_traffic.md")
    # written by paper_2003_10561_amd/profsum.py from FETCH_SIZE / WRITE_SIZE runs of this bench
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            m = re.match(r"^- (\w+): (\S+)\s*$", line)
            if m:
                kv[m.group(1)] = m.group(2)
    if kv.get("source_sha256") != stage_source_sha(source) or "bytes_per_launch" not in kv:
        return None
    return float(kv["bytes_per_launch"])


def calib_copy(torch, mib):
    """A plain device copy of known size: the reference the HBM counters are scaled by."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes_each_way": n * 4, "launches": 3}), flush=True)


def batch_specs(seed0=1000):
    """64 runs: 16 each of N = 32, 64, 96, 128 (PE tiles 16^3 at N = 32, else 32^3), M_t ~ U[0.1, 0.5],
    mu_ref = default(N) x logU[0.5, 2], delays CAA or SAA with equal odds, L ~ U{1, 2, 3}; run i seeded
    with seed0 + i."""
    specs = []
    for i in range(64):
        rng = np.random.default_rng(seed0 + i)
        n = (32, 64, 96, 128)[i // 16]
        specs.append(dict(n=n, p=2 if n == 32 else n // 32, mt=float(rng.uniform(0.1, 0.5)),
                          mu_scale=float(np.exp(rng.uniform(np.log(0.5), np.log(2.0)))),
                          mode="caa" if rng.random() < 0.5 else "saa", L=int(rng.integers(1, 4)),
                          seed=seed0 + i))
    return specs


def _run_delayed_fraction(sp, first, steps):
    """Delayed fraction of a batched run's (step, face) pairs over steps [first, first + steps): exact
    for periodic delays (every face at n mod c_r after c_r warm-up steps), the expectation L / (L + 1)
    after the L + 3 warm-up steps for random ones."""
    L = sp["L"]
    rng = range(first, first + steps)
    if sp["mode"] == "caa":
        return sum(1 for n in rng if n >= L + 1 and n % (L + 1) != 0) / steps
    return sum(L / (L + 1) for n in rng if n >= L + 3) / steps


def batched_workload(torch, atns, W, steps, warmup, cache):
    specs = batch_specs()
    sims = []
    # the warm-up chunk has the timed chunk's length, so that the timed chunk replays its graph
    warmup = steps
    total = warmup + steps + 1
    for sp in specs:
        n = sp["n"]
        q = W.make_field(n, sp["seed"], sp["mt"])
        cfg = atns.Config(n=(n,) * 3, p=(sp["p"],) * 3, dt=W.default_dt(q), mu_ref=W.default_mu(n) * sp["mu_scale"],
                          max_delay=sp["L"], precision="fp32")
        s = atns.Sim(cfg)
        s.init_field(q)
        if sp["mode"] == "caa":
            s.set_delay_schedule(atns.CAA, L=sp["L"], c_r=sp["L"] + 1, n_steps=total)
        else:
            s.set_delay_schedule(atns.SAA, L=sp["L"], seed=sp["seed"], n_steps=total)
        sims.append(s)
    b = atns.Batch("fp32")
    for s in sims:
        b.add(s)
    tune_ms = b.autotune(cache, reps=3)
    tile, zc, tile_d, zc_d = b.get_stage_tuning()
    b.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    b.step(steps)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    pts = sum(sp["n"] ** 3 for sp in specs)
    from paper_2003_10561_amd import traffic
    step_bytes = sum(4 * sp["n"] ** 3 * traffic.words_per_point_step((sp["n"],) * 3, (sp["p"],) * 3,
                                                                     _run_delayed_fraction(sp, warmup, steps))
                     for sp in specs)
    gbs = step_bytes / (ms / steps * 1e-3) / 1e9
    caps, reps = b.graph_stats()
    nonfinite = sum(s.stats()["nonfinite"] for s in sims)
    b.close()
    del sims
    torch.cuda.empty_cache()
    ref = same_pe_single_run(torch, atns, W)
    return {"value": pts * steps / (ms * 1e-3), "unit": "grid-pt-steps/s", "runs": len(specs), "points": pts,
            "same_pe_single_run": ref, "batched_over_same_pe_single": pts * steps / (ms * 1e-3) / ref["value"],
            "steps": steps, "warmup": warmup, "ms_per_step": ms / steps, "tile": tile, "zchunk": zc,
            "tile_delayed": tile_d, "zchunk_delayed": zc_d,
            "autotune_stage_ms": tune_ms, "graph_captures": caps, "graph_replays": reps,
            "roofline": {"bound": "hbm", "kernel": "batched step (all launches)", "achieved": gbs,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                         "algorithmic_bytes_per_step": step_bytes},
            "nonfinite_runs": int(nonfinite),
            "workload": "64 runs (16 each of 32^3, 64^3, 96^3, 128^3), CAA/SAA L in 1..3, FP32, one batched "
                        "launch per kernel per RK stage from a HIP graph"}


def same_pe_single_run(torch, atns, W, n=256, pe=8, steps=10, warmup=3):
    """The per-point reference for the batched and served workloads, whose members run on PEs of 32^3
    (16^3 at N = 32): one unforced FP32 run of 256^3 on 8x8x8 PEs of 32^3, CAA L=3 c_r=4, autotuned
    launch shapes (the 512^3 headline runs on PEs of 64^3, with half the face work per point)."""
    q = W.make_field(n, 77, 0.3)
    cfg = atns.Config(n=(n,) * 3, p=(pe,) * 3, dt=W.default_dt(q), mu_ref=W.default_mu(n), max_delay=3,
                      precision="fp32")
    sim = atns.Sim(cfg)
    sim.init_field(q)
    sim.set_delay_schedule(atns.CAA, L=3, c_r=4, n_steps=warmup + steps + 8)
    b = atns.Batch("fp32")
    b.add(sim)
    b.autotune(None, reps=2)
    shapes = b.get_stage_tuning()
    b.remove(sim)
    b.close()
    sim.set_stage_tuning(*shapes)
    ms = time_window(torch, sim, steps, warmup=warmup)
    sim.close()
    torch.cuda.empty_cache()
    return {"value": n ** 3 * steps / (ms * 1e-3), "ms_per_step": ms / steps, "launch": list(shapes),
            "workload": f"one run of {n}^3 on {pe}x{pe}x{pe} PEs of {n // pe}^3, CAA L=3 c_r=4, unforced, FP32"}


def served_workload(atns, W, seconds, seed=5, tile=-1, zchunk=64, tile_delayed=-1, zchunk_delayed=64):
    """Poisson arrivals at 20/s for `seconds`; N = 32 round(exp(U(ln 32, ln 256)) / 32); steps ~ U{20..200};
    delays as in the batched workload; request j seeded with 5000 + j.  Initial fields come from a pool of
    two seeded fields per size (building one per request on the host would dominate the latency)."""
    rng = np.random.default_rng(seed)
    t, reqs = 0.0, []
    pool = {}
    while True:
        t += float(rng.exponential(1.0 / 20.0))
        if t > seconds:
            break
        j = len(reqs)
        n = int(32 * round(float(np.exp(rng.uniform(np.log(32), np.log(256)))) / 32))
        n = max(32, n)
        key = (n, j % 2)
        if key not in pool:
            q = W.make_field(n, 5000 + 10 * n + key[1], 0.3)
            pool[key] = (q, W.default_dt(q))
        q, dt = pool[key]
        mode = atns.CAA if rng.random() < 0.5 else atns.SAA
        L = int(rng.integers(1, 4))
        reqs.append(dict(arrival_s=t, n=n, p=2 if n == 32 else n // 32, steps=int(rng.integers(20, 201)),
                         mode=mode, L=L, seed=5000 + j, dt=dt, mu_ref=W.default_mu(n), q0=q))
    res, makespan = atns.serve(reqs, precision="fp32", max_active=64, hbm_budget_bytes=200e9, tile=tile,
                               zchunk=zchunk, tile_delayed=tile_delayed, zchunk_delayed=zchunk_delayed)
    ok = [o for o in res if o["status"] == 0]
    lat = np.array([o["done_s"] - r["arrival_s"] for r, o in zip(reqs, res) if o["status"] == 0])
    queue = np.array([o["admit_s"] - r["arrival_s"] for r, o in zip(reqs, res) if o["status"] == 0])
    service = np.array([o["done_s"] - o["admit_s"] for o in res if o["status"] == 0])
    work = sum(r["n"] ** 3 * r["steps"] for r, o in zip(reqs, res) if o["status"] == 0)
    offered = sum(r["n"] ** 3 * r["steps"] for r in reqs) / seconds
    return {"requests": len(reqs), "served": len(ok), "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)), "throughput": work / makespan,
            "p50_queue_s": float(np.percentile(queue, 50)), "p99_queue_s": float(np.percentile(queue, 99)),
            "p50_service_s": float(np.percentile(service, 50)), "p99_service_s": float(np.percentile(service, 99)),
            "unit": "grid-pt-steps/s", "offered_load": offered, "makespan_s": makespan,
            "arrival_window_s": seconds, "nonfinite": int(sum(o["stats"]["nonfinite"] for o in ok)),
            "tile": tile, "zchunk": zchunk, "tile_delayed": tile_delayed, "zchunk_delayed": zchunk_delayed,
            "workload": "Poisson 20/s, N log-uniform 32..256 (multiples of 32), 20..200 steps, CAA/SAA L 1..3, "
                        "FP32, continuous batching"}


def _oracle_threads(n):
    """Set the OpenMP thread count of the oracle's runtime (its library links libgomp)."""
    import ctypes
    ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))


def _oracle_rate(W, n, pe, steps, mode, L, seed, field_seed, forcing, reps):
    """pt-steps/s of the oracle over `steps` RK3 steps after initialisation (not timed); median of
    `reps` runs."""
    from oracle import Oracle, OracleConfig
    q = W.make_field(n, field_seed, 0.3)
    dt, mu = W.default_dt(q), W.default_mu(n)
    fh = W.make_forcing(303, steps + 2, dt, 1.0, 0.1 * W.urms_of(q)) if forcing else None
    rates, secs = [], []
    for _ in range(reps):
        o = Oracle(OracleConfig(n=(n, n, n), p=pe, dt=dt, mu_ref=mu, max_delay=max(L, 1), forcing=forcing))
        o.init_field(q)
        if mode == "caa":
            o.set_schedule(1, L=L, c_r=L + 1, n_steps=steps + 2)
        else:
            o.set_schedule(2, L=L, seed=seed, n_steps=steps + 2)
        if forcing:
            o.set_forcing(fh)
        t = time.perf_counter()
        o.rk_step(steps)
        el = time.perf_counter() - t
        o.close()
        secs.append(el)
        rates.append(n ** 3 * steps / el)
    return float(np.median(rates)), float(np.median(secs))


def cpu_baseline(W, n, steps):
    """The CPU FP64 oracle on the host's cores, timed as the baseline protocol asks: median of 3 runs
    with initialisation excluded.  `value` is a 128^3 sample with the headline's PE shape (64^3),
    delays and forcing; beside it the 32^3 plain-method configuration in full, a few steps of the
    256^3 decaying configuration, and the 1-thread rate of the 128^3 sample (fewer steps)."""
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    pe = max(1, n // 64)
    v, el = _oracle_rate(W, n, (pe,) * 3, steps, "caa", 3, 0, 3, True, 3)
    cfg1, el1 = _oracle_rate(W, 32, (2, 2, 1), 10, "caa", 3, 0, 1, False, 3)
    cfg2, el2 = _oracle_rate(W, 256, (4, 4, 4), 7, "saa", 2, 102, 2, False, 1)
    _oracle_threads(1)
    one, el_one = _oracle_rate(W, n, (pe,) * 3, 2, "caa", 3, 0, 3, True, 1)
    _oracle_threads(cores)
    return {"value": v, "unit": "grid-pt-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{n}^3, {pe}x{pe}x{pe} PEs of 64^3, CAA L=3, forced, FP64, {steps} RK3 steps, median of 3 "
                      f"({el:.1f} s each)",
            "cfg1_full": {"value": cfg1, "sample": "32^3, 2x2x1 PEs, CAA L=3, FP64, 10 RK3 steps (the whole "
                                                   f"configuration), median of 3 ({el1:.2f} s each)"},
            "cfg2_sample": {"value": cfg2, "sample": f"256^3, 4x4x4 PEs, SAA L=2 seed 102, FP64, first 7 of its "
                                                     f"100 RK3 steps ({el2:.1f} s)"},
            "one_thread": {"value": one, "cores": 1, "sample": f"{n}^3 as value, 2 RK3 steps ({el_one:.1f} s)"}}


def field_rel_l2(a, b):
    """Relative L2 error of each conserved component of a against b."""
    return [float(np.linalg.norm((a[c] - b[c]).ravel()) / np.linalg.norm(b[c].ravel())) for c in range(a.shape[0])]


def order6_leg(torch, atns, W, traffic, n, pe, q, dt, mu, Wm, K):
    """The sixth-order AT scheme ((1,6) rows, 4-level extrapolation) on the same 512^3 field, FP32,
    unforced (decaying), CAA c_r = 4: timed window, then a kernel-event window for the roofline of
    its two launches per stage and its extrapolated face values (one launch per delayed step)."""
    total = Wm + 2 * K + 2
    cfg = atns.Config(n=(n,) * 3, p=(pe,) * 3, dt=dt, mu_ref=mu, max_delay=3, precision="fp32", order=6)
    sim = atns.Sim(cfg)
    sim.init_field(q)
    sim.set_delay_schedule(atns.CAA, L=3, c_r=4, n_steps=total)
    ms = time_window(torch, sim, K, warmup=Wm)
    ms_ev, kt = kernel_window(torch, sim, K)
    st = sim.stats()
    sim.close()
    torch.cuda.empty_cache()
    pd = sum(1 for s in range(Wm + K, Wm + 2 * K) if s >= 4 and s % 4) / K
    rf = roofline(kt, n, pe, 4, pd, K, kernels=("k6_gradflux", "k6_divupdate", "k6_ghosts"), order=6)
    rf["traffic"] = measured_traffic(f"k6_stage_{n}_pe{pe}_fp32", "stage6.hip")
    return {"value": n ** 3 * K / (ms * 1e-3), "unit": "grid-pt-steps/s", "ms_per_step": ms / K, "steps": K,
            "kernels_ms": {k: v[0] / max(v[1], 1) for k, v in kt.items()}, "roofline": rf,
            "delayed_fraction": pd, "nonfinite": st["nonfinite"],
            "workload": f"decaying turbulence {n}^3, {pe}x{pe}x{pe} PEs, sixth-order AT scheme, CAA L=3, FP32"}


def decaying_cfg2(torch, atns, W, traffic, steps):
    """The decaying-turbulence configuration: FP64, 256^3 on 4x4x4 PEs of 64^3, random (SAA) delays
    uniform in {0, 1, 2} from seed 102 after the L + 3 = 5 synchronous warm-up steps, seeded field 2,
    statistics read back after every step.  Pass 1 times the steps with their statistics (no
    per-kernel events); pass 2 repeats them from the same initial field with kernel events, for
    the roofline of the stage kernels and the cost of the statistics."""
    n, pe, L = 256, 4, 2
    q = W.make_field(n, 2, 0.3)
    dt, mu = W.default_dt(q), W.default_mu(n)
    cfg = atns.Config(n=(n,) * 3, p=(pe,) * 3, dt=dt, mu_ref=mu, max_delay=L, precision="fp64")
    sim = atns.Sim(cfg)
    sim.init_field(q)
    sim.set_delay_schedule(atns.SAA, L=L, seed=102, n_steps=steps + 1)
    b = atns.Batch("fp64")
    b.add(sim)
    b.autotune(None, reps=2)
    shapes = b.get_stage_tuning()
    b.remove(sim)
    b.close()
    sim.set_stage_tuning(*shapes)

    def run(with_events):
        sim.init_field(q)
        if with_events:
            sim.set_kernel_timing(True)
        stream = torch.cuda.current_stream()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record(stream)
        last = None
        for _ in range(steps):
            sim.rk_step(1)
            last = sim.stats()  # synchronises: the statistics of every step reach the host
        t1.record(stream)
        torch.cuda.synchronize()
        kt = sim.kernel_timing() if with_events else None
        if with_events:
            sim.set_kernel_timing(False)
        return t0.elapsed_time(t1), kt, last

    ms, _, st = run(False)
    ms_ev, kt, _ = run(True)
    # delayed fraction: after the warm-up every draw is uniform in {0..L}; its expectation (the
    # 36k draws of the window match it to about 0.5%)
    pd = max(0, steps - (L + 3)) / steps * L / (L + 1)
    rf = roofline(kt, n, pe, 8, pd, steps)
    sim.close()
    torch.cuda.empty_cache()
    return {"value": n ** 3 * steps / (ms * 1e-3), "unit": "grid-pt-steps/s", "ms_per_step": ms / steps,
            "steps": steps, "launch": dict(zip(("tile", "zchunk", "tile_delayed", "zchunk_delayed"), shapes)),
            "stats_ms_per_step": kt.get("k_stats", (0.0, 1))[0] / steps, "delayed_fraction": pd,
            "roofline": rf, "stats_last": {k: st[k] for k in ("step", "K", "eps", "enstrophy", "Mt", "nonfinite")},
            "workload": "decaying turbulence 256^3, 4x4x4 virtual PEs of 64^3, SAA L=2 seed 102, FP64, "
                        "statistics every step"}


PAPER_KERNELS = ("kp_publish", "kp_grad", "kp_rhs")


def paper_leg(torch, atns, W, traffic, n, pe, q, dt, mu, Wm, K, with_ab2=True):
    """The paper's own discretisation (internal-energy form, (2,4) AT second derivatives, three-step
    mixed derivatives, Sutherland's law) on the same 512^3 field, FP32, unforced, CAA c_r = 4: RK3
    steps (timed window, then a kernel-event window for the roofline), then AB2 steps, the paper's
    own integrator."""
    cv = W.GAS_R / (W.GAMMA - 1.0)
    qp = q.copy()
    qp[4] = q[4] - 0.5 * (q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / q[0]  # rho e = E - rho |u|^2 / 2
    total = Wm + 3 * K + 4
    cfg = atns.Config(n=(n,) * 3, p=(pe,) * 3, dt=dt, mu_ref=mu, max_delay=3, precision="fp32", form=1,
                      visc_law=1, sutherland_s=0.4)
    sim = atns.Sim(cfg)
    sim.init_field(qp)
    del qp
    sim.set_delay_schedule(atns.CAA, L=3, c_r=4, n_steps=total)
    ms = time_window(torch, sim, K, warmup=Wm)
    ms_ev, kt = kernel_window(torch, sim, K)
    pd = sum(1 for s in range(Wm + K, Wm + 2 * K) if s >= 4 and s % 4) / K
    stage_ms = sum(kt[k][0] for k in kt if k in PAPER_KERNELS) / (3 * K)
    words = traffic.paper_words_per_point_step((n,) * 3, (pe,) * 3, pd) / 3.0
    gbs = words * 4 * n ** 3 / (stage_ms * 1e-3) / 1e9
    ab2 = None
    if with_ab2:
        sim.ab2_step(2)
        ms_ab2, kt_ab2 = kernel_window(torch, sim, K, sim.ab2_step)
        pd_ab2 = sum(1 for s in range(Wm + 2 * K + 4, Wm + 3 * K + 4) if s >= 4 and s % 4) / K
        step_ab2 = sum(kt_ab2[k][0] for k in kt_ab2 if k in PAPER_KERNELS) / K
        gbs_ab2 = traffic.paper_words_per_point_step((n,) * 3, (pe,) * 3, pd_ab2, ab2=True) * 4 * n ** 3 / (
            step_ab2 * 1e-3) / 1e9
        ab2 = {"value": n ** 3 * K / (ms_ab2 * 1e-3), "ms_per_step": ms_ab2 / K,
               "roofline": {"bound": "hbm", "achieved": gbs_ab2, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": gbs_ab2 / HBM_PEAK_GBS,
                            "algorithmic_bytes_per_point_step":
                                4 * traffic.paper_words_per_point_step((n,) * 3, (pe,) * 3, pd_ab2, ab2=True)},
               "timing": "kernel events"}
    st = sim.stats()
    sim.close()
    torch.cuda.empty_cache()
    return {"value": n ** 3 * K / (ms * 1e-3), "unit": "grid-pt-steps/s", "ms_per_step": ms / K, "steps": K,
            "kernels_ms": {k: v[0] / max(v[1], 1) for k, v in kt.items()},
            "roofline": {"bound": "hbm", "kernel": "+".join(PAPER_KERNELS), "achieved": gbs, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "avg_stage_ms": stage_ms,
                         "algorithmic_bytes_per_point_step": words * 3 * 4,
                         "traffic": measured_traffic(f"kp_stage_{n}_pe{pe}_fp32", "stagep.hip")},
            "delayed_fraction": pd, "ab2": ab2,
            "nonfinite": st["nonfinite"], "stats_after": {k: st[k] for k in ("K", "eps", "enstrophy", "Mt")},
            "workload": f"decaying turbulence {n}^3, {pe}x{pe}x{pe} PEs, the paper's internal-energy form "
                        "((2,4) AT second derivatives, three-step mixed derivatives, Sutherland S = 0.4), "
                        "CAA L=3, FP32"}


def diag_leg(torch, atns, sim, n, reps=3):
    """Turbulence diagnostics (Sec. 4.1: E(kappa), E_p(kappa), S and F of du/dx, PDFs of eps/<eps> and
    Omega/<Omega>) of the headline run's final FP32 state, timed with HIP events on the run's stream."""
    nshell = int(math.isqrt(3 * (n // 2) ** 2)) + 2
    nbins, emax, omax = 200, 20.0, 40.0
    ws = torch.empty(atns.diag_workspace_bytes(sim.cfg, nshell, nbins, emax, omax), dtype=torch.uint8, device="cuda")
    raw = torch.empty(2 * nshell + atns.DIAG_N_SCALARS + 2 * (nbins + 1), dtype=torch.float64, device="cuda")
    st = sim.stream
    qp = sim.field_device_ptr()

    def call():
        atns.field_diagnostics(sim.cfg, qp, nshell, nbins, emax, omax, workspace=ws, stream=st, out=raw, sync=False)

    call()
    st.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        call()
    e1.record(st)
    st.synchronize()
    ms = e0.elapsed_time(e1) / reps
    d = atns.diag_dict(raw.cpu().numpy(), nshell, nbins)
    del ws, raw
    # algorithmic bytes per point: the field read by the moment, histogram and x-transform passes
    # (3 x 5 FP32 words), and the half spectra of u, v, w, p (4 x 16 B x (n/2 + 1) / n) written by
    # the x pass, read and written by the y pass and read by the z pass
    bpp = 3 * 5 * 4 + 4 * 16 * (n // 2 + 1) / n * 4
    gbs = bpp * n ** 3 / (ms * 1e-3) / 1e9
    E = d["E"]
    return {"ms_per_call": ms, "calls": reps, "points": n ** 3, "nshell": nshell, "nbins": nbins,
            "roofline": {"bound": "hbm", "kernel": "all diagnostics launches", "achieved": gbs,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                         "algorithmic_bytes_per_point": bpp, "traffic": None},
            "S": d["S"], "F": d["F"], "eps_mean": d["eps_mean"], "ens_mean": d["ens_mean"],
            "E_total": float(E.sum()), "E_peak_shell": int(np.argmax(E[1:]) + 1),
            "Ep_total_fluct": float(d["Ep"][1:].sum()),
            "eps_pdf_tail_gt10": int(d["eps_pdf"][nbins * 10 // int(emax):].sum()),
            "ens_pdf_tail_gt10": int(d["ens_pdf"][nbins * 10 // int(omax):].sum()),
            "workload": f"{n}^3 FP32 state after the timed RK3 steps; {nshell} shells, {nbins} PDF bins "
                        f"on [0, {emax:g}) and [0, {omax:g}), FP64 arithmetic"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch

    if args.calib_copy_mib:
        calib_copy(torch, args.calib_copy_mib)
        return
    from paper_2003_10561_amd import atns, traffic, workload as W

    n, pe, K, Wm = args.n, args.pe, args.steps, args.warmup
    AB2_WARM = 2
    # warm-up, the timed window, the kernel-event window, then the Adams-Bashforth steps
    total = Wm + 2 * K + 2 + AB2_WARM + K
    t = time.perf_counter()
    q = W.make_field(n, 3, 0.3, log=log)
    dt, mu = W.default_dt(q), W.default_mu(n)
    fh = W.make_forcing(303, total, dt, 1.0, 0.1 * W.urms_of(q))
    log(f"inputs {n}^3 ready in {time.perf_counter() - t:.1f} s; dt={dt:.4e} mu={mu:.4e}")
    ntiles = pe ** 3
    sched = np.zeros((total, ntiles, 6), np.int8)
    for s in range(4, total):
        sched[s] = s % 4
    pd = traffic.delayed_fraction(sched[Wm:Wm + K])
    pd_k = traffic.delayed_fraction(sched[Wm + K:Wm + 2 * K])

    sim, tuned = build_sim(atns, W, n, pe, "fp32", total, q, dt, mu, fh, args.tile, args.zchunk, not args.no_autotune)
    launch32 = dict(zip(("tile", "zchunk", "tile_delayed", "zchunk_delayed"), sim.get_stage_tuning()),
                    autotuned=tuned)
    log(f"fp32 simulation initialised (launch {launch32}); timing")
    ms32 = time_window(torch, sim, K, warmup=Wm)
    ms32_ev, kt32 = kernel_window(torch, sim, K)
    st32 = sim.stats()
    diag = None
    if not args.no_diag:
        diag = diag_leg(torch, atns, sim, n)
        log(f"diagnostics: {diag}")
    f32 = sim.get_field() if not args.no_fp64 else None
    if not args.no_ab2:
        sim.ab2_step(AB2_WARM)
        ms_ab2, kt_ab2 = kernel_window(torch, sim, K, sim.ab2_step)
        st_ab2 = sim.stats()
    del sim
    torch.cuda.empty_cache()
    log(f"fp32: {ms32 / K:.3f} ms/step ({ms32_ev / K:.3f} with kernel events); kernels {kt32}")
    rf = roofline(kt32, n, pe, 4, pd_k, K)
    rf["traffic"] = measured_traffic(f"k_stage_{n}_pe{pe}_fp32")
    value = n ** 3 * K / (ms32 * 1e-3)
    out = {"metric": METRIC, "value": value, "unit": "grid-pt-steps/s", "n_gpus": 1, "steps": K,
           "warmup": Wm, "ms_per_step": ms32 / K, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"forced turbulence {n}^3, {pe}x{pe}x{pe} virtual PEs "
                                  f"({n // pe}^3 each), CAA delays c_r=4 (L=3), OU forcing |k|<=2.5, "
                                  "FP32 fields / FP64 reductions, LS-RK3",
                      "n": n, "pe": [pe, pe, pe], "delays": "CAA L=3", "precision": "fp32"},
           "launch": launch32,
           "roofline": rf,
           "kernel_window": {"steps": K, "ms_per_step": ms32_ev / K, "delayed_fraction": pd_k,
                             "kernels_ms": {k: v[0] / max(v[1], 1) for k, v in kt32.items()},
                             "launches": {k: v[1] for k, v in kt32.items()}},
           "hbm_gbs_algorithmic": traffic.bytes_per_point_step((n,) * 3, (pe,) * 3, pd, 4) * value / 1e9,
           "stats_after": {k: st32[k] for k in ("K", "eps", "enstrophy", "Mt", "nonfinite")}}
    if diag is not None:
        out["diagnostics"] = diag
    if not args.no_ab2:
        # the paper's own integrator (Sec. 2.2, Eq. time_ab): one RHS per step; not the headline
        pd_ab2 = traffic.delayed_fraction(sched[Wm + 2 * K + AB2_WARM:Wm + 3 * K + AB2_WARM])
        stage_ab2 = sum(kt_ab2[k][0] for k in kt_ab2 if k in STAGE_KERNELS) / K
        gbs_ab2 = traffic.ab2_words_per_point_step((n,) * 3, (pe,) * 3, pd_ab2) * 4 * n ** 3 / (stage_ab2 * 1e-3) / 1e9
        out["ab2"] = {"value": n ** 3 * K / (ms_ab2 * 1e-3), "unit": "grid-pt-steps/s", "ms_per_step": ms_ab2 / K,
                       "steps": K, "warmup": AB2_WARM, "stage_ms": stage_ab2, "delayed_fraction": pd_ab2,
                       "roofline": {"bound": "hbm", "achieved": gbs_ab2, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                    "frac": gbs_ab2 / HBM_PEAK_GBS,
                                    "algorithmic_bytes_per_point_step":
                                        4 * traffic.ab2_words_per_point_step((n,) * 3, (pe,) * 3, pd_ab2)},
                       "nonfinite": st_ab2["nonfinite"],
                       "workload": "the same run continued with second-order Adams-Bashforth steps (timed with "
                                   "kernel events)"}
    if not args.no_fp64:
        sim, _ = build_sim(atns, W, n, pe, "fp64", total, q, dt, mu, fh, args.tile, args.zchunk, not args.no_autotune)
        launch64 = dict(zip(("tile", "zchunk", "tile_delayed", "zchunk_delayed"), sim.get_stage_tuning()))
        log("fp64 simulation initialised; timing")
        ms64 = time_window(torch, sim, K, warmup=Wm)
        ms64_ev, kt64 = kernel_window(torch, sim, K)
        st64 = sim.stats()
        f64 = sim.get_field()
        del sim
        torch.cuda.empty_cache()
        log(f"fp64: {ms64 / K:.3f} ms/step")
        v64 = n ** 3 * K / (ms64 * 1e-3)
        rf64 = roofline(kt64, n, pe, 8, pd_k, K)
        rf64["traffic"] = measured_traffic(f"k_stage_{n}_pe{pe}_fp64")
        errs = field_rel_l2(f32, f64)
        del f32, f64
        out["fp64"] = {"value": v64, "ms_per_step": ms64 / K, "roofline_frac": rf64["frac"], "launch": launch64,
                       "achieved_gbs": rf64["achieved"], "avg_launch_ms": rf64["avg_launch_ms"],
                       "roofline": rf64,
                       "hbm_gbs_algorithmic": traffic.bytes_per_point_step((n,) * 3, (pe,) * 3, pd, 8) * v64 / 1e9,
                       "fp32_speedup": value / v64,
                       "fp32_vs_fp64_field_rel_l2": dict(zip(("rho", "rho_u", "rho_v", "rho_w", "E"), errs)),
                       "fp32_vs_fp64_stats_rel": {k: abs(st32[k] - st64[k]) / abs(st64[k])
                                                  for k in ("K", "eps", "enstrophy", "Mt")},
                       "error_note": f"FP32 and FP64 runs after the same {Wm + 2 * K} RK3 steps; the FP64 path "
                                     "matches the FP64 oracle at this size"}
    if not args.no_order6:
        log("sixth-order scheme ...")
        out["order6"] = order6_leg(torch, atns, W, traffic, n, pe, q, dt, mu, Wm, K)
        log(f"order6: {out['order6']}")
    if not args.no_paper:
        log("the paper's own discretisation ...")
        out["paper_form"] = paper_leg(torch, atns, W, traffic, n, pe, q, dt, mu, Wm, K, not args.no_paper_ab2)
        log(f"paper_form: {out['paper_form']}")
    if not args.no_cfg2:
        log("decaying 256^3 FP64 configuration ...")
        out["decaying_256"] = decaying_cfg2(torch, atns, W, traffic, args.cfg2_steps)
        log(f"decaying_256: {out['decaying_256']}")
    if not args.no_batch:
        log("batched 64-run workload ...")
        out["batched"] = batched_workload(torch, atns, W, args.batch_steps, args.batch_steps, args.tune_cache)
        log(f"batched: {out['batched']}")
    if not args.no_serve:
        log("served trace ...")
        # the launch shape the autotuner chose for the batched mix (same kind of runs), if measured
        bt = out.get("batched", {})
        out["served"] = served_workload(atns, W, args.serve_seconds, tile=bt.get("tile", -1),
                                        zchunk=bt.get("zchunk", 64), tile_delayed=bt.get("tile_delayed", -1),
                                        zchunk_delayed=bt.get("zchunk_delayed", 64))
        log(f"served: {out['served']}")
    if not args.no_cpu:
        log("cpu oracle baseline ...")
        out["cpu_baseline"] = cpu_baseline(W, args.cpu_n, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
