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
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--tile", type=int, default=None, help="fused-stage tile shape (default: library)")
    ap.add_argument("--zchunk", type=int, default=None)
    return ap.parse_args()


def build_sim(atns, W, n, pe, precision, n_steps_total, q, dt, mu, fh, tile=None, zchunk=None):
    cfg = atns.Config(n=(n, n, n), p=(pe, pe, pe), dt=dt, mu_ref=mu, max_delay=3,
                      precision=precision, forcing=True)
    sim = atns.Sim(cfg)
    if tile is not None or zchunk is not None:
        t0, z0 = sim.get_tuning()
        sim.set_tuning(t0 if tile is None else tile, z0 if zchunk is None else zchunk)
    sim.init_field(q)
    sim.set_delay_schedule(atns.CAA, L=3, c_r=4, n_steps=n_steps_total)
    sim.set_forcing(fh)
    return sim


def time_steps(torch, sim, warmup, steps):
    sim.rk_step(warmup)
    torch.cuda.synchronize()
    sim.set_kernel_timing(True)
    stream = torch.cuda.current_stream()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    sim.rk_step(steps)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    kt = sim.kernel_timing()
    sim.set_kernel_timing(False)
    return ms, kt


def roofline(kt, n, pe, word, pd, steps):
    """Dominant launch = one RK stage (its kernels); algorithmic bytes per stage launch."""
    from paper_2003_10561_amd import traffic
    stage_kernels = [k for k in kt if k in ("k_grad", "k_flux", "k_update", "k_stage")]
    launches = steps * 3
    stage_ms = sum(kt[k][0] for k in stage_kernels) / launches
    words = traffic.words_per_point_step((n,) * 3, (pe,) * 3, pd) / 3.0
    bytes_per_launch = words * word * n ** 3
    achieved = bytes_per_launch / (stage_ms * 1e-3) / 1e9
    name = "+".join(stage_kernels)
    return {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "bytes_per_launch": bytes_per_launch, "avg_launch_ms": stage_ms,
            "algorithmic_bytes_per_point_step": words * 3 * word}


def cpu_baseline(W, n, steps):
    """The CPU FP64 oracle on a bounded sample with the same PE shape (64^3), delays and forcing."""
    from oracle import Oracle, OracleConfig
    pe = max(1, n // 64)
    q = W.make_field(n, 3, 0.3)
    dt, mu = W.default_dt(q), W.default_mu(n)
    fh = W.make_forcing(303, steps + 2, dt, 1.0, 0.1 * W.urms_of(q))
    o = Oracle(OracleConfig(n=(n, n, n), p=(pe, pe, pe), dt=dt, mu_ref=mu, max_delay=3, forcing=True))
    o.init_field(q)
    o.set_schedule(1, L=3, c_r=4, n_steps=steps + 2)
    o.set_forcing(fh)
    t = time.perf_counter()
    o.rk_step(steps)
    el = time.perf_counter() - t
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": n ** 3 * steps / el, "unit": "grid-pt-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{n}^3, {pe}x{pe}x{pe} PEs of 64^3, CAA L=3, forced, FP64, {steps} RK3 steps "
                      f"({el:.1f} s)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2003_10561_amd import atns, traffic, workload as W

    n, pe, K, Wm = args.n, args.pe, args.steps, args.warmup
    total = Wm + K + 2
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

    sim = build_sim(atns, W, n, pe, "fp32", total, q, dt, mu, fh, args.tile, args.zchunk)
    log("fp32 simulation initialised; timing")
    ms32, kt32 = time_steps(torch, sim, Wm, K)
    st32 = sim.stats()
    del sim
    torch.cuda.empty_cache()
    log(f"fp32: {ms32 / K:.3f} ms/step; tuning {args.tile, args.zchunk}; kernels {kt32}")
    rf = roofline(kt32, n, pe, 4, pd, K)
    value = n ** 3 * K / (ms32 * 1e-3)
    out = {"metric": METRIC, "value": value, "unit": "grid-pt-steps/s", "n_gpus": 1, "steps": K,
           "warmup": Wm, "ms_per_step": ms32 / K, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"forced turbulence {n}^3, {pe}x{pe}x{pe} virtual PEs "
                                  f"({n // pe}^3 each), CAA delays c_r=4 (L=3), OU forcing |k|<=2.5, "
                                  "FP32 fields / FP64 reductions, LS-RK3",
                      "n": n, "pe": [pe, pe, pe], "delays": "CAA L=3", "precision": "fp32"},
           "roofline": rf,
           "hbm_gbs_algorithmic": traffic.bytes_per_point_step((n,) * 3, (pe,) * 3, pd, 4) * value / 1e9,
           "stats_after": {k: st32[k] for k in ("K", "eps", "enstrophy", "Mt", "nonfinite")}}
    if not args.no_fp64:
        sim = build_sim(atns, W, n, pe, "fp64", total, q, dt, mu, fh, args.tile, args.zchunk)
        log("fp64 simulation initialised; timing")
        ms64, kt64 = time_steps(torch, sim, Wm, K)
        st64 = sim.stats()
        del sim
        torch.cuda.empty_cache()
        log(f"fp64: {ms64 / K:.3f} ms/step")
        v64 = n ** 3 * K / (ms64 * 1e-3)
        rf64 = roofline(kt64, n, pe, 8, pd, K)
        out["fp64"] = {"value": v64, "ms_per_step": ms64 / K, "roofline_frac": rf64["frac"],
                       "achieved_gbs": rf64["achieved"],
                       "hbm_gbs_algorithmic": traffic.bytes_per_point_step((n,) * 3, (pe,) * 3, pd, 8) * v64 / 1e9,
                       "fp32_speedup": value / v64,
                       "fp32_vs_fp64_stats_rel": {k: abs(st32[k] - st64[k]) / abs(st64[k])
                                                  for k in ("K", "eps", "enstrophy", "Mt")}}
    if not args.no_cpu:
        log("cpu oracle baseline ...")
        out["cpu_baseline"] = cpu_baseline(W, args.cpu_n, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
