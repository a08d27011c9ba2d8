"""Summaries of rocprofv3 output for the stage kernels (the text files kept under profiles/).

Reads a `--kernel-trace --stats` run and two `--pmc` runs (FETCH_SIZE, then WRITE_SIZE) of the same
bench command, plus the same two counters for a plain device copy of known size, and writes:

* <out>_trace.md: per-kernel call counts and durations, and the per-stage time over the timed
  window (the last `timed` stage launches, with the AT face-view launches among them);
* <out>_traffic.md: HBM bytes per stage launch over the same window, each counter scaled by the
  ratio (bytes the copy moved) / (bytes the counter reported for it), and the sha256 of the stage
  kernel source the counters were taken on (bench.py reports the traffic only while it matches).

Usage: python -m paper_2003_10561_amd.profsum --trace DIR --fetch DIR --write DIR --copy-fetch DIR
       --copy-write DIR --copy-bytes B --timed 30 --out profiles/k_stage_512_pe8_fp32 --command "..."
       [--stage k_stage< --aux k_at_sums<]

--stage names the launch that ends each RK stage (one per stage), --aux the launches that belong to
the stage before it (the AT sums of the fourth-order scheme; the gradient / flux launch of the
sixth-order one, whose divergence / update launch is the stage launch).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os

HERE = os.path.dirname(os.path.abspath(__file__))
STAGE = "k_stage<"  # defaults; main() takes --stage / --aux
VIEWS = ("k_at_sums<",)


def is_aux(k):
    return STAGE not in k and any(v in k for v in VIEWS)


def short_name(k):
    """Kernel name without return type, namespaces and argument list."""
    k = k.replace("void ", "").replace("atns::(anonymous namespace)::", "").replace("atns::", "")
    k = k.replace("(anonymous namespace)::", "")
    return k.split("(")[0]


def _one(pattern):
    hits = sorted(glob.glob(pattern))
    if not hits:
        raise FileNotFoundError(pattern)
    return hits[0]


def dispatches(trace_dir):
    rows = list(csv.DictReader(open(_one(os.path.join(trace_dir, "*kernel_trace.csv")))))
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return [(r["Kernel_Name"], (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6) for r in rows]


def counters(pmc_dir):
    rows = list(csv.DictReader(open(_one(os.path.join(pmc_dir, "*counter_collection.csv")))))
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return [(r["Kernel_Name"], float(r["Counter_Value"])) for r in rows]


def timed_window(seq, timed):
    """Entries from the `timed`-th last stage launch on (the auxiliary launches before it included)."""
    idx = [i for i, (k, _) in enumerate(seq) if STAGE in k]
    if len(idx) < timed:
        raise ValueError(f"only {len(idx)} stage launches")
    first = idx[-timed]
    # the auxiliary launches of a stage come just before its stage launch
    while first > 0 and is_aux(seq[first - 1][0]):
        first -= 1
    last = idx[-1]
    return seq[first:last + 1]


def copy_factor(pmc_dir, nbytes):
    vals = [v for k, v in counters(pmc_dir) if "copyBuffer" in k or "elementwise" in k]
    big = max(vals)
    return nbytes / (big * 1024.0)


SOURCE = "stage_fused.hip"


def source_sha():
    with open(os.path.join(HERE, "csrc", SOURCE), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def main():
    ap = argparse.ArgumentParser()
    for k in ("trace", "fetch", "write", "copy_fetch", "copy_write", "out", "command"):
        ap.add_argument("--" + k.replace("_", "-"), required=True)
    ap.add_argument("--copy-bytes", type=float, required=True)
    ap.add_argument("--timed", type=int, required=True)
    ap.add_argument("--workload", default="")
    ap.add_argument("--stage", default="k_stage<")
    ap.add_argument("--aux", default="k_at_sums<", help="comma-separated patterns of the auxiliary launches")
    ap.add_argument("--summary", default="", help="comma-separated kernel patterns: per-kernel table only")
    ap.add_argument("--source", default="stage_fused.hip", help="kernel source whose sha256 is recorded")
    a = ap.parse_args()
    global STAGE, VIEWS, SOURCE
    STAGE, VIEWS, SOURCE = a.stage, tuple(a.aux.split(",")), a.source
    if a.summary:
        return summary(a)

    seq = dispatches(a.trace)
    win = timed_window(seq, a.timed)
    st_ms = sum(d for k, d in win if STAGE in k)
    gv_ms = sum(d for k, d in win if is_aux(k))
    n_gv = sum(1 for k, _ in win if is_aux(k))
    def table(entries, top):
        per_kernel = {}
        for k, d in entries:
            c, t = per_kernel.get(k, (0, 0.0))
            per_kernel[k] = (c + 1, t + d)
        rows = ["| kernel | calls | avg ms | total ms |", "|---|---|---|---|"]
        for k, (c, t) in sorted(per_kernel.items(), key=lambda kv: -kv[1][1])[:top]:
            rows.append(f"| `{short_name(k)[:80]}` | {c} | {t / c:.3f} | {t:.1f} |")
        return rows

    lines = [f"# Kernel trace: {STAGE.rstrip('<')} and {', '.join(v.rstrip('<') for v in VIEWS)}, {a.workload}", "",
             "Command (R = the repository root; run from /tmp with `export TMPDIR=/tmp`):", "",
             "```", a.command.split(" ;; ")[0], "```", "",
             f"Kernels of the timed window (the last {a.timed} stage launches of the single-run workload):", ""]
    lines += table(win, 12)
    lines += ["", "Whole run, the 12 kernels with the most time (other workloads of the command included):", ""]
    lines += table(seq, 12)
    lines += ["", f"Timed window (last {a.timed} stage launches):", "",
              f"- stage_launch: {STAGE.rstrip('<')}",
              f"- aux_launch: {', '.join(v.rstrip('<') for v in VIEWS)}",
              f"- stage_launch_avg_ms: {st_ms / a.timed:.4f}",
              f"- aux_launches: {n_gv}",
              f"- aux_ms_per_stage: {gv_ms / a.timed:.4f}",
              f"- stage_avg_ms: {(st_ms + gv_ms) / a.timed:.4f}",
              f"- source_sha256: {source_sha()}", ""]
    with open(a.out + "_trace.md", "w") as f:
        f.write("\n".join(lines))

    ff = copy_factor(a.copy_fetch, a.copy_bytes)
    fw = copy_factor(a.copy_write, a.copy_bytes)
    fetch = timed_window(counters(a.fetch), a.timed)
    write = timed_window(counters(a.write), a.timed)
    fb = sum(v for k, v in fetch if STAGE in k or is_aux(k)) * 1024.0 * ff / a.timed
    wb = sum(v for k, v in write if STAGE in k or is_aux(k)) * 1024.0 * fw / a.timed
    sf = [v * 1024.0 * ff for k, v in fetch if STAGE in k]
    sw = [v * 1024.0 * fw for k, v in write if STAGE in k]
    cmds = a.command.split(" ;; ")
    lines = [f"# HBM traffic: {STAGE.rstrip('<')} and {', '.join(v.rstrip('<') for v in VIEWS)}, {a.workload}", "",
             "Commands (R = the repository root; run from /tmp with `export TMPDIR=/tmp`):", "", "```"]
    lines += cmds[1:] if len(cmds) > 1 else cmds
    lines += ["```", "",
              f"Copy calibration: for a device copy of {a.copy_bytes:.0f} bytes each way, bytes moved / "
              f"bytes reported is {ff:.4f} for FETCH_SIZE and {fw:.4f} for WRITE_SIZE; these factors scale "
              "the stage counters below.", "",
              f"Per stage over the timed window ({STAGE.rstrip('<')} plus {', '.join(v.rstrip('<') for v in VIEWS)}):",
              "",
              f"- fetch_bytes_per_launch: {fb:.6e}",
              f"- write_bytes_per_launch: {wb:.6e}",
              f"- bytes_per_launch: {fb + wb:.6e}",
              f"- fetch_scale: {ff:.6f}",
              f"- write_scale: {fw:.6f}",
              f"- source_sha256: {source_sha()}", "",
              f"{STAGE.rstrip('<')} alone, per launch in the window (GB fetched / written):", "",
              "| launch | fetch GB | write GB |", "|---|---|---|"]
    for i, (x, y) in enumerate(zip(sf, sw)):
        lines.append(f"| {i} | {x / 1e9:.3f} | {y / 1e9:.3f} |")
    with open(a.out + "_traffic.md", "w") as f:
        f.write("\n".join(lines) + "\n")


def summary(a):
    """Per-kernel calls and durations over the whole traced run for the kernels matching the
    --summary patterns (workloads measured per call rather than per stage)."""
    pats = a.summary.split(",")
    per = {}
    for k, d in dispatches(a.trace):
        if any(p in k for p in pats):
            c, t = per.get(k, (0, 0.0))
            per[k] = (c + 1, t + d)
    rows = ["| kernel | calls | avg ms | total ms |", "|---|---|---|---|"]
    tot = 0.0
    for k, (c, t) in sorted(per.items(), key=lambda kv: -kv[1][1]):
        rows.append(f"| `{short_name(k)[:80]}` | {c} | {t / c:.3f} | {t:.1f} |")
        tot += t
    calls = max((c for c, _ in per.values()), default=0)
    lines = [f"# Kernel trace: {a.workload}", "",
             "Command (R = the repository root; run from /tmp with `export TMPDIR=/tmp`):", "",
             "```", a.command, "```", "", "Kernels matching " + ", ".join(f"`{p}`" for p in pats) + ":", ""]
    lines += rows
    lines += ["", f"- calls_per_kernel: {calls}",
              f"- ms_per_call_sum_of_kernels: {tot / max(calls, 1):.4f}",
              f"- source_sha256: {source_sha()}", ""]
    with open(a.out + "_trace.md", "w") as f:
        f.write("\n".join(lines))


if __name__ == "__main__":
    main()
