"""Profiling support: the program rocprofv3 runs, and the summaries of its
output kept with the sources.

  python -m paper_2208_04371_amd.profiling step --workload microstrip --steps 200
      runs `steps` fused steps of a workload in its default launch shape,
      then five 1 GiB streaming copies (the calibration kernel);
  python -m paper_2208_04371_amd.profiling summarize --workload microstrip \\
      --stats DIR [--fetch DIR --write DIR] --command "..." --out profiles
      writes <out>/fused_step_<workload>_stats.txt from a --kernel-trace
      --stats run and, given the FETCH_SIZE and WRITE_SIZE runs,
      <out>/fused_step_<workload>_traffic.json and .txt (HBM-side bytes per
      step, each counter scaled by what it reads for the copy of known size).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 1 << 30
COPY_REPS = 5
WORKLOADS = {
    "microstrip": ("single_microstrip", "microstrip_400x120x80"),
    "line": ("large_line", "line_1024x512x256"),
}


# The sources that decide what the profiled single-plan step launches and
# moves (kernels, their headers, the plan layout and tile sets) and the copy
# kernel the counters are calibrated against.  Batching, the autotuner and
# the host post-processing do not enter a profiled step.
PROFILED_SOURCES = ("copy.hip", "fused.hip", "internal.hpp", "kernels.hip", "plan.cpp",
                    "probe.hpp", "source.hpp")


def source_hash() -> str:
    """Hash of the profiled sources: a counter summary holds for these only."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2208_04371_amd", "csrc")
    for fn in PROFILED_SOURCES:
        with open(os.path.join(d, fn), "rb") as f:
            h.update(fn.encode() + f.read())
    return h.hexdigest()[:16]


def run_step(workload: str, steps: int):
    sys.path.insert(0, ROOT)
    import torch
    import paper_2208_04371_amd as fd
    import workloads as W
    gen, _ = WORKLOADS[workload]
    prob = getattr(W, gen)()
    sim = fd.Simulation(prob, fused=True)
    sim.run(steps)
    torch.cuda.synchronize()
    rows, z = fd.fdtd_plan_get_config(sim.handle)
    sim.close()
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(COPY_REPS):
        fd.fdtd_device_copy(b, a)
    torch.cuda.synchronize()
    print(f"ran {steps} steps of {prob.name} (rows {rows}, zchunk {z}) and {COPY_REPS} copies "
          f"of {COPY_BYTES} B", flush=True)


def _rows(d: str, pattern: str):
    out = []
    for fn in glob.glob(os.path.join(d, "**", pattern), recursive=True):
        with open(fn, newline="") as f:
            out += list(csv.DictReader(f))
    return out


def _kernel_class(name: str) -> str:
    m = re.search(r"k_fused<\s*\d+\s*,\s*(true|false)", name)
    if m:
        return "boundary" if m.group(1) == "true" else "interior"
    if "k_copy" in name and "tail" not in name:
        return "copy"
    return "other"


def kernel_stats(d: str):
    """{name: (calls, average ns)} from a --stats run."""
    out = {}
    for r in _rows(d, "*kernel_stats.csv"):
        out[r["Name"]] = (int(r["Calls"]), float(r["AverageNs"]))
    return out


def counter_per_class(d: str, counter: str):
    """Average counter value per dispatch for each kernel class."""
    acc = {}
    for r in _rows(d, "*counter_collection.csv"):
        if r.get("Counter_Name") != counter:
            continue
        k = _kernel_class(r.get("Kernel_Name", ""))
        s, n = acc.get(k, (0.0, 0))
        acc[k] = (s + float(r["Counter_Value"]), n + 1)
    return {k: s / n for k, (s, n) in acc.items()}


def summarize(a):
    _, tag = WORKLOADS[a.workload]
    os.makedirs(a.out, exist_ok=True)
    stats = kernel_stats(a.stats)
    lines = [f"# rocprofv3 kernel statistics: fused step, {tag}", "",
             "command:", f"  {a.command}", "", f"sources: {source_hash()}", "",
             f"{'kernel':70s} {'calls':>6s} {'avg_us':>10s}"]
    step_us = 0.0
    for name, (calls, avg) in sorted(stats.items(), key=lambda kv: -kv[1][0] * kv[1][1]):
        short = name if len(name) <= 70 else name[:67] + "..."
        lines.append(f"{short:70s} {calls:6d} {avg / 1e3:10.3f}")
        if _kernel_class(name) in ("boundary", "interior"):
            step_us += avg / 1e3
    lines += ["", f"fused step (boundary + interior launch): {step_us:.3f} us"]
    with open(os.path.join(a.out, f"fused_step_{tag}_stats.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    if not (a.fetch and a.write):
        return
    fetch = counter_per_class(a.fetch, "FETCH_SIZE")
    write = counter_per_class(a.write, "WRITE_SIZE")
    # each counter in KiB per dispatch; the copy moves COPY_BYTES each way
    kf = COPY_BYTES / (fetch["copy"] * 1024.0)
    kw = COPY_BYTES / (write["copy"] * 1024.0)
    per = {c: fetch.get(c, 0.0) * 1024.0 * kf + write.get(c, 0.0) * 1024.0 * kw
           for c in ("boundary", "interior")}
    d = {"workload": tag, "source_hash": source_hash(),
         "bytes_per_launch": round(per["boundary"] + per["interior"]),
         "bytes_boundary": round(per["boundary"]), "bytes_interior": round(per["interior"]),
         "fetch_kib": {k: round(v, 1) for k, v in fetch.items()},
         "write_kib": {k: round(v, 1) for k, v in write.items()},
         "copy_scale": {"fetch": kf, "write": kw}, "copy_bytes": COPY_BYTES,
         "command": a.command}
    with open(os.path.join(a.out, f"fused_step_{tag}_traffic.json"), "w") as f:
        json.dump(d, f, indent=1)
        f.write("\n")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("step")
    s.add_argument("--workload", choices=sorted(WORKLOADS), default="microstrip")
    s.add_argument("--steps", type=int, default=200)
    m = sub.add_parser("summarize")
    m.add_argument("--workload", choices=sorted(WORKLOADS), default="microstrip")
    m.add_argument("--stats", required=True)
    m.add_argument("--fetch")
    m.add_argument("--write")
    m.add_argument("--command", default="")
    m.add_argument("--out", default=os.path.join(ROOT, "profiles"))
    a = ap.parse_args()
    if a.cmd == "step":
        run_step(a.workload, a.steps)
    else:
        summarize(a)


if __name__ == "__main__":
    main()
