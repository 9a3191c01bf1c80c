"""Profiling support: the program rocprofv3 runs, and the summaries of its
output kept with the sources.

  python -m paper_2208_04371_amd.profiling step --workload line --steps 200 [--temporal M]
      runs `steps` fused steps of a workload in its default launch shape
      (two-level steps as the plan chooses them, or as --temporal sets),
      then five 1 GiB streaming copies (the calibration kernel);
  python -m paper_2208_04371_amd.profiling summarize --workload line --steps 200 \\
      --stats DIR [--counter-steps 20 --fetch DIR --write DIR --sizes DIR] --command "..."
      writes <out>/fused_step_<workload>_stats.txt from a --kernel-trace
      --stats run and, given the counter runs, <out>/fused_step_<workload>_traffic.json:
        --fetch: FETCH_SIZE, --write: WRITE_SIZE (KiB per dispatch), each
                 scaled by what it reads for the copy of known size;
        --sizes: TCC_EA0_RDREQ_32B/64B/128B, the read requests by size, which
                 show what the FETCH_SIZE scale stands for.
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
STEP_CLASSES = ("boundary", "interior", "two_level")


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


def run_step(workload: str, steps: int, temporal=None):
    sys.path.insert(0, ROOT)
    import torch
    import paper_2208_04371_amd as fd
    import workloads as W
    gen, _ = WORKLOADS[workload]
    prob = getattr(W, gen)()
    sim = fd.Simulation(prob, fused=True, temporal=temporal)
    sim.run(steps)
    torch.cuda.synchronize()
    rows, z = fd.fdtd_plan_get_config(sim.handle)
    tb = sim.temporal()
    sim.close()
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(COPY_REPS):
        fd.fdtd_device_copy(b, a)
    torch.cuda.synchronize()
    print(f"ran {steps} steps of {prob.name} (rows {rows}, zchunk {z}; two-level {tb}) and "
          f"{COPY_REPS} copies of {COPY_BYTES} B", flush=True)


def _rows(d: str, pattern: str):
    out = []
    for fn in glob.glob(os.path.join(d, "**", pattern), recursive=True):
        with open(fn, newline="") as f:
            out += list(csv.DictReader(f))
    return out


def _kernel_class(name: str) -> str:
    if re.search(r"\bk_tb<", name):
        return "two_level"
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
    """{class: (average counter value per dispatch, dispatches)}."""
    acc = {}
    for r in _rows(d, "*counter_collection.csv"):
        if r.get("Counter_Name") != counter:
            continue
        k = _kernel_class(r.get("Kernel_Name", ""))
        s, n = acc.get(k, (0.0, 0))
        acc[k] = (s + float(r["Counter_Value"]), n + 1)
    return {k: (s / n, n) for k, (s, n) in acc.items()}


def summarize(a):
    _, tag = WORKLOADS[a.workload]
    os.makedirs(a.out, exist_ok=True)
    stats = kernel_stats(a.stats)
    lines = [f"# rocprofv3 kernel statistics: fused step, {tag}", "",
             "command:", f"  {a.command}", "", f"sources: {source_hash()}", "",
             f"{'kernel':70s} {'calls':>6s} {'avg_us':>10s}"]
    total_us = 0.0
    per_class = {}
    for name, (calls, avg) in sorted(stats.items(), key=lambda kv: -kv[1][0] * kv[1][1]):
        short = name if len(name) <= 70 else name[:67] + "..."
        lines.append(f"{short:70s} {calls:6d} {avg / 1e3:10.3f}")
        c = _kernel_class(name)
        if c in STEP_CLASSES:
            total_us += calls * avg / 1e3
            per_class[c] = (calls, avg / 1e3)
    step_us = total_us / a.steps
    lines += ["", f"leapfrog steps profiled: {a.steps}"]
    for c in STEP_CLASSES:
        if c in per_class:
            lines.append(f"  {c:10s} launches {per_class[c][0]:6d}, average {per_class[c][1]:.3f} us")
    lines += [f"fused step (all field-update launches / steps): {step_us:.3f} us"]
    with open(os.path.join(a.out, f"fused_step_{tag}_stats.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    if not (a.fetch and a.write):
        return
    csteps = a.counter_steps or a.steps
    fetch = counter_per_class(a.fetch, "FETCH_SIZE")
    write = counter_per_class(a.write, "WRITE_SIZE")
    # each counter in KiB per dispatch; the copy moves COPY_BYTES each way
    kf = COPY_BYTES / (fetch["copy"][0] * 1024.0)
    kw = COPY_BYTES / (write["copy"][0] * 1024.0)
    per = {}
    for c in STEP_CLASSES:
        if c in fetch:
            per[c] = {"dispatches_per_step": fetch[c][1] / csteps,
                      "bytes_per_dispatch": round(fetch[c][0] * 1024.0 * kf +
                                                  write.get(c, (0.0, 0))[0] * 1024.0 * kw)}
    step_bytes = sum(v["bytes_per_dispatch"] * v["dispatches_per_step"] for v in per.values())
    d = {"workload": tag, "source_hash": source_hash(), "steps": csteps,
         "bytes_per_launch": round(step_bytes),
         "per_kernel": per,
         "fetch_kib": {k: round(v[0], 1) for k, v in fetch.items()},
         "write_kib": {k: round(v[0], 1) for k, v in write.items()},
         "copy_scale": {"fetch": kf, "write": kw}, "copy_bytes": COPY_BYTES,
         "command": a.command}
    if a.sizes:
        # read requests by size: the FETCH_SIZE scale of the copy holds for a
        # kernel whose reads are all of the copy's request size
        sz = {}
        for s in ("32B", "64B", "128B"):
            for k, (v, _) in counter_per_class(a.sizes, f"TCC_EA0_RDREQ_{s}_sum").items():
                sz.setdefault(k, {})[s] = v
        d["read_requests_per_dispatch"] = sz
        d["read_bytes_from_request_sizes"] = {
            k: round(v.get("32B", 0) * 32 + v.get("64B", 0) * 64 + v.get("128B", 0) * 128)
            for k, v in sz.items()}
    with open(os.path.join(a.out, f"fused_step_{tag}_traffic.json"), "w") as f:
        json.dump(d, f, indent=1)
        f.write("\n")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("step")
    s.add_argument("--workload", choices=sorted(WORKLOADS), default="microstrip")
    s.add_argument("--steps", type=int, default=200)
    s.add_argument("--temporal", type=int, default=None)
    m = sub.add_parser("summarize")
    m.add_argument("--workload", choices=sorted(WORKLOADS), default="microstrip")
    m.add_argument("--steps", type=int, required=True)
    m.add_argument("--counter-steps", type=int, default=0)
    m.add_argument("--stats", required=True)
    m.add_argument("--fetch")
    m.add_argument("--write")
    m.add_argument("--sizes")
    m.add_argument("--command", default="")
    m.add_argument("--out", default=os.path.join(ROOT, "profiles"))
    a = ap.parse_args()
    if a.cmd == "step":
        run_step(a.workload, a.steps, a.temporal)
    else:
        summarize(a)


if __name__ == "__main__":
    main()
