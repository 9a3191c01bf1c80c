"""Benchmark of the FDTD S-parameter hot path on one MI355X.

One benchmark step = one complete S-parameter run of the 400x120x80
microstrip (5 nm cells, silicon substrate, PEC ground and strip, 10-cell
absorbing layers, Gaussian-modulated sine at x = 20, probes at x = 60 and
x = 340, 64 frequencies 10-300 GHz): reset, 20000 fused FP32 leapfrog steps
with per-step port V/I sampling and FP64 running DFTs, spectra to the host
and the FP64 post-processing into S*, S(50 ohm), Z_r, Z0 and phase delay.
Inputs are resident on the GPU before the timed region starts.

Prints one JSON line (see the fields below).  Also measured and reported:
  * roofline: achieved bytes/s of the fused step kernel, from HIP events
    around every launch in the timed region, against 8 TB/s;
  * cpu_baseline: the FP64 CPU oracle on a bounded sample of the same grid;
  * variants: the plain FP64 and plain FP32 kernels on the same grid and the
    batched launch of the 12-instance S-matrix workload;
  * accuracy: S*/S/Z0 against stored oracle results when present.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "Mcell-updates/s and % of HBM peak, FP32/batched vs FP64 plain at |dS|<=1e-3"
HBM_PEAK_GBS = 8000.0
# step durations come from HIP events around windows of 16 consecutive
# steps (covering every step of the timed region): a pair of events around
# every step costs the host about a microstrip step's time and adds its own
# latency on the GPU, which would slow the timed runs themselves
TIMING_EVERY = 16
PROFILE_DIR = os.path.join(ROOT, "profiles")


def algorithmic_bytes(p, field_bytes=4, id_bytes=1, fused=True):
    """Bytes one leapfrog step must move for grid p: every field component
    read and written once (12 values per cell), three per-edge material ids,
    and for every absorbing-layer cell the four auxiliaries of that layer
    read and written.  Unfused H/E kernels re-read E (H pass) and H (E pass):
    18 field values per cell instead of 12."""
    cells = p.nx * p.ny * p.nz
    n = (p.nx, p.ny, p.nz)
    layer = 0
    for a in range(3):
        L = sum(p.pml_cells[2 * a + s] for s in (0, 1) if p.faces[2 * a + s] == 1)
        others = cells // n[a]
        layer += L * others
    vals = 12 if fused else 18
    return cells * (vals * field_bytes + 3 * id_bytes) + layer * 8 * field_bytes, cells, layer


def load_traffic(workload):
    """HBM-side bytes per fused step from the committed rocprofv3 counter
    summary, if it was taken on the current kernel sources."""
    from paper_2208_04371_amd.profiling import source_hash
    path = os.path.join(PROFILE_DIR, f"fused_step_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != source_hash():
        return None
    return d.get("bytes_per_launch")


def golden_accuracy(freqs, r):
    path = os.path.join(ROOT, "tests", "golden", "microstrip_400x120x80_oracle.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        g = json.load(f)
    c = lambda d: np.array(d["re"]) + 1j * np.array(d["im"])
    out = {
        "max_abs_dS_star": float(np.max(np.abs(r["S_star"] - c(g["S_star"])))),
        "max_abs_dS": float(np.max(np.abs(r["S"] - c(g["S"])))),
        "max_rel_dZ0": float(np.max(np.abs(r["Z0"] / c(g["Z0"]) - 1))),
        "reference": "FP64 CPU oracle, 20000 steps (tests/golden)",
    }
    return out


def stream_copy(fd, nbytes=1 << 30, reps=5):
    """The library's streaming copy of a known size (on torch's current
    stream): the practical bandwidth ceiling of the GPU and the calibration
    kernel of the counter-based traffic."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    fd.fdtd_device_copy(b, a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fd.fdtd_device_copy(b, a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * nbytes / (ms * 1e-3) / 1e9


def one_run(sim, fd, post_inputs):
    sim.reset()
    sim.run()
    V, I = sim.spectra()
    Vinc, Iinc, Vtot = post_inputs(V, I)
    return V, I, fd.fdtd_sparams(sim.prob.freqs, Vinc, Iinc, Vtot)


def protocol(V, I):
    # uniform mirror-symmetric line driven once at port 1: the port-2 run is
    # its mirror image, and incident and total runs coincide
    Vinc = np.stack([V[0], V[0]])
    Iinc = np.stack([I[0], I[0]])
    Vtot = np.stack([np.stack([V[0], V[1]]), np.stack([V[1], V[0]])])
    return Vinc, Iinc, Vtot


def measure_variant(fd, prob, fused, precision, steps):
    import torch
    sim = fd.Simulation(prob, fused=fused, precision=precision)
    sim.run(20)
    sim.reset()
    fd.fdtd_plan_set_timing(sim.handle, TIMING_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.run(steps)
    sim.spectra()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kms, launches = fd.fdtd_plan_get_kernel_time(sim.handle)
    sim.close()
    return dt, kms / max(launches, 1)


def cpu_baseline(prob, budget_s=15.0):
    import oracle
    o = oracle.Oracle(prob)
    t = time.perf_counter()
    o.run(5)
    per = (time.perf_counter() - t) / 5
    steps = max(5, int(budget_s / max(per, 1e-6)))
    steps = min(steps, prob.nsteps)
    t = time.perf_counter()
    o.run(steps)
    dt = time.perf_counter() - t
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": round(prob.ncells * steps / dt / 1e6, 3),
        "unit": "Mcell-updates/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{steps} of {prob.nsteps} leapfrog steps (after 5 warm-up steps) of the same "
                  f"{prob.nx}x{prob.ny}x{prob.nz} grid, FP64, probes and DFT included",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (the path runs "
              "one process on one GPU; sharding across GPUs is not built).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2208_04371_amd import build as hb
    if not os.path.exists(hb.LIB):
        hb.build()
    import paper_2208_04371_amd as fd
    import workloads as W

    torch.cuda.set_device(0)
    prob = W.single_microstrip(twin=False)
    copy_gbs = stream_copy(fd)

    sim = fd.Simulation(prob, fused=True)
    for _ in range(args.warmup):
        one_run(sim, fd, protocol)
    fd.fdtd_plan_set_timing(sim.handle, TIMING_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        V, I, res = one_run(sim, fd, protocol)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms, launches = fd.fdtd_plan_get_kernel_time(sim.handle)
    rows, zchunk = fd.fdtd_plan_get_config(sim.handle)
    sim.close()

    nsteps = prob.nsteps
    updates = prob.ncells * nsteps * args.steps
    value = updates / wall / 1e6
    bytes_launch, cells, layer_cells = algorithmic_bytes(prob)
    kavg_s = kms / max(launches, 1) * 1e-3
    achieved = bytes_launch / kavg_s / 1e9
    traffic = load_traffic("microstrip_400x120x80")

    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "microstrip_400x120x80 single 2-port run, fused FP32 fields + FP64 DFT",
            "cells": cells, "timesteps_per_run": nsteps, "frequencies": len(prob.freqs),
            "layer_cells": layer_cells, "tile_rows": rows, "zchunk": zchunk,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            # counted DRAM-side bytes (FETCH_SIZE + WRITE_SIZE, scaled by the
            # copy calibration) over the same event-timed step: the measured
            # fraction of peak (reads served by the memory-side cache count)
            "traffic_frac": (round(traffic / kavg_s / 1e9 / HBM_PEAK_GBS, 4)
                             if traffic else None),
            "kernel": "k_fused<R, layers>: one leapfrog step = boundary-tile launch + "
                      "interior-tile launch, timed together by HIP events on the run "
                      "stream around windows of 16 consecutive steps",
            "bytes_per_launch": bytes_launch,
            "avg_launch_us": round(kavg_s * 1e6, 3),
            "launches": launches,
            "stream_copy_GBs": round(copy_gbs, 1),
        },
    }
    acc = golden_accuracy(prob.freqs, res)
    if acc is not None:
        line["accuracy"] = acc

    if not args.no_variants:
        var = {}
        for name, fused, prec in (("fp64_plain", False, fd.FP64), ("fp32_plain", False, fd.FP32)):
            steps = 2000
            dt, kavg_ms = measure_variant(fd, prob, fused, prec, steps)
            vb, _, _ = algorithmic_bytes(prob, 8 if prec == fd.FP64 else 4, 1, fused=False)
            var[name] = {"value": round(prob.ncells * steps / dt / 1e6, 1),
                         "unit": "Mcell-updates/s", "timesteps": steps,
                         "avg_step_us": round(kavg_ms * 1e3, 2),
                         "hbm_frac": round(vb / (kavg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        probs = W.batched_smatrix(nsteps=2000)
        bs = fd.BatchSimulation(probs)
        # launch shape from the autotuner (searched outside the timed region;
        # it resets the members)
        bpick = bs.autotune(trial_steps=16)
        brows, bz = bs.get_config()
        border = bs.tile_order()
        bs.set_timing(TIMING_EVERY)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bs.run(2000)
        for q in range(len(probs)):
            bs.spectra(q)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        bms, _ = bs.kernel_time()
        groups = bs.groups()
        cells_b = sum(p.ncells for p in probs)
        bytes_b = sum(algorithmic_bytes(p)[0] for p in probs)
        # GPU time per batch step (with several groups, each group's launches
        # are timed as steps of their own)
        step_ms = bms / 2000
        var["batched_fp32_12x"] = {
            "value": round(cells_b * 2000 / dt / 1e6, 1), "unit": "Mcell-updates/s",
            "timesteps": 2000, "instances": len(probs), "cells": cells_b, "groups": groups,
            "autotuned": {"candidate": bpick, "tile_rows": brows, "zchunk": bz,
                          "tile_order": "automatic" if border[0] < 0 else border[0]},
            "avg_step_us": round(step_ms * 1e3, 2),
            "hbm_frac": round(bytes_b / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        bs.close()
        # the same twelve members run one after the other as single plans
        # (default launch shape each, kernel timer on as in the batch run),
        # for a like-for-like comparison
        solo = 0.0
        for p in probs:
            sim1 = fd.Simulation(p, fused=True)
            sim1.run(20)
            sim1.reset()
            fd.fdtd_plan_set_timing(sim1.handle, TIMING_EVERY)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            sim1.run(2000)
            sim1.spectra()
            torch.cuda.synchronize()
            solo += time.perf_counter() - t1
            sim1.close()
        var["batched_fp32_12x"]["members_one_at_a_time"] = {
            "value": round(cells_b * 2000 / solo / 1e6, 1), "unit": "Mcell-updates/s"}
        var["batched_fp32_12x"]["vs_members_one_at_a_time"] = round(solo / dt, 3)
        # the 16-instance geometry sweep of uneven shapes with its launch
        # shape chosen by the autotuner (no cache file: searched here, and
        # the search is outside the timed region)
        sp = W.geometry_sweep(nsteps=600)
        ss = fd.BatchSimulation(sp)
        pick = ss.autotune(trial_steps=16)
        srows, sz = ss.get_config()
        sorder = ss.tile_order()
        ss.set_timing(TIMING_EVERY)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ss.run(600)
        for q in range(len(sp)):
            ss.spectra(q)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        sms, _ = ss.kernel_time()
        cells_s = sum(p.ncells for p in sp)
        bytes_s = sum(algorithmic_bytes(p)[0] for p in sp)
        var["sweep_16x_autotuned"] = {
            "value": round(cells_s * 600 / dt / 1e6, 1), "unit": "Mcell-updates/s",
            "timesteps": 600, "instances": len(sp), "cells": cells_s, "groups": ss.groups(),
            "autotuned": {"candidate": pick, "tile_rows": srows, "zchunk": sz,
                          "tile_order": "automatic" if sorder[0] < 0 else sorder[0]},
            "avg_step_us": round(sms / 600 * 1e3, 2),
            "hbm_frac": round(bytes_s / (sms / 600 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        ss.close()
        # the 1024x512x256 layered lossy line: the grid far larger than the
        # caches, in its default launch shape
        lp = W.large_line(nsteps=300)
        dt, kavg_ms = measure_variant(fd, lp, True, fd.FP32, 300)
        lb, lcells, llayer = algorithmic_bytes(lp)
        ltraffic = load_traffic("line_1024x512x256")
        var["line_1024x512x256_fused"] = {
            "value": round(lp.ncells * 300 / dt / 1e6, 1), "unit": "Mcell-updates/s",
            "timesteps": 300, "cells": lcells, "layer_cells": llayer,
            "avg_step_us": round(kavg_ms * 1e3, 2), "bytes_per_step": lb,
            "achieved_GBs": round(lb / (kavg_ms * 1e-3) / 1e9, 1),
            "hbm_frac": round(lb / (kavg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": ltraffic,
            "traffic_frac": (round(ltraffic / (kavg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                             if ltraffic else None)}
        line["variants"] = var

    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
