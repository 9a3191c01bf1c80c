"""Benchmark of the FDTD S-parameter hot path on one MI355X.

One benchmark step = one run of the 1024x512x256 layered lossy line (2 nm
cells, 134.2 M cells: silicon/oxide layer stack below z = 96, a 32-cell
lossy metal strip of 5.8e7 S/m, PEC ground, 12-cell absorbing layers,
Gaussian-modulated sine at x = 24, ports at x = 64 and x = 960, 64
frequencies 10-300 THz) over 2000 steps: reset, 2000 fused FP32 leapfrog
steps with per-step port V/I sampling and FP64 running DFTs, spectra to the
host and the FP64 post-processing (S*, S at 50 ohm, Z_r, Z0, delay).  It is
the largest single-GPU workload, and its 7.6 GB state streams from HBM every
step (the 400x120x80 microstrip's fits the 256 MB memory-side cache).
Inputs are resident on the GPU before the timed region starts.

Prints one JSON line.  Besides the metric:
  * roofline: algorithmic bytes of one fused step over its duration from
    HIP events on the run stream (windows of 16 steps), against 8 TB/s;
    traffic: counted L2-to-memory bytes of the committed rocprofv3 counter
    runs (null once the kernel sources changed since they were taken);
  * accuracy: the timed run's port spectra against the oracle's stored run
    of the same 2000 steps, and the S-parameters of whole runs against the
    oracle's stored results;
  * variants: the same line by single steps and with the autotuner's
    launch shape and temporal-block depth, plain FP64 and plain FP32
    kernels on it (each fraction from the same single-pass algorithmic
    bytes), the 400x120x80 microstrip, the 12-instance batched S-matrix
    (20 000 steps; grouped, in lockstep, and its members run one at a time),
    the 16-instance sweep;
  * ceilings: streaming copies of 1 GiB (the library's kernel, torch's);
  * cpu_baseline: the FP64 CPU oracle on a bounded sample of the same line,
    on all host threads and on one;
  * paper: the paper's own throughput figure with its hardware (context).
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
GOLD = os.path.join(ROOT, "tests", "golden")
LINE_STEPS = 2000


def algorithmic_bytes(p, field_bytes=4, id_bytes=1, fields=12):
    """Bytes one leapfrog step must move for grid p in one pass: every
    field component read and written once (12 values per cell), three
    per-edge material ids, and for every absorbing-layer cell the four
    auxiliaries of that layer read and written (a cell in two layers counts
    twice).  fields=18: what two unfused H and E passes move (E re-read by
    the H pass, H by the E pass)."""
    cells = p.nx * p.ny * p.nz
    n = (p.nx, p.ny, p.nz)
    layer = 0
    for a in range(3):
        L = sum(p.pml_cells[2 * a + s] for s in (0, 1) if p.faces[2 * a + s] == 1)
        layer += L * (cells // n[a])
    return cells * (fields * field_bytes + 3 * id_bytes) + layer * 8 * field_bytes, cells, layer


def load_traffic(workload):
    """Counted bytes per fused step from the committed rocprofv3 counter
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


def _gold(name):
    path = os.path.join(GOLD, name + "_oracle.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def _c(d):
    return np.asarray(d["re"]) + 1j * np.asarray(d["im"])


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def s_errors(r, g):
    gt = np.asarray(g["tau"])
    return {
        "max_abs_dS_star": float(np.max(np.abs(r["S_star"] - _c(g["S_star"])))),
        "max_abs_dS": float(np.max(np.abs(r["S"] - _c(g["S"])))),
        "max_rel_dZ0": float(np.max(np.abs(r["Z0"] / _c(g["Z0"]) - 1))),
        "max_rel_dtau": float(np.max(np.abs(r["tau"][:, 1, 0] / gt[:, 1, 0] - 1))),
    }


def spectra_errors(V, I, g, key=None):
    src = g if key is None else g[key]
    return {"V": _rel(V, np.array([_c(x) for x in src["V"]])),
            "I": _rel(I, np.array([_c(x) for x in src["I"]]))}


def copy_ceilings(fd, nbytes=1 << 30, reps=5):
    """GB/s of streaming copies of a known size on torch's current stream:
    the library's copy kernel (also the calibration kernel of the counter
    traffic) and torch's device-to-device copy."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    out = {}
    for name, fn in (("fdtd_device_copy", lambda: fd.fdtd_device_copy(b, a)),
                     ("torch_copy", lambda: b.copy_(a))):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = round(2 * nbytes / (ms * 1e-3) / 1e9, 1)
    del a, b
    return out


def timed_plan_run(fd, sim, steps):
    """Reset, `steps` steps, spectra: wall seconds and the event-timed
    average step (ms)."""
    import torch
    sim.reset()
    fd.fdtd_plan_set_timing(sim.handle, TIMING_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.run(steps)
    V, I = sim.spectra()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kms, launches = fd.fdtd_plan_get_kernel_time(sim.handle)
    return dt, kms / max(launches, 1), V, I


def measure_plain(fd, prob, precision, steps):
    sim = fd.Simulation(prob, fused=False, precision=precision)
    sim.run(10)
    dt, kavg_ms, V, I = timed_plan_run(fd, sim, steps)
    sim.close()
    fb = 8 if precision == fd.FP64 else 4
    one, _, _ = algorithmic_bytes(prob, fb)
    two, _, _ = algorithmic_bytes(prob, fb, fields=18)
    s = kavg_ms * 1e-3
    return {"value": round(prob.ncells * steps / dt / 1e6, 1), "unit": "Mcell-updates/s",
            "timesteps": steps, "avg_step_us": round(kavg_ms * 1e3, 2),
            "bytes_per_step": one,
            "hbm_frac": round(one / s / 1e9 / HBM_PEAK_GBS, 4),
            "unfused_bytes_per_step": two,
            "unfused_bytes_frac": round(two / s / 1e9 / HBM_PEAK_GBS, 4)}, V, I


def cpu_baseline(prob, budget_s=12.0):
    """The FP64 oracle as it stands on a bounded sample of the same grid:
    a few leapfrog steps (probes and DFT included) on every host thread
    after one untimed step, then one step on one thread.  Set-up
    (coefficients, tables) is not timed."""
    import oracle
    o = oracle.Oracle(prob)
    nthreads = oracle.threads()
    t = time.perf_counter()
    o.run(1)
    per = time.perf_counter() - t
    steps = max(1, min(int(budget_s / max(per, 1e-6)), 50))
    t = time.perf_counter()
    o.run(steps)
    rate = prob.ncells * steps / (time.perf_counter() - t) / 1e6
    oracle.set_threads(1)
    t = time.perf_counter()
    o.run(1)
    rate1 = prob.ncells / (time.perf_counter() - t) / 1e6
    oracle.set_threads(nthreads)
    del o
    return {
        "value": round(rate, 3), "unit": "Mcell-updates/s", "cores": nthreads, "kind": "oracle",
        "single_thread_value": round(rate1, 3),
        "sample": f"{steps} leapfrog steps on {nthreads} threads (after one untimed step), then "
                  f"one step on 1 thread, of the same {prob.nx}x{prob.ny}x{prob.nz} line, FP64, "
                  "probes and DFT included; threads from omp_get_max_threads",
    }


PAPER = {
    "value": 182.0, "unit": "Mcell-updates/s",
    "hardware": "one Perlmutter node, 4x NVIDIA A100",
    "workload": "CMOS transmission line, 200x120x800 = 19.2 M cells, 1.4 M steps in 41 h "
                "(Sec. III; per-run wall time), precision not stated",
    "derived": "19.2e6 cells x 1.4e6 steps / (41 x 3600 s)",
    "note": "context only: another machine, workload and (unstated) precision",
}


def bench_batch(fd, W, torch):
    """The 12-instance S-matrix (THz band) over its 20 000 steps, autotuned
    launch shape, S per strip width from each excitation pair; then the same
    members one at a time as single plans."""
    probs = W.batched_smatrix(twin=True)
    nsteps = probs[0].nsteps
    bs = fd.BatchSimulation(probs)
    # outside the timed region; resets.  The search covers the schedule
    # (grouped under the cache-sized budget, or lockstep) and the launch
    # shape; 64 trial steps because a grouped trial runs each group's steps
    # in turn and a group's first steps refill the memory-side cache
    pick = bs.autotune(trial_steps=64)
    rows, zc = bs.get_config()
    order = bs.tile_order()
    bs.set_timing(TIMING_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bs.run(nsteps)
    spectra = [bs.spectra(q) for q in range(len(probs))]
    res = []
    for w_idx in range(len(W.BATCH_WIDTHS)):
        sp = {"inc1": spectra[2 * w_idx], "tot1": spectra[2 * w_idx],
              "inc2": spectra[2 * w_idx + 1], "tot2": spectra[2 * w_idx + 1]}
        res.append(fd.fdtd_sparams(probs[0].freqs, *fd.protocol_from_runs(sp)))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    bms, _ = bs.kernel_time()
    groups = bs.groups()
    bs.close()
    cells = sum(p.ncells for p in probs)
    nbytes = sum(algorithmic_bytes(p)[0] for p in probs)
    step_ms = bms / nsteps
    out = {"value": round(cells * nsteps / dt / 1e6, 1), "unit": "Mcell-updates/s",
           "timesteps": nsteps, "instances": len(probs), "cells": cells, "groups": groups,
           "schedule": "lockstep" if groups == 1 else "grouped",
           "autotuned": {"candidate": pick, "tile_rows": rows, "zchunk": zc,
                         "tile_order": "automatic" if order[0] < 0 else order[0]},
           "avg_step_us": round(step_ms * 1e3, 2),
           "hbm_frac": round(nbytes / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "s_matrices": len(res)}
    acc = {}
    widths = list(W.BATCH_WIDTHS)
    for w, name in ((4, "smatrix_w4_ny100_thz"), (16, "smatrix_w16_ny140_thz")):
        g = _gold(name)
        if g is not None:
            acc[f"w{w}"] = s_errors(res[widths.index(w)], g)
    if acc:
        acc["reference"] = "FP64 CPU oracle runs of the same excitation pairs (tests/golden)"
        out["accuracy"] = acc
    # the same batch in lockstep: one launch pair per step over all twelve
    # members (one group), autotuned for that schedule
    lk = fd.BatchSimulation(probs)
    lk.set_group_bytes(0)
    lpick = lk.autotune(trial_steps=64)
    lrows, lzc = lk.get_config()
    lk.set_timing(TIMING_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lk.run(nsteps)
    for q in range(len(probs)):
        lk.spectra(q)
    torch.cuda.synchronize()
    dl = time.perf_counter() - t0
    lms, _ = lk.kernel_time()
    lgroups = lk.groups()
    lk.close()
    out["lockstep"] = {"value": round(cells * nsteps / dl / 1e6, 1), "unit": "Mcell-updates/s",
                       "groups": lgroups, "avg_step_us": round(lms / nsteps * 1e3, 2),
                       "autotuned": {"candidate": lpick, "tile_rows": lrows, "zchunk": lzc}}
    solo = 0.0
    for p in probs:
        sim = fd.Simulation(p, fused=True)
        sim.run(10)
        d1, _, _, _ = timed_plan_run(fd, sim, nsteps)
        solo += d1
        sim.close()
    out["members_one_at_a_time"] = {"value": round(cells * nsteps / solo / 1e6, 1),
                                    "unit": "Mcell-updates/s"}
    out["vs_members_one_at_a_time"] = round(solo / dt, 3)
    return out


def bench_sweep(fd, W, torch, nsteps=600):
    sp = W.geometry_sweep(nsteps=nsteps)
    ss = fd.BatchSimulation(sp)
    pick = ss.autotune(trial_steps=64)     # schedule and shape, as for the S-matrix batch
    rows, zc = ss.get_config()
    order = ss.tile_order()
    ss.set_timing(TIMING_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ss.run(nsteps)
    for q in range(len(sp)):
        ss.spectra(q)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sms, _ = ss.kernel_time()
    groups = ss.groups()
    ss.close()
    cells = sum(p.ncells for p in sp)
    nbytes = sum(algorithmic_bytes(p)[0] for p in sp)
    return {"value": round(cells * nsteps / dt / 1e6, 1), "unit": "Mcell-updates/s",
            "timesteps": nsteps, "instances": len(sp), "cells": cells, "groups": groups,
            "schedule": "lockstep" if groups == 1 else "grouped",
            "autotuned": {"candidate": pick, "tile_rows": rows, "zchunk": zc,
                          "tile_order": "automatic" if order[0] < 0 else order[0]},
            "avg_step_us": round(sms / nsteps * 1e3, 2),
            "hbm_frac": round(nbytes / (sms / nsteps * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def bench_microstrip(fd, W, torch):
    """The 400x120x80 microstrip, whole 20 000-step runs in both readings,
    S-parameters against the oracle's stored runs."""
    out = {}
    for twin in (True, False):
        p = W.single_microstrip(twin=twin)
        sim = fd.Simulation(p, fused=True)
        sim.run(10)
        dt, kavg_ms, V, I = timed_plan_run(fd, sim, p.nsteps)
        sim.close()
        r = fd.fdtd_sparams(p.freqs, *fd.protocol_from_runs(
            {"inc1": (V, I), "tot1": (V, I), "inc2": (V[::-1], I[::-1]),
             "tot2": (V[::-1], I[::-1])}))
        b, cells, layer = algorithmic_bytes(p)
        e = {"value": round(cells * p.nsteps / dt / 1e6, 1), "unit": "Mcell-updates/s",
             "timesteps": p.nsteps, "avg_step_us": round(kavg_ms * 1e3, 2),
             "bytes_per_step": b,
             "hbm_frac": round(b / (kavg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        g = _gold(p.name)
        if g is not None:
            e["accuracy"] = s_errors(r, g)
            e["accuracy"]["reference"] = "FP64 CPU oracle, 20000 steps (tests/golden)"
            if not twin:
                e["accuracy"]["note"] = ("GHz band on 5 nm cells: the pulse stays in its "
                                         "leading tail for the whole run, so this checks that "
                                         "the sums agree, not the S-parameters of a developed "
                                         "pulse")
        out["microstrip_400x120x80" + ("_thz" if twin else "_ghz")] = e
    return out


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
        raise SystemExit(f"{hb.LIB} is not built: run `python __graft_entry__.py build` first")
    import paper_2208_04371_amd as fd
    import workloads as W

    torch.cuda.set_device(0)
    prob = W.large_line(nsteps=LINE_STEPS)
    ceilings = copy_ceilings(fd)

    sim = fd.Simulation(prob, fused=True)
    for _ in range(args.warmup):
        sim.reset()
        sim.run()
        sim.spectra()
    fd.fdtd_plan_set_timing(sim.handle, TIMING_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sim.reset()
        sim.run()
        V, I = sim.spectra()
        res = fd.fdtd_sparams(prob.freqs, *fd.protocol_from_runs(
            {"inc1": (V, I), "tot1": (V, I), "inc2": (V[::-1], I[::-1]),
             "tot2": (V[::-1], I[::-1])}))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms, launches = fd.fdtd_plan_get_kernel_time(sim.handle)
    rows, zchunk = fd.fdtd_plan_get_config(sim.handle)
    order = fd.fdtd_plan_get_tile_order(sim.handle)
    sstores = fd.fdtd_plan_get_stream_stores(sim.handle)
    tmode, tused, trows, tzc, ttiles = sim.temporal()
    sim.close()
    assert np.all(np.isfinite(V)) and res is not None

    updates = prob.ncells * LINE_STEPS * args.steps
    value = updates / wall / 1e6
    bytes_step, cells, layer_cells = algorithmic_bytes(prob)
    kavg_s = kms / max(launches, 1) * 1e-3
    achieved = bytes_step / kavg_s / 1e9
    traffic = load_traffic("line_1024x512x256")

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
            "workload": "line_1024x512x256: 2 nm layered lossy line, 2000-step run, "
                        "fused FP32 fields + FP64 probes/DFT/post",
            "cells": cells, "timesteps_per_run": LINE_STEPS, "frequencies": len(prob.freqs),
            "layer_cells": layer_cells, "tile_rows": rows, "zchunk": zchunk,
            "tile_order": order[1], "stream_stores": sstores[1],
            "two_level": {"used": bool(tused and ttiles > 0), "tiles": ttiles,
                          "tile": [60, trows, tzc]},
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            # counted L2-to-memory bytes (FETCH_SIZE + WRITE_SIZE scaled by
            # the copy calibration) over the same event-timed step; they
            # include halo over-fetch and reads served by the memory-side
            # cache, so this is not a DRAM fraction
            "counted_frac": (round(traffic / kavg_s / 1e9 / HBM_PEAK_GBS, 4)
                             if traffic else None),
            "kernel": "one leapfrog step: with two-level steps a pair of steps is the "
                      "boundary-tile launch k_fused<R, true>, the two-level launch k_tb "
                      "over the interior tiles and k_fused<R, true> again, timed together "
                      "by HIP events on the run stream around windows of 16 consecutive "
                      "steps; achieved = the single-pass algorithmic bytes of a step over "
                      "the step time (the effective rate: a two-level pass moves the "
                      "interior's fields once for two steps)",
            "bytes_per_launch": bytes_step,
            "avg_launch_us": round(kavg_s * 1e6, 3),
            "launches": launches,
            "copy_ceiling_GBs": ceilings,
        },
        "paper": PAPER,
    }
    g = _gold("line_1024x512x256_2000")
    if g is not None:
        line["accuracy"] = {"line_2000_spectra_vs_oracle": spectra_errors(V, I, g),
                            "reference": "FP64 CPU oracle run of the same 2000 steps "
                                         "(tests/golden)"}

    if not args.no_variants:
        var = {}
        # the same runs by single steps only: the fraction of the single-pass
        # fused kernel
        sim = fd.Simulation(prob, fused=True, temporal=0)
        sim.run(10)
        d1, k1, V1, I1 = timed_plan_run(fd, sim, LINE_STEPS)
        sim.close()
        var["line_fused_single_steps"] = {
            "value": round(prob.ncells * LINE_STEPS / d1 / 1e6, 1), "unit": "Mcell-updates/s",
            "timesteps": LINE_STEPS, "avg_step_us": round(k1 * 1e3, 2),
            "bytes_per_step": bytes_step,
            "hbm_frac": round(bytes_step / (k1 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        if g is not None:
            var["line_fused_single_steps"]["spectra_vs_oracle"] = spectra_errors(V1, I1, g)
        # launch shape and temporal-block depth chosen by the autotuner
        # (first stage: rows x z-chunk x order; second: two-level tile
        # shapes and single steps)
        sim = fd.Simulation(prob, fused=True)
        t_tune = time.perf_counter()
        best = sim.autotune(trial_steps=16)
        t_tune = time.perf_counter() - t_tune
        da, ka, Va, Ia = timed_plan_run(fd, sim, LINE_STEPS)
        ar, az = fd.fdtd_plan_get_config(sim.handle)
        ao = fd.fdtd_plan_get_tile_order(sim.handle)
        _, aused, atr, atz, atiles = sim.temporal()
        sim.close()
        var["line_autotuned"] = {
            "value": round(prob.ncells * LINE_STEPS / da / 1e6, 1), "unit": "Mcell-updates/s",
            "timesteps": LINE_STEPS, "avg_step_us": round(ka * 1e3, 2),
            "hbm_frac": round(bytes_step / (ka * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "choice": {"index": best, "tile_rows": ar, "zchunk": az, "tile_order": ao[1],
                       "two_level": {"used": bool(aused and atiles > 0), "tiles": atiles,
                                     "tile": [60, atr, atz]}},
            "search_s": round(t_tune, 2)}
        if g is not None:
            var["line_autotuned"]["spectra_vs_oracle"] = spectra_errors(Va, Ia, g)
        for name, prec in (("line_fp64_plain", fd.FP64), ("line_fp32_plain", fd.FP32)):
            e, Vp, Ip = measure_plain(fd, prob, prec, LINE_STEPS)
            if g is not None:
                e["spectra_vs_oracle"] = spectra_errors(Vp, Ip, g)
            var[name] = e
        var.update(bench_microstrip(fd, W, torch))
        var["batched_smatrix_12x"] = bench_batch(fd, W, torch)
        var["sweep_16x_autotuned"] = bench_sweep(fd, W, torch)
        line["variants"] = var

    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
