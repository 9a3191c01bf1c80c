"""Precision chain on the 1024x512x256 lossy line over a full-length run.

The CPU oracle cannot run this grid for long (1.3e11 cell updates per 1000
steps), so the fused FP32 kernel is checked against the library's plain FP64
kernels, which the GPU tests tie to the oracle element by element.  Both
runs take the line's full 200 000 steps (the 10-300 THz band at 2 nm cells;
about 760 fs, long after the pulse has crossed the line and the lossy strip
has rung down) and are post-processed the same way (single-excitation
protocol of a uniform line, then S*, S at 50 ohm, Z0 and the delay).

The two runs do not fit one time-limited job, so each writes its spectra
and derived quantities to a JSON file and `compare` checks them (a run
stops early when its projected duration exceeds BUDGET_S seconds):

    python tests/long_line_chain.py run fp64 OUT64.json [BUDGET_S]
    python tests/long_line_chain.py run fp32 OUT32.json [BUDGET_S]
    python tests/long_line_chain.py compare OUT64.json OUT32.json

Bars: |dS*|, |dS| <= 1e-3 and Z0 within 0.5 % over the band, the delay
within 0.5 %.  Not collected by pytest (one run takes minutes).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

NSTEPS = 200_000
REPORT_EVERY = 10_000


def _c(a):
    a = np.asarray(a)
    return {"re": a.real.tolist(), "im": a.imag.tolist()}


def _uc(d):
    return np.asarray(d["re"]) + 1j * np.asarray(d["im"])


def run(prec: str, out: str, budget_s: float) -> None:
    import torch
    import paper_2208_04371_amd as fd
    from oracle import post
    import workloads as W

    p = W.large_line(nsteps=NSTEPS)
    fused = prec == "fp32"
    precision = fd.FP32 if fused else fd.FP64
    print(f"line {p.nx}x{p.ny}x{p.nz}, {prec} {'fused' if fused else 'plain'}, "
          f"{NSTEPS} steps", flush=True)
    sim = fd.Simulation(p, fused=fused, precision=precision)
    t0 = time.perf_counter()
    done = 0
    while done < NSTEPS:
        n = min(REPORT_EVERY, NSTEPS - done)
        sim.run(n)
        torch.cuda.synchronize()
        done += n
        el = time.perf_counter() - t0
        print(f"  step {done}  {el:.1f} s", flush=True)
        if el * NSTEPS / done > budget_s:
            sys.exit(f"projected {el * NSTEPS / done:.0f} s exceeds the {budget_s:.0f} s budget")
    V, I = sim.spectra()
    wall = time.perf_counter() - t0
    r = fd.fdtd_sparams(p.freqs, *post.single_excitation_protocol(V, I))
    cfg = sim.get_config() if fused else None
    sim.close()
    rec = {"precision": prec, "steps": NSTEPS, "wall_s": wall, "launch": cfg,
           "freqs": p.freqs.tolist(), "V": [_c(v) for v in V], "I": [_c(i) for i in I],
           "S_star": _c(r["S_star"]), "S": _c(r["S"]), "Z0": _c(r["Z0"]),
           "tau": np.asarray(r["tau"]).tolist()}
    with open(out, "w") as f:
        json.dump(rec, f)
    print(f"wrote {out} ({wall:.0f} s)", flush=True)


def compare(ref_path: str, test_path: str) -> int:
    with open(ref_path) as f:
        a = json.load(f)
    with open(test_path) as f:
        b = json.load(f)
    assert a["freqs"] == b["freqs"] and a["steps"] == b["steps"]
    ds_star = np.max(np.abs(_uc(a["S_star"]) - _uc(b["S_star"])))
    ds = np.max(np.abs(_uc(a["S"]) - _uc(b["S"])))
    z0a, z0b = _uc(a["Z0"]), _uc(b["Z0"])
    dz0 = np.max(np.abs(z0b / z0a - 1))
    # delay of S*21 (S*11 of the matched protocol is zero and has no phase)
    ta, tb = np.asarray(a["tau"])[:, 1, 0], np.asarray(b["tau"])[:, 1, 0]
    dtau = np.max(np.abs(tb / ta - 1))
    dv = max(np.max(np.abs(_uc(x) - _uc(y))) / np.max(np.abs(_uc(x)))
             for x, y in zip(a["V"], b["V"]))
    di = max(np.max(np.abs(_uc(x) - _uc(y))) / np.max(np.abs(_uc(x)))
             for x, y in zip(a["I"], b["I"]))
    s21 = np.abs(_uc(a["S_star"]))[:, 1, 0]
    print(f"{a['precision']} ({a['wall_s']:.0f} s) vs {b['precision']} ({b['wall_s']:.0f} s), "
          f"{a['steps']} steps")
    print(f"  spectra: max |dV|/max|V| {dv:.2e}, max |dI|/max|I| {di:.2e}")
    print(f"  |dS*| {ds_star:.2e}  |dS| {ds:.2e}  Z0 rel {dz0:.2e}  tau rel {dtau:.2e}")
    print(f"  |S*21| {s21.min():.4f}..{s21.max():.4f}, "
          f"Re Z0 {z0a.real.min():.2f}..{z0a.real.max():.2f} ohm, "
          f"tau {ta.min() * 1e15:.2f}..{ta.max() * 1e15:.2f} fs")
    ok = ds_star <= 1e-3 and ds <= 1e-3 and dz0 <= 5e-3 and dtau <= 5e-3
    print("PASS" if ok else "FAIL")
    return 0 if ok else 1


if __name__ == "__main__":
    if len(sys.argv) in (4, 5) and sys.argv[1] == "run" and sys.argv[2] in ("fp32", "fp64"):
        run(sys.argv[2], sys.argv[3], float(sys.argv[4]) if len(sys.argv) == 5 else 1e9)
    elif len(sys.argv) == 4 and sys.argv[1] == "compare":
        sys.exit(compare(sys.argv[2], sys.argv[3]))
    else:
        sys.exit(__doc__)
