"""Write stored oracle results for the full-size workloads.

Calls only the CPU oracle (oracle/) and the seeded problem descriptions
(workloads/).  Output: one JSON file per case next to this script with
the DFT spectra of every probe and, for the uniform lines, the oracle's S*,
S, Z_r, Z0 and delay.

Case kinds:
  * single runs (the 400x120x80 microstrip, sweep members): spectra, and
    for the uniform lines the S-matrix of the single-excitation protocol;
  * excitation pairs of the 12-instance S-matrix batch: the runs driven next
    to port 1 and next to port 2 of one strip width, their spectra and the
    S-matrix the per-port protocol (Sec. II-A) forms from the pair;
  * the 1024x512x256 line after its first steps: port spectra and field
    values at stored positions (both port planes around the strip, and a
    seeded sample of the whole grid);
  * the four runs of the step circuit's per-port protocol (the appendix's
    pulse-width check): every run's spectra and the resulting S-matrix.

    python tests/golden/make_golden.py [name ...]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from oracle import post  # noqa: E402
import workloads as W  # noqa: E402


def _pair(w, twin):
    ps = [p for p in W.batched_smatrix(twin=twin) if f"_w{w}_" in p.name]
    assert len(ps) == 2
    return ps


CASES = {
    "microstrip_400x120x80": lambda: W.single_microstrip(twin=False),
    "microstrip_400x120x80_thz": lambda: W.single_microstrip(twin=True),
    # the smallest and largest member of the 16-grid geometry sweep; their
    # inclusions make them non-uniform, so only the spectra are stored (an
    # S-matrix would need the runs of every excitation)
    "sweep_00_128x128x128": lambda: W.geometry_sweep()[0],
    "sweep_15_320x160x96": lambda: W.geometry_sweep()[15],
    # excitation pairs of the batched S-matrix workload (narrowest and widest
    # strip), THz band: 20 000 steps each run
    "smatrix_w4_ny100_thz": lambda: _pair(4, True),
    "smatrix_w16_ny140_thz": lambda: _pair(16, True),
    "smatrix_w4_ny100": lambda: _pair(4, False),
    # first 2000 steps of the 1024x512x256 layered lossy line
    "line_1024x512x256_2000": lambda: W.large_line(nsteps=2000),
    # the paper's own verification microstrip (Sec. II-B), 60 000 steps
    "paper_microstrip_1000x200x50": lambda: W.paper_microstrip(),
    # the appendix's pulse-width check on the step circuit: the four runs of
    # the per-port protocol driven by eq. 3 pulses of two widths, PEC strip
    # (9000 steps) and 5.8e7 S/m strip (36 000 steps)
    "step_pulse_pec_1p5fs": lambda: W.small_step_circuit(pulse_width=1.5e-15),
    "step_pulse_pec_2p25fs": lambda: W.small_step_circuit(pulse_width=2.25e-15),
    "step_pulse_lossy_1p5fs": lambda: W.small_step_circuit(pulse_width=1.5e-15, lossy=True),
    "step_pulse_lossy_2p25fs": lambda: W.small_step_circuit(pulse_width=2.25e-15, lossy=True),
}
SPECTRA_ONLY = {"sweep_00_128x128x128", "sweep_15_320x160x96"}
PAIRS = {"smatrix_w4_ny100_thz", "smatrix_w16_ny140_thz", "smatrix_w4_ny100"}
FIELD_CASES = {"line_1024x512x256_2000"}
PROTOCOLS = {"step_pulse_pec_1p5fs", "step_pulse_pec_2p25fs", "step_pulse_lossy_1p5fs",
             "step_pulse_lossy_2p25fs"}


def _c(z):
    z = np.asarray(z)
    return {"re": z.real.tolist(), "im": z.imag.tolist()}


def _run(name, p, t):
    o = oracle.Oracle(p)
    chunk = 1000 if p.ncells < 20_000_000 else 100
    while o.step < p.nsteps:
        o.run(min(chunk, p.nsteps - o.step))
        print(f"{name}/{p.name}: step {o.step}/{p.nsteps} ({time.time() - t:.0f} s)", flush=True)
    return o


def field_positions(p, seed=11, nrand=4096, pad=8, zwin=(88, 108)):
    """Positions (comp, i, j, k) stored for a field case: every component
    on both port planes over the strip's rows +- pad and the planes of
    zwin, then nrand seeded positions anywhere in the grid."""
    pos = []
    for q in p.ports:
        for c in range(6):
            for k in range(*zwin):
                for j in range(q.y0 - pad, q.y1 + pad):
                    pos.append((c, q.i, j, k))
    rng = np.random.default_rng(seed)
    for _ in range(nrand):
        c = int(rng.integers(0, 6))
        pos.append((c, int(rng.integers(0, p.nx)), int(rng.integers(0, p.ny)),
                    int(rng.integers(0, p.nz))))
    return pos


def make(name):
    t = time.time()
    made = CASES[name]()
    out = {"_about": f"FP64 CPU oracle results for {name} "
                     "(written by tests/golden/make_golden.py)."}
    if name in PROTOCOLS:
        spectra = {}
        for key, p in made.items():
            o = _run(name, p, t)
            V, I = o.spectra()
            spectra[key] = (V, I)
            out[key] = {"name": p.name, "V": [_c(v) for v in V], "I": [_c(i) for i in I]}
            out["dt"] = o.dt
            del o
        p1 = made["tot1"]
        r = post.sparams(p1.freqs, *post.protocol_from_runs(spectra))
        out.update({"nsteps": p1.nsteps, "freqs": p1.freqs.tolist(),
                    "S_star": _c(r["S_star"]), "S": _c(r["S"]), "Zr": _c(r["Zr"]),
                    "Z0": _c(r["Z0"]), "tau": r["tau"].tolist()})
    elif name in PAIRS:
        p1, p2 = made
        runs = {}
        for key, p in (("p1", p1), ("p2", p2)):
            o = _run(name, p, t)
            V, I = o.spectra()
            runs[key] = (V, I)
            out[key] = {"name": p.name, "V": [_c(v) for v in V], "I": [_c(i) for i in I]}
            out["dt"] = o.dt
            del o
        # a uniform line: incident and total runs coincide for each port
        sp = {"inc1": runs["p1"], "tot1": runs["p1"], "inc2": runs["p2"], "tot2": runs["p2"]}
        r = post.sparams(p1.freqs, *post.protocol_from_runs(sp))
        out.update({"nsteps": p1.nsteps, "freqs": p1.freqs.tolist(),
                    "S_star": _c(r["S_star"]), "S": _c(r["S"]), "Zr": _c(r["Zr"]),
                    "Z0": _c(r["Z0"]), "tau": r["tau"].tolist()})
    else:
        p = made
        o = _run(name, p, t)
        V, I = o.spectra()
        out.update({"nsteps": p.nsteps, "freqs": p.freqs.tolist(), "dt": o.dt,
                    "V": [_c(v) for v in V], "I": [_c(i) for i in I]})
        if name in FIELD_CASES:
            pos = field_positions(p)
            vals = [float(o.field(c)[k, j, i]) for (c, i, j, k) in pos]
            out["positions"] = pos
            out["values"] = vals
        elif name not in SPECTRA_ONLY:
            r = post.sparams(p.freqs, *post.single_excitation_protocol(V, I))
            out.update({"S_star": _c(r["S_star"]), "S": _c(r["S"]), "Zr": _c(r["Zr"]),
                        "Z0": _c(r["Z0"]), "tau": r["tau"].tolist()})
    out["seconds"] = time.time() - t
    out["threads"] = oracle.threads()
    tmp = os.path.join(HERE, f"{name}_oracle.json.tmp")
    with open(tmp, "w") as f:
        json.dump(out, f)
    os.replace(tmp, os.path.join(HERE, f"{name}_oracle.json"))
    print(f"{name}: done in {time.time() - t:.0f} s", flush=True)


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(CASES)):
        make(n)
