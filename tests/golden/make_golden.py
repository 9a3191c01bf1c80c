"""Write stored oracle results for the full-size workloads.

Calls only the CPU oracle (oracle/) and the seeded problem descriptions
(workloads/).  Output: one JSON file per workload next to this script with
the DFT spectra of every probe and, for the uniform lines, the oracle's S*,
S, Z_r, Z0 and delay.

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

CASES = {
    "microstrip_400x120x80": lambda: W.single_microstrip(twin=False),
    "microstrip_400x120x80_thz": lambda: W.single_microstrip(twin=True),
    # the smallest and largest member of the 16-grid geometry sweep; their
    # inclusions make them non-uniform, so only the spectra are stored (an
    # S-matrix would need the runs of every excitation)
    "sweep_00_128x128x128": lambda: W.geometry_sweep()[0],
    "sweep_15_320x160x96": lambda: W.geometry_sweep()[15],
}
SPECTRA_ONLY = {"sweep_00_128x128x128", "sweep_15_320x160x96"}


def _c(z):
    z = np.asarray(z)
    return {"re": z.real.tolist(), "im": z.imag.tolist()}


def make(name):
    p = CASES[name]()
    t = time.time()
    o = oracle.Oracle(p)
    chunk = 1000
    while o.step < p.nsteps:
        o.run(min(chunk, p.nsteps - o.step))
        print(f"{name}: step {o.step}/{p.nsteps} ({time.time() - t:.0f} s)", flush=True)
    V, I = o.spectra()
    out = {
        "_about": f"FP64 CPU oracle results for {name} after {p.nsteps} steps "
                  "(written by tests/golden/make_golden.py).",
        "nsteps": p.nsteps, "freqs": p.freqs.tolist(), "dt": o.dt,
        "V": [_c(v) for v in V], "I": [_c(i) for i in I],
    }
    if name not in SPECTRA_ONLY:
        r = post.sparams(p.freqs, *post.single_excitation_protocol(V, I))
        out.update({"S_star": _c(r["S_star"]), "S": _c(r["S"]), "Zr": _c(r["Zr"]),
                    "Z0": _c(r["Z0"]), "tau": r["tau"].tolist()})
    out["seconds"] = time.time() - t
    with open(os.path.join(HERE, f"{name}_oracle.json"), "w") as f:
        json.dump(out, f)
    print(f"{name}: done in {time.time() - t:.0f} s", flush=True)


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(CASES)):
        make(n)
