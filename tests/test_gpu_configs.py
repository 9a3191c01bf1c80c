"""The full-size workloads against the oracle's stored runs (tests/golden,
written by tests/golden/make_golden.py, which calls the CPU oracle only).

  * The 12-instance batched S-matrix (six strip widths times the two
    excitations of a 2-port, uneven y extents, one batch): the S-matrix of
    each strip width formed from its port-1 / port-2 excitation pair by the
    per-port protocol (Sec. II-A) through fdtd_sparams; the narrowest and
    widest pairs against the oracle's runs of the same pairs.
  * The 1024x512x256 layered lossy line over its first 2000 steps: port
    spectra and field values on both port planes and at seeded positions,
    from the plain FP64 kernels (to rounding) and the fused FP32 kernel
    (FP32 bars): the first link of the parity chain on that grid.

Bars (FP32): spectra 1e-4 of their largest value, |dS| <= 1e-3, Z0 and
delay within 0.5 %.  FP64 plain: 1e-10.
"""
import json
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def fd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2208_04371_amd import build as hb
    if not os.path.exists(hb.LIB):
        hb.build()
    import paper_2208_04371_amd as fd
    return fd


def _say(msg):
    print(msg, flush=True)


def _c(d):
    return np.asarray(d["re"]) + 1j * np.asarray(d["im"])


def _load(name):
    path = os.path.join(GOLD, name + "_oracle.json")
    if not os.path.exists(path):
        pytest.skip(f"stored oracle run missing: {path} (tests/golden/make_golden.py)")
    with open(path) as f:
        return json.load(f)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def pair_sparams(fd, freqs, run1, run2):
    """S-matrix of a uniform 2-port from the runs driven next to port 1 and
    next to port 2: on a uniform line each run is both the incident and
    the total run of its port (per-port protocol, Sec. II-A)."""
    sp = {"inc1": run1, "tot1": run1, "inc2": run2, "tot2": run2}
    return fd.fdtd_sparams(freqs, *fd.protocol_from_runs(sp))


def _compare_s(r, g, tag):
    ds_star = float(np.max(np.abs(r["S_star"] - _c(g["S_star"]))))
    ds = float(np.max(np.abs(r["S"] - _c(g["S"]))))
    dz0 = float(np.max(np.abs(r["Z0"] / _c(g["Z0"]) - 1)))
    gt = np.asarray(g["tau"])
    dtau = max(float(np.max(np.abs(r["tau"][:, 1, 0] / gt[:, 1, 0] - 1))),
               float(np.max(np.abs(r["tau"][:, 0, 1] / gt[:, 0, 1] - 1))))
    _say(f"  {tag}: |dS*| {ds_star:.1e} |dS| {ds:.1e} Z0 {dz0:.1e} tau {dtau:.1e}")
    return ds_star, ds, dz0, dtau


def test_batched_smatrix_pairs_match_stored_oracle(fd):
    """The 12-instance batch over its 20 000 steps (THz reading, autotuned
    launch shape): every strip width's S-matrix from its excitation pair;
    the w = 4 and w = 16 pairs against the oracle's runs of those pairs."""
    names = {4: "smatrix_w4_ny100_thz", 16: "smatrix_w16_ny140_thz"}
    golds = {w: _load(n) for w, n in names.items()}
    probs = W.batched_smatrix(twin=True)
    assert len(probs) == 12 and probs[0].nsteps == 20000
    _say(f"batched S-matrix, {len(probs)} instances, {probs[0].nsteps} steps")
    bs = fd.BatchSimulation(probs)
    bs.autotune(trial_steps=16)          # leaves the members reset
    _say(f"  launch shape {bs.get_config()}, groups {bs.groups()}")
    bs.run(probs[0].nsteps)
    spectra = [bs.spectra(q) for q in range(len(probs))]
    bs.close()
    freqs = probs[0].freqs
    for w_idx, w in enumerate(W.BATCH_WIDTHS):
        p1, p2 = probs[2 * w_idx], probs[2 * w_idx + 1]
        assert f"_w{w}_" in p1.name and p1.name.endswith("_p1") and p2.name.endswith("_p2")
        r = pair_sparams(fd, freqs, spectra[2 * w_idx], spectra[2 * w_idx + 1])
        s21 = np.abs(r["S_star"][:, 1, 0])
        _say(f"  w {w}: |S*21| {s21.min():.3f}..{s21.max():.3f}, "
             f"Re Z0 {r['Z0'].real.min():.1f}..{r['Z0'].real.max():.1f} ohm")
        # a passive uniform line: the wave reaches the far port, Z0 has a
        # positive real part, the delay is positive
        assert np.all(np.isfinite(r["S"])) and np.all(r["Z0"].real > 0)
        assert np.all(r["tau"][:, 1, 0] > 0) and np.all(r["tau"][:, 0, 1] > 0)
        if w not in golds:
            continue
        g = golds[w]
        assert np.array_equal(freqs, g["freqs"]) and g["nsteps"] == p1.nsteps
        for key, q in (("p1", 2 * w_idx), ("p2", 2 * w_idx + 1)):
            assert g[key]["name"] == probs[q].name
            V, I = spectra[q]
            ev = _rel(V, np.array([_c(x) for x in g[key]["V"]]))
            ei = _rel(I, np.array([_c(x) for x in g[key]["I"]]))
            _say(f"  w {w} {key}: spectra V {ev:.1e} I {ei:.1e}")
            assert ev < 1e-4 and ei < 1e-4
        ds_star, ds, dz0, dtau = _compare_s(r, g, f"w {w}")
        assert ds_star <= 1e-3 and ds <= 1e-3 and dz0 <= 5e-3 and dtau <= 5e-3


@pytest.mark.parametrize("kernel", ["fp64", "fused"])
def test_line_first_2000_steps_match_stored_oracle(fd, kernel):
    """The 1024x512x256 layered lossy line after 2000 steps, in the launch
    shape the benchmark times: port spectra and the stored field values
    (both port planes around the strip, seeded positions anywhere)."""
    g = _load("line_1024x512x256_2000")
    p = W.large_line(nsteps=2000)
    assert g["nsteps"] == p.nsteps and np.array_equal(p.freqs, g["freqs"])
    _say(f"line {p.nx}x{p.ny}x{p.nz}, {kernel}, {p.nsteps} steps")
    if kernel == "fused":
        sim = fd.Simulation(p, fused=True)
    else:
        sim = fd.Simulation(p, fused=False, precision=fd.FP64)
    sim.run()
    V, I = sim.spectra()
    ev = _rel(V, np.array([_c(x) for x in g["V"]]))
    ei = _rel(I, np.array([_c(x) for x in g["I"]]))
    pos = np.asarray(g["positions"], dtype=np.int64)
    ref = np.asarray(g["values"])
    got = np.zeros_like(ref)
    for c in range(6):
        sel = np.nonzero(pos[:, 0] == c)[0]
        f = sim.field(c)
        got[sel] = f[pos[sel, 3], pos[sel, 2], pos[sel, 1]]
        del f
    sim.close()
    errs = []
    for grp in ((0, 1, 2), (3, 4, 5)):
        sel = np.isin(pos[:, 0], grp)
        scale = np.max(np.abs(ref[sel]))
        assert scale > 0
        errs.append(float(np.max(np.abs(got[sel] - ref[sel])) / scale))
    _say(f"  spectra V {ev:.1e} I {ei:.1e}; fields E {errs[0]:.1e} H {errs[1]:.1e}")
    tol = 1e-10 if kernel == "fp64" else 1e-4
    assert ev < tol and ei < tol and max(errs) < tol


def test_line_long_run_fused_matches_plain_fp64(fd):
    """The second link of the parity chain on the 1024x512x256 line: the
    fused FP32 run (two-level steps, the benchmark's launch shape) against
    the plain FP64 kernels, which the first link ties to the oracle, over
    20 000 steps (the pulse has crossed the line; 2.7e12 cell updates):
    port spectra, and S*, Z0 and delay where both ports' spectra are within
    20 dB of their peaks."""
    p = W.large_line(nsteps=20000)
    out = {}
    for kernel in ("fused", "fp64"):
        _say(f"line {p.nx}x{p.ny}x{p.nz}, {kernel}, {p.nsteps} steps")
        if kernel == "fused":
            sim = fd.Simulation(p, fused=True)
            _say(f"  two-level {sim.temporal()}")
        else:
            sim = fd.Simulation(p, fused=False, precision=fd.FP64)
        sim.run()
        out[kernel] = sim.spectra()
        sim.close()
    (Vf, If), (Vd, Id) = out["fused"], out["fp64"]
    ev, ei = _rel(Vf, Vd), _rel(If, Id)
    rf = pair_sparams(fd, p.freqs, (Vf, If), (Vf[::-1], If[::-1]))
    rd = pair_sparams(fd, p.freqs, (Vd, Id), (Vd[::-1], Id[::-1]))
    strong = np.ones(len(p.freqs), bool)
    for q in range(2):
        a = np.abs(Vd[q])
        strong &= a > 0.1 * a.max()
    ds = float(np.max(np.abs(rf["S_star"][strong] - rd["S_star"][strong])))
    dz0 = float(np.max(np.abs(rf["Z0"][strong] / rd["Z0"][strong] - 1)))
    dtau = float(np.max(np.abs(rf["tau"][strong, 1, 0] / rd["tau"][strong, 1, 0] - 1)))
    _say(f"  spectra V {ev:.1e} I {ei:.1e}; over {strong.sum()} frequencies |dS*| {ds:.1e} "
         f"Z0 {dz0:.1e} tau {dtau:.1e}")
    assert strong.sum() >= 8
    assert ev < 1e-4 and ei < 1e-4
    assert ds <= 1e-3 and dz0 <= 5e-3 and dtau <= 5e-3
