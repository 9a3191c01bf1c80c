"""The stored oracle runs under tests/golden (CPU only).

Every stored file must describe the problem its name stands for today (step
count, frequency grid, run names), so that a later change to a workload
cannot leave a GPU test comparing against a run of another problem; and a
stored run must come out of the committed oracle again: one run of the
smallest case is recomputed here and compared with the file.
"""
import glob
import json
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden")
sys.path.insert(0, GOLD)

import make_golden as MG  # noqa: E402


def _stored():
    out = {}
    for path in sorted(glob.glob(os.path.join(GOLD, "*_oracle.json"))):
        name = os.path.basename(path)[:-len("_oracle.json")]
        with open(path) as f:
            out[name] = json.load(f)
    return out


def _c(d):
    return np.asarray(d["re"]) + 1j * np.asarray(d["im"])


def test_stored_runs_describe_the_current_workloads():
    stored = _stored()
    assert stored, "no stored oracle runs"
    for name, g in stored.items():
        assert name in MG.CASES, name
        made = MG.CASES[name]()
        if name in MG.PROTOCOLS:
            runs = made
            first = runs["tot1"]
            for key, p in runs.items():
                assert g[key]["name"] == p.name and len(g[key]["V"]) == len(p.ports)
        elif name in MG.PAIRS:
            first = made[0]
            for key, p in zip(("p1", "p2"), made):
                assert g[key]["name"] == p.name and len(g[key]["V"]) == len(p.ports)
        else:
            first = made
            assert len(g["V"]) == len(first.ports)
        assert g["nsteps"] == first.nsteps, name
        assert np.array_equal(np.asarray(g["freqs"]), first.freqs), name
        if name in MG.FIELD_CASES:
            assert len(g["positions"]) == len(g["values"]) > 0
            assert [tuple(q) for q in g["positions"]] == \
                [tuple(q) for q in MG.field_positions(first)], name


def test_stored_run_reproduces_from_the_oracle():
    """The incident run of port 1 of the PEC step circuit driven by the
    1.5 fs pulse (96x40x28, 9000 steps): the oracle run now against the
    stored file (its sums run in a fixed order, so only the thread count
    could move the last bits; the bar is far below any kernel tolerance)."""
    name = "step_pulse_pec_1p5fs"
    path = os.path.join(GOLD, name + "_oracle.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written yet")
    with open(path) as f:
        g = json.load(f)
    import oracle
    p = MG.CASES[name]()["inc1"]
    o = oracle.Oracle(p).run(p.nsteps)
    V, I = o.spectra()
    Vs = np.array([_c(x) for x in g["inc1"]["V"]])
    Is = np.array([_c(x) for x in g["inc1"]["I"]])
    ev = np.max(np.abs(V - Vs)) / np.max(np.abs(Vs))
    ei = np.max(np.abs(I - Is)) / np.max(np.abs(Is))
    assert ev < 1e-12 and ei < 1e-12, (ev, ei)
