"""Two-level (temporally blocked) steps against single steps and the oracle.

A 256x64x48 microstrip has two-level tiles in its interior box (x 64..191,
y 8..55, z 0..39 with 6-cell absorbing layers); its source and both ports lie
inside that box, so the two-level pass also handles the source, the probe
tiles (whose intermediate level the probes read) and the bottom chunk on the
PEC ground.  The plan with two-level steps must match the same plan run by
single steps bit for bit, and the FP64 oracle to the FP32 bars, for several
two-level tile shapes, odd and even step counts, resumed runs and
checkpoints.
"""
import os

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


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


def _grid(nsteps, src_i=80, ports=(100, 180), sigma_strip=0.0):
    return W.small_microstrip(nx=256, ny=64, nz=48, strip_w=8, sub_top=12, pml=6, src_i=src_i,
                              ports=ports, nsteps=nsteps, nf=16, seed=7,
                              sigma_strip=sigma_strip)


def _run(fd, p, temporal, chunks, tcfg=None):
    sim = fd.Simulation(p, fused=True, temporal=temporal, temporal_config=tcfg)
    for n in chunks:
        sim.run(n)
    V, I = sim.spectra()
    F = [sim.field(c) for c in range(6)]
    info = sim.temporal()
    sim.close()
    return V, I, F, info


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _compare(got, ref, tol, tag, bitwise=False):
    Vg, Ig, Fg = got[:3]
    Vr, Ir, Fr = ref[:3]
    ev = float(np.max(np.abs(Vg - Vr)) / np.max(np.abs(Vr)))
    ei = float(np.max(np.abs(Ig - Ir)) / np.max(np.abs(Ir)))
    ef = []
    for grp in ((0, 1, 2), (3, 4, 5)):
        scale = np.sqrt(sum(np.sum(Fr[c] ** 2) for c in grp))
        ef += [float(np.linalg.norm(Fg[c] - Fr[c]) / scale) for c in grp]
    same = all(np.array_equal(Fg[c], Fr[c]) for c in range(6)) and np.array_equal(Vg, Vr)
    _say(f"  {tag}: spectra V {ev:.1e} I {ei:.1e}; fields (l2) " +
         " ".join(f"{e:.1e}" for e in ef) + ("; bitwise equal" if same else ""))
    assert ev < tol and ei < tol and max(ef) < tol
    if bitwise:
        assert same, "two-level steps differ from single steps in the last bits"


@pytest.mark.parametrize("tcfg", [(8, 32), (10, 4), (13, 16), (13, 32)],
                         ids=["r8z32", "r10z4", "r13z16", "r13z32"])
def test_two_level_equals_single_steps(fd, tcfg):
    """151 steps (75 two-level passes and a single step) against the plan
    run by single steps only: the same bits (both kernels pin the rounding
    of the update formulas)."""
    p = _grid(151)
    _say(f"two-level {tcfg} vs single steps, {p.nx}x{p.ny}x{p.nz}, {p.nsteps} steps")
    tb = _run(fd, p, 1, [p.nsteps], tcfg)
    mode, used, rows, zc, tiles = tb[3]
    _say(f"  two-level tiles {tiles} ({rows} rows, z-chunk {zc})")
    assert used == 1 and tiles > 0 and (rows, zc) == tcfg
    ref = _run(fd, p, 0, [p.nsteps])
    assert ref[3][1] == 0
    _compare(tb, ref, 1e-5, "two-level vs single", bitwise=True)


def test_two_level_matches_oracle(fd):
    """Every field and the port spectra after 120 steps against the FP64
    oracle (FP32 bars), with a lossy strip."""
    p = _grid(120, sigma_strip=5.8e7)
    _say(f"two-level vs oracle, {p.nsteps} steps")
    tb = _run(fd, p, 1, [p.nsteps])
    o = oracle.Oracle(p).run(p.nsteps)
    Vo, Io = o.spectra()
    ref = (Vo, Io, [o.field(c) for c in range(6)])
    _compare(tb, ref, 1e-4, "two-level vs oracle")


def test_two_level_source_and_ports_outside_the_box(fd):
    """Source and ports in boundary tiles (x 20, 30 and 230): the two-level
    tiles only see their waves."""
    p = _grid(101, src_i=20, ports=(30, 230))
    tb = _run(fd, p, 1, [p.nsteps])
    ref = _run(fd, p, 0, [p.nsteps])
    _compare(tb, ref, 1e-5, "outside the box", bitwise=True)


def test_two_level_resumed_and_checkpoint(fd):
    """Runs split 37 + 50 + 14 (odd splits change which steps are single)
    against one run of 101 steps; a checkpoint taken mid-run and resumed
    gives bitwise the uninterrupted run."""
    p = _grid(101)
    one = _run(fd, p, 1, [101])
    split = _run(fd, p, 1, [37, 50, 14])
    _compare(split, one, 1e-5, "split run", bitwise=True)
    sim = fd.Simulation(p, fused=True, temporal=1)
    sim.run(61)
    ck = sim.checkpoint()
    sim.run(40)
    Va, _ = sim.spectra()
    Fa = [sim.field(c) for c in range(6)]
    sim.restore(ck)
    sim.run(40)
    Vb, _ = sim.spectra()
    Fb = [sim.field(c) for c in range(6)]
    sim.close()
    assert np.array_equal(Va, Vb)
    for c in range(6):
        assert np.array_equal(Fa[c], Fb[c]), c


def test_two_level_not_used_where_no_tile_qualifies(fd):
    """A grid made of absorbing layers and their margins has no two-level
    tile: the plan still runs, by single steps, and matches the oracle."""
    p = W.small_microstrip(nsteps=60)      # 96x40x28, 8-cell layers
    tb = _run(fd, p, 1, [p.nsteps])
    assert tb[3][1] == 1 and tb[3][4] == 0
    o = oracle.Oracle(p).run(p.nsteps)
    Vo, Io = o.spectra()
    _compare(tb, (Vo, Io, [o.field(c) for c in range(6)]), 1e-4, "no two-level tiles")
