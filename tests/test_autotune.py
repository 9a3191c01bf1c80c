"""Launch-shape autotuner of batches and single fused plans (the tile height
x z-chunk search with its JSON cache keyed by GPU architecture and grid
shapes)."""
import json
import os

import numpy as np
import pytest

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


def _probs():
    return [W.small_microstrip(nsteps=60, ny=36 + 4 * q, seed=q) for q in range(3)]


def test_autotune_picks_caches_and_resets(fd, tmp_path):
    cache = str(tmp_path / "tune.json")
    bs = fd.BatchSimulation(_probs())
    best = bs.autotune(trial_steps=3, cache_path=cache)
    rows, z = bs.get_config()
    print("autotune picked", best, rows, z, flush=True)
    assert best >= 0
    assert rows in (2, 4, 8, 12, 16) and z in (4, 8, 16, 32, 64)
    # the cache holds one entry for this device and these member shapes
    with open(cache) as f:
        entries = json.load(f)
    assert len(entries) == 1
    (key, val), = entries.items()
    assert key.endswith("96x36x28;96x40x28;96x44x28;")
    order = bs.tile_order()[0]
    assert order in (-1, 16)
    assert val[:2] == [rows, z] and val[2] > 0 and val[3] == order
    # the members were reset: a run now equals a fresh batch in that shape
    bs.run(60)
    ref = fd.BatchSimulation(_probs(), config=(rows, z))
    ref.run(60)
    for q in range(3):
        assert np.array_equal(bs.field(q, W.EZ), ref.field(q, W.EZ))
        Va, Ia = bs.spectra(q)
        Vb, Ib = ref.spectra(q)
        assert np.array_equal(Va, Vb) and np.array_equal(Ia, Ib)
    # a second batch of the same shapes takes the cached choice untimed
    again = fd.BatchSimulation(_probs())
    assert again.autotune(trial_steps=3, cache_path=cache) == -1
    assert again.get_config() == (rows, z) and again.tile_order()[0] == order
    for x in (bs, ref, again):
        x.close()


def test_plan_autotune_picks_caches_and_resets(fd, tmp_path):
    cache = str(tmp_path / "tune.json")
    p = W.small_microstrip(nsteps=60, ny=40, seed=5)
    sim = fd.Simulation(p, fused=True)
    sim.run(7)                       # the search starts from any state
    best = sim.autotune(trial_steps=3, cache_path=cache)
    rows, z = sim.get_config()
    print("plan autotune picked", best, rows, z, flush=True)
    assert 0 <= best < 50
    assert rows in (2, 4, 8, 12, 16) and z in (4, 8, 16, 32, 64)
    order = sim.tile_order()[0]
    assert order in (-1, 16) and best % 2 == (order == 16)
    assert sim.step == 0
    with open(cache) as f:
        entries = json.load(f)
    (key, val), = entries.items()
    assert key.endswith("|96x40x28;")
    assert val[:2] == [rows, z] and val[2] > 0 and val[3] == order
    # the plan was reset: a run now equals a fresh plan in that shape
    sim.run()
    ref = fd.Simulation(p, fused=True, config=(rows, z))
    ref.set_tile_order(order)
    ref.run()
    assert np.array_equal(sim.field(W.EZ), ref.field(W.EZ))
    Va, Ia = sim.spectra()
    Vb, Ib = ref.spectra()
    assert np.array_equal(Va, Vb) and np.array_equal(Ia, Ib)
    # a one-member batch of the same shape shares the cache entry
    bs = fd.BatchSimulation([p])
    assert bs.autotune(trial_steps=3, cache_path=cache) == -1
    assert bs.get_config() == (rows, z) and bs.tile_order()[0] == order
    # plain kernels have no launch shape to tune
    plain = fd.Simulation(p, fused=False)
    with pytest.raises(fd.FdtdError) as e:
        plain.autotune(trial_steps=3)
    assert e.value.code == -3
    for x in (sim, ref, bs, plain):
        x.close()


def _tb_grid(nsteps):
    # the 256x64x48 microstrip whose interior box holds two-level tiles
    return W.small_microstrip(nx=256, ny=64, nz=48, strip_w=8, sub_top=12, pml=6, src_i=80,
                              ports=(100, 180), nsteps=nsteps, nf=16, seed=7)


def test_plan_autotune_chooses_temporal_depth(fd, tmp_path):
    """A plan with two-level steps: the search also times two-level tile
    shapes and single steps (12 + 1 candidates after the first stage).
    Whatever it picks, the run equals the plan run by single steps bit for
    bit, and a second plan of the same shape takes the cached choice,
    depth and two-level shape included."""
    cache = str(tmp_path / "tune.json")
    p = _tb_grid(151)
    sim = fd.Simulation(p, fused=True, temporal=1)
    sim.run(5)
    best = sim.autotune(trial_steps=4, cache_path=cache)
    rows, z = sim.get_config()
    order = sim.tile_order()[0]
    mode, used, tbr, tbz, tiles = sim.temporal()
    i1, i2 = best % 50, best // 50
    print(f"plan autotune picked {best}: rows {rows} z {z} order {order}; two-level "
          f"used {used} ({tbr} x {tbz}, {tiles} tiles)", flush=True)
    assert 0 <= best < 50 * 13 and sim.step == 0
    assert best % 2 == (order == 16)
    if i2 == 12:
        assert used == 0 and tiles == 0          # single steps chosen
    else:
        assert used == 1 and (tbr, tbz) == ((8, 10, 13)[i2 // 4], (8, 16, 32, 64)[i2 % 4])
    with open(cache) as f:
        entries = json.load(f)
    (key, val), = entries.items()
    assert key.endswith("|256x64x48;two-level")
    assert val[:2] == [rows, z] and val[3] == order
    assert val[4] == (1 if i2 == 12 else 2) and val[5:7] == [tbr, tbz] and val[7] == 0
    sim.run()
    ref = fd.Simulation(p, fused=True, temporal=0, config=(rows, z))
    ref.set_tile_order(order)
    ref.run()
    for c in range(6):
        assert np.array_equal(sim.field(c), ref.field(c)), c
    Va, Ia = sim.spectra()
    Vb, Ib = ref.spectra()
    assert np.array_equal(Va, Vb) and np.array_equal(Ia, Ib)
    # the cached choice, applied untimed
    again = fd.Simulation(p, fused=True, temporal=1)
    assert again.autotune(trial_steps=4, cache_path=cache) == -1
    assert again.get_config() == (rows, z) and again.tile_order()[0] == order
    assert again.temporal()[1:4] == (used, tbr, tbz)
    # a tile shape set by the caller brings two-level passes back
    fd.fdtd_plan_set_temporal_config(again.handle, 13, 16)
    assert again.temporal()[1:4] == (1, 13, 16)
    for x in (sim, ref, again):
        x.close()


def test_batch_autotune_chooses_the_schedule(fd, tmp_path):
    """A batch split into groups (a 1-byte budget: one member per group):
    the search times every shape grouped and in lockstep (100 candidates)
    and applies the winner's schedule; results equal the single runs bit for
    bit either way, and the cached choice brings the schedule back."""
    cache = str(tmp_path / "tune.json")
    probs = _probs()
    bs = fd.BatchSimulation(probs)
    bs.set_group_bytes(1)
    assert bs.groups() == 3
    best = bs.autotune(trial_steps=8, cache_path=cache)
    rows, z = bs.get_config()
    lock = best // 50
    print(f"batch autotune picked {best}: {'lockstep' if lock else 'grouped'}, rows {rows} "
          f"z {z}", flush=True)
    assert 0 <= best < 100
    assert bs.groups() == (1 if lock else 3)
    with open(cache) as f:
        entries = json.load(f)
    (key, val), = entries.items()
    assert key.endswith("96x36x28;96x40x28;96x44x28;groups=3;")
    assert val[:2] == [rows, z] and val[7] == lock
    bs.run(60)
    for q, p in enumerate(probs):
        ref = fd.Simulation(p, fused=True, config=(rows, z))
        ref.run(60)
        assert np.array_equal(bs.field(q, W.EZ), ref.field(W.EZ))
        Va, Ia = bs.spectra(q)
        Vb, Ib = ref.spectra()
        assert np.array_equal(Va, Vb) and np.array_equal(Ia, Ib)
        ref.close()
    again = fd.BatchSimulation(probs)
    again.set_group_bytes(1)
    assert again.autotune(trial_steps=8, cache_path=cache) == -1
    assert again.get_config() == (rows, z) and again.groups() == bs.groups()
    # a budget set by the caller takes the schedule back from the autotuner
    again.set_group_bytes(1)
    assert again.groups() == 3
    for x in (bs, again):
        x.close()


def test_autotune_cache_entries_bad_and_old(fd, tmp_path):
    """The cache is a file anyone can edit: an entry whose values are out of
    range is ignored (the search runs and rewrites it), and an entry in the
    older four-value form (rows, z-chunk, ms, order) still applies, with the
    other fields at their defaults."""
    cache = str(tmp_path / "tune.json")
    p = W.small_microstrip(nsteps=30, ny=40, seed=5)
    sim = fd.Simulation(p, fused=True)
    assert sim.autotune(trial_steps=2, cache_path=cache) >= 0
    with open(cache) as f:
        (key, val), = json.load(f).items()
    assert len(val) == 8
    with open(cache, "w") as f:
        f.write('{\n"%s": [7, 16, 0.05, 16, 2, 13, 32, 0],\nnot an entry\n}\n' % key)
    assert sim.autotune(trial_steps=2, cache_path=cache) >= 0     # rows 7: ignored
    with open(cache) as f:
        val = json.load(f)[key]
    assert val[0] in (2, 4, 8, 12, 16)
    with open(cache, "w") as f:
        f.write('{\n"%s": [4, 16, 0.05, 16]\n}\n' % key)
    assert sim.autotune(trial_steps=2, cache_path=cache) == -1
    assert sim.get_config() == (4, 16) and sim.tile_order()[0] == 16
    sim.run()
    ref = fd.Simulation(p, fused=True, config=(4, 16))
    ref.set_tile_order(16)
    ref.run()
    Va, Ia = sim.spectra()
    Vb, Ib = ref.spectra()
    assert np.array_equal(Va, Vb) and np.array_equal(Ia, Ib)
    for x in (sim, ref):
        x.close()
