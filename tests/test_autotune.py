"""Launch-shape autotuner of batches (the tile height x z-chunk search with
its JSON cache keyed by GPU architecture and member shapes)."""
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
    assert val[:2] == [rows, z] and val[2] > 0
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
    assert again.get_config() == (rows, z)
    for x in (bs, ref, again):
        x.close()
