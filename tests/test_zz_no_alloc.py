"""fdtd_run_noalloc (the run entry point for callers that cannot allocate
device memory) against fdtd_run, through the C ABI: the same fields and
spectra, bit for bit, on two calls in a row (the second on a smaller
grid, with the static ring still holding the first call's samples), on a
resumed run, on the plain FP64 kernels, and the size limit of its static
history ring."""
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


def _say(msg):
    print(msg, flush=True)


def _both(fd, p, fused, precision, chunks, temporal=None):
    """The problem run by fdtd_run and, on a second plan, by
    fdtd_run_noalloc in the given step chunks; fields and spectra of each."""
    out = []
    for noalloc in (False, True):
        sim = fd.Simulation(p, fused=fused, precision=precision, temporal=temporal)
        for n in chunks:
            if noalloc:
                fd.fdtd_run_noalloc(sim.handle, n)
            else:
                fd.fdtd_run(sim.handle, n)
        V, I = sim.spectra()
        fields = [sim.field(c) for c in range(6)]
        sim.close()
        out.append((V, I, fields))
    return out


def _assert_same(a, b):
    Va, Ia, Fa = a
    Vb, Ib, Fb = b
    assert np.any(Va != 0) and np.any(Ia != 0)
    assert np.array_equal(Va, Vb) and np.array_equal(Ia, Ib)
    for c in range(6):
        assert np.array_equal(Fa[c], Fb[c]), c


def test_noalloc_equals_run_two_calls_second_smaller(fd):
    """Fused FP32: a 96x40x28 microstrip, then a smaller 64x24x20 one."""
    for dims, n in (((96, 40, 28), 300), ((64, 24, 20), 200)):
        p = W.small_microstrip(nx=dims[0], ny=dims[1], nz=dims[2], strip_w=4, sub_top=6,
                               pml=6, src_i=10, ports=(16, dims[0] - 16), nsteps=n)
        _say(f"noalloc vs run, fused, {dims}, {n} steps")
        a, b = _both(fd, p, True, fd.FP32, [n])
        _assert_same(a, b)


def test_noalloc_resumed_equals_one_run(fd):
    """Calls of 130 and 170 steps (over a DFT fold) equal one 300-step run."""
    p = W.small_microstrip(nsteps=300)
    _say("noalloc resumed, fused, 300 steps")
    a, _ = _both(fd, p, True, fd.FP32, [300])
    _, b = _both(fd, p, True, fd.FP32, [130, 170])
    _assert_same(a, b)


def test_noalloc_two_level_steps(fd):
    """A plan with two-level steps (its source and ports inside the
    two-level box), 101 steps in calls of 50 and 51."""
    p = W.small_microstrip(nx=256, ny=64, nz=48, strip_w=8, sub_top=12, pml=6, src_i=80,
                           ports=(100, 180), nsteps=101, nf=16, seed=7)
    _say("noalloc vs run, two-level steps, 101 steps")
    a, b = _both(fd, p, True, fd.FP32, [50, 51], temporal=1)
    _assert_same(a, b)


def test_noalloc_plain_fp64(fd):
    p = W.small_microstrip(nsteps=120, fp32=False)
    _say("noalloc vs run, plain fp64, 120 steps")
    a, b = _both(fd, p, False, fd.FP64, [120])
    _assert_same(a, b)


def test_noalloc_rejects_rings_beyond_its_static_size(fd):
    """32 probes fit the 256 KiB ring; 33 are refused with INVALID_ARG,
    and the plan still runs through fdtd_run."""
    p = W.small_microstrip(nsteps=10)
    p.ports = []
    for npts in (32, 33):
        p.points = [W.PointProbe(W.EZ, 20 + q, 20, 3) for q in range(npts)]
        sim = fd.Simulation(p, fused=True)
        if npts == 32:
            fd.fdtd_run_noalloc(sim.handle, 10)
        else:
            with pytest.raises(fd.FdtdError) as e:
                fd.fdtd_run_noalloc(sim.handle, 10)
            assert e.value.code == -1
            fd.fdtd_run(sim.handle, 10)
        V, _ = sim.spectra()
        assert np.any(V != 0)
        sim.close()
