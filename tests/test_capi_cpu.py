"""Host-only checks of the C-ABI library: it loads, exports every function
include/fdtd.h declares, validates its arguments, and its host FP64
arithmetic (time step, post-processing) agrees with the oracle's."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from oracle import post
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def fd():
    from paper_2208_04371_amd import build as hb
    if not os.path.exists(hb.LIB):
        hb.build()
    import paper_2208_04371_amd as fd
    fd.lib()
    return fd


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(fdtd_[a-z0-9_]+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol(fd):
    names = _declared()
    assert len(names) >= 39
    L = C.CDLL(fd._capi.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing
    # and the binding declares a signature for each of them
    assert names <= set(fd._capi.SIGNATURES), names - set(fd._capi.SIGNATURES)


def test_status_strings(fd):
    L = fd.lib()
    assert L.fdtd_status_string(0) == b"ok"
    assert L.fdtd_status_string(-6) == b"diverged"


def test_create_rejects_bad_grids(fd):
    with pytest.raises(fd.FdtdError) as e:
        fd._plan_create = None
        from paper_2208_04371_amd import fdtd_plan_create
        fdtd_plan_create(0, 10, 10, 1, 1, 1, 0.9)
    assert e.value.code == -1
    from paper_2208_04371_amd import fdtd_plan_create
    with pytest.raises(fd.FdtdError) as e:
        fdtd_plan_create(10, 10, 10, 1, 1, 1, 0.9, precision=fd.FP64, kernel=fd.KERNEL_FUSED)
    assert e.value.code == -3
    with pytest.raises(fd.FdtdError):
        fdtd_plan_create(10, 10, 10, -1, 1, 1, 0.9)
    # fewer than two cells along an axis
    for dims in ((1, 1, 1), (1, 8, 8), (8, 1, 8), (8, 8, 1)):
        with pytest.raises(fd.FdtdError) as e:
            fdtd_plan_create(*dims, 1, 1, 1, 0.9)
        assert e.value.code == -1
    h = fdtd_plan_create(2, 2, 2, 1, 1, 1, 0.9)
    fd.fdtd_plan_destroy(h)


def test_fused_plan_refuses_arrays_of_4_gib(fd):
    """The fused kernels address every array with 32-bit byte offsets: a
    grid whose field arrays would reach 4 GiB (1600 x 1024 x 660 cells:
    4.43 GB per component) is refused as UNSUPPORTED when the plan is
    finalized."""
    from paper_2208_04371_amd import describe, fdtd_plan_destroy, fdtd_plan_workspace_size
    nx, ny, nz = 1600, 1024, 660
    p = W.Problem(name="over_4gib", nx=nx, ny=ny, nz=nz, dx=5e-9, dy=5e-9, dz=5e-9,
                  courant=0.99, normalized=False, materials=[W.Material(1.0)],
                  cells=np.zeros((nz, ny, nx), dtype=np.uint8),
                  faces=(W.PEC,) * 6, freqs=np.array([1e12]), nsteps=1, fp32=True)
    h = describe(p, fused=True)
    try:
        with pytest.raises(fd.FdtdError) as e:
            fdtd_plan_workspace_size(h)
        assert e.value.code == -3 and "4 GiB" in str(e.value)
    finally:
        fdtd_plan_destroy(h)


def test_call_order_and_argument_errors(fd):
    from paper_2208_04371_amd import (describe, fdtd_plan_add_port, fdtd_plan_autotune,
                                      fdtd_plan_create, fdtd_plan_destroy,
                                      fdtd_plan_workspace_size, fdtd_run, fdtd_plan_set_materials)
    p = W.small_microstrip()
    h = describe(p)
    # run or autotune before bind
    with pytest.raises(fd.FdtdError) as e:
        fdtd_run(h, 10, stream=0)
    assert e.value.code == -2
    with pytest.raises(fd.FdtdError) as e:
        fdtd_plan_autotune(h, 3, stream=0)
    assert e.value.code == -2
    # tile order: -1 (automatic) by default, [0, 4096] accepted
    assert fd.fdtd_plan_get_tile_order(h)[0] == -1
    for bad in (-2, 4097):
        with pytest.raises(fd.FdtdError) as e:
            fd.fdtd_plan_set_tile_order(h, bad)
        assert e.value.code == -1
    fd.fdtd_plan_set_tile_order(h, 16)
    assert fd.fdtd_plan_get_tile_order(h) == (16, 16)
    fd.fdtd_plan_set_tile_order(h, -1)
    # streaming stores: -1 (automatic), 0, 1
    assert fd.fdtd_plan_get_stream_stores(h) == (-1, 0)   # 9 MB workspace: off
    for bad in (-2, 2):
        with pytest.raises(fd.FdtdError) as e:
            fd.fdtd_plan_set_stream_stores(h, bad)
        assert e.value.code == -1
    fd.fdtd_plan_set_stream_stores(h, 1)
    assert fd.fdtd_plan_get_stream_stores(h) == (1, 1)
    fd.fdtd_plan_set_stream_stores(h, -1)
    big = describe(W.large_line(nsteps=10))
    fdtd_plan_workspace_size(big)
    assert fd.fdtd_plan_get_stream_stores(big) == (-1, 1)
    assert fd.fdtd_plan_get_tile_order(big) == (-1, 16)
    fdtd_plan_destroy(big)
    # timing stride: 0 off, n >= 1 every n-th step, negative refused
    with pytest.raises(fd.FdtdError) as e:
        fd.fdtd_plan_set_timing(h, -1)
    assert e.value.code == -1
    fd.fdtd_plan_set_timing(h, 16)
    assert fd.fdtd_plan_get_kernel_time(h) == (0.0, 0)
    fd.fdtd_plan_set_timing(h, 0)
    # port whose current loop would leave the grid
    h2 = fdtd_plan_create(20, 20, 20, 1, 1, 1, 0.9, units=fd.NORMALIZED)
    with pytest.raises(fd.FdtdError) as e:
        fdtd_plan_add_port(h2, 5, 1, 0, 4, 2, 4)
    assert e.value.code == -1
    with pytest.raises(fd.FdtdError) as e:
        fdtd_plan_add_port(h2, 5, 2, 3, 6, 2, 4)
    assert e.value.code == -1
    # material id out of range
    cells = np.full((20, 20, 20), 3, np.uint8)
    with pytest.raises(fd.FdtdError) as e:
        fdtd_plan_set_materials(h2, cells, [W.Material(1.0)])
    assert e.value.code == -1
    # workspace query before materials
    with pytest.raises(fd.FdtdError) as e:
        fdtd_plan_workspace_size(h2)
    assert e.value.code == -2
    assert fdtd_plan_workspace_size(h) > 0
    # describe refuses magnetic walls, which only the oracle models
    with pytest.raises(fd.FdtdError):
        describe(W.parallel_plate())
    fdtd_plan_destroy(h)
    fdtd_plan_destroy(h2)


@pytest.mark.parametrize("make", [
    lambda: W.pec_cavity(),
    lambda: W.single_microstrip(),
    lambda: W.large_line(),
    lambda: W.small_microstrip(),
])
def test_time_step_agrees_with_oracle(fd, make):
    from paper_2208_04371_amd import describe, fdtd_plan_destroy, fdtd_plan_get_dt, \
        fdtd_plan_workspace_size
    p = make()
    h = describe(p)
    fdtd_plan_workspace_size(h)
    dt = fdtd_plan_get_dt(h)
    fdtd_plan_destroy(h)
    o = oracle.Oracle(W.Problem(name="t", nx=2, ny=2, nz=2, dx=p.dx, dy=p.dy, dz=p.dz,
                                courant=p.courant, normalized=p.normalized,
                                materials=[W.Material()], cells=np.zeros((2, 2, 2), np.uint8),
                                faces=(0,) * 6))
    assert dt == pytest.approx(o.dt, rel=1e-15)


def test_workspace_grows_with_ping_pong(fd):
    from paper_2208_04371_amd import describe, fdtd_plan_destroy, fdtd_plan_workspace_size
    p = W.small_microstrip()
    hf = describe(p, fused=True)
    hp = describe(p, fused=False)
    sf, sp = fdtd_plan_workspace_size(hf), fdtd_plan_workspace_size(hp)
    # fields and H auxiliaries are kept twice; E auxiliaries are updated in
    # place and the ids are packed
    assert sf > 1.6 * sp
    fdtd_plan_destroy(hf)
    fdtd_plan_destroy(hp)


def _random_protocol(rng, n, nf):
    c = lambda *s: rng.normal(size=s) + 1j * rng.normal(size=s)
    Vinc = c(n, nf)
    Iinc = Vinc / (rng.uniform(10, 90, (n, nf)) + 1j * rng.uniform(-10, 10, (n, nf)))
    Vtot = c(n, n, nf) * 0.4
    for j in range(n):
        Vtot[j, j] = Vinc[j] * (1 + 0.3 * c(nf))
    return Vinc, Iinc, Vtot


@pytest.mark.parametrize("n", [1, 2, 3])
def test_sparams_matches_oracle_post(fd, n):
    rng = np.random.default_rng(40 + n)
    nf = 9
    f = np.linspace(1e12, 9e12, nf)
    Vinc, Iinc, Vtot = _random_protocol(rng, n, nf)
    got = fd.fdtd_sparams(f, Vinc, Iinc, Vtot)
    ref = post.sparams(f, Vinc, Iinc, Vtot)
    for key in ("S_star", "S", "Zr"):
        assert np.max(np.abs(got[key] - ref[key])) < 1e-12 * max(1, np.max(np.abs(ref[key])))
    if n == 2:
        assert np.max(np.abs(got["Z0"] - ref["Z0"])) < 1e-10 * np.max(np.abs(ref["Z0"]))
    # phase delays agree where the unwrapped phase is smooth enough to define them
    assert np.allclose(got["tau"], ref["tau"], rtol=1e-9, atol=1e-25)


def test_sparams_uniform_line_closed_form(fd):
    """Library post-processing of a reflectionless 25 ohm line matches eq. 7
    (typo fixed) after renormalization to 50 ohm, and Z0 = 25 ohm."""
    f = np.linspace(1e9, 60e9, 40)
    tau = 30e-12
    k = np.exp(-2j * np.pi * f * tau)
    Vinc = np.stack([np.ones_like(k), np.ones_like(k)])
    Iinc = Vinc / 25.0
    Vtot = np.stack([np.stack([Vinc[0], k]), np.stack([k, Vinc[1]])])
    r = fd.fdtd_sparams(f, Vinc, Iinc, Vtot)
    s11, s21 = post.lossless_line_s(-1.0 / 3.0, k)
    assert np.max(np.abs(r["S"][:, 0, 0] - s11)) < 1e-13
    assert np.max(np.abs(r["S"][:, 1, 0] - s21)) < 1e-13
    assert np.max(np.abs(r["Z0"] - 25.0)) < 1e-10
    assert np.max(np.abs(r["tau"][:, 1, 0] / tau - 1)) < 1e-12


def test_sparams_rejects_bad_input(fd):
    with pytest.raises(fd.FdtdError) as e:
        fd.fdtd_sparams(np.zeros(0), np.zeros((1, 0)), np.zeros((1, 0)), np.zeros((1, 1, 0)))
    assert e.value.code == -1


def test_sparams_reports_divergence(fd):
    """A non-finite spectrum (a run that blew up) is reported as DIVERGED,
    not turned into numbers."""
    f = np.array([1e9, 2e9])
    V = np.ones((2, 2), complex)
    I = 0.02 * np.ones((2, 2), complex)
    # a lossy, slightly mismatched 2-port: S* = [[0.1, 0.7], [0.7, 0.1]]
    Vt = np.empty((2, 2, 2), complex)
    Vt[0, 0] = Vt[1, 1] = 1.1
    Vt[0, 1] = Vt[1, 0] = 0.7
    r = fd.fdtd_sparams(f, V, I, Vt)
    assert np.all(np.isfinite(r["S"])) and np.all(np.isfinite(r["Z0"]))
    V[1, 0] = np.nan
    with pytest.raises(fd.FdtdError) as e:
        fd.fdtd_sparams(f, V, I, Vt)
    assert e.value.code == -6


def test_device_copy_validates_arguments(fd):
    """Argument checks of the streaming copy happen before any HIP call."""
    L = fd.lib()
    assert L.fdtd_device_copy(None, None, 0, None) == 0           # nothing to copy
    assert L.fdtd_device_copy(None, C.c_void_p(4096), 64, None) == -1
    assert L.fdtd_device_copy(C.c_void_p(4096), C.c_void_p(8192 + 8), 64, None) == -1
    assert L.fdtd_device_copy(C.c_void_p(4096), C.c_void_p(8192), 60, None) == -1
    assert L.fdtd_device_copy(C.c_void_p(4096), C.c_void_p(4096 + 32), 64, None) == -1


def test_source_samples_validation(fd):
    import dataclasses
    from paper_2208_04371_amd import describe, fdtd_plan_destroy, fdtd_plan_workspace_size
    p = W.small_microstrip(nsteps=10)
    # a SAMPLED source without samples cannot be finalized
    ps = dataclasses.replace(p, source=dataclasses.replace(p.source, kind=W.SAMPLED))
    h = describe(ps, fused=True)
    with pytest.raises(fd.FdtdError) as e:
        fdtd_plan_workspace_size(h)
    assert e.value.code == -2
    L = fd.lib()
    assert L.fdtd_plan_set_source_samples(h, None, 5) == -1
    fdtd_plan_destroy(h)
    # with samples it finalizes
    ps = dataclasses.replace(ps, source=dataclasses.replace(ps.source, samples=np.ones(8)))
    h = describe(ps, fused=True)
    assert fdtd_plan_workspace_size(h) > 0
    fdtd_plan_destroy(h)


def test_coefficient_set_limits(fd):
    """More than 256 distinct edge coefficient sets: plain plans switch to
    16-bit ids, fused plans (ids in LDS-indexed 8-bit fields) refuse the grid
    with UNSUPPORTED when it is finalized."""
    from paper_2208_04371_amd import describe, fdtd_plan_destroy, fdtd_plan_workspace_size
    rng = np.random.default_rng(7)
    p = W.small_microstrip(nx=40, ny=24, nz=16, nsteps=10, pml=4, src_i=6, ports=(10, 30))
    # irregular permittivities: the averages over the cells of an edge differ
    p.materials = [W.Material(float(e)) for e in 1.0 + 10.0 * rng.random(40)]
    p.cells = rng.integers(0, 40, size=p.cells.shape).astype(np.uint8)
    h = describe(p, fused=False)
    assert fdtd_plan_workspace_size(h) > 0
    fdtd_plan_destroy(h)
    with pytest.raises(fd.FdtdError) as e:
        h = describe(p, fused=True)
        fdtd_plan_workspace_size(h)
    assert e.value.code == -3


def test_two_level_mode_and_shape_arguments(fd):
    """Two-level steps: the mode is set before the plan is finalized (STATE
    after), the tile shape is checked, PLAIN plans refuse mode 1, automatic
    mode leaves small plans at two buffers and turns the third on for the
    1024x512x256 line (its state with two buffers is 7.6 GB), and a plan
    with two-level steps cannot join a batch.  Host-only calls."""
    from paper_2208_04371_amd import (describe, fdtd_plan_destroy, fdtd_plan_get_temporal,
                                      fdtd_plan_set_temporal, fdtd_plan_set_temporal_config,
                                      fdtd_plan_workspace_size)
    p = W.small_microstrip()
    h = describe(p, fused=True)
    try:
        assert fdtd_plan_get_temporal(h)[:4] == (-1, 0, 13, 32)
        for bad in (-2, 2):
            with pytest.raises(fd.FdtdError) as e:
                fdtd_plan_set_temporal(h, bad)
            assert e.value.code == -1
        for rows, z in ((5, 16), (12, 16), (13, 3), (13, 257)):
            with pytest.raises(fd.FdtdError) as e:
                fdtd_plan_set_temporal_config(h, rows, z)
            assert e.value.code == -1
        fdtd_plan_set_temporal_config(h, 8, 32)
        two = fdtd_plan_workspace_size(h)          # automatic: a 9 MB state stays at two
        assert fdtd_plan_get_temporal(h)[:4] == (-1, 0, 8, 32)
        with pytest.raises(fd.FdtdError) as e:
            fdtd_plan_set_temporal(h, 1)
        assert e.value.code == -2
    finally:
        fdtd_plan_destroy(h)
    h = describe(p, fused=True)
    try:
        fdtd_plan_set_temporal(h, 1)
        three = fdtd_plan_workspace_size(h)
        assert fdtd_plan_get_temporal(h)[1] == 1
        assert three > two                         # the third field buffer
        with pytest.raises(fd.FdtdError) as e:
            arr = (C.c_void_p * 1)(h.value)
            out = C.c_void_p()
            fd._capi.check(fd.lib().fdtd_batch_create(arr, 1, C.byref(out)), "fdtd_batch_create",
                           None, batch=True)
        assert e.value.code == -3
    finally:
        fdtd_plan_destroy(h)
    hp = describe(p, fused=False)
    try:
        with pytest.raises(fd.FdtdError) as e:
            fdtd_plan_set_temporal(hp, 1)
        assert e.value.code == -3
    finally:
        fdtd_plan_destroy(hp)
    # automatic mode on the 1024x512x256 line: three buffers, two-level tiles
    hl = describe(W.large_line(nsteps=2), fused=True)
    try:
        fdtd_plan_workspace_size(hl)
        mode, used, rows, z, tiles = fdtd_plan_get_temporal(hl)
        assert mode == -1 and used == 1 and tiles > 0
    finally:
        fdtd_plan_destroy(hl)
