"""GPU path vs the FP64 CPU oracle, element by element, through the C ABI.

Tolerances: plain FP64 kernels agree with the oracle to 1e-10 relative
(rounding order only); FP32 fields to a relative L2 of 1e-4, S-parameters to
|dS| <= 1e-3 and Z0 to 0.5 %.
"""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import post
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


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _fields(x):
    return [x.field(c) for c in range(6)]


def _field_errors(got, ref, norm="max"):
    """Per-component error relative to the scale of its group (E or H):
    max-norm (norm="max") or L2 over the group (norm="l2")."""
    errs = []
    for grp in ((0, 1, 2), (3, 4, 5)):
        if norm == "max":
            scale = max(np.max(np.abs(ref[c])) for c in grp)
            errs += [float(np.max(np.abs(got[c] - ref[c])) / scale) for c in grp]
        else:
            scale = math.sqrt(sum(np.sum(ref[c] ** 2) for c in grp))
            errs += [float(np.linalg.norm(got[c] - ref[c]) / scale) for c in grp]
    return errs


def _check_fields(sim, o, tol, norm="max"):
    errs = _field_errors(_fields(sim), _fields(o), norm)
    _say(f"  field errors ({norm}): " + " ".join(f"{e:.1e}" for e in errs))
    assert max(errs) < tol, f"field error {max(errs):.3e} >= {tol}"


# ---------------------------------------------------------------------------
# plain FP64
# ---------------------------------------------------------------------------

def test_cavity_fp64_plain_matches_oracle(fd):
    p = W.pec_cavity()
    _say(f"cavity fp64 plain {p.nx}^3 x {p.nsteps}")
    sim = fd.Simulation(p, fused=False)
    sim.run()
    o = oracle.Oracle(p).run(p.nsteps)
    _check_fields(sim, o, 1e-10)
    Vg, _ = sim.spectra()
    Vo, _ = o.spectra()
    assert _rel(Vg, Vo) < 1e-10


def test_small_microstrip_fp64_plain_matches_oracle(fd):
    p = W.small_microstrip(nsteps=500, fp32=False)
    _say("small microstrip fp64 plain")
    sim = fd.Simulation(p, fused=False)
    sim.run()
    o = oracle.Oracle(p).run(p.nsteps)
    _check_fields(sim, o, 1e-10)
    Vg, Ig = sim.spectra()
    Vo, Io = o.spectra()
    assert _rel(Vg, Vo) < 1e-10
    assert _rel(Ig, Io) < 1e-10


def test_layered_lossy_fp64_plain_matches_oracle(fd):
    p = W.small_microstrip(nsteps=400, fp32=False, seed=9, sigma_strip=5.8e7)
    _say("layered lossy microstrip fp64 plain")
    sim = fd.Simulation(p, fused=False)
    sim.run()
    o = oracle.Oracle(p).run(p.nsteps)
    _check_fields(sim, o, 1e-10)


@pytest.mark.parametrize("fused", [False, True])
def test_eigenmode_on_gpu(fd, fused):
    """The TM_210 standing mode of the PEC cube evolves as cos(w n dt) with
    the Yee dispersion relation, on the GPU too."""
    N, m, n = 32, 2, 1
    p = W.pec_cavity(n=N, source=False, fp32=fused)
    sim = fd.Simulation(p, fused=fused)
    dt = sim.dt
    a, b = m * math.pi / N, n * math.pi / N
    w = 2 * math.asin(dt * math.sqrt(math.sin(a / 2) ** 2 + math.sin(b / 2) ** 2)) / dt
    kk, jj, ii = np.meshgrid(np.arange(N + 1), np.arange(N + 1), np.arange(N + 1), indexing="ij")
    Ez = np.sin(a * ii) * np.sin(b * jj)
    Ez[N] = 0
    Hx = 0.5 * dt * np.sin(a * ii) * 2 * np.cos(b * (jj + 0.5)) * math.sin(b / 2)
    Hy = -0.5 * dt * np.sin(b * jj) * 2 * np.cos(a * (ii + 0.5)) * math.sin(a / 2)
    Hx[:, N, :] = 0; Hx[N] = 0
    Hy[:, :, N] = 0; Hy[N] = 0
    sim.set_field(W.EZ, Ez)
    sim.set_field(W.HX, Hx)
    sim.set_field(W.HY, Hy)
    steps = 1000
    sim.run(steps)
    err = _rel(sim.field(W.EZ), math.cos(w * steps * dt) * Ez)
    assert np.isfinite(err)
    _say(f"eigenmode fused={fused} err {err:.2e}")
    assert err < (1e-4 if fused else 1e-11)


# ---------------------------------------------------------------------------
# FP32 plain and fused
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def small_ref():
    p = W.small_microstrip(nsteps=800)
    o = oracle.Oracle(p).run(p.nsteps)
    return p, o


@pytest.mark.parametrize("fused", [False, True])
def test_small_microstrip_fp32_matches_oracle(fd, small_ref, fused):
    p, o = small_ref
    _say(f"small microstrip fp32 fused={fused}")
    sim = fd.Simulation(p, fused=fused)
    sim.run()
    _check_fields(sim, o, 1e-4, norm="l2")
    Vg, Ig = sim.spectra()
    Vo, Io = o.spectra()
    assert _rel(Vg, Vo) < 1e-4
    assert _rel(Ig, Io) < 1e-4
    rg = fd.fdtd_sparams(p.freqs, *post.single_excitation_protocol(Vg, Ig))
    ro = post.sparams(p.freqs, *post.single_excitation_protocol(Vo, Io))
    assert np.max(np.abs(rg["S_star"] - ro["S_star"])) < 1e-3
    assert np.max(np.abs(rg["S"] - ro["S"])) < 1e-3
    assert np.max(np.abs(rg["Z0"] / ro["Z0"] - 1)) < 5e-3


@pytest.mark.parametrize("rows,zchunk", [(2, 64), (2, 5), (4, 1), (4, 32), (8, 7), (12, 9), (16, 3)])
def test_fused_launch_shapes_agree(fd, rows, zchunk):
    """Every tile height and z-chunk (ragged tails in x, y and z) gives the
    same fields and port spectra as the reference launch shape (the probes
    are sampled by blocks of 64 x R threads: 12 rows is not a power of two)."""
    p = W.small_microstrip(nsteps=150, seed=4)
    ref = fd.Simulation(p, fused=True, config=(4, 32)).run()
    sim = fd.Simulation(p, fused=True, config=(rows, zchunk)).run()
    errs = _field_errors(_fields(sim), _fields(ref))
    assert max(errs) < 1e-6, errs
    Vs, Is = sim.spectra()
    Vr, Ir = ref.spectra()
    assert _rel(Vs[0], Vr[0]) < 1e-6 and _rel(Is[0], Ir[0]) < 1e-6
    # the same shape with a dealt tile order and streaming stores: same bits
    alt = fd.Simulation(p, fused=True, config=(rows, zchunk))
    alt.set_tile_order(5)
    alt.set_stream_stores(1)
    alt.run()
    assert all(np.array_equal(a, b) for a, b in zip(_fields(alt), _fields(sim)))
    Va, Ia = alt.spectra()
    assert np.array_equal(Va, Vs) and np.array_equal(Ia, Is)


@pytest.mark.parametrize("nx,rows", [(30, 8), (69, 2), (69, 16), (80, 8), (81, 4), (104, 8),
                                     (128, 12)])
def test_ragged_x_column_matches_oracle(fd, nx, rows):
    """Grids whose last x column holds 1..32 cells run it as 16-wide tiles of
    4R rows (one or two sub-columns; nx = 30 has no 64-wide tile at all,
    R = 16 gives narrow tiles taller than the grid); 104 = 64 + 40 keeps
    one partial 64-wide tile and 128 has no ragged column."""
    p = W.small_microstrip(nx=nx, nsteps=150, pml=6, src_i=8, ports=(10, nx - 10), seed=7)
    _say(f"ragged x column nx={nx} rows={rows}")
    o = oracle.Oracle(p).run(p.nsteps)
    sim = fd.Simulation(p, fused=True, config=(rows, 8)).run()
    _check_fields(sim, o, 1e-4, norm="l2")
    Vg, Ig = sim.spectra()
    Vo, Io = o.spectra()
    assert _rel(Vg, Vo) < 1e-4 and _rel(Ig, Io) < 1e-4


def test_tile_order_changes_timing_only(fd):
    """Any block-to-tile order, and streaming or cached field stores, give
    bit-identical fields and spectra."""
    p = W.small_microstrip(nsteps=120, seed=3)
    ref = None
    for order in (0, 1, 7, 16):
        sim = fd.Simulation(p, fused=True, config=(4, 4))
        sim.set_tile_order(order)
        assert sim.tile_order() == (order, order)
        sim.run()
        got = (_fields(sim), sim.spectra())
        if ref is None:
            ref = got
        else:
            assert all(np.array_equal(a, b) for a, b in zip(got[0], ref[0])), order
            assert all(np.array_equal(a, b) for a, b in zip(got[1], ref[1])), order
        sim.close()
    for stream in (0, 1):
        sim = fd.Simulation(p, fused=True, config=(4, 4))
        sim.set_stream_stores(stream)
        assert sim.stream_stores() == (stream, stream)
        sim.run()
        assert all(np.array_equal(a, b) for a, b in zip(_fields(sim), ref[0])), stream
        assert all(np.array_equal(a, b) for a, b in zip(sim.spectra(), ref[1])), stream
        sim.close()
    probs = [W.small_microstrip(nsteps=60, ny=36 + 4 * q, seed=q) for q in range(3)]
    out = []
    for order in (0, 3):
        bs = fd.BatchSimulation(probs, config=(8, 4))
        bs.set_tile_order(order)
        bs.set_stream_stores(order > 0)
        bs.run(60)
        out.append([bs.field(q, W.EZ) for q in range(3)])
        bs.close()
    assert all(np.array_equal(a, b) for a, b in zip(*out))


def test_kernel_timer_windows_cover_every_step(fd):
    p = W.small_microstrip(nsteps=40)
    sim = fd.Simulation(p, fused=True)
    for every in (1, 4, 16, 64):
        fd.fdtd_plan_set_timing(sim.handle, every)
        sim.reset()
        sim.run(23)                  # windows end with each run
        sim.run(17)
        ms, n = fd.fdtd_plan_get_kernel_time(sim.handle)
        assert n == 40 and ms > 0, (every, n, ms)
    fd.fdtd_plan_set_timing(sim.handle, 0)
    sim.run(5)
    assert fd.fdtd_plan_get_kernel_time(sim.handle) == (0.0, 0)
    sim.close()


@pytest.mark.parametrize("fused", [False, True])
def test_anisotropic_cells_match_oracle(fd, fused):
    """Cells of unequal sides (dy = 1.3 dx, dz = 0.8 dx) with absorbing
    layers, a layered substrate, a strip and both probes: every per-axis
    coefficient (curl terms, layer profiles, probe weights) differs."""
    p = W.small_microstrip(nx=81, nsteps=400, seed=11)
    p.dy = 1.3 * p.dx
    p.dz = 0.8 * p.dx
    p.fp32 = fused
    _say(f"anisotropic cells fused={fused}")
    o = oracle.Oracle(p).run(p.nsteps)
    sim = fd.Simulation(p, fused=fused, precision=None if fused else fd.FP64).run()
    if fused:
        _check_fields(sim, o, 1e-4, norm="l2")
        tol = 1e-4
    else:
        _check_fields(sim, o, 1e-10)
        tol = 1e-10
    Vg, Ig = sim.spectra()
    Vo, Io = o.spectra()
    assert _rel(Vg, Vo) < tol and _rel(Ig, Io) < tol
    sim.close()


def test_batch_of_ragged_grids_equals_single_runs(fd):
    """Members whose last x column is ragged in different ways (none, one or
    two narrow sub-columns, a partial 64-wide tile, no 64-wide tile at all),
    run one per group with a dealt tile order and streaming stores, give the
    bits of their single runs."""
    probs = [W.small_microstrip(nx=nx, nsteps=120, pml=6, src_i=8, ports=(10, nx - 10), seed=q)
             for q, nx in enumerate((30, 69, 81, 104, 128))]
    bs = fd.BatchSimulation(probs, config=(8, 4))
    bs.set_group_bytes(1)
    bs.set_tile_order(3)
    bs.set_stream_stores(1)
    assert bs.groups() == len(probs)
    bs.run(120)
    for q, p in enumerate(probs):
        s = fd.Simulation(p, fused=True, config=(8, 4)).run()
        Vb, Ib = bs.spectra(q)
        Vs, Is = s.spectra()
        assert np.array_equal(Vb, Vs) and np.array_equal(Ib, Is), f"member {q} spectra"
        for c in range(6):
            assert np.array_equal(bs.field(q, c), s.field(c)), f"member {q} component {c}"
        s.close()
    bs.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_plain_kernels_with_16bit_ids_match_oracle(fd, prec):
    """More than 256 distinct edge coefficient sets (40 irregular dielectrics
    in random cells) put the plain kernels on 16-bit ids."""
    rng = np.random.default_rng(7)
    p = W.small_microstrip(nx=40, ny=24, nz=16, nsteps=200, pml=4, src_i=6, ports=(10, 30))
    p.materials = [W.Material(float(e)) for e in 1.0 + 10.0 * rng.random(40)]
    p.cells = rng.integers(0, 40, size=p.cells.shape).astype(np.uint8)
    _say(f"16-bit ids, plain {prec}")
    o = oracle.Oracle(p).run(p.nsteps)
    sim = fd.Simulation(p, fused=False, precision=fd.FP64 if prec == "fp64" else fd.FP32).run()
    if prec == "fp64":
        _check_fields(sim, o, 1e-10)
    else:
        _check_fields(sim, o, 1e-4, norm="l2")
    sim.close()


@pytest.mark.parametrize("fused", [False, True])
def test_blow_up_is_reported_as_divergence(fd, fused):
    """Non-finite field values (NaN written into Ez, as a run that blew up
    would hold) reach the probe sums; fdtd_get_spectra reports DIVERGED
    instead of returning them.  Only the float values change: every index
    and address is the same as in a normal run."""
    p = W.small_microstrip(nsteps=60)
    sim = fd.Simulation(p, fused=fused)
    sim.run(5)
    ez = sim.field(W.EZ)
    ez[: p.nz, :, :] = np.nan
    sim.set_field(W.EZ, ez)
    sim.run(40)
    with pytest.raises(fd.FdtdError) as e:
        sim.spectra()
    assert e.value.code == -6
    sim.close()


@pytest.mark.parametrize("fused,steps", [(True, 600), (False, 2000)], ids=["fused", "plain64"])
def test_unstable_time_step_is_reported_as_divergence(fd, fused, steps):
    """A time step 1.2 times the 3-D stability limit on a grid with vacuum
    cells: the leapfrog grows without bound until the fields overflow, and
    fdtd_get_spectra reports DIVERGED rather than returning the sums.  (The
    runs differ from normal ones only in the values, never in an index.)"""
    p = W.small_microstrip(nsteps=steps)
    p.courant = 1.2
    sim = fd.Simulation(p, fused=fused, precision=fd.FP32 if fused else fd.FP64)
    sim.run()
    assert not np.all(np.isfinite(sim.field(W.EZ)))
    with pytest.raises(fd.FdtdError) as e:
        sim.spectra()
    assert e.value.code == -6
    sim.close()


def test_fused_equals_plain_fp32(fd):
    p = W.small_microstrip(nsteps=300, seed=2, sigma_strip=5.8e7)
    a = fd.Simulation(p, fused=True).run()
    b = fd.Simulation(p, fused=False).run()
    errs = _field_errors(_fields(a), _fields(b))
    assert max(errs) < 1e-5, errs


def test_fused_deterministic(fd):
    p = W.small_microstrip(nsteps=200)
    a = fd.Simulation(p, fused=True).run()
    b = fd.Simulation(p, fused=True).run()
    Va, Ia = a.spectra()
    Vb, Ib = b.spectra()
    assert np.array_equal(Va, Vb) and np.array_equal(Ia, Ib)
    for comp in range(6):
        assert np.array_equal(a.field(comp), b.field(comp)), comp


@pytest.mark.parametrize("fused", [False, True])
def test_checkpoint_resume_bitwise(fd, fused):
    p = W.small_microstrip(nsteps=300)
    a = fd.Simulation(p, fused=fused).run(300)
    b = fd.Simulation(p, fused=fused).run(137)
    ck = b.checkpoint()
    b.run(163)
    c = fd.Simulation(p, fused=fused)
    c.restore(ck)
    c.run(163)
    Va, Ia = a.spectra()
    for x in (b, c):
        Vx, Ix = x.spectra()
        assert np.array_equal(Va, Vx) and np.array_equal(Ia, Ix)
        for comp in range(6):
            assert np.array_equal(a.field(comp), x.field(comp)), comp


def test_resumed_runs_equal_one_run(fd):
    p = W.small_microstrip(nsteps=1200)
    a = fd.Simulation(p, fused=True).run(1200)
    b = fd.Simulation(p, fused=True)
    for n in (1, 511, 512, 176):
        b.run(n)
    assert b.step == 1200
    Va, Ia = a.spectra()
    Vb, Ib = b.spectra()
    assert np.array_equal(Va, Vb) and np.array_equal(Ia, Ib)


# ---------------------------------------------------------------------------
# batches
# ---------------------------------------------------------------------------

def test_batch_equals_single_runs(fd):
    probs = [W.small_microstrip(nsteps=200, ny=36 + 4 * q, seed=q) for q in range(4)]
    probs.append(W.pec_cavity(n=20, nsteps=200, fp32=True))
    _say("batch of 5 uneven instances")
    bs = fd.BatchSimulation(probs)
    bs.run(200)
    for q, p in enumerate(probs):
        s = fd.Simulation(p, fused=True, config=bs.get_config()).run(200)
        Vb, Ib = bs.spectra(q)
        Vs, Is = s.spectra()
        assert np.array_equal(Vb, Vs) and np.array_equal(Ib, Is), f"instance {q} spectra"
        assert np.array_equal(bs.field(q, W.EZ), s.field(W.EZ)), f"instance {q} Ez"


@pytest.mark.parametrize("fused", [False, True])
def test_sampled_and_eq3_sources_match_oracle(fd, fused):
    """A pulse given point by point (SAMPLED) and the differential Gaussian
    of eq. 3 drive the GPU grid as they drive the oracle."""
    import dataclasses
    p = W.small_microstrip(nsteps=300, fp32=fused)
    box = p.source.box
    dt = oracle.Oracle(p).dt
    rng = np.random.default_rng(31)
    srcs = [W.Source(W.SAMPLED, box, samples=rng.standard_normal(250) * np.hanning(250)),
            W.Source(W.DIFF_GAUSSIAN, box, width=40 * dt)]
    for src in srcs:
        q = dataclasses.replace(p, source=src)
        sim = fd.Simulation(q, fused=fused).run()
        o = oracle.Oracle(q).run(q.nsteps)
        _say(f"source kind {src.kind} fused={fused}")
        if fused:
            _check_fields(sim, o, 1e-4, norm="l2")
        else:
            _check_fields(sim, o, 1e-10)
        Vg, _ = sim.spectra()
        Vo, _ = o.spectra()
        assert _rel(Vg, Vo) < (1e-4 if fused else 1e-10)


def _many_materials(nmat=4, seed=21, block=(8, 8, 16)):
    """The small microstrip with its dielectric replaced by blocks of nmat
    random materials: 54 distinct edge coefficients for the defaults (more
    than the 32 a 16-bit id word holds), so its ids need 32-bit words."""
    p = W.small_microstrip(nsteps=120, seed=seed)
    rng = np.random.default_rng(seed)
    base = len(p.materials)
    p.materials += [W.Material(float(e)) for e in rng.uniform(2.0, 12.0, nmat)]
    nz, ny, nx = p.cells.shape
    bz, by, bx = block
    ids = rng.integers(0, nmat, size=(-(-nz // bz), -(-ny // by), -(-nx // bx)))
    full = np.repeat(np.repeat(np.repeat(ids, bz, 0), by, 1), bx, 2)[:nz, :ny, :nx]
    sub = p.cells < 2   # keep the strip
    p.cells[sub] = (base + full[sub]).astype(np.uint8)
    return p


@pytest.mark.parametrize("budget", [0, 1, 20 << 20])
def test_batch_group_schedules_agree(fd, budget):
    """A batch run group by group (each member alone: budget 1; groups of a
    few members: 20 MiB) gives the same bits as lockstep and as the single
    runs, across a mid-run DFT fold (600 steps) and a split run."""
    probs = [W.small_microstrip(nsteps=600, ny=36 + 4 * q, seed=q) for q in range(4)]
    probs.append(W.pec_cavity(n=20, nsteps=600, fp32=True))
    bs = fd.BatchSimulation(probs)
    bs.set_group_bytes(budget)
    ng = bs.groups()
    _say(f"batch group budget {budget}: {ng} groups")
    assert ng == {0: 1, 1: len(probs), 20 << 20: 3}[budget]
    bs.run(250)
    bs.run(350)
    for q, p in enumerate(probs):
        s = fd.Simulation(p, fused=True, config=bs.get_config()).run(600)
        Vb, Ib = bs.spectra(q)
        Vs, Is = s.spectra()
        assert np.array_equal(Vb, Vs) and np.array_equal(Ib, Is), f"instance {q} spectra"
        assert np.array_equal(bs.field(q, W.EZ), s.field(W.EZ)), f"instance {q} Ez"
        s.close()
    bs.close()


def test_batch_mixed_id_widths(fd):
    """A member with more than 32 coefficient sets makes the whole batch use
    32-bit id words; every member still equals its own single run."""
    probs = [_many_materials(), W.small_microstrip(nsteps=120, seed=6)]
    bs = fd.BatchSimulation(probs)
    bs.run(120)
    for q, p in enumerate(probs):
        s = fd.Simulation(p, fused=True, config=bs.get_config()).run(120)
        Vb, Ib = bs.spectra(q)
        Vs, Is = s.spectra()
        assert np.array_equal(Vb, Vs) and np.array_equal(Ib, Is), f"instance {q}"
        for comp in range(6):
            assert np.array_equal(bs.field(q, comp), s.field(comp)), (q, comp)
    bs.close()


def test_many_materials_fused_matches_oracle(fd):
    p = _many_materials()
    sim = fd.Simulation(p, fused=True).run()
    o = oracle.Oracle(p).run(p.nsteps)
    _check_fields(sim, o, 1e-4, norm="l2")


# ---------------------------------------------------------------------------
# the 400x120x80 microstrip at full size, in the benchmark's launch shape
# ---------------------------------------------------------------------------

def test_full_size_microstrip_window(fd):
    """The full 400x120x80 grid for a 300-step window of the resolved
    (THz) reading: every field against the oracle."""
    p = W.single_microstrip(twin=True, nsteps=300)
    _say("full-size microstrip window, 300 steps")
    sim = fd.Simulation(p, fused=True).run()
    o = oracle.Oracle(p).run(p.nsteps)
    _check_fields(sim, o, 1e-4, norm="l2")
    Vg, Ig = sim.spectra()
    Vo, Io = o.spectra()
    assert _rel(Vg, Vo) < 1e-4 and _rel(Ig, Io) < 1e-4


def _golden(name):
    import json
    with open(os.path.join(os.path.dirname(__file__), "golden", name + "_oracle.json")) as f:
        g = json.load(f)
    c = lambda d: np.asarray(d["re"]) + 1j * np.asarray(d["im"])
    return {k: (c(v) if isinstance(v, dict) else
                np.array([c(x) for x in v]) if k in ("V", "I") else np.asarray(v))
            for k, v in g.items() if k in ("V", "I", "S_star", "S", "Zr", "Z0", "tau", "freqs")}


@pytest.mark.parametrize("twin,kernel", [(False, "fused"), (True, "fused"), (False, "fp64")])
def test_full_run_matches_stored_oracle(fd, twin, kernel):
    """The whole 20 000-step S-parameter run of the 400x120x80 microstrip
    (literal GHz band, and its THz twin) against the oracle's stored
    spectra and post-processed results (tests/golden, written by the CPU
    oracle alone): the fused FP32 path within the S-parameter bars, the
    plain FP64 kernels to rounding."""
    name = "microstrip_400x120x80" + ("_thz" if twin else "")
    g = _golden(name)
    p = W.single_microstrip(twin=twin)
    assert p.nsteps == 20000 and np.array_equal(p.freqs, g["freqs"])
    _say(f"full run {name}, {kernel}, {p.nsteps} steps")
    if kernel == "fused":
        sim = fd.Simulation(p, fused=True)
    else:
        sim = fd.Simulation(p, fused=False, precision=fd.FP64)
    sim.run()
    V, I = sim.spectra()
    sim.close()
    r = fd.fdtd_sparams(p.freqs, *post.single_excitation_protocol(V, I))
    ev, ei = _rel(V, g["V"]), _rel(I, g["I"])
    ds_star = float(np.max(np.abs(r["S_star"] - g["S_star"])))
    ds = float(np.max(np.abs(r["S"] - g["S"])))
    dz0 = float(np.max(np.abs(r["Z0"] / g["Z0"] - 1)))
    dtau = float(np.max(np.abs(r["tau"][:, 1, 0] / g["tau"][:, 1, 0] - 1)))
    _say(f"  spectra V {ev:.1e} I {ei:.1e}; |dS*| {ds_star:.1e} |dS| {ds:.1e} "
         f"Z0 {dz0:.1e} tau {dtau:.1e}")
    if kernel == "fused":
        assert ev < 1e-4 and ei < 1e-4
        assert ds_star <= 1e-3 and ds <= 1e-3 and dz0 <= 5e-3 and dtau <= 5e-3
    else:
        assert ev < 1e-10 and ei < 1e-10
        assert ds_star < 1e-9 and ds < 1e-9 and dz0 < 1e-9 and dtau < 1e-9


def _check_groups(got, ref, tol):
    """L2 error of each component relative to its group (E or H); a group
    whose reference is all zero must come out exactly zero."""
    for grp in ((0, 1, 2), (3, 4, 5)):
        if all(np.max(np.abs(ref[c])) == 0 for c in grp):
            assert all(np.max(np.abs(got[c])) == 0 for c in grp), grp
            continue
        scale = math.sqrt(sum(np.sum(ref[c] ** 2) for c in grp))
        for c in grp:
            assert np.linalg.norm(got[c] - ref[c]) / scale < tol, c


def _tiny_grid(nx, ny, nz, pml, src, nsteps=30):
    """A small grid with a dielectric lower half, absorbing layers of `pml`
    cells on every face (PEC faces when 0) and a Gaussian pulse (t0 10,
    width 4 steps) on the Ez edge at `src`, sampled by a point probe."""
    faces = (W.CPML,) * 6 if pml else (W.PEC,) * 6
    cells = np.zeros((nz, ny, nx), dtype=np.uint8)
    cells[: max(1, nz // 2)] = 1
    i, j, k = src
    return W.Problem(name=f"tiny_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, dx=5e-9, dy=5e-9,
                     dz=5e-9, courant=0.99, normalized=False,
                     materials=[W.Material(1.0), W.Material(3.0)], cells=cells, faces=faces,
                     pml_cells=(pml,) * 6,
                     source=W.Source(W.GAUSSIAN_STEPS, (i, i, j, j, k, k), t0=10, width=4),
                     points=[W.PointProbe(W.EZ, i, j, k)], freqs=W.linear_freqs(1e13, 1e15, 4),
                     nsteps=nsteps, fp32=True)


TINY = [((2, 2, 2), 0, (1, 1, 0)),       # the smallest grid a plan accepts
        ((2, 3, 4), 1, (1, 1, 1)),       # one-cell layers on every face
        ((20, 20, 20), 10, (10, 10, 10)),  # all cells in layers: no interior tile
        ((65, 9, 5), 2, (32, 4, 2))]     # one cell past a 64-wide tile in x


@pytest.mark.parametrize("kernel", ["fused", "fp64"])
@pytest.mark.parametrize("dims,pml,src", TINY, ids=["2x2x2", "2x3x4", "20x20x20", "65x9x5"])
def test_degenerate_grids_match_oracle(fd, dims, pml, src, kernel):
    """Grids far smaller than a tile, or made of absorbing layers only,
    after 30 steps: every field and the probe's spectra against the oracle
    (all-zero references must come out exactly zero)."""
    p = _tiny_grid(*dims, pml, src)
    _say(f"degenerate grid {dims} layers {pml} {kernel}")
    if kernel == "fused":
        sim = fd.Simulation(p, fused=True)
    else:
        sim = fd.Simulation(p, fused=False, precision=fd.FP64)
    sim.run()
    o = oracle.Oracle(p).run(p.nsteps)
    tol = 1e-4 if kernel == "fused" else 1e-10
    _check_groups(_fields(sim), _fields(o), tol)
    Vg, _ = sim.spectra()
    Vo, _ = o.spectra()
    assert np.max(np.abs(Vo)) > 0 and _rel(Vg, Vo) < tol
    sim.close()


def test_zero_and_single_steps(fd):
    """A run of zero steps changes nothing (fields and spectra exactly zero,
    for a plan and a batch); runs of one and two steps match the oracle."""
    p = W.small_microstrip(nsteps=2, seed=5)
    _say("zero, one and two steps")
    sim = fd.Simulation(p, fused=True)
    sim.run(0)
    assert sim.step == 0
    assert all(np.max(np.abs(f)) == 0 for f in _fields(sim))
    V, I = sim.spectra()
    assert np.max(np.abs(V)) == 0 and np.max(np.abs(I)) == 0
    o = oracle.Oracle(p)
    for n in (1, 2):
        sim.run(1)
        o.run(1)
        assert sim.step == n
        _check_groups(_fields(sim), _fields(o), 1e-4)
    sim.close()
    bs = fd.BatchSimulation([W.small_microstrip(nsteps=2, seed=5), W.small_microstrip(nsteps=2, seed=6)])
    bs.run(0)
    for q in range(2):
        assert all(np.max(np.abs(bs.field(q, c))) == 0 for c in range(6))
        V, I = bs.spectra(q)
        assert np.max(np.abs(V)) == 0 and np.max(np.abs(I)) == 0
    bs.close()


def _largest_fused_grid(nz=600, nsteps=60):
    """1600 x 1024 x nz cells at 5 nm: a dielectric (eps_r 4) slab under
    vacuum, PEC ground, 10-cell absorbing layers on the other faces, and a
    Gaussian pulse (t0 30, width 10 steps) on an Ez line near the far top
    corner, sampled by a point probe.  At nz = 600 each field array of a
    fused plan takes 4.03 GB, just under the 4 GiB its 32-bit byte offsets
    allow; nz = 660 is over it."""
    nx, ny = 1600, 1024
    cells = np.zeros((nz, ny, nx), dtype=np.uint8)
    cells[: nz // 4] = 1
    src = W.Source(W.GAUSSIAN_STEPS, (nx - 40, nx - 40, ny - 40, ny - 40, nz - 45, nz - 35),
                   t0=30, width=10)
    return W.Problem(name=f"largest_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, dx=5e-9, dy=5e-9,
                     dz=5e-9, courant=0.99, normalized=False,
                     materials=[W.Material(1.0), W.Material(4.0)], cells=cells,
                     faces=(W.CPML,) * 4 + (W.PEC, W.CPML), pml_cells=(10,) * 6, source=src,
                     points=[W.PointProbe(W.EZ, nx - 40, ny - 40, nz - 40)],
                     freqs=W.linear_freqs(1e12, 1e14, 8), nsteps=nsteps, fp32=True)


def test_largest_fused_grid_light_cone(fd):
    """The largest grid one fused plan accepts (field arrays of 4.03 GB,
    51.5 GB of state, default launch shape, streaming stores): a 140-cell
    window at the far top corner (the highest addresses, its absorbing
    layers and the source) against the oracle run on that window, every
    field component and the probe's spectra."""
    n = 60
    p = _largest_fused_grid(nsteps=n)
    _say(f"largest fused grid {p.nx}x{p.ny}x{p.nz}, {n} steps, corner window")
    sim = fd.Simulation(p, fused=True)
    assert sim.stream_stores()[1] == 1
    sim.run()
    Vg, _ = sim.spectra()
    box = (p.nx - 140, p.nx, p.ny - 140, p.ny, p.nz - 140, p.nz)
    wp = W.window(p, box)
    wp.points = [W.PointProbe(W.EZ, 100, 100, 100)]
    o = oracle.Oracle(wp).run(n)
    m = n + 2
    full_sl = (slice(box[4] + m, None), slice(box[2] + m, None), slice(box[0] + m, None))
    win_sl = (slice(m, None), slice(m, None), slice(m, None))
    got = []
    for c in range(6):
        f = sim.field(c)
        got.append(f[full_sl].copy())
        del f
    sim.close()
    ref = [o.field(c)[win_sl] for c in range(6)]
    assert max(np.max(np.abs(r)) for r in ref[:3]) > 0
    errs = _field_errors(got, ref, "l2")
    Vo, _ = o.spectra()
    ev = _rel(Vg, Vo)
    _say("  field errors (l2): " + " ".join(f"{e:.1e}" for e in errs) + f"; probe {ev:.1e}")
    assert max(errs) < 1e-4 and ev < 1e-4


# ---------------------------------------------------------------------------
# the 1024x512x256 line and the 16-instance sweep at full size, in their
# default launch shapes
# ---------------------------------------------------------------------------

def test_full_size_line_light_cone(fd):
    """The full 1024x512x256 layered lossy line for 100 steps.  The oracle
    runs a window around the source whose cut faces lie 102 cells beyond the
    checked box: inside the light cone the two must agree (the window
    property itself is checked on the CPU)."""
    n = 100
    p = W.large_line(nsteps=n)
    _say(f"full-size line {p.nx}x{p.ny}x{p.nz}, {n} steps, light-cone window")
    sim = fd.Simulation(p, fused=True).run()
    box = (0, 140, 140, 372, 0, 200)
    o = oracle.Oracle(W.window(p, box)).run(n)
    m = n + 2
    full_sl = (slice(0, box[5] - m), slice(box[2] + m, box[3] - m), slice(0, box[1] - m))
    win_sl = (slice(0, box[5] - m), slice(m, box[3] - box[2] - m), slice(0, box[1] - m))
    got = [sim.field(c)[full_sl].copy() for c in range(6)]
    sim.close()
    ref = [o.field(c)[win_sl] for c in range(6)]
    assert max(np.max(np.abs(r)) for r in ref[:3]) > 0
    errs = _field_errors(got, ref, "l2")
    _say("  field errors (l2): " + " ".join(f"{e:.1e}" for e in errs))
    assert max(errs) < 1e-4


def test_geometry_sweep_batch_matches_oracle(fd):
    """The 16 uneven sweep instances as one batch for 120 steps; the
    smallest and the largest instance checked whole against the oracle."""
    n = 120
    probs = W.geometry_sweep(nsteps=n)
    _say(f"sweep batch of {len(probs)}, {n} steps")
    bs = fd.BatchSimulation(probs)
    bs.run(n)
    for q in (0, len(probs) - 1):
        p = probs[q]
        o = oracle.Oracle(p).run(n)
        errs = _field_errors([bs.field(q, c) for c in range(6)], _fields(o), "l2")
        _say(f"  instance {q} {p.nx}x{p.ny}x{p.nz} field errors (l2): " +
             " ".join(f"{e:.1e}" for e in errs))
        assert max(errs) < 1e-4
        Vb, Ib = bs.spectra(q)
        Vo, Io = o.spectra()
        assert _rel(Vb, Vo) < 1e-4 and _rel(Ib, Io) < 1e-4
    bs.close()


def test_geometry_sweep_full_run_matches_stored_oracle(fd):
    """The 16-instance sweep as one batch over its whole 50 000 steps, in
    the launch shape its autotuner picks: the spectra of the smallest and
    the largest instance against the oracle's stored full runs."""
    probs = W.geometry_sweep()
    assert probs[0].nsteps == 50000
    for q in (0, len(probs) - 1):
        path = os.path.join(os.path.dirname(__file__), "golden", probs[q].name + "_oracle.json")
        if not os.path.exists(path):
            pytest.skip(f"stored oracle run missing: {path} (tests/golden/make_golden.py)")
    _say(f"sweep batch of {len(probs)}, autotuned, {probs[0].nsteps} steps")
    bs = fd.BatchSimulation(probs)
    bs.autotune(trial_steps=16)       # leaves the members reset
    _say(f"  launch shape {bs.get_config()}, tile order {bs.tile_order()}")
    bs.run(probs[0].nsteps)
    for q in (0, len(probs) - 1):
        p = probs[q]
        g = _golden(p.name)
        assert np.array_equal(p.freqs, g["freqs"])
        V, I = bs.spectra(q)
        ev, ei = _rel(V, g["V"]), _rel(I, g["I"])
        _say(f"  instance {q} {p.nx}x{p.ny}x{p.nz}: spectra V {ev:.1e} I {ei:.1e}")
        assert ev < 1e-4 and ei < 1e-4
    bs.close()
