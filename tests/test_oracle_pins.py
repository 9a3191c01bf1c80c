"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: numbers the
paper prints, closed forms, exact invariants of the Yee scheme, or library
routines for special cases.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import post
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")
C0 = 299792458.0


def _pins():
    with open(os.path.join(GOLD, "paper_pins.json")) as f:
        return json.load(f)


def _tiny(dx, dy, dz, courant=0.99, normalized=False, **kw):
    cells = np.zeros((2, 2, 2), np.uint8)
    return W.Problem(name="tiny", nx=2, ny=2, nz=2, dx=dx, dy=dy, dz=dz, courant=courant,
                     normalized=normalized, materials=[W.Material()], cells=cells,
                     faces=(W.PEC,) * 6, **kw)


# ---------------------------------------------------------------------------
# numbers printed in the paper
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("key", ["dt_microstrip", "dt_cmos_line"])
def test_time_step_matches_paper(key):
    pin = _pins()[key]
    o = oracle.Oracle(_tiny(*pin["cells_m"], courant=pin["courant"]))
    assert abs(o.dt / pin["dt_s"] - 1) < pin["rel_tol"]


def test_lowest_resolved_frequency_matches_paper():
    """The lowest frequency a run resolves is one over its duration: the
    paper's step counts at the oracle's time steps (cells and CFL of
    Sec. II-B and Sec. III) give its 0.1 GHz and 50 GHz."""
    pins = _pins()
    pin = pins["lowest_frequency"]
    steps = {60000: pins["dt_microstrip"], 1400000: pins["dt_cmos_line"]}
    for n, dt_paper, f_low in pin["cases"]:
        grid = steps[n]
        o = oracle.Oracle(_tiny(*grid["cells_m"], courant=grid["courant"]))
        assert abs(o.dt / dt_paper - 1) < grid["rel_tol"]
        assert abs(1.0 / (n * o.dt) / f_low - 1) < pin["rel_tol"], (n, 1.0 / (n * o.dt), f_low)


def _waveform_spectrum(sigma, kind=W.DIFF_GAUSSIAN, fc=0.0, bw=0.0, t0=0.0, per=200, span=12):
    # pick cubic cells so that dt = sigma / per
    dt = sigma / per
    d = dt * C0 * math.sqrt(3.0) / 0.99
    src = W.Source(kind, (1, 1, 1, 1, 0, 0), t0=t0, width=sigma, fc=fc, bandwidth=bw)
    o = oracle.Oracle(_tiny(d, d, d, source=src))
    assert abs(o.dt / dt - 1) < 1e-12
    n = int(span * per)
    s = o.waveform(0, n)
    return o.dt, s


def test_peak_frequency_matches_paper():
    pin = _pins()["peak_frequency"]
    for sigma, fp in pin["cases"]:
        dt, s = _waveform_spectrum(sigma)
        pad = 64
        X = np.abs(np.fft.rfft(s, n=len(s) * pad))
        f = np.fft.rfftfreq(len(s) * pad, d=dt)
        assert abs(f[np.argmax(X)] / fp - 1) < pin["rel_tol"], (sigma, f[np.argmax(X)], fp)


def test_band_edges_match_paper():
    pin = _pins()["band_edges"]
    sigma = pin["sigma_s"]
    dt, s = _waveform_spectrum(sigma, per=400, span=14)
    t = np.arange(len(s)) * dt
    f_peak = 1.0 / (math.sqrt(2) * math.pi * sigma)

    def mag(f):
        return abs(np.sum(s * np.exp(-2j * np.pi * f * t)) * dt)

    for fe in pin["edges_hz"]:
        r = mag(fe) / mag(f_peak)
        assert pin["level"] / pin["factor"] < r < pin["level"] * pin["factor"], (fe, r)


def test_mismatch_gamma_matches_paper():
    """A port matched to its own 25 ohm line, referred to 50 ohm through the
    renormalization, reflects Gamma = (25 - 50)/(25 + 50)."""
    pin = _pins()["mismatch_gamma"]
    S_star = np.zeros((1, 1, 1), dtype=complex)
    Zr = np.full((1, 1), pin["z_line"], dtype=complex)
    S = post.renormalize(S_star, Zr, pin["z_ref"])
    assert abs(S[0, 0, 0] - pin["gamma"]) < pin["abs_tol"]


# ---------------------------------------------------------------------------
# exact properties of the Yee scheme
# ---------------------------------------------------------------------------

def test_energy_invariant_pec_cavity():
    """The discrete energy eps|E^n|^2 + mu H^{n-1/2}.H^{n+1/2} is conserved
    exactly by a lossless PEC cavity once the source is off."""
    p = W.pec_cavity()
    o = oracle.Oracle(p, history=1000, energy=True).run(1000)
    E = o.energy
    ref = E[150]
    assert ref > 0
    assert np.max(np.abs(E[150:1000] - ref)) / ref < 1e-12


def test_energy_invariant_with_metal_and_dielectric():
    """Same invariant with internal PEC blocks and several dielectrics."""
    p = W.pec_cavity(n=20, nsteps=600)
    rng = np.random.default_rng(7)
    p.materials = [W.Material(1.0), W.Material(4.0), W.Material(11.7), W.Material(pec=True)]
    p.cells = rng.integers(0, 3, size=(20, 20, 20)).astype(np.uint8)
    p.cells[4:7, 3:15, 5:9] = 3
    p.cells[12:14, 8:10, 2:18] = 3
    p.source = W.Source(W.GAUSSIAN_STEPS, (10, 10, 10, 10, 10, 10), t0=30, width=8)
    o = oracle.Oracle(p, history=600, energy=True).run(600)
    E = o.energy
    assert np.max(np.abs(E[120:600] - E[120])) / E[120] < 1e-12


@pytest.mark.parametrize("m,n", [(1, 1), (2, 1), (3, 2)])
def test_single_eigenmode_follows_yee_dispersion(m, n):
    """A TM_mn0 standing mode of the PEC cube evolves as cos(w n dt) with w
    from the Yee dispersion relation
    sin^2(w dt/2) = (c dt)^2 sum_d sin^2(k_d D/2)/D^2."""
    N = 32
    p = W.pec_cavity(n=N, source=False)
    o = oracle.Oracle(p)
    dt = o.dt
    a, b = m * math.pi / N, n * math.pi / N
    sw = dt * math.sqrt(math.sin(a / 2) ** 2 + math.sin(b / 2) ** 2)
    w = 2 * math.asin(sw) / dt
    kk, jj, ii = np.meshgrid(np.arange(N + 1), np.arange(N + 1), np.arange(N + 1), indexing="ij")
    Ez = np.sin(a * ii) * np.sin(b * jj)
    Ez[N, :, :] = 0.0              # Ez has k in [0, N)
    # H^{-1/2} = (dt/2) curl E^0 for the pure cos(w t) standing mode
    curl_x = np.sin(a * ii) * 2 * np.cos(b * (jj + 0.5)) * math.sin(b / 2)
    curl_y = -np.sin(b * jj) * 2 * np.cos(a * (ii + 0.5)) * math.sin(a / 2)
    Hx = 0.5 * dt * curl_x
    Hy = 0.5 * dt * curl_y
    Hx[:, N, :] = 0; Hx[N, :, :] = 0
    Hy[:, :, N] = 0; Hy[N, :, :] = 0
    o.set_field(W.EZ, Ez)
    o.set_field(W.HX, Hx)
    o.set_field(W.HY, Hy)
    steps = 1000
    o.run(steps)
    expect = math.cos(w * steps * dt) * Ez
    err = np.max(np.abs(o.field(W.EZ) - expect)) / np.max(np.abs(Ez))
    assert err < 1e-12, err


@pytest.mark.parametrize("comp,layers", [("z", "x"), ("z", "y"), ("x", "y"), ("x", "z")])
def test_interface_averaging_in_one_cell_layers(comp, layers):
    """Edge permittivity is the mean over the cells that share the edge (the
    reading taken for material interfaces).  With 1-cell layers of eps 2 and
    5 alternating along an axis across the edges, every edge of the mode's
    component is shared by two cells of each, so a standing mode uniform
    along that component (TM_mn0 for Ez, its rotation for Ex) evolves
    exactly as in a uniform eps 3.5, at the exact Yee frequency.  A harmonic
    mean, or a mean over the wrong cells, changes the frequency."""
    N = 24
    eps = (2.0, 5.0)
    p = W.pec_cavity(n=N, source=False)
    p.materials = [W.Material(eps[0]), W.Material(eps[1])]
    kk, jj, ii = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    p.cells = ({"x": ii, "y": jj, "z": kk}[layers] % 2).astype(np.uint8)
    o = oracle.Oracle(p)
    dt = o.dt
    a, b = 2 * math.pi / N, math.pi / N
    s2 = math.sin(a / 2) ** 2 + math.sin(b / 2) ** 2

    def omega(e):
        return 2 * math.asin(dt * math.sqrt(s2 / e)) / dt

    kk, jj, ii = np.meshgrid(np.arange(N + 1), np.arange(N + 1), np.arange(N + 1), indexing="ij")
    if comp == "z":
        # Ez = sin(a i) sin(b j); H^{-1/2} = (dt/2) curl E^0
        E = np.sin(a * ii) * np.sin(b * jj)
        E[N, :, :] = 0.0
        H1 = 0.5 * dt * np.sin(a * ii) * 2 * np.cos(b * (jj + 0.5)) * math.sin(b / 2)
        H2 = -0.5 * dt * np.sin(b * jj) * 2 * np.cos(a * (ii + 0.5)) * math.sin(a / 2)
        H1[:, N, :] = 0; H1[N, :, :] = 0
        H2[:, :, N] = 0; H2[N, :, :] = 0
        ce, c1, c2 = W.EZ, W.HX, W.HY
    else:
        # Ex = sin(a j) sin(b k): Hy = (dt/2) dEx/dz, Hz = -(dt/2) dEx/dy
        E = np.sin(a * jj) * np.sin(b * kk)
        E[:, :, N] = 0.0
        H1 = 0.5 * dt * np.sin(a * jj) * 2 * np.cos(b * (kk + 0.5)) * math.sin(b / 2)
        H2 = -0.5 * dt * np.sin(b * kk) * 2 * np.cos(a * (jj + 0.5)) * math.sin(a / 2)
        H1[:, :, N] = 0; H1[N, :, :] = 0
        H2[:, :, N] = 0; H2[:, N, :] = 0
        ce, c1, c2 = W.EX, W.HY, W.HZ
    o.set_field(ce, E)
    o.set_field(c1, H1)
    o.set_field(c2, H2)
    steps = 600
    o.run(steps)
    got = o.field(ce)
    expect = math.cos(omega(0.5 * (eps[0] + eps[1])) * steps * dt) * E
    err = np.max(np.abs(got - expect)) / np.max(np.abs(E))
    assert err < 1e-11, err
    # the harmonic mean would be far off
    wrong = math.cos(omega(2 / (1 / eps[0] + 1 / eps[1])) * steps * dt) * E
    assert np.max(np.abs(got - wrong)) / np.max(np.abs(E)) > 1e-2


def test_cavity_resonances():
    """The probe spectrum of the soft-driven PEC cube peaks at the Yee
    frequencies of the modes the centre source excites (odd m, n)."""
    p = W.pec_cavity()
    o = oracle.Oracle(p, history=p.nsteps).run(p.nsteps)
    x = o.history()[0][0]
    x = x - x[200:].mean()          # the soft source leaves a static field
    dt, N = o.dt, 32
    pad = 32
    X = np.abs(np.fft.rfft(x * np.hanning(len(x)), n=len(x) * pad))
    f = np.fft.rfftfreq(len(x) * pad, d=dt)
    peaks = [f[i] for i in range(1, len(X) - 1)
             if X[i] > X[i - 1] and X[i] > X[i + 1] and X[i] > 0.3 * X.max()]

    def fyee(m, n, q):
        s = sum(math.sin(v * math.pi / (2 * N)) ** 2 for v in (m, n, q))
        return math.asin(dt * math.sqrt(s)) / (math.pi * dt)

    half_bin = 0.5 / (len(x) * dt)
    for mode in [(1, 1, 0), (1, 1, 2), (3, 1, 0), (3, 1, 2)]:
        fm = fyee(*mode)
        assert min(abs(pk - fm) for pk in peaks) < half_bin, (mode, fm, peaks)
    # every strong peak is one of the excitable modes
    excit = [fyee(m, n, q) for m in range(1, 9, 2) for n in range(1, 9, 2) for q in range(0, 9)]
    for pk in peaks:
        assert min(abs(pk - fe) for fe in excit) < half_bin


def test_lossy_medium_decay():
    """A uniform static Ez between magnetic side walls decays only through
    the conductivity: E^n -> exp(-sigma t / eps) up to the O((sigma dt/eps)^3)
    per-step error of the centred (semi-implicit) loss term."""
    n = 6
    cells = np.zeros((n, n, n), np.uint8)
    eps_r = 2.0
    p = W.Problem(name="lossy", nx=n, ny=n, nz=n, dx=1.0, dy=1.0, dz=1.0, courant=0.99,
                  normalized=True, materials=[W.Material(eps_r, sigma=0.0)], cells=cells,
                  faces=(W.PMC, W.PMC, W.PMC, W.PMC, W.PEC, W.PEC), fp32=False)
    dt = oracle.Oracle(p).dt
    x = 0.0125
    p.materials[0].sigma = 2 * x * eps_r / dt     # sigma dt / (2 eps) = x
    o = oracle.Oracle(p)
    Ez = np.ones((n + 1, n + 1, n + 1))
    Ez[n] = 0
    o.set_field(W.EZ, Ez)
    steps = 100
    o.run(steps)
    ez = o.field(W.EZ)[:n]
    expect = math.exp(-2 * x * steps)
    assert np.allclose(ez, ez[0, 0, 0], rtol=0, atol=1e-14)
    assert abs(ez[0, 0, 0] / expect - 1) < steps * x ** 3


def test_contour_current_is_discrete_ampere():
    """The port current loop around a (here dielectric) strip equals the sum
    of (curl H)_x over the Ex edges it encloses, recovered from two
    successive Ex levels: Cb (curl H)_x = Ex^{n} - Ca Ex^{n-1}."""
    p = W.small_microstrip(nsteps=0)
    p.materials[2] = W.Material(3.0)        # strip made of dielectric
    o = oracle.Oracle(p, history=400)
    o.run(299)
    ex_prev = o.field(W.EX).copy()
    o.run(1)
    ex_now = o.field(W.EX)
    _, I = o.history()
    port = p.ports[0]
    total = 0.0
    for m in (port.i - 1, port.i):
        sl = (slice(port.z0, port.z1 + 1), slice(port.y0, port.y1 + 1), m)
        ca, cb = o.ca[0][sl], o.cb[0][sl]
        total += np.sum((ex_now[sl] - ca * ex_prev[sl]) / cb) * p.dy * p.dz
    expect = port.direction * 0.5 * total
    assert abs(I[0, 299] - expect) <= 1e-9 * abs(expect)


# ---------------------------------------------------------------------------
# transmission-line pins on an exact discrete TEM line
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def plate():
    p = W.parallel_plate()
    o = oracle.Oracle(p, history=p.nsteps).run(p.nsteps)
    V, I = o.spectra()
    eps_r = p.materials[0].eps_r
    v = 1.0 / math.sqrt(eps_r)
    w = 2 * np.pi * p.freqs
    k = 2 * np.arcsin(np.sin(w * o.dt / 2) / (v * o.dt))      # dx = 1
    d, width = 6.0, 2.0
    z_exact = (d / width) / math.sqrt(eps_r) / np.cos(k / 2)
    return p, o, V, I, k, z_exact


def test_parallel_plate_impedance(plate):
    """Z_r = (eta d / w) / cos(k dx / 2): the exact discrete TEM impedance
    of V at a node plane over I averaged from the two neighbouring H planes."""
    p, o, V, I, k, z = plate
    zr1 = post.reference_impedance(V[0], I[0])
    zr2 = post.reference_impedance(V[1], -I[1])    # outgoing wave at port 2
    assert np.max(np.abs(zr1 / z - 1)) < 2e-4
    assert np.max(np.abs(zr2 / z - 1)) < 2e-4
    # raw eta d / w is off by the 1/cos(k dx/2) staggering bias
    bias = np.max(np.abs(1 / np.cos(k / 2) - 1))
    assert bias > 1e-3


def test_parallel_plate_transmission_and_delay(plate):
    p, o, V, I, k, z = plate
    Vinc, Iinc, Vtot = post.single_excitation_protocol(V, I)
    r = post.sparams(p.freqs, Vinc, Iinc, Vtot)
    length = p.ports[1].i - p.ports[0].i
    s21 = r["S_star"][:, 1, 0]
    assert np.max(np.abs(s21 - np.exp(-1j * k * length))) < 2e-4
    tau = r["tau"][:, 1, 0]
    tau_exact = k * length / (2 * np.pi * p.freqs)
    assert np.max(np.abs(tau / tau_exact - 1)) < 2e-4
    # overall Z0 of a uniform line through ABCD equals its line impedance
    assert np.max(np.abs(r["Z0"] / z - 1)) < 5e-4


def test_matched_line_reflection(plate):
    """Wave split a, b = (V +/- Z I)/2 at port 1 with the exact line
    impedance: only the absorbing layer reflects."""
    p, o, V, I, k, z = plate
    a = 0.5 * (V[0] + z * I[0])
    b = 0.5 * (V[0] - z * I[0])
    assert np.max(np.abs(b / a)) < 1e-3


# ---------------------------------------------------------------------------
# source spectrum, DFT accumulation, checkpoint
# ---------------------------------------------------------------------------

def test_gauss_sine_spectrum_closed_form():
    """DFT of the sampled Gaussian-modulated sine equals its continuous
    Fourier transform
    e^{-j2pi f t0} (tau sqrt(pi) / 2j) [e^{-pi^2 tau^2 (f-fc)^2} - e^{-pi^2 tau^2 (f+fc)^2}]."""
    fc, bw = 150e12, 300e12
    tau = 2 * math.sqrt(math.log(1000.0)) / (math.pi * bw)
    t0 = 6 * tau
    dt, s = _waveform_spectrum(tau, kind=W.GAUSS_SINE, fc=fc, bw=bw, t0=t0, per=60, span=13)
    t = np.arange(len(s)) * dt
    f = np.linspace(10e12, 300e12, 30)
    X = np.array([np.sum(s * np.exp(-2j * np.pi * fk * t)) * dt for fk in f])
    ex = (np.exp(-2j * np.pi * f * t0) * tau * math.sqrt(math.pi) / 2j *
          (np.exp(-(math.pi * tau * (f - fc)) ** 2) - np.exp(-(math.pi * tau * (f + fc)) ** 2)))
    peak = tau * math.sqrt(math.pi) / 2
    assert np.max(np.abs(X - ex)) < 1e-9 * peak


def test_running_dft_matches_fft_bins():
    """With frequencies on the FFT grid of the run, the running DFT of the
    port signals equals numpy's FFT of their recorded histories."""
    p = W.small_microstrip(nsteps=256)
    dt = oracle.Oracle(p).dt
    N = 256
    bins = np.array([1, 3, 7, 20, 51])
    p.freqs = bins / (N * dt)
    o = oracle.Oracle(p, history=N).run(N)
    V, I = o.spectra()
    hv, hi = o.history()
    for q in range(2):
        # sample n (1..N) sits at FFT index n-1, so the sum picks up e^{-j2pi m/N};
        # the current is sampled half a step earlier
        FV = np.fft.fft(hv[q])[bins] * np.exp(-2j * np.pi * bins / N) * dt
        FI = np.fft.fft(hi[q])[bins] * np.exp(-2j * np.pi * bins * 0.5 / N) * dt
        assert np.max(np.abs(V[q] - FV)) < 1e-11 * np.max(np.abs(FV))
        assert np.max(np.abs(I[q] - FI)) < 1e-11 * np.max(np.abs(FI))


def test_checkpoint_resume_bitwise():
    p = W.small_microstrip(nsteps=400)
    a = oracle.Oracle(p, history=400).run(400)
    b = oracle.Oracle(p, history=400).run(150)
    ck = b.checkpoint()
    b.run(250)
    c = oracle.Oracle(p, history=400)
    c.restore(ck)
    c.run(250)
    for x in (b, c):
        assert np.array_equal(a.acc, x.acc)
        for comp in range(6):
            assert np.array_equal(a.field(comp), x.field(comp))


# ---------------------------------------------------------------------------
# pins for the other two axes, magnetic walls, source timing, face zeros
# ---------------------------------------------------------------------------

def _tem_line(axis: int, pol: int, n_len=240, pml=16, eps_r=2.25):
    """Exact discrete TEM line along ``axis`` with E along ``pol``: PEC
    faces normal to ``pol``, magnetic walls normal to the third axis,
    absorbing layers on both ends of ``axis``; probed by two E points 120
    cells apart."""
    third = 3 - axis - pol
    n = [0, 0, 0]
    n[axis], n[pol], n[third] = n_len, 6, 2
    faces = [0] * 6
    pcells = [0] * 6
    faces[2 * axis] = faces[2 * axis + 1] = W.CPML
    pcells[2 * axis] = pcells[2 * axis + 1] = pml
    faces[2 * pol] = faces[2 * pol + 1] = W.PEC
    faces[2 * third] = faces[2 * third + 1] = W.PMC
    lo, hi = [0, 0, 0], [0, 0, 0]
    lo[axis] = hi[axis] = 30
    lo[pol], hi[pol] = 0, n[pol] - 1
    lo[third], hi[third] = 0, n[third]
    box = (lo[0], hi[0], lo[1], hi[1], lo[2], hi[2])
    src = W.Source(W.GAUSS_SINE, box, fc=0.035, bandwidth=0.09, comp=pol)
    pts = []
    for pos in (60, 180):
        q = [0, 0, 0]
        q[axis], q[pol], q[third] = pos, 2, 1
        pts.append(W.PointProbe(pol, *q))
    return W.Problem(name=f"tem_{axis}{pol}", nx=n[0], ny=n[1], nz=n[2], dx=1.0, dy=1.0,
                     dz=1.0, courant=0.99, normalized=True, materials=[W.Material(eps_r)],
                     cells=np.zeros((n[2], n[1], n[0]), np.uint8), faces=tuple(faces),
                     pml_cells=tuple(pcells), source=src, points=pts,
                     freqs=W.linear_freqs(0.01, 0.06, 32), nsteps=2400, fp32=False)


@pytest.mark.parametrize("axis,pol", [(0, 1), (0, 2), (1, 0), (1, 2), (2, 0), (2, 1)])
def test_tem_line_every_axis_and_polarization(axis, pol):
    """The absorbing layers of every axis terminate an exact TEM line of
    either polarization: E at two points 120 cells apart differs by exactly
    exp(-j k 120) with the Yee wavenumber k."""
    p = _tem_line(axis, pol)
    o = oracle.Oracle(p).run(p.nsteps)
    V, _ = o.spectra()
    v = 1.0 / math.sqrt(2.25)
    w = 2 * np.pi * p.freqs
    k = 2 * np.arcsin(np.sin(w * o.dt / 2) / (v * o.dt))
    assert np.max(np.abs(V[1] / V[0] - np.exp(-1j * k * 120))) < 2e-4


@pytest.mark.parametrize("walls", ["pec", "pmc_x"])
def test_eigenmode_anisotropic_cells(walls):
    """TM_mn0 mode on a non-cubic grid with unequal cell sides; with
    magnetic x walls the mode is cos(m pi x / a) sin(n pi y / b) and the
    tangential Ez on those walls evolves through the image currents."""
    nx, ny, nz = 24, 30, 4
    dx, dy, dz = 1.0, 1.3, 0.8
    m, n = 2, 1
    faces = (W.PEC,) * 6 if walls == "pec" else (W.PMC, W.PMC, W.PEC, W.PEC, W.PEC, W.PEC)
    p = W.Problem(name="aniso", nx=nx, ny=ny, nz=nz, dx=dx, dy=dy, dz=dz, courant=0.95,
                  normalized=True, materials=[W.Material(1.0)],
                  cells=np.zeros((nz, ny, nx), np.uint8), faces=faces, fp32=False)
    o = oracle.Oracle(p)
    dt = o.dt
    a, b = m * math.pi / nx, n * math.pi / ny
    sw = dt * math.sqrt(math.sin(a / 2) ** 2 / dx ** 2 + math.sin(b / 2) ** 2 / dy ** 2)
    w = 2 * math.asin(sw) / dt
    kk, jj, ii = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1),
                             indexing="ij")
    if walls == "pec":
        fx = np.sin(a * ii)
        dfx = 2 * np.cos(a * (ii + 0.5)) * math.sin(a / 2)        # f(i+1) - f(i)
    else:
        fx = np.cos(a * ii)
        dfx = -2 * np.sin(a * (ii + 0.5)) * math.sin(a / 2)
    gy = np.sin(b * jj)
    dgy = 2 * np.cos(b * (jj + 0.5)) * math.sin(b / 2)
    Ez = fx * gy
    Ez[nz] = 0
    Hx = 0.5 * dt * fx * dgy / dy          # (dt/2) (dEz/dy)
    Hy = -0.5 * dt * dfx * gy / dx         # (dt/2) (-dEz/dx)
    Hx[:, ny, :] = 0; Hx[nz] = 0
    Hy[:, :, nx] = 0; Hy[nz] = 0
    if walls == "pec":
        Hx[:, :, 0] = 0; Hx[:, :, nx] = 0
    o.set_field(W.EZ, Ez); o.set_field(W.HX, Hx); o.set_field(W.HY, Hy)
    steps = 700
    o.run(steps)
    err = np.max(np.abs(o.field(W.EZ) - math.cos(w * steps * dt) * Ez)) / np.max(np.abs(Ez))
    assert err < 1e-11, err


def test_source_enters_at_the_new_time_level():
    """After the first step of a cavity at rest the driven node holds
    exactly s(t_1): the Gaussian of the source evaluated at step 1."""
    p = W.pec_cavity(nsteps=3)
    c = p.nx // 2
    p.points = [W.PointProbe(W.EZ, c, c, c)]
    o = oracle.Oracle(p, history=3).run(1)
    v, _ = o.history()
    assert v[0, 0] == pytest.approx(math.exp(-((1 - 40.0) / 12.0) ** 2), rel=1e-14)


def test_tangential_e_vanishes_on_pec_and_absorbing_faces():
    """The absorbing layers are backed by PEC: after a run every E component
    tangential to a PEC or absorbing face is exactly zero, while a magnetic
    wall carries tangential E."""
    p = W.small_microstrip(nsteps=200)
    o = oracle.Oracle(p).run(200)
    Ex, Ey, Ez = (o.field(c) for c in (W.EX, W.EY, W.EZ))
    nx, ny, nz = p.nx, p.ny, p.nz
    for F, sl in ((Ey, np.s_[:, :, 0]), (Ey, np.s_[:, :, nx]), (Ez, np.s_[:, :, 0]),
                  (Ez, np.s_[:, :, nx]), (Ex, np.s_[:, 0, :]), (Ex, np.s_[:, ny, :]),
                  (Ez, np.s_[:, 0, :]), (Ez, np.s_[:, ny, :]), (Ex, np.s_[0]),
                  (Ex, np.s_[nz]), (Ey, np.s_[0]), (Ey, np.s_[nz])):
        assert np.all(F[sl] == 0.0)
    q = _tem_line(1, 2)                     # magnetic walls normal to x
    oq = oracle.Oracle(q).run(300)
    assert np.max(np.abs(oq.field(W.EZ)[:q.nz, :, 0])) > 1e-3


def test_sampled_source_reproduces_the_analytic_pulse():
    """A source given point by point (value m at level m + 1) drives the grid
    exactly as the analytic pulse it samples; past the last sample it adds
    nothing."""
    import dataclasses
    p = W.small_microstrip(nsteps=120, fp32=False)
    ref = oracle.Oracle(p)
    vals = ref.waveform(1, 80)            # levels 1..80 of the Gaussian sine
    assert np.max(np.abs(vals)) > 0
    ps = dataclasses.replace(p, source=dataclasses.replace(p.source, kind=W.SAMPLED,
                                                           samples=vals))
    o = oracle.Oracle(ps)
    got = o.waveform(1, 100)
    assert np.array_equal(got[:80], vals) and np.all(got[80:] == 0)
    # the analytic pulse truncated after level 80 drives the same fields
    ref_t = oracle.Oracle(dataclasses.replace(ps, nsteps=80))
    ref_t.run(80)
    o.run(80)
    ref.run(80)
    for c in range(6):
        assert np.array_equal(o.field(c), ref.field(c)), c
