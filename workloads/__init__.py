"""Seeded synthetic problem descriptions shared by the oracle and the HIP path.

This module holds geometry and parameters only: grid sizes, cell material
maps, boundary kinds, port and source placement, waveform parameters and the
analysis frequencies.  It contains none of the method's arithmetic (no time
step, no coefficients, no waveform values, no update equations); each side
derives those on its own from these raw inputs.

The problems follow the structure of the paper's workloads (Sec. II-B and
Sec. III): a PEC ground under a dielectric, a conductor strip on top running
along the propagation axis (x here), port planes near both ends, an
absorbing layer on every face except the ground and a soft pulse on an
excitation plane between strip and ground.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

# boundary kinds per face, faces ordered x-, x+, y-, y+, z-, z+
PEC, CPML, PMC = 0, 1, 2
# waveform kinds
GAUSSIAN_STEPS, GAUSS_SINE, DIFF_GAUSSIAN, SAMPLED = 1, 2, 3, 4
# field components
EX, EY, EZ, HX, HY, HZ = 0, 1, 2, 3, 4, 5


@dataclass
class Material:
    eps_r: float = 1.0
    sigma: float = 0.0
    pec: bool = False


@dataclass
class Port:
    """A port plane at node index ``i`` normal to x.

    ``direction`` is +1 when the port's inward direction is +x, -1 otherwise.
    The strip conductor occupies cells y in [y0, y1), z in [z0, z1); the
    ground is the z = 0 face.  The voltage surface spans the Ez edges of the
    plane between ground and strip bottom; the current contour encloses the
    strip one half cell outside its metal.
    """
    i: int
    direction: int
    y0: int
    y1: int
    z0: int
    z1: int


@dataclass
class PointProbe:
    comp: int
    i: int
    j: int
    k: int


@dataclass
class Source:
    """Soft source added to one E component (Ez unless ``comp`` says
    otherwise) on the inclusive node box below.

    Ez node (i, j, k) is the edge from z = k to z = k + 1 (likewise Ex, Ey
    along their own axes).
    ``t0`` / ``width`` are in steps for GAUSSIAN_STEPS and in seconds (or
    normalized time units) otherwise; ``t0 <= 0`` asks for the default delay
    of three pulse widths.  ``bandwidth`` is the full width of the band
    where the spectrum stays within three orders of magnitude of its peak.
    """
    kind: int
    box: Tuple[int, int, int, int, int, int]  # i0, i1, j0, j1, k0, k1 (inclusive)
    t0: float = 0.0
    width: float = 0.0
    fc: float = 0.0
    bandwidth: float = 0.0
    amplitude: float = 1.0
    comp: int = EZ
    samples: Optional[np.ndarray] = None   # SAMPLED: value m added at level m + 1


@dataclass
class Problem:
    name: str
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    courant: float                  # fraction of the 3-D stability limit
    normalized: bool                # True: c = eps0 = mu0 = 1
    materials: List[Material]
    cells: np.ndarray               # uint8 [nz, ny, nx], x fastest
    faces: Tuple[int, int, int, int, int, int]
    pml_cells: Tuple[int, int, int, int, int, int] = (0, 0, 0, 0, 0, 0)
    pml_m: float = 3.0
    pml_sigma_max: float = 0.0      # <= 0: default optimum for the axis
    pml_kappa_max: float = 1.0
    pml_alpha_max: float = 0.0
    source: Optional[Source] = None
    ports: List[Port] = field(default_factory=list)
    points: List[PointProbe] = field(default_factory=list)
    freqs: np.ndarray = field(default_factory=lambda: np.zeros(0))
    nsteps: int = 0
    fp32: bool = True

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz

    def n_probes(self) -> int:
        return len(self.ports) + len(self.points)


def linear_freqs(f_lo: float, f_hi: float, n: int) -> np.ndarray:
    """Inclusive linear frequency grid."""
    if n == 1:
        return np.array([f_lo], dtype=np.float64)
    return f_lo + (f_hi - f_lo) * np.arange(n, dtype=np.float64) / (n - 1)


# ---------------------------------------------------------------------------
# PEC cavity (normalized units)
# ---------------------------------------------------------------------------

def cavity_probe_node(n: int = 32, seed: int = 0) -> Tuple[int, int, int]:
    rng = np.random.default_rng(seed)
    c = n // 2
    while True:
        p = tuple(int(v) for v in rng.integers(1, n, 3))
        if p != (c, c, c):
            return p


def pec_cavity(n: int = 32, nsteps: int = 1000, nf: int = 64, fp32: bool = False,
               source: bool = True) -> Problem:
    """Vacuum cube with PEC walls, soft Gaussian Ez at the centre node,
    Ez point probe at a seeded off-centre node."""
    cells = np.zeros((n, n, n), dtype=np.uint8)
    c = n // 2
    pi, pj, pk = cavity_probe_node(n)
    src = Source(GAUSSIAN_STEPS, (c, c, c, c, c, c), t0=40.0, width=12.0) if source else None
    return Problem(
        name=f"pec_cavity_{n}", nx=n, ny=n, nz=n, dx=1.0, dy=1.0, dz=1.0,
        courant=0.99, normalized=True, materials=[Material(1.0)], cells=cells,
        faces=(PEC,) * 6, source=src, points=[PointProbe(EZ, pi, pj, pk)],
        freqs=linear_freqs(0.005, 0.1, nf), nsteps=nsteps, fp32=fp32)


# ---------------------------------------------------------------------------
# Microstrip lines (SI units)
# ---------------------------------------------------------------------------

def _microstrip_cells(nx, ny, nz, sub_top, eps_id, strip_y0, strip_y1, strip_z0, strip_z1,
                      pec_id):
    cells = np.zeros((nz, ny, nx), dtype=np.uint8)
    cells[:sub_top, :, :] = eps_id
    cells[strip_z0:strip_z1, strip_y0:strip_y1, :] = pec_id
    return cells


def microstrip(name="microstrip_400x120x80", nx=400, ny=120, nz=80, delta=5e-9,
               eps_sub=11.7, sub_top=20, strip_w=8, strip_t=2, pml=10,
               src_i=20, ports=(60, 340), nsteps=20000, nf=64, band=(10e9, 300e9),
               fc=150e9, bw=300e9, fp32=True) -> Problem:
    """Single 2-port microstrip: substrate below ``sub_top``, PEC ground at
    z = 0, PEC strip ``strip_w`` cells wide centred in y on the substrate,
    absorbing layers on the five other faces, Gaussian-modulated sine on the
    excitation plane at ``src_i``."""
    y0 = (ny - strip_w) // 2
    y1 = y0 + strip_w
    z0, z1 = sub_top, sub_top + strip_t
    mats = [Material(1.0), Material(eps_sub), Material(1.0, pec=True)]
    cells = _microstrip_cells(nx, ny, nz, sub_top, 1, y0, y1, z0, z1, 2)
    src = Source(GAUSS_SINE, (src_i, src_i, y0, y1, 0, z0 - 1), fc=fc, bandwidth=bw)
    plist = [Port(ports[0], +1, y0, y1, z0, z1), Port(ports[1], -1, y0, y1, z0, z1)]
    return Problem(
        name=name, nx=nx, ny=ny, nz=nz, dx=delta, dy=delta, dz=delta, courant=0.99,
        normalized=False, materials=mats, cells=cells,
        faces=(CPML, CPML, CPML, CPML, PEC, CPML), pml_cells=(pml,) * 6,
        source=src, ports=plist, freqs=linear_freqs(band[0], band[1], nf),
        nsteps=nsteps, fp32=fp32)


def single_microstrip(twin: bool = False, nsteps: int = 20000) -> Problem:
    """400x120x80 cells at 5 nm, silicon substrate below z = 20, 8-cell PEC
    strip, 10-cell absorbing layers, source at x = 20, probes at x = 60 and
    x = 340, 64 frequencies.  ``twin`` reads the band in THz (10-300 THz,
    pulse centred at 150 THz, 300 THz wide): the same discrete problem as
    5 um cells at 10-300 GHz."""
    s = 1e3 if twin else 1.0
    return microstrip(name="microstrip_400x120x80" + ("_thz" if twin else ""),
                      band=(10e9 * s, 300e9 * s), fc=150e9 * s, bw=300e9 * s,
                      nsteps=nsteps)


BATCH_WIDTHS = {4: 100, 6: 108, 8: 116, 10: 124, 12: 132, 16: 140}


def batched_smatrix(twin: bool = False, nsteps: int = 20000) -> List[Problem]:
    """Six strip widths, each on its own y extent, times the two
    excitations of a 2-port (source next to port 1 or next to port 2):
    12 uneven instances."""
    s = 1e3 if twin else 1.0
    out = []
    for w, ny in BATCH_WIDTHS.items():
        for exc, src_i in ((1, 20), (2, 380)):
            p = microstrip(name=f"microstrip_w{w}_ny{ny}_p{exc}", ny=ny, strip_w=w,
                           src_i=src_i, band=(10e9 * s, 300e9 * s), fc=150e9 * s,
                           bw=300e9 * s, nsteps=nsteps)
            out.append(p)
    return out


def large_line(nsteps: int = 2000, seed: int = 3) -> Problem:
    """1024x512x256 cells at 2 nm: substrate below z = 96 built from runs of
    2-8 cells, each silicon or oxide with probability 1/2; a lossy metal strip
    (5.8e7 S/m) 32 cells wide and 4 thick on top; PEC ground; 12-cell
    absorbing layers; band 10-300 THz."""
    nx, ny, nz = 1024, 512, 256
    rng = np.random.default_rng(seed)
    mats = [Material(1.0), Material(11.7), Material(3.9), Material(1.0, sigma=5.8e7)]
    cells = np.zeros((nz, ny, nx), dtype=np.uint8)
    k = 0
    while k < 96:
        run = int(rng.integers(2, 9))
        mid = 1 if rng.random() < 0.5 else 2
        cells[k:min(96, k + run)] = mid
        k += run
    y0 = (ny - 32) // 2
    y1 = y0 + 32
    cells[96:100, y0:y1, :] = 3
    src = Source(GAUSS_SINE, (24, 24, y0, y1, 0, 95), fc=150e12, bandwidth=300e12)
    plist = [Port(64, +1, y0, y1, 96, 100), Port(960, -1, y0, y1, 96, 100)]
    return Problem(
        name="large_line_1024x512x256", nx=nx, ny=ny, nz=nz, dx=2e-9, dy=2e-9, dz=2e-9,
        courant=0.99, normalized=False, materials=mats, cells=cells,
        faces=(CPML, CPML, CPML, CPML, PEC, CPML), pml_cells=(12,) * 6, source=src,
        ports=plist, freqs=linear_freqs(10e12, 300e12, 64), nsteps=nsteps, fp32=True)


SWEEP_SHAPES = [
    (128, 128, 128), (144, 128, 128), (152, 136, 120), (168, 136, 120),
    (176, 136, 120), (192, 136, 120), (208, 144, 112), (216, 144, 112),
    (232, 144, 112), (240, 144, 112), (256, 152, 104), (272, 152, 104),
    (280, 152, 104), (296, 152, 104), (304, 160, 96), (320, 160, 96),
]


def geometry_sweep(nsteps: int = 50000, shapes=None) -> List[Problem]:
    """16 microstrips of uneven size, each with 5-20 seeded rectangular
    dielectric inclusions (eps_r uniform in [2, 12], sides 4-16 cells) in the
    interior outside the absorbing layers; one excited port each."""
    out = []
    pml = 10
    for idx, (nx, ny, nz) in enumerate(shapes or SWEEP_SHAPES):
        rng = np.random.default_rng(5000 + idx)
        sub_top = nz // 4
        p = microstrip(name=f"sweep_{idx:02d}_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz,
                       sub_top=sub_top, pml=pml, src_i=20, ports=(60, nx - 60),
                       nsteps=nsteps, nf=32, band=(10e12, 300e12), fc=150e12, bw=300e12)
        count = int(rng.integers(5, 21))
        for _ in range(count):
            sx, sy, sz = (int(v) for v in rng.integers(4, 17, 3))
            eps = float(rng.uniform(2.0, 12.0))
            x0 = int(rng.integers(pml, nx - pml - sx + 1))
            y0 = int(rng.integers(pml, ny - pml - sy + 1))
            z0 = int(rng.integers(0, nz - pml - sz + 1))
            p.materials.append(Material(eps))
            p.cells[z0:z0 + sz, y0:y0 + sy, x0:x0 + sx] = len(p.materials) - 1
        # the strip stays a conductor wherever an inclusion overlapped it
        port = p.ports[0]
        p.cells[port.z0:port.z1, port.y0:port.y1, :] = 2
        out.append(p)
    return out


def paper_microstrip(nsteps: int = 60000, nf: int = 240, pml: int = 10, strip_cells: int = 1,
                     ports=(100, 900), src_i: int = 40) -> Problem:
    """The verification line of the paper's Sec. II-B, with x as the
    propagation axis: 1000 (x) by 200 (y) by 50 (z) cells of 0.1 mm, oxide
    (eps_r 3.8) 1 mm thick (10 cells) on a PEC ground, a PEC strip 5.7 mm
    (57 cells) wide along the whole line, CFL 0.9, differential Gaussian
    sigma = 11.254 ps (t0 = 3 sigma), 60 000 steps, absorbing layers on the
    other five faces.  The strip thickness, the port positions and the
    frequency grid are not given in the paper: one cell, ports 800 cells
    apart, and 240 frequencies over 0.25-60 GHz (the phase of the 80 mm line
    then turns by under a radian between neighbouring frequencies, so its
    delay unwraps unambiguously)."""
    nx, ny, nz = 1000, 200, 50
    h, w = 10, 57
    y0 = (ny - w) // 2
    y1 = y0 + w
    mats = [Material(1.0), Material(3.8), Material(1.0, pec=True)]
    cells = np.zeros((nz, ny, nx), dtype=np.uint8)
    cells[:h] = 1
    cells[h:h + strip_cells, y0:y1, :] = 2
    src = Source(DIFF_GAUSSIAN, (src_i, src_i, y0, y1, 0, h - 1), width=11.254e-12)
    plist = [Port(ports[0], +1, y0, y1, h, h + strip_cells),
             Port(ports[1], -1, y0, y1, h, h + strip_cells)]
    return Problem(
        name="paper_microstrip_1000x200x50", nx=nx, ny=ny, nz=nz, dx=1e-4, dy=1e-4, dz=1e-4,
        courant=0.9, normalized=False, materials=mats, cells=cells,
        faces=(CPML, CPML, CPML, CPML, PEC, CPML), pml_cells=(pml,) * 6, source=src,
        ports=plist, freqs=linear_freqs(0.25e9, 60e9, nf), nsteps=nsteps, fp32=True)


# ---------------------------------------------------------------------------
# Non-uniform 2-port: the four runs of the incident/total protocol
# ---------------------------------------------------------------------------

def step_circuit(nx=400, ny=120, nz=80, delta=5e-9, w1=8, w2=16, step_x=200, sub_top=20,
                 strip_t=2, pml=10, src_margin=20, port_margin=60, nsteps=20000, nf=64,
                 twin=True, fp32=True, z_step=0):
    """A microstrip whose strip changes width (w1 -> w2 cells) and, with
    ``z_step`` > 0, also rises by that many cells at x = ``step_x``.

    Returns the runs of the per-port protocol as a dict:
      inc1 / inc2: a uniform line with port 1's / port 2's cross-section,
                   driven next to that port (no internal reflections);
      tot1 / tot2: the full circuit driven next to port 1 / port 2.
    Every run carries both ports (port 1 at x = port_margin, inward +x;
    port 2 at x = nx - port_margin, inward -x)."""
    s = 1e3 if twin else 1.0
    band = (10e9 * s, 300e9 * s)
    mats = [Material(1.0), Material(11.7), Material(1.0, pec=True)]

    def strip_box(w, zlift):
        y0 = (ny - w) // 2
        return y0, y0 + w, sub_top + zlift, sub_top + zlift + strip_t

    b1, b2 = strip_box(w1, 0), strip_box(w2, z_step)

    def cells_for(kind):
        c = np.zeros((nz, ny, nx), dtype=np.uint8)
        c[:sub_top] = 1
        if kind == "uniform1":
            c[b1[2]:b1[3], b1[0]:b1[1], :] = 2
        elif kind == "uniform2":
            c[:sub_top + z_step] = 1
            c[b2[2]:b2[3], b2[0]:b2[1], :] = 2
        else:
            c[b1[2]:b1[3], b1[0]:b1[1], :step_x] = 2
            c[sub_top:sub_top + z_step, :, step_x:] = 1
            c[b2[2]:b2[3], b2[0]:b2[1], step_x:] = 2
        return c

    ports = [Port(port_margin, +1, b1[0], b1[1], b1[2], b1[3]),
             Port(nx - port_margin, -1, b2[0], b2[1], b2[2], b2[3])]
    src1 = Source(GAUSS_SINE, (src_margin, src_margin, b1[0], b1[1], 0, b1[2] - 1),
                  fc=150e9 * s, bandwidth=300e9 * s)
    src2 = Source(GAUSS_SINE, (nx - src_margin, nx - src_margin, b2[0], b2[1], 0, b2[2] - 1),
                  fc=150e9 * s, bandwidth=300e9 * s)

    def prob(name, kind, src):
        return Problem(name=f"step_{name}_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, dx=delta,
                       dy=delta, dz=delta, courant=0.99, normalized=False,
                       materials=[Material(m.eps_r, m.sigma, m.pec) for m in mats],
                       cells=cells_for(kind), faces=(CPML, CPML, CPML, CPML, PEC, CPML),
                       pml_cells=(pml,) * 6, source=src, ports=list(ports),
                       freqs=linear_freqs(band[0], band[1], nf), nsteps=nsteps, fp32=fp32)

    return {"inc1": prob("inc1", "uniform1", src1), "tot1": prob("tot1", "step", src1),
            "inc2": prob("inc2", "uniform2", src2), "tot2": prob("tot2", "step", src2)}


def small_step_circuit(fp32: bool = True, pulse_width: Optional[float] = None,
                       lossy: bool = False, scale: int = 1) -> dict:
    """The 96x40x28 step circuit of the convergence checks (5 nm cells: a
    4-cell strip on an 8-cell silicon substrate that widens to 8 cells and
    rises by one cell halfway; 8-cell absorbing layers; 16 frequencies over
    10-300 THz; 9000 steps), as the four runs of the per-port protocol.
    ``pulse_width``: excite with eq. 3's differential Gaussian of that sigma
    (seconds) instead of the Gaussian-modulated sine; ``lossy``: the strip is
    a 5.8e7 S/m metal instead of PEC and the runs last 36 000 steps (the
    lossy line rings down slowly); ``scale``: cells ``scale`` times finer,
    every feature and the step count scaled with them."""
    s = scale
    runs = step_circuit(nx=96 * s, ny=40 * s, nz=28 * s, delta=5e-9 / s, w1=4 * s, w2=8 * s,
                        step_x=48 * s, sub_top=8 * s, strip_t=2 * s, pml=8 * s,
                        src_margin=12 * s, port_margin=24 * s,
                        nsteps=(36000 if lossy else 9000) * s, nf=16, fp32=fp32, z_step=1 * s)
    for p in runs.values():
        if pulse_width is not None:
            p.source = Source(DIFF_GAUSSIAN, p.source.box, width=pulse_width)
        if lossy:
            p.materials[2] = Material(1.0, sigma=5.8e7)
    return runs


def window(p: Problem, box: Tuple[int, int, int, int, int, int], name: str = "") -> Problem:
    """The cells [x0, x1) x [y0, y1) x [z0, z1) of ``p`` as a problem of
    their own, for light-cone checks: faces that are faces of ``p`` keep their
    boundary and layers, cut faces become PEC.  The source is clipped to the
    window (its nodes re-indexed); ports and point probes are dropped.  After
    n steps the fields of the window agree with those of ``p`` on every cell
    more than n + 1 cells away from a cut face."""
    x0, x1, y0, y1, z0, z1 = box
    lo, hi = (x0, y0, z0), (x1, y1, z1)
    n = (p.nx, p.ny, p.nz)
    assert all(0 <= lo[a] < hi[a] <= n[a] for a in range(3))
    faces, pml = [], []
    for a in range(3):
        for side, cut in ((0, lo[a] > 0), (1, hi[a] < n[a])):
            faces.append(PEC if cut else p.faces[2 * a + side])
            pml.append(0 if cut else p.pml_cells[2 * a + side])
    src = None
    if p.source is not None:
        s = p.source
        b = list(s.box)
        clipped = []
        for a in range(3):
            c0, c1 = max(b[2 * a], lo[a]), min(b[2 * a + 1], hi[a] - 1)
            clipped += [c0 - lo[a], c1 - lo[a]]
        if all(clipped[2 * a] <= clipped[2 * a + 1] for a in range(3)):
            src = Source(s.kind, tuple(clipped), s.t0, s.width, s.fc, s.bandwidth, s.amplitude,
                         s.comp, s.samples)
    return Problem(
        name=name or f"{p.name}_window", nx=x1 - x0, ny=y1 - y0, nz=z1 - z0, dx=p.dx, dy=p.dy,
        dz=p.dz, courant=p.courant, normalized=p.normalized,
        materials=[Material(m.eps_r, m.sigma, m.pec) for m in p.materials],
        cells=np.ascontiguousarray(p.cells[z0:z1, y0:y1, x0:x1]), faces=tuple(faces),
        pml_cells=tuple(pml), pml_m=p.pml_m, pml_sigma_max=p.pml_sigma_max,
        pml_kappa_max=p.pml_kappa_max, pml_alpha_max=p.pml_alpha_max, source=src,
        freqs=p.freqs.copy(), nsteps=p.nsteps, fp32=p.fp32)


# ---------------------------------------------------------------------------
# Test-only geometries
# ---------------------------------------------------------------------------

def parallel_plate(nx=240, ny=2, gap=6, top=4, eps_r=2.25, pml=16, src_i=30,
                   ports=(60, 180), nsteps=2400, nf=32, band=(0.01, 0.06),
                   fc=0.035, bw=0.09) -> Problem:
    """TEM parallel-plate line in normalized units: PEC ground at z = 0, a
    PEC plate filling z >= ``gap`` up to the top face, magnetic walls on both
    y faces (an infinitely wide plate), absorbing layers on both x faces.
    The plate spans the full width, so w = ny cells and d = gap cells."""
    nz = gap + top
    mats = [Material(eps_r), Material(1.0, pec=True)]
    cells = np.zeros((nz, ny, nx), dtype=np.uint8)
    cells[gap:, :, :] = 1
    src = Source(GAUSS_SINE, (src_i, src_i, 0, ny, 0, gap - 1), fc=fc, bandwidth=bw)
    plist = [Port(ports[0], +1, 0, ny, gap, nz), Port(ports[1], -1, 0, ny, gap, nz)]
    return Problem(
        name="parallel_plate", nx=nx, ny=ny, nz=nz, dx=1.0, dy=1.0, dz=1.0, courant=0.99,
        normalized=True, materials=mats, cells=cells,
        faces=(CPML, CPML, PMC, PMC, PEC, PEC), pml_cells=(pml, pml, 0, 0, 0, 0),
        source=src, ports=plist, freqs=linear_freqs(band[0], band[1], nf),
        nsteps=nsteps, fp32=False)


def small_microstrip(nx=96, ny=40, nz=28, strip_w=6, sub_top=8, pml=8, src_i=14,
                     ports=(24, 72), nsteps=600, nf=16, twin=True, fp32=True,
                     eps_sub=11.7, sigma_strip=0.0, seed=None) -> Problem:
    """A small microstrip with the same structure as the 400x120x80 line,
    sized so that the oracle finishes in seconds while the grid still spans
    several kernel tiles and ragged tile tails in every axis.  With ``seed``
    the substrate gets a seeded layer stack and the strip can be lossy."""
    s = 1e3 if twin else 1.0
    p = microstrip(name=f"small_microstrip_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz,
                   sub_top=sub_top, strip_w=strip_w, pml=pml, src_i=src_i, ports=ports,
                   nsteps=nsteps, nf=nf, band=(10e9 * s, 300e9 * s), fc=150e9 * s,
                   bw=300e9 * s, fp32=fp32, eps_sub=eps_sub)
    if seed is not None:
        rng = np.random.default_rng(seed)
        p.materials.append(Material(3.9))
        k = 0
        while k < sub_top:
            run = int(rng.integers(1, 4))
            if rng.random() < 0.5:
                p.cells[k:min(sub_top, k + run)] = len(p.materials) - 1
            k += run
    if sigma_strip > 0:
        p.materials[2] = Material(1.0, sigma=sigma_strip)
    return p
