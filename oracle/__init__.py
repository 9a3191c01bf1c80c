"""FP64 CPU oracle for the FDTD S-parameter path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this package.  It shares no code
with the GPU library: the time stepping lives in ``fdtd64.c`` (plain C,
FP64), the post-processing in ``post.py`` (numpy, FP64).  Problems come from
the ``workloads`` package, which holds geometry only.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle64.so")
SRC_PATH = os.path.join(HERE, "fdtd64.c")


def build(force: bool = True) -> str:
    """Compile the oracle with the host C compiler."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-Wno-unused-function", "-o", LIB_PATH + ".tmp", SRC_PATH, "-lm"]
        subprocess.check_call(cmd)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.or_dt.restype = C.c_double
        L.or_dt.argtypes = [C.POINTER(OrProblem)]
        L.or_setup.restype = C.c_int
        L.or_setup.argtypes = [C.POINTER(OrProblem), C.POINTER(OrState)]
        L.or_run.restype = C.c_int
        L.or_run.argtypes = [C.POINTER(OrProblem), C.POINTER(OrState), C.c_int64]
        L.or_max_threads.restype = C.c_int
        L.or_max_threads.argtypes = []
        L.or_set_threads.restype = None
        L.or_set_threads.argtypes = [C.c_int]
        L.or_waveform.restype = None
        L.or_waveform.argtypes = [C.POINTER(OrProblem), C.c_int64, C.c_int64,
                                  C.POINTER(C.c_double)]
        _lib = L
    return _lib


def threads() -> int:
    """Threads the oracle's parallel loops use (omp_get_max_threads)."""
    return int(lib().or_max_threads())


def set_threads(n: int) -> None:
    """Run the oracle's parallel loops on n threads from now on."""
    lib().or_set_threads(int(n))


PD = C.POINTER(C.c_double)
PI32 = C.POINTER(C.c_int32)


class OrProblem(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
        ("courant", C.c_double), ("normalized", C.c_int32),
        ("nmat", C.c_int32), ("mat_eps", PD), ("mat_sigma", PD), ("mat_pec", PI32),
        ("cells", C.POINTER(C.c_uint8)),
        ("face", C.c_int32 * 6), ("pml_cells", C.c_int32 * 6),
        ("pml_m", C.c_double), ("pml_sigma_max", C.c_double),
        ("pml_kappa_max", C.c_double), ("pml_alpha_max", C.c_double),
        ("src_kind", C.c_int32), ("src_comp", C.c_int32), ("src_box", C.c_int32 * 6),
        ("src_t0", C.c_double), ("src_width", C.c_double), ("src_fc", C.c_double),
        ("src_bw", C.c_double), ("src_amp", C.c_double),
        ("nport", C.c_int32), ("ports", PI32),
        ("npoint", C.c_int32), ("points", PI32),
        ("nf", C.c_int32), ("freqs", PD),
        ("src_nsamp", C.c_int64), ("src_samples", PD),
    ]


class OrState(C.Structure):
    _fields_ = [
        ("e", PD * 3), ("h", PD * 3), ("psi", PD * 12), ("ca", PD * 3), ("cb", PD * 3),
        ("bE", PD * 3), ("cE", PD * 3), ("ikE", PD * 3),
        ("bH", PD * 3), ("cH", PD * 3), ("ikH", PD * 3),
        ("inE", PI32 * 3), ("inH", PI32 * 3),
        ("acc", PD), ("hist", PD), ("hist_len", C.c_int64), ("energy", PD),
        ("step", C.c_int64),
    ]


def _pd(a):
    return a.ctypes.data_as(PD)


def _pi(a):
    return a.ctypes.data_as(PI32)


class Oracle:
    """One simulation of a ``workloads.Problem`` on the CPU in FP64.

    Arrays are numpy-owned; ``checkpoint``/``restore`` copy them.
    Field arrays have shape (nz+1, ny+1, nx+1), x fastest.
    """

    def __init__(self, prob, history: int = 0, energy: bool = False):
        self.prob = prob
        p = prob
        self._keep = []
        keep = self._keep.append
        self.mat_eps = np.array([m.eps_r for m in p.materials], dtype=np.float64)
        self.mat_sigma = np.array([m.sigma for m in p.materials], dtype=np.float64)
        self.mat_pec = np.array([1 if m.pec else 0 for m in p.materials], dtype=np.int32)
        self.cells = np.ascontiguousarray(p.cells, dtype=np.uint8)
        assert self.cells.shape == (p.nz, p.ny, p.nx)
        ports = np.array([[q.i, q.direction, q.y0, q.y1, q.z0, q.z1] for q in p.ports],
                         dtype=np.int32).reshape(-1)
        points = np.array([[q.comp, q.i, q.j, q.k] for q in p.points],
                          dtype=np.int32).reshape(-1)
        if ports.size == 0:
            ports = np.zeros(1, np.int32)
        if points.size == 0:
            points = np.zeros(1, np.int32)
        self.freqs = np.ascontiguousarray(p.freqs, dtype=np.float64)
        if self.freqs.size == 0:
            self.freqs = np.zeros(1)
        for a in (self.mat_eps, self.mat_sigma, self.mat_pec, self.cells, ports, points,
                  self.freqs):
            keep(a)
        pr = OrProblem()
        pr.nx, pr.ny, pr.nz = p.nx, p.ny, p.nz
        pr.dx, pr.dy, pr.dz = p.dx, p.dy, p.dz
        pr.courant = p.courant
        pr.normalized = 1 if p.normalized else 0
        pr.nmat = len(p.materials)
        pr.mat_eps, pr.mat_sigma, pr.mat_pec = _pd(self.mat_eps), _pd(self.mat_sigma), _pi(self.mat_pec)
        pr.cells = self.cells.ctypes.data_as(C.POINTER(C.c_uint8))
        pr.face = (C.c_int32 * 6)(*p.faces)
        pr.pml_cells = (C.c_int32 * 6)(*p.pml_cells)
        pr.pml_m, pr.pml_sigma_max = p.pml_m, p.pml_sigma_max
        pr.pml_kappa_max, pr.pml_alpha_max = p.pml_kappa_max, p.pml_alpha_max
        if p.source is not None:
            s = p.source
            pr.src_kind = s.kind
            pr.src_comp = s.comp
            pr.src_box = (C.c_int32 * 6)(*s.box)
            pr.src_t0, pr.src_width, pr.src_fc = s.t0, s.width, s.fc
            pr.src_bw, pr.src_amp = s.bandwidth, s.amplitude
            if getattr(s, "samples", None) is not None:
                self.src_samples = np.ascontiguousarray(s.samples, dtype=np.float64)
                pr.src_nsamp, pr.src_samples = len(self.src_samples), _pd(self.src_samples)
        pr.nport, pr.ports = len(p.ports), _pi(ports)
        pr.npoint, pr.points = len(p.points), _pi(points)
        pr.nf, pr.freqs = len(p.freqs), _pd(self.freqs)
        self.pr = pr

        shape = (p.nz + 1, p.ny + 1, p.nx + 1)
        self.e = [np.zeros(shape) for _ in range(3)]
        self.h = [np.zeros(shape) for _ in range(3)]
        self.psi = [np.zeros(shape) for _ in range(12)]
        self.ca = [np.zeros(shape) for _ in range(3)]
        self.cb = [np.zeros(shape) for _ in range(3)]
        n = (p.nx, p.ny, p.nz)
        self.prof = {k: [np.zeros(n[a] + 1) for a in range(3)]
                     for k in ("bE", "cE", "ikE", "bH", "cH", "ikH")}
        self.inE = [np.zeros(n[a] + 1, np.int32) for a in range(3)]
        self.inH = [np.zeros(n[a] + 1, np.int32) for a in range(3)]
        nprobe = p.n_probes()
        self.acc = np.zeros((max(nprobe, 1), 2, max(len(p.freqs), 1), 2))
        self.hist_len = int(history)
        self.hist = np.zeros((max(nprobe, 1), 2, max(self.hist_len, 1)))
        self.energy = np.zeros(max(self.hist_len, 1)) if energy else None

        st = OrState()
        for a in range(3):
            st.e[a], st.h[a] = _pd(self.e[a]), _pd(self.h[a])
            st.ca[a], st.cb[a] = _pd(self.ca[a]), _pd(self.cb[a])
            for k in ("bE", "cE", "ikE", "bH", "cH", "ikH"):
                getattr(st, k)[a] = _pd(self.prof[k][a])
            st.inE[a], st.inH[a] = _pi(self.inE[a]), _pi(self.inH[a])
        for q in range(12):
            st.psi[q] = _pd(self.psi[q])
        st.acc = _pd(self.acc)
        st.hist = _pd(self.hist) if self.hist_len > 0 else None
        st.hist_len = self.hist_len
        st.energy = _pd(self.energy) if energy else None
        st.step = 0
        self.st = st
        lib().or_setup(C.byref(self.pr), C.byref(self.st))

    # -- stepping ------------------------------------------------------------
    @property
    def dt(self) -> float:
        return lib().or_dt(C.byref(self.pr))

    @property
    def step(self) -> int:
        return int(self.st.step)

    def run(self, nsteps: int):
        lib().or_run(C.byref(self.pr), C.byref(self.st), int(nsteps))
        return self

    def waveform(self, first_level: int, count: int) -> np.ndarray:
        out = np.zeros(count)
        lib().or_waveform(C.byref(self.pr), int(first_level), int(count), _pd(out))
        return out

    # -- results -------------------------------------------------------------
    def spectra(self):
        """Complex DFTs: V[probe, f], I[probe, f]."""
        a = self.acc[..., 0] + 1j * self.acc[..., 1]
        return a[:, 0, :].copy(), a[:, 1, :].copy()

    def history(self):
        return self.hist[:, 0, :].copy(), self.hist[:, 1, :].copy()

    def field(self, comp: int) -> np.ndarray:
        return (self.e + self.h)[comp]

    def set_field(self, comp: int, values: np.ndarray):
        (self.e + self.h)[comp][...] = values

    # -- checkpoint ----------------------------------------------------------
    def checkpoint(self):
        arrs = self.e + self.h + self.psi + [self.acc, self.hist]
        if self.energy is not None:
            arrs.append(self.energy)
        return ([a.copy() for a in arrs], int(self.st.step))

    def restore(self, ck):
        arrs, step = ck
        dst = self.e + self.h + self.psi + [self.acc, self.hist]
        if self.energy is not None:
            dst.append(self.energy)
        for d, s in zip(dst, arrs):
            d[...] = s
        self.st.step = step


def run_problem(prob, nsteps=None, history=0, energy=False) -> Oracle:
    o = Oracle(prob, history=history, energy=energy)
    o.run(prob.nsteps if nsteps is None else nsteps)
    return o
