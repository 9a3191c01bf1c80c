"""MI355X FDTD S-parameter library: Python binding of include/fdtd.h.

The functions named ``fdtd_*`` forward one-to-one to the C interface
(argument marshalling only; all computation happens in libfdtd.so).  The
``Simulation`` and ``BatchSimulation`` helpers issue the C calls that
describe a ``workloads.Problem`` and hold the device workspace as a torch
uint8 tensor; torch supplies device memory and the stream, nothing else.
"""
from __future__ import annotations

import ctypes as C
from typing import List, Optional, Sequence

import numpy as np

from ._capi import (FACE_CPML, FACE_PEC, FP32, FP64, KERNEL_FUSED, KERNEL_PLAIN, NORMALIZED,
                    SI, FdtdError, check, fdtd_boundary, fdtd_grid, fdtd_material, fdtd_port,
                    fdtd_source, lib)

__all__ = ["FdtdError", "Simulation", "BatchSimulation", "fdtd_sparams", "lib"]

_PD = C.POINTER(C.c_double)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_PD)


def _stream(stream=None):
    if stream is not None:
        return C.c_void_p(int(stream))
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


# ---------------------------------------------------------------------------
# thin wrappers with the C names
# ---------------------------------------------------------------------------

def fdtd_plan_create(nx, ny, nz, dx, dy, dz, courant, precision=FP32, units=SI,
                     kernel=KERNEL_PLAIN):
    g = fdtd_grid(nx, ny, nz, dx, dy, dz, courant, precision, units, kernel)
    h = C.c_void_p()
    check(lib().fdtd_plan_create(C.byref(g), C.byref(h)), "fdtd_plan_create")
    return h


def fdtd_plan_set_materials(plan, cells: np.ndarray, table):
    cells = np.ascontiguousarray(cells, dtype=np.uint8)
    mats = (fdtd_material * len(table))(*[fdtd_material(m.eps_r, m.sigma, 1 if m.pec else 0)
                                          for m in table])
    check(lib().fdtd_plan_set_materials(plan, cells.ctypes.data_as(C.POINTER(C.c_uint8)),
                                        mats, len(table)), "fdtd_plan_set_materials", plan)


def fdtd_plan_set_boundary(plan, faces, cells, m=3.0, sigma_max=0.0, kappa_max=1.0,
                           alpha_max=0.0):
    b = fdtd_boundary((C.c_int32 * 6)(*faces), (C.c_int32 * 6)(*cells), m, sigma_max,
                      kappa_max, alpha_max)
    check(lib().fdtd_plan_set_boundary(plan, C.byref(b)), "fdtd_plan_set_boundary", plan)


def fdtd_plan_add_port(plan, i, direction, y0, y1, z0, z1) -> int:
    q = fdtd_port(i, direction, y0, y1, z0, z1)
    out = C.c_int32()
    check(lib().fdtd_plan_add_port(plan, C.byref(q), C.byref(out)), "fdtd_plan_add_port", plan)
    return out.value


def fdtd_plan_add_point_probe(plan, comp, i, j, k) -> int:
    out = C.c_int32()
    check(lib().fdtd_plan_add_point_probe(plan, comp, i, j, k, C.byref(out)),
          "fdtd_plan_add_point_probe", plan)
    return out.value


def fdtd_plan_set_source(plan, kind, box, t0=0.0, width=0.0, fc=0.0, bandwidth=0.0,
                         amplitude=1.0):
    s = fdtd_source(kind, (C.c_int32 * 6)(*box), t0, width, fc, bandwidth, amplitude)
    check(lib().fdtd_plan_set_source(plan, C.byref(s)), "fdtd_plan_set_source", plan)


def fdtd_plan_set_source_samples(plan, samples):
    s = np.ascontiguousarray(samples, dtype=np.float64)
    check(lib().fdtd_plan_set_source_samples(plan, _ptr(s), len(s)),
          "fdtd_plan_set_source_samples", plan)


def fdtd_plan_set_frequencies(plan, freqs):
    f = np.ascontiguousarray(freqs, dtype=np.float64)
    check(lib().fdtd_plan_set_frequencies(plan, _ptr(f), len(f)), "fdtd_plan_set_frequencies", plan)


def fdtd_plan_workspace_size(plan) -> int:
    n = C.c_size_t()
    check(lib().fdtd_plan_workspace_size(plan, C.byref(n)), "fdtd_plan_workspace_size", plan)
    return n.value


def fdtd_plan_get_dt(plan) -> float:
    v = C.c_double()
    check(lib().fdtd_plan_get_dt(plan, C.byref(v)), "fdtd_plan_get_dt", plan)
    return v.value


def fdtd_plan_bind(plan, dptr: int, nbytes: int, stream=None):
    check(lib().fdtd_plan_bind(plan, C.c_void_p(dptr), nbytes, _stream(stream)),
          "fdtd_plan_bind", plan)


def fdtd_reset(plan, stream=None):
    check(lib().fdtd_reset(plan, _stream(stream)), "fdtd_reset", plan)


def fdtd_run(plan, nsteps: int, stream=None):
    check(lib().fdtd_run(plan, int(nsteps), _stream(stream)), "fdtd_run", plan)


def fdtd_run_noalloc(plan, nsteps: int, stream=None):
    check(lib().fdtd_run_noalloc(plan, int(nsteps), _stream(stream)), "fdtd_run_noalloc", plan)


def fdtd_get_step(plan) -> int:
    v = C.c_int64()
    check(lib().fdtd_get_step(plan, C.byref(v)), "fdtd_get_step", plan)
    return v.value


def fdtd_get_spectra(plan, probe: int, nf: int, stream=None):
    V = np.zeros(2 * nf)
    I = np.zeros(2 * nf)
    check(lib().fdtd_get_spectra(plan, probe, _ptr(V), _ptr(I), _stream(stream)),
          "fdtd_get_spectra", plan)
    return V[0::2] + 1j * V[1::2], I[0::2] + 1j * I[1::2]


def fdtd_read_field(plan, comp: int, shape, stream=None) -> np.ndarray:
    out = np.zeros(shape)
    check(lib().fdtd_read_field(plan, comp, _ptr(out), _stream(stream)), "fdtd_read_field", plan)
    return out


def fdtd_write_field(plan, comp: int, values: np.ndarray, stream=None):
    v = np.ascontiguousarray(values, dtype=np.float64)
    check(lib().fdtd_write_field(plan, comp, _ptr(v), _stream(stream)), "fdtd_write_field", plan)


def fdtd_checkpoint_size(plan) -> int:
    n = C.c_size_t()
    check(lib().fdtd_checkpoint_size(plan, C.byref(n)), "fdtd_checkpoint_size", plan)
    return n.value


def fdtd_checkpoint_save(plan, stream=None) -> np.ndarray:
    buf = np.zeros(fdtd_checkpoint_size(plan), dtype=np.uint8)
    check(lib().fdtd_checkpoint_save(plan, buf.ctypes.data_as(C.c_void_p), buf.nbytes,
                                     _stream(stream)), "fdtd_checkpoint_save", plan)
    return buf


def fdtd_checkpoint_load(plan, buf: np.ndarray, stream=None):
    check(lib().fdtd_checkpoint_load(plan, buf.ctypes.data_as(C.c_void_p), buf.nbytes,
                                     _stream(stream)), "fdtd_checkpoint_load", plan)


def fdtd_plan_set_config(plan, rows: int, zchunk: int):
    check(lib().fdtd_plan_set_config(plan, rows, zchunk), "fdtd_plan_set_config", plan)


def fdtd_plan_get_config(plan):
    r, z = C.c_int32(), C.c_int32()
    check(lib().fdtd_plan_get_config(plan, C.byref(r), C.byref(z)), "fdtd_plan_get_config", plan)
    return r.value, z.value


def fdtd_plan_set_tile_order(plan, order: int):
    check(lib().fdtd_plan_set_tile_order(plan, order), "fdtd_plan_set_tile_order", plan)


def fdtd_plan_get_tile_order(plan):
    o, u = C.c_int32(), C.c_int32()
    check(lib().fdtd_plan_get_tile_order(plan, C.byref(o), C.byref(u)),
          "fdtd_plan_get_tile_order", plan)
    return o.value, u.value


def fdtd_plan_set_stream_stores(plan, mode: int):
    check(lib().fdtd_plan_set_stream_stores(plan, mode), "fdtd_plan_set_stream_stores", plan)


def fdtd_plan_get_stream_stores(plan):
    m, u = C.c_int32(), C.c_int32()
    check(lib().fdtd_plan_get_stream_stores(plan, C.byref(m), C.byref(u)),
          "fdtd_plan_get_stream_stores", plan)
    return m.value, u.value


def fdtd_plan_set_temporal(plan, mode: int):
    check(lib().fdtd_plan_set_temporal(plan, mode), "fdtd_plan_set_temporal", plan)


def fdtd_plan_set_temporal_config(plan, rows: int, zchunk: int):
    check(lib().fdtd_plan_set_temporal_config(plan, rows, zchunk),
          "fdtd_plan_set_temporal_config", plan)


def fdtd_plan_get_temporal(plan):
    """(mode, used, tile_rows, zchunk, tiles)."""
    v = [C.c_int32() for _ in range(5)]
    check(lib().fdtd_plan_get_temporal(plan, *[C.byref(x) for x in v]),
          "fdtd_plan_get_temporal", plan)
    return tuple(x.value for x in v)


def fdtd_plan_autotune(plan, trial_steps: int = 20, cache_path: Optional[str] = None,
                       stream=None) -> int:
    best = C.c_int32()
    path = cache_path.encode() if cache_path else None
    check(lib().fdtd_plan_autotune(plan, trial_steps, path, _stream(stream), C.byref(best)),
          "fdtd_plan_autotune", plan)
    return best.value


def fdtd_plan_set_timing(plan, enable):
    """enable: False/0 off, True/1 every step, n > 1 every n-th step."""
    check(lib().fdtd_plan_set_timing(plan, int(enable)), "fdtd_plan_set_timing", plan)


def fdtd_plan_get_kernel_time(plan):
    ms, n = C.c_double(), C.c_int64()
    check(lib().fdtd_plan_get_kernel_time(plan, C.byref(ms), C.byref(n)),
          "fdtd_plan_get_kernel_time", plan)
    return ms.value, n.value


def fdtd_plan_destroy(plan):
    if plan:
        lib().fdtd_plan_destroy(plan)


def fdtd_sparams(freqs, Vinc, Iinc, Vtot, z_ref=50.0):
    """Host FP64 post-processing in the library (eqs. 1, 2, 5-8 and the
    ABCD step).  Vinc, Iinc: [np, nf] complex; Vtot: [np, np, nf] complex.
    Returns dict with S_star [nf, np, np], S, Zr [nf, np], Z0 [nf] (2-ports)
    and tau [nf, np, np]."""
    f = np.ascontiguousarray(freqs, dtype=np.float64)
    nf = len(f)
    n = Vinc.shape[0]

    def inter(z):
        z = np.asarray(z, dtype=complex)
        out = np.empty(z.shape + (2,))
        out[..., 0], out[..., 1] = z.real, z.imag
        return np.ascontiguousarray(out)

    vi, ii, vt = inter(Vinc), inter(Iinc), inter(Vtot)
    Ss = np.zeros((nf, n, n, 2))
    S = np.zeros((nf, n, n, 2))
    Zr = np.zeros((nf, n, 2))
    Z0 = np.zeros((nf, 2))
    tau = np.zeros((nf, n, n))
    check(lib().fdtd_sparams(n, nf, _ptr(f), _ptr(vi), _ptr(ii), _ptr(vt), z_ref, _ptr(Ss),
                             _ptr(S), _ptr(Zr), _ptr(Z0), _ptr(tau)), "fdtd_sparams")
    c = lambda a: a[..., 0] + 1j * a[..., 1]
    return {"S_star": c(Ss), "S": c(S), "Zr": c(Zr), "Z0": c(Z0) if n == 2 else None, "tau": tau}


def fdtd_device_copy(dst, src, stream=None):
    """Copy the device tensor ``src`` into ``dst`` (same byte size, 16-byte
    multiples, no overlap) with the library's streaming copy kernel."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("fdtd_device_copy: size mismatch")
    check(lib().fdtd_device_copy(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), nbytes,
                                 _stream(stream)), "fdtd_device_copy")


def protocol_from_runs(spectra):
    """Arrange the spectra of the four runs of a 2-port's protocol ("inc1",
    "inc2": port j driven on its uniform line; "tot1", "tot2": the full
    circuit driven at port j; each (V[probe, f], I[probe, f]), probe 0 =
    port 1) into the Vinc, Iinc, Vtot arrays fdtd_sparams takes."""
    V1, I1 = spectra["inc1"]
    V2, I2 = spectra["inc2"]
    T1 = spectra["tot1"][0]
    T2 = spectra["tot2"][0]
    return (np.stack([V1[0], V2[1]]), np.stack([I1[0], I2[1]]),
            np.stack([np.stack([T1[0], T1[1]]), np.stack([T2[0], T2[1]])]))


# ---------------------------------------------------------------------------
# helpers that describe a workloads.Problem through the calls above
# ---------------------------------------------------------------------------

def describe(prob, fused: bool = True, precision: Optional[int] = None):
    """Create and fill a plan for ``prob`` (a workloads.Problem)."""
    if precision is None:
        precision = FP32 if prob.fp32 else FP64
    kernel = KERNEL_FUSED if (fused and precision == FP32) else KERNEL_PLAIN
    h = fdtd_plan_create(prob.nx, prob.ny, prob.nz, prob.dx, prob.dy, prob.dz, prob.courant,
                         precision, NORMALIZED if prob.normalized else SI, kernel)
    try:
        fdtd_plan_set_materials(h, prob.cells, prob.materials)
        for f in prob.faces:
            if f not in (FACE_PEC, FACE_CPML):
                raise FdtdError(-3, "describe", "only PEC and CPML faces run on the GPU")
        fdtd_plan_set_boundary(h, prob.faces, prob.pml_cells, prob.pml_m, prob.pml_sigma_max,
                               prob.pml_kappa_max, prob.pml_alpha_max)
        for q in prob.ports:
            fdtd_plan_add_port(h, q.i, q.direction, q.y0, q.y1, q.z0, q.z1)
        for q in prob.points:
            fdtd_plan_add_point_probe(h, q.comp, q.i, q.j, q.k)
        if prob.source is not None:
            s = prob.source
            if s.comp != 2:
                raise FdtdError(-3, "describe", "the GPU source drives Ez")
            fdtd_plan_set_source(h, s.kind, s.box, s.t0, s.width, s.fc, s.bandwidth, s.amplitude)
            if getattr(s, "samples", None) is not None:
                fdtd_plan_set_source_samples(h, s.samples)
        fdtd_plan_set_frequencies(h, prob.freqs)
    except Exception:
        fdtd_plan_destroy(h)
        raise
    return h


class Simulation:
    """One plan bound to a torch-owned device workspace."""

    def __init__(self, prob, fused: bool = True, precision: Optional[int] = None,
                 config=None, device: str = "cuda", temporal: Optional[int] = None,
                 temporal_config=None):
        import torch
        self.prob = prob
        self.handle = describe(prob, fused=fused, precision=precision)
        if config is not None:
            fdtd_plan_set_config(self.handle, *config)
        if temporal is not None:
            fdtd_plan_set_temporal(self.handle, temporal)
        if temporal_config is not None:
            fdtd_plan_set_temporal_config(self.handle, *temporal_config)
        self.nbytes = fdtd_plan_workspace_size(self.handle)
        self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        fdtd_plan_bind(self.handle, self.workspace.data_ptr(), self.nbytes)
        self.dt = fdtd_plan_get_dt(self.handle)
        self.nf = len(prob.freqs)

    def run(self, nsteps: Optional[int] = None):
        fdtd_run(self.handle, self.prob.nsteps if nsteps is None else nsteps)
        return self

    def reset(self):
        fdtd_reset(self.handle)

    def autotune(self, trial_steps: int = 20, cache_path: Optional[str] = None) -> int:
        return fdtd_plan_autotune(self.handle, trial_steps, cache_path)

    def set_tile_order(self, order: int):
        fdtd_plan_set_tile_order(self.handle, order)

    def set_stream_stores(self, mode: int):
        fdtd_plan_set_stream_stores(self.handle, mode)

    def stream_stores(self):
        return fdtd_plan_get_stream_stores(self.handle)

    def tile_order(self):
        return fdtd_plan_get_tile_order(self.handle)

    def get_config(self):
        return fdtd_plan_get_config(self.handle)

    def temporal(self):
        """(mode, used, tile_rows, zchunk, two-level tiles)."""
        return fdtd_plan_get_temporal(self.handle)

    @property
    def step(self) -> int:
        return fdtd_get_step(self.handle)

    def spectra(self):
        V, I = [], []
        for q in range(self.prob.n_probes()):
            v, i = fdtd_get_spectra(self.handle, q, self.nf)
            V.append(v)
            I.append(i)
        return np.array(V), np.array(I)

    def field(self, comp: int) -> np.ndarray:
        p = self.prob
        return fdtd_read_field(self.handle, comp, (p.nz + 1, p.ny + 1, p.nx + 1))

    def set_field(self, comp: int, values: np.ndarray):
        fdtd_write_field(self.handle, comp, values)

    def checkpoint(self) -> np.ndarray:
        return fdtd_checkpoint_save(self.handle)

    def restore(self, buf: np.ndarray):
        fdtd_checkpoint_load(self.handle, buf)

    def close(self):
        if self.handle:
            fdtd_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchSimulation:
    """Many FP32 fused plans stepped together by one launch per step."""

    def __init__(self, probs: Sequence, config=None, device: str = "cuda"):
        import torch
        self.probs = list(probs)
        self.handles = [describe(p, fused=True, precision=FP32) for p in self.probs]
        arr = (C.c_void_p * len(self.handles))(*[h.value for h in self.handles])
        self.handle = C.c_void_p()
        check(lib().fdtd_batch_create(arr, len(self.handles), C.byref(self.handle)),
              "fdtd_batch_create", None, batch=True)
        if config is not None:
            self.set_config(*config)
        n = C.c_size_t()
        check(lib().fdtd_batch_workspace_size(self.handle, C.byref(n)),
              "fdtd_batch_workspace_size", self.handle, batch=True)
        self.nbytes = n.value
        self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        check(lib().fdtd_batch_bind(self.handle, C.c_void_p(self.workspace.data_ptr()),
                                    self.nbytes, _stream()), "fdtd_batch_bind", self.handle,
              batch=True)

    def run(self, nsteps: int):
        check(lib().fdtd_batch_run(self.handle, int(nsteps), _stream()), "fdtd_batch_run",
              self.handle, batch=True)
        return self

    def reset(self):
        check(lib().fdtd_batch_reset(self.handle, _stream()), "fdtd_batch_reset", self.handle,
              batch=True)

    def set_config(self, rows: int, zchunk: int):
        check(lib().fdtd_batch_set_config(self.handle, rows, zchunk), "fdtd_batch_set_config",
              self.handle, batch=True)

    def set_tile_order(self, order: int):
        check(lib().fdtd_batch_set_tile_order(self.handle, order), "fdtd_batch_set_tile_order",
              self.handle, batch=True)

    def set_stream_stores(self, mode: int):
        check(lib().fdtd_batch_set_stream_stores(self.handle, mode),
              "fdtd_batch_set_stream_stores", self.handle, batch=True)

    def set_group_bytes(self, nbytes: int):
        check(lib().fdtd_batch_set_group_bytes(self.handle, nbytes), "fdtd_batch_set_group_bytes",
              self.handle, batch=True)

    def groups(self) -> int:
        n = C.c_int32()
        check(lib().fdtd_batch_get_groups(self.handle, C.byref(n)), "fdtd_batch_get_groups",
              self.handle, batch=True)
        return n.value

    def tile_order(self):
        o, u = C.c_int32(), C.c_int32()
        check(lib().fdtd_batch_get_tile_order(self.handle, C.byref(o), C.byref(u)),
              "fdtd_batch_get_tile_order", self.handle, batch=True)
        return o.value, u.value

    def get_config(self):
        r, z = C.c_int32(), C.c_int32()
        check(lib().fdtd_batch_get_config(self.handle, C.byref(r), C.byref(z)),
              "fdtd_batch_get_config", self.handle, batch=True)
        return r.value, z.value

    def autotune(self, trial_steps: int = 20, cache_path: Optional[str] = None) -> int:
        best = C.c_int32()
        path = cache_path.encode() if cache_path else None
        check(lib().fdtd_batch_autotune(self.handle, trial_steps, path, _stream(),
                                        C.byref(best)), "fdtd_batch_autotune", self.handle,
              batch=True)
        return best.value

    def set_timing(self, enable):
        check(lib().fdtd_batch_set_timing(self.handle, int(enable)),
              "fdtd_batch_set_timing", self.handle, batch=True)

    def kernel_time(self):
        ms, n = C.c_double(), C.c_int64()
        check(lib().fdtd_batch_get_kernel_time(self.handle, C.byref(ms), C.byref(n)),
              "fdtd_batch_get_kernel_time", self.handle, batch=True)
        return ms.value, n.value

    def spectra(self, idx: int):
        p = self.probs[idx]
        V, I = [], []
        for q in range(p.n_probes()):
            v, i = fdtd_get_spectra(self.handles[idx], q, len(p.freqs))
            V.append(v)
            I.append(i)
        return np.array(V), np.array(I)

    def field(self, idx: int, comp: int) -> np.ndarray:
        p = self.probs[idx]
        return fdtd_read_field(self.handles[idx], comp, (p.nz + 1, p.ny + 1, p.nx + 1))

    def close(self):
        if self.handle:
            lib().fdtd_batch_destroy(self.handle)
            self.handle = None
        for h in self.handles:
            fdtd_plan_destroy(h)
        self.handles = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
