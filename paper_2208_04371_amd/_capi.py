"""ctypes declarations of the C interface in include/fdtd.h.

Argument marshalling only: every function here forwards to libfdtd.so.
Errors come back as FdtdError carrying the status code and the library's
message.  The library must have been built (paper_2208_04371_amd.build);
loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfdtd.so")

FDTD_OK = 0
STATUS = {0: "OK", -1: "E_INVALID_ARG", -2: "E_STATE", -3: "E_UNSUPPORTED", -4: "E_HIP",
          -5: "E_NOMEM", -6: "E_DIVERGED"}
FP32, FP64 = 0, 1
SI, NORMALIZED = 0, 1
KERNEL_PLAIN, KERNEL_FUSED = 0, 1
FACE_PEC, FACE_CPML = 0, 1


class FdtdError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str = ""):
        self.code = code
        super().__init__(f"{where}: {STATUS.get(code, code)} {msg}".strip())


class fdtd_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("courant", C.c_double), ("precision", C.c_int32), ("units", C.c_int32),
                ("kernel", C.c_int32)]


class fdtd_material(C.Structure):
    _fields_ = [("eps_r", C.c_double), ("sigma", C.c_double), ("is_pec", C.c_int32)]


class fdtd_boundary(C.Structure):
    _fields_ = [("face", C.c_int32 * 6), ("cells", C.c_int32 * 6), ("m", C.c_double),
                ("sigma_max", C.c_double), ("kappa_max", C.c_double), ("alpha_max", C.c_double)]


class fdtd_port(C.Structure):
    _fields_ = [("i", C.c_int32), ("dir", C.c_int32), ("y0", C.c_int32), ("y1", C.c_int32),
                ("z0", C.c_int32), ("z1", C.c_int32)]


class fdtd_source(C.Structure):
    _fields_ = [("kind", C.c_int32), ("box", C.c_int32 * 6), ("t0", C.c_double),
                ("width", C.c_double), ("fc", C.c_double), ("bandwidth", C.c_double),
                ("amplitude", C.c_double)]


P = C.c_void_p
PD = C.POINTER(C.c_double)
I32, I64, SZ = C.c_int32, C.c_int64, C.c_size_t

# name -> (restype, argtypes)
SIGNATURES = {
    "fdtd_plan_create": (I32, [C.POINTER(fdtd_grid), C.POINTER(P)]),
    "fdtd_plan_set_materials": (I32, [P, C.POINTER(C.c_uint8), C.POINTER(fdtd_material), I32]),
    "fdtd_plan_set_boundary": (I32, [P, C.POINTER(fdtd_boundary)]),
    "fdtd_plan_add_port": (I32, [P, C.POINTER(fdtd_port), C.POINTER(I32)]),
    "fdtd_plan_add_point_probe": (I32, [P, I32, I32, I32, I32, C.POINTER(I32)]),
    "fdtd_plan_set_source": (I32, [P, C.POINTER(fdtd_source)]),
    "fdtd_plan_set_frequencies": (I32, [P, PD, I32]),
    "fdtd_plan_workspace_size": (I32, [P, C.POINTER(SZ)]),
    "fdtd_plan_get_dt": (I32, [P, PD]),
    "fdtd_plan_bind": (I32, [P, P, SZ, P]),
    "fdtd_reset": (I32, [P, P]),
    "fdtd_run": (I32, [P, I64, P]),
    "fdtd_run_noalloc": (I32, [P, I64, P]),
    "fdtd_get_step": (I32, [P, C.POINTER(I64)]),
    "fdtd_get_spectra": (I32, [P, I32, PD, PD, P]),
    "fdtd_read_field": (I32, [P, I32, PD, P]),
    "fdtd_write_field": (I32, [P, I32, PD, P]),
    "fdtd_checkpoint_size": (I32, [P, C.POINTER(SZ)]),
    "fdtd_checkpoint_save": (I32, [P, P, SZ, P]),
    "fdtd_checkpoint_load": (I32, [P, P, SZ, P]),
    "fdtd_last_error": (C.c_char_p, [P]),
    "fdtd_plan_destroy": (None, [P]),
    "fdtd_batch_create": (I32, [C.POINTER(P), I32, C.POINTER(P)]),
    "fdtd_batch_workspace_size": (I32, [P, C.POINTER(SZ)]),
    "fdtd_batch_bind": (I32, [P, P, SZ, P]),
    "fdtd_batch_reset": (I32, [P, P]),
    "fdtd_batch_run": (I32, [P, I64, P]),
    "fdtd_batch_autotune": (I32, [P, I32, C.c_char_p, P, C.POINTER(I32)]),
    "fdtd_batch_get_config": (I32, [P, C.POINTER(I32), C.POINTER(I32)]),
    "fdtd_batch_set_config": (I32, [P, I32, I32]),
    "fdtd_batch_last_error": (C.c_char_p, [P]),
    "fdtd_batch_destroy": (None, [P]),
    "fdtd_plan_get_config": (I32, [P, C.POINTER(I32), C.POINTER(I32)]),
    "fdtd_plan_set_config": (I32, [P, I32, I32]),
    "fdtd_plan_autotune": (I32, [P, I32, C.c_char_p, P, C.POINTER(I32)]),
    "fdtd_plan_set_tile_order": (I32, [P, I32]),
    "fdtd_plan_get_tile_order": (I32, [P, C.POINTER(I32), C.POINTER(I32)]),
    "fdtd_batch_set_tile_order": (I32, [P, I32]),
    "fdtd_batch_set_group_bytes": (I32, [P, C.c_uint64]),
    "fdtd_batch_set_stream_stores": (I32, [P, I32]),
    "fdtd_plan_set_stream_stores": (I32, [P, I32]),
    "fdtd_plan_set_temporal": (I32, [P, I32]),
    "fdtd_plan_set_temporal_config": (I32, [P, I32, I32]),
    "fdtd_plan_get_temporal": (I32, [P, C.POINTER(I32), C.POINTER(I32), C.POINTER(I32),
                                     C.POINTER(I32), C.POINTER(I32)]),
    "fdtd_plan_get_stream_stores": (I32, [P, C.POINTER(I32), C.POINTER(I32)]),
    "fdtd_batch_get_groups": (I32, [P, C.POINTER(I32)]),
    "fdtd_batch_get_tile_order": (I32, [P, C.POINTER(I32), C.POINTER(I32)]),
    "fdtd_plan_set_timing": (I32, [P, I32]),
    "fdtd_plan_get_kernel_time": (I32, [P, PD, C.POINTER(I64)]),
    "fdtd_batch_set_timing": (I32, [P, I32]),
    "fdtd_batch_get_kernel_time": (I32, [P, PD, C.POINTER(I64)]),
    "fdtd_sparams": (I32, [I32, I32, PD, PD, PD, PD, C.c_double, PD, PD, PD, PD, PD]),
    "fdtd_status_string": (C.c_char_p, [I32]),
    "fdtd_device_copy": (I32, [P, P, C.c_size_t, P]),
    "fdtd_plan_set_source_samples": (I32, [P, C.POINTER(C.c_double), C.c_int64]),
}

_lib = None


def lib():
    """Load libfdtd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -m paper_2208_04371_amd.build)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(code: int, where: str, handle=None, batch=False):
    if code != FDTD_OK:
        msg = ""
        if handle or batch:
            # a batch call without a handle is fdtd_batch_create: its message
            # is kept per thread and read with a NULL handle
            fn = lib().fdtd_batch_last_error if batch else lib().fdtd_last_error
            msg = (fn(handle) or b"").decode()
        raise FdtdError(code, where, msg)
