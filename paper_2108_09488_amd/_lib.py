"""ctypes binding of libadesph.so (the C ABI of include/adesph.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  If the library has not been built, loading fails
loudly; there is no fallback path.
"""
from __future__ import annotations

import ctypes as ct
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libadesph.so")

ADE_OK, ADE_EINVAL, ADE_EWORKSPACE, ADE_EHIP, ADE_EUNSTABLE, ADE_ENONFINITE, ADE_ESTATE = 0, -1, -2, -3, -4, -5, -6
ADE_WENDLAND_C2, ADE_WENDLAND_C4 = 2, 4
ADE_EULER, ADE_PC = 1, 2
ADE_STRICT_DT, ADE_CHECK_FINITE, ADE_VELOCITY_FIELD = 1, 2, 4
ADE_TUNE_KEEP_LANES = 1

ERROR_NAMES = {0: "ADE_OK", -1: "ADE_EINVAL", -2: "ADE_EWORKSPACE", -3: "ADE_EHIP",
               -4: "ADE_EUNSTABLE", -5: "ADE_ENONFINITE", -6: "ADE_ESTATE"}

# every entry point declared in include/adesph.h
EXPORTS = ["ade_workspace_bytes", "ade_create", "ade_init_particles", "ade_set_velocities", "ade_build_cells",
           "ade_coincident",
           "ade_step", "ade_step_graph", "ade_rhs", "ade_read_C", "ade_read_x", "ade_mass", "ade_conc_range",
           "ade_neighbours", "ade_sensor_interp", "ade_adjoint_workspace_bytes", "ade_adjoint",
           "ade_adjoint_noalloc", "ade_adjoint_noalloc_max_bytes",
           "ade_kernel_timing", "ade_autotune", "ade_set_tuning", "ade_get_tuning", "ade_info",
           "ade_state_bytes", "ade_save_state", "ade_load_state", "ade_destroy", "ade_last_error",
           "ade_version"]


class AdeParams(ct.Structure):
    _fields_ = [("dim", ct.c_int32), ("real_bytes", ct.c_int32), ("kernel", ct.c_int32),
                ("integrator", ct.c_int32), ("H", ct.c_double), ("L", ct.c_double),
                ("alpha_L", ct.c_double), ("alpha_T", ct.c_double), ("D_m", ct.c_double),
                ("v", ct.c_double * 3), ("dt", ct.c_double), ("rho0", ct.c_double),
                ("mass", ct.c_double), ("flags", ct.c_uint32), ("cell_rows", ct.c_int32),
                ("cell_xsub", ct.c_int32), ("reserved", ct.c_int32)]


class AdeTuning(ct.Structure):
    _fields_ = [("block", ct.c_int32), ("lanes", ct.c_int32), ("xcd_group", ct.c_int32),
                ("persistent", ct.c_int32), ("targets", ct.c_int32)]


class AdeError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib() -> ct.CDLL:
    """Load libadesph.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2108_09488_amd.build` "
                          "(the HIP library has no fallback)")
    L = ct.CDLL(LIB_PATH)
    p, i32, i64, sz = ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_size_t
    P = ct.POINTER(AdeParams)
    T = ct.POINTER(AdeTuning)
    pi64, pd, psz = ct.POINTER(ct.c_int64), ct.POINTER(ct.c_double), ct.POINTER(ct.c_size_t)
    sigs = {
        "ade_workspace_bytes": [P, p, i32, psz],
        "ade_create": [P, p, i32, p, sz, p, ct.POINTER(p)],
        "ade_init_particles": [p, p, p],
        "ade_set_velocities": [p, p],
        "ade_build_cells": [p],
        "ade_step": [p, i64],
        "ade_step_graph": [p, i64],
        "ade_rhs": [p, p],
        "ade_read_C": [p, p],
        "ade_read_x": [p, p],
        "ade_mass": [p, p],
        "ade_conc_range": [p, p],
        "ade_neighbours": [p, p, p, i64, pi64],
        "ade_sensor_interp": [p, p, i32, p],
        "ade_adjoint_workspace_bytes": [p, i64, i32, i32, psz],
        "ade_adjoint": [p, i64, i32, p, i32, p, p, sz, pd, pd],
        "ade_adjoint_noalloc": [p, i64, i32, p, i32, p, pd, pd],
        "ade_adjoint_noalloc_max_bytes": [psz],
        "ade_kernel_timing": [p, i32, pd, pi64],
        "ade_autotune": [p, i32, i32, T],
        "ade_set_tuning": [p, T],
        "ade_get_tuning": [p, T],
        "ade_info": [p, i32, pi64, pi64, pi64, pd, pi64],
        "ade_coincident": [p, ct.POINTER(ct.c_int32)],
        "ade_state_bytes": [p, psz],
        "ade_save_state": [p, p, sz],
        "ade_load_state": [p, p, sz],
        "ade_destroy": [p],
    }
    for name, args in sigs.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ct.c_int
    L.ade_last_error.restype = ct.c_char_p
    L.ade_last_error.argtypes = []
    L.ade_version.restype = ct.c_char_p
    L.ade_version.argtypes = []
    _lib = L
    return L


def check(rc: int) -> None:
    if rc != ADE_OK:
        raise AdeError(rc, lib().ade_last_error().decode())
