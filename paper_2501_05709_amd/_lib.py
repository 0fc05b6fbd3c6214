"""ctypes declarations of the C ABI in include/fr.h.

Loading fails loudly when libfr.so has not been built: there is no CPU
fallback for any entry point.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libfr.so")

FR_OK, FR_E_ARG, FR_E_MESH, FR_E_NOMEM, FR_E_DEVICE, FR_E_NONFINITE, FR_E_STATE, FR_E_UNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6, -7)
FR_FP64, FR_FP32 = 0, 1
FR_BC_WALL, FR_BC_FARFIELD = 1, 2

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)


class MeshDesc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("order", ctypes.c_int32), ("geom_order", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("n_nodes", ctypes.c_int64), ("nodes", _dp),
        ("n_elems", ctypes.c_int64), ("elem_nodes", _i64p),
        ("n_periodic", ctypes.c_int32), ("periodic_shift", _dp),
        ("n_bfaces", ctypes.c_int64), ("bfaces", _i64p),
        ("gamma", ctypes.c_double), ("prandtl", ctypes.c_double), ("mu", ctypes.c_double),
        ("freestream", ctypes.c_double * 5),
        ("ref_area", ctypes.c_double), ("lift_dir", ctypes.c_double * 3), ("drag_dir", ctypes.c_double * 3),
        ("dt", ctypes.c_double),
        ("device", ctypes.c_int32), ("stream", ctypes.c_void_p),
        ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_ctx", ctypes.c_void_p),
        ("elem_order", ctypes.POINTER(ctypes.c_int32)),
    ]


class FwhDesc(ctypes.Structure):
    _fields_ = [
        ("n_points", ctypes.c_int64), ("points", _dp), ("normals", _dp), ("areas", _dp),
        ("n_copies", ctypes.c_int32), ("copy_shift", ctypes.c_double * 3), ("mach", ctypes.c_double * 3),
        ("c0", ctypes.c_double), ("rho0", ctypes.c_double), ("p0", ctypes.c_double),
        ("dt", ctypes.c_double), ("tau0", ctypes.c_double), ("capacity", ctypes.c_int64),
        ("device", ctypes.c_int32), ("stream", ctypes.c_void_p),
        ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_ctx", ctypes.c_void_p),
    ]


class PoolSurface(ctypes.Structure):
    _fields_ = [
        ("n_points", ctypes.c_int64), ("points", _dp), ("normals", _dp), ("areas", _dp),
        ("n_copies", ctypes.c_int32), ("copy_shift", ctypes.c_double * 3),
        ("warmup", ctypes.c_int64), ("every", ctypes.c_int64), ("n_samples", ctypes.c_int64),
    ]


# every function declared in include/fr.h: name -> (restype, argtypes)
SIGNATURES = {
    "fr_mesh_create": (ctypes.c_int, [ctypes.POINTER(MeshDesc), ctypes.POINTER(ctypes.c_void_p)]),
    "fr_batch_create": (ctypes.c_int, [ctypes.POINTER(MeshDesc), ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]),
    "fr_mesh_destroy": (None, [ctypes.c_void_p]),
    "fr_mesh_info": (ctypes.c_int, [ctypes.c_void_p, _i64p]),
    "fr_design_range": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _i64p, _i64p]),
    "fr_solution_points": (ctypes.c_int, [ctypes.c_void_p, _dp]),
    "fr_neighbours": (ctypes.c_int, [ctypes.c_void_p, _i64p]),
    "fr_connectivity": (ctypes.c_int, [ctypes.POINTER(MeshDesc), _i64p, _dp]),
    "fr_set_state": (ctypes.c_int, [ctypes.c_void_p, _dp]),
    "fr_get_state": (ctypes.c_int, [ctypes.c_void_p, _dp]),
    "fr_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "fr_step_async": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "fr_sync": (ctypes.c_int, [ctypes.c_void_p]),
    "fr_forces": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _dp]),
    "fr_residual": (ctypes.c_int, [ctypes.c_void_p, _dp, _dp]),
    "fr_state_device": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), _i64p]),
    "fr_select_kernels": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "fr_selected_kernels": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "fr_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32)]),
    "fr_profile_kernels": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, _dp, _i64p]),
    "fr_pool_create": (ctypes.c_int, [ctypes.c_size_t, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]),
    "fr_pool_destroy": (None, [ctypes.c_void_p]),
    "fr_footprint": (ctypes.c_int, [ctypes.POINTER(MeshDesc), ctypes.POINTER(ctypes.c_size_t)]),
    "fr_pool_admit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(MeshDesc), _dp, ctypes.c_int64, _i64p]),
    "fr_pool_tick": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, _i64p, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_int32)]),
    "fr_pool_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "fr_pool_collect": (ctypes.c_int, [ctypes.c_void_p, _i64p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "fr_pool_result": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, _dp, _dp]),
    "fr_pool_usage": (ctypes.c_int, [ctypes.c_void_p, _i64p]),
    "fr_mesh_points": (ctypes.c_int, [ctypes.c_void_p, _i64p]),
    "fr_pool_admit_sampled": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(MeshDesc), _dp,
                                             ctypes.POINTER(PoolSurface), _i64p]),
    "fr_pool_pressure": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, _dp, ctypes.c_int64, _dp, _i64p, _dp]),
    "fr_probe_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(MeshDesc), ctypes.c_int32, ctypes.c_int64, _dp,
                                       ctypes.POINTER(ctypes.c_void_p)]),
    "fr_probe_destroy": (None, [ctypes.c_void_p]),
    "fr_probe_locate": (ctypes.c_int, [ctypes.c_void_p, _i64p, _dp]),
    "fr_probe_sample": (ctypes.c_int, [ctypes.c_void_p, _dp]),
    "fr_fwh_create": (ctypes.c_int, [ctypes.POINTER(FwhDesc), ctypes.POINTER(ctypes.c_void_p)]),
    "fr_fwh_destroy": (None, [ctypes.c_void_p]),
    "fr_fwh_append": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, _dp]),
    "fr_fwh_append_probe": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "fr_fwh_samples": (ctypes.c_int, [ctypes.c_void_p, _i64p]),
    "fr_fwh_window": (ctypes.c_int, [ctypes.c_void_p, _dp, _dp, _i64p]),
    "fr_fwh_pressure": (ctypes.c_int, [ctypes.c_void_p, _dp, ctypes.c_int64, _dp, _i64p, _dp, _dp, _dp]),
    "fr_fwh_pressure_at": (ctypes.c_int, [ctypes.c_void_p, _dp, ctypes.c_double, ctypes.c_int64, _dp, _dp, _dp]),
    "fr_fwh_pressure_at_noalloc": (ctypes.c_int, [ctypes.c_void_p, _dp, ctypes.c_double, ctypes.c_int64, _dp, _dp,
                                                  _dp]),
    "fr_fwh_time_ms": (ctypes.c_int, [ctypes.c_void_p, _dp]),
    "fr_last_error": (ctypes.c_char_p, []),
}

_lib = None


class FRError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (fr_status {code})")
        self.code = code


def load():
    """Load libfr.so; raises if it has not been built.

    torch is imported first when it is installed: its bundled HIP runtime
    carries the same soname as the system one, so libfr.so then binds to the
    runtime torch already holds and the process has a single HIP runtime.
    """
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2501_05709_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(code, what=""):
    if code != FR_OK:
        msg = load().fr_last_error().decode(errors="replace")
        raise FRError(code, f"{what}: {msg}" if what else msg)
