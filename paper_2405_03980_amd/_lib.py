"""ctypes declarations of the C ABI in include/sph4he.h (argument marshalling only).

The shared library is built in-tree (paper_2405_03980_amd/libsph4he.so).  There is no
fallback: if it is missing, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsph4he.so")

ABI_VERSION = 3

OK, E_INVALID, E_WORKSPACE, E_HIP, E_STATE, E_DOMAIN, E_NONFINITE, E_UNSUPPORTED, E_CAPACITY = range(9)
STATUS_NAMES = {0: "OK", 1: "E_INVALID", 2: "E_WORKSPACE", 3: "E_HIP", 4: "E_STATE",
                5: "E_DOMAIN", 6: "E_NONFINITE", 7: "E_UNSUPPORTED", 8: "E_CAPACITY"}

KERNEL_CUBIC, KERNEL_WENDLAND_C2 = 0, 1
FP64, FP32_MIXED = 0, 1
GEOM_PERIODIC_BOX, GEOM_CYLINDER_Z, GEOM_OPEN = 0, 1, 2


class SphParams(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32), ("kernel", C.c_int32), ("precision", C.c_int32),
        ("geometry", C.c_int32),
        ("dx", C.c_double), ("h", C.c_double),
        ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("rho0", C.c_double), ("c0", C.c_double), ("gamma", C.c_double),
        ("mass", C.c_double * 2),
        ("eta", C.c_double), ("sigma_T", C.c_double), ("C_l", C.c_double),
        ("kappa_I", C.c_double),
        ("cell_factor", C.c_int32), ("pressure_filter", C.c_int32),
        ("coll_alpha", C.c_double), ("coll_e", C.c_double),
    ]


class SphTuning(C.Structure):
    _fields_ = [("block_density", C.c_int32), ("block_force", C.c_int32),
                ("block_stream", C.c_int32), ("use_graph", C.c_int32), ("sweep", C.c_int32),
                ("xcd_run", C.c_int32), ("list_targets", C.c_int32)]


# name -> (restype, argtypes)
_vp = C.c_void_p
_PROTOS = {
    "sph_params_init": (C.c_int, [C.POINTER(SphParams)]),
    "sph_grid_dims": (C.c_int, [C.POINTER(SphParams), C.POINTER(C.c_int32)]),
    "sph_workspace_bytes": (C.c_int, [C.POINTER(SphParams), C.c_int64, C.POINTER(C.c_size_t)]),
    "sph_create": (C.c_int, [C.POINTER(SphParams), C.c_int64, _vp, C.c_size_t, _vp, C.POINTER(_vp)]),
    "sph_init_particles": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "sph_step": (C.c_int, [_vp, C.c_double, C.c_double, C.c_int32]),
    "sph_read_fields": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "sph_diagnostics": (C.c_int, [_vp, C.POINTER(C.c_double)]),
    "sph_debug_cells": (C.c_int, [_vp, _vp, _vp, _vp]),
    "sph_debug_neighbors": (C.c_int, [_vp, _vp, _vp, C.c_int64, C.POINTER(C.c_int64)]),
    "sph_debug_masks": (C.c_int, [_vp, _vp, _vp, C.c_int64, C.POINTER(C.c_int64)]),
    "sph_debug_near": (C.c_int, [_vp, _vp, _vp]),
    "sph_vortex_dims": (C.c_int, [C.POINTER(SphParams), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "sph_vortex_image": (C.c_int, [_vp, C.c_double, C.c_double, C.c_int32, _vp, _vp, _vp,
                                   C.POINTER(C.c_int32)]),
    "sph_vortex_image_noalloc": (C.c_int, [_vp, C.c_double, C.c_double, C.c_int32, _vp, _vp,
                                           C.POINTER(C.c_int32)]),
    "sph_set_tuning": (C.c_int, [_vp, C.POINTER(SphTuning)]),
    "sph_get_tuning": (C.c_int, [_vp, C.POINTER(SphTuning)]),
    "sph_sync": (C.c_int, [_vp]),
    "sph_status_str": (C.c_char_p, [C.c_int]),
    "sph_last_error": (C.c_char_p, [_vp]),
    "sph_destroy": (None, [_vp]),
    "sph_batch_workspace_bytes": (C.c_int, [C.c_int32, C.POINTER(SphParams), C.POINTER(C.c_int64), C.POINTER(C.c_size_t)]),
    "sph_batch_create": (C.c_int, [C.c_int32, C.POINTER(SphParams), C.POINTER(C.c_int64), _vp, C.c_size_t, _vp, C.POINTER(_vp)]),
    "sph_batch_init": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "sph_batch_step": (C.c_int, [_vp, C.c_double, C.POINTER(C.c_double), C.c_int32]),
    "sph_batch_read_fields": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "sph_batch_diagnostics": (C.c_int, [_vp, C.POINTER(C.c_double)]),
    "sph_batch_set_tuning": (C.c_int, [_vp, C.POINTER(SphTuning)]),
    "sph_batch_sync": (C.c_int, [_vp]),
    "sph_batch_last_error": (C.c_char_p, [_vp]),
    "sph_batch_destroy": (None, [_vp]),
    "sph_profile_begin": (C.c_int, [_vp]),
    "sph_profile_end": (C.c_int, [_vp, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "sph_batch_profile_begin": (C.c_int, [_vp]),
    "sph_batch_profile_end": (C.c_int, [_vp, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
}

KERNEL_GROUPS = ("keys", "scan", "scatter", "reorder", "density", "force", "collide", "filter")

_lib = None


def lib() -> C.CDLL:
    """Load libsph4he.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2405_03980_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class SphError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{where}: SPH_{name}" + (f" ({detail})" if detail else ""))


def make_params(d: dict, precision: int | None = None) -> SphParams:
    """sph_params from a workload parameter dict (as built by inputs.base_params)."""
    p = SphParams()
    lib().sph_params_init(C.byref(p))
    p.kernel = int(d["kernel"])
    p.precision = int(d.get("precision", FP32_MIXED) if precision is None else precision)
    p.geometry = int(d["geometry"])
    p.dx, p.h = float(d["dx"]), float(d["h"])
    for a in range(3):
        p.lo[a], p.hi[a] = float(d["lo"][a]), float(d["hi"][a])
    p.rho0, p.c0, p.gamma = float(d["rho0"]), float(d["c0"]), float(d["gamma"])
    p.mass[0], p.mass[1] = float(d["mass"][0]), float(d["mass"][1])
    p.eta, p.sigma_T, p.C_l = float(d["eta"]), float(d["sigma_T"]), float(d["C_l"])
    p.kappa_I = float(d["kappa_I"])
    p.cell_factor = int(d.get("cell_factor", 1))
    p.pressure_filter = int(d.get("pressure_filter", 0))
    p.coll_alpha, p.coll_e = float(d.get("coll_alpha", 0.0)), float(d.get("coll_e", 0.0))
    return p


def header_symbols(header_path: str) -> list[str]:
    """Function names declared in a C header (for export checks)."""
    import re
    txt = open(header_path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sph_[a-z_]+)\s*\(", txt)))
