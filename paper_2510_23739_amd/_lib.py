"""ctypes declarations of the C ABI in include/psoam.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpsoam.so")

OK, EINVAL, EUNSUPPORTED, EHIP, ENOMEM, EDIVERGED = range(6)
PREC = {"fp32": 0, "bf16": 1, "fp16": 2, "bf16_split": 3, "fp16_split": 4, "bf16_refined": 5}


class Geom(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("n_species", C.c_int32), ("n_pulses", C.c_int32), ("nt", C.c_int32),
                ("f", C.c_int32), ("phi_per_voxel", C.c_int32), ("separable", C.c_int32)]


class Species(C.Structure):
    _fields_ = [("a", C.c_double * 8), ("b", C.c_double * 8), ("tau", C.c_double * 8),
                ("gamma", C.c_double)]


class Shell(C.Structure):
    _fields_ = [("dr", C.c_double), ("z_focus", C.c_double), ("t_focus", C.c_int32),
                ("n_eir", C.c_int32), ("eir_origin", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("lambda_tv", C.c_double), ("lambda_l1", C.c_double),
                ("k1", C.c_int32), ("k2", C.c_int32),
                ("eps1", C.c_double), ("eps2", C.c_double), ("alpha1", C.c_double),
                ("n_power", C.c_int32), ("literal_momentum", C.c_int32), ("warm_inner", C.c_int32),
                ("v0", C.c_void_p), ("trace", C.POINTER(C.c_double)), ("lambda_tvs", C.c_double),
                ("device_stop", C.c_int32)]


class SolveStats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("status", C.c_int32), ("alpha1", C.c_double),
                ("lambda_max", C.c_double), ("objective", C.c_double)]


class PlanInfo(C.Structure):
    _fields_ = [("useful_macs", C.c_int64 * 2), ("chunks", C.c_int64 * 2),
                ("executed_macs", C.c_int64 * 2), ("operand_bytes", C.c_int64 * 2),
                ("lds_bytes", C.c_int64 * 2), ("lds_rows", C.c_int32 * 2)]


class TuneReport(C.Structure):
    _fields_ = [("h_rows", C.c_int32), ("ht_rows", C.c_int32), ("ht_shift", C.c_int32),
                ("candidates", C.c_int32), ("from_cache", C.c_int32),
                ("h_ms", C.c_double), ("ht_ms", C.c_double),
                ("h_ms_default", C.c_double), ("ht_ms_default", C.c_double),
                ("h_loaders", C.c_int32), ("tv_tile", C.c_int32 * 4),
                ("tv_ms", C.c_double), ("tv_ms_default", C.c_double),
                ("fp32_runs", C.c_int32 * 2)]


EXPORTS = {
    "psoam_plan_create": (C.c_int, [C.POINTER(Geom), C.POINTER(Species), C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                    C.POINTER(C.c_void_p)]),
    "psoam_plan_create_tuned": (C.c_int, [C.POINTER(Geom), C.POINTER(Species), C.c_void_p,
                                          C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                          C.c_void_p, C.POINTER(C.c_void_p),
                                          C.POINTER(TuneReport)]),
    "psoam_plan_destroy": (C.c_int, [C.c_void_p]),
    "psoam_plan_create_acoustic": (C.c_int, [C.POINTER(Geom), C.c_void_p, C.c_void_p, C.c_int32,
                                             C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]),
    "psoam_plan_create_factorised": (C.c_int, [C.POINTER(Geom), C.POINTER(Species), C.c_void_p,
                                               C.c_void_p, C.c_void_p, C.POINTER(Shell),
                                               C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]),
    "psoam_unmix": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(SolveOpts),
                              C.POINTER(SolveStats), C.c_void_p]),
    "psoam_plan_geom": (C.c_int, [C.c_void_p, C.POINTER(Geom)]),
    "psoam_apply_A": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "psoam_apply_AT": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "psoam_prox_l1": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_float, C.c_int32,
                                C.c_void_p]),
    "psoam_prox_tv_ws_bytes": (C.c_size_t, [C.c_void_p]),
    "psoam_prox_r3_ws_bytes": (C.c_size_t, [C.c_void_p]),
    "psoam_prox_r3": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_float, C.c_float,
                                C.c_float, C.c_int32, C.c_void_p, C.c_void_p]),
    "psoam_prox_tv": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_float, C.c_int32,
                                C.c_int32, C.c_void_p, C.c_void_p]),
    "psoam_prox_tv_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_float, C.c_int32,
                                        C.c_int32, C.c_void_p]),
    "psoam_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(SolveOpts),
                              C.POINTER(SolveStats), C.c_void_p]),
    "psoam_solve_batch": (C.c_int, [C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                    C.POINTER(C.c_void_p), C.POINTER(SolveOpts),
                                    C.POINTER(SolveStats), C.c_void_p]),
    "psoam_plan_stats": (C.c_int, [C.c_void_p, C.POINTER(PlanInfo)]),
    "psoam_band_only": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "psoam_last_error": (C.c_char_p, []),
}

_lib = None


def load() -> C.CDLL:
    """Load the in-tree libpsoam.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2510_23739_amd.build`")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class PsoamError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"psoam error {code}: {msg}")
        self.code = code


def check(rc: int) -> None:
    if rc != OK:
        raise PsoamError(rc, load().psoam_last_error().decode())
