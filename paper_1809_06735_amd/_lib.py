"""ctypes binding of libpaper_lbm.so (the C ABI declared in include/lbm.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpaper_lbm.so")

LBM_OK = 0
LBM_E_INVALID = -1
LBM_E_NOMEM = -2
LBM_E_HIP = -3
LBM_E_DIVERGED = -4
LBM_E_STATE = -5
LBM_E_UNSUPPORTED = -6
LBM_E_TIMEOUT = -7
LBM_F32 = 0
LBM_F64 = 1
LBM_LAYOUT_PLANES = 0
LBM_LAYOUT_ROWS = 1
LAYOUTS = {"planes": LBM_LAYOUT_PLANES, "rows": LBM_LAYOUT_ROWS}
LBM_FORCE_GUO = 0
LBM_FORCE_EDM = 1
SCHEMES = {"guo": LBM_FORCE_GUO, "edm": LBM_FORCE_EDM}
LBM_COLLISION_BGK = 0
LBM_COLLISION_ENTROPIC = 1
COLLISIONS = {"bgk": LBM_COLLISION_BGK, "entropic": LBM_COLLISION_ENTROPIC}
LBM_BATCH_PERSISTENT = 0
LBM_BATCH_PER_STEP = 1
LBM_BATCH_MULTI_STEP = 2
LBM_BATCH_PERSISTENT_MULTI = 3
NTERMS = 13
NWVALS = 16   # per explicit window: 13 box means, delta^E, delta^Omega, Ma
TERM_NAMES = ("lhs_E", "e1", "e2", "e3", "e4", "e5",
              "lhs_Z", "z1", "z2", "z3", "z4", "z5", "usq")
SCALAR_NAMES = ("mass", "mom_x", "mom_y", "energy", "max_speed", "min_rho", "nonfinite", "time")
NTERMS3 = 14
TERM_NAMES3 = ("lhs_E", "e1", "e2", "e3", "e4", "e5",
               "lhs_Z", "z1", "z2", "z3", "z4", "z5", "z6", "usq")
SCALAR_NAMES3 = ("mass", "mom_x", "mom_y", "mom_z", "energy", "max_speed", "min_rho", "nonfinite",
                 "time")


class LBMError(RuntimeError):
    """A non-zero status returned by the library."""

    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class Config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("dtype", C.c_int32),
                ("has_force", C.c_int32), ("with_balance", C.c_int32), ("layout", C.c_int32),
                ("tau", C.c_double), ("drag_alpha", C.c_double),
                ("force_scheme", C.c_int32), ("collision", C.c_int32),
                ("damp_f0", C.c_double), ("damp_kmin", C.c_double), ("damp_kmax", C.c_double),
                ("stream", C.c_void_p)]


class BalanceStats(C.Structure):
    _fields_ = [("L", C.c_int32), ("reserved", C.c_int32),
                ("count_dE", C.c_int64), ("nan_dE", C.c_int64), ("count_dZ", C.c_int64),
                ("nan_dZ", C.c_int64), ("count_Ma", C.c_int64),
                ("mean_dE", C.c_double), ("std_dE", C.c_double), ("min_dE", C.c_double),
                ("max_dE", C.c_double),
                ("mean_dZ", C.c_double), ("std_dZ", C.c_double), ("min_dZ", C.c_double),
                ("max_dZ", C.c_double),
                ("mean_Ma", C.c_double), ("std_Ma", C.c_double), ("min_Ma", C.c_double),
                ("max_Ma", C.c_double)]


class Tile(C.Structure):
    _fields_ = [("bx", C.c_int32), ("by", C.c_int32), ("vx", C.c_int32), ("ry", C.c_int32),
                ("nt", C.c_int32), ("fuse", C.c_int32), ("pf", C.c_int32), ("halo", C.c_int32)]


class BalanceInput(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nu", C.c_double),
                ("rho", C.c_void_p * 3), ("ux", C.c_void_p * 3), ("uy", C.c_void_p * 3),
                ("fx", C.c_void_p), ("fy", C.c_void_p), ("stream", C.c_void_p),
                ("nu_field", C.c_void_p)]


LBM_MAX_EDGES = 1024
LBM_MAX_SHELLS = 4096


class BalanceExtra(C.Structure):
    _fields_ = [("edges", C.POINTER(C.c_double)), ("nedges", C.c_int32), ("accumulate", C.c_int32),
                ("hist", C.POINTER(C.c_int64)), ("sample_xy", C.c_void_p),
                ("sample_counts", C.POINTER(C.c_int32)), ("sample_out", C.POINTER(BalanceStats)),
                ("sample_hist", C.POINTER(C.c_int64))]


class AdjointConfig(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("dtype", C.c_int32), ("box", C.c_int32),
                ("ckpt_every", C.c_int32), ("reserved", C.c_int32), ("steps", C.c_int64),
                ("tau", C.c_double), ("stream", C.c_void_p)]


_P = C.c_void_p
_I = C.c_int
_I32 = C.c_int32
class Tile3(C.Structure):
    _fields_ = [("fuse", C.c_int32), ("bx", C.c_int32), ("by", C.c_int32), ("bz", C.c_int32)]


class Config3(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("dtype", C.c_int32),
                ("has_force", C.c_int32), ("with_balance", C.c_int32), ("tau", C.c_double),
                ("stream", C.c_void_p), ("lattice", C.c_int32), ("reserved", C.c_int32)]


LATTICES3 = {"d3q19": 0, "d3q27": 1}


_I64 = C.c_int64
_SZ = C.c_size_t
_DP = C.POINTER(C.c_double)
_PP = C.POINTER(C.c_void_p)

# name -> (restype, argtypes)
SIGNATURES = {
    "lbm_version": (C.c_char_p, []),
    "lbm_strerror": (C.c_char_p, [_I]),
    "lbm_last_error": (C.c_char_p, []),
    "lbm_workspace_bytes": (_I, [C.POINTER(Config), C.POINTER(_SZ)]),
    "lbm_init": (_I, [C.POINTER(Config), _P, _SZ, _P, _P, _P, _P, _P, C.POINTER(_P)]),
    "lbm_step": (_I, [_P, _I64]),
    "lbm_moments": (_I, [_P, _P, _P, _P, _I32, _DP]),
    "lbm_subvolume_balance": (_I, [_P, C.POINTER(_I32), _I32, C.POINTER(BalanceStats), _P,
                                   C.POINTER(_I32), _I32, _DP, _P]),
    "lbm_subvolume_balance_ex": (_I, [_P, C.POINTER(_I32), _I32, C.POINTER(BalanceStats), _P,
                                      C.POINTER(_I32), _I32, _DP, _P, C.POINTER(BalanceExtra)]),
    "lbm_balance_begin": (_I, [_P, C.POINTER(_I32), _I32]),
    "lbm_balance_end": (_I, [_P, C.POINTER(BalanceStats)]),
    "lbm_energy_spectrum": (_I, [_P, _DP, _I32]),
    "lbm_enstrophy": (_I, [_P, _DP]),
    "lbm_relaxation": (_I, [_P, _P, _P]),
    "lbm_spectrum_workspace_bytes": (_I, [_I32, _I32, C.POINTER(_SZ)]),
    "lbm_spectrum_fields": (_I, [_I32, _I32, _P, _P, _P, _SZ, _DP, _I32, _P]),
    "lbm_time": (_I, [_P, C.POINTER(_I64)]),
    "lbm_state_bytes": (_I, [_P, C.POINTER(_SZ)]),
    "lbm_save": (_I, [_P, _P]),
    "lbm_load": (_I, [_P, _P]),
    "lbm_set_tile": (_I, [_P, C.POINTER(Tile)]),
    "lbm_get_tile": (_I, [_P, C.POINTER(Tile)]),
    "lbm_autotune": (_I, [_P, _I32, C.POINTER(Tile)]),
    "lbm_set_tuned_tile": (_I, [C.POINTER(Config), C.POINTER(Tile)]),
    "lbm_set_graph": (_I, [_P, _I32]),
    "lbm_step_timing": (_I, [_P, _I32]),
    "lbm_step_time": (_I, [_P, _DP, C.POINTER(_I64), _I32]),
    "lbm_destroy": (_I, [_P]),
    "lbm_balance_workspace_bytes": (_I, [_I32, _I32, C.POINTER(_SZ)]),
    "lbm_balance_fields": (_I, [C.POINTER(BalanceInput), _P, _SZ, C.POINTER(_I32), _I32,
                                C.POINTER(BalanceStats), _P, C.POINTER(_I32), _I32, _DP, _P]),
    "lbm_balance_fields_noalloc": (_I, [C.POINTER(BalanceInput), C.POINTER(_I32), _I32,
                                        C.POINTER(BalanceStats), _P, C.POINTER(_I32), _I32, _DP, _P]),
    "lbm_balance_fields_ex": (_I, [C.POINTER(BalanceInput), _P, _SZ, C.POINTER(_I32), _I32,
                                   C.POINTER(BalanceStats), _P, C.POINTER(_I32), _I32, _DP, _P,
                                   C.POINTER(BalanceExtra)]),
    "lbm_batch_workspace_bytes": (_I, [C.POINTER(Config), _I32, C.POINTER(_SZ)]),
    "lbm_batch_init": (_I, [C.POINTER(Config), _I32, _P, _SZ, _PP, _PP, _PP, _PP, _PP,
                            C.POINTER(_P)]),
    "lbm_batch_set_mode": (_I, [_P, _I32, _I32]),
    "lbm_batch_set_tile": (_I, [_P, _I32, _I32, _I32]),
    "lbm_batch_autotune": (_I, [_P, _I32, C.POINTER(_I32), C.POINTER(_I32), C.POINTER(_I32)]),
    "lbm_batch_get_mode": (_I, [_P, C.POINTER(_I32), C.POINTER(_I32)]),
    "lbm_batch_set_multi": (_I, [_P, C.POINTER(Tile)]),
    "lbm_batch_get_multi": (_I, [_P, C.POINTER(Tile)]),
    "lbm_batch_step": (_I, [_P, _I64]),
    "lbm_batch_moments": (_I, [_P, _I32, _P, _P, _P, _I32, _DP]),
    "lbm_batch_time": (_I, [_P, C.POINTER(_I64)]),
    "lbm_batch_sites": (_I64, [_P]),
    "lbm_batch_destroy": (_I, [_P]),
    "lbm_adjoint_workspace_bytes": (_I, [C.POINTER(AdjointConfig), C.POINTER(_SZ)]),
    "lbm_adjoint_run": (_I, [C.POINTER(AdjointConfig), _P, _SZ, _P, _P, _DP, _P, _P, _DP]),
    "lbm_copy": (_I, [_P, _P, _SZ, _P]),
    "lbm3_workspace_bytes": (_I, [C.POINTER(Config3), C.POINTER(_SZ)]),
    "lbm3_init": (_I, [C.POINTER(Config3), _P, _SZ, _P, _P, _P, _P, _P, _P, _P, C.POINTER(_P)]),
    "lbm3_step": (_I, [_P, _I64]),
    "lbm3_moments": (_I, [_P, _P, _P, _P, _P, _DP]),
    "lbm3_time": (_I, [_P, C.POINTER(_I64)]),
    "lbm3_subvolume_balance": (_I, [_P, C.POINTER(_I32), _I32, C.POINTER(BalanceStats), _P]),
    "lbm3_destroy": (_I, [_P]),
    "lbm3_set_tile": (_I, [_P, C.POINTER(Tile3)]),
    "lbm3_get_tile": (_I, [_P, C.POINTER(Tile3)]),
    "lbm3_autotune": (_I, [_P, _I32, C.POINTER(Tile3)]),
}

_lock = threading.Lock()
_lib = None


def load():
    """Load the built library (once) and declare every signature."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"HIP library {LIB_PATH} is not built; run `python -m paper_1809_06735_amd.build` "
                "(the library has no CPU fallback)")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


def check(rc: int, what: str = ""):
    """Raise LBMError for a non-zero status."""
    if rc != LBM_OK:
        lib = load()
        msg = lib.lbm_last_error().decode(errors="replace")
        raise LBMError(rc, f"{what}: {lib.lbm_strerror(rc).decode()}: {msg}")
