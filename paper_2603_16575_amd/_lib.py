"""ctypes binding of libmbe3osv (include/mbe3osv.h).

Argument marshalling only: every step of the hot path runs in the HIP
library.  Device arrays are passed as raw pointers taken from torch tensors
(torch supplies device memory and streams); host lists as numpy arrays.
Importing this module fails loudly when the shared library is missing.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libmbe3osv.so")

MBE3_OK = 0
MBE3_EINVAL = -1
MBE3_ENOMEM = -2
MBE3_EHIP = -3
MBE3_ENOCONV = -4
MBE3_ENONFINITE = -5
MBE3_FP64 = 0
MBE3_MIXED_BF16 = 1
MBE3_MIXED_BF16_PROJ = 2
MBE3_GRAD_SLAB = 0
MBE3_GRAD_GAMMA = 1
MBE3_GRAD_PROBE = 2

EXPORTS = [
    "mbe3_create", "mbe3_destroy", "mbe3_last_error", "mbe3_get_layout",
    "mbe3_gamma_offsets", "mbe3_k_offsets", "mbe3_basis_offsets",
    "osv_project", "pair_K", "fragment_solve", "mbe3_energy",
    "mbe3_pair_basis", "mbe3_plan_check", "mbe3_set_timing",
    "mbe3_get_timing", "mbe3_backward", "mbe3_graph_begin", "mbe3_graph_end",
    "mbe3_graph_launch", "mbe3_autotune", "mbe3_set_gemm_shape",
    "mbe3_tune_report", "mbe3_screen", "mbe3_weak_pairs", "mbe3_fit_metric",
    "mbe3_fit_mask", "mbe3_project_fit", "mbe3_pair_K_fit", "mbe3_first_order_dE",
    "mbe3_screen_lists", "mbe3_screen_noalloc", "mbe3_rosv", "mbe3_pm_localize",
    "mbe3_set_slab_shift",
]
GEMM_SHAPES = ["64x64", "128x128", "32x32", "32x128", "64x128", "96x96"]
PHASES = ["regen", "project", "pair_K", "bases", "pairs", "cross", "solve",
          "energy", "grad", "backward"]


class Mbe3Problem(ctypes.Structure):
    _fields_ = [
        ("n_occ", ctypes.c_int32), ("n_vir", ctypes.c_int32),
        ("n_aux", ctypes.c_int32),
        ("r", ctypes.c_void_p), ("Q", ctypes.c_void_p),
        ("eps_vir", ctypes.c_void_p), ("f_occ", ctypes.c_void_p),
        ("seed", ctypes.c_uint64),
        ("w_ia", ctypes.c_void_p), ("w_iP", ctypes.c_void_p),
        ("slab", ctypes.c_void_p),
        ("n_pair", ctypes.c_int64), ("pairs", ctypes.c_void_p),
        ("n_frag", ctypes.c_int64), ("frags", ctypes.c_void_p),
        ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
        ("tau_S", ctypes.c_double), ("precision", ctypes.c_int32),
        ("warm_start", ctypes.c_int32),
    ]


class Mbe3Layout(ctypes.Structure):
    _fields_ = [("n_slot", ctypes.c_int64), ("gamma_rows", ctypes.c_int64),
                ("gamma_elems", ctypes.c_int64), ("k_elems", ctypes.c_int64),
                ("n_frag", ctypes.c_int64)]


class Mbe3Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mbe3 status {code}: {msg}")
        self.code = code


_lib = None


def load():
    """Load the shared library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libmbe3osv is not built ({LIB_PATH}); run "
                          "`python -m paper_2603_16575_amd.build` first")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "mbe3_create": [ctypes.POINTER(vp), ctypes.POINTER(Mbe3Problem), vp],
        "mbe3_destroy": [vp],
        "mbe3_get_layout": [vp, ctypes.POINTER(Mbe3Layout)],
        "mbe3_gamma_offsets": [vp, vp],
        "mbe3_k_offsets": [vp, vp],
        "mbe3_basis_offsets": [vp, vp, vp],
        "osv_project": [vp, vp, i64],
        "pair_K": [vp, vp, vp, i64],
        "fragment_solve": [vp, vp, vp, vp, vp],
        "mbe3_energy": [vp, vp, vp, vp],
        "mbe3_pair_basis": [vp, vp, vp, vp],
        "mbe3_plan_check": [ctypes.POINTER(Mbe3Problem), ctypes.POINTER(Mbe3Layout)],
        "mbe3_set_timing": [vp, ctypes.c_int],
        "mbe3_get_timing": [vp, vp, vp],
        "mbe3_backward": [vp, ctypes.c_double, vp, vp, ctypes.c_int, vp, i64,
                          vp, vp],
        "mbe3_graph_begin": [vp, ctypes.c_int],
        "mbe3_graph_end": [vp],
        "mbe3_graph_launch": [vp, vp],
        "mbe3_autotune": [vp, vp, i64, vp, i64, vp, i64, ctypes.c_int],
        "mbe3_set_gemm_shape": [vp, ctypes.c_int, ctypes.c_int],
        "mbe3_screen": [vp, vp, i64, vp],
        "mbe3_weak_pairs": [vp, vp, i64, vp, vp, vp],
        "mbe3_fit_metric": [vp, vp],
        "mbe3_fit_mask": [vp, vp, ctypes.c_double, vp, i64],
        "mbe3_project_fit": [vp, vp, ctypes.c_double, vp, i64],
        "mbe3_pair_K_fit": [vp, vp, ctypes.c_double, vp, i64],
        "mbe3_first_order_dE": [vp, vp, vp, vp, vp, vp],
        "mbe3_screen_noalloc": [vp, vp, i64, vp],
        "mbe3_set_slab_shift": [vp, ctypes.c_double],
        "mbe3_pm_localize": [vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                             ctypes.c_double, ctypes.c_int32, vp, vp, vp, vp, vp, vp],
        "mbe3_rosv": [vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_int, vp, vp, vp, vp],
        "mbe3_screen_lists": [ctypes.c_int32, vp, i64, vp, ctypes.c_double, ctypes.c_double,
                              ctypes.c_double, vp, vp, vp, vp, vp, vp, i64, vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.mbe3_last_error.argtypes = [vp]
    lib.mbe3_last_error.restype = ctypes.c_char_p
    lib.mbe3_tune_report.argtypes = [vp]
    lib.mbe3_tune_report.restype = ctypes.c_char_p
    lib.mbe3_screen_noalloc_max_bytes.argtypes = []
    lib.mbe3_screen_noalloc_max_bytes.restype = ctypes.c_int64
    _lib = lib
    return lib


def check(code, handle=None):
    if code != MBE3_OK:
        msg = load().mbe3_last_error(handle).decode()
        raise Mbe3Error(code, msg)
    return code


def ptr(t):
    """Raw pointer of a torch tensor / numpy array (None -> NULL)."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()
