"""ctypes declarations of libmtp.so (the C ABI of include/mtp.h).

Argument marshalling only.  The library is loaded from this package folder;
if it is missing the import of any entry point raises -- there is no other
implementation to fall back to.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmtp.so")

MTP_FP64, MTP_MIXED = 0, 1
MTP_GRADE_FULL, MTP_GRADE_LINEAR, MTP_GRADE_FULL_CFG, MTP_GRADE_LINEAR_CFG = 0, 1, 2, 3

STATUS = {0: "MTP_OK", -1: "MTP_E_INVAL", -2: "MTP_E_IO", -3: "MTP_E_PARSE", -4: "MTP_E_OVERLAP",
          -5: "MTP_E_CAPACITY", -6: "MTP_E_SINGULAR", -7: "MTP_E_HIP", -8: "MTP_E_NOMEM", -9: "MTP_E_UNSUPPORTED"}

# every symbol declared in include/mtp.h
EXPORTS = ("mtp_load", "mtp_save", "mtp_create", "mtp_free", "mtp_info", "mtp_set_params", "mtp_get_params", "mtp_kept_columns",
           "mtp_set_active_set", "mtp_get_active_set", "mtp_nbrs_create", "mtp_nbrs_free", "mtp_build_neighbors",
           "mtp_nbrs_status", "mtp_nbrs_export", "mtp_energy_forces_stress", "mtp_energy_forces_stress_noalloc", "mtp_grade", "mtp_grade_rows", "mtp_grade_cfg", "mtp_evaluate",
           "mtp_evaluate_select", "mtp_b_rows", "mtp_select", "mtp_maxvol_update", "mtp_cut_neighborhood", "mtp_md_run", "mtp_relax_fire", "mtp_fit_bfgs", "mtp_efs_backward", "mtp_basis_describe",
           "mtp_compiled_levels", "mtp_last_error", "mtp_profile_enable", "mtp_profile_read", "mtp_tune", "mtp_mfma_rate")


class MtpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


class ModelInfo(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("n_types", ctypes.c_int32), ("n_polyn", ctypes.c_int32),
                ("n_lin", ctypes.c_int32), ("n_rad", ctypes.c_int32), ("n_comp", ctypes.c_int32),
                ("n_theta", ctypes.c_int32), ("m_full", ctypes.c_int32), ("m_linear", ctypes.c_int32),
                ("r_min", ctypes.c_double), ("r_cut", ctypes.c_double),
                ("has_active_full", ctypes.c_int32), ("has_active_linear", ctypes.c_int32),
                ("contraction_flops", ctypes.c_int64)]


class System(ctypes.Structure):
    _fields_ = [("n_cfg", ctypes.c_int32), ("n_atoms", ctypes.c_int64), ("cfg_off", ctypes.c_void_p),
                ("pos", ctypes.c_void_p), ("type", ctypes.c_void_p), ("cell", ctypes.c_void_p),
                ("pbc", ctypes.c_void_p)]


_lib = None


def lib():
    """The loaded library (raises FileNotFoundError if it was never built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FileNotFoundError(f"{LIB_PATH} is missing: build it with `python -m paper_2304_13144_amd.build` "
                                "(or __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    PP = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "mtp_load": [ctypes.c_char_p, ctypes.c_int, PP],
        "mtp_save": [P, ctypes.c_char_p],
        "mtp_create": [I32, I32, D, D, ctypes.c_int, PP],
        "mtp_free": [P],
        "mtp_info": [P, ctypes.POINTER(ModelInfo)],
        "mtp_set_params": [P, P, P],
        "mtp_get_params": [P, ctypes.POINTER(D)],
        "mtp_kept_columns": [P, P],
        "mtp_set_active_set": [P, ctypes.c_int, P, P],
        "mtp_get_active_set": [P, ctypes.c_int, P, P, P],
        "mtp_nbrs_create": [PP],
        "mtp_nbrs_free": [P],
        "mtp_build_neighbors": [P, ctypes.POINTER(System), I32, P, P],
        "mtp_nbrs_status": [P, P],
        "mtp_nbrs_export": [P, P, P, P, ctypes.POINTER(I32), P],
        "mtp_energy_forces_stress": [P, ctypes.POINTER(System), P, ctypes.c_int, P, P, P, P, P],
        "mtp_energy_forces_stress_noalloc": [P, ctypes.POINTER(System), P, ctypes.c_int, P, P, P, P, P],
        "mtp_grade": [P, ctypes.POINTER(System), P, ctypes.c_int, ctypes.c_int, P, P, P, P],
        "mtp_evaluate": [P, ctypes.POINTER(System), P, ctypes.c_int, ctypes.c_int, P, P, P, P, P, P, P],
        "mtp_grade_cfg": [P, ctypes.POINTER(System), P, ctypes.c_int, ctypes.c_int, P, P, P, P],
        "mtp_grade_rows": [P, ctypes.c_int, ctypes.c_int, P, I64, I64, I32, P, P, P],
        "mtp_evaluate_select": [P, ctypes.POINTER(System), P, ctypes.c_int, ctypes.c_int, P, P, P, P, P, P, D, P, I32,
                                P, P],
        "mtp_b_rows": [P, ctypes.POINTER(System), P, ctypes.c_int, P, I32, P, P],
        "mtp_select": [P, I64, D, P, I32, P, P],
        "mtp_maxvol_update": [P, ctypes.c_int, P, I64, D, I32, P, P, ctypes.POINTER(I32), P],
        "mtp_cut_neighborhood": [ctypes.POINTER(System), P, D, I32, P, P, P, P, ctypes.POINTER(I32),
                                 ctypes.POINTER(I32), P],
        "mtp_fit_bfgs": [P, ctypes.POINTER(System), P, ctypes.c_int, P, P, P, D, D, D, I32, D, ctypes.POINTER(D),
                         ctypes.POINTER(D), ctypes.POINTER(I32), P],
        "mtp_relax_fire": [P, ctypes.POINTER(System), P, I32, P, ctypes.POINTER(D), D, D, D, I32, ctypes.c_int,
                           ctypes.c_int, D, D, ctypes.POINTER(D), ctypes.POINTER(I32), ctypes.POINTER(I32),
                           ctypes.POINTER(I32), ctypes.POINTER(I32), P],
        "mtp_md_run": [P, ctypes.POINTER(System), P, I32, P, P, ctypes.POINTER(D), D, I32, ctypes.c_int, ctypes.c_int,
                       D, D, ctypes.POINTER(D), ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I32), P],
        "mtp_efs_backward": [P, ctypes.POINTER(System), P, ctypes.c_int, P, P, P, P, P],
        "mtp_basis_describe": [I32, ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(I32)],
        "mtp_compiled_levels": [ctypes.POINTER(I32), I32],
        "mtp_profile_enable": [ctypes.c_int],
        "mtp_tune": [P, ctypes.POINTER(System), P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(I32),
                     ctypes.POINTER(I32), P],
        "mtp_profile_read": [ctypes.c_char_p, ctypes.POINTER(D), ctypes.POINTER(I64)],
        "mtp_mfma_rate": [ctypes.c_int, ctypes.c_int32, ctypes.POINTER(D), P],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.mtp_last_error.argtypes = []
    L.mtp_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def check(code):
    if code != 0:
        raise MtpError(code, lib().mtp_last_error().decode(errors="replace"))
    return code
