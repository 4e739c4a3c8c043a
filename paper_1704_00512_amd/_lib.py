"""ctypes binding of the C interface declared in include/chess.h.

Argument marshalling only: every step of the computation runs in the HIP
library (libchess.so next to this file).  If the library is missing this
module raises ImportError; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libchess.so")

CHESS_OK = 0
CHESS_F64, CHESS_F32, CHESS_BF16, CHESS_BF16X3 = 0, 1, 2, 3
CHESS_ERFC, CHESS_FERMI_DIRAC = 0, 1
CHESS_BOUNDS_GERSHGORIN, CHESS_BOUNDS_LANCZOS, CHESS_BOUNDS_LEARNED, CHESS_BOUNDS_LEARNED_LANCZOS = 0, 1, 2, 3
CHESS_FN_ERFC, CHESS_FN_FERMI_DIRAC, CHESS_FN_POWER, CHESS_FN_PENALTY = 0, 1, 2, 3

ERRORS = {
    -1: "CHESS_E_ARG", -2: "CHESS_E_PATTERN", -3: "CHESS_E_NOT_SPD", -4: "CHESS_E_BOUNDS",
    -5: "CHESS_E_NOCONV", -6: "CHESS_E_OOM", -7: "CHESS_E_HIP", -8: "CHESS_E_UNSUPPORTED",
    -9: "CHESS_E_CAPACITY",
}


class chess_pattern(ctypes.Structure):
    _fields_ = [("b", ctypes.c_int32), ("nbrows", ctypes.c_int32), ("nnzb", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p)]


class chess_matrix(ctypes.Structure):
    _fields_ = [("pat", chess_pattern), ("val", ctypes.c_void_p), ("dtype", ctypes.c_int32)]


class chess_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("smearing", ctypes.c_int32),
                ("bounds_mode", ctypes.c_int32), ("n_pl", ctypes.c_int32),
                ("n_pl_s", ctypes.c_int32), ("store_history", ctypes.c_int32),
                ("max_reexpand", ctypes.c_int32), ("lanczos_steps", ctypes.c_int32),
                ("tol_fit", ctypes.c_double), ("tol_fit_s", ctypes.c_double),
                ("tol_ne", ctypes.c_double), ("bounds", ctypes.c_double * 2),
                ("s_bounds", ctypes.c_double * 2), ("mu", ctypes.c_double),
                ("mu_bracket", ctypes.c_double * 2), ("eig_width", ctypes.c_double),
                ("bound_margin", ctypes.c_double), ("adapt_kt", ctypes.c_int32),
                ("max_kt_halvings", ctypes.c_int32), ("kt_ratio", ctypes.c_double),
                ("tol_energy", ctypes.c_double), ("sinvhalf_in", ctypes.c_void_p),
                ("sinvhalf_out", ctypes.c_void_p)]


class chess_info(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double), ("lo", ctypes.c_double), ("hi", ctypes.c_double),
                ("s_lo", ctypes.c_double), ("s_hi", ctypes.c_double), ("tr_ks", ctypes.c_double),
                ("ne_chain", ctypes.c_double), ("penalty", ctypes.c_double),
                ("n_pl", ctypes.c_int32), ("n_pl_s", ctypes.c_int32), ("passes", ctypes.c_int32),
                ("bisect_iters", ctypes.c_int32), ("reexpansions", ctypes.c_int32),
                ("chain_steps", ctypes.c_int32),
                ("ms_total", ctypes.c_double), ("ms_setup", ctypes.c_double),
                ("ms_s_chain", ctypes.c_double), ("ms_transform", ctypes.c_double),
                ("ms_h_chain", ctypes.c_double), ("ms_mu", ctypes.c_double),
                ("ms_post", ctypes.c_double), ("ms_chain_kernel", ctypes.c_double),
                ("kernel_variant", ctypes.c_int32), ("fallback", ctypes.c_int32),
                ("pred_lo", ctypes.c_double), ("pred_hi", ctypes.c_double),
                ("pred_mu", ctypes.c_double), ("ms_learned", ctypes.c_double),
                ("energy", ctypes.c_double), ("energy_wide", ctypes.c_double),
                ("kt_used", ctypes.c_double), ("kt_halvings", ctypes.c_int32),
                ("homo", ctypes.c_double), ("lumo", ctypes.c_double),
                ("ms_chain_kernel_acc", ctypes.c_double), ("kernel_variant_moments", ctypes.c_int32),
                ("tile_rows", ctypes.c_int32), ("moment_products", ctypes.c_int32),
                ("s_penalty", ctypes.c_double), ("s_check_terms", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class chess_batch_item(ctypes.Structure):
    _fields_ = [("H", ctypes.POINTER(chess_matrix)), ("S", ctypes.POINTER(chess_matrix)),
                ("pattern", ctypes.POINTER(chess_pattern)), ("n_electrons", ctypes.c_double),
                ("kT", ctypes.c_double), ("mu_trial", ctypes.c_double * 3),
                ("K_out", ctypes.POINTER(chess_matrix) * 3),
                ("Sinvhalf_out", ctypes.POINTER(chess_matrix)),
                ("Sinv_out", ctypes.POINTER(chess_matrix)),
                ("ne_trial", ctypes.POINTER(ctypes.c_double)),
                ("info", ctypes.POINTER(chess_info))]


EXPORTS = ["chess_default_opts", "chess_create", "chess_destroy", "chess_last_error",
           "chess_fermi_operator", "chess_matrix_power", "chess_eigs_in_interval",
           "chess_chebyshev", "chess_masked_product", "chess_set_progress",
           "chess_features", "chess_mlp_forward", "chess_mlp_grad", "chess_mlp_adam",
           "chess_model_load", "chess_model_save", "chess_fermi_operator_batched",
           "chess_ssf_to_bcsr", "chess_bcsr_to_ssf", "chess_degree", "chess_mlp_grad_noalloc"]

N_FEATURES, MLP_HIDDEN, MLP_OUT = 64, 128, 3
MLP_PARAMS = MLP_HIDDEN * N_FEATURES + MLP_HIDDEN + MLP_OUT * MLP_HIDDEN + MLP_OUT
MLP_NORM = 2 * N_FEATURES + 2 * MLP_OUT
MODEL_FLOATS = MLP_NORM + 3 + MLP_PARAMS
NOALLOC_MAX_BATCH = 4096

PROGRESS_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_char_p, ctypes.c_int64,
                               ctypes.c_int64)

_lib = None


def load():
    """Loads libchess.so (ImportError if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it first (build())")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    L.chess_default_opts.argtypes = [P(chess_opts)]
    L.chess_default_opts.restype = None
    L.chess_create.argtypes = [P(vp), ctypes.c_int, vp]
    L.chess_destroy.argtypes = [vp]
    L.chess_last_error.argtypes = [vp]
    L.chess_last_error.restype = ctypes.c_char_p
    L.chess_fermi_operator.argtypes = [vp, P(chess_matrix), P(chess_matrix), P(chess_pattern),
                                       ctypes.c_double, ctypes.c_double, P(chess_matrix),
                                       P(chess_info), P(chess_opts)]
    L.chess_matrix_power.argtypes = [vp, P(chess_matrix), ctypes.c_double, P(chess_pattern),
                                     P(chess_matrix), P(chess_info), P(chess_opts)]
    L.chess_eigs_in_interval.argtypes = [vp, P(chess_matrix), P(chess_matrix), ctypes.c_double,
                                         ctypes.c_double, P(chess_pattern), P(ctypes.c_double),
                                         ctypes.c_int64, P(ctypes.c_int64), P(chess_info),
                                         P(chess_opts)]
    L.chess_chebyshev.argtypes = [vp, P(chess_matrix), ctypes.c_double, ctypes.c_double,
                                  P(chess_pattern), ctypes.c_int32, ctypes.c_int32,
                                  P(ctypes.c_double), P(chess_matrix), P(ctypes.c_double),
                                  P(chess_opts)]
    L.chess_masked_product.argtypes = [vp, P(chess_matrix), P(chess_matrix), P(chess_matrix)]
    L.chess_set_progress.argtypes = [vp, PROGRESS_FN, vp, ctypes.c_int32]
    fp = P(ctypes.c_float)
    L.chess_features.argtypes = [vp, P(chess_matrix), P(chess_matrix), P(chess_pattern),
                                 ctypes.c_double, ctypes.c_double, fp, P(ctypes.c_double),
                                 P(chess_opts)]
    L.chess_mlp_forward.argtypes = [vp, vp, vp, vp, ctypes.c_int32, vp, vp]
    L.chess_mlp_grad.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.c_int32, vp, vp,
                                 P(ctypes.c_double)]
    L.chess_mlp_grad_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.c_int32, vp,
                                         P(ctypes.c_double)]
    L.chess_mlp_adam.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int64, ctypes.c_float,
                                 ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_int32]
    L.chess_fermi_operator_batched.argtypes = [vp, ctypes.c_int32, P(chess_batch_item),
                                               P(chess_opts)]
    L.chess_model_load.argtypes = [vp, fp, ctypes.c_int64]
    L.chess_model_save.argtypes = [vp, fp, ctypes.c_int64]
    i64, i32 = ctypes.c_int64, ctypes.c_int32
    L.chess_ssf_to_bcsr.argtypes = [i32, i64, i64, vp, vp, vp, i64, vp, vp, vp, i64, P(i64)]
    L.chess_bcsr_to_ssf.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, i64, P(i64), P(i64)]
    L.chess_degree.argtypes = [i32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, P(i32)]
    for name in EXPORTS:
        if name not in ("chess_default_opts", "chess_last_error"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L
