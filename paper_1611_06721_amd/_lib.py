"""ctypes view of the C-ABI in include/ec.h (argument marshalling only).

The shared library is loaded after torch so that both use the same HIP
runtime.  A missing library raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libec.so")

EC_OK = 0
EC_ERR_ARG, EC_ERR_HIP, EC_ERR_NOT_CONVERGED, EC_ERR_BREAKDOWN = -1, -2, -3, -4
EC_ERR_CFL, EC_ERR_NONFINITE, EC_ERR_STATE, EC_ERR_SINGULAR_PROJ = -5, -6, -7, -8
WF_DC, WF_SIN, WF_RAMP, WF_EXP = 0, 1, 2, 3
SEQ_SRC, SEQ_CPL, SEQ_ADJ, SEQ_USER = 0, 1, 2, 3
SV_ZERO, SV_PREV, SV_SPE, SV_POD = 0, 1, 2, 3
PREC_FP64, PREC_FP32_REFINED = 0, 1
OP_KN, OP_KCN_T, OP_KC_KCN = 0, 1, 2
MASS_LUMPED, MASS_CONSISTENT = 0, 1
MAX_WINDOW = 20
STATIC_MAX_NPAD = 1195904

STATUS_NAMES = {0: "OK", -1: "ARG", -2: "HIP", -3: "NOT_CONVERGED", -4: "BREAKDOWN",
                -5: "CFL", -6: "NONFINITE", -7: "STATE", -8: "SINGULAR_PROJ"}


class Grid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("len", C.c_double * 3)]


class Material(C.Structure):
    _fields_ = [("sigma", C.c_double), ("k1", C.c_double), ("k2", C.c_double),
                ("k3", C.c_double)]


class Materials(C.Structure):
    _fields_ = [("cell_mat", C.POINTER(C.c_uint8)), ("mats", C.POINTER(Material)),
                ("n_mats", C.c_int32), ("nu0", C.c_double)]


class Source(C.Structure):
    _fields_ = [("edge_current", C.POINTER(C.c_double)), ("waveform", C.c_int32),
                ("amp", C.c_double), ("freq", C.c_double), ("tau", C.c_double),
                ("ramp_steps", C.c_int64)]


class SolveOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("maxit", C.c_int32), ("precision", C.c_int32),
                ("inner_rtol", C.c_double), ("inner_maxit", C.c_int32),
                ("outer_max", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("outer_iters", C.c_int32), ("status", C.c_int32),
                ("basis_cols", C.c_int32), ("rel_res", C.c_double), ("b_norm", C.c_double),
                ("pod_info", C.c_double), ("r0_rel", C.c_double)]


class ImplicitOpts(C.Structure):
    _fields_ = [("newton_rtol", C.c_double), ("max_newton", C.c_int32), ("gmres_m", C.c_int32),
                ("gmres_max", C.c_int32), ("gmres_rtol", C.c_double), ("inner_rtol", C.c_double),
                ("start_method", C.c_int32), ("window", C.c_int32)]


class ImplicitInfo(C.Structure):
    _fields_ = [("newton_iters", C.c_int32), ("gmres_iters", C.c_int32), ("kn_solves", C.c_int32),
                ("status", C.c_int32), ("res0", C.c_double), ("res", C.c_double)]


class StepOpts(C.Structure):
    _fields_ = [("start_method", C.c_int32), ("window", C.c_int32), ("pod_kmax", C.c_int32),
                ("pod_eps", C.c_double), ("solve", SolveOpts), ("graph_iters", C.c_int32 * 2),
                ("graph_serial", C.c_int32)]


# every symbol the header declares, with its signature
_H = C.c_void_p
_P = C.c_void_p
SIGNATURES = {
    "ec_create": (C.c_int32, [C.POINTER(Grid), C.POINTER(Materials), C.POINTER(Source),
                              C.POINTER(_H)]),
    "ec_destroy": (C.c_int32, [_H]),
    "ec_sizes": (C.c_int32, [_H, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                             C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "ec_bind": (C.c_int32, [_H, _P, _P, C.c_int64, C.c_int32]),
    "ec_apply": (C.c_int32, [_H, C.c_int32, _P, _P]),
    "ec_set_gauge_penalty": (C.c_int32, [_H, C.c_double]),
    "ec_set_dependency_tol": (C.c_int32, [_H, C.c_double]),
    "ec_set_pcg_kernel": (C.c_int32, [_H, C.c_int32]),
    "ec_tune_pcg": (C.c_int32, [_H, C.c_char_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                C.POINTER(C.c_double)]),
    "ec_history_reset": (C.c_int32, [_H, C.c_int32]),
    "ec_history_push": (C.c_int32, [_H, C.c_int32, C.c_int32, C.c_int32, _P]),
    "ec_start_vector": (C.c_int32, [_H, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_double,
                                    _P, _P, _P]),
    "ec_solve": (C.c_int32, [_H, C.c_int32, C.c_int32, C.c_int32, _P, _P,
                             C.POINTER(SolveOpts), _P]),
    "ec_set_state": (C.c_int32, [_H, _P, C.POINTER(SolveOpts)]),
    "ec_step": (C.c_int32, [_H, C.c_int64, C.c_double, _P, C.POINTER(StepOpts), _P]),
    "ec_run": (C.c_int32, [_H, C.c_int64, C.c_int64, C.c_double, _P, C.POINTER(StepOpts), _P]),
    "ec_counters": (C.c_int32, [_H, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                C.POINTER(C.c_int32)]),
    "ec_counters_reset": (C.c_int32, [_H]),
    "ec_set_step": (C.c_int32, [_H, C.c_int64]),
    "ec_cfl": (C.c_int32, [_H, _P, C.c_int32, C.c_double, C.POINTER(C.c_double)]),
    "ec_set_material": (C.c_int32, [_H, C.c_int32, C.POINTER(Material)]),
    "ec_cfl_estimate": (C.c_int32, [_H, _P, C.c_int32, C.c_double, C.c_int32, C.c_int32,
                                    C.c_int32, _P, _P]),
    "ec_set_adaptive_dt": (C.c_int32, [_H, _P, C.c_double]),
    "ec_set_mass": (C.c_int32, [_H, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_int32]),
    "ec_implicit_step": (C.c_int32, [_H, C.c_int64, C.c_double, _P, C.POINTER(ImplicitOpts),
                                     C.POINTER(ImplicitInfo)]),
    "ec_mass_apply": (C.c_int32, [_H, _P, _P]),
    "ec_mass_solve": (C.c_int32, [_H, _P, _P, _P]),
    "ec_mass_counters": (C.c_int32, [_H, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "ec_clock": (C.c_int32, [_H, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                             C.POINTER(C.c_double)]),
    "ec_adjoint_sizes": (C.c_int32, [_H, C.c_int64, C.c_int32, C.POINTER(C.c_int64)]),
    "ec_adjoint_forward": (C.c_int32, [_H, C.c_int64, C.c_double, C.c_int32, C.POINTER(StepOpts),
                                       _P, C.c_int64, _P, _P]),
    "ec_adjoint_backward": (C.c_int32, [_H, C.c_int64, C.c_double, C.c_int32,
                                        C.POINTER(StepOpts), _P, C.c_int64, C.c_int32, _P]),
    "ec_batch_sizes": (C.c_int32, [C.c_int32, C.POINTER(_H), C.POINTER(C.c_int64)]),
    "ec_batch_create": (C.c_int32, [C.c_int32, C.POINTER(_H), _P, C.c_int64, C.POINTER(_P)]),
    "ec_batch_destroy": (C.c_int32, [_P]),
    "ec_batch_step": (C.c_int32, [_P, C.c_int64, C.POINTER(C.c_double), C.POINTER(_P),
                                  C.POINTER(StepOpts)]),
    "ec_batch_run": (C.c_int32, [_P, C.c_int64, C.c_int64, C.POINTER(C.c_double),
                                 C.POINTER(_P), C.POINTER(StepOpts)]),
    "ec_batch_graph_capture": (C.c_int32, [_P, C.POINTER(C.c_double), C.POINTER(_P),
                                           C.POINTER(StepOpts), C.POINTER(C.c_void_p)]),
    "ec_batch_set_tiles": (C.c_int32, [_P, C.c_int32]),
    "ec_batch_autotune": (C.c_int32, [_P, C.c_char_p, C.POINTER(C.c_int32),
                                      C.POINTER(C.c_double)]),
    "ec_graph_capture_step": (C.c_int32, [_H, C.c_double, _P, C.POINTER(StepOpts), _P,
                                          C.POINTER(C.c_void_p)]),
    "ec_graph_launch": (C.c_int32, [_P, _P]),
    "ec_graph_destroy": (C.c_int32, [_P]),
    "ec_solve_static": (C.c_int32, [_H, C.c_int32, _P, _P, C.POINTER(SolveOpts), _P]),
    "ec_last_error": (C.c_char_p, [_H]),
}

_lib = None


def load():
    """Load libec.so (after torch, so that one HIP runtime serves both)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads the HIP runtime first)
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() "
                           "(hipcc --offload-arch=gfx950); there is no fallback path")
    L = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


class ECError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code, handle=None):
    if code != EC_OK:
        msg = load().ec_last_error(handle)
        raise ECError(code, msg.decode() if msg else "")
    return code
