"""MI355X (gfx950) implementation of the semi-explicit eddy-current scheme with
multiple right-hand-side start vectors (Dutine, Clemens, Schoeps).

The compute path is the HIP library ``libec.so`` behind the C-ABI of
``include/ec.h``; this package only marshals arguments (ctypes) and takes
device memory and streams from torch.
"""
from ._lib import (EC_ERR_ARG, EC_ERR_BREAKDOWN, EC_ERR_CFL, EC_ERR_HIP,  # noqa
                   EC_ERR_NONFINITE, EC_ERR_NOT_CONVERGED, EC_ERR_SINGULAR_PROJ, EC_ERR_STATE,
                   EC_OK, MASS_CONSISTENT, MASS_LUMPED, MAX_WINDOW, OP_KC_KCN, OP_KCN_T, OP_KN, PREC_FP32_REFINED, PREC_FP64,
                   SEQ_ADJ, SEQ_CPL, SEQ_SRC, SEQ_USER, STATIC_MAX_NPAD, SV_POD, SV_PREV,
                   SV_SPE, SV_ZERO,
                   ECError, LIB_PATH)


def __getattr__(name):
    # torch-dependent pieces load lazily
    if name in ("Problem", "Graph", "Batch", "solve_opts", "step_opts", "info_array",
                "INFO_BYTES"):
        from . import problem
        return getattr(problem, name)
    if name in ("EddyLoss", "eddy_loss"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
