"""ctypes declarations of the C ABI in include/isis_mg.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libisis_mg.so")

ISIS_OK = 0
ISIS_ERR_INVALID_ARG = -1
ISIS_ERR_NOT_CONVERGED = -2
ISIS_ERR_DIVERGED = -3
ISIS_ERR_HIP = -4
ISIS_ERR_UNSUPPORTED = -5

ISIS_SYMMETRON, ISIS_FR_HS, ISIS_LINEAR, ISIS_CHAMELEON = 0, 1, 2, 3
ISIS_FP64, ISIS_MIXED = 0, 1
MAX_HIST = 128


class ModelParamsC(C.Structure):
    _fields_ = [("model", C.c_int), ("lambda0", C.c_double), ("a_ssb", C.c_double),
                ("beta", C.c_double), ("n", C.c_double), ("fR0_abs", C.c_double),
                ("omega_m", C.c_double), ("omega_l", C.c_double), ("kappa", C.c_double),
                ("m2", C.c_double), ("cham_alpha", C.c_double), ("cham_mu", C.c_double),
                ("cham_n", C.c_double), ("paper_u", C.c_int)]


class DescC(C.Structure):
    _fields_ = [("N", C.c_int), ("box", C.c_double), ("nu_pre", C.c_int), ("nu_post", C.c_int),
                ("nu_coarse", C.c_int), ("max_cycles", C.c_int), ("precision", C.c_int),
                ("fp32_floor", C.c_double), ("temporal_block", C.c_int), ("stream", C.c_void_p),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
                ("guess_accept", C.c_double), ("restriction", C.c_int),
                ("judge_skip", C.c_int), ("prolongation", C.c_int)]


class StatsC(C.Structure):
    _fields_ = [("cycles", C.c_int), ("cycles_fp32", C.c_int), ("r_ref", C.c_double),
                ("r0", C.c_double), ("rel_res", C.c_double),
                ("rel_hist", C.c_double * MAX_HIST), ("ms_total", C.c_double),
                ("cell_updates", C.c_double), ("used_guess", C.c_int),
                ("fine_sweep_ms", C.c_double * 2), ("fine_sweep_launches", C.c_int * 2),
                ("fine_sweep_updates", C.c_double * 2), ("fine_sweep_bytes", C.c_double * 2),
                ("temporal_block", C.c_int), ("rho_hist", C.c_double * MAX_HIST),
                ("safeguard_hits", C.c_longlong), ("ms_smooth", C.c_double),
                ("restriction", C.c_int), ("judged_cycles", C.c_int),
                ("fine_prol_ms", C.c_double * 2), ("fine_prol_launches", C.c_int * 2),
                ("fine_prol_bytes", C.c_double * 2), ("nu_pre", C.c_int), ("nu_post", C.c_int),
                ("prolongation", C.c_int), ("judged_fp32", C.c_int)]


_lib = None

# (name, restype, argtypes) for every function of the header.
_P = C.c_void_p
_D = C.c_double
_I = C.c_int
SIGNATURES = [
    ("isis_mg_workspace_size", C.c_size_t, [C.POINTER(DescC)]),
    ("isis_mg_create", _I, [C.POINTER(DescC), C.POINTER(_P)]),
    ("isis_mg_solve", _I, [_P, _P, _P, C.POINTER(ModelParamsC), _D, _D, _I, C.POINTER(StatsC)]),
    ("isis_mg_residual", _I, [_P, _P, _P, C.POINTER(ModelParamsC), _D, _P, C.POINTER(_D)]),
    ("isis_mg_residual_noalloc", _I, [C.POINTER(ModelParamsC), _D, _I, _D, _P, _P, _P,
                                      C.POINTER(_D), _P]),
    ("isis_mg_destroy", None, [_P]),
    ("isis_mg_last_error", C.c_char_p, [_P]),
    ("isis_mg_set_profiling", _I, [_P, _I]),
    ("isis_op_halfsweep", _I, [C.POINTER(ModelParamsC), _D, _I, _D, _P, _P, _P, _I, _P]),
    ("isis_force", _I, [C.POINTER(ModelParamsC), _D, _I, _D, _P, _P, _P, _P, _P, _P]),
    ("isis_op_sweeps", _I, [C.POINTER(ModelParamsC), _D, _I, _D, _P, _P, _P, _P, _I, _I, _P]),
    ("isis_op_prolong_sweeps", _I,
     [C.POINTER(ModelParamsC), _D, _I, _D, _P, _P, _P, _P, _P, _P, _I, _I, _P]),
    ("isis_op_defect", _I, [C.POINTER(ModelParamsC), _D, _I, _D, _P, _P, _P, _P, _P]),
    ("isis_op_restrict", _I, [_I, _P, _P, _P]),
    ("isis_op_fas_descend", _I, [C.POINTER(ModelParamsC), _D, _I, _D, _P, _P, _P, _P, _P, _P,
                                 _P, _P, _P, _P]),
    ("isis_op_restrict_fw", _I, [_I, _P, _P, _P]),
    ("isis_op_masked_defect", _I, [C.POINTER(ModelParamsC), _D, _I, _D, _P, _P, _P, _P, _P, _P,
                                   _P, _P]),
    ("isis_op_masked_halfsweep", _I, [C.POINTER(ModelParamsC), _D, _I, _D, _P, _P, _P, _P, _P,
                                      _P, _I, _P]),
    ("isis_patch_workspace_size", C.c_size_t, [_I]),
    ("isis_patch_solve", _I, [C.POINTER(ModelParamsC), _D, _I, _D, _P, _P, _P, _P, _I, _I, _D,
                              _P, C.c_size_t, C.POINTER(_I), C.POINTER(_D), _P]),
    ("isis_op_prolong_correct", _I, [_I, _P, _P, _P, _P]),
    ("isis_op_prolong_correct_w", _I, [_I, _P, _P, _P, _P]),
    ("isis_op_coarse_solve", _I, [C.POINTER(ModelParamsC), _D, _D, _P, _P, _P, _I, _P]),
    ("isis_op_cold_start", _I, [C.POINTER(ModelParamsC), _D, C.c_long, _P, _P, _P]),
    ("isis_unet_param_count", C.c_size_t, []),
    ("isis_unet_workspace_size", C.c_size_t, [_I, _I]),
    ("isis_unet_predict", _I, [_P, _P, _P, _D, _I, _P, _P, _P, C.c_size_t, _P]),
    ("isis_unet_train_step", _I, [_P, _P, _P, _I, C.c_float, _P, _P, _P, _D, _I, _P, C.c_size_t,
                                  C.POINTER(C.c_float), _P, _P]),
    ("isis_unet_forward", _I, [_P, _P, _P, _D, _I, _P, _P, C.c_size_t, _P]),
    ("isis_unet_backward", _I, [_P, _P, _P, _I, _P, C.c_size_t, _P, C.POINTER(C.c_float), _P]),
    ("isis_unet_adam_step", _I, [_P, _P, _P, _P, C.c_long, _I, C.c_float, _P]),
    ("isis_unet_tensor", _I, [_P, _I, _I, C.POINTER(_P), C.POINTER(C.c_long),
                              C.POINTER(_I)]),
    ("isis_unet_last_error", C.c_char_p, []),
    ("isis_conv3_fwd", _I, [_P, _I, _I, _P, _P, _I, _I, _P, _P, _P]),
    ("isis_conv3_flip_weights", _I, [_P, _I, _I, _P, _P]),
    ("isis_conv3_bwd_weight_workspace", C.c_size_t, [_I, _I, _I]),
    ("isis_conv3_bwd_weight", _I, [_P, _I, _I, _P, _I, _P, _P, _P, C.c_size_t, _P]),
]


def lib():
    """Load libisis_mg.so (raises if it has not been built: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1307_6748_amd.build` "
                "(the solver has no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib
