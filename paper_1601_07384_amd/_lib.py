"""ctypes binding of ``libstdg.so`` (the C ABI in ``include/stdg.h``).

Argument marshalling only: every step of the computation runs in the HIP
library.  Loading fails loudly when the library has not been built.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstdg.so")

STDG_OK = 0
STDG_NOT_CONVERGED = 1
STDG_ERR_ARG = -1
STDG_ERR_MESH = -2
STDG_ERR_NUMERIC = -3
STDG_ERR_DEVICE = -4
STDG_ERR_NOMEM = -5
STDG_LAYOUT_ELEMENT = 0
STDG_LAYOUT_RUN = 1
STDG_FP64 = 0
STDG_FP32 = 1
STDG_AUTO = 0
STDG_CG = 1
STDG_GMRES = 2
STDG_CG_TIME = 3


class Config(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("p_gamma", ctypes.c_int32),
                ("nu", ctypes.c_double), ("dt", ctypes.c_double),
                ("periodic", ctypes.c_int32),
                ("box_lo", ctypes.c_double * 3), ("box_hi", ctypes.c_double * 3),
                ("anchor_tet", ctypes.c_int64), ("anchor_node", ctypes.c_int32),
                ("reorder", ctypes.c_int32)]


class MeshInfo(ctypes.Structure):
    _fields_ = [("n_tet", ctypes.c_int64), ("n_face", ctypes.c_int64),
                ("n_interior_face", ctypes.c_int64),
                ("N", ctypes.c_int32), ("G", ctypes.c_int32), ("Nst", ctypes.c_int32),
                ("n_classes", ctypes.c_int32), ("anchor_internal", ctypes.c_int64),
                ("inner_layout", ctypes.c_int32), ("inner_len", ctypes.c_int64),
                ("inner_per_element", ctypes.c_int32)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("rtol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("inner_rtol", ctypes.c_double),
                ("max_outer", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("precond", ctypes.c_int32)]


class SolveReport(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("outer_iters", ctypes.c_int32),
                ("inner_iters", ctypes.c_int32), ("applies", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("seconds", ctypes.c_double),
                ("initial_rel_residual", ctypes.c_double), ("fused_iter_us", ctypes.c_double)]


STDG_GUESS_ZERO = 0
STDG_GUESS_PREVIOUS = 1
STDG_BICGSTAB = 4
STDG_PRECOND_NONE = 0
STDG_PRECOND_BLOCK_JACOBI = 1
STDG_KRYLOV_ZERO = 0
STDG_KRYLOV_PREVIOUS = 1
STDG_KRYLOV_EXTRAPOLATE = 2
STDG_KRYLOV_LEARNED = 3
STDG_LOSS_MSE = 0
STDG_LOSS_RESIDUAL = 1


class StepOpts(ctypes.Structure):
    _fields_ = [("n_picard", ctypes.c_int32), ("pressure_guess", ctypes.c_int32),
                ("pressure", SolveOpts), ("viscous", SolveOpts),
                ("krylov_guess", ctypes.c_int32), ("model", ctypes.c_void_p),
                ("hist", ctypes.c_void_p), ("rec_b", ctypes.c_void_p),
                ("rec_x", ctypes.c_void_p), ("theta", ctypes.c_double)]


class StepReport(ctypes.Structure):
    _fields_ = [("pressure_iters", ctypes.c_int32), ("viscous_iters", ctypes.c_int32),
                ("max_pressure_residual", ctypes.c_double),
                ("max_viscous_residual", ctypes.c_double), ("seconds", ctypes.c_double),
                ("pressure_seconds", ctypes.c_double), ("viscous_seconds", ctypes.c_double),
                ("pressure_applies", ctypes.c_int32), ("first_pressure_iters", ctypes.c_int32),
                ("first_pressure_seconds", ctypes.c_double),
                ("first_initial_residual", ctypes.c_double),
                ("pressure_fused_iter_us", ctypes.c_double),
                ("guess_weight_network", ctypes.c_double), ("status", ctypes.c_int32)]


class ModelConfig(ctypes.Structure):
    _fields_ = [("hidden", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("lr", ctypes.c_double), ("beta1", ctypes.c_double),
                ("beta2", ctypes.c_double), ("eps", ctypes.c_double),
                ("init_scale_out", ctypes.c_double), ("loss", ctypes.c_int32)]


class TrainReport(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("samples", ctypes.c_int64),
                ("first_loss", ctypes.c_double), ("last_loss", ctypes.c_double),
                ("seconds", ctypes.c_double)]


# (name, restype, argtypes) of every symbol declared in include/stdg.h
_P = ctypes.c_void_p
SIGNATURES = [
    ("stdg_mesh_build", ctypes.c_int, [_P, ctypes.c_int64, _P, ctypes.c_int64,
                                        ctypes.POINTER(Config), ctypes.POINTER(_P)]),
    ("stdg_mesh_build_host", ctypes.c_int, [_P, ctypes.c_int64, _P, ctypes.c_int64,
                                             ctypes.POINTER(Config), ctypes.POINTER(_P)]),
    ("stdg_mesh_build_curved", ctypes.c_int, [_P, ctypes.c_int64, _P, ctypes.c_int64, _P, ctypes.c_int32,
                                               ctypes.POINTER(Config), ctypes.POINTER(_P)]),
    ("stdg_mesh_blocks", ctypes.c_int, [_P, _P, _P, _P, _P]),
    ("stdg_mesh_info_get", ctypes.c_int, [_P, ctypes.POINTER(MeshInfo)]),
    ("stdg_mesh_permutation", ctypes.c_int, [_P, _P]),
    ("stdg_mesh_faces", ctypes.c_int, [_P, _P, _P, _P, _P]),
    ("stdg_mesh_free", None, [_P]),
    ("stdg_pressure_apply", ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P]),
    ("stdg_pressure_apply_f32", ctypes.c_int, [_P, _P, _P, _P]),
    ("stdg_pressure_apply_spatial_f32", ctypes.c_int, [_P, _P, _P, _P]),
    ("stdg_inner_from_f64", ctypes.c_int, [_P, _P, ctypes.c_double, _P, _P]),
    ("stdg_inner_to_f64", ctypes.c_int, [_P, _P, ctypes.c_double, _P, _P]),
    ("stdg_solve_opts_default", None, [ctypes.POINTER(SolveOpts)]),
    ("stdg_pressure_solve", ctypes.c_int, [_P, _P, _P, ctypes.POINTER(SolveOpts),
                                            ctypes.POINTER(SolveReport), _P]),
    ("stdg_pressure_solve_noalloc", ctypes.c_int, [_P, _P, _P, ctypes.POINTER(SolveOpts),
                                                    ctypes.POINTER(SolveReport), _P]),
    ("stdg_step_opts_default", None, [ctypes.POINTER(StepOpts)]),
    ("stdg_picard_step", ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.POINTER(StepOpts),
                                         ctypes.POINTER(StepReport), _P]),
    ("stdg_dual_from_main", ctypes.c_int, [_P, _P, _P, _P]),
    ("stdg_main_from_dual", ctypes.c_int, [_P, _P, _P, _P]),
    ("stdg_divergence", ctypes.c_int, [_P, _P, _P, _P]),
    ("stdg_model_config_default", None, [ctypes.POINTER(ModelConfig)]),
    ("stdg_model_create", ctypes.c_int, [_P, ctypes.POINTER(ModelConfig), ctypes.POINTER(_P)]),
    ("stdg_model_free", ctypes.c_int, [_P]),
    ("stdg_model_info", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    ("stdg_model_set_params", ctypes.c_int, [_P, _P]),
    ("stdg_model_get_params", ctypes.c_int, [_P, _P]),
    ("stdg_model_get_grads", ctypes.c_int, [_P, _P]),
    ("stdg_model_features", ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    ("stdg_model_forward", ctypes.c_int, [_P, _P, ctypes.c_int64, _P, _P]),
    ("stdg_model_loss_grad", ctypes.c_int, [_P, _P, _P, ctypes.c_int64,
                                             ctypes.POINTER(ctypes.c_double), _P]),
    ("stdg_model_residual_loss_grad", ctypes.c_int, [_P, _P, _P, _P, _P, _P, ctypes.POINTER(ctypes.c_double),
                                                      _P]),
    ("stdg_model_adam_step", ctypes.c_int, [_P, _P]),
    ("stdg_model_train", ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P, _P, _P, ctypes.c_int32,
                                         ctypes.POINTER(TrainReport), _P]),
    ("stdg_model_predict", ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    ("stdg_last_error", ctypes.c_char_p, []),
]

_lib = None


def load():
    """Load libstdg.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run paper_1601_07384_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class StdgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"stdg error {code}: {msg}")
        self.code = code


def check(code, allow=(STDG_OK,)):
    if code in allow:
        return code
    raise StdgError(code, load().stdg_last_error().decode())
