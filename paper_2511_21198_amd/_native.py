"""ctypes binding of libfsd.so (include/fsd.h).  Argument marshalling only:
every step of the solver runs in the HIP library.

The library is loaded after ``torch`` so that it shares torch's HIP runtime
(same device memory, same streams).  A missing library raises at import
time; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (loads the HIP runtime the library binds to)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfsd.so")

# fsd_status
OK, EINVAL, ENOTCONV, EBREAKDOWN, ENONFINITE, ESMALLWS, EHIP, EUNSUPPORTED, ENOTBOUND = range(9)
# fsd_solver
SOLVER_AUTO, SOLVER_PCG, SOLVER_PGMRES, SOLVER_PGMRES2 = 0, 1, 2, 3
# fsd_precision
PREC_FP64, PREC_MIXED = 0, 1
# fsd_x0_mode
X0_PREV, X0_ZERO, X0_EXTERNAL, X0_EXTRAP, X0_GUARDED = 0, 1, 2, 3, 4
# fsd_precond
PC_TAU, PC_NONE, PC_TCHAN, PC_STRANG = 0, 1, 2, 3
# engines and passes (fsd_set_engine)
ENGINES = {"auto": 0, "wave": 1, "col": 2, "colh": 3, "stage": 4, "stage_half": 5, "wave1": 6}
PASSES = {"toep_x": 0, "toep_y": 1, "toep_z": 2, "dst_x": 3, "dst_y": 4, "dsts_last": 5}


class Params(C.Structure):
    _fields_ = [
        ("dim", C.c_int),
        ("n", C.c_int * 3),
        ("a", C.c_double * 3),
        ("b", C.c_double * 3),
        ("delta", C.c_double * 3),
        ("kplus", C.c_double * 3),
        ("kminus", C.c_double * 3),
        ("M", C.c_int),
        ("T", C.c_double),
        ("solver", C.c_int),
        ("restart", C.c_int),
        ("tol", C.c_double),
        ("maxit", C.c_long),
        ("precision", C.c_int),
        ("inner_tol", C.c_double),
        ("max_outer", C.c_int),
        ("x0_mode", C.c_int),
        ("allow_delta_zero", C.c_int),
        ("dst_mfma", C.c_int),
        ("reorth_eta2", C.c_double),
        ("precond", C.c_int),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("iters", C.c_long),
        ("outer_iters", C.c_int),
        ("converged", C.c_int),
        ("relres", C.c_double),
        ("solver_relres", C.c_double),
        ("status", C.c_int),
        ("x0_fallback", C.c_int),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ProfileEntry(C.Structure):
    _fields_ = [
        ("name", C.c_char * 32),
        ("launches", C.c_long),
        ("total_ms", C.c_double),
        ("bytes", C.c_double),
    ]


# Every symbol declared in include/fsd.h, include/fsd_nn.h and
# include/fsd_batch.h, with (restype, argtypes).
_VP = C.c_void_p
SIGNATURES = {
    "fsd_default_params": (C.c_int, [C.POINTER(Params)]),
    "fsd_init_problem": (C.c_int, [C.POINTER(Params), C.POINTER(_VP)]),
    "fsd_destroy": (None, [_VP]),
    "fsd_workspace_bytes": (C.c_size_t, [_VP]),
    "fsd_bind": (C.c_int, [_VP, _VP, C.c_size_t, _VP]),
    "fsd_apply_A": (C.c_int, [_VP, _VP, _VP]),
    "fsd_apply_rhs": (C.c_int, [_VP, _VP, _VP, _VP]),
    "fsd_apply_Pinv": (C.c_int, [_VP, _VP, _VP]),
    "fsd_apply_A32": (C.c_int, [_VP, _VP, _VP]),
    "fsd_apply_A_noalloc": (C.c_int, [_VP, _VP, _VP]),
    "fsd_noalloc_scratch_bytes": (C.c_size_t, []),
    "fsd_apply_Pinv32": (C.c_int, [_VP, _VP, _VP]),
    "fsd_solve": (C.c_int, [_VP, _VP, _VP, C.POINTER(Stats)]),
    "fsd_cn_step": (C.c_int, [_VP, _VP, _VP, _VP, _VP, C.POINTER(Stats)]),
    "fsd_get_coefficients": (C.c_int, [_VP, C.c_int, C.POINTER(C.c_double),
                                       C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "fsd_reset_history": (C.c_int, [_VP]),
    "fsd_set_graphs": (C.c_int, [_VP, C.c_int]),
    "fsd_set_engine": (C.c_int, [_VP, C.c_int, C.c_int, C.c_int]),
    "fsd_autotune": (C.c_int, [_VP]),
    "fsd_engines": (C.c_int, [_VP, C.c_char_p, C.c_int]),
    "fsd_profile_enable": (C.c_int, [_VP, C.c_int]),
    "fsd_profile_read": (C.c_int, [_VP, C.POINTER(ProfileEntry), C.c_int]),
    "fsd_hbm_copy": (C.c_int, [_VP, _VP, C.c_size_t, _VP]),
    "fsd_status_string": (C.c_char_p, [C.c_int]),
    "fsd_last_error": (C.c_char_p, []),
    "fsd_version": (C.c_char_p, []),
    # fsd_nn.h
    "fsd_nn_param_count": (C.c_long, []),
    "fsd_nn_layer": (C.c_int, [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "fsd_nn_create": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(_VP)]),
    "fsd_nn_destroy": (None, [_VP]),
    "fsd_nn_workspace_bytes": (C.c_size_t, [_VP]),
    "fsd_nn_bind": (C.c_int, [_VP, _VP, C.c_size_t, _VP]),
    "fsd_nn_features": (C.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, C.c_double, C.POINTER(C.c_double),
                                  _VP, _VP, _VP]),
    "fsd_nn_crop": (C.c_int, [_VP, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                              C.c_int, C.c_int, C.c_int, _VP, _VP]),
    "fsd_nn_forward": (C.c_int, [_VP, _VP, _VP, _VP]),
    "fsd_nn_loss_grad": (C.c_int, [_VP, _VP, _VP, _VP, C.c_int, _VP, _VP]),
    "fsd_nn_adam": (C.c_int, [C.c_long, _VP, _VP, _VP, _VP, C.c_int, C.c_double, C.c_double,
                              C.c_double, C.c_double, _VP]),
    "fsd_nn_predict": (C.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, C.c_double,
                                 C.POINTER(C.c_double), _VP]),
    # fsd_batch.h
    "fsd_batch_create": (C.c_int, [C.POINTER(Params), C.c_int, C.POINTER(_VP)]),
    "fsd_batch_destroy": (None, [_VP]),
    "fsd_batch_workspace_bytes": (C.c_size_t, [_VP]),
    "fsd_batch_offset": (C.c_size_t, [_VP, C.c_int]),
    "fsd_batch_bind": (C.c_int, [_VP, _VP, C.c_size_t, C.POINTER(_VP), C.c_int]),
    "fsd_batch_set_lanes": (C.c_int, [_VP, C.c_int]),
    "fsd_batch_lanes": (C.c_int, [_VP]),
    "fsd_batch_set_graphs": (C.c_int, [_VP, C.c_int]),
    "fsd_batch_graphs": (C.c_int, [_VP]),
    "fsd_batch_cn_step": (C.c_int, [_VP, C.POINTER(_VP), C.POINTER(_VP), C.POINTER(_VP),
                                    C.POINTER(_VP), C.POINTER(Stats)]),
    "fsd_batch_autotune": (C.c_int, [_VP, C.POINTER(_VP), C.POINTER(_VP), C.POINTER(_VP),
                                     C.POINTER(C.c_double)]),
    "fsd_batch_problem": (_VP, [_VP, C.c_int]),
}


def load(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with `python -m paper_2511_21198_amd.build` "
            "(the solver has no CPU fallback)")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = load()


class FsdError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib.fsd_last_error().decode()
        super().__init__(f"{where}: {lib.fsd_status_string(status).decode()} ({msg})")


def check(status: int, where: str):
    if status != OK:
        raise FsdError(status, where)
