"""ctypes declarations of the C interface in include/stmlmc.h.

Loading fails loudly when the built library is absent: there is no fallback.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("STM_LIBRARY", os.path.join(HERE, "libstmlmc.so"))

STM_MAX_LEVELS = 8

STATUS = {
    0: "STM_OK", -1: "STM_E_INVALID", -2: "STM_E_NOMEM", -3: "STM_E_DEVICE",
    -4: "STM_E_NOT_CONVERGED", -5: "STM_E_NONFINITE", -6: "STM_E_UNSUPPORTED",
}
FIBER_LAWS = {"diag2d": 0, "rot3d": 1, "x": 2, "diag": 3}
PRECISIONS = {"fp64": 0, "mixed": 1}
FIELD_KINDS = {"lognormal": 0, "additive": 1}
IC_KINDS = {"ball": 0, "gauss": 1}
QOIS = {"activation": 0, "spacetime": 1}


class StmLevel(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("m", ctypes.c_int),
                ("smooth_sweeps", ctypes.c_int), ("cheb_ratio", ctypes.c_double),
                ("team_seconds", ctypes.c_double * 32)]


class StmProblem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double),
        ("T", ctypes.c_double),
        ("k_react", ctypes.c_double), ("a_react", ctypes.c_double),
        ("sigma_f0", ctypes.c_double), ("transverse_ratio", ctypes.c_double),
        ("fiber_law", ctypes.c_int),
        ("ic_center", ctypes.c_double * 3), ("ic_radius", ctypes.c_double),
        ("threshold", ctypes.c_double),
        ("n_levels", ctypes.c_int),
        ("levels", StmLevel * STM_MAX_LEVELS),
        ("n_modes", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("newton_tol", ctypes.c_double),
        ("newton_max", ctypes.c_int),
        ("gmres_rtol", ctypes.c_double),
        ("gmres_restart", ctypes.c_int),
        ("mg_levels", ctypes.c_int),
        ("smooth_steps", ctypes.c_int),
        ("smooth_omega", ctypes.c_double),
        ("coarse_sweeps", ctypes.c_int),
        ("smoother", ctypes.c_int),
        ("cheb_ratio", ctypes.c_double),
        ("lds_kb", ctypes.c_int),
        ("block_threads", ctypes.c_int),
        ("max_lanes", ctypes.c_int),
        ("team_size", ctypes.c_int),
        ("theta", ctypes.c_double),
        ("field_kind", ctypes.c_int),
        ("tau_relative", ctypes.c_int),
        ("ic_kind", ctypes.c_int),
        ("qoi", ctypes.c_int),
        ("newton_damping", ctypes.c_int),
        ("st_mode", ctypes.c_int),
    ]


class StmSolveStats(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int), ("newton_max_per_slab", ctypes.c_int),
        ("newton_iters", ctypes.c_int64), ("krylov_iters", ctypes.c_int64),
        ("final_step", ctypes.c_double), ("device_seconds", ctypes.c_double),
        ("algorithmic_bytes", ctypes.c_double),
        ("phase_seconds", ctypes.c_double * 8),
        ("model_bytes", ctypes.c_double),
        ("damped_steps", ctypes.c_int64),
    ]


class StmTimings(ctypes.Structure):
    _fields_ = [
        ("kl_ms", ctypes.c_double), ("solve_ms", ctypes.c_double), ("stats_ms", ctypes.c_double),
        ("solve_bytes", ctypes.c_double), ("solve_launches", ctypes.c_int),
        ("solve_teams", ctypes.c_int), ("solve_blocks", ctypes.c_int), ("solve_block", ctypes.c_int),
        ("solve_bytes_model", ctypes.c_double),
    ]


class StmMlmcResult(ctypes.Structure):
    _fields_ = [
        ("mean", ctypes.c_void_p), ("var", ctypes.c_void_p),
        ("level_mean", ctypes.c_void_p), ("level_var", ctypes.c_void_p),
        ("N", ctypes.c_int * STM_MAX_LEVELS),
        ("V", ctypes.c_double * STM_MAX_LEVELS),
        ("cost", ctypes.c_double * STM_MAX_LEVELS),
        ("bias_estimate", ctypes.c_double),
        ("newton_iters", ctypes.c_int64), ("krylov_iters", ctypes.c_int64),
        ("censored", ctypes.c_int64),
        ("rounds", ctypes.c_int), ("worst_status", ctypes.c_int),
        ("algorithmic_bytes", ctypes.c_double), ("dof_steps", ctypes.c_int64),
        ("model_bytes", ctypes.c_double),
    ]


# every symbol include/stmlmc.h declares, with (restype, argtypes)
_P = ctypes.c_void_p
SIGNATURES = {
    "stm_create": (ctypes.c_int, [ctypes.POINTER(StmProblem), _P, ctypes.POINTER(_P)]),
    "stm_destroy": (None, [_P]),
    "stm_last_error": (ctypes.c_char_p, [_P]),
    "stm_get_timings": (ctypes.c_int, [_P, ctypes.POINTER(StmTimings)]),
    "stm_level_size": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "stm_kl_synthesize": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, ctypes.c_int, _P]),
    "stm_st_solve": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, ctypes.c_int, _P,
                                    ctypes.POINTER(StmSolveStats)]),
    "stm_st_solve_noalloc": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, ctypes.c_int, _P,
                                            ctypes.POINTER(StmSolveStats)]),
    "stm_activation_map": (ctypes.c_int, [_P, ctypes.c_int, _P, ctypes.c_int, _P,
                                          ctypes.POINTER(ctypes.c_int)]),
    "stm_prolong_st": (ctypes.c_int, [_P, ctypes.c_int, _P, ctypes.c_int, _P]),
    "stm_mlmc_estimate": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_P),
                                         ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_int),
                                         ctypes.c_double, ctypes.c_int,
                                         ctypes.POINTER(StmMlmcResult)]),
}

_lib = None


def load(path=LIB_PATH):
    """Load libstmlmc.so and declare its symbols; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            "libstmlmc.so not found at %s: build it first (python -m paper_1911_06066_amd.build); "
            "this package has no CPU fallback" % path)
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
