"""ctypes declarations of the pmgfr C ABI (include/pmgfr.h). Loads libpmgfr.so from this
package directory and fails loudly when it is missing: there is no fallback path."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpmgfr.so")

pmg_status = C.c_int32
pmg_level = C.c_void_p
pmg_factors = C.c_void_p
pmg_batch = C.c_void_p

PMG_OK = 0
PMG_E_ARG = -1
PMG_E_SHAPE = -2
PMG_E_HIP = -3
PMG_E_SINGULAR = -4
PMG_E_NONFINITE = -5
PMG_E_NOT_CONVERGED = -6
PMG_E_NOMEM = -7
PMG_BC_SLIP_WALL = -1
PMG_BC_FAR_FIELD = -2
PMG_BC_NOSLIP_WALL = -3

STATUS_NAMES = {0: "PMG_OK", -1: "PMG_E_ARG", -2: "PMG_E_SHAPE", -3: "PMG_E_HIP", -4: "PMG_E_SINGULAR",
                -5: "PMG_E_NONFINITE", -6: "PMG_E_NOT_CONVERGED", -7: "PMG_E_NOMEM"}


class LevelDesc(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("P", C.c_int32), ("geom_order", C.c_int32), ("n_elements", C.c_int32),
        ("nodes", C.POINTER(C.c_double)), ("face_nbr", C.POINTER(C.c_int32)),
        ("face_nbr_face", C.POINTER(C.c_int32)), ("face_orient", C.POINTER(C.c_int32)),
        ("gamma", C.c_double), ("rgas", C.c_double), ("eps_mode", C.c_int32),
        ("ma_inf", C.c_double), ("kappa", C.c_double), ("q_inf", C.c_double * 5), ("q_ref", C.c_double * 5),
        ("device", C.c_int32), ("mu", C.c_double), ("prandtl", C.c_double), ("br2_penalty", C.c_double),
    ]


class SolveOpts(C.Structure):
    _fields_ = [
        ("n_levels", C.c_int32), ("levels", C.POINTER(pmg_level)), ("factors", C.POINTER(pmg_factors)),
        ("n_smooth", C.POINTER(C.c_int32)), ("dtau_init", C.c_double), ("dtau_max", C.c_double),
        ("ser_exponent", C.c_double), ("refresh_every", C.c_int32), ("freeze_at_max", C.c_int32),
        ("tol_rel", C.c_double), ("max_vcycles", C.c_int32), ("alpha_r", C.c_double),
        ("use_graph", C.c_int32), ("use_cfl", C.c_int32), ("cfl_init", C.c_double), ("cfl_max", C.c_double),
        ("stage_guess", C.c_int32),
        ("ser_floor", C.c_int32),
        ("lookahead", C.c_int32),
    ]


class SolveStats(C.Structure):
    _fields_ = [
        ("n_vcycles", C.c_int32), ("n_refresh", C.c_int32), ("r0", C.c_double), ("r_final", C.c_double),
        ("history", C.POINTER(C.c_double)), ("history_capacity", C.c_int32), ("status", C.c_int32),
        ("seconds", C.c_double), ("dtau_min", C.c_double),
    ]


class NkOpts(C.Structure):
    _fields_ = [
        ("krylov_dim", C.c_int32), ("max_newton", C.c_int32), ("eta", C.c_double), ("fd_rel", C.c_double),
        ("pc_rel", C.c_double), ("precondition", C.c_int32),
    ]


DP = C.c_void_p   # device pointers travel as plain addresses

SIGNATURES = {
    "pmg_last_error": (C.c_char_p, []),
    "pmg_abi_version": (C.c_int32, []),
    "pmg_level_create": (pmg_status, [C.POINTER(LevelDesc), C.POINTER(pmg_level)]),
    "pmg_level_destroy": (pmg_status, [pmg_level]),
    "pmg_level_info": (pmg_status, [pmg_level, C.POINTER(C.c_int32)]),
    "pmg_level_points": (pmg_status, [pmg_level, C.POINTER(C.c_double)]),
    "pmg_level_status": (pmg_status, [pmg_level, C.POINTER(C.c_int32)]),
    "pmg_level_dx": (pmg_status, [pmg_level, C.POINTER(C.c_double)]),
    "pmg_level_epw": (pmg_status, [pmg_level, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "pmg_level_set_epw": (pmg_status, [pmg_level, C.c_int32]),
    "pmg_level_autotune": (pmg_status, [pmg_level, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                        C.POINTER(C.c_double), C.c_void_p]),
    "pmg_dtau_min": (pmg_status, [pmg_level, DP, C.POINTER(C.c_double), C.c_void_p]),
    "pmg_factors_create": (pmg_status, [pmg_level, C.c_int32, C.POINTER(pmg_factors)]),
    "pmg_factors_destroy": (pmg_status, [pmg_factors]),
    "pmg_line_factors_create": (pmg_status, [pmg_level, C.c_int32, C.POINTER(C.c_int32), C.c_int32, C.c_int32,
                                             C.POINTER(pmg_factors)]),
    "pmg_line_blocks": (pmg_status, [pmg_factors, DP, C.c_double, C.c_double, DP, DP, DP, C.c_void_p]),
    "fr_residual": (pmg_status, [pmg_level, DP, DP, DP, C.c_double, DP, DP, C.c_void_p]),
    "fr_residual_noalloc": (pmg_status, [pmg_level, DP, DP, DP, C.c_double, DP, DP, C.c_void_p]),
    "fr_conservative": (pmg_status, [pmg_level, DP, DP, C.c_void_p]),
    "fr_element_jacobian": (pmg_status, [pmg_level, DP, C.c_double, C.c_double, DP, pmg_factors, C.c_void_p]),
    "ejacobi_sweep": (pmg_status, [pmg_level, pmg_factors, DP, DP, DP, C.c_double, C.c_int32, C.c_double, DP, DP,
                                   C.c_void_p]),
    "pmg_restrict": (pmg_status, [pmg_level, pmg_level, DP, DP, C.c_int32, C.c_void_p]),
    "pmg_prolong": (pmg_status, [pmg_level, pmg_level, DP, DP, C.c_int32, C.c_void_p]),
    "esdirk_stage_solve": (pmg_status, [C.POINTER(SolveOpts), C.c_double, C.c_double, DP, C.POINTER(DP),
                                        C.POINTER(C.c_double), C.c_int32, DP, DP, C.POINTER(SolveStats),
                                        C.c_void_p]),
    "esdirk_step": (pmg_status, [C.POINTER(SolveOpts), C.c_int32, C.c_double, DP, DP, C.POINTER(SolveStats),
                                 C.c_int32, C.c_void_p]),
    "esdirk_stages": (C.c_int32, [C.c_int32]),
    "esdirk_butcher": (C.c_int32, [C.c_int32, C.POINTER(C.c_double)]),
    "nk_work_elems": (C.c_int64, [pmg_level, C.c_int32]),
    "nk_stage_solve": (pmg_status, [C.POINTER(SolveOpts), C.POINTER(NkOpts), C.c_double, C.c_double, DP,
                                    C.POINTER(DP), C.POINTER(C.c_double), C.c_int32, DP, DP, C.POINTER(SolveStats),
                                    C.POINTER(C.c_int32), C.c_void_p]),
    "pmg_batch_create": (pmg_status, [C.POINTER(SolveOpts), C.c_int32, C.POINTER(pmg_batch)]),
    "pmg_batch_destroy": (pmg_status, [pmg_batch]),
    "pmg_batch_size": (C.c_int32, [pmg_batch]),
    "esdirk_stage_solve_batched": (pmg_status, [pmg_batch, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                                C.POINTER(DP), C.POINTER(C.POINTER(DP)), C.POINTER(C.POINTER(C.c_double)),
                                                C.POINTER(C.c_int32), C.POINTER(DP), C.POINTER(DP),
                                                C.POINTER(SolveStats), C.c_void_p]),
    "esdirk_step_batched": (pmg_status, [pmg_batch, C.c_int32, C.POINTER(C.c_double), C.POINTER(DP), C.POINTER(DP),
                                         C.POINTER(SolveStats), C.c_void_p]),
}

_lib = None


def lib() -> C.CDLL:
    """The loaded library, with argument and return types declared."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1908_03972_amd.build` "
                               "(the HIP library is required; there is no fallback)")
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib


class PmgError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        super().__init__(f"{where} failed with {STATUS_NAMES.get(status, status)}: {message}")


def check(status: int, where: str) -> None:
    if status != PMG_OK:
        msg = lib().pmg_last_error()
        raise PmgError(status, where, msg.decode() if msg else "")
