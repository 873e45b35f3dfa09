"""ctypes declarations of libkktfwi.so (the C ABI in include/kktfwi.h).

The shared library is required: there is no CPU or Python fallback.  If it is
missing, importing the package still works but every call raises.
"""

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkktfwi.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "kktfwi.h")

KF_OK, KF_EINVAL, KF_ESHAPE, KF_ENOMEM, KF_EHIP, KF_ENOCONV, KF_EBREAKDOWN, KF_ENAN, KF_ESTATE = range(9)
STATUS_NAMES = {0: "KF_OK", 1: "KF_EINVAL", 2: "KF_ESHAPE", 3: "KF_ENOMEM", 4: "KF_EHIP", 5: "KF_ENOCONV",
                6: "KF_EBREAKDOWN", 7: "KF_ENAN", 8: "KF_ESTATE"}
KF_C128, KF_C64, KF_MIXED = 0, 1, 2
KF_PC_EXACT, KF_PC_INEXACT, KF_PC_MULTIGRID = 0, 1, 2
KF_OUTER_FGMRES, KF_OUTER_BICGSTAB = 0, 1


class KfDesc(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("nz", C.c_int32), ("h", C.c_double), ("npml", C.c_int32),
        ("pml_r0", C.c_double), ("pml_cref", C.c_double), ("omega", C.c_double),
        ("K", C.c_int32), ("src_ix", C.POINTER(C.c_int32)), ("src_iz", C.POINTER(C.c_int32)),
        ("nrec", C.c_int32), ("rec_ix", C.POINTER(C.c_int32)), ("rec_iz", C.POINTER(C.c_int32)),
        ("w", C.POINTER(C.c_double)), ("eps", C.c_double), ("reg_on_update", C.c_int32),
    ]


class KfNewtonOpts(C.Structure):
    _fields_ = [
        ("rtol", C.c_double), ("restart", C.c_int32), ("maxit", C.c_int32), ("pc", C.c_int32),
        ("fwd_prec", C.c_int32), ("fwd_rtol", C.c_double), ("misfit_after", C.c_int32),
        ("reorth_eta", C.c_double), ("outer", C.c_int32),
    ]


class KfNewtonStats(C.Structure):
    _fields_ = [
        ("outer_iters", C.c_int32), ("restarts", C.c_int32), ("rel_res", C.c_double),
        ("rel_res_hist", C.c_double * 512), ("misfit_before", C.c_double), ("misfit_after", C.c_double),
        ("phi_before", C.c_double), ("ds_imag_ratio", C.c_double), ("t_factor_ms", C.c_double),
        ("t_forward_ms", C.c_double), ("t_precond_ms", C.c_double), ("t_matvec_ms", C.c_double),
        ("t_orth_ms", C.c_double), ("t_total_ms", C.c_double), ("fwd_refine_iters", C.c_int32),
        ("reorth_passes", C.c_int32),
    ]


class KfTuneEntry(C.Structure):
    _fields_ = [("chunks", C.c_int32), ("sources_per_group", C.c_int32), ("t_factor_ms", C.c_double),
                ("t_solve_ms", C.c_double), ("score_ms", C.c_double)]


class KfCgOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("maxit", C.c_int32), ("solve_prec", C.c_int32), ("solve_rtol", C.c_double),
                ("real_constrained", C.c_int32), ("fwd_prec", C.c_int32), ("fwd_rtol", C.c_double)]


class KfCgStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("solves", C.c_int32), ("rel_res", C.c_double), ("true_rel_res", C.c_double),
                ("rel_res_hist", C.c_double * 512), ("misfit_before", C.c_double), ("phi_before", C.c_double),
                ("t_factor_ms", C.c_double), ("t_forward_ms", C.c_double), ("t_cg_ms", C.c_double),
                ("t_total_ms", C.c_double)]


class KfMgStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("vcycles", C.c_int32), ("levels", C.c_int32), ("rel_res_max", C.c_double)]


class KfSolveStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("rel_res_max", C.c_double)]


P = C.c_void_p
_SIGNATURES = {
    "kf_version": (C.c_char_p, []),
    "kf_last_error": (C.c_char_p, []),
    "kf_create": (C.c_int, [C.POINTER(KfDesc), P, C.c_int32, P, C.POINTER(P)]),
    "kf_destroy": (C.c_int, [P]),
    "kf_set_gamma": (C.c_int, [P, P]),
    "kf_get_gamma": (C.c_int, [P, P]),
    "kf_set_background": (C.c_int, [P, P]),
    "kf_get_background": (C.c_int, [P, P]),
    "kf_set_stream": (C.c_int, [P, P]),
    "kf_factor": (C.c_int, [P, C.c_int32, C.POINTER(C.c_double)]),
    "kf_set_solver_shape": (C.c_int, [P, C.c_int32, C.c_int32]),
    "kf_get_solver_shape": (C.c_int, [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "kf_autotune": (C.c_int, [P, C.c_int32, C.c_double, C.POINTER(KfTuneEntry), C.c_int32, C.POINTER(C.c_int32)]),
    "kf_stencil_apply": (C.c_int, [P, C.c_int32, C.c_int32, P, P]),
    "helmholtz_solve": (C.c_int, [P, C.c_int32, C.c_int32, P, P, C.c_double, C.c_int32,
                                  C.POINTER(KfSolveStats)]),
    "kkt_apply": (C.c_int, [P, P, P]),
    "kkt_apply_noalloc": (C.c_int, [P, P, P]),
    "precond_apply": (C.c_int, [P, C.c_int32, P, P]),
    "newton_step": (C.c_int, [P, P, C.POINTER(KfNewtonOpts), P, P, C.c_int32, C.POINTER(KfNewtonStats)]),
    "helmholtz_adjoint_gradient": (C.c_int, [P, C.c_int32, P, P, P]),
    "newton_continuation": (C.c_int, [C.POINTER(P), C.c_int32, C.POINTER(P), C.POINTER(C.c_int32),
                                      C.POINTER(KfNewtonOpts), P, C.POINTER(KfNewtonStats)]),
    "newton_step_concurrent": (C.c_int, [C.POINTER(P), C.c_int32, C.POINTER(P), C.POINTER(KfNewtonOpts),
                                         C.POINTER(P), C.POINTER(P), C.c_int32, C.POINTER(KfNewtonStats)]),
    "rsgn_cg_step": (C.c_int, [P, P, C.POINTER(KfCgOpts), P, P, C.c_int32, C.POINTER(KfCgStats)]),
    "kf_sources": (C.c_int, [P, P]),
    "kf_set_hblock": (C.c_int, [P, C.c_int32, C.c_int32]),
    "kf_hblock_add_pair": (C.c_int, [P, P, P]),
    "kf_set_multigrid": (C.c_int, [P, C.c_int32, C.c_double, C.c_double, C.c_int32, C.c_int32]),
    "helmholtz_solve_mg": (C.c_int, [P, C.c_int32, P, P, C.c_double, C.c_int32, C.POINTER(KfMgStats)]),
    "kf_mg_vcycle": (C.c_int, [P, P, P]),
    "kf_mg_levels": (C.c_int, [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "kf_sizes": (C.c_int, [P, C.POINTER(C.c_int64)]),
    "kf_batch_create": (C.c_int, [C.POINTER(P), C.c_int32, P, C.POINTER(P)]),
    "kf_batch_destroy": (C.c_int, [P]),
    "kf_batch_factor": (C.c_int, [P, C.c_int32, C.POINTER(C.c_double)]),
    "helmholtz_solve_batched": (C.c_int, [P, C.c_int32, C.c_int32, C.POINTER(P), C.POINTER(P)]),
    "newton_step_batched": (C.c_int, [P, C.POINTER(P), C.POINTER(KfNewtonOpts), C.POINTER(P), C.POINTER(P),
                                      C.c_int32, C.c_int32, C.POINTER(KfNewtonStats)]),
    "kf_profile_enable": (C.c_int, [P, C.c_int32]),
    "kf_profile_read": (C.c_int, [P, C.c_char_p, C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
    "kf_profile_only": (C.c_int, [P, C.c_char_p]),
    "kf_profile_work": (C.c_int, [P, C.c_char_p, C.POINTER(C.c_double)]),
}

_lib = None


class KFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2204_06489_amd.build` "
                               "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status, allow=()):
    if status != KF_OK and status not in allow:
        raise KFError(status, lib().kf_last_error().decode())
    return status


def header_functions():
    """Names of the functions declared in include/kktfwi.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(?:kf_status|const char \*)\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", text)))
