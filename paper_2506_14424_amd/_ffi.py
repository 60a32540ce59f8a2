"""ctypes declarations mirroring include/sipg.h."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsipg.so")

PART_CELL, PART_INTERIOR, PART_BOUNDARY, PART_ALL = 1, 2, 4, 7
PRECOND = {"chebyshev": 0, "multigrid": 1}
F64, F32 = 0, 1
VISCOUS, POISSON, PENALTY = 0, 1, 2
OPS = {"viscous": VISCOUS, "poisson": POISSON, "penalty": PENALTY}
BC = {"D": 0, "N": 1}
LAW = {"const": 0, "sine": 1, "logfield": 2, "carreau": 3, "arrays": 4}
MAX_MODES = 16

STATUS = {
    0: "SIPG_OK", -1: "SIPG_ERR_INVALID", -2: "SIPG_ERR_OOM", -3: "SIPG_ERR_HIP",
    -4: "SIPG_ERR_NOT_CONVERGED", -5: "SIPG_ERR_BREAKDOWN", -6: "SIPG_ERR_UNSUPPORTED",
    -7: "SIPG_ERR_STATE",
}


class SipgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Mesh(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("vertices", C.POINTER(C.c_double)), ("bc", C.c_int32 * 6)]


class Viscosity(C.Structure):
    _fields_ = [("kind", C.c_int32), ("mu", C.c_double), ("amp", C.c_double),
                ("contrast", C.c_double), ("rmin", C.c_double), ("rmax", C.c_double),
                ("mu0", C.c_double), ("mu_inf", C.c_double), ("lam", C.c_double),
                ("n_exp", C.c_double), ("kappa", C.c_double), ("a_exp", C.c_double),
                ("n_modes", C.c_int32), ("k", C.POINTER(C.c_int32)), ("a", C.POINTER(C.c_double)),
                ("v", C.POINTER(C.c_double)), ("phi", C.POINTER(C.c_double)),
                ("mu_cell", C.POINTER(C.c_double)), ("mu_face", C.POINTER(C.c_double))]


class Params(C.Structure):
    _fields_ = [("op", C.c_int32), ("degree", C.c_int32), ("alpha", C.c_double),
                ("penalty", C.c_double), ("tau_div", C.POINTER(C.c_double)),
                ("tau_cont", C.POINTER(C.c_double))]


class SolveOpts(C.Structure):
    _fields_ = [("rel_tol", C.c_double), ("max_iter", C.c_int32), ("precond_precision", C.c_int32),
                ("cheb_degree", C.c_int32), ("cheb_ratio", C.c_double), ("cheb_safety", C.c_double),
                ("lanczos_steps", C.c_int32), ("check_every", C.c_int32), ("max_restarts", C.c_int32),
                ("precond_kind", C.c_int32), ("use_graph", C.c_int32),
                ("reuse_eigs", C.c_int32)]


class MgOpts(C.Structure):
    _fields_ = [("coarse_degree", C.c_int32), ("min_cells", C.c_int32), ("max_levels", C.c_int32),
                ("h_coarsen", C.c_int32), ("continuous", C.c_int32), ("direct_max", C.c_int32)]


PICARD_HISTORY = 64
PICARD_NOALLOC_MAX_DOF = 2097152   # SIPG_PICARD_NOALLOC_MAX_DOF


class PicardOpts(C.Structure):
    _fields_ = [("rel_tol", C.c_double), ("abs_tol", C.c_double), ("max_iter", C.c_int32), ("aitken", C.c_int32)]


class PicardInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("linear_iterations", C.c_int32), ("residual_initial", C.c_double),
                ("residual_final", C.c_double), ("status", C.c_int32), ("recorded", C.c_int32),
                ("residual_norms", C.c_double * PICARD_HISTORY), ("omegas", C.c_double * PICARD_HISTORY)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("restarts", C.c_int32), ("rel_residual", C.c_double),
                ("lambda_max", C.c_double), ("status", C.c_int32)]


class SplitOpts(C.Structure):
    _fields_ = [("pressure", SolveOpts), ("viscous", SolveOpts), ("penalty", SolveOpts), ("zeta", C.c_double),
                ("warm_start", C.c_int32)]


class SplitInfo(C.Structure):
    _fields_ = [("pressure", SolveInfo), ("viscous", SolveInfo), ("penalty", SolveInfo)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2506_14424_amd.build` "
                          "(there is no CPU fallback)")
    # torch ships its own HIP runtime; importing it first makes the library
    # bind to that runtime (by soname) instead of loading a second HIP and HSA
    # runtime into the process, which cannot share streams or device pointers
    # with torch's and crashes the process
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    st = C.c_int32
    sig = {
        "sipg_abi_version": (C.c_int32, []),
        "sipg_last_error": (C.c_char_p, []),
        "sipg_plan_create": (st, [C.POINTER(Mesh), C.POINTER(Viscosity), C.POINTER(Params), C.POINTER(P)]),
        "sipg_plan_destroy": (None, [P]),
        "sipg_dof_count": (C.c_int64, [P]),
        "sipg_face_count": (C.c_int64, [P]),
        "sipg_plan_workspace_bytes": (st, [P, C.c_int32, C.POINTER(C.c_size_t)]),
        "sipg_plan_bind": (st, [P, P, C.c_size_t, C.c_int32, P]),
        "sipg_apply": (st, [P, C.c_int32, P, P, P]),
        "sipg_apply_parts": (st, [P, C.c_int32, C.c_int32, P, P, P]),
        "sipg_diagonal": (st, [P, C.c_int32, C.c_int32, P, P]),
        "sipg_viscosity_values": (st, [P, P, P, P]),
        "sipg_solve_opts_default": (None, [C.POINTER(SolveOpts)]),
        "sipg_solve": (st, [P, P, P, C.POINTER(SolveOpts), C.POINTER(SolveInfo), P]),
        "sipg_solve_begin": (st, [P, P, P, C.POINTER(SolveOpts), P]),
        "sipg_solve_advance": (st, [P, C.c_int32]),
        "sipg_solve_poll": (st, [P, C.POINTER(C.c_int32), C.POINTER(SolveInfo)]),
        "sipg_mg_opts_default": (None, [C.POINTER(MgOpts)]),
        "sipg_plan_set_multigrid": (st, [P, C.POINTER(MgOpts)]),
        "sipg_multigrid_levels": (C.c_int32, [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_int32]),
        "sipg_precondition": (st, [P, P, P, C.POINTER(SolveOpts), P]),
        "sipg_multigrid_transfer": (st, [P, C.c_int32, C.c_int32, C.c_int32, P, P, P]),
        "sipg_update_viscosity": (st, [P, P, P]),
        "sipg_picard_opts_default": (None, [C.POINTER(PicardOpts)]),
        "sipg_picard_work_bytes": (C.c_size_t, [P]),
        "sipg_picard_solve": (st, [P, P, P, P, C.POINTER(SolveOpts), C.POINTER(PicardOpts), C.POINTER(PicardInfo), P]),
        "sipg_picard_solve_noalloc": (st, [P, P, P, C.POINTER(SolveOpts), C.POINTER(PicardOpts), C.POINTER(PicardInfo), P]),
        "sipg_convective_step": (st, [P, P, P, P, P, C.c_double, P, P]),
        "sipg_pressure_rhs": (st, [P, P, P, P, P, P, P, C.c_double, P, P]),
        "sipg_wall_load": (st, [P, P, P, P]),
        "sipg_projection": (st, [P, P, P, P, C.c_int32, C.c_double, P, P, P]),
        "sipg_update_penalty_factors": (st, [P, P, C.c_double, C.c_double, P]),
        "sipg_split_opts_default": (None, [C.POINTER(SplitOpts)]),
        "sipg_split_work_bytes": (C.c_size_t, [P, P]),
        "sipg_split_step": (st, [P, P, P, P, P, P, P, C.c_double, P, P, P, C.POINTER(SplitOpts),
                                 C.POINTER(SplitInfo), P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


lib = _load()


def check(code: int) -> None:
    if code != 0:
        raise SipgError(code, lib.sipg_last_error().decode())
