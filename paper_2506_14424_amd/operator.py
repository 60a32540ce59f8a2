"""Operator: one plan of libsipg with its workspace in device memory."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _ffi as F
from ._ffi import check, lib


@dataclass
class SolveOptions:
    rel_tol: float = 1e-8
    max_iter: int = 5000
    precond_precision: str = "f32"   # "f32" (mixed) or "f64"
    cheb_degree: int = 5
    cheb_ratio: float = 20.0
    cheb_safety: float = 1.2
    lanczos_steps: int = 20
    check_every: int = 10
    max_restarts: int = 3
    precond: str = "chebyshev"       # or "multigrid" (after Operator.set_multigrid)
    use_graph: bool = False          # replay captured HIP graphs of the iteration chunks
    reuse_eigs: bool = False         # keep eigenvalue estimates across viscosity / penalty-factor updates

    def to_c(self) -> F.SolveOpts:
        o = F.SolveOpts()
        o.rel_tol = self.rel_tol
        o.max_iter = self.max_iter
        o.precond_precision = F.F32 if self.precond_precision == "f32" else F.F64
        o.cheb_degree = self.cheb_degree
        o.cheb_ratio = self.cheb_ratio
        o.cheb_safety = self.cheb_safety
        o.lanczos_steps = self.lanczos_steps
        o.check_every = self.check_every
        o.max_restarts = self.max_restarts
        o.precond_kind = F.PRECOND[self.precond]
        o.use_graph = int(self.use_graph)
        o.reuse_eigs = int(self.reuse_eigs)
        return o


def _stream_handle(stream) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _law_struct(law: dict | None, keep: list) -> F.Viscosity:
    v = F.Viscosity()
    if law is None:
        v.kind = F.LAW["const"]
        v.mu = 1.0
        return v
    kind = law["kind"]
    v.kind = F.LAW[kind]
    if kind == "const":
        v.mu = law["mu"]
    elif kind == "sine":
        v.mu, v.amp = law["mu"], law["amp"]
    elif kind == "arrays":
        mc = np.ascontiguousarray(law["mu_cell"], dtype=np.float64).reshape(-1)
        mf = np.ascontiguousarray(law["mu_face"], dtype=np.float64).reshape(-1)
        keep += [mc, mf]
        v.mu_cell = mc.ctypes.data_as(C.POINTER(C.c_double))
        v.mu_face = mf.ctypes.data_as(C.POINTER(C.c_double))
    elif kind in ("logfield", "carreau"):
        k = np.ascontiguousarray(law["k"], dtype=np.int32).reshape(-1)
        phi = np.ascontiguousarray(law["phi"], dtype=np.float64)
        keep += [k, phi]
        v.n_modes = len(phi)
        v.k = k.ctypes.data_as(C.POINTER(C.c_int32))
        v.phi = phi.ctypes.data_as(C.POINTER(C.c_double))
        if kind == "logfield":
            a = np.ascontiguousarray(law["a"], dtype=np.float64)
            keep.append(a)
            v.a = a.ctypes.data_as(C.POINTER(C.c_double))
            v.contrast, v.rmin, v.rmax = law["contrast"], law["rmin"], law["rmax"]
        else:
            vel = np.ascontiguousarray(law["v"], dtype=np.float64).reshape(-1)
            keep.append(vel)
            v.v = vel.ctypes.data_as(C.POINTER(C.c_double))
            v.mu0, v.mu_inf, v.lam = law["mu0"], law["mu_inf"], law["lam"]
            v.n_exp, v.kappa, v.a_exp = law["n_exp"], law["kappa"], law["a_exp"]
    else:
        raise ValueError(f"unknown law {kind}")
    return v


class Operator:
    """SIPG viscous ("viscous"), SIPG Poisson ("poisson") or penalty-step
    ("penalty": mass + divergence and normal-continuity penalties with
    per-cell factors tau_div, tau_cont) operator on a structured nx*ny*nz box
    mesh; see include/sipg.h for the discretisation."""

    def __init__(self, nx: int, ny: int, nz: int, degree: int, op: str = "viscous",
                 alpha: float = 0.0, penalty: float = 1.0, law: dict | None = None,
                 vertices: np.ndarray | None = None, bc=("D",) * 6,
                 tau_div: np.ndarray | None = None, tau_cont: np.ndarray | None = None):
        keep: list = []
        mesh = F.Mesh()
        mesh.nx, mesh.ny, mesh.nz = nx, ny, nz
        if vertices is not None:
            vv = np.ascontiguousarray(vertices, dtype=np.float64).reshape(-1)
            keep.append(vv)
            mesh.vertices = vv.ctypes.data_as(C.POINTER(C.c_double))
        for i, b in enumerate(bc):
            mesh.bc[i] = F.BC[b]
        par = F.Params()
        if op not in F.OPS:
            raise ValueError(f"unknown operator {op}")
        par.op = F.OPS[op]
        par.degree, par.alpha, par.penalty = degree, alpha, penalty
        if op == "penalty":
            if tau_div is None or tau_cont is None:
                raise ValueError("the penalty operator needs tau_div and tau_cont (one value per cell)")
            for name, t in (("tau_div", tau_div), ("tau_cont", tau_cont)):
                a = np.ascontiguousarray(t, dtype=np.float64).reshape(-1)
                if a.size != nx * ny * nz:
                    raise ValueError(f"{name} needs {nx * ny * nz} values, got {a.size}")
                keep.append(a)
                setattr(par, name, a.ctypes.data_as(C.POINTER(C.c_double)))
        lw = _law_struct(law if op == "viscous" else None, keep)
        h = C.c_void_p()
        check(lib.sipg_plan_create(C.byref(mesh), C.byref(lw), C.byref(par), C.byref(h)))
        self._h = h
        self.nx, self.ny, self.nz, self.degree, self.op = nx, ny, nz, degree, op
        self.n = degree + 1
        self.C = 1 if op == "poisson" else 3
        self.ndof = int(lib.sipg_dof_count(h))
        self.nface = int(lib.sipg_face_count(h))
        self.ncell = nx * ny * nz
        self.workspace = None
        self._with_solver = False

    @classmethod
    def from_config(cls, cfg: dict, vertices=None) -> "Operator":
        return cls(cfg["nx"], cfg["ny"], cfg["nz"], cfg["degree"], cfg["op"], cfg["alpha"],
                   cfg["penalty"], cfg.get("law"), vertices, cfg["bc"], cfg.get("tau_div"), cfg.get("tau_cont"))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib.sipg_plan_destroy(h)
            self._h = None

    # ------------------------------------------------------------- setup
    def set_multigrid(self, coarse_degree: int = 12, min_cells: int = 2, max_levels: int = 16,
                      h_coarsen: bool = True, continuous: bool = True, direct_max: int = 1024):
        """Build the hp-multigrid hierarchy (before bind); see sipg_plan_set_multigrid.
        continuous: the cph hierarchy (DG level, then continuous levels, direct
        coarse solve up to direct_max unknowns); False: all levels DG."""
        o = F.MgOpts()
        o.coarse_degree, o.min_cells, o.max_levels, o.h_coarsen = coarse_degree, min_cells, max_levels, int(h_coarsen)
        o.continuous, o.direct_max = int(continuous), direct_max
        check(lib.sipg_plan_set_multigrid(self._h, C.byref(o)))
        return self

    def multigrid_levels(self) -> list[tuple[int, int, int, int]]:
        """(degree, nx, ny, nz) of every level, finest first."""
        nl = int(lib.sipg_multigrid_levels(self._h, None, None, 0))
        deg = (C.c_int32 * nl)()
        cells = (C.c_int32 * (3 * nl))()
        lib.sipg_multigrid_levels(self._h, deg, cells, nl)
        return [(deg[l], cells[3 * l], cells[3 * l + 1], cells[3 * l + 2]) for l in range(nl)]

    def multigrid_transfer(self, level: int, x, restrict: bool, out=None, stream=None):
        """restrict: P^T x from level to level+1; else out += P x from level+1 to level."""
        import torch
        if out is None:
            raise ValueError("pass the output vector (prolongation adds into it)")
        prec = self._prec(x)
        check(lib.sipg_multigrid_transfer(self._h, int(level), int(restrict), prec, C.c_void_p(x.data_ptr()),
                                          C.c_void_p(out.data_ptr()), C.c_void_p(_stream_handle(stream))))
        return out

    def workspace_bytes(self, with_solver: bool = True) -> int:
        b = C.c_size_t()
        check(lib.sipg_plan_workspace_bytes(self._h, int(with_solver), C.byref(b)))
        return int(b.value)

    def bind(self, with_solver: bool = True, stream=None, workspace=None, device="cuda"):
        import torch
        nbytes = self.workspace_bytes(with_solver)
        if workspace is None:
            workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        ptr = workspace.data_ptr()
        off = (-ptr) % 256
        check(lib.sipg_plan_bind(self._h, C.c_void_p(ptr + off), workspace.numel() - off, int(with_solver),
                                 C.c_void_p(_stream_handle(stream))))
        self.workspace = workspace
        self._with_solver = with_solver
        return self

    # ------------------------------------------------------------- operator
    @staticmethod
    def _prec(t) -> int:
        import torch
        if t.dtype == torch.float64:
            return F.F64
        if t.dtype == torch.float32:
            return F.F32
        raise TypeError(f"unsupported dtype {t.dtype}")

    def _check_vec(self, t):
        if not t.is_cuda or not t.is_contiguous() or t.numel() != self.ndof:
            raise ValueError(f"expected a contiguous device vector of {self.ndof} entries")

    def apply(self, x, y=None, parts: int = F.PART_ALL, stream=None):
        import torch
        self._check_vec(x)
        if y is None:
            y = torch.empty_like(x)
        self._check_vec(y)
        if y.dtype != x.dtype:
            raise TypeError("x and y must have the same dtype")
        check(lib.sipg_apply_parts(self._h, self._prec(x), parts, C.c_void_p(x.data_ptr()),
                                   C.c_void_p(y.data_ptr()), C.c_void_p(_stream_handle(stream))))
        return y

    def diagonal(self, dtype=None, inverse: bool = False, out=None, stream=None):
        import torch
        dtype = dtype or torch.float64
        if out is None:
            out = torch.empty(self.ndof, dtype=dtype, device="cuda")
        self._check_vec(out)
        check(lib.sipg_diagonal(self._h, self._prec(out), int(inverse), C.c_void_p(out.data_ptr()),
                                C.c_void_p(_stream_handle(stream))))
        return out

    def viscosity_values(self, stream=None):
        import torch
        mc = torch.empty(self.ncell * self.n ** 3, dtype=torch.float64, device="cuda")
        mf = torch.empty(self.nface * self.n ** 2, dtype=torch.float64, device="cuda")
        check(lib.sipg_viscosity_values(self._h, C.c_void_p(mc.data_ptr()), C.c_void_p(mf.data_ptr()),
                                        C.c_void_p(_stream_handle(stream))))
        return mc, mf

    # ------------------------------------------------------------- solve
    @staticmethod
    def _info(ci: F.SolveInfo) -> dict:
        return {"iterations": ci.iterations, "restarts": ci.restarts, "rel_residual": ci.rel_residual,
                "lambda_max": ci.lambda_max, "status": F.STATUS.get(ci.status, ci.status)}

    def solve(self, b, x=None, opts: SolveOptions | None = None, stream=None, raise_on_error=True):
        import torch
        self._check_vec(b)
        if b.dtype != torch.float64:
            raise TypeError("solve takes FP64 vectors")
        if x is None:
            x = torch.empty_like(b)
        o = (opts or SolveOptions()).to_c()
        info = F.SolveInfo()
        rc = lib.sipg_solve(self._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), C.byref(o),
                            C.byref(info), C.c_void_p(_stream_handle(stream)))
        if rc != 0 and (raise_on_error or rc not in (-4, -5)):
            check(rc)
        return x, self._info(info)

    # ------------------------------------------------------------- nonlinear viscous step
    def update_viscosity(self, u, stream=None):
        """Viscosity at every quadrature point (all multigrid levels) from the
        velocity u, then the diagonals; see sipg_update_viscosity."""
        import torch
        self._check_vec(u)
        if u.dtype != torch.float64:
            raise TypeError("update_viscosity takes an FP64 vector")
        check(lib.sipg_update_viscosity(self._h, C.c_void_p(u.data_ptr()), C.c_void_p(_stream_handle(stream))))

    def picard_work_bytes(self) -> int:
        return int(lib.sipg_picard_work_bytes(self._h))

    def picard_solve(self, b, x=None, opts: SolveOptions | None = None, rel_tol: float = 1e-8,
                     abs_tol: float = 0.0, max_iter: int = 50, aitken: bool = True, work=None, stream=None,
                     raise_on_error=True):
        """A(nu(x)) x = b by Picard iterations with Aitken relaxation; x holds
        the initial iterate (zero if None).  `opts` configures the linear
        solves (rel_tol relative to the current residual).  Returns (x, info)."""
        import torch
        self._check_vec(b)
        if b.dtype != torch.float64:
            raise TypeError("picard_solve takes FP64 vectors")
        nbytes = self.picard_work_bytes()
        if work is None:
            work = torch.empty(nbytes + 256, dtype=torch.uint8, device=b.device)
        ptr = work.data_ptr()
        off = (-ptr) % 256
        if work.numel() - off < nbytes:
            raise ValueError(f"work needs {nbytes} bytes after 256-byte alignment")
        return self._picard(b, x, opts, rel_tol, abs_tol, max_iter, aitken, ptr + off, stream, raise_on_error)

    def picard_solve_noalloc(self, b, x=None, opts: SolveOptions | None = None, rel_tol: float = 1e-8,
                             abs_tol: float = 0.0, max_iter: int = 50, aitken: bool = True, stream=None,
                             raise_on_error=True):
        """picard_solve with the work area in the library's static device
        array (sipg_picard_solve_noalloc: no device allocation by the call;
        at most PICARD_NOALLOC_MAX_DOF unknowns; calls overlapping on one
        GPU race)."""
        import torch
        self._check_vec(b)
        if b.dtype != torch.float64:
            raise TypeError("picard_solve_noalloc takes FP64 vectors")
        return self._picard(b, x, opts, rel_tol, abs_tol, max_iter, aitken, None, stream, raise_on_error)

    def _picard(self, b, x, opts, rel_tol, abs_tol, max_iter, aitken, work_ptr, stream, raise_on_error):
        import torch
        x = torch.zeros_like(b) if x is None else x
        self._check_vec(x)
        po = F.PicardOpts()
        po.rel_tol, po.abs_tol, po.max_iter, po.aitken = rel_tol, abs_tol, max_iter, int(aitken)
        lo = (opts or SolveOptions(rel_tol=1e-3)).to_c()
        info = F.PicardInfo()
        if work_ptr is None:
            rc = lib.sipg_picard_solve_noalloc(self._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                                               C.byref(lo), C.byref(po), C.byref(info),
                                               C.c_void_p(_stream_handle(stream)))
        else:
            rc = lib.sipg_picard_solve(self._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                                       C.c_void_p(work_ptr), C.byref(lo), C.byref(po), C.byref(info),
                                       C.c_void_p(_stream_handle(stream)))
        if rc != 0 and raise_on_error:
            check(rc)
        k = info.recorded
        return x, {"iterations": info.iterations, "linear_iterations": info.linear_iterations,
                   "residual_initial": info.residual_initial, "residual_final": info.residual_final,
                   "status": F.STATUS.get(info.status, info.status),
                   "residual_norms": list(info.residual_norms[:k]),
                   "omegas": list(info.omegas[:max(0, min(info.iterations, F.PICARD_HISTORY))])}

    def precondition(self, r, z=None, opts: SolveOptions | None = None, stream=None):
        """One application z = M r of the solve's preconditioner (FP64 vectors)."""
        import torch
        self._check_vec(r)
        if r.dtype != torch.float64:
            raise TypeError("precondition takes FP64 vectors")
        if z is None:
            z = torch.empty_like(r)
        o = (opts or SolveOptions()).to_c()
        check(lib.sipg_precondition(self._h, C.c_void_p(r.data_ptr()), C.c_void_p(z.data_ptr()), C.byref(o),
                                    C.c_void_p(_stream_handle(stream))))
        return z

    def solve_begin(self, b, x, opts: SolveOptions | None = None, stream=None):
        o = (opts or SolveOptions()).to_c()
        check(lib.sipg_solve_begin(self._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                                   C.byref(o), C.c_void_p(_stream_handle(stream))))

    def solve_advance(self, iters: int):
        check(lib.sipg_solve_advance(self._h, int(iters)))

    def solve_poll(self):
        done = C.c_int32()
        info = F.SolveInfo()
        check(lib.sipg_solve_poll(self._h, C.byref(done), C.byref(info)))
        return bool(done.value), (self._info(info) if done.value else None)
