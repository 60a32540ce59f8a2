"""SplitStep: the three plans of one dual-splitting time step (velocity
viscous step, pressure Poisson, penalty step) and the library's step
operators; see the dual-splitting section of include/sipg.h."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np

from . import _ffi as F
from ._ffi import check, lib
from .operator import Operator, SolveOptions, _stream_handle


@dataclass
class SplitOptions:
    # 10-step Lanczos estimates, as sipg_split_opts_default
    pressure: SolveOptions = field(default_factory=lambda: SolveOptions(rel_tol=1e-10, lanczos_steps=10))
    viscous: SolveOptions = field(default_factory=lambda: SolveOptions(rel_tol=1e-10, lanczos_steps=10))
    penalty: SolveOptions = field(default_factory=lambda: SolveOptions(rel_tol=1e-10, lanczos_steps=10))
    zeta: float = 1.0
    warm_start: bool = False         # viscous solve from uhh, penalty solve from u_visc

    def to_c(self) -> F.SplitOpts:
        o = F.SplitOpts()
        o.pressure, o.viscous, o.penalty = self.pressure.to_c(), self.viscous.to_c(), self.penalty.to_c()
        o.zeta = self.zeta
        o.warm_start = int(self.warm_start)
        return o


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


class SplitStep:
    """BDF order 1 or 2 (order 2: every step takes u_prev).  Velocity DG_k
    (viscous plan with alpha = gamma_0/dt and the Carreau law
    `law`), pressure DG_{k-1} (pure-Neumann Poisson) and the penalty step
    (alpha = 1, factors recomputed from the velocity) on one mesh whose six
    sides are walls: no-slip, or with the velocity data `g_wall` of the step
    calls (layout of include/sipg.h)."""

    def __init__(self, nx: int, ny: int, nz: int, degree: int, dt: float, law: dict, vertices=None,
                 penalty: float = 1.0, order: int = 1):
        if law.get("kind") != "carreau":
            raise ValueError("the splitting step takes a Carreau law (viscosity updated from the velocity)")
        if order not in (1, 2):
            raise ValueError("BDF order 1 or 2")
        self.dt, self.order = float(dt), order
        gamma0 = 1.0 if order == 1 else 1.5
        self.vel = Operator(nx, ny, nz, degree, "viscous", gamma0 / dt, penalty, law, vertices, ("D",) * 6)
        self.pres = Operator(nx, ny, nz, degree - 1, "poisson", 0.0, penalty, None, vertices, ("N",) * 6)
        zero = np.zeros(nx * ny * nz)
        self.pen = Operator(nx, ny, nz, degree, "penalty", 1.0, 1.0, None, vertices, ("D",) * 6, zero, zero)
        self.ndof_u, self.ndof_p = self.vel.ndof, self.pres.ndof
        self._work = None

    def set_multigrid(self, penalty: bool = False, **kw) -> "SplitStep":
        """hp-multigrid for the viscous and pressure solves and, with
        penalty=True, for the penalty step (its levels' factors follow every
        update)."""
        self.vel.set_multigrid(**kw)
        self.pres.set_multigrid(**kw)
        if penalty:
            self.pen.set_multigrid(**kw)
        return self

    def bind(self, stream=None) -> "SplitStep":
        for op in (self.vel, self.pres, self.pen):
            op.bind(with_solver=True, stream=stream)
        return self

    def _vec(self, t, n, name):
        import torch
        if t is None or not t.is_cuda or not t.is_contiguous() or t.numel() != n or t.dtype != torch.float64:
            raise ValueError(f"{name}: expected a contiguous FP64 device vector of {n} entries")

    def wall_count(self) -> int:
        """Rows of the wall data: one per boundary face (see include/sipg.h)."""
        v = self.vel
        return 2 * (v.ny * v.nz + v.nx * v.nz + v.nx * v.ny)

    def _wall(self, g):
        if g is not None:
            self._vec(g, self.wall_count() * self.vel.n ** 2 * 3, "g_wall")

    def _prev(self, u_prev):
        if (u_prev is None) != (self.order == 1):
            raise ValueError("u_prev (the velocity before u) is needed for BDF2 and only there")
        if u_prev is not None:
            self._vec(u_prev, self.ndof_u, "u_prev")

    def convective_step(self, u, b=None, uhat=None, g_wall=None, u_prev=None, stream=None):
        import torch
        self._vec(u, self.ndof_u, "u")
        self._prev(u_prev)
        if b is not None:
            self._vec(b, self.ndof_u, "b")
        self._wall(g_wall)
        uhat = torch.empty_like(u) if uhat is None else uhat
        check(lib.sipg_convective_step(self.vel._h, _ptr(u), _ptr(u_prev), _ptr(b), _ptr(g_wall), self.dt,
                                       _ptr(uhat), C.c_void_p(_stream_handle(stream))))
        return uhat

    def pressure_rhs(self, uhat, u_old, b=None, f=None, g_wall=None, u_prev=None, stream=None):
        import torch
        self._vec(uhat, self.ndof_u, "uhat")
        self._vec(u_old, self.ndof_u, "u_old")
        self._prev(u_prev)
        self._wall(g_wall)
        f = torch.empty(self.ndof_p, dtype=torch.float64, device=uhat.device) if f is None else f
        check(lib.sipg_pressure_rhs(self.vel._h, self.pres._h, _ptr(uhat), _ptr(u_old), _ptr(u_prev), _ptr(b),
                                    _ptr(g_wall), self.dt, _ptr(f), C.c_void_p(_stream_handle(stream))))
        return f

    def wall_load(self, op: Operator, g_wall, y, stream=None):
        """y += the load of the wall data for the viscous (self.vel) or
        penalty (self.pen) plan."""
        self._wall(g_wall)
        self._vec(y, self.ndof_u, "y")
        check(lib.sipg_wall_load(op._h, _ptr(g_wall), _ptr(y), C.c_void_p(_stream_handle(stream))))
        return y

    def projection(self, uhat, p, stream=None):
        import torch
        self._vec(uhat, self.ndof_u, "uhat")
        self._vec(p, self.ndof_p, "p")
        uhh, rhs = torch.empty_like(uhat), torch.empty_like(uhat)
        check(lib.sipg_projection(self.vel._h, self.pres._h, _ptr(uhat), _ptr(p), self.order, self.dt, _ptr(uhh),
                                  _ptr(rhs), C.c_void_p(_stream_handle(stream))))
        return uhh, rhs

    def update_penalty_factors(self, u, zeta: float = 1.0, stream=None):
        self._vec(u, self.ndof_u, "u")
        check(lib.sipg_update_penalty_factors(self.pen._h, _ptr(u), self.dt, float(zeta),
                                              C.c_void_p(_stream_handle(stream))))

    def work_bytes(self) -> int:
        return int(lib.sipg_split_work_bytes(self.vel._h, self.pres._h))

    def step(self, u_old, b=None, u_new=None, p=None, opts: SplitOptions | None = None, g_wall=None, u_prev=None,
             stream=None):
        """One step (BDF1, or BDF2 with u_prev = u^{n-1}); returns (u_new, p, info)."""
        import torch
        self._vec(u_old, self.ndof_u, "u_old")
        self._prev(u_prev)
        self._wall(g_wall)
        u_new = torch.empty_like(u_old) if u_new is None else u_new
        p = torch.empty(self.ndof_p, dtype=torch.float64, device=u_old.device) if p is None else p
        nbytes = self.work_bytes()
        if self._work is None or self._work.numel() < nbytes + 256:
            self._work = torch.empty(nbytes + 256, dtype=torch.uint8, device=u_old.device)
        ptr = self._work.data_ptr()
        off = (-ptr) % 256
        o = (opts or SplitOptions()).to_c()
        info = F.SplitInfo()
        check(lib.sipg_split_step(self.vel._h, self.pres._h, self.pen._h, _ptr(u_old), _ptr(u_prev), _ptr(b),
                                  _ptr(g_wall), self.dt,
                                  _ptr(u_new), _ptr(p), C.c_void_p(ptr + off), C.byref(o), C.byref(info),
                                  C.c_void_p(_stream_handle(stream))))
        return u_new, p, {k: Operator._info(getattr(info, k)) for k in ("pressure", "viscous", "penalty")}
