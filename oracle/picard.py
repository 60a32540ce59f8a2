"""Picard update of the viscosity from the velocity and the relaxed
fixed-point iteration of the nonlinear viscous step.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 4.1 (paragraph "Viscous Step", eq. viscosity_pointwise) updates the
apparent viscosity pointwise from the last velocity iterate,
nu^{k+1} = eta(gdot(grad^S u^k)), with gdot = sqrt(2 eps:eps) and eta the
generalised Newtonian law of Sec. 2; Sec. 5.1 (projection solver, Alg. 1)
repeats viscosity update and linear viscous solve until the residual of the
nonlinear viscous step has dropped by eps_rel or below eps_abs, and
accelerates the fixed-point iteration by Aitken's adaptive relaxation
(Irons and Tuck 1969), computing the relaxation factor from the full
nonlinear residual rather than from the increment.  Readings taken here:

* the velocity's shear rate at a cell point is that of the DG function in
  the cell; at a face point it is that of the mean of the two traces'
  symmetric gradients (interior faces) or of the interior trace (boundary
  faces), so one value per face point as for the prescribed laws;
* multigrid levels evaluate the shear rate of the finest velocity at their
  own quadrature points: a point of a coarse cell lies in the fine cell
  (2^L e + floor(2^L xi)) at the fine reference point frac(2^L xi) per
  direction (L mesh steps; degree steps keep the cell), with the traces of
  the fine cells on either side of a coarse face;
* residual R(u) = b - A(mu(u)) u with the viscosity updated from u; the
  linear step solves A(mu(u_k)) delta = R(u_k) and sets
  u_{k+1} = u_k + omega_k delta, omega_0 = 1,
  omega_k = -omega_{k-1} R_{k-1}.(R_k - R_{k-1}) / |R_k - R_{k-1}|^2;
* the iteration stops as soon as either criterion holds (the text says
  "or"; the listing's loop condition would need both).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .basis import cell_points, face_points, tensor_tables
from .forms import Problem, apply as op_apply
from .laws import generalized_newtonian


def _jacobian_at(mesh, cells, pts):
    """J[p, i, d] = d x_i / d xi_d of cell cells[p] at reference point pts[p]."""
    X = mesh.corners(cells)                       # (P, 2, 2, 2, 3)
    _, G = mesh._shape(pts)                       # (P, 2, 2, 2, 3)
    return np.einsum("pabcd,pabci->pid", G, X)


def velocity_gradient(fine: Problem, u, cells, pts):
    """Physical gradient grad u [p, c, i] = d u_c / d x_i of the fine DG
    velocity u in cell cells[p] at reference point pts[p]."""
    n, C = fine.n, fine.C
    U = np.asarray(u, dtype=np.float64).reshape(fine.mesh.ncells, C, n ** 3)
    _, G = tensor_tables(n, pts)                  # (P, n^3, 3)
    gref = np.einsum("pcj,pjd->pcd", U[cells], G)
    Jinv = np.linalg.inv(_jacobian_at(fine.mesh, cells, pts))    # [p, d, i] = d xi_d / d x_i
    return np.einsum("pcd,pdi->pci", gref, Jinv)


def _shear_rate(grad):
    eps = 0.5 * (grad + np.swapaxes(grad, -1, -2))
    return np.sqrt(2.0 * np.einsum("...ij,...ij->...", eps, eps))


def _ratio(level: Problem, fine: Problem) -> int:
    r = fine.mesh.nx // level.mesh.nx
    assert (level.mesh.nx * r, level.mesh.ny * r, level.mesh.nz * r) == (fine.mesh.nx, fine.mesh.ny, fine.mesh.nz)
    assert r & (r - 1) == 0
    return r


def _locate(level: Problem, fine: Problem, cells, pts, d=None, side=None):
    """Fine cell and fine reference point of each (level cell, level point)
    pair; for face points (d, side) the fine cell touching that face."""
    r = _ratio(level, fine)
    ex, ey, ez = level.mesh.cell_ijk(cells)
    E, P = len(cells), len(pts)
    t = r * np.broadcast_to(pts, (E, P, 3))
    k = np.floor(t).astype(np.int64)
    k = np.minimum(k, r - 1)                      # xi = 1 on a face: last fine cell, fine xi = 1
    xi = t - k
    if d is not None:
        k[..., d] = 0 if side == 0 else r - 1
        xi[..., d] = float(side)
    fx = r * ex[:, None] + k[..., 0]
    fy = r * ey[:, None] + k[..., 1]
    fz = r * ez[:, None] + k[..., 2]
    fcell = (fz * fine.mesh.ny + fy) * fine.mesh.nx + fx
    return fcell.reshape(-1), xi.reshape(-1, 3)


def shear_rate_values(level: Problem, fine: Problem, u, cells=None, faces=None):
    """(gdot at level cell points [ncells, n^3], gdot at level face points
    [nfaces, n^2], faces numbered by Mesh.face_index) of the fine velocity u.
    With `cells` / `faces` given only those rows are evaluated (the cell rows
    in the order given; face rows not asked for are NaN)."""
    m, n = level.mesh, level.n
    cells = np.arange(m.ncells) if cells is None else np.asarray(cells)
    want = None if faces is None else np.zeros(m.nfaces, dtype=bool)
    if want is not None:
        want[np.asarray(faces)] = True
    pts, _ = cell_points(n)
    fc, xi = _locate(level, fine, cells, pts)
    gd_cell = _shear_rate(velocity_gradient(fine, u, fc, xi)).reshape(len(cells), n ** 3)
    gd_face = np.zeros((m.nfaces, n * n)) if want is None else np.full((m.nfaces, n * n), np.nan)
    for d in range(3):
        fpts, _ = face_points(n, d, 1)
        fpts0, _ = face_points(n, d, 0)
        em, ep = m.interior_faces(d)
        if want is not None:
            keep = want[m.face_index(d, em, 1)]
            em, ep = em[keep], ep[keep]
        if len(em):
            fm, xm = _locate(level, fine, em, fpts, d, 1)
            fp, xp = _locate(level, fine, ep, fpts0, d, 0)
            gm = velocity_gradient(fine, u, fm, xm)
            gp = velocity_gradient(fine, u, fp, xp)
            gd_face[m.face_index(d, em, 1)] = _shear_rate(0.5 * (gm + gp)).reshape(len(em), n * n)
        for side in (0, 1):
            bc = m.boundary_cells(d, side)
            if want is not None:
                bc = bc[want[m.face_index(d, bc, side)]]
            if len(bc) == 0:
                continue
            sp, _ = face_points(n, d, side)
            fb, xb = _locate(level, fine, bc, sp, d, side)
            gd_face[m.face_index(d, bc, side)] = _shear_rate(velocity_gradient(fine, u, fb, xb)).reshape(
                len(bc), n * n)
    return gd_cell, gd_face


def viscosity_values(level: Problem, fine: Problem, u, law: dict):
    """eta(gdot) at the level's cell and face points (Sec. 4.1,
    eq. viscosity_pointwise) for the generalised Newtonian law's
    parameters in `law` (its prescribed velocity modes are not used)."""
    gc, gf = shear_rate_values(level, fine, u)
    return generalized_newtonian(law, gc), generalized_newtonian(law, gf)


def with_velocity_viscosity(level: Problem, fine: Problem, u, law: dict) -> Problem:
    """The level's operator with the viscosity updated from the fine velocity."""
    return dataclasses.replace(level, mu_values=viscosity_values(level, fine, u, law))


def aitken_omega(omega_prev: float, R_prev, R) -> float:
    """Adaptive relaxation factor from two consecutive residuals."""
    dR = R - R_prev
    den = float(dR @ dR)
    if den == 0.0:
        return omega_prev
    return -omega_prev * float(R_prev @ dR) / den


def relaxed_fixed_point(residual, solve, u0, rel_tol: float, abs_tol: float, max_iter: int,
                        aitken: bool = True):
    """u_{k+1} = u_k + omega_k solve(u_k, R(u_k)) until |R| <= rel_tol |R_0|
    or |R| <= abs_tol.  `residual(u)` returns R(u) (updating whatever the
    operator depends on), `solve(u, R)` the correction.  Returns
    (u, info) with the residual norms and relaxation factors."""
    u = np.array(u0, dtype=np.float64, copy=True)
    R = residual(u)
    r0 = float(np.linalg.norm(R))
    norms, omegas = [r0], []
    omega, R_prev = 1.0, None
    status = "not_converged"
    k = 0
    while True:
        rn = norms[-1]
        if rn <= rel_tol * r0 or rn <= abs_tol:
            status = "ok"
            break
        if k >= max_iter:
            break
        if aitken and R_prev is not None:
            omega = aitken_omega(omega, R_prev, R)
        delta = solve(u, R)
        u = u + omega * delta
        omegas.append(omega)
        R_prev, R = R, residual(u)
        norms.append(float(np.linalg.norm(R)))
        k += 1
    return u, {"iterations": k, "residual_norms": norms, "omegas": omegas, "status": status}


def picard_solve(pb: Problem, law: dict, b, u0, linear_solve, rel_tol: float = 1e-8,
                 abs_tol: float = 0.0, max_iter: int = 50, aitken: bool = True):
    """The nonlinear viscous step A(mu(u)) u = b by Picard iterations with
    Aitken relaxation.  linear_solve(pb_k, R) returns the correction for the
    operator pb_k whose viscosity was updated from the current iterate."""
    state = {}

    def residual(u):
        state["pb"] = with_velocity_viscosity(pb, pb, u, law)
        return b - op_apply(state["pb"], u)

    def solve(u, R):
        return linear_solve(state["pb"], R)

    return relaxed_fixed_point(residual, solve, u0, rel_tol, abs_tol, max_iter, aitken)
