"""One time step of the dual splitting scheme -- test infrastructure.

Follows Sec. 3 ("Splitting Scheme": eqs. convective_step, projection_step,
pressure_step, pressure_Neumann_BC, viscous_step_with_convection), the weak
forms of Sec. 4.1 (eqs. convective_step_weak, convective_term_weak,
pressure_step_weak, guhat_consistent_BC, projection_step_weak, the viscous
step) and the order of Alg. 1 (Sec. 5.1): convective step, pressure step,
velocity projection, viscous step, divergence and continuity penalty step.
Only tests, the package's smoke check and the benchmark's CPU baseline use
this module.

Scope and readings taken here:
  * BDF1 (m = 1: gamma_0 = alpha_0 = beta_0 = 1; m_p = min(m - 1, 2) = 0, so
    h_p has no extrapolated convective or viscous terms) or, given u^{n-1},
    BDF2 with a constant step (m = 2: gamma_0 = 3/2, alpha = (2, -1/2),
    beta = (2, -1); m_p = 1, beta_bar = (1), u^dd = u^n);
  * the vorticity omega = curl u^dd is the element-local L2 projection onto
    DG_k (Alg. 1), and nu^dd = eta(gdot(grad^S u^dd)) enters h_p with its
    value at the wall point (interior trace) and the gradient of its
    element-local L2 projection onto DG_k (the paper does not say how its
    gradient is formed);
  * every boundary is a wall with velocity Dirichlet data g_u constant in
    time (d_t g_u = 0; g_u = 0 for no-slip, a moving lid otherwise), given
    at the velocity's face quadrature points of the boundary faces (layout of
    ``wall_rows``), pressure Neumann with h_p of eq. pressure_Neumann_BC; the
    pressure level is fixed by removing the mean of the right-hand side and
    taking the solution of zero nodal mean;
  * the body force b is given as nodal values of DG_k (constant in time);
  * the pressure space is DG_{k-1} on the same mesh (nodal at its own k
    Gauss points); every integral of the mixed forms (pressure right-hand
    side, projection) uses the velocity's (k+1)-point Gauss rule;
  * the convective term is (w . grad) u (the paper's notation) with the
    upwind flux u_dag = {u} + sign({w}.n) [u]_oriented / 2 and the mirror
    principle on the walls (u+ = 2 g_u - u-, w+ likewise);
  * the data enter the viscous step's right-hand side through the mirror
    principle of the SIPG form (the load of ``forms.load_vector``) and the
    penalty step's through its oriented jump u - g_u on the walls;
  * [c(u, u)]^# in g_uhat on the walls is evaluated from the interior trace
    of u^n and of its gradient;
  * viscosity linear implicit, nu^# = eta(gdot(grad^S u^#)) with the
    extrapolation u^# = sum_i beta_i u^{n-i} (Alg. 1 leaves the loop after
    one pass in this case); the penalty factors use u^# as well;
  * penalty step factors (Fehn et al. 2018, restated in the penalty-step
    reading of this package): |u_e| = volume mean of |u^#| over the cell,
    h_e = |cell|^(1/3), tau_div = zeta |u_e| h_e dt / (k + 1),
    tau_cont = zeta |u_e| dt.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import picard as PC
from .basis import cell_points, face_points, tensor_tables
from .laws import generalized_newtonian
from .forms import (Problem, _cell_geo, _face_geo, _mu_face, _phys_grad, _sym, _tau, _tau_face, _test_project,
                    assemble, cell_sizes, penalty_geometry)
from .mesh import Mesh

# BDF1 coefficients (m = 1)
GAMMA0, ALPHA0, BETA0 = 1.0, 1.0, 1.0


def bdf(order: int) -> dict:
    """gamma_0, alpha_i, beta_i (extrapolation of order m) and beta_bar_i
    (extrapolation of order m_p = min(m - 1, 2)) for a constant step."""
    if order == 1:
        return {"gamma0": 1.0, "alpha": (1.0,), "beta": (1.0,), "beta_bar": ()}
    if order == 2:
        return {"gamma0": 1.5, "alpha": (2.0, -0.5), "beta": (2.0, -1.0), "beta_bar": (1.0,)}
    raise ValueError("BDF order 1 or 2")


def pressure_problem(mesh: Mesh, degree_u: int) -> Problem:
    """The pressure Poisson problem: DG_{k-1}, Neumann on every wall."""
    return Problem(Mesh(mesh.nx, mesh.ny, mesh.nz, mesh.vertices.reshape(-1, 3), ("N",) * 6), degree_u - 1,
                   "poisson", 0.0, 1.0)


def _walls(pb: Problem):
    if any(b != "D" for b in pb.mesh.bc):
        raise ValueError("the splitting step is defined here for no-slip walls on every side")


def wall_rows(mesh: Mesh) -> dict:
    """Rows of the wall-data array per wall (d, side): sides in the order
    -x, +x, -y, +y, -z, +z, each side's faces in the order of
    ``mesh.boundary_cells(d, side)``; each row holds the n^2 face points
    (index b n + a, a along the lower tangential axis) times 3 components."""
    sizes = (mesh.ny * mesh.nz, mesh.nx * mesh.nz, mesh.nx * mesh.ny)
    out, off = {}, 0
    for d in range(3):
        for side in (0, 1):
            out[(d, side)] = slice(off, off + sizes[d])
            off += sizes[d]
    return out


def wall_count(mesh: Mesh) -> int:
    return 2 * (mesh.ny * mesh.nz + mesh.nx * mesh.nz + mesh.nx * mesh.ny)


def _wall_g(pb: Problem, g_wall, d: int, side: int) -> np.ndarray:
    """g_u at the face points of wall (d, side): (cells, n^2, 3)."""
    rows = wall_rows(pb.mesh)[(d, side)]
    if g_wall is None:
        return np.zeros((rows.stop - rows.start, pb.n ** 2, 3))
    return np.asarray(g_wall, dtype=np.float64).reshape(wall_count(pb.mesh), pb.n ** 2, 3)[rows]


def _values(pb: Problem, X, V):
    """X (E, C, n^3) at points with tables V (P, n^3) -> (E, P, C)."""
    return np.einsum("pj,ecj->epc", V, X)


# ---------------------------------------------------------------------------
# mass matrix (per cell; nodal basis at the quadrature points)
# ---------------------------------------------------------------------------

def mass_apply(pb: Problem, x) -> np.ndarray:
    """M x with M_IJ = (phi_I, phi_J) on the n-point Gauss rule."""
    n, C = pb.n, pb.C
    X = np.asarray(x, dtype=np.float64).reshape(pb.mesh.ncells, C, n ** 3)
    pts, _ = cell_points(n)
    V, G = tensor_tables(n, pts)
    cells = np.arange(pb.mesh.ncells)
    _, Jinv, JxW = _cell_geo(pb, cells)
    Y = _test_project(V, G, Jinv, _values(pb, X, V), np.zeros((len(cells), len(pts), C, 3)), JxW)
    return Y.reshape(-1)


def mass_solve(pb: Problem, y) -> np.ndarray:
    """M^-1 y, cell by cell (the mass matrix is block diagonal in DG)."""
    n, C = pb.n, pb.C
    Y = np.asarray(y, dtype=np.float64).reshape(pb.mesh.ncells, C, n ** 3)
    pts, _ = cell_points(n)
    V, _ = tensor_tables(n, pts)
    _, _, JxW = _cell_geo(pb, np.arange(pb.mesh.ncells))
    M = np.einsum("pi,ep,pj->eij", V, JxW, V)                      # (E, n^3, n^3), one per component
    return np.linalg.solve(M[:, None], Y[..., None])[..., 0].reshape(-1)


# ---------------------------------------------------------------------------
# convective term (eq. convective_term_weak)
# ---------------------------------------------------------------------------

def _upwind_face(um, up, wm, wp, nrm):
    """(({w}.n)(u_dag - u-)) on the "-" side of a face with normal nrm out of "-"."""
    wn = 0.5 * np.einsum("epc,epc->ep", wm + wp, nrm)
    udag = 0.5 * (um + up) + 0.5 * np.sign(wn)[..., None] * (um - up)
    return wn[..., None] * (udag - um)


def convective_form(pb: Problem, u, w, g_wall=None) -> np.ndarray:
    """c_h(phi_I, u; w) summed over the cells, for every test function:
    (v, (w . grad) u)_e - (v, ({w}.n) u)_de + (v, ({w}.n) u_dag)_de; on the
    walls u+ = 2 g_u - u-, w+ = 2 g_u - w-."""
    _walls(pb)
    mesh, n = pb.mesh, pb.n
    U = np.asarray(u, dtype=np.float64).reshape(mesh.ncells, 3, n ** 3)
    W = np.asarray(w, dtype=np.float64).reshape(mesh.ncells, 3, n ** 3)
    Y = np.zeros_like(U)
    cells = np.arange(mesh.ncells)
    pts, _ = cell_points(n)
    V, G = tensor_tables(n, pts)
    _, Jinv, JxW = _cell_geo(pb, cells)
    gu = _phys_grad(U, G, Jinv)                                    # d u_c / d x_i
    a = np.einsum("epci,epi->epc", gu, _values(pb, W, V))         # (w . grad) u
    Y += _test_project(V, G, Jinv, a, np.zeros(a.shape + (3,)), JxW)
    zero = None
    for d in range(3):
        em, ep = mesh.interior_faces(d)
        if len(em):
            Vm, Gm = tensor_tables(n, face_points(n, d, 1)[0])
            Vp, Gp = tensor_tables(n, face_points(n, d, 0)[0])
            _, _, Jim, nrm, ds = _face_geo(pb, em, d, 1)
            _, _, Jip, _, _ = _face_geo(pb, ep, d, 0)
            um, up = _values(pb, U[em], Vm), _values(pb, U[ep], Vp)
            wm, wp = _values(pb, W[em], Vm), _values(pb, W[ep], Vp)
            zero = np.zeros(um.shape + (3,))
            Y[em] += _test_project(Vm, Gm, Jim, _upwind_face(um, up, wm, wp, nrm), zero, ds)
            Y[ep] += _test_project(Vp, Gp, Jip, _upwind_face(up, um, wp, wm, -nrm), zero, ds)
        for side in (0, 1):                                        # walls: mirror principle
            bc = mesh.boundary_cells(d, side)
            Vf, Gf = tensor_tables(n, face_points(n, d, side)[0])
            _, _, Ji, nrm, ds = _face_geo(pb, bc, d, side)
            ui, wi = _values(pb, U[bc], Vf), _values(pb, W[bc], Vf)
            g = _wall_g(pb, g_wall, d, side)
            Y[bc] += _test_project(Vf, Gf, Ji, _upwind_face(ui, 2 * g - ui, wi, 2 * g - wi, nrm),
                                   np.zeros(ui.shape + (3,)), ds)
    return Y.reshape(-1)


def convective_step(pb: Problem, u, b, dt: float, g_wall=None, u_prev=None) -> np.ndarray:
    """uhat from eq. convective_step_weak:
    (gamma_0/dt)(v, uhat) = (v, b) + sum_i (alpha_i/dt)(v, u^{n-i}) - sum_i beta_i c_h(v, u^{n-i}; u^{n-i})
    (BDF1, or BDF2 with u_prev = u^{n-1})."""
    olds = [np.asarray(u, dtype=np.float64)] + ([] if u_prev is None else [np.asarray(u_prev, dtype=np.float64)])
    c = bdf(len(olds))
    rhs = mass_apply(pb, b)
    for a_i, b_i, ui in zip(c["alpha"], c["beta"], olds):
        rhs = rhs + a_i / dt * mass_apply(pb, ui) - b_i * convective_form(pb, ui, ui, g_wall)
    return dt / c["gamma0"] * mass_solve(pb, rhs)


def _curl(G):
    """curl from G[..., c, i] = d u_c / d x_i."""
    return np.stack([G[..., 2, 1] - G[..., 1, 2], G[..., 0, 2] - G[..., 2, 0], G[..., 1, 0] - G[..., 0, 1]], -1)


def l2_project(pb: Problem, values) -> np.ndarray:
    """Element-local L2 projection onto DG_k of values (cells, P, C) at the
    cell quadrature points: per cell M_e x = (phi_j, values)_e; (cells, C, n^3)."""
    n = pb.n
    pts, _ = cell_points(n)
    V, _ = tensor_tables(n, pts)
    _, _, JxW = _cell_geo(pb, np.arange(pb.mesh.ncells))
    rhs = np.einsum("pj,ep,epc->ecj", V, JxW, values)
    M = np.einsum("pi,ep,pj->eij", V, JxW, V)
    return np.linalg.solve(M[:, None], rhs[..., None])[..., 0]


def vorticity(pb: Problem, u) -> np.ndarray:
    """omega_h = element-local L2 projection of curl u onto DG_k (Alg. 1)."""
    n = pb.n
    U = np.asarray(u, dtype=np.float64).reshape(pb.mesh.ncells, 3, n ** 3)
    pts, _ = cell_points(n)
    _, G = tensor_tables(n, pts)
    _, Jinv, _ = _cell_geo(pb, np.arange(pb.mesh.ncells))
    return l2_project(pb, _curl(_phys_grad(U, G, Jinv)))


def viscosity_projection(pb: Problem, u, law: dict) -> np.ndarray:
    """eta(gdot(grad^S u)) at the cell points, projected element-locally onto DG_k."""
    n = pb.n
    U = np.asarray(u, dtype=np.float64).reshape(pb.mesh.ncells, 3, n ** 3)
    pts, _ = cell_points(n)
    _, G = tensor_tables(n, pts)
    _, Jinv, _ = _cell_geo(pb, np.arange(pb.mesh.ncells))
    nu = generalized_newtonian(law, PC._shear_rate(_phys_grad(U, G, Jinv)))
    return l2_project(pb, nu[..., None])


# ---------------------------------------------------------------------------
# pressure step (eqs. pressure_step_weak, guhat_consistent_BC, pressure_Neumann_BC)
# ---------------------------------------------------------------------------

def wall_data(pb: Problem, u_old, b, dt: float, d: int, side: int, g_wall=None, u_prev=None, law=None):
    """On the wall xi_d = side: g_uhat and h_p at the face points of the
    boundary cells, with the velocities and b taken from the interior traces.
    g_uhat = (dt/gamma_0) (b - sum_i beta_i (grad u^{n-i}) u^{n-i}) + sum_i (alpha_i/gamma_0) g_u,
    h_p = n.b - n.d_t g_u - sum_{i<m_p} beta_bar_i n.((grad u^{n-i}) u^{n-i})
          - nu^dd n.curl(omega^dd) + 2 n.(grad^S u^dd . grad nu^dd)   (the last two for m_p >= 1),
    u^dd = sum_{i<m_p} beta_bar_i u^{n-i}."""
    n = pb.n
    olds = [u_old] + ([] if u_prev is None else [u_prev])
    c = bdf(len(olds))
    Us = [np.asarray(v, dtype=np.float64).reshape(pb.mesh.ncells, 3, n ** 3) for v in olds]
    B = np.asarray(b, dtype=np.float64).reshape(pb.mesh.ncells, 3, n ** 3)
    bc = pb.mesh.boundary_cells(d, side)
    Vf, Gf = tensor_tables(n, face_points(n, d, side)[0])
    _, _, Ji, nrm, ds = _face_geo(pb, bc, d, side)
    bi = _values(pb, B[bc], Vf)
    convs = [np.einsum("epci,epi->epc", _phys_grad(U[bc], Gf, Ji), _values(pb, U[bc], Vf)) for U in Us]
    g_u = _wall_g(pb, g_wall, d, side)
    dt_g_u = np.zeros_like(bi)                                   # data constant in time
    g_uhat = dt / c["gamma0"] * (bi - sum(b_i * cv for b_i, cv in zip(c["beta"], convs))) \
        + sum(c["alpha"]) / c["gamma0"] * g_u
    h_p = np.einsum("epc,epc->ep", nrm, bi) - np.einsum("epc,epc->ep", nrm, dt_g_u)
    for bb_i, cv in zip(c["beta_bar"], convs):
        h_p = h_p - bb_i * np.einsum("epc,epc->ep", nrm, cv)
    if c["beta_bar"]:
        if law is None:
            raise ValueError("BDF2 wall data need the viscosity law")
        udd = sum(bb_i * v for bb_i, v in zip(c["beta_bar"], olds))
        Udd = np.asarray(udd, dtype=np.float64).reshape(pb.mesh.ncells, 3, n ** 3)
        gu = _phys_grad(Udd[bc], Gf, Ji)                           # grad u^dd at the wall points
        nu = generalized_newtonian(law, PC._shear_rate(gu))
        curl_om = _curl(_phys_grad(vorticity(pb, udd)[bc], Gf, Ji))
        grad_nu = _phys_grad(viscosity_projection(pb, udd, law)[bc], Gf, Ji)[..., 0, :]
        S = 0.5 * (gu + np.swapaxes(gu, -1, -2))
        h_p = h_p - nu * np.einsum("epc,epc->ep", nrm, curl_om) \
            + 2.0 * np.einsum("epi,epij,epj->ep", nrm, S, grad_nu)
    return bc, g_uhat, h_p


def divergence_form(pb_u: Problem, pb_p: Problem, uhat, wall_value) -> np.ndarray:
    """sum_e (grad q, uhat)_e - (q, {uhat}.n)_de for every pressure test
    function q, on the velocity's quadrature; {uhat} on a wall is
    wall_value(d, side) (E_b, P, 3)."""
    mesh, n, npr = pb_u.mesh, pb_u.n, pb_p.n
    U = np.asarray(uhat, dtype=np.float64).reshape(mesh.ncells, 3, n ** 3)
    F = np.zeros((mesh.ncells, 1, npr ** 3))
    cells = np.arange(mesh.ncells)
    pts, _ = cell_points(n)
    Vu, _ = tensor_tables(n, pts)
    Vq, Gq = tensor_tables(npr, pts)
    _, Jinv, JxW = _cell_geo(pb_u, cells)
    B = _values(pb_u, U, Vu)[:, :, None, :]                       # (E, P, 1, 3)
    F += _test_project(Vq, Gq, Jinv, np.zeros(B.shape[:3]), B, JxW)
    for d in range(3):
        em, ep = mesh.interior_faces(d)
        if len(em):
            ptm, ptp = face_points(n, d, 1)[0], face_points(n, d, 0)[0]
            Vum, _ = tensor_tables(n, ptm)
            Vup, _ = tensor_tables(n, ptp)
            Vqm, Gqm = tensor_tables(npr, ptm)
            Vqp, Gqp = tensor_tables(npr, ptp)
            _, _, Jim, nrm, ds = _face_geo(pb_u, em, d, 1)
            _, _, Jip, _, _ = _face_geo(pb_u, ep, d, 0)
            avg = 0.5 * (_values(pb_u, U[em], Vum) + _values(pb_u, U[ep], Vup))
            an = np.einsum("epc,epc->ep", avg, nrm)[..., None]
            zero = np.zeros(an.shape + (3,))
            F[em] += _test_project(Vqm, Gqm, Jim, -an, zero, ds)
            F[ep] += _test_project(Vqp, Gqp, Jip, an, zero, ds)
        for side in (0, 1):
            bc = mesh.boundary_cells(d, side)
            pt = face_points(n, d, side)[0]
            Vqf, Gqf = tensor_tables(npr, pt)
            _, _, Ji, nrm, ds = _face_geo(pb_u, bc, d, side)
            an = np.einsum("epc,epc->ep", wall_value(d, side), nrm)[..., None]
            F[bc] += _test_project(Vqf, Gqf, Ji, -an, np.zeros(an.shape + (3,)), ds)
    return F.reshape(-1)


def wall_neumann_form(pb_u: Problem, pb_p: Problem, h_value) -> np.ndarray:
    """(q, h_p) on the walls for every pressure test function."""
    mesh, n, npr = pb_u.mesh, pb_u.n, pb_p.n
    F = np.zeros((mesh.ncells, 1, npr ** 3))
    for d in range(3):
        for side in (0, 1):
            bc = mesh.boundary_cells(d, side)
            Vqf, Gqf = tensor_tables(npr, face_points(n, d, side)[0])
            _, _, Ji, _, ds = _face_geo(pb_u, bc, d, side)
            h = h_value(d, side)[..., None]
            F[bc] += _test_project(Vqf, Gqf, Ji, h, np.zeros(h.shape + (3,)), ds)
    return F.reshape(-1)


def ppe_rhs(pb_u: Problem, pb_p: Problem, uhat, u_old, b, dt: float, g_wall=None, u_prev=None,
            law=None) -> np.ndarray:
    """Right-hand side of eq. pressure_step_weak with the wall data moved
    over: (gamma_0/dt) [(grad q, uhat) - (q, {uhat}.n)] + (q, h_p)_walls,
    {uhat} = g_uhat on the walls (mirror principle)."""
    _walls(pb_u)
    g0 = bdf(1 if u_prev is None else 2)["gamma0"]
    data = {(d, s): wall_data(pb_u, u_old, b, dt, d, s, g_wall, u_prev, law) for d in range(3) for s in (0, 1)}
    div = divergence_form(pb_u, pb_p, uhat, lambda d, s: data[(d, s)][1])
    return g0 / dt * div + wall_neumann_form(pb_u, pb_p, lambda d, s: data[(d, s)][2])


def pressure_solve(pb_p: Problem, f) -> np.ndarray:
    """Pure-Neumann SIPG Poisson solve: the right-hand side's mean removed,
    the solution of zero nodal mean (a direct sparse solve of the bordered
    system)."""
    A = assemble(pb_p).tocsr()
    N = A.shape[0]
    f0 = np.asarray(f, dtype=np.float64) - np.mean(f)
    one = sp.csr_matrix(np.ones((N, 1)))
    K = sp.bmat([[A, one], [one.T, None]]).tocsc()
    sol = spla.spsolve(K, np.concatenate([f0, [0.0]]))
    return sol[:N]


# ---------------------------------------------------------------------------
# velocity projection (eq. projection_step_weak)
# ---------------------------------------------------------------------------

def projection_form(pb_u: Problem, pb_p: Problem, p) -> np.ndarray:
    """(div v, p)_e - (v, {p} n)_de for every velocity test function;
    {p} = p- on the walls (pressure Neumann: mirror p+ = p-)."""
    mesh, n, npr = pb_u.mesh, pb_u.n, pb_p.n
    Pn = np.asarray(p, dtype=np.float64).reshape(mesh.ncells, 1, npr ** 3)
    Y = np.zeros((mesh.ncells, 3, n ** 3))
    cells = np.arange(mesh.ncells)
    pts, _ = cell_points(n)
    Vu, Gu = tensor_tables(n, pts)
    Vq, _ = tensor_tables(npr, pts)
    _, Jinv, JxW = _cell_geo(pb_u, cells)
    pq = _values(pb_u, Pn, Vq)[..., 0]                             # (E, P)
    B = pq[..., None, None] * np.eye(3)                            # grad v : (p I) = p div v
    Y += _test_project(Vu, Gu, Jinv, np.zeros(B.shape[:3]), B, JxW)
    for d in range(3):
        em, ep = mesh.interior_faces(d)
        if len(em):
            ptm, ptp = face_points(n, d, 1)[0], face_points(n, d, 0)[0]
            Vum, Gum = tensor_tables(n, ptm)
            Vup, Gup = tensor_tables(n, ptp)
            Vqm, _ = tensor_tables(npr, ptm)
            Vqp, _ = tensor_tables(npr, ptp)
            _, _, Jim, nrm, ds = _face_geo(pb_u, em, d, 1)
            _, _, Jip, _, _ = _face_geo(pb_u, ep, d, 0)
            pavg = 0.5 * (_values(pb_u, Pn[em], Vqm) + _values(pb_u, Pn[ep], Vqp))   # (E, P, 1)
            a = pavg * nrm
            zero = np.zeros(a.shape + (3,))
            Y[em] += _test_project(Vum, Gum, Jim, -a, zero, ds)
            Y[ep] += _test_project(Vup, Gup, Jip, a, zero, ds)
        for side in (0, 1):
            bc = mesh.boundary_cells(d, side)
            pt = face_points(n, d, side)[0]
            Vuf, Guf = tensor_tables(n, pt)
            Vqf, _ = tensor_tables(npr, pt)
            _, _, Ji, nrm, ds = _face_geo(pb_u, bc, d, side)
            a = _values(pb_u, Pn[bc], Vqf) * nrm
            Y[bc] += _test_project(Vuf, Guf, Ji, -a, np.zeros(a.shape + (3,)), ds)
    return Y.reshape(-1)


def projection(pb_u: Problem, pb_p: Problem, uhat, p, dt: float, gamma0: float = GAMMA0):
    """uhh from (gamma_0/dt)(v, uhh) = (gamma_0/dt)(v, uhat) + (div v, p) - (v, {p} n),
    and the viscous step's right-hand side (gamma_0/dt) M uhh."""
    _walls(pb_u)
    uhh = np.asarray(uhat, dtype=np.float64) + dt / gamma0 * mass_solve(pb_u, projection_form(pb_u, pb_p, p))
    return uhh, gamma0 / dt * mass_apply(pb_u, uhh)


# ---------------------------------------------------------------------------
# penalty step factors and the whole step
# ---------------------------------------------------------------------------

def penalty_factors(pb: Problem, u, dt: float, zeta: float = 1.0):
    """Per-cell tau_div = zeta |u_e| h_e dt/(k+1) and tau_cont = zeta |u_e| dt,
    |u_e| the volume mean of |u| over the cell, h_e = |cell|^(1/3)."""
    n = pb.n
    U = np.asarray(u, dtype=np.float64).reshape(pb.mesh.ncells, 3, n ** 3)
    pts, _ = cell_points(n)
    V, _ = tensor_tables(n, pts)
    _, _, JxW = _cell_geo(pb, np.arange(pb.mesh.ncells))
    speed = np.linalg.norm(_values(pb, U, V), axis=-1)
    ue = np.sum(JxW * speed, axis=1) / np.sum(JxW, axis=1)
    h = cell_sizes(pb)
    return zeta * ue * h * dt / (pb.degree + 1), zeta * ue * dt


def viscous_wall_load(pb: Problem, g_wall) -> np.ndarray:
    """The viscous step's load of the wall data (mirror principle of the
    SIPG form): int -2 mu eps(v):(g (x) n) + 2 tau (v.g + (v.n)(g.n)) over the
    walls, mu the problem's viscosity at the face points."""
    mesh, n = pb.mesh, pb.n
    Y = np.zeros((mesh.ncells, 3, n ** 3))
    sig = penalty_geometry(pb)
    for d in range(3):
        for side in (0, 1):
            bc = mesh.boundary_cells(d, side)
            Vf, Gf = tensor_tables(n, face_points(n, d, side)[0])
            _, xq, Ji, nrm, ds = _face_geo(pb, bc, d, side)
            mu = _mu_face(pb, d, bc, side, xq)
            tau = _tau(pb, mu, sig[bc])
            g = _wall_g(pb, g_wall, d, side)
            gn = np.einsum("epc,epc->ep", g, nrm)
            a = 2.0 * tau[..., None] * (g + nrm * gn[..., None])
            B = -2.0 * mu[..., None, None] * _sym(g[..., :, None] * nrm[..., None, :])
            Y[bc] += _test_project(Vf, Gf, Ji, a, B, ds)
    return Y.reshape(-1)


def penalty_wall_load(pb: Problem, g_wall) -> np.ndarray:
    """The penalty step's load of the wall data: int tau_e (v.n)(g.n) over
    the walls (oriented jump u - g with the cell's own continuity factor)."""
    mesh, n = pb.mesh, pb.n
    Y = np.zeros((mesh.ncells, 3, n ** 3))
    for d in range(3):
        for side in (0, 1):
            bc = mesh.boundary_cells(d, side)
            Vf, Gf = tensor_tables(n, face_points(n, d, side)[0])
            _, _, Ji, nrm, ds = _face_geo(pb, bc, d, side)
            g = _wall_g(pb, g_wall, d, side)
            tf = _tau_face(pb, bc)[:, None]
            a = tf[..., None] * nrm * np.einsum("epc,epc->ep", g, nrm)[..., None]
            Y[bc] += _test_project(Vf, Gf, Ji, a, np.zeros(a.shape + (3,)), ds)
    return Y.reshape(-1)


def split_step(pb_visc: Problem, law: dict, u_old, b, dt: float, zeta: float = 1.0, g_wall=None,
               u_prev=None) -> dict:
    """One step of Alg. 1 (BDF1, or BDF2 given u_prev = u^{n-1}) with
    linear-implicit viscosity: convective step, pressure step, projection,
    viscous step, penalty step.  pb_visc is the viscous problem with
    alpha = gamma_0/dt on the velocity mesh (walls); every linear system is
    solved directly."""
    c = bdf(1 if u_prev is None else 2)
    if abs(pb_visc.alpha * dt - c["gamma0"]) > 1e-12 * c["gamma0"]:
        raise ValueError("the viscous problem's mass coefficient must be gamma_0/dt")
    olds = [np.asarray(u_old, dtype=np.float64)] + ([] if u_prev is None else [np.asarray(u_prev, dtype=np.float64)])
    u_ex = sum(b_i * v for b_i, v in zip(c["beta"], olds))     # u^#
    pb_p = pressure_problem(pb_visc.mesh, pb_visc.degree)
    uhat = convective_step(pb_visc, u_old, b, dt, g_wall, u_prev)
    f = ppe_rhs(pb_visc, pb_p, uhat, u_old, b, dt, g_wall, u_prev, law)
    p = pressure_solve(pb_p, f)
    uhh, rhs_v = projection(pb_visc, pb_p, uhat, p, dt, c["gamma0"])
    pb_v = PC.with_velocity_viscosity(pb_visc, pb_visc, u_ex, law)
    if g_wall is not None:
        rhs_v = rhs_v + viscous_wall_load(pb_v, g_wall)
    u_visc = spla.spsolve(assemble(pb_v).tocsc(), rhs_v)
    td, tc = penalty_factors(pb_visc, u_ex, dt, zeta)
    pb_pen = Problem(pb_visc.mesh, pb_visc.degree, "penalty", 1.0, 1.0, tau_div=td, tau_cont=tc)
    rhs_pen = mass_apply(pb_pen, u_visc)
    if g_wall is not None:
        rhs_pen = rhs_pen + penalty_wall_load(pb_pen, g_wall)
    u_new = spla.spsolve(assemble(pb_pen).tocsc(), rhs_pen)
    return {"uhat": uhat, "ppe_rhs": f, "p": p, "uhh": uhh, "rhs_visc": rhs_v, "u_visc": u_visc,
            "tau_div": td, "tau_cont": tc, "u_new": u_new, "pb_p": pb_p}
