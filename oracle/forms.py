"""SIPG bilinear forms, their assembly, their direct application and diagonal.

Viscous operator (Sec. 4.1, paragraph "Viscous Step"): the form v_h^e of the
viscous step, built from tau_1 = nu grad u and tau_2 = nu (grad u)^T with the
SIPG fluxes u^dag = {{u}}, tau_1^dag = {{nu grad u}} - tau [[u]],
tau_2^dag = (tau_1^dag)^T, plus the mass term (gamma_0/dt)(v, u) of the viscous
step; alpha below is gamma_0/dt.  Summed over the cells and rewritten face by
face (u - u^dag = [u]/2, [[u]] = [u] (x) n) this reads

  a(v, u) = sum_cells int  alpha v.u + 2 mu eps(v):eps(u)
          + sum_interior int  -2 {{mu eps(v)}}:([u](x)n) - 2 {{mu eps(u)}}:([v](x)n)
                              + tau ([v].[u] + ([v].n)([u].n))
          + sum_Dirichlet int -2 mu eps(v):(u(x)n) - 2 mu eps(u):(v(x)n)
                              + 2 tau (v.u + (v.n)(u.n))

with [w] = w^- - w^+ (Sec. 4), n the unit normal from the "-" to the "+"
cell, and the boundary terms from the mirror principle (Dirichlet:
u^+ = -u^-, grad u^+ = grad u^-; Neumann: u^+ = u^-, grad u^+ = -grad u^-,
which cancels every term).

Poisson operator (Sec. 4.1, paragraph "Pressure Step"), coercive SIPG sign:

  a_p(q, p) = sum_cells int alpha q p + grad q . grad p
            + sum_interior int -{{grad q}}.n [p] - {{grad p}}.n [q] + tau_p [q][p]
            + sum_Dirichlet int -(grad q . n) p - (grad p . n) q + 2 tau_p q p

Penalty step (Sec. 4.3, "Consistent Stabilization", eq. penalty_step): per cell
(v, u) + (div v, tau_div^e div u) + (v.n, tau_cont^e [[u]].n) on the cell
boundary.  Summed over cells with the face factor taken as the mean of the
two cells' tau_cont (a reading: it keeps the form symmetric) and the
oriented jump u - g on Dirichlet faces (no mirror doubling):

  a_pen(v, u) = sum_cells int alpha v.u + tau_div div v div u
              + sum_interior int tau_F ([v].n)([u].n)
              + sum_Dirichlet int tau_e (v.n)(u.n)

with alpha = 1 for the paper's form; the factors come per cell as inputs.

Penalty of the SIPG forms (Sec. 4.1 takes it from Hillewaert 2013 and omits
the formula): tau = P (k+1)^2 mu(x) sigma_F, where sigma_e is the cell's
surface-to-volume ratio with interior faces weighted by one half,
  sigma_e = (sum_{faces f of e} w_f |f|) / |e|,  w_f = 1/2 inside, 1 on the boundary,
sigma_F = max(sigma^-, sigma^+) on an interior face and the cell's own value on
a boundary face, mu the pointwise viscosity at the face point (mu = 1 for the
Poisson operator).  For a cube of edge h inside the mesh sigma_e = 3/h.

Degrees of freedom: nodal values at the Gauss points; vector index
((e*C + c)*n + i3)*n^2 + i2*n + i1.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from .basis import cell_points, face_points, tensor_tables, gauss_points
from .laws import viscosity
from .mesh import Mesh


@dataclass
class Problem:
    mesh: Mesh
    degree: int
    op: str = "viscous"          # "viscous" (3 components), "poisson" (1) or "penalty" (3)
    alpha: float = 0.0           # gamma_0 / dt in front of the mass term (1 for the penalty step)
    penalty: float = 1.0         # P in tau = P (k+1)^2 mu sigma_F
    law: object = field(default_factory=lambda: {"kind": "const", "mu": 1.0})
    tau_div: object = None       # penalty step: tau_div per cell
    tau_cont: object = None      # penalty step: tau_cont per cell
    mu_values: object = None     # viscous: (mu_cell [ncells, n^3], mu_face [nfaces, n^2]) given
                                 # pointwise (e.g. from a velocity, Sec. 4.1 eq. viscosity_pointwise)
                                 # in place of the law; faces numbered by Mesh.face_index

    @property
    def n(self) -> int:
        return self.degree + 1

    @property
    def C(self) -> int:
        return 1 if self.op == "poisson" else 3

    @property
    def nloc(self) -> int:
        return self.C * self.n ** 3

    @property
    def ndof(self) -> int:
        return self.mesh.ncells * self.nloc

    @staticmethod
    def from_config(cfg: dict, vertices=None) -> "Problem":
        """Build from a ``workloads.config`` dictionary (vertices drawn there)."""
        mesh = Mesh(cfg["nx"], cfg["ny"], cfg["nz"], vertices, cfg["bc"])
        return Problem(mesh, cfg["degree"], cfg["op"], cfg["alpha"], cfg["penalty"], cfg["law"],
                       cfg.get("tau_div"), cfg.get("tau_cont"))


# ---------------------------------------------------------------------------
# geometry
# ---------------------------------------------------------------------------

def cell_sizes(pb: Problem, cells=None) -> np.ndarray:
    """h_e = (int_e 1 dx)^(1/3); the n-point rule is exact for trilinear cells.
    With `cells` given only those entries are computed (the others are NaN)."""
    pts, w = cell_points(pb.n)
    if cells is None:
        J = pb.mesh.jacobian(np.arange(pb.mesh.ncells), pts)
        return (np.linalg.det(J) @ w) ** (1.0 / 3.0)
    cells = np.unique(np.asarray(cells))
    h = np.full(pb.mesh.ncells, np.nan)
    h[cells] = (np.linalg.det(pb.mesh.jacobian(cells, pts)) @ w) ** (1.0 / 3.0)
    return h


def penalty_geometry(pb: Problem, cells=None) -> np.ndarray:
    """sigma_e = (sum_f w_f |f|) / |e| per cell: face areas |f| = sum of ds
    over the face rule, w_f = 1/2 for a face shared with another cell and 1
    for a face on the boundary of the box, |e| = sum of JxW.  With `cells`
    given only those entries are computed (the others are NaN)."""
    mesh = pb.mesh
    sel = np.arange(mesh.ncells) if cells is None else np.unique(np.asarray(cells))
    sig = np.full(mesh.ncells, np.nan)
    if len(sel) == 0:
        return sig
    _, _, JxW = _cell_geo(pb, sel)
    vol = JxW.sum(axis=1)
    ijk = mesh.cell_ijk(sel)
    surf = np.zeros(len(sel))
    for d in range(3):
        lim = (mesh.nx, mesh.ny, mesh.nz)[d]
        for side in (0, 1):
            _, _, _, _, ds = _face_geo(pb, sel, d, side)
            on_boundary = ijk[d] == (lim - 1 if side == 1 else 0)
            surf += np.where(on_boundary, 1.0, 0.5) * ds.sum(axis=1)
    sig[sel] = surf / vol
    return sig


def _with_neighbours(mesh, cells) -> np.ndarray:
    """The cells and the (up to six) cells sharing a face with them."""
    ex, ey, ez = mesh.cell_ijk(np.asarray(cells))
    out = [np.asarray(cells)]
    for d, (lim, stride) in enumerate(((mesh.nx, 1), (mesh.ny, mesh.nx), (mesh.nz, mesh.nx * mesh.ny))):
        pos = (ex, ey, ez)[d]
        out.append(np.asarray(cells)[pos > 0] - stride)
        out.append(np.asarray(cells)[pos < lim - 1] + stride)
    return np.unique(np.concatenate(out))


def _cell_geo(pb: Problem, cells):
    pts, w = cell_points(pb.n)
    J = pb.mesh.jacobian(cells, pts)
    det = np.linalg.det(J)
    if np.any(det <= 0):
        raise ValueError("inverted cell")
    Jinv = np.linalg.inv(J)                  # Jinv[e, q, d, i] = d xi_d / d x_i
    xq = pb.mesh.map(cells, pts)
    return xq, Jinv, det * w


def _face_geo(pb: Problem, cells, d, side):
    """Geometry on face xi_d = side of each cell: points, Jinv, unit normal
    pointing out of that cell, surface measure ds = det J |J^-T e_d| w."""
    pts, wf = face_points(pb.n, d, side)
    J = pb.mesh.jacobian(cells, pts)
    det = np.linalg.det(J)
    Jinv = np.linalg.inv(J)
    v = Jinv[..., d, :]                      # J^-T e_d
    nv = np.linalg.norm(v, axis=-1)
    normal = (1.0 if side == 1 else -1.0) * v / nv[..., None]
    ds = det * nv * wf
    xq = pb.mesh.map(cells, pts)
    return pts, xq, Jinv, normal, ds


def _mu(pb: Problem, x):
    if pb.op != "viscous":
        return np.ones(x.shape[:-1])
    return viscosity(pb.law, x)


def _mu_cell(pb: Problem, cells, x):
    """mu at the cell points x (E, n^3, 3) of `cells`."""
    if pb.op == "viscous" and pb.mu_values is not None:
        return np.asarray(pb.mu_values[0], dtype=np.float64)[np.asarray(cells)]
    return _mu(pb, x)


def _mu_face(pb: Problem, d, cells, side, x):
    """mu at the points x (E, n^2, 3) of the faces xi_d = side of `cells`."""
    if pb.op == "viscous" and pb.mu_values is not None:
        return np.asarray(pb.mu_values[1], dtype=np.float64)[pb.mesh.face_index(d, np.asarray(cells), side)]
    return _mu(pb, x)


def _tau(pb: Problem, mu, sigF):
    """tau = P (k+1)^2 mu sigma_F at the face points (mu: (F, points))."""
    return pb.penalty * (pb.degree + 1) ** 2 * mu * sigF[:, None]


def _sym(G):
    return 0.5 * (G + np.swapaxes(G, -1, -2))


# ---------------------------------------------------------------------------
# the two face forms, literally, for broadcast arrays of test and trial traces
# ---------------------------------------------------------------------------

def viscous_face_form(vm, vp, Gvm, Gvp, um, up, Gum, Gup, mu, tau, n):
    """Interior-face integrand for test traces (vm, vp, Gvm, Gvp) of shape
    (I, 3) / (I, 3, 3) and trial traces of shape (J, 3) / (J, 3, 3) at one
    point; returns the (I, J) matrix of
    -2{{mu eps(v)}}:([u](x)n) - 2{{mu eps(u)}}:([v](x)n) + tau([v].[u] + ([v].n)([u].n))."""
    jv, ju = vm - vp, um - up
    ev = 0.5 * mu * (_sym(Gvm) + _sym(Gvp))
    eu = 0.5 * mu * (_sym(Gum) + _sym(Gup))
    return (-2.0 * (ev @ n) @ ju.T - 2.0 * jv @ (eu @ n).T
            + tau * (jv @ ju.T + np.outer(jv @ n, ju @ n)))


def viscous_dirichlet_form(v, Gv, u, Gu, mu, tau, n):
    """-2 mu eps(v):(u(x)n) - 2 mu eps(u):(v(x)n) + 2 tau (v.u + (v.n)(u.n))."""
    ev, eu = mu * _sym(Gv), mu * _sym(Gu)
    return (-2.0 * (ev @ n) @ u.T - 2.0 * v @ (eu @ n).T
            + 2.0 * tau * (v @ u.T + np.outer(v @ n, u @ n)))


def poisson_face_form(qm, qp, Gqm, Gqp, pm, pp, Gpm, Gpp, tau, n):
    """-{{grad q}}.n [p] - {{grad p}}.n [q] + tau [q][p] for (I,) / (I, 3) test
    and (J,) / (J, 3) trial traces."""
    jq, jp = qm - qp, pm - pp
    aq = 0.5 * (Gqm + Gqp) @ n
    ap = 0.5 * (Gpm + Gpp) @ n
    return -np.outer(aq, jp) - np.outer(jq, ap) + tau * np.outer(jq, jp)


def penalty_face_form(vm, vp, um, up, tau, n):
    """Continuity penalty of the penalty step on an interior face:
    tau ([v].n)([u].n) for (I, 3) test and (J, 3) trial traces."""
    return tau * np.outer((vm - vp) @ n, (um - up) @ n)


def penalty_dirichlet_form(v, u, tau, n):
    """tau (v.n)(u.n): the oriented jump on a Dirichlet face is u - g."""
    return tau * np.outer(v @ n, u @ n)


def _div(g):
    """Divergence of vector basis functions from their gradients (..., C, 3)."""
    return np.einsum("...cc->...", g)


def _tau_face(pb: Problem, a, b=None):
    """Penalty step: face value of tau_cont, the mean of the two cells'
    values inside and the cell's own value on the boundary."""
    t = np.asarray(pb.tau_cont, dtype=np.float64)
    return t[a] if b is None else 0.5 * (t[a] + t[b])


def poisson_dirichlet_form(q, Gq, p, Gp, tau, n):
    """-(grad q.n) p - (grad p.n) q + 2 tau q p."""
    return -np.outer(Gq @ n, p) - np.outer(q, Gp @ n) + 2.0 * tau * np.outer(q, p)


# ---------------------------------------------------------------------------
# basis traces of one cell: every local basis function at a set of points
# ---------------------------------------------------------------------------

def _basis_traces(pb: Problem, V, G, Jinv):
    """For points with tables V (P, n^3), G (P, n^3, 3) and one cell's Jinv
    (P, 3, 3): values (P, nloc, C) and physical gradients (P, nloc, C, 3)
    of all local basis functions phi_{c,j} = phi_j e_c (index c*n^3 + j)."""
    C, n3 = pb.C, pb.n ** 3
    P = V.shape[0]
    grad = np.einsum("pjd,pdi->pji", G, Jinv)            # (P, n^3, 3)
    vals = np.zeros((P, C * n3, C))
    grads = np.zeros((P, C * n3, C, 3))
    for c in range(C):
        vals[:, c * n3:(c + 1) * n3, c] = V
        grads[:, c * n3:(c + 1) * n3, c, :] = grad
    return vals, grads


# ---------------------------------------------------------------------------
# O2: assembled sparse matrix
# ---------------------------------------------------------------------------

PARTS_ALL = ("cell", "interior", "boundary")


def assemble(pb: Problem, parts=PARTS_ALL) -> sp.csr_matrix:
    """Global matrix A_IJ = a(phi_I, phi_J), element by element, face by face."""
    mesh, n, C, nloc = pb.mesh, pb.n, pb.C, pb.nloc
    rows, cols, vals = [], [], []
    loc = np.arange(nloc)
    sig = penalty_geometry(pb)

    def add(block, dofs_r, dofs_c):
        R, Cc = np.meshgrid(dofs_r, dofs_c, indexing="ij")
        rows.append(R.ravel()); cols.append(Cc.ravel()); vals.append(block.ravel())

    if "cell" in parts:
        pts, _ = cell_points(n)
        V, G = tensor_tables(n, pts)
        for e in range(mesh.ncells):
            xq, Jinv, JxW = _cell_geo(pb, np.array([e]))
            mu = _mu_cell(pb, np.array([e]), xq)[0]
            v, g = _basis_traces(pb, V, G, Jinv[0])
            K = np.zeros((nloc, nloc))
            for q in range(len(JxW[0])):
                if pb.op == "viscous":
                    E = _sym(g[q]).reshape(nloc, 9)
                    K += JxW[0, q] * (pb.alpha * v[q] @ v[q].T + 2.0 * mu[q] * E @ E.T)
                elif pb.op == "penalty":
                    dv = _div(g[q])
                    K += JxW[0, q] * (pb.alpha * v[q] @ v[q].T + pb.tau_div[e] * np.outer(dv, dv))
                else:
                    gg = g[q][:, 0, :]
                    K += JxW[0, q] * (pb.alpha * v[q] @ v[q].T + gg @ gg.T)
            add(K, e * nloc + loc, e * nloc + loc)

    if "interior" in parts:
        for d in range(3):
            em, ep = mesh.interior_faces(d)
            ptm, _ = face_points(n, d, 1)
            ptp, _ = face_points(n, d, 0)
            Vm, Gm = tensor_tables(n, ptm)
            Vp, Gp = tensor_tables(n, ptp)
            for a, b in zip(em, ep):
                _, xq, Jim, nrm, ds = _face_geo(pb, np.array([a]), d, 1)
                _, _, Jip, _, _ = _face_geo(pb, np.array([b]), d, 0)
                mu = _mu_face(pb, d, np.array([a]), 1, xq)[0]
                tau = _tau(pb, mu[None], np.array([max(sig[a], sig[b])]))[0]
                vm_, gm_ = _basis_traces(pb, Vm, Gm, Jim[0])
                vp_, gp_ = _basis_traces(pb, Vp, Gp, Jip[0])
                # test/trial functions of both cells: first the "-" cell's, then the "+" cell's
                K = np.zeros((2 * nloc, 2 * nloc))
                z = np.zeros_like(vm_[0]); zg = np.zeros_like(gm_[0])
                for f in range(len(ds[0])):
                    Vminus = np.concatenate([vm_[f], z]); Vplus = np.concatenate([z, vp_[f]])
                    Gminus = np.concatenate([gm_[f], zg]); Gplus = np.concatenate([zg, gp_[f]])
                    if pb.op == "viscous":
                        blk = viscous_face_form(Vminus, Vplus, Gminus, Gplus,
                                                Vminus, Vplus, Gminus, Gplus,
                                                mu[f], tau[f], nrm[0, f])
                    elif pb.op == "penalty":
                        blk = penalty_face_form(Vminus, Vplus, Vminus, Vplus, _tau_face(pb, a, b), nrm[0, f])
                    else:
                        blk = poisson_face_form(Vminus[:, 0], Vplus[:, 0], Gminus[:, 0], Gplus[:, 0],
                                                Vminus[:, 0], Vplus[:, 0], Gminus[:, 0], Gplus[:, 0],
                                                tau[f], nrm[0, f])
                    K += ds[0, f] * blk
                dofs = np.concatenate([a * nloc + loc, b * nloc + loc])
                add(K, dofs, dofs)

    if "boundary" in parts:
        for d in range(3):
            for side in (0, 1):
                if mesh.bc[2 * d + side] != "D":
                    continue
                pts, _ = face_points(n, d, side)
                Vf, Gf = tensor_tables(n, pts)
                for e in mesh.boundary_cells(d, side):
                    _, xq, Ji, nrm, ds = _face_geo(pb, np.array([e]), d, side)
                    mu = _mu_face(pb, d, np.array([e]), side, xq)[0]
                    tau = _tau(pb, mu[None], np.array([sig[e]]))[0]
                    v, g = _basis_traces(pb, Vf, Gf, Ji[0])
                    K = np.zeros((nloc, nloc))
                    for f in range(len(ds[0])):
                        if pb.op == "viscous":
                            blk = viscous_dirichlet_form(v[f], g[f], v[f], g[f], mu[f], tau[f], nrm[0, f])
                        elif pb.op == "penalty":
                            blk = penalty_dirichlet_form(v[f], v[f], _tau_face(pb, e), nrm[0, f])
                        else:
                            blk = poisson_dirichlet_form(v[f][:, 0], g[f][:, 0], v[f][:, 0], g[f][:, 0],
                                                         tau[f], nrm[0, f])
                        K += ds[0, f] * blk
                    add(K, e * nloc + loc, e * nloc + loc)

    N = pb.ndof
    if not rows:
        return sp.csr_matrix((N, N))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    return A.tocsr()


# ---------------------------------------------------------------------------
# O3: the same quadrature sums applied directly to a vector
# ---------------------------------------------------------------------------

def _phys_grad(X, G, Jinv):
    """X (E, C, n^3), tables G (P, n^3, 3), Jinv (E, P, 3, 3) -> grad (E, P, C, 3)."""
    ref = np.einsum("pjd,ecj->epcd", G, X, optimize=True)
    return np.einsum("epcd,epdi->epci", ref, Jinv, optimize=True)


def _test_project(V, G, Jinv, a, B, w):
    """sum_p w[e,p] (V[p,j] a[e,p,c] + grad phi_j(p) . B[e,p,c,:]) -> (E, C, n^3)."""
    Bref = np.einsum("epdi,epci->epcd", Jinv, B, optimize=True)
    return (np.einsum("pj,ep,epc->ecj", V, w, a, optimize=True)
            + np.einsum("pjd,ep,epcd->ecj", G, w, Bref, optimize=True))


def apply(pb: Problem, x: np.ndarray, parts=PARTS_ALL, batch: int = 4096, cells=None) -> np.ndarray:
    """y = A x evaluated directly from the quadrature sums (no global matrix).

    With `cells` given, only the rows of those cells are evaluated (the other
    rows are returned as zero), so single entries of large problems can be
    checked without evaluating the whole operator."""
    mesh, n, C = pb.mesh, pb.n, pb.C
    X = np.asarray(x, dtype=np.float64).reshape(mesh.ncells, C, n ** 3)
    Y = np.zeros_like(X)
    sig = penalty_geometry(pb) if cells is None else penalty_geometry(pb, _with_neighbours(mesh, cells))
    sel = np.ones(mesh.ncells, dtype=bool)
    if cells is not None:
        sel[:] = False
        sel[np.asarray(cells)] = True
    own = np.nonzero(sel)[0]

    if "cell" in parts:
        pts, _ = cell_points(n)
        V, G = tensor_tables(n, pts)
        for s in range(0, len(own), batch):
            cells = own[s:s + batch]
            xq, Jinv, JxW = _cell_geo(pb, cells)
            mu = _mu_cell(pb, cells, xq)
            Xc = X[cells]
            u = np.einsum("pj,ecj->epc", V, Xc)
            gu = _phys_grad(Xc, G, Jinv)
            if pb.op == "viscous":
                B = 2.0 * mu[..., None, None] * _sym(gu)
            elif pb.op == "penalty":
                td = np.asarray(pb.tau_div, dtype=np.float64)[cells]
                B = (td[:, None] * _div(gu))[..., None, None] * np.eye(3)
            else:
                B = gu
            Y[cells] += _test_project(V, G, Jinv, pb.alpha * u, B, JxW)

    if "interior" in parts:
        for d in range(3):
            em_all, ep_all = mesh.interior_faces(d)
            keep = sel[em_all] | sel[ep_all]
            em_all, ep_all = em_all[keep], ep_all[keep]
            ptm, _ = face_points(n, d, 1)
            ptp, _ = face_points(n, d, 0)
            Vm, Gm = tensor_tables(n, ptm)
            Vp, Gp = tensor_tables(n, ptp)
            for s in range(0, len(em_all), batch):
                em, ep = em_all[s:s + batch], ep_all[s:s + batch]
                _, xq, Jim, nrm, ds = _face_geo(pb, em, d, 1)
                _, _, Jip, _, _ = _face_geo(pb, ep, d, 0)
                mu = _mu_face(pb, d, em, 1, xq)
                tau = _tau(pb, mu, np.maximum(sig[em], sig[ep]))
                um = np.einsum("pj,ecj->epc", Vm, X[em]); up = np.einsum("pj,ecj->epc", Vp, X[ep])
                gm = _phys_grad(X[em], Gm, Jim); gp = _phys_grad(X[ep], Gp, Jip)
                if pb.op == "penalty":
                    ju = um - up
                    tf = _tau_face(pb, em, ep)[:, None]
                    a_m = tf[..., None] * nrm * np.einsum("epc,epc->ep", ju, nrm)[..., None]
                    B = np.zeros(ju.shape + (3,))
                elif pb.op == "viscous":
                    ju = um - up
                    avg = 0.5 * mu[..., None, None] * (_sym(gm) + _sym(gp))
                    a_m = (-2.0 * np.einsum("epci,epi->epc", avg, nrm)
                           + tau[..., None] * (ju + nrm * np.einsum("epc,epc->ep", ju, nrm)[..., None]))
                    B = -mu[..., None, None] * _sym(ju[..., :, None] * nrm[..., None, :])
                else:
                    ju = um - up
                    avgn = 0.5 * np.einsum("epci,epi->epc", gm + gp, nrm)
                    a_m = -avgn + tau[..., None] * ju
                    B = -0.5 * ju[..., :, None] * nrm[..., None, :]
                Y[em] += _test_project(Vm, Gm, Jim, a_m, B, ds)
                Y[ep] += _test_project(Vp, Gp, Jip, -a_m, B, ds)

    if "boundary" in parts:
        for d in range(3):
            for side in (0, 1):
                if mesh.bc[2 * d + side] != "D":
                    continue
                pts, _ = face_points(n, d, side)
                Vf, Gf = tensor_tables(n, pts)
                cells = mesh.boundary_cells(d, side)
                cells = cells[sel[cells]]
                if len(cells) == 0:
                    continue
                _, xq, Ji, nrm, ds = _face_geo(pb, cells, d, side)
                mu = _mu_face(pb, d, cells, side, xq)
                tau = _tau(pb, mu, sig[cells])
                u = np.einsum("pj,ecj->epc", Vf, X[cells])
                gu = _phys_grad(X[cells], Gf, Ji)
                if pb.op == "penalty":
                    tf = _tau_face(pb, cells)[:, None]
                    a = tf[..., None] * nrm * np.einsum("epc,epc->ep", u, nrm)[..., None]
                    B = np.zeros(u.shape + (3,))
                elif pb.op == "viscous":
                    a = (-2.0 * mu[..., None] * np.einsum("epci,epi->epc", _sym(gu), nrm)
                         + 2.0 * tau[..., None] * (u + nrm * np.einsum("epc,epc->ep", u, nrm)[..., None]))
                    B = -2.0 * mu[..., None, None] * _sym(u[..., :, None] * nrm[..., None, :])
                else:
                    a = -np.einsum("epci,epi->epc", gu, nrm) + 2.0 * tau[..., None] * u
                    B = -u[..., :, None] * nrm[..., None, :]
                Y[cells] += _test_project(Vf, Gf, Ji, a, B, ds)

    Y[~sel] = 0.0
    return Y.reshape(-1)


# ---------------------------------------------------------------------------
# diagonal a(phi_I, phi_I) without assembling
# ---------------------------------------------------------------------------

def diagonal(pb: Problem, batch: int = 1024) -> np.ndarray:
    """d_I = a(phi_I, phi_I), evaluated with the face forms above for every
    local basis function (the matrix diagonal that Sec. 5.3 inverts for the
    Jacobi-type smoother)."""
    mesh, n, C, nloc = pb.mesh, pb.n, pb.C, pb.nloc
    D = np.zeros((mesh.ncells, nloc))
    sig = penalty_geometry(pb)
    pts, _ = cell_points(n)
    V, G = tensor_tables(n, pts)
    for s in range(0, mesh.ncells, batch):
        cells = np.arange(s, min(s + batch, mesh.ncells))
        xq, Jinv, JxW = _cell_geo(pb, cells)
        mu = _mu_cell(pb, cells, xq)
        grad = np.einsum("pjd,epdi->epji", G, Jinv, optimize=True)   # (E, P, n^3, 3)
        g2 = np.einsum("epji,epji->epj", grad, grad)
        for c in range(C):
            if pb.op == "viscous":
                # 2 mu eps(phi e_c):eps(phi e_c) = mu (|grad phi|^2 + (d_c phi)^2)
                dens = pb.alpha * V[None] ** 2 + mu[..., None] * (g2 + grad[..., c] ** 2)
            elif pb.op == "penalty":
                # div(phi e_c) = d_c phi
                td = np.asarray(pb.tau_div, dtype=np.float64)[cells]
                dens = pb.alpha * V[None] ** 2 + td[:, None, None] * grad[..., c] ** 2
            else:
                dens = pb.alpha * V[None] ** 2 + g2
            D[cells, c * n ** 3:(c + 1) * n ** 3] += np.einsum("ep,epj->ej", JxW, dens)

    def face_self(cells, d, side, sigF, dirichlet, tau_p=None):
        pts, _ = face_points(n, d, side)
        Vf, Gf = tensor_tables(n, pts)
        _, xq, Ji, nrm, ds = _face_geo(pb, cells, d, side)
        mu = _mu_face(pb, d, cells, side, xq)
        tau = _tau(pb, mu, sigF)
        out = np.zeros((len(cells), nloc))
        for ii, e in enumerate(cells):
            v, g = _basis_traces(pb, Vf, Gf, Ji[ii])
            for f in range(len(pts)):
                if pb.op == "penalty":
                    # tau ((phi e_c).n)^2 on interior and Dirichlet faces alike
                    m = penalty_dirichlet_form(v[f], v[f], tau_p[ii], nrm[ii, f])
                elif pb.op == "viscous":
                    if dirichlet:
                        m = viscous_dirichlet_form(v[f], g[f], v[f], g[f], mu[ii, f], tau[ii, f], nrm[ii, f])
                    else:
                        z, zg = np.zeros_like(v[f]), np.zeros_like(g[f])
                        # own side is "-" when side == 1 (normal points out of it)
                        if side == 1:
                            m = viscous_face_form(v[f], z, g[f], zg, v[f], z, g[f], zg,
                                                  mu[ii, f], tau[ii, f], nrm[ii, f])
                        else:
                            m = viscous_face_form(z, v[f], zg, g[f], z, v[f], zg, g[f],
                                                  mu[ii, f], tau[ii, f], -nrm[ii, f])
                else:
                    q, gq = v[f][:, 0], g[f][:, 0]
                    if dirichlet:
                        m = poisson_dirichlet_form(q, gq, q, gq, tau[ii, f], nrm[ii, f])
                    else:
                        z, zg = np.zeros_like(q), np.zeros_like(gq)
                        if side == 1:
                            m = poisson_face_form(q, z, gq, zg, q, z, gq, zg, tau[ii, f], nrm[ii, f])
                        else:
                            m = poisson_face_form(z, q, zg, gq, z, q, zg, gq, tau[ii, f], -nrm[ii, f])
                out[ii] += ds[ii, f] * np.diag(m)
        return out

    pen = pb.op == "penalty"
    for d in range(3):
        em, ep = mesh.interior_faces(d)
        if len(em):
            sF = np.maximum(sig[em], sig[ep])
            tp = _tau_face(pb, em, ep) if pen else None
            D[em] += face_self(em, d, 1, sF, False, tp)
            D[ep] += face_self(ep, d, 0, sF, False, tp)
        for side in (0, 1):
            if mesh.bc[2 * d + side] == "D":
                cells = mesh.boundary_cells(d, side)
                D[cells] += face_self(cells, d, side, sig[cells], True, _tau_face(pb, cells) if pen else None)
    return D.reshape(-1)


# ---------------------------------------------------------------------------
# right-hand sides, interpolation and errors (for the consistency pins)
# ---------------------------------------------------------------------------

def node_points(pb: Problem) -> np.ndarray:
    """Physical node positions (ncells, n^3, 3)."""
    pts, _ = cell_points(pb.n)
    return pb.mesh.map(np.arange(pb.mesh.ncells), pts)


def interpolate(pb: Problem, fn) -> np.ndarray:
    """Nodal interpolant of fn: (P, 3) -> (P, C) (or (P,) for C = 1)."""
    xn = node_points(pb)
    E, P = xn.shape[:2]
    vals = np.asarray(fn(xn.reshape(-1, 3))).reshape(E, P, -1)     # (E, P, C)
    return np.transpose(vals, (0, 2, 1)).reshape(-1)


def load_vector(pb: Problem, f, g=None, hN=None) -> np.ndarray:
    """l(v) = sum_cells int f.v + boundary terms of the mirror principle:
    Dirichlet data g enters through u^+ = -u^- + 2g, i.e.
    viscous: int -2 mu eps(v):(g(x)n) + 2 tau (v.g + (v.n)(g.n));
    Poisson: int -(grad q.n) g + 2 tau q g;
    Neumann data hN (traction 2 mu eps(u) n, resp. grad p.n): int v.hN.
    f, g: callables (P, 3) -> (P, C) (or (P,) for C = 1); hN(x, n) also
    receives the outward unit normal at the points."""
    mesh, n, C = pb.mesh, pb.n, pb.C
    Y = np.zeros((mesh.ncells, C, n ** 3))
    sig = penalty_geometry(pb)
    pts, _ = cell_points(n)
    V, G = tensor_tables(n, pts)
    cells = np.arange(mesh.ncells)
    xq, Jinv, JxW = _cell_geo(pb, cells)
    fv = np.asarray(f(xq.reshape(-1, 3))).reshape(len(cells), len(JxW[0]), C)
    Y += np.einsum("pj,ep,epc->ecj", V, JxW, fv)

    for d in range(3):
        for side in (0, 1):
            kind = mesh.bc[2 * d + side]
            fpts, _ = face_points(n, d, side)
            Vf, Gf = tensor_tables(n, fpts)
            bc_cells = mesh.boundary_cells(d, side)
            _, xq, Ji, nrm, ds = _face_geo(pb, bc_cells, d, side)
            E, P = xq.shape[:2]
            if kind == "D" and g is not None:
                mu = _mu_face(pb, d, bc_cells, side, xq)
                tau = _tau(pb, mu, sig[bc_cells])
                gv = np.asarray(g(xq.reshape(-1, 3))).reshape(E, P, C)
                if pb.op == "viscous":
                    a = 2.0 * tau[..., None] * (gv + nrm * np.einsum("epc,epc->ep", gv, nrm)[..., None])
                    B = -2.0 * mu[..., None, None] * _sym(gv[..., :, None] * nrm[..., None, :])
                else:
                    a = 2.0 * tau[..., None] * gv
                    B = -gv[..., :, None] * nrm[..., None, :]
                Y[bc_cells] += _test_project(Vf, Gf, Ji, a, B, ds)
            if kind == "N" and hN is not None:
                hv = np.asarray(hN(xq.reshape(-1, 3), nrm.reshape(-1, 3))).reshape(E, P, C)
                Y[bc_cells] += np.einsum("pj,ep,epc->ecj", Vf, ds, hv)
    return Y.reshape(-1)


def l2_error(pb: Problem, x: np.ndarray, exact, nq: int | None = None) -> tuple[float, float]:
    """(||u_h - u||_L2, ||u||_L2) with an nq-point Gauss rule per direction."""
    nq = nq or pb.n + 2
    g, w = gauss_points(nq)
    Q3, Q2, Q1 = np.meshgrid(np.arange(nq), np.arange(nq), np.arange(nq), indexing="ij")
    pts = np.stack([g[Q1.ravel()], g[Q2.ravel()], g[Q3.ravel()]], axis=1)
    wq = w[Q1.ravel()] * w[Q2.ravel()] * w[Q3.ravel()]
    V, _ = tensor_tables(pb.n, pts)
    cells = np.arange(pb.mesh.ncells)
    J = pb.mesh.jacobian(cells, pts)
    JxW = np.linalg.det(J) * wq
    xq = pb.mesh.map(cells, pts)
    X = np.asarray(x).reshape(len(cells), pb.C, pb.n ** 3)
    uh = np.einsum("pj,ecj->epc", V, X)
    ue = np.asarray(exact(xq.reshape(-1, 3))).reshape(uh.shape)
    err = np.sqrt(np.sum(JxW[..., None] * (uh - ue) ** 2))
    ref = np.sqrt(np.sum(JxW[..., None] * ue ** 2))
    return float(err), float(ref)
