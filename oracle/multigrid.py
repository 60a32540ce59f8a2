"""Geometric hp-multigrid V-cycle used as the preconditioner of the FP64 CG
(Sec. 5.3, paragraph on preconditioning the viscous terms).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 5.3 builds the hierarchy by lowering the polynomial degree recursively
from k to k-1 and then coarsening the mesh, smooths every level with
Chebyshev-accelerated Jacobi on that level's inverse diagonal and operator
action, runs standard V-cycles, and keeps the viscosity at the integration
points of every level.  Two hierarchies are defined: the paper's own
(cph: the DG level, then continuous levels, a direct coarse solve), in
`CphHierarchy` at the end of this file, and an all-DG one (`Hierarchy`),
whose readings are:

* levels stay discontinuous: DG_k, DG_{k-1}, ..., DG_1 on the given mesh,
  then DG_1 on meshes with half as many cells per direction (every other
  vertex of the finer mesh) while all cell counts stay even and at least
  ``min_cells``;
* transfers are the natural embeddings of the coarse space in the fine
  one in reference coordinates: the coarse polynomial of a cell evaluated at
  the fine nodes (p: same cell; h: the child cell's nodes mapped into the
  parent's reference cell, xi_parent = (child + xi_child) / 2 per direction),
  restriction is the transpose;
* every level evaluates the viscosity law at its own quadrature points; for
  the penalty step a coarse cell takes the mean of its children's penalty
  factors;
* smoothing: the same Chebyshev-Jacobi polynomial as the one-level
  preconditioner (interval [lam/20, lam], lam = 1.2 x the largest Ritz value
  of 20 Lanczos steps) of degree ``smooth_degree`` before and after the
  coarse correction; the coarsest level is approximated by the same kind of
  polynomial of degree ``coarse_degree`` in place of AMG cycles.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .basis import gauss_points, lagrange_values
from .forms import Problem, apply as op_apply, assemble, diagonal
from .mesh import Mesh
from .solvers import chebyshev_jacobi, lanczos_max


def level_problems(pb: Problem, h_coarsen: bool = True, min_cells: int = 2,
                   max_levels: int = 16) -> list[Problem]:
    """The hierarchy, finest first."""
    levels = [pb]
    k = pb.degree
    while k > 1 and len(levels) < max_levels:
        k -= 1
        levels.append(Problem(pb.mesh, k, pb.op, pb.alpha, pb.penalty, pb.law, pb.tau_div, pb.tau_cont))
    m = levels[-1].mesh
    td, tc = pb.tau_div, pb.tau_cont
    while (h_coarsen and len(levels) < max_levels
           and all(c % 2 == 0 and c // 2 >= min_cells for c in (m.nx, m.ny, m.nz))):
        if td is not None:     # penalty step: a coarse cell takes the mean of its 8 children's factors
            td, tc = (np.asarray(t, float).reshape(m.nz // 2, 2, m.ny // 2, 2, m.nx // 2, 2)
                      .mean(axis=(1, 3, 5)).reshape(-1) for t in (td, tc))
        verts = m.vertices[::2, ::2, ::2].reshape(-1, 3)
        m = Mesh(m.nx // 2, m.ny // 2, m.nz // 2, verts, m.bc)
        levels.append(Problem(m, levels[-1].degree, pb.op, pb.alpha, pb.penalty, pb.law, td, tc))
    return levels


def _kron3(A, B, C):
    """Matrix of the map on tensor-product node arrays with index
    i3*n^2 + i2*n + i1 (A acts on i3, B on i2, C on i1)."""
    return np.kron(A, np.kron(B, C))


def p_matrix(nf: int, nc: int) -> np.ndarray:
    """1D prolongation DG_{nc-1} -> DG_{nf-1} on one interval: the coarse
    Lagrange basis evaluated at the fine Gauss nodes, shape (nf, nc)."""
    return lagrange_values(gauss_points(nc)[0], gauss_points(nf)[0])


def h_matrix(n: int, child: int) -> np.ndarray:
    """1D prolongation from an interval to its half number `child` (0: lower,
    1: upper): the parent's basis at the child's nodes, shape (n, n)."""
    x = gauss_points(n)[0]
    return lagrange_values(x, (child + x) / 2.0)


def prolongation(fine: Problem, coarse: Problem) -> sp.csr_matrix:
    """Global prolongation matrix (fine ndof x coarse ndof)."""
    C = fine.C
    if fine.mesh.ncells == coarse.mesh.ncells:        # p-level
        Pm = p_matrix(fine.n, coarse.n)
        block = sp.csr_matrix(np.kron(np.eye(C), _kron3(Pm, Pm, Pm)))
        return sp.block_diag([block] * fine.mesh.ncells, format="csr")
    # h-level: same degree, fine cell (fx, fy, fz) is child (fx%2, fy%2, fz%2) of (fx//2, fy//2, fz//2)
    fm, cm = fine.mesh, coarse.mesh
    n = fine.n
    H = [h_matrix(n, 0), h_matrix(n, 1)]
    nl_f, nl_c = fine.nloc, coarse.nloc
    rows, cols, vals = [], [], []
    for fz in range(fm.nz):
        for fy in range(fm.ny):
            for fx in range(fm.nx):
                ef = (fz * fm.ny + fy) * fm.nx + fx
                ec = ((fz // 2) * cm.ny + fy // 2) * cm.nx + fx // 2
                loc = np.kron(np.eye(C), _kron3(H[fz % 2], H[fy % 2], H[fx % 2]))
                r, c = np.nonzero(np.abs(loc) > 0.0)
                rows.append(ef * nl_f + r)
                cols.append(ec * nl_c + c)
                vals.append(loc[r, c])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(fine.ndof, coarse.ndof))


class Hierarchy:
    """Levels with their operators, inverse diagonals, Chebyshev intervals and
    the prolongations between consecutive levels."""

    def __init__(self, pb: Problem, smooth_degree: int = 5, coarse_degree: int = 12,
                 h_coarsen: bool = True, min_cells: int = 2, max_levels: int = 16,
                 ratio: float = 20.0, safety: float = 1.2, lanczos_steps: int = 20,
                 seed: int = 12345, levels: list[Problem] | None = None):
        # `levels` replaces the hierarchy of level_problems (e.g. the same
        # levels with the viscosity updated from a velocity)
        self.levels = levels if levels is not None else level_problems(pb, h_coarsen, min_cells, max_levels)
        self.smooth_degree, self.coarse_degree = smooth_degree, coarse_degree
        self.ops = [(lambda x, p=p: op_apply(p, x)) for p in self.levels]
        self.dinv = [1.0 / diagonal(p) for p in self.levels]
        self.lam = [lanczos_max(a, d, lanczos_steps, seed) for a, d in zip(self.ops, self.dinv)]
        self.interval = [(safety * l, safety * l / ratio) for l in self.lam]
        self.P = [prolongation(self.levels[i], self.levels[i + 1])
                  for i in range(len(self.levels) - 1)]

    def smooth(self, l: int, r: np.ndarray, degree: int) -> np.ndarray:
        hi, lo = self.interval[l]
        return chebyshev_jacobi(self.ops[l], self.dinv[l], r, degree, hi, lo)

    def vcycle(self, r: np.ndarray, l: int = 0) -> np.ndarray:
        """z ~ A_l^-1 r by one V-cycle from zero."""
        if l == len(self.levels) - 1:
            return self.smooth(l, r, self.coarse_degree)
        A = self.ops[l]
        z = self.smooth(l, r, self.smooth_degree)                   # pre-smoothing
        zc = self.vcycle(self.P[l].T @ (r - A(z)), l + 1)          # restricted residual
        z = z + self.P[l] @ zc                                      # coarse correction
        return z + self.smooth(l, r - A(z), self.smooth_degree)    # post-smoothing


# ---------------------------------------------------------------------------
# cph-multigrid: continuous levels below the DG level (Sec. 5.3)
# ---------------------------------------------------------------------------
#
# Sec. 5.3 first transfers the DG solution to continuous elements of the same
# degree, then lowers the degree of the continuous space, then coarsens the
# mesh, and solves the coarsest level with AMG or a direct solver.  Readings
# taken here:
#
# * the continuous space Q_j^c on a level's mesh is nodal at the Gauss-Lobatto
#   points of every cell (shared nodes on shared faces, edges and vertices);
#   it is a subspace of the level's DG_j space, and the embedding G evaluates
#   a cell's Lobatto interpolant at its Gauss nodes;
# * the continuous level's operator is the Galerkin restriction G^T A G of
#   the level's DG operator: for continuous functions every interior-face
#   term of the SIPG form vanishes, so only cell and boundary-face terms are
#   kept (the weak Dirichlet conditions stay as in the DG form);
# * the continuous levels are Q_k^c, Q_{k-1}^c, ..., Q_1^c on the given mesh,
#   then Q_1^c on the coarser meshes of `level_problems`; transfers between
#   them are embeddings (same reference-coordinate nesting as the DG levels);
# * every continuous level is smoothed by the same Chebyshev-Jacobi
#   polynomial as the DG levels (its own diagonal and Lanczos estimate); the
#   coarsest is solved directly in FP64 when it has at most `direct_max`
#   unknowns (for the pure-Neumann Poisson problem with the operator plus
#   mean(diag) 1 1^T / n, whose inverse is the pseudo-inverse on mean-zero
#   vectors) when it is of degree 1 (the hierarchy reaches degree 1 unless
#   `max_levels` cuts it short) and has at most `direct_max` unknowns, else
#   approximated by the Chebyshev-Jacobi polynomial of degree `coarse_degree`.

def gll_points(j: int) -> np.ndarray:
    """The j + 1 Gauss-Lobatto-Legendre points of [0, 1]: the end points and
    the roots of P_j' (ascending)."""
    if j == 1:
        return np.array([0.0, 1.0])
    c = np.zeros(j + 1)
    c[-1] = 1.0
    inner = np.polynomial.legendre.legroots(np.polynomial.legendre.legder(c))
    return np.concatenate([[0.0], (np.sort(inner) + 1.0) / 2.0, [1.0]])


def cg_shape(mesh: Mesh, j: int) -> tuple[int, int, int]:
    """Nodes per direction of the continuous Q_j space on `mesh`."""
    return j * mesh.nx + 1, j * mesh.ny + 1, j * mesh.nz + 1


def cg_ndof(level: Problem) -> int:
    Mx, My, Mz = cg_shape(level.mesh, level.degree)
    return level.C * Mx * My * Mz


def cg_embedding(level: Problem) -> sp.csr_matrix:
    """G (level.ndof x cg_ndof): continuous Q_j values (index
    c*Mx*My*Mz + (gz*My + gy)*Mx + gx, node g = j*cell + local index) ->
    the level's DG_j values at the Gauss nodes of every cell."""
    j, n, C, mesh = level.degree, level.n, level.C, level.mesh
    Mx, My, Mz = cg_shape(mesh, j)
    nv = Mx * My * Mz
    L = lagrange_values(gll_points(j), gauss_points(n)[0])          # (Gauss q, Lobatto a)
    loc = _kron3(L, L, L)                                            # (q3 q2 q1, a3 a2 a1)
    a3, a2, a1 = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    a1, a2, a3 = a1.ravel(), a2.ravel(), a3.ravel()
    R, Cc = np.meshgrid(np.arange(n ** 3), np.arange(n ** 3), indexing="ij")
    R, Cc = R.ravel(), Cc.ravel()
    rows, cols, vals = [], [], []
    for e in range(mesh.ncells):
        ex, ey, ez = (int(v[0]) for v in mesh.cell_ijk(np.array([e])))
        g = ((ez * j + a3) * My + ey * j + a2) * Mx + ex * j + a1      # global node of each local one
        for c in range(C):
            rows.append((e * C + c) * n ** 3 + R)
            cols.append(c * nv + g[Cc])
            vals.append(loc.ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(level.ndof, C * nv))


def _cg_1d(ncell: int, jf: int, jc: int, mesh_step: bool) -> np.ndarray:
    """1D prolongation between continuous nodal spaces along one direction."""
    if mesh_step:                          # degree 1: fine vertex 2i <- i, 2i+1 <- (i + i+1)/2
        R = np.zeros((2 * ncell + 1, ncell + 1))
        for i in range(2 * ncell + 1):
            if i % 2 == 0:
                R[i, i // 2] = 1.0
            else:
                R[i, i // 2] = R[i, i // 2 + 1] = 0.5
        return R
    L = lagrange_values(gll_points(jc), gll_points(jf))              # (fine a, coarse b)
    R = np.zeros((jf * ncell + 1, jc * ncell + 1))
    for e in range(ncell):
        R[e * jf:e * jf + jf + 1, e * jc:e * jc + jc + 1] = L
    return R


def cg_prolongation(fine: Problem, coarse: Problem) -> sp.csr_matrix:
    """Continuous Q_coarse -> Q_fine: a degree step on the same mesh (the
    coarse Lobatto interpolant at the fine Lobatto nodes of each cell) or a
    mesh step at degree 1 (the coarse trilinear function at the fine
    vertices in the coarse cell's reference coordinates)."""
    step = fine.mesh.ncells != coarse.mesh.ncells
    m = coarse.mesh
    R = [_cg_1d(nc, fine.degree, coarse.degree, step) for nc in (m.nx, m.ny, m.nz)]
    return sp.block_diag([sp.csr_matrix(_kron3(R[2], R[1], R[0]))] * fine.C, format="csr")


def _mean_zero(pb: Problem) -> bool:
    return pb.op == "poisson" and pb.alpha == 0.0 and all(b == "N" for b in pb.mesh.bc)


class CphHierarchy:
    """The DG level, then the continuous levels with their Galerkin
    operators, inverse diagonals, Chebyshev intervals, prolongations and the
    coarsest level's direct inverse."""

    def __init__(self, pb: Problem, smooth_degree: int = 5, coarse_degree: int = 12,
                 h_coarsen: bool = True, min_cells: int = 2, max_levels: int = 16,
                 ratio: float = 20.0, safety: float = 1.2, lanczos_steps: int = 20,
                 seed: int = 12345, direct_max: int = 1024, levels: list[Problem] | None = None):
        self.pb = pb
        self.carriers = levels if levels is not None else level_problems(pb, h_coarsen, min_cells, max_levels)
        self.smooth_degree, self.coarse_degree = smooth_degree, coarse_degree
        self.G = cg_embedding(self.carriers[0])
        self.A = []
        for c in self.carriers:
            Gc = cg_embedding(c)
            self.A.append((Gc.T @ assemble(c, ("cell", "boundary")) @ Gc).tocsr())
        self.P = [cg_prolongation(self.carriers[i], self.carriers[i + 1])
                  for i in range(len(self.carriers) - 1)]
        self.top_op = lambda x: op_apply(pb, x)
        self.top_dinv = 1.0 / diagonal(pb)
        self.dinv = [1.0 / A.diagonal() for A in self.A]
        lam = lanczos_max(self.top_op, self.top_dinv, lanczos_steps, seed)
        self.top_interval = (safety * lam, safety * lam / ratio)
        self.lam = [lanczos_max(lambda v, A=A: A @ v, d, lanczos_steps, seed) for A, d in zip(self.A, self.dinv)]
        self.interval = [(safety * l, safety * l / ratio) for l in self.lam]
        Ac = self.A[-1]
        self.direct = self.carriers[-1].degree == 1 and Ac.shape[0] <= direct_max
        if self.direct:
            M = Ac.toarray()
            if _mean_zero(pb):
                M = M + np.mean(np.diag(M)) * np.ones_like(M) / M.shape[0]
            self.coarse_inverse = np.linalg.inv(M)

    def smooth(self, l: int, r: np.ndarray, degree: int) -> np.ndarray:
        hi, lo = self.interval[l]
        return chebyshev_jacobi(lambda v: self.A[l] @ v, self.dinv[l], r, degree, hi, lo)

    def cg_vcycle(self, r: np.ndarray, l: int = 0) -> np.ndarray:
        """z ~ A_l^-1 r on continuous level l by one V-cycle from zero."""
        if l == len(self.A) - 1:
            if self.direct:
                return self.coarse_inverse @ r
            return self.smooth(l, r, self.coarse_degree)
        A = self.A[l]
        z = self.smooth(l, r, self.smooth_degree)
        z = z + self.P[l] @ self.cg_vcycle(self.P[l].T @ (r - A @ z), l + 1)
        return z + self.smooth(l, r - A @ z, self.smooth_degree)

    def vcycle(self, r: np.ndarray) -> np.ndarray:
        """One V-cycle from zero on the DG level: Chebyshev-Jacobi smoothing
        on the DG operator around the correction from the continuous levels."""
        hi, lo = self.top_interval
        sm = lambda v: chebyshev_jacobi(self.top_op, self.top_dinv, v, self.smooth_degree, hi, lo)
        z = sm(r)
        z = z + self.G @ self.cg_vcycle(self.G.T @ (r - self.top_op(z)))
        return z + sm(r - self.top_op(z))
