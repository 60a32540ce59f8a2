"""Geometric hp-multigrid V-cycle used as the preconditioner of the FP64 CG
(Sec. 5.3, paragraph on preconditioning the viscous terms).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 5.3 builds the hierarchy by lowering the polynomial degree recursively
from k to k-1 and then coarsening the mesh, smooths every level with
Chebyshev-accelerated Jacobi on that level's inverse diagonal and operator
action, runs standard V-cycles, and keeps the viscosity at the integration
points of every level.  Readings taken here (the paper's own hierarchy first
converts the DG space to a continuous one and solves the coarsest level with
AMG cycles or a direct solver):

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
from .forms import Problem, apply as op_apply, diagonal
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
