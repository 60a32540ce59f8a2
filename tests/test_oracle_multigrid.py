"""Pins of the oracle's hp-multigrid preconditioner (Sec. 5.3: degree lowered
from k to k-1, then mesh coarsening, Chebyshev-Jacobi smoothing, V-cycles),
checked against what the definitions fix rather than against the oracle
itself: the transfers embed coarse functions exactly, restriction is the
adjoint of prolongation, the V-cycle is a symmetric positive definite
operator, and it preconditions better than one-level Chebyshev-Jacobi."""
import numpy as np
import pytest

import workloads as W
from oracle import multigrid as MG
from oracle.forms import Problem, apply, interpolate
from oracle.mesh import Mesh
from oracle.solvers import solve


def _poly(deg, C, seed):
    """A random tensor polynomial of degree <= deg per variable, C components."""
    rng = np.random.default_rng(seed)
    coef = rng.standard_normal((C, deg + 1, deg + 1, deg + 1))

    def f(x):
        out = np.zeros((len(x), C))
        for c in range(C):
            for a in range(deg + 1):
                for b in range(deg + 1):
                    for d in range(deg + 1):
                        out[:, c] += coef[c, a, b, d] * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** d
        return out if C > 1 else out[:, 0]
    return f


def test_hierarchy_lowers_degree_then_coarsens_mesh():
    pb = Problem(Mesh(8, 8, 4), 3, "viscous", 1.0, 1.0, {"kind": "const", "mu": 1.0})
    L = MG.level_problems(pb, min_cells=2)
    assert [(p.degree, p.mesh.nx, p.mesh.ny, p.mesh.nz) for p in L] == \
        [(3, 8, 8, 4), (2, 8, 8, 4), (1, 8, 8, 4), (1, 4, 4, 2)]
    # an odd cell count stops the mesh coarsening
    assert len(MG.level_problems(Problem(Mesh(6, 6, 6), 2), min_cells=2)) == 3   # 2, 1 on 6^3, 1 on 3^3
    assert len(MG.level_problems(Problem(Mesh(5, 4, 4), 2))) == 2


@pytest.mark.parametrize("op", ["viscous", "poisson"])
def test_p_prolongation_embeds_coarse_polynomials(op):
    """DG_{k-1} is a subspace of DG_k: prolongating the interpolant of a
    polynomial of degree k-1 gives the fine interpolant of the same polynomial."""
    mesh = Mesh(2, 3, 2, W.box_vertices(2, 3, 2, 0.1))
    fine, coarse = Problem(mesh, 4, op), Problem(mesh, 3, op)
    f = _poly(3, fine.C, 1)
    P = MG.prolongation(fine, coarse)
    assert P.shape == (fine.ndof, coarse.ndof)
    np.testing.assert_allclose(P @ interpolate(coarse, f), interpolate(fine, f), rtol=0, atol=1e-11)


@pytest.mark.parametrize("deg", [1, 2])
def test_h_prolongation_embeds_coarse_mesh_polynomials(deg):
    """On straight cells a polynomial of degree k is represented exactly on
    both meshes: prolongation maps the coarse-mesh interpolant to the
    fine-mesh one (fixes the child numbering and the parent coordinates)."""
    fine = Problem(Mesh(4, 2, 6), deg, "viscous")
    coarse = Problem(Mesh(2, 1, 3), deg, "viscous")
    f = _poly(deg, 3, 2)
    P = MG.prolongation(fine, coarse)
    np.testing.assert_allclose(P @ interpolate(coarse, f), interpolate(fine, f), rtol=0, atol=1e-11)


def test_h_prolongation_of_one_cell_function():
    """A function supported on one coarse cell is supported on its 8 children
    only, and there it is the same polynomial in the parent's coordinates."""
    fine, coarse = Problem(Mesh(4, 4, 4), 1, "poisson"), Problem(Mesh(2, 2, 2), 1, "poisson")
    xc = np.zeros(coarse.ndof)
    xc[5 * 8:6 * 8] = np.arange(1.0, 9.0)          # coarse cell 5 = (1, 0, 1)
    xf = (MG.prolongation(fine, coarse) @ xc).reshape(64, 8)
    support = sorted(np.nonzero(np.abs(xf).sum(1))[0])
    children = sorted(((2 * 1 + cz) * 4 + (2 * 0 + cy)) * 4 + 2 * 1 + cx
                      for cx in (0, 1) for cy in (0, 1) for cz in (0, 1))
    assert support == children


def test_vcycle_is_symmetric_positive_definite():
    """Equal pre- and post-smoothing polynomials and a fixed coarsest
    polynomial make the V-cycle a symmetric operator; it is positive
    definite on an SPD problem."""
    cfg = W.config("c1")
    H = MG.Hierarchy(Problem.from_config(cfg), smooth_degree=3, coarse_degree=8)
    rng = np.random.default_rng(3)
    r1, r2 = rng.standard_normal((2, H.levels[0].ndof))
    a, b = H.vcycle(r1) @ r2, r1 @ H.vcycle(r2)
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))
    for r in (r1, r2):
        assert H.vcycle(r) @ r > 0


def test_vcycle_preconditions_better_than_one_level_chebyshev():
    """Curved 4^3 cells, k = 3, viscosity contrast 1e3 (levels k = 3, 2, 1 on
    4^3, k = 1 on 2^3): the V-cycle cuts the CG iterations to well under half
    of one-level Chebyshev-Jacobi's, and the solve reaches the tolerance."""
    cfg = W.config("c2")
    cfg.update(nx=4, ny=4, nz=4)
    V = W.box_vertices(4, 4, 4, cfg["perturb"])
    pb = Problem.from_config(cfg, V)
    A = lambda x: apply(pb, x)
    b = W.uniform_vector(2, pb.ndof)
    H = MG.Hierarchy(pb, smooth_degree=3, coarse_degree=12)
    _, cheb = solve(A, 1.0 / H.dinv[0], b, tol=1e-6)
    x, mg = solve(A, 1.0 / H.dinv[0], b, tol=1e-6, precond=H.vcycle)
    assert cheb["status"] == "ok" and mg["status"] == "ok"
    assert np.linalg.norm(b - A(x)) <= 1e-6 * np.linalg.norm(b) * 1.0001
    assert mg["iterations"] < 0.5 * cheb["iterations"], (mg, cheb)
