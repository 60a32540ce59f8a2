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


# ------------------------------------------------ continuous (cph) levels ---

def test_gll_points_closed_forms():
    """Gauss-Lobatto points on [0, 1]: end points and the roots of P_j'
    (j = 2: 1/2; j = 3: (1 -+ 1/sqrt 5)/2; j = 4: 1/2, (1 -+ sqrt(3/7))/2)."""
    assert np.allclose(MG.gll_points(1), [0, 1])
    assert np.allclose(MG.gll_points(2), [0, 0.5, 1], atol=1e-15)
    s5 = 1 / np.sqrt(5)
    assert np.allclose(MG.gll_points(3), [0, (1 - s5) / 2, (1 + s5) / 2, 1], atol=1e-15)
    s = np.sqrt(3 / 7)
    assert np.allclose(MG.gll_points(4), [0, (1 - s) / 2, 0.5, (1 + s) / 2, 1], atol=1e-15)


def _face_jumps(pb, u):
    """Largest difference of the two cells' traces at the Gauss points of
    every interior face (the DG function's discontinuity)."""
    from oracle.basis import face_points, tensor_tables
    X = u.reshape(pb.mesh.ncells, pb.C, -1)
    worst = 0.0
    for d in range(3):
        em, ep = pb.mesh.interior_faces(d)
        Vm, _ = tensor_tables(pb.n, face_points(pb.n, d, 1)[0])
        Vp, _ = tensor_tables(pb.n, face_points(pb.n, d, 0)[0])
        tm = np.einsum("pj,ecj->epc", Vm, X[em])
        tp = np.einsum("pj,ecj->epc", Vp, X[ep])
        worst = max(worst, float(np.abs(tm - tp).max()))
    return worst


@pytest.mark.parametrize("deg", [1, 2, 3])
def test_cg_embedding_gives_continuous_functions(deg):
    """G maps any vector of Lobatto-node values to a DG function whose traces
    agree on every interior face (curved mesh, 3 components); a DG function
    of random nodal values does not."""
    pb = Problem(Mesh(3, 2, 2, W.box_vertices(3, 2, 2, 0.1)), deg, "viscous", 1.0, 1.0, W.const_law(1.0))
    G = MG.cg_embedding(pb)
    u = np.random.default_rng(deg).uniform(-1, 1, G.shape[1])
    assert _face_jumps(pb, G @ u) <= 1e-13
    assert _face_jumps(pb, np.random.default_rng(9).uniform(-1, 1, pb.ndof)) > 1e-2


@pytest.mark.parametrize("deg", [1, 2, 3])
def test_cg_embedding_reproduces_polynomials(deg):
    """On an affine mesh a global polynomial of degree <= deg per variable is
    in the continuous space: its Lobatto-node values embed to its values at
    every cell's Gauss nodes."""
    pb = Problem(Mesh(2, 3, 2), deg, "poisson", 0.0, 1.0)
    f = _poly(deg, 1, deg)
    Mx, My, Mz = MG.cg_shape(pb.mesh, deg)
    t = [np.concatenate([e + MG.gll_points(deg)[:-1] for e in range(m)] + [[m]]) / m
         for m in (pb.mesh.nx, pb.mesh.ny, pb.mesh.nz)]
    Z, Y, X = np.meshgrid(t[2], t[1], t[0], indexing="ij")
    nodes = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    assert len(nodes) == Mx * My * Mz
    assert np.abs(MG.cg_embedding(pb) @ f(nodes) - interpolate(pb, f)).max() <= 1e-12


@pytest.mark.parametrize("step", ["degree", "mesh"])
def test_cg_transfers_commute_with_dg_transfers(step):
    """Embedding then DG prolongation equals continuous prolongation then
    embedding: G_f P_cg = P_dg G_c, for a degree step (3 -> 2) and a mesh
    step (degree 1, 4^3 -> 2^3 cells) on a curved mesh."""
    pb = Problem(Mesh(4, 4, 4, W.box_vertices(4, 4, 4, 0.1)), 3, "viscous", 1.0, 1.0, W.const_law(1.0))
    L = MG.level_problems(pb, min_cells=2)
    f, c = (L[0], L[1]) if step == "degree" else (L[2], L[3])
    assert (f.mesh.ncells != c.mesh.ncells) == (step == "mesh")
    lhs = MG.cg_embedding(f) @ MG.cg_prolongation(f, c)
    rhs = MG.prolongation(f, c) @ MG.cg_embedding(c)
    assert abs(lhs - rhs).max() <= 1e-13


def test_cg_operator_is_the_sipg_form_on_continuous_functions():
    """For continuous functions every interior-face term of the SIPG form
    vanishes: G^T A G with the whole operator equals the cell-and-boundary
    operator the continuous levels use (viscous, curved, variable viscosity;
    Poisson with mixed conditions)."""
    from oracle.forms import assemble
    for pb in (Problem(Mesh(3, 2, 2, W.box_vertices(3, 2, 2, 0.1)), 2, "viscous", 2.0, 1.0, W.logfield_law(2, 1e2)),
               Problem(Mesh(2, 3, 2, None, ("D", "N", "N", "D", "N", "N")), 3, "poisson", 0.0, 1.0)):
        G = MG.cg_embedding(pb)
        full = (G.T @ assemble(pb) @ G).toarray()
        part = (G.T @ assemble(pb, ("cell", "boundary")) @ G).toarray()
        assert np.abs(full - part).max() <= 1e-12 * np.abs(full).max()


def _vcycle_matrix(H, n):
    return np.column_stack([H.vcycle(e) for e in np.eye(n)])


def test_cph_vcycle_is_spd_and_beats_the_dg_hierarchy():
    """The cph V-cycle (DG smoothing, continuous levels, direct coarse
    solve) is a symmetric positive definite operator, and with the
    surface-to-volume penalty it needs far fewer CG iterations than the
    all-DG hierarchy on a curved high-contrast problem."""
    pb = Problem(Mesh(2, 1, 1, W.box_vertices(2, 1, 1, 0.1)), 2, "viscous", 10.0, 1.0, W.logfield_law(2, 1e3))
    H = MG.CphHierarchy(pb, smooth_degree=3, min_cells=1)
    assert H.direct
    M = _vcycle_matrix(H, pb.ndof)
    assert np.abs(M - M.T).max() <= 1e-10 * np.abs(M).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T))[0] > 0
    pb = Problem(Mesh(2, 2, 2, W.box_vertices(2, 2, 2, 0.1)), 3, "viscous", 10.0, 1.0, W.logfield_law(2, 1e3))
    A = lambda v: apply(pb, v)
    b = W.uniform_vector(3, pb.ndof)
    Hc = MG.CphHierarchy(pb, smooth_degree=4, min_cells=1)
    Hd = MG.Hierarchy(pb, smooth_degree=4, min_cells=1)
    d = 1.0 / Hd.dinv[0]
    _, ic = solve(A, d, b, tol=1e-8, precond=Hc.vcycle)
    _, idg = solve(A, d, b, tol=1e-8, precond=Hd.vcycle)
    assert ic["status"] == "ok" and ic["iterations"] <= 10 and ic["iterations"] < idg["iterations"] / 2, (ic, idg)


def test_cph_coarse_direct_solve_pure_neumann():
    """The coarsest continuous level of the pure-Neumann Poisson problem is
    singular (constants); its direct inverse is that of the operator plus
    mean(diag) 1 1^T / n, which solves A z = r for every mean-zero r, and the
    whole cph V-cycle keeps mean-zero vectors' solves converging."""
    pb = Problem(Mesh(4, 4, 4, None, ("N",) * 6), 2, "poisson", 0.0, 1.0)
    H = MG.CphHierarchy(pb, smooth_degree=3)
    Ac = H.A[-1].toarray()
    assert np.abs(Ac @ np.ones(len(Ac))).max() <= 1e-12 * np.abs(Ac).max()
    r = np.random.default_rng(1).uniform(-1, 1, len(Ac))
    r -= r.mean()
    z = H.coarse_inverse @ r
    assert np.abs(Ac @ z - r).max() <= 1e-10 * np.abs(r).max()
    b = W.uniform_vector(4, pb.ndof)
    _, info = solve(lambda v: apply(pb, v), 1.0 / H.top_dinv, b, tol=1e-8, precond=H.vcycle, mean_zero=True)
    assert info["status"] == "ok" and info["iterations"] <= 12, info
