"""Pins of the oracle's Picard viscosity update (Sec. 4.1, eq.
viscosity_pointwise) and Aitken-relaxed fixed-point iteration (Sec. 5.1,
Alg. 1): closed-form shear rates of polynomial velocities on every multigrid
level, the face-averaging reading on a piecewise-linear field, the law at
zero shear, the face numbering, the pointwise-table path of the forms, the
relaxation formula's two-step exactness on linear problems, the Newtonian
limit, and the fixed point checked by a direct solve."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import multigrid as MG
from oracle import picard as PC
from oracle.basis import cell_points, face_points
from oracle.forms import Problem, apply, assemble, interpolate, _cell_geo, _face_geo
from oracle.laws import generalized_newtonian, viscosity
from oracle.mesh import Mesh


def test_face_numbering_is_a_bijection():
    m = Mesh(3, 2, 4)
    seen = []
    for d in range(3):
        em, ep = m.interior_faces(d)
        a, b = m.face_index(d, em, 1), m.face_index(d, ep, 0)
        assert np.array_equal(a, b)                    # both cells name the same face
        seen.append(a)
        for side in (0, 1):
            seen.append(m.face_index(d, m.boundary_cells(d, side), side))
    allf = np.sort(np.concatenate(seen))
    assert np.array_equal(allf, np.arange(m.nfaces))


def test_pointwise_table_equals_the_law():
    """Tabulating the law at every cell and face point and passing the table
    reproduces the law's operator exactly (pins the table indexing)."""
    m = Mesh(3, 2, 2, W.box_vertices(3, 2, 2, 0.1), ("D", "N", "D", "D", "N", "D"))
    law = W.sine_law(1.0, 0.5)
    pb = Problem(m, 2, "viscous", 3.0, 1.0, law)
    n = pb.n
    mu_c = viscosity(law, _cell_geo(pb, np.arange(m.ncells))[0])
    mu_f = np.zeros((m.nfaces, n * n))
    for d in range(3):
        for side in (0, 1):
            cells = np.arange(m.ncells)
            _, xq, _, _, _ = _face_geo(pb, cells, d, side)
            mu_f[m.face_index(d, cells, side)] = viscosity(law, xq)
    tab = Problem(m, 2, "viscous", 3.0, 1.0, {"kind": "const", "mu": 123.0}, mu_values=(mu_c, mu_f))
    x = W.uniform_vector(2, pb.ndof)
    ref = apply(pb, x)
    assert np.abs(apply(tab, x) - ref).max() <= 1e-13 * np.abs(ref).max()
    A, At = assemble(pb), assemble(tab)
    assert abs(A - At).max() <= 1e-13 * abs(A).max()


def _levels(pb):
    return MG.level_problems(pb, min_cells=1)


def test_shear_rate_of_a_linear_field_on_every_level():
    """u = G x + c lies in the space on trilinear cells: gdot =
    sqrt(2 eps:eps) of the constant sym(G) at every point of every level."""
    m = Mesh(4, 4, 4, W.box_vertices(4, 4, 4, 0.1))
    pb = Problem(m, 2, "viscous", 10.0, 1.0, W.carreau_law(3))
    G = np.array([[0.3, -1.2, 0.5], [0.7, 0.1, -0.4], [0.2, 0.9, -0.6]])
    u = interpolate(pb, lambda X: X @ G.T + np.array([1.0, 2.0, 3.0]))
    E = 0.5 * (G + G.T)
    expect = np.sqrt(2.0 * np.sum(E * E))
    levels = _levels(pb)
    assert [(p.degree, p.mesh.nx) for p in levels] == [(2, 4), (1, 4), (1, 2), (1, 1)]
    for L in levels:
        gc, gf = PC.shear_rate_values(L, pb, u)
        assert gc.shape == (L.mesh.ncells, L.n ** 3) and gf.shape == (L.mesh.nfaces, L.n ** 2)
        assert np.abs(gc - expect).max() <= 1e-12 and np.abs(gf - expect).max() <= 1e-12


def test_rigid_motion_has_zero_shear_and_the_zero_shear_viscosity():
    m = Mesh(2, 3, 2, W.box_vertices(2, 3, 2, 0.1))
    law = W.carreau_law(3)
    pb = Problem(m, 3, "viscous", 10.0, 1.0, law)
    w = np.array([0.4, -1.1, 0.7])
    u = interpolate(pb, lambda X: np.cross(w, X) + np.array([0.5, 0.0, -2.0]))
    mc, mf = PC.viscosity_values(pb, pb, u, law)
    eta0 = law["mu_inf"] + (law["mu0"] - law["mu_inf"]) * law["kappa"] ** ((law["n_exp"] - 1) / law["a_exp"])
    assert np.abs(mc - eta0).max() <= 1e-12 and np.abs(mf - eta0).max() <= 1e-12


def test_shear_rate_of_a_quadratic_field_at_the_level_points():
    """u = (y^2, x z, 0) on a straight mesh: gdot = sqrt((2y + z)^2 + x^2)
    at the physical position of every cell and face point of every level
    (pins where a coarse point lands among the fine cells)."""
    m = Mesh(4, 2, 4)
    pb = Problem(m, 2, "viscous", 1.0, 1.0, W.carreau_law(3))
    u = interpolate(pb, lambda X: np.stack([X[:, 1] ** 2, X[:, 0] * X[:, 2], 0 * X[:, 0]], axis=1))
    exact = lambda X: np.sqrt((2 * X[..., 1] + X[..., 2]) ** 2 + X[..., 0] ** 2)
    for L in MG.level_problems(pb, min_cells=1):
        gc, gf = PC.shear_rate_values(L, pb, u)
        lm, n = L.mesh, L.n
        pts, _ = cell_points(n)
        assert np.abs(gc - exact(lm.map(np.arange(lm.ncells), pts))).max() <= 1e-12
        for d in range(3):
            for side in (0, 1):
                cells = np.arange(lm.ncells)
                fp, _ = face_points(n, d, side)
                ref = exact(lm.map(cells, fp))
                assert np.abs(gf[lm.face_index(d, cells, side)] - ref).max() <= 1e-12


def test_face_shear_rate_averages_the_two_traces():
    """Piecewise-linear velocity with a different gradient G_e per cell:
    cell points see sym(G_e); an interior face point the mean of the two
    cells' symmetric gradients; a boundary face point its cell's."""
    m = Mesh(3, 2, 2, W.box_vertices(3, 2, 2, 0.1))
    pb = Problem(m, 1, "viscous", 1.0, 1.0, W.carreau_law(3))
    rng = np.random.default_rng(3)
    Gs = rng.uniform(-1, 1, (m.ncells, 3, 3))
    pts, _ = cell_points(pb.n)
    X = m.map(np.arange(m.ncells), pts)                       # (E, n^3, 3)
    u = np.einsum("eij,epj->eip", Gs, X).reshape(-1)          # layout (e, c, node)
    sym = 0.5 * (Gs + np.swapaxes(Gs, 1, 2))
    gd = lambda E: np.sqrt(2.0 * np.einsum("...ij,...ij->...", E, E))
    gc, gf = PC.shear_rate_values(pb, pb, u)
    assert np.abs(gc - gd(sym)[:, None]).max() <= 1e-12
    for d in range(3):
        em, ep = m.interior_faces(d)
        ref = gd(0.5 * (sym[em] + sym[ep]))
        assert np.abs(gf[m.face_index(d, em, 1)] - ref[:, None]).max() <= 1e-12
        for side in (0, 1):
            bc = m.boundary_cells(d, side)
            assert np.abs(gf[m.face_index(d, bc, side)] - gd(sym[bc])[:, None]).max() <= 1e-12


@pytest.mark.parametrize("n", [1, 5])
def test_aitken_relaxation_solves_a_linear_problem_in_two_steps(n):
    """R(u) = b - a u with the correction s R, s a wrong scale: plain
    iteration contracts by |1 - a s| per step; the relaxed one lands on
    b / a at the second step (omega_1 = 1 / (a s))."""
    a, s = 3.0, 0.1
    b = np.linspace(1.0, 2.0, n)
    res = lambda u: b - a * u
    sol = lambda u, R: s * R
    u, info = PC.relaxed_fixed_point(res, sol, np.zeros(n), 1e-14, 0.0, 10, aitken=True)
    assert info["iterations"] == 2 and info["status"] == "ok"
    assert abs(info["omegas"][1] - 1.0 / (a * s)) <= 1e-14
    assert np.abs(u - b / a).max() <= 1e-14
    _, plain = PC.relaxed_fixed_point(res, sol, np.zeros(n), 1e-6, 0.0, 100, aitken=False)
    assert plain["iterations"] == int(np.ceil(np.log(1e-6) / np.log(1 - a * s)))


def _direct(pbk, R):
    return spla.spsolve(assemble(pbk).tocsc(), R)


def test_newtonian_limit_converges_in_one_iteration():
    """Flow index b = 1: eta = eta_0 whatever the shear, so the first
    linear solve is already the solution."""
    m = Mesh(2, 2, 2, W.box_vertices(2, 2, 2, 0.1))
    law = dict(W.carreau_law(3), n_exp=1.0)
    pb = Problem(m, 2, "viscous", 10.0, 1.0, law)
    b = W.uniform_vector(7, pb.ndof)
    u, info = PC.picard_solve(pb, law, b, np.zeros(pb.ndof), _direct, rel_tol=1e-10)
    assert info["iterations"] == 1 and info["status"] == "ok"
    const = Problem(m, 2, "viscous", 10.0, 1.0, {"kind": "const", "mu": law["mu0"]})
    ref = _direct(const, b)
    assert np.abs(u - ref).max() <= 1e-10 * np.abs(ref).max()


def test_shear_thinning_fixed_point():
    """Carreau with b = 0.5: plain and relaxed iterations reach the same
    velocity, which solves the linear problem of its own viscosity; the
    relaxed one needs fewer iterations on this case."""
    m = Mesh(2, 2, 2, W.box_vertices(2, 2, 2, 0.1))
    law = W.carreau_law(3)
    pb = Problem(m, 2, "viscous", 10.0, 1.0, law)
    b = W.uniform_vector(7, pb.ndof) * 100.0 * 10.0 / (8 * 27)
    u1, i1 = PC.picard_solve(pb, law, b, np.zeros(pb.ndof), _direct, rel_tol=1e-10, max_iter=60, aitken=True)
    u0, i0 = PC.picard_solve(pb, law, b, np.zeros(pb.ndof), _direct, rel_tol=1e-10, max_iter=60, aitken=False)
    assert i1["status"] == "ok" and i0["status"] == "ok"
    assert i1["iterations"] < i0["iterations"]
    assert np.abs(u1 - u0).max() <= 1e-8 * np.abs(u0).max()
    mu = PC.viscosity_values(pb, pb, u1, law)
    assert mu[0].min() < 0.5 * mu[0].max()                 # the viscosity really varies
    fixed = _direct(Problem(m, 2, "viscous", 10.0, 1.0, law, mu_values=mu), b)
    assert np.abs(fixed - u1).max() <= 1e-8 * np.abs(u1).max()
