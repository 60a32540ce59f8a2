"""Pins of the CPU oracle against facts that do not come from the oracle itself:
exactness of quadrature, closed-form energies, null spaces, symmetry and
definiteness of SIPG (Sec. 4.1 calls both forms symmetric interior penalty),
reproduction of discrete solutions (Galerkin consistency), the patch test on
curved cells, the relation between the viscous and the Poisson form for
constant viscosity, the optimal order k+1 (Sec. 6.1), a brute-force
recomputation of matrix entries, and published values of the random
generator.  All CPU only.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import sympy as sy

import workloads as W
from oracle import solvers
from oracle.basis import gauss_points, lagrange_values, lagrange_derivatives
from oracle.forms import (Problem, apply, assemble, diagonal, interpolate, l2_error,
                          load_vector, cell_sizes)
from oracle.laws import viscosity, shear_rate_of_modes
from oracle.mesh import Mesh

pytestmark = pytest.mark.filterwarnings("ignore::scipy.sparse.SparseEfficiencyWarning")


def jittered_vertices(n, amp, seed=7):
    """Unit-cube vertices with interior vertices moved randomly by up to amp*h."""
    t = np.linspace(0, 1, n + 1)
    Z, Y, X = np.meshgrid(t, t, t, indexing="ij")
    V = np.stack([X, Y, Z], -1)
    rng = np.random.default_rng(seed)
    d = rng.uniform(-amp / n, amp / n, size=V.shape)
    inner = np.zeros(V.shape[:3], bool)
    inner[1:-1, 1:-1, 1:-1] = True
    V[inner] += d[inner]
    return V.reshape(-1, 3)


# ---------------------------------------------------------------- basis ---

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_gauss_rule_exact_to_degree_2n_minus_1(n):
    x, w = gauss_points(n)
    for m in range(2 * n):
        assert abs(w @ x ** m - 1.0 / (m + 1)) < 1e-14
    assert abs(w @ x ** (2 * n) - 1.0 / (2 * n + 1)) > 1e-8


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_lagrange_cardinal_and_derivative_vs_polyfit(n):
    x, _ = gauss_points(n)
    assert np.allclose(lagrange_values(x, x), np.eye(n), atol=1e-14)
    t = np.linspace(-0.3, 1.2, 17)
    D = lagrange_derivatives(x, t)
    V = lagrange_values(x, t)
    for j in range(n):
        e = np.zeros(n); e[j] = 1.0
        c = np.polyfit(x, e, n - 1)
        assert np.allclose(V[:, j], np.polyval(c, t), atol=1e-10)
        assert np.allclose(D[:, j], np.polyval(np.polyder(c), t), atol=1e-9)


# ------------------------------------------------- structural properties ---

def _problems():
    return [
        Problem(Mesh(3, 3, 3, W.box_vertices(3, 3, 3, 0.1)), 2, "viscous", 10.0, 1.0, W.logfield_law(2, 1e3)),
        Problem(Mesh(3, 3, 2, None, ("D", "N", "D", "D", "N", "D")),
                3, "viscous", 0.0, 1.0, W.sine_law()),
        Problem(Mesh(3, 3, 3, jittered_vertices(3, 0.25)), 2, "viscous", 1.0, 1.0, W.carreau_law(3)),
        Problem(Mesh(3, 3, 3, jittered_vertices(3, 0.25)), 3, "poisson", 0.0, 1.0),
        Problem(Mesh(2, 3, 2, None, ("N",) * 6), 4, "poisson", 0.0, 1.0),
    ]


@pytest.mark.parametrize("i", range(5))
def test_symmetric(i):
    pb = _problems()[i]
    A = assemble(pb)
    assert abs(A - A.T).max() <= 1e-14 * abs(A).max()
    rng = np.random.default_rng(i)
    u, v = rng.standard_normal(pb.ndof), rng.standard_normal(pb.ndof)
    assert abs(v @ apply(pb, u) - u @ apply(pb, v)) <= 1e-12 * np.linalg.norm(u) * np.linalg.norm(v) * abs(A).max()


@pytest.mark.parametrize("op,deg,alpha", [("viscous", 2, 0.0), ("viscous", 3, 5.0), ("poisson", 2, 0.0), ("poisson", 3, 0.0)])
def test_dirichlet_operator_is_positive_definite(op, deg, alpha):
    pb = Problem(Mesh(2, 2, 2, jittered_vertices(2, 0.0)), deg, op, alpha, 1.0, W.logfield_law(4, 1e2))
    ev = np.linalg.eigvalsh(assemble(pb).toarray())
    assert ev[0] > 1e-8 * ev[-1]


def test_neumann_poisson_annihilates_constants_on_curved_mesh():
    pb = Problem(Mesh(3, 3, 3, jittered_vertices(3, 0.25), ("N",) * 6), 3, "poisson", 0.0, 1.0)
    A = assemble(pb)
    assert np.abs(A @ np.ones(pb.ndof)).max() <= 1e-13 * abs(A).max()
    assert np.abs(apply(pb, np.ones(pb.ndof))).max() <= 1e-13 * abs(A).max()


def test_neumann_viscous_annihilates_rigid_motions_on_curved_mesh():
    """eps(u) = 0 and [u] = 0 for translations and rotations w x x, which lie in
    the mapped Q_k space because physical linear functions are trilinear in xi."""
    pb = Problem(Mesh(3, 3, 3, jittered_vertices(3, 0.25), ("N",) * 6), 2, "viscous", 0.0, 1.0,
                 W.logfield_law(1, 1e3))
    A = assemble(pb)
    scale = abs(A).max()
    modes = [lambda x, c=c: np.eye(3)[c][None, :].repeat(len(x), 0) for c in range(3)]
    for w in np.eye(3):
        modes.append(lambda x, w=w: np.cross(w[None, :], x))
    for m in modes:
        r = interpolate(pb, m)
        assert np.abs(A @ r).max() <= 1e-12 * scale * np.abs(r).max()
    # a stretching mode is not in the null space: a(u,u) = int 2 mu eps:eps = 2 mu |Omega| for u = (x,0,0)
    pbc = Problem(pb.mesh, 2, "viscous", 0.0, 1.0, W.const_law(0.7))
    u = interpolate(pbc, lambda x: np.stack([x[:, 0], 0 * x[:, 0], 0 * x[:, 0]], 1))
    assert abs(u @ apply(pbc, u) - 2 * 0.7) < 1e-12


def test_poisson_energy_of_linear_function_is_exact():
    pb = Problem(Mesh(3, 3, 3, jittered_vertices(3, 0.25), ("N",) * 6), 2, "poisson", 0.0, 1.0)
    p = interpolate(pb, lambda x: 2.0 * x[:, 1] - x[:, 2])
    assert abs(p @ apply(pb, p) - 5.0) < 1e-12    # int |(0, 2, -1)|^2 over the unit cube


def test_zero_viscosity_leaves_diagonal_mass_of_domain_volume():
    """mu = 0 => tau = 0 and A = alpha M; collocation at Gauss points makes M
    diagonal, and the entries of one component sum to alpha |Omega| = alpha."""
    pb = Problem(Mesh(3, 3, 3, jittered_vertices(3, 0.25)), 3, "viscous", 4.0, 1.0, W.const_law(0.0))
    A = assemble(pb).toarray()
    off = A - np.diag(np.diag(A))
    assert np.abs(off).max() <= 1e-14 * np.abs(A).max()
    d = np.diag(A).reshape(pb.mesh.ncells, 3, -1)
    for c in range(3):
        assert abs(d[:, c].sum() - 4.0) < 1e-12


def _indicator_energy(pb, cell, comp=0):
    u = np.zeros(pb.ndof)
    n3 = pb.n ** 3
    u[(cell * pb.C + comp) * n3:(cell * pb.C + comp + 1) * n3] = 1.0
    return u @ apply(pb, u)


@pytest.mark.parametrize("deg", [2, 3])
def test_penalty_energy_of_cell_indicator(deg):
    """Piecewise constant on one cell of an affine 3^3 mesh (h = 1/3, all
    Dirichlet): only the penalty survives, tau = (k+1)^2 mu sigma_F on each of
    the cell's six faces of area h^2 (interior faces tau [q]^2, Dirichlet faces
    2 tau q^2; viscous component c: (1 + n_c^2) times that).
    sigma_e with half-weighted interior faces: corner cell (3 boundary faces)
    4.5/h, centre cell 3/h, a centre cell's face neighbour (1 boundary face)
    3.5/h, an edge cell's neighbour along the edge 4/h.
      corner cell: every face takes max(4.5, 4)/h = 4.5/h;
        Poisson 3 tau h^2 + 3 * 2 tau h^2 = 40.5 (k+1)^2 h,
        viscous 4 tau h^2 + 8 tau h^2 = 54 (k+1)^2 mu h;
      centre cell: every face takes the neighbour's 3.5/h (the max; the min
        or either side's own value would give 3/h on some faces):
        Poisson 6 tau h^2 = 21 (k+1)^2 h, viscous 8 tau h^2 = 28 (k+1)^2 mu h."""
    N, h = 3, 1.0 / 3
    k2 = (deg + 1) ** 2
    pbp = Problem(Mesh(N, N, N), deg, "poisson", 0.0, 1.0)
    assert abs(_indicator_energy(pbp, 0) - 40.5 * k2 * h) < 1e-12
    assert abs(_indicator_energy(pbp, 13) - 21.0 * k2 * h) < 1e-12
    mu = 0.3
    pbv = Problem(Mesh(N, N, N), deg, "viscous", 0.0, 1.0, W.const_law(mu))
    for c in range(3):
        assert abs(_indicator_energy(pbv, 0, c) - 54.0 * k2 * mu * h) < 1e-12
        assert abs(_indicator_energy(pbv, 13, c) - 28.0 * k2 * mu * h) < 1e-12


@pytest.mark.parametrize("a", [0.7, 0.3])
def test_penalty_takes_the_larger_surface_to_volume_ratio_of_unequal_cells(a):
    """Two affine cells [0,a]x[0,1]^2 and [a,1]x[0,1]^2 (all Dirichlet).
    sigma of a cell of width w: (boundary x-face 1 + half the shared face 1/2
    + four boundary side faces 4w) / w.  An indicator of either cell sees
    tau_F = (k+1)^2 max(sigma_0, sigma_1) on the shared face and its own
    sigma on its five boundary faces (area 1 + 4w, factor 2):
      E_i = (k+1)^2 (max(sigma_0, sigma_1) + 2 sigma_i (1 + 4 w_i)).
    Both widths are tried so that the narrower (larger-sigma) cell is once
    the "-" and once the "+" cell: a one-sided choice, the minimum, or a
    penalty in terms of h_e = |e|^(1/3) all miss one of the four values."""
    deg = 2
    k2 = (deg + 1) ** 2
    V = Mesh(2, 1, 1).vertices.copy()
    V[:, :, 1, 0] = a
    pb = Problem(Mesh(2, 1, 1, V.reshape(-1, 3)), deg, "poisson", 0.0, 1.0)
    w = np.array([a, 1.0 - a])
    sig = (1.5 + 4 * w) / w
    for i in range(2):
        ref = k2 * (sig.max() + 2 * sig[i] * (1 + 4 * w[i]))
        assert abs(_indicator_energy(pb, i) - ref) < 1e-11 * ref
    # the alternatives differ from the pinned values by far more than the tolerance
    for i in range(2):
        ref = k2 * (sig.max() + 2 * sig[i] * (1 + 4 * w[i]))
        for alt in (sig.min(), sig[0], sig[1]):
            if alt != sig.max():
                assert abs(k2 * (alt + 2 * sig[i] * (1 + 4 * w[i])) - ref) > 1e-3 * ref


def test_constant_viscosity_reduces_to_laplacian():
    """Affine mesh, x/y sides Dirichlet, z sides Neumann, constant mu: for
    u = f e_3 and v = g e_3 with f, g independent of z,
    a(v, u) = mu a_p(g, f) + alpha (g, f)  (2 eps(f e3):eps(g e3) = grad f.grad g)."""
    N, deg, mu, alpha = 3, 2, 0.6, 3.0
    bc = ("D", "D", "D", "D", "N", "N")
    n = deg + 1
    pbv = Problem(Mesh(N, N, N, None, bc), deg, "viscous", alpha, 1.0, W.const_law(mu))
    pbp = Problem(Mesh(N, N, N, None, bc), deg, "poisson", alpha / mu, 1.0)
    rng = np.random.default_rng(3)

    def zindep():
        base = rng.standard_normal((N, N, n, n))          # (ey, ex, i2, i1)
        F = np.zeros((N, N, N, n, n, n))                  # (ez, ey, ex, i3, i2, i1)
        F[:] = base[None, :, :, None, :, :]
        return F.reshape(N ** 3, n ** 3)

    f, g = zindep(), zindep()
    uf = np.zeros((N ** 3, 3, n ** 3)); uf[:, 2] = f
    ug = np.zeros((N ** 3, 3, n ** 3)); ug[:, 2] = g
    lhs = ug.ravel() @ apply(pbv, uf.ravel())
    rhs = mu * (g.ravel() @ apply(pbp, f.ravel()))
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)


# --------------------------------------------------- consistency pins ---

X = sy.symbols("x y z")


def _visc_rhs(u, mu, alpha):
    """f = alpha u - div(2 mu eps(u)) symbolically."""
    G = sy.Matrix(3, 3, lambda i, j: sy.diff(u[i], X[j]))
    S = mu * (G + G.T)
    return [sy.simplify(alpha * u[i] - sum(sy.diff(S[i, j], X[j]) for j in range(3))) for i in range(3)]


def _vec_fn(exprs):
    fs = [sy.lambdify(X, e, "numpy") for e in exprs]
    return lambda P: np.stack([np.broadcast_to(f(P[:, 0], P[:, 1], P[:, 2]), (len(P),)) for f in fs], 1)


def _scal_fn(expr):
    f = sy.lambdify(X, expr, "numpy")
    return lambda P: np.broadcast_to(f(P[:, 0], P[:, 1], P[:, 2]), (len(P),)).copy()


@pytest.mark.parametrize("mu_expr", ["const", "multilinear"])
@pytest.mark.parametrize("deg", [2, 3])
def test_viscous_reproduces_polynomial_solution(mu_expr, deg):
    """u* in [Q_2]^3 vanishing on the boundary; with mu constant or multilinear
    every integrand is of degree <= 2k+1 per direction, so the discrete
    solution equals the interpolant of u* (Galerkin consistency)."""
    x, y, z = X
    b0 = x * (1 - x) * y * (1 - y) * z * (1 - z)
    u = [b0, 2 * b0, 3 * b0]
    mu = sy.Float(0.8) if mu_expr == "const" else 1 + x / 2 + y / 3 + z / 4 + x * y * z / 5
    alpha = 2.0
    f = _visc_rhs(u, mu, alpha)
    pb = Problem(Mesh(3, 2, 2), deg, "viscous", alpha, 1.0, _scal_fn(mu + 0 * x))
    A = assemble(pb)
    b = load_vector(pb, _vec_fn(f))
    sol = spla.spsolve(A.tocsc(), b)
    ref = interpolate(pb, _vec_fn(u))
    assert np.abs(sol - ref).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("deg", [2, 3])
def test_poisson_reproduces_polynomial_solution(deg):
    x, y, z = X
    p = x * (1 - x) * y * (1 - y) * z * (1 - z)
    f = -(sy.diff(p, x, 2) + sy.diff(p, y, 2) + sy.diff(p, z, 2))
    pb = Problem(Mesh(2, 3, 2), deg, "poisson", 0.0, 1.0)
    sol = spla.spsolve(assemble(pb).tocsc(), load_vector(pb, _scal_fn(f)))
    ref = interpolate(pb, _scal_fn(p))
    assert np.abs(sol - ref).max() <= 1e-10 * np.abs(ref).max()


def test_neumann_poisson_reproduces_polynomial_solution():
    """p* = q(x)q(y)q(z), q = 3t^2 - 2t^3 has zero normal derivative on the
    box; with alpha = 1 the Neumann problem is regular."""
    x, y, z = X
    q = lambda t: 3 * t ** 2 - 2 * t ** 3
    p = q(x) * q(y) * q(z)
    f = p - (sy.diff(p, x, 2) + sy.diff(p, y, 2) + sy.diff(p, z, 2))
    pb = Problem(Mesh(2, 2, 3, None, ("N",) * 6), 3, "poisson", 1.0, 1.0)
    sol = spla.spsolve(assemble(pb).tocsc(), load_vector(pb, _scal_fn(f)))
    ref = interpolate(pb, _scal_fn(p))
    assert np.abs(sol - ref).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("deg", [2, 3])
def test_viscous_patch_test_on_curved_cells(deg):
    """Linear u* with inhomogeneous Dirichlet data on four sides and the exact
    traction 2 mu eps(u*) n on two; on trilinear cells every integrand stays of
    degree <= k+2 per direction, so the solution reproduces u* exactly."""
    Amat = np.array([[0.3, -0.2, 0.5], [0.1, 0.4, -0.3], [-0.6, 0.2, 0.1]])
    c0 = np.array([0.2, -0.1, 0.4])
    ustar = lambda P: P @ Amat.T + c0
    mu, alpha = 1.7, 3.0
    eps = 0.5 * (Amat + Amat.T)
    bc = ("D", "D", "N", "D", "D", "N")
    pb = Problem(Mesh(3, 3, 3, jittered_vertices(3, 0.25), bc), deg, "viscous", alpha, 1.0, W.const_law(mu))

    def traction(P, nrm):
        return 2 * mu * nrm @ eps.T

    b = load_vector(pb, lambda P: alpha * ustar(P), g=ustar, hN=traction)
    sol = spla.spsolve(assemble(pb).tocsc(), b)
    ref = interpolate(pb, ustar)
    assert np.abs(sol - ref).max() <= 1e-10


def test_poisson_patch_test_on_curved_cells():
    gvec = np.array([0.4, -1.1, 0.7])
    pstar = lambda P: P @ gvec + 0.3
    bc = ("D", "N", "D", "D", "N", "D")
    pb = Problem(Mesh(3, 3, 3, jittered_vertices(3, 0.25), bc), 2, "poisson", 0.0, 1.0)
    b = load_vector(pb, lambda P: 0.0 * P[:, 0], g=pstar, hN=lambda P, nrm: nrm @ gvec)
    sol = spla.spsolve(assemble(pb).tocsc(), b)
    assert np.abs(sol - interpolate(pb, pstar)).max() <= 1e-10


@pytest.mark.slow
@pytest.mark.parametrize("deg,Ns,curved", [(2, (3, 4), False), (3, (3, 4), False), (2, (3, 4), True)])
def test_viscous_converges_at_order_k_plus_1(deg, Ns, curved):
    """Sec. 6.1 reports optimal k+1 L2 convergence; here for the viscous
    operator alone with the smooth viscosity 1 + 0.5 sin sin sin."""
    x, y, z = X
    s = sy.sin
    pi = sy.pi
    u = [s(pi * x) * s(pi * y) * s(pi * z), s(2 * pi * x) * s(pi * y) * s(pi * z),
         s(pi * x) * s(2 * pi * y) * s(pi * z)]
    mu = 1 + sy.Rational(1, 2) * s(2 * pi * x) * s(2 * pi * y) * s(2 * pi * z)
    alpha = 10.0
    f = _visc_rhs(u, mu, alpha)
    errs = []
    for N in Ns:
        V = W.box_vertices(N, N, N, 0.1) if curved else None
        pb = Problem(Mesh(N, N, N, V), deg, "viscous", alpha, 1.0, W.sine_law(1.0, 0.5))
        sol = spla.spsolve(assemble(pb).tocsc(), load_vector(pb, _vec_fn(f)))
        e, r = l2_error(pb, sol, _vec_fn(u))
        errs.append(e / r)
    rates = [np.log(errs[i] / errs[i + 1]) / np.log(Ns[i + 1] / Ns[i]) for i in range(len(Ns) - 1)]
    assert abs(rates[-1] - (deg + 1)) < 0.3, rates


def test_bruteforce_poisson_entries_affine_two_cells():
    """Recompute entries of the Poisson matrix on two affine cells with an
    independent construction: 1D basis from numpy's polynomial fit through
    the Legendre roots, physical coordinates directly (J = h I), a
    (k+3)-point rule (integrands are polynomials, both rules are exact), and
    faces enumerated by hand.  (The viscous form is recomputed on curved
    cells with variable viscosity by the test below.)"""
    deg, hx = 2, 0.5
    n = deg + 1
    roots = (np.polynomial.legendre.legroots([0] * n + [1]) + 1) / 2
    polys = [np.polynomial.Polynomial.fit(roots, np.eye(n)[j], n - 1).convert() for j in range(n)]
    dpolys = [p.deriv() for p in polys]
    gq, gw = np.polynomial.legendre.leggauss(n + 3)
    gq, gw = (gq + 1) / 2, gw / 2
    # two cells [0,.5]x[0,1]^2 and [.5,1]x[0,1]^2 (nx=2, ny=nz=1), all Dirichlet
    cells = [(0.0, 0.0, 0.0), (0.5, 0.0, 0.0)]
    size = np.array([0.5, 1.0, 1.0])

    def phi(cell, i, P):      # value and physical gradient of node i=(i1,i2,i3) of cell at points P
        xi = (P - np.array(cells[cell])) / size
        inside = np.all((xi >= -1e-12) & (xi <= 1 + 1e-12), axis=1)
        v = [polys[i[d]](xi[:, d]) for d in range(3)]
        dv = [dpolys[i[d]](xi[:, d]) / size[d] for d in range(3)]
        val = v[0] * v[1] * v[2] * inside
        grad = np.stack([dv[0] * v[1] * v[2], v[0] * dv[1] * v[2], v[0] * v[1] * dv[2]], 1) * inside[:, None]
        return val, grad

    def vol_pts(cell):
        T = np.array(np.meshgrid(gq, gq, gq, indexing="ij")).reshape(3, -1).T
        Wt = np.prod(np.array(np.meshgrid(gw, gw, gw, indexing="ij")).reshape(3, -1).T, 1)
        return np.array(cells[cell]) + T * size, Wt * np.prod(size)

    def face_pts(x0, d, lo, hi):   # plane x_d = x0 over the rectangle lo..hi in the other two dims
        t = [k for k in range(3) if k != d]
        A, B = np.meshgrid(gq, gq, indexing="ij")
        P = np.zeros((A.size, 3)); P[:, d] = x0
        P[:, t[0]] = lo[0] + A.ravel() * (hi[0] - lo[0]); P[:, t[1]] = lo[1] + B.ravel() * (hi[1] - lo[1])
        Wt = np.outer(gw, gw).ravel() * (hi[0] - lo[0]) * (hi[1] - lo[1])
        return P, Wt

    def side(P, cell, d, s):       # trace from inside `cell`, nudged towards its interior
        Q = P.copy(); Q[:, d] += (-1e-13 if s == 1 else 1e-13)
        return Q

    # sigma of each 0.5 x 1 x 1 cell: (x wall 1 + half the shared face 1/2 + four side walls 0.5) / 0.5
    sigma = (1.0 + 0.5 + 4 * 0.5) / 0.5
    tau_p = (deg + 1) ** 2 * sigma
    # face list: (plane coordinate, direction, normal sign for the owning cell, owner, neighbour or None)
    faces = [(0.0, 0, -1, 0, None), (0.5, 0, +1, 0, 1), (1.0, 0, +1, 1, None)]
    for cell in (0, 1):
        for d in (1, 2):
            for s in (0, 1):
                faces.append((float(s), d, 2 * s - 1, cell, None))

    def poisson_entry(I, J):
        ci, ni = I; cj, nj = J
        val = 0.0
        for cell in (0, 1):
            P, Wt = vol_pts(cell)
            vi, gi = phi(ci, ni, P); vj, gj = phi(cj, nj, P)
            val += Wt @ np.einsum("pi,pi->p", gi, gj)
        for x0, d, sgn, own, nb in faces:
            o = np.array(cells[own])
            lo = [o[k] for k in range(3) if k != d]; hi = [o[k] + size[k] for k in range(3) if k != d]
            P, Wt = face_pts(x0, d, lo, hi)
            nrm = np.zeros(3); nrm[d] = sgn
            sm = 1 if sgn > 0 else 0
            qm, gqm = phi(ci, ni, side(P, own, d, sm)) if ci == own else (0 * Wt, 0 * P)
            pm, gpm = phi(cj, nj, side(P, own, d, sm)) if cj == own else (0 * Wt, 0 * P)
            if nb is None:
                val += Wt @ (-(gqm @ nrm) * pm - (gpm @ nrm) * qm + 2 * tau_p * qm * pm)
            else:
                qp, gqp = phi(ci, ni, side(P, nb, d, 1 - sm)) if ci == nb else (0 * Wt, 0 * P)
                pp, gpp = phi(cj, nj, side(P, nb, d, 1 - sm)) if cj == nb else (0 * Wt, 0 * P)
                jq, jp = qm - qp, pm - pp
                val += Wt @ (-0.5 * ((gqm + gqp) @ nrm) * jp - 0.5 * ((gpm + gpp) @ nrm) * jq + tau_p * jq * jp)
        return val

    pb = Problem(Mesh(2, 1, 1), deg, "poisson", 0.0, 1.0)
    A = assemble(pb).toarray()
    rng = np.random.default_rng(0)
    idx = lambda cell, i: cell * n ** 3 + i[2] * n * n + i[1] * n + i[0]
    for _ in range(25):
        I = (int(rng.integers(2)), tuple(int(v) for v in rng.integers(0, n, 3)))
        J = (int(rng.integers(2)), tuple(int(v) for v in rng.integers(0, n, 3)))
        ref = poisson_entry(I, J)
        # the 1e-13 nudge that picks a side of a face costs ~1e-12 in the traces
        assert abs(A[idx(*I), idx(*J)] - ref) <= 1e-10 * np.abs(A).max(), (I, J)


class _NaiveCells:
    """A second, deliberately plain construction of the viscous form for a
    pins test: its own 1D Lagrange basis (numpy polynomial fit through the
    Legendre roots), its own trilinear map written out vertex by vertex,
    physical points looped one at a time, face normals and area elements from
    the cross product of the two tangent vectors, and the "+" side's
    reference point of a face point found by Newton's method on that cell's
    map (no assumption that the two cells share face coordinates)."""

    def __init__(self, V, nx, deg, alpha, mu_fn):
        self.V = V                      # (2, 2, nx + 1, 3): vertices (k, j, i)
        self.nx, self.n, self.alpha, self.mu = nx, deg + 1, alpha, mu_fn
        n = self.n
        roots = (np.polynomial.legendre.legroots([0] * n + [1]) + 1) / 2
        self.p = [np.polynomial.Polynomial.fit(roots, np.eye(n)[j], n - 1).convert() for j in range(n)]
        self.dp = [q.deriv() for q in self.p]
        g, w = np.polynomial.legendre.leggauss(n)
        self.g, self.w = (g + 1) / 2, w / 2
        self.k2 = (deg + 1) ** 2
        self.sigma = [self._sigma(e) for e in range(nx)]

    def map(self, e, xi):
        x, J = np.zeros(3), np.zeros((3, 3))
        for a in (0, 1):
            for b in (0, 1):
                for c in (0, 1):
                    X = self.V[c, b, e + a]
                    L = [1 - xi[0] if a == 0 else xi[0], 1 - xi[1] if b == 0 else xi[1],
                         1 - xi[2] if c == 0 else xi[2]]
                    dL = [-1.0 if a == 0 else 1.0, -1.0 if b == 0 else 1.0, -1.0 if c == 0 else 1.0]
                    x += X * L[0] * L[1] * L[2]
                    J[:, 0] += X * dL[0] * L[1] * L[2]
                    J[:, 1] += X * L[0] * dL[1] * L[2]
                    J[:, 2] += X * L[0] * L[1] * dL[2]
        return x, J

    def inverse_map(self, e, P):
        xi = np.full(3, 0.5)
        for _ in range(50):
            x, J = self.map(e, xi)
            step = np.linalg.solve(J, x - P)
            xi = xi - step
            if np.abs(step).max() < 1e-16:
                break
        return xi

    def face_point(self, e, d, side, qa, qb):
        """Physical point, outward unit normal and area weight of face point (qa, qb)."""
        t1, t2 = (d + 1) % 3, (d + 2) % 3
        xi = np.zeros(3); xi[d] = side; xi[t1] = self.g[qa]; xi[t2] = self.g[qb]
        x, J = self.map(e, xi)
        c = np.cross(J[:, t1], J[:, t2])       # along +xi_d for the cyclic tangent order
        area = np.linalg.norm(c)
        return x, (1.0 if side == 1 else -1.0) * c / area, area * self.w[qa] * self.w[qb]

    def _sigma(self, e):
        vol = 0.0
        for q in np.ndindex(self.n, self.n, self.n):
            vol += np.linalg.det(self.map(e, self.g[list(q)])[1]) * np.prod(self.w[list(q)])
        surf = 0.0
        for d in range(3):
            for side in (0, 1):
                inner = d == 0 and ((side == 1 and e < self.nx - 1) or (side == 0 and e > 0))
                A = sum(self.face_point(e, d, side, qa, qb)[2] for qa in range(self.n) for qb in range(self.n))
                surf += (0.5 if inner else 1.0) * A
        return surf / vol

    def basis(self, I, e, xi, J):
        """Value (3,) and gradient (3, 3) [component, direction] of the vector
        basis function I = (cell, component, (i1, i2, i3)) inside cell e."""
        cell, comp, (i1, i2, i3) = I
        val, grad = np.zeros(3), np.zeros((3, 3))
        if cell != e:
            return val, grad
        v = [self.p[i](t) for i, t in zip((i1, i2, i3), xi)]
        dv = [self.dp[i](t) for i, t in zip((i1, i2, i3), xi)]
        ref = np.array([dv[0] * v[1] * v[2], v[0] * dv[1] * v[2], v[0] * v[1] * dv[2]])
        val[comp] = v[0] * v[1] * v[2]
        grad[comp] = np.linalg.solve(J.T, ref)
        return val, grad

    def entry(self, I, Jt):
        """(cell, interior-face, boundary-face) parts of a(phi_I, phi_J)."""
        eps = lambda G: 0.5 * (G + G.T)
        cellp = intp = bndp = 0.0
        for e in {I[0], Jt[0]}:
            for q in np.ndindex(self.n, self.n, self.n):
                xi = self.g[list(q)]
                x, J = self.map(e, xi)
                wq = np.linalg.det(J) * np.prod(self.w[list(q)])
                v, Gv = self.basis(I, e, xi, J)
                u, Gu = self.basis(Jt, e, xi, J)
                cellp += wq * (self.alpha * v @ u + 2 * self.mu(x) * np.sum(eps(Gv) * eps(Gu)))
        for e in range(self.nx):
            for d in range(3):
                for side in (0, 1):
                    nb = e + 1 if (d == 0 and side == 1 and e < self.nx - 1) else None
                    if d == 0 and side == 0 and e > 0:
                        continue                   # counted from the "-" cell
                    if e not in (I[0], Jt[0]) and nb not in (I[0], Jt[0]):
                        continue
                    for qa in range(self.n):
                        for qb in range(self.n):
                            x, nrm, ds = self.face_point(e, d, side, qa, qb)
                            mu = self.mu(x)
                            xm = self.inverse_map(e, x)
                            Jm = self.map(e, xm)[1]
                            vm, Gvm = self.basis(I, e, xm, Jm)
                            um, Gum = self.basis(Jt, e, xm, Jm)
                            if nb is None:       # Dirichlet wall, mirror principle
                                tau = self.k2 * mu * self.sigma[e]
                                bndp += ds * (-2 * mu * np.sum(eps(Gvm) * np.outer(um, nrm))
                                              - 2 * mu * np.sum(eps(Gum) * np.outer(vm, nrm))
                                              + 2 * tau * (vm @ um + (vm @ nrm) * (um @ nrm)))
                                continue
                            xp = self.inverse_map(nb, x)
                            Jp = self.map(nb, xp)[1]
                            vp, Gvp = self.basis(I, nb, xp, Jp)
                            up, Gup = self.basis(Jt, nb, xp, Jp)
                            tau = self.k2 * mu * max(self.sigma[e], self.sigma[nb])
                            jv, ju = vm - vp, um - up
                            av = 0.5 * mu * (eps(Gvm) + eps(Gvp))
                            au = 0.5 * mu * (eps(Gum) + eps(Gup))
                            intp += ds * (-2 * np.sum(av * np.outer(ju, nrm)) - 2 * np.sum(au * np.outer(jv, nrm))
                                          + tau * (jv @ ju + (jv @ nrm) * (ju @ nrm)))
        return cellp, intp, bndp


@pytest.mark.parametrize("deg", [2, 3])
def test_bruteforce_viscous_entries_curved_cells_variable_viscosity(deg):
    """Entries of the viscous matrix (cell terms, the interior face, Dirichlet
    mirror faces) on two trilinear cells with randomly moved vertices and the
    viscosity 1 + 0.5 sin 2pi x sin 2pi y sin 2pi z, recomputed by the plain
    construction above with the same n-point Gauss rules, part by part."""
    rng = np.random.default_rng(12 + deg)
    V = Mesh(2, 1, 1).vertices.copy()
    V += rng.uniform(-0.08, 0.08, V.shape)
    alpha = 4.0
    mu_fn = lambda x: 1 + 0.5 * np.sin(2 * np.pi * x[0]) * np.sin(2 * np.pi * x[1]) * np.sin(2 * np.pi * x[2])
    pb = Problem(Mesh(2, 1, 1, V.reshape(-1, 3)), deg, "viscous", alpha, 1.0, W.sine_law(1.0, 0.5))
    parts = [assemble(pb, (p,)).toarray() for p in ("cell", "interior", "boundary")]
    scale = np.abs(sum(parts)).max()
    bf = _NaiveCells(V, 2, deg, alpha, mu_fn)
    n = deg + 1
    idx = lambda I: (I[0] * 3 + I[1]) * n ** 3 + I[2][2] * n * n + I[2][1] * n + I[2][0]
    draw = lambda: (int(rng.integers(2)), int(rng.integers(3)), tuple(int(v) for v in rng.integers(0, n, 3)))
    pairs = [(draw(), draw()) for _ in range(14)]
    # pairs across the interior face, and a node pair on a wall of the same cell
    pairs += [((0, 0, (n - 1, 1, 0)), (1, 2, (0, 1, n - 1))), ((1, 1, (0, 0, 0)), (0, 1, (n - 1, 0, 0))),
              ((0, 2, (0, 0, 0)), (0, 0, (0, 1, 0)))]
    for I, J in pairs:
        ref = bf.entry(I, J)
        for got, want in zip((P[idx(I), idx(J)] for P in parts), ref):
            assert abs(got - want) <= 1e-13 * scale, (I, J, got, want)


def test_sampled_cell_apply_equals_rows_of_full_apply():
    """apply(pb, x, cells=S) returns the rows of the full apply for the cells
    in S (and zero elsewhere) on a curved 4^3 mesh with mixed boundary
    conditions, for a corner, an edge, a face and an interior cell, every part
    and the viscous and Poisson operators."""
    Vt = W.box_vertices(4, 4, 4, 0.1)
    bc = ("D", "N", "D", "D", "N", "D")
    S = np.array([0, 2, 5, 21, 63])         # corner, edge, face, interior, corner
    for op, law in (("viscous", W.logfield_law(3, 1e2)), ("poisson", W.const_law(1.0))):
        pb = Problem(Mesh(4, 4, 4, Vt, bc), 2, op, 3.0, 1.0, law)
        x = np.random.default_rng(5).uniform(-1, 1, pb.ndof)
        for parts in (("cell", "interior", "boundary"), ("cell",), ("interior",), ("boundary",)):
            full = apply(pb, x, parts).reshape(64, -1)
            part = apply(pb, x, parts, cells=S).reshape(64, -1)
            assert np.abs(part[S] - full[S]).max() <= 1e-14 * np.abs(full).max()
            others = np.setdiff1d(np.arange(64), S)
            assert not np.any(part[others])


def test_oracle_modes_agree():
    """The assembled matrix (O2) and the direct quadrature apply (O3)."""
    for pb in _problems():
        A = assemble(pb)
        x = np.random.default_rng(1).uniform(-1, 1, pb.ndof)
        y2, y3 = A @ x, apply(pb, x)
        assert np.abs(y2 - y3).max() <= 1e-13 * np.abs(y2).max()
        for parts in (("cell",), ("interior",), ("boundary",)):
            Ap = assemble(pb, parts)
            assert np.abs(Ap @ x - apply(pb, x, parts)).max() <= 1e-13 * np.abs(y2).max()
        assert np.abs(diagonal(pb) - A.diagonal()).max() <= 1e-13 * np.abs(A.diagonal()).max()


# --------------------------------------------------------------- laws ---

def test_sine_law_values():
    law = W.sine_law(2.0, 0.5)
    P = np.array([[0.25, 0.25, 0.25], [0.75, 0.25, 0.25], [0.5, 0.3, 0.9]])
    assert np.allclose(viscosity(law, P), [3.0, 1.0, 2.0], atol=1e-14)


def test_logfield_range_and_contrast():
    law = W.logfield_law(2, 1e3)
    P = np.random.default_rng(0).uniform(0, 1, (20000, 3))
    mu = viscosity(law, P)
    assert mu.min() >= 1.0 - 1e-14 and mu.max() <= 1e3 * (1 + 1e-14)
    assert mu.max() / mu.min() > 1e2


def test_generalized_newtonian_special_cases():
    base = W.carreau_law(3)
    P = np.random.default_rng(1).uniform(0, 1, (50, 3))
    gd = shear_rate_of_modes(base, P)
    newt = dict(base, mu0=0.7, mu_inf=0.7)
    assert np.allclose(viscosity(newt, P), 0.7)
    power = dict(base, kappa=0.0, mu_inf=0.0, a_exp=2.0, n_exp=0.4, lam=2.0, mu0=1.5)
    assert np.allclose(viscosity(power, P), 1.5 * (2.0 * gd) ** (0.4 - 1.0), rtol=1e-12)
    car = viscosity(base, P)   # Carreau: mu_inf + (mu0 - mu_inf)(1 + (lam g)^2)^((n-1)/2)
    assert np.allclose(car, 1e-4 + (1 - 1e-4) * (1 + gd ** 2) ** (-0.25), rtol=1e-12)


def test_shear_rate_matches_finite_differences_and_field_is_solenoidal():
    law = W.carreau_law(3)
    k, v, phi = law["k"].astype(float), law["v"], law["phi"]
    w = lambda P: np.cos(2 * np.pi * P @ k.T + phi) @ v
    P = np.random.default_rng(2).uniform(0, 1, (30, 3))
    hh = 1e-6
    G = np.stack([(w(P + hh * e) - w(P - hh * e)) / (2 * hh) for e in np.eye(3)], 2)  # G[p,i,j]=dw_i/dx_j
    eps = 0.5 * (G + G.transpose(0, 2, 1))
    gd = np.sqrt(2 * np.einsum("pij,pij->p", eps, eps))
    assert np.allclose(shear_rate_of_modes(law, P), gd, rtol=1e-6)
    assert np.abs(np.trace(G, axis1=1, axis2=2)).max() < 1e-6 * np.abs(G).max()


# ------------------------------------------------------------ solvers ---

def test_splitmix64_published_outputs():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed0.txt")
    ref = [int(l, 16) for l in open(path) if l.strip() and not l.startswith("#")]
    u = solvers.splitmix64_uniform(0, 3)
    bits = ((u + 1.0) / 2.0 * 2.0 ** 53).astype(np.uint64)
    assert [int(b) for b in bits] == [r >> 11 for r in ref]


def test_chebyshev_matches_closed_form_polynomial():
    """For diagonal A and D = I, the error after the Chebyshev iteration from
    0 is the scaled Chebyshev polynomial T_d((theta - l)/delta) / T_d(theta/delta)."""
    lam = np.linspace(0.05, 2.0, 40)
    A = lambda v: lam * v
    r = np.ones_like(lam)
    lo, hi, deg = 0.1, 2.1, 5
    z = solvers.chebyshev_jacobi(A, np.ones_like(lam), r, deg, hi, lo)
    theta, delta = (hi + lo) / 2, (hi - lo) / 2
    T = np.polynomial.chebyshev.Chebyshev.basis(deg)
    resid = 1 - lam * z                       # error polynomial at each eigenvalue
    assert np.allclose(resid, T((theta - lam) / delta) / T(theta / delta), atol=1e-13)


def test_lanczos_recovers_largest_eigenvalue():
    rng = np.random.default_rng(0)
    Q, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    M = Q @ np.diag(np.linspace(1, 9, 12)) @ Q.T
    d = np.diag(M)
    est = solvers.lanczos_max(lambda v: M @ v, 1 / d, steps=12)
    S = M / np.sqrt(np.outer(d, d))
    assert abs(est - np.linalg.eigvalsh(S)[-1]) < 1e-9


def test_flexible_cg_solves_and_reports():
    pb = Problem(Mesh(3, 3, 3, jittered_vertices(3, 0.2)), 2, "viscous", 10.0, 1.0, W.sine_law())
    A = assemble(pb).tocsc()
    b = W.uniform_vector(1, pb.ndof)
    x, info = solvers.solve(lambda v: A @ v, A.diagonal(), b, tol=1e-10)
    assert info["status"] == "ok" and info["rel_residual"] <= 1e-10
    assert np.abs(x - spla.spsolve(A, b)).max() <= 1e-7 * np.abs(x).max()


def test_neumann_poisson_solve_is_mean_zero():
    pb = Problem(Mesh(3, 3, 3, None, ("N",) * 6), 3, "poisson", 0.0, 1.0)
    A = assemble(pb).tocsr()
    b = W.uniform_vector(4, pb.ndof)
    x, info = solvers.solve(lambda v: A @ v, A.diagonal(), b, tol=1e-8, mean_zero=True)
    assert info["status"] == "ok" and abs(x.mean()) < 1e-14
    bz = b - b.mean()
    assert np.linalg.norm(bz - A @ x) <= 1e-8 * np.linalg.norm(bz)


@pytest.mark.slow
def test_high_contrast_request_is_positive_definite():
    """Sec. 4.1 remarks that the pointwise viscosity does not by itself make
    the operator positive.  A 3^3, k = 3 request of the serving stream with a
    viscosity contrast of 1e4 across the unit cube is positive definite with
    the surface-to-volume penalty (3.5-4.5 (k+1)^2 mu / h on this mesh); with
    a quarter of it (about the plain (k+1)^2 mu / h scaling) the matrix has
    negative eigenvalues."""
    cfg = W.serving_requests(seed=11, count=12, rate=200.0, nmin=2, nmax=6)[3]["cfg"]
    assert (cfg["nx"], cfg["degree"], cfg["law"]["contrast"]) == (3, 3, 1e4)

    def lam_min(P):
        pb = Problem(Mesh(3, 3, 3), 3, "viscous", cfg["alpha"], P, cfg["law"])
        A = assemble(pb)
        d = 1.0 / np.sqrt(A.diagonal())
        return np.linalg.eigvalsh((A.multiply(np.outer(d, d))).toarray())[0]
    assert lam_min(1.0) > 0.0
    assert lam_min(0.25) < 0.0
