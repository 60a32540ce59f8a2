"""Pins of the oracle's dual-splitting step (Sec. 3 "Splitting Scheme",
Sec. 4.1 weak forms, Sec. 5.1 Alg. 1), each against a closed form that does
not come from the oracle's own tables: the mass matrix integrates the
domain's volume; the convective term of a linear field is (u . grad) u at
every node and the upwind flux of a piecewise-constant field takes the
inflow side's value (1D Lagrange values from scipy, Gauss weights from
numpy); the divergence form of a linear field is -div(u) times the integral
of each pressure basis function; the pressure right-hand side sums to the
wall flux of (grad u) u, i.e. tr(B^2) for u = B x + d; the projection of a
linear pressure removes its constant gradient and a piecewise-constant
pressure acts through half its jump; the penalty factors of a constant
velocity; the whole step keeps a fluid at rest under a gradient body
force with the hydrostatic pressure; and with velocity data on the walls:
the viscous load equals the forms' SIPG load vector, a uniform flow through
the box stays uniform with zero pressure, the inflow flux of a wall, and the
penalty step's wall load in closed form.  BDF2: the coefficients reproduce
constants, a quadratic's derivative and a linear extrapolation; the
vorticity of a polynomial field and the projected viscosity of a law that
is polynomial in the gradient are exact; the wall data h_p of s(y^2, 0, 0)
in closed form (curl curl, the viscosity gradient term); equal linear states
make the right-hand side sum vanish; the convective step of two linear
fields; rest and uniform flow through whole BDF2 steps."""
import numpy as np
import pytest
from scipy.interpolate import lagrange

import workloads as W
from oracle import splitting as SP
from oracle.forms import Problem, interpolate, node_points
from oracle.mesh import Mesh


def gauss01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return (x + 1) / 2, w / 2


def ends(n):
    """l_j(0), l_j(1) of the n Gauss points' Lagrange basis (scipy)."""
    g, _ = gauss01(n)
    l0, l1 = np.zeros(n), np.zeros(n)
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        P = lagrange(g, e)
        l0[j], l1[j] = P(0.0), P(1.0)
    return l0, l1


def velocity_problem(nx, ny, nz, deg, perturb=0.0, dt=0.1):
    V = W.box_vertices(nx, ny, nz, perturb) if perturb else None
    return Problem(Mesh(nx, ny, nz, V), deg, "viscous", 1.0 / dt, 1.0)


def aniso_box(nx, ny, nz, sx, sy, sz):
    x = np.linspace(0, sx, nx + 1)
    y = np.linspace(0, sy, ny + 1)
    z = np.linspace(0, sz, nz + 1)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return np.stack([X, Y, Z], -1).reshape(-1, 3)


A = np.array([[0.3, -1.2, 0.5], [0.7, 0.1, -0.4], [-0.6, 0.9, 0.2]])
c0 = np.array([0.25, -0.5, 1.0])


def linear(M, c):
    return lambda x: x @ M.T + c


@pytest.mark.parametrize("perturb", [0.0, 0.1])
def test_mass_integrates_the_volume(perturb):
    pb = velocity_problem(3, 2, 2, 3, perturb)
    one = np.ones(pb.ndof)
    m = SP.mass_apply(pb, one).reshape(pb.mesh.ncells, 3, -1)
    assert np.allclose(m.sum(axis=(0, 2)), 1.0, rtol=0, atol=1e-13)
    x = W.uniform_vector(1, pb.ndof)
    assert np.allclose(SP.mass_solve(pb, SP.mass_apply(pb, x)), x, rtol=0, atol=1e-12)


@pytest.mark.parametrize("perturb,deg", [(0.0, 2), (0.1, 3)])
def test_convective_term_of_a_linear_field(perturb, deg):
    """u = A x + c is continuous and in the space (also on trilinear cells):
    the face terms vanish (no jump; {u} = g_u = 0 on the walls) and M^-1 c_h
    at each node is (u . grad) u = A (A x + c)."""
    pb = velocity_problem(3, 2, 2, deg, perturb)
    u = interpolate(pb, linear(A, c0))
    got = SP.mass_solve(pb, SP.convective_form(pb, u, u))
    ref = interpolate(pb, lambda x: (x @ A.T + c0) @ A.T)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    dt = 0.05
    b = W.uniform_vector(2, pb.ndof)
    uhat = SP.convective_step(pb, u, b, dt)
    assert np.abs(uhat - (u + dt * (b - ref))).max() <= 1e-13


@pytest.mark.parametrize("inflow_from_right", [True, False])
def test_upwind_flux_of_piecewise_constants(inflow_from_right):
    """Two cells along x (widths hx = 0.5, heights 0.7 x 1.3), u constant per
    cell: only the shared face acts; on the side where {u}.n < 0 the node
    value is l_i1(face) / (hx w_i1) ({u}.n) (u_other - u_own), zero on the
    outflow side."""
    deg = 3
    n = deg + 1
    m = Mesh(2, 1, 1, aniso_box(2, 1, 1, 1.0, 0.7, 1.3))
    pb = Problem(m, deg, "viscous", 1.0, 1.0)
    ua = np.array([-3.0, 1.0, 0.25]) if inflow_from_right else np.array([2.0, -1.0, 0.5])
    ub = np.array([1.0, 0.5, -2.0]) if inflow_from_right else np.array([-0.5, 2.0, 1.5])
    U = np.zeros((2, 3, n ** 3))
    U[0] = ua[:, None]
    U[1] = ub[:, None]
    got = SP.mass_solve(pb, SP.convective_form(pb, U.reshape(-1), U.reshape(-1))).reshape(2, 3, n, n, n)
    g, w = gauss01(n)
    l0, l1 = ends(n)
    hx = 0.5
    wn = 0.5 * (ua[0] + ub[0])          # {u}.n with n = +x out of cell 0
    ref = np.zeros_like(got)
    if wn < 0:
        ref[0] = (wn * (ub - ua))[:, None, None, None] * (l1 / (hx * w))[None, None, None, :]
    else:
        ref[1] = (-wn * (ua - ub))[:, None, None, None] * (l0 / (hx * w))[None, None, None, :]
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("deg", [2, 4])
def test_divergence_form_of_a_linear_field(deg):
    """sum_e (grad q, u)_e - (q, {u}.n)_de = -(q, div u) for a continuous
    u = A x + c with its own trace on the walls; on an affine box of cell
    sizes hx, hy, hz, int q_j = hx hy hz w_j1 w_j2 w_j3 (k-point weights)."""
    nx, ny, nz = 3, 2, 2
    m = Mesh(nx, ny, nz, aniso_box(nx, ny, nz, 1.2, 0.8, 1.0))
    pb = Problem(m, deg, "viscous", 1.0, 1.0)
    pp = SP.pressure_problem(m, deg)
    u = interpolate(pb, linear(A, c0))
    U = u.reshape(m.ncells, 3, -1)
    from oracle.basis import face_points, tensor_tables

    def trace(d, s):
        V, _ = tensor_tables(pb.n, face_points(pb.n, d, s)[0])
        return np.einsum("pj,ecj->epc", V, U[m.boundary_cells(d, s)])

    got = SP.divergence_form(pb, pp, u, trace).reshape(m.ncells, deg, deg, deg)
    _, wq = gauss01(deg)
    vol = (1.2 / nx) * (0.8 / ny) * (1.0 / nz)
    ref = -np.trace(A) * vol * wq[None, :, None, None] * wq[None, None, :, None] * wq[None, None, None, :]
    assert np.abs(got - np.broadcast_to(ref, got.shape)).max() <= 1e-13


@pytest.mark.parametrize("perturb", [0.0, 0.1])
def test_pressure_rhs_sums_to_the_wall_flux(perturb):
    """Summed over the pressure basis (a partition of unity) the interior
    face terms cancel and the walls leave int (grad u^n) u^n . n = tr(B^2)
    on the unit cube for u^n = B x + d, whatever uhat and b are."""
    pb = velocity_problem(2, 3, 2, 3, perturb)
    pp = SP.pressure_problem(pb.mesh, pb.degree)
    B = np.array([[0.5, 0.2, -0.3], [0.1, -0.4, 0.6], [0.8, 0.3, 0.1]])
    u_old = interpolate(pb, linear(B, np.array([1.0, -2.0, 0.5])))
    uhat = W.uniform_vector(3, pb.ndof)
    b = W.uniform_vector(4, pb.ndof)
    f = SP.ppe_rhs(pb, pp, uhat, u_old, b, 0.05)
    assert abs(f.sum() - np.trace(B @ B)) <= 1e-11


@pytest.mark.parametrize("perturb,deg", [(0.0, 2), (0.0, 4), (0.1, 3)])
def test_projection_of_a_linear_pressure(perturb, deg):
    """p = g.x + p0 is continuous ({p} = p, also on the walls): the form
    is -(v, grad p), so M^-1 of it is -g at every velocity node."""
    pb = velocity_problem(2, 2, 3, deg, perturb)
    pp = SP.pressure_problem(pb.mesh, deg)
    gvec = np.array([0.7, -1.1, 0.4])
    p = interpolate(pp, lambda x: x @ gvec + 0.3)
    got = SP.mass_solve(pb, SP.projection_form(pb, pp, p)).reshape(pb.mesh.ncells, 3, -1)
    assert np.abs(got + gvec[None, :, None]).max() <= 1e-12


def test_projection_of_piecewise_constant_pressure():
    """Two cells along x, p constant per cell: (div v, p_e) - (v, {p} n) =
    sum over faces (p_e - {p}) v.n, i.e. half the jump on the shared face
    and nothing on the walls."""
    deg = 3
    n = deg + 1
    m = Mesh(2, 1, 1, aniso_box(2, 1, 1, 1.0, 0.7, 1.3))
    pb = Problem(m, deg, "viscous", 1.0, 1.0)
    pp = SP.pressure_problem(m, deg)
    p0, p1 = 2.0, -0.5
    p = np.concatenate([np.full(deg ** 3, p0), np.full(deg ** 3, p1)])
    got = SP.mass_solve(pb, SP.projection_form(pb, pp, p)).reshape(2, 3, n, n, n)
    _, w = gauss01(n)
    l0, l1 = ends(n)
    ref = np.zeros_like(got)
    ref[0, 0] = (0.5 * (p0 - p1) * l1 / (0.5 * w))[None, None, :]
    ref[1, 0] = (-0.5 * (p1 - p0) * l0 / (0.5 * w))[None, None, :]
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_penalty_factors_of_a_constant_velocity():
    nx, ny, nz, deg, dt, zeta = 3, 2, 4, 3, 0.02, 1.5
    m = Mesh(nx, ny, nz, aniso_box(nx, ny, nz, 1.2, 0.8, 1.0))
    pb = Problem(m, deg, "viscous", 1.0 / dt, 1.0)
    c = np.array([0.3, -0.4, 1.2])
    td, tc = SP.penalty_factors(pb, interpolate(pb, lambda x: np.broadcast_to(c, x.shape)), dt, zeta)
    h = ((1.2 / nx) * (0.8 / ny) * (1.0 / nz)) ** (1 / 3)
    speed = np.linalg.norm(c)
    assert np.allclose(td, zeta * speed * h * dt / (deg + 1), rtol=1e-13, atol=0)
    assert np.allclose(tc, zeta * speed * dt, rtol=1e-13, atol=0)


@pytest.mark.parametrize("perturb,deg", [(0.0, 2), (0.1, 3)])
def test_rest_under_a_gradient_force(perturb, deg):
    """u^n = 0 and b = g (= grad(g.x)): uhat = dt g, the pressure solves
    -lap p = 0 with grad p.n = g.n, so p = g.x up to the level (linear, in
    the space: SIPG is exact), the projection removes dt grad p, and the
    fluid stays at rest through the viscous and penalty steps."""
    dt = 0.05
    pb = velocity_problem(2, 2, 2, deg, perturb, dt)
    gvec = np.array([0.4, -1.0, 2.5])
    b = interpolate(pb, lambda x: np.broadcast_to(gvec, x.shape))
    law = W.carreau_law(3)
    out = SP.split_step(pb, law, np.zeros(pb.ndof), b, dt)
    assert np.abs(out["uhat"] - dt * b).max() <= 1e-14
    pe = node_points(out["pb_p"]).reshape(-1, 3) @ gvec
    pe -= pe.mean()
    assert np.abs(out["p"] - pe).max() <= 1e-10
    assert np.abs(out["uhh"]).max() <= 1e-10
    assert np.abs(out["u_new"]).max() <= 1e-10
    assert np.all(out["tau_div"] == 0.0) and np.all(out["tau_cont"] == 0.0)


def test_step_rejects_other_boundaries_and_mass_coefficients():
    pb = Problem(Mesh(2, 2, 2, None, ("D", "N", "D", "D", "D", "D")), 2, "viscous", 10.0, 1.0)
    with pytest.raises(ValueError):
        SP.convective_form(pb, np.zeros(pb.ndof), np.zeros(pb.ndof))
    pb = velocity_problem(2, 2, 2, 2, 0.0, 0.1)
    with pytest.raises(ValueError):
        SP.split_step(pb, W.carreau_law(3), np.zeros(pb.ndof), np.zeros(pb.ndof), 0.2)


def test_penalty_factor_speed_is_the_volume_mean():
    """u = (x^2, 0, 0) (in Q_2): the volume mean of |u| over a cell
    [a, a + hx] x ... is a^2 + a hx + hx^2/3."""
    nx, ny, nz, deg, dt = 4, 1, 2, 2, 0.1
    m = Mesh(nx, ny, nz, aniso_box(nx, ny, nz, 1.6, 0.5, 1.0))
    pb = Problem(m, deg, "viscous", 1.0 / dt, 1.0)
    u = interpolate(pb, lambda x: np.stack([x[:, 0] ** 2, 0 * x[:, 0], 0 * x[:, 0]], -1))
    _, tc = SP.penalty_factors(pb, u, dt, 1.0)
    hx = 1.6 / nx
    a = hx * (np.arange(m.ncells) % nx)
    assert np.allclose(tc, (a ** 2 + a * hx + hx ** 2 / 3) * dt, rtol=1e-13, atol=0)


def _g_wall_from(pb, fn):
    """Wall-data array of the callable fn at the walls' face points."""
    from oracle.forms import _face_geo
    rows = SP.wall_rows(pb.mesh)
    g = np.zeros((SP.wall_count(pb.mesh), pb.n ** 2, 3))
    for (d, side), sl in rows.items():
        _, xq, _, _, _ = _face_geo(pb, pb.mesh.boundary_cells(d, side), d, side)
        g[sl] = fn(xq.reshape(-1, 3)).reshape(xq.shape)
    return g.reshape(-1)


def test_viscous_wall_load_equals_the_forms_load():
    """The wall-data load of the viscous step equals the SIPG load vector of
    the forms (pinned there by patch tests with inhomogeneous data)."""
    from oracle import picard as PC
    from oracle.forms import load_vector
    pb = velocity_problem(3, 2, 2, 3, 0.1)
    pbv = PC.with_velocity_viscosity(pb, pb, W.uniform_vector(3, pb.ndof), W.carreau_law(3))
    fn = linear(A, c0)
    ref = load_vector(pbv, lambda x: np.zeros_like(x), fn)
    got = SP.viscous_wall_load(pbv, _g_wall_from(pbv, fn))
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("perturb,deg", [(0.0, 2), (0.1, 3)])
def test_uniform_flow_through_the_box_is_steady(perturb, deg):
    """u^n = c, g_u = c on every wall (inflow and outflow), b = 0: no
    convection, a zero pressure, and the viscous (SIPG consistency) and
    penalty steps (no divergence, no jump against g) return c."""
    dt = 0.05
    pb = velocity_problem(2, 2, 2, deg, perturb, dt)
    c = np.array([0.7, -0.4, 0.25])
    const = lambda x: np.broadcast_to(c, x.shape)
    u = interpolate(pb, const)
    out = SP.split_step(pb, W.carreau_law(3), u, np.zeros(pb.ndof), dt, g_wall=_g_wall_from(pb, const))
    assert np.abs(out["uhat"] - u).max() <= 1e-13
    assert np.abs(out["p"]).max() <= 1e-10
    assert np.abs(out["u_new"] - u).max() <= 1e-10
    assert np.all(out["tau_div"] > 0)


@pytest.mark.parametrize("gx", [0.8, -0.8])
def test_wall_inflow_flux(gx):
    """Two cells along x, u = c in both; data g only on the -x wall: the
    inflow case (g.n < 0) gives l_i1(0) / (hx w_i1) (g.n)(2g - 2c) at the
    nodes of the first cell, the outflow case nothing."""
    deg = 3
    n = deg + 1
    m = Mesh(2, 1, 1, aniso_box(2, 1, 1, 1.0, 0.7, 1.3))
    pb = Problem(m, deg, "viscous", 1.0, 1.0)
    c = np.array([0.3, -0.2, 0.5])
    g = np.array([gx, 0.4, -0.1])
    U = np.tile(c[None, :, None], (2, 1, n ** 3)).reshape(-1)
    gw = np.zeros((SP.wall_count(m), n * n, 3))
    gw[SP.wall_rows(m)[(0, 0)]] = g
    got = SP.mass_solve(pb, SP.convective_form(pb, U, U, gw.reshape(-1))).reshape(2, 3, n, n, n)
    _, w = gauss01(n)
    l0, _ = ends(n)
    gn = -g[0]
    ref = np.zeros_like(got)
    if gn < 0:
        ref[0] = (gn * (2 * g - 2 * c))[:, None, None, None] * (l0 / (0.5 * w))[None, None, None, :]
    scale = max(np.abs(ref).max(), 1.0)
    assert np.abs(got - ref).max() <= 1e-12 * scale


def test_penalty_wall_load_closed_form():
    """One cell, tau_cont = t: the load of g = (gx, 0, 0) on the -x wall is
    t (g.n)(v.n) integrated: at node i, -l_i1(0) t gx (-1) hy hz w_i2 w_i3 for
    the x component, zero elsewhere."""
    deg = 2
    n = deg + 1
    m = Mesh(1, 1, 1, aniso_box(1, 1, 1, 0.6, 0.7, 1.3))
    t = 0.37
    pb = Problem(m, deg, "penalty", 1.0, 1.0, tau_div=np.array([0.1]), tau_cont=np.array([t]))
    gx = 1.3
    gw = np.zeros((SP.wall_count(m), n * n, 3))
    gw[SP.wall_rows(m)[(0, 0)], :, 0] = gx
    got = SP.penalty_wall_load(pb, gw.reshape(-1)).reshape(3, n, n, n)
    _, w = gauss01(n)
    l0, _ = ends(n)
    ref = np.zeros_like(got)
    # (g.n)(v.n) with n = -e_x: (-gx)(-v_x) = gx v_x
    ref[0] = t * gx * 0.7 * 1.3 * w[None, :, None] * w[:, None, None] * l0[None, None, :]
    assert np.abs(got - ref).max() <= 1e-13


# ---------------------------------------------------------------- BDF2

def poly_law(mu0=1.0, mu_inf=0.2, lam=0.7):
    """Carreau parameters with kappa = 0, a = 2, n = 3: eta = mu_inf + (mu0 - mu_inf) (lam gdot)^2,
    a polynomial in the velocity gradient."""
    law = dict(W.carreau_law(3))
    law.update(mu0=mu0, mu_inf=mu_inf, lam=lam, kappa=0.0, a_exp=2.0, n_exp=3.0)
    return law


def test_bdf2_coefficients():
    for m in (1, 2):
        c = SP.bdf(m)
        assert abs(sum(c["alpha"]) - c["gamma0"]) <= 1e-15          # constants are steady
        assert abs(sum(c["beta"]) - 1.0) <= 1e-15                   # extrapolation of constants
    c = SP.bdf(2)
    # BDF2 differentiates t^2 exactly at t = 1 from t = 0, -1: (3/2 - 2*0 + 1/2*1) = 2
    assert abs(c["gamma0"] * 1.0 - c["alpha"][0] * 0.0 - c["alpha"][1] * 1.0 - 2.0) <= 1e-15
    # second-order extrapolation: 2 f(0) - f(-1) = f(1) for linear f
    assert abs(c["beta"][0] * 0.0 + c["beta"][1] * (-1.0) - 1.0) <= 1e-15


def test_vorticity_of_a_polynomial_field():
    deg = 2
    m = Mesh(3, 2, 2, aniso_box(3, 2, 2, 1.2, 0.8, 1.0))
    pb = Problem(m, deg, "viscous", 1.0, 1.0)
    u = interpolate(pb, lambda x: np.stack([x[:, 1] ** 2, x[:, 2] * x[:, 0], x[:, 0] * x[:, 1]], -1))
    ref = interpolate(pb, lambda x: np.stack([0 * x[:, 0], -x[:, 1], x[:, 2] - 2 * x[:, 1]], -1))
    got = SP.vorticity(pb, u).reshape(-1)
    assert np.abs(got - ref).max() <= 1e-12


def test_viscosity_projection_of_a_polynomial_law():
    deg = 3
    m = Mesh(2, 3, 2, aniso_box(2, 3, 2, 1.0, 0.9, 1.1))
    pb = Problem(m, deg, "viscous", 1.0, 1.0)
    law, s = poly_law(), 0.8
    u = interpolate(pb, lambda x: np.stack([s * x[:, 1] ** 2, 0 * x[:, 0], 0 * x[:, 0]], -1))
    nu = lambda y: law["mu_inf"] + (law["mu0"] - law["mu_inf"]) * law["lam"] ** 2 * 4 * s ** 2 * y ** 2
    ref = interpolate(Problem(m, deg, "poisson"), lambda x: nu(x[:, 1]))
    assert np.abs(SP.viscosity_projection(pb, u, law).reshape(-1) - ref).max() <= 1e-12


def test_bdf2_wall_data_closed_form():
    """u^n = u^{n-1} = s (y^2, 0, 0), b = 0, no wall data, polynomial law:
    (grad u) u = 0, curl curl u = (-2s, 0, 0), grad^S u . grad nu = (s y nu', 0, 0),
    so h_p = n_x 2 s (nu + y nu') and g_uhat = 0 on the x walls."""
    deg, dt = 3, 0.05
    m = Mesh(2, 2, 3, aniso_box(2, 2, 3, 1.0, 1.0, 1.0))
    pb = Problem(m, deg, "viscous", 1.5 / dt, 1.0)
    law, s = poly_law(), 0.6
    u = interpolate(pb, lambda x: np.stack([s * x[:, 1] ** 2, 0 * x[:, 0], 0 * x[:, 0]], -1))
    k2 = (law["mu0"] - law["mu_inf"]) * law["lam"] ** 2 * 4 * s ** 2
    from oracle.forms import _face_geo
    for side, nx_ in ((0, -1.0), (1, 1.0)):
        bc, g_uhat, h_p = SP.wall_data(pb, u, np.zeros(pb.ndof), dt, 0, side, None, u, law)
        _, xq, _, _, _ = _face_geo(pb, bc, 0, side)
        y = xq[..., 1]
        nu = law["mu_inf"] + k2 * y ** 2
        ref = nx_ * 2 * s * (nu + y * 2 * k2 * y)
        assert np.abs(h_p - ref).max() <= 1e-11 * np.abs(ref).max()
        assert np.abs(g_uhat).max() <= 1e-13


@pytest.mark.parametrize("perturb", [0.0, 0.1])
def test_bdf2_pressure_rhs_sum_for_equal_linear_states(perturb):
    """u^n = u^{n-1} = B x + d: the wall terms of sum_i beta_i (2 - 1 = 1) and
    beta_bar_0 (= 1) cancel, the vorticity and the viscosity are constant:
    the right-hand side sums to zero (BDF1 gives tr(B^2))."""
    pb = velocity_problem(2, 3, 2, 3, perturb)
    pp = SP.pressure_problem(pb.mesh, pb.degree)
    B = np.array([[0.5, 0.2, -0.3], [0.1, -0.4, 0.6], [0.8, 0.3, 0.1]])
    u = interpolate(pb, linear(B, np.array([1.0, -2.0, 0.5])))
    f = SP.ppe_rhs(pb, pp, W.uniform_vector(3, pb.ndof), u, W.uniform_vector(4, pb.ndof), 0.05, None, u,
                   W.carreau_law(3))
    assert abs(f.sum()) <= 1e-10


def test_bdf2_convective_step_of_linear_fields():
    pb = velocity_problem(3, 2, 2, 2, 0.1)
    A2 = np.array([[-0.2, 0.4, 0.1], [0.3, 0.5, -0.6], [0.2, -0.1, 0.3]])
    c2 = np.array([0.1, 0.4, -0.3])
    u1, u0 = interpolate(pb, linear(A, c0)), interpolate(pb, linear(A2, c2))
    b, dt = W.uniform_vector(2, pb.ndof), 0.05
    conv1 = interpolate(pb, lambda x: (x @ A.T + c0) @ A.T)
    conv0 = interpolate(pb, lambda x: (x @ A2.T + c2) @ A2.T)
    ref = (2 * u1 - 0.5 * u0) / 1.5 + dt / 1.5 * (b - 2 * conv1 + conv0)
    got = SP.convective_step(pb, u1, b, dt, None, u0)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("perturb", [0.0, 0.1])
def test_bdf2_rest_and_uniform_flow(perturb):
    """BDF2 steps of a fluid at rest under a gradient force (p = g.x) and of
    a uniform flow through the box (u = c, p = 0)."""
    dt = 0.05
    nx = 2
    V = W.box_vertices(nx, nx, nx, perturb) if perturb else None
    pb = Problem(Mesh(nx, nx, nx, V), 3, "viscous", 1.5 / dt, 1.0)
    law = W.carreau_law(3)
    g = np.array([0.4, -1.0, 2.5])
    b = interpolate(pb, lambda x: np.broadcast_to(g, x.shape))
    out = SP.split_step(pb, law, np.zeros(pb.ndof), b, dt, u_prev=np.zeros(pb.ndof))
    pe = node_points(out["pb_p"]).reshape(-1, 3) @ g
    assert np.abs(out["p"] - (pe - pe.mean())).max() <= 1e-10 and np.abs(out["u_new"]).max() <= 1e-10
    c = np.array([0.7, -0.4, 0.25])
    const = lambda x: np.broadcast_to(c, x.shape)
    u = interpolate(pb, const)
    out = SP.split_step(pb, law, u, np.zeros(pb.ndof), dt, g_wall=_g_wall_from(pb, const), u_prev=u)
    assert np.abs(out["u_new"] - u).max() <= 1e-10 and np.abs(out["p"]).max() <= 1e-10
