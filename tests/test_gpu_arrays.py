"""GPU parity of the viscous operator with a tabulated viscosity (ARRAYS
law: mu given at every cell and face quadrature point, Sec. 4.1 stores it
pointwise) with the oracle's table path: a law tabulated at the points
reproduces the law's operator, and a rough random table (contrast 1e3)
matches the oracle per part, in FP32, on the diagonal and through a solve."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle.forms import Problem, apply as oracle_apply, diagonal as oracle_diagonal, _cell_geo, _face_geo  # noqa: E402
from oracle.laws import viscosity  # noqa: E402
from oracle.mesh import Mesh  # noqa: E402
from paper_2506_14424_amd import Operator, SolveOptions, PART_CELL, PART_INTERIOR, PART_BOUNDARY  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return max(float(np.abs(a - b).max() / np.abs(b).max()), float(np.linalg.norm(a - b) / np.linalg.norm(b)))


def tabulate(pb, law):
    m, n = pb.mesh, pb.n
    mu_c = viscosity(law, _cell_geo(pb, np.arange(m.ncells))[0])
    mu_f = np.zeros((m.nfaces, n * n))
    for d in range(3):
        for side in (0, 1):
            cells = np.arange(m.ncells)
            _, xq, _, _, _ = _face_geo(pb, cells, d, side)
            mu_f[m.face_index(d, cells, side)] = viscosity(law, xq)
    return mu_c, mu_f


def test_tabulated_law_equals_the_law():
    nx, ny, nz, deg = 3, 2, 4, 3
    V = W.box_vertices(nx, ny, nz, 0.1)
    bc = ("D", "N", "D", "D", "N", "D")
    law = W.sine_law(1.0, 0.5)
    pb = Problem(Mesh(nx, ny, nz, V, bc), deg, "viscous", 10.0, 1.0, law)
    mu_c, mu_f = tabulate(pb, law)
    tab = Operator(nx, ny, nz, deg, "viscous", 10.0, 1.0, {"kind": "arrays", "mu_cell": mu_c, "mu_face": mu_f},
                   V, bc).bind(with_solver=False)
    ref_op = Operator(nx, ny, nz, deg, "viscous", 10.0, 1.0, law, V, bc).bind(with_solver=False)
    x = torch.from_numpy(W.uniform_vector(3, pb.ndof)).cuda()
    y, yl = tab.apply(x).cpu().numpy(), ref_op.apply(x).cpu().numpy()
    e_or, e_law = rel(y, oracle_apply(pb, x.cpu().numpy())), rel(y, yl)
    say(f"[arrays] tabulated sine law: vs oracle {e_or:.2e}, vs the law on the GPU {e_law:.2e}")
    assert e_or <= 1e-12 and e_law <= 1e-12
    mc, mf = (t.cpu().numpy() for t in tab.viscosity_values())
    assert np.array_equal(mc, mu_c.reshape(-1)) and np.array_equal(mf, mu_f.reshape(-1))


@pytest.mark.parametrize("deg", [2, 4])
def test_rough_table_matches_oracle(deg):
    nx, ny, nz = 4, 3, 2
    V = W.box_vertices(nx, ny, nz, 0.1)
    m = Mesh(nx, ny, nz, V)
    n = deg + 1
    # per-cell level c_e ~ 10^U(0,3), cell points within 10 % above it, face
    # points at most 0.9 of the smaller adjacent level (face values above a
    # cell's would break the coercivity of the SIPG form)
    rng = np.random.default_rng(deg)
    c = 10.0 ** rng.uniform(0, 3, m.ncells)
    mu_c = c[:, None] * rng.uniform(1.0, 1.1, (m.ncells, n ** 3))
    lo = np.full(m.nfaces, np.inf)
    for d in range(3):
        em, ep = m.interior_faces(d)
        f = m.face_index(d, em, 1)
        lo[f] = np.minimum(c[em], c[ep])
        for side in (0, 1):
            bc = m.boundary_cells(d, side)
            lo[m.face_index(d, bc, side)] = c[bc]
    assert np.isfinite(lo).all()
    mu_f = 0.9 * lo[:, None] * rng.uniform(0.8, 1.0, (m.nfaces, n * n))
    pb = Problem(m, deg, "viscous", 10.0, 1.0, {"kind": "const", "mu": 0.0}, mu_values=(mu_c, mu_f))
    op = Operator(nx, ny, nz, deg, "viscous", 10.0, 1.0, {"kind": "arrays", "mu_cell": mu_c, "mu_face": mu_f},
                  V).bind(with_solver=True)
    x = W.uniform_vector(5, pb.ndof)
    xt = torch.from_numpy(x).cuda()
    for parts, pname in ((PART_CELL, ("cell",)), (PART_INTERIOR, ("interior",)), (PART_BOUNDARY, ("boundary",)),
                         (7, ("cell", "interior", "boundary"))):
        e = rel(op.apply(xt, parts=parts).cpu().numpy(), oracle_apply(pb, x, pname))
        say(f"[arrays] k={deg} parts={pname} fp64 err={e:.2e}")
        assert e <= 1e-12
    x32 = xt.float()
    e32 = rel(op.apply(x32).double().cpu().numpy(), oracle_apply(pb, x32.double().cpu().numpy()))
    assert e32 <= 1e-5
    assert rel(op.diagonal(torch.float64).cpu().numpy(), oracle_diagonal(pb)) <= 1e-12
    b = torch.from_numpy(W.uniform_vector(6, pb.ndof)).cuda()
    sol, info = op.solve(b, opts=SolveOptions(rel_tol=1e-10))
    res = float(np.linalg.norm(b.cpu().numpy() - oracle_apply(pb, sol.cpu().numpy())) / np.linalg.norm(b.cpu().numpy()))
    say(f"[arrays] k={deg} solve {info}; oracle residual {res:.2e}")
    assert info["status"] == "SIPG_OK" and res <= 1.0001e-10
