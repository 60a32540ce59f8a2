"""Parity of the HIP operator, diagonal and viscosity evaluation with the CPU
oracle, element by element on seeded inputs.

Bars: FP64 results within 1e-12 relative (max |gpu - ref| / max |ref| and the
2-norm ratio), FP32 results within 1e-5 on the same measures, input values
identical on both sides (the FP32 input is the rounded vector, which the
oracle then evaluates in FP64).  Small meshes span several workgroups and a
ragged last workgroup; the full workload sizes are checked on sampled cells
the oracle evaluates one by one, plus properties that hold at any size.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle.basis import face_points
from oracle.forms import Problem, apply as oracle_apply, assemble, diagonal as oracle_diagonal, _cell_geo
from oracle.laws import viscosity as oracle_viscosity
from oracle.mesh import Mesh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2506_14424_amd import Operator, PART_CELL, PART_INTERIOR, PART_BOUNDARY  # noqa: E402

TOL64, TOL32 = 1e-12, 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def vertices_of(cfg):
    return W.box_vertices(cfg["nx"], cfg["ny"], cfg["nz"], cfg["perturb"])


def rel_err(y, ref):
    y, ref = np.asarray(y, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    scale = np.abs(ref).max()
    return max(np.abs(y - ref).max() / scale, np.linalg.norm(y - ref) / np.linalg.norm(ref))


def small_cases():
    out = [
        ("c1", W.config("c1")),
        ("c2@5", W.config("c2", 5)),
        ("c3@3", W.config("c3", 3)),
        ("c4p@3", W.config("c4p", 3)),
        ("c4v@3", W.config("c4v", 3)),
    ]
    mixed = W.config("c2", 3)
    mixed.update(nx=3, ny=4, nz=2, degree=1, bc=("D", "N", "N", "D", "D", "N"), name="mixed-k1")
    out.append(("mixed-k1", mixed))
    m2 = W.config("c3", 3)
    m2.update(nx=2, ny=3, nz=5, degree=2, bc=("N", "D", "D", "N", "N", "D"), name="mixed-k2")
    out.append(("mixed-k2", m2))
    p1 = W.config("c4p", 3)
    p1.update(nx=4, ny=3, nz=2, degree=4, alpha=2.5, bc=("D", "N", "D", "D", "N", "D"), perturb=0.1,
              name="poisson-curved")
    out.append(("poisson-curved", p1))
    # degenerate and ragged meshes for the octant cell order (a dimension of
    # one cell, odd counts, a partial last workgroup) on the matrix-core
    # instance (k = 3) and on k = 4
    t1 = W.config("c2", 3)
    t1.update(nx=1, ny=5, nz=3, bc=("D", "N", "D", "D", "N", "D"), name="thin-k3")
    out.append(("thin-k3", t1))
    t2 = W.config("c2", 3)
    t2.update(nx=7, ny=1, nz=2, name="ragged-k3")
    out.append(("ragged-k3", t2))
    t3 = W.config("c3", 3)
    t3.update(nx=1, ny=1, nz=1, name="single-k4")
    out.append(("single-k4", t3))
    return out


def mixed_vertices(cfg):
    if cfg["perturb"] == 0.0:
        return None
    # box_vertices scales the perturbation with 1/max(n); fine for non-cubic boxes too
    return W.box_vertices(cfg["nx"], cfg["ny"], cfg["nz"], cfg["perturb"])


@pytest.mark.parametrize("name,cfg", small_cases(), ids=[c[0] for c in small_cases()])
def test_apply_matches_oracle_small(name, cfg):
    V = mixed_vertices(cfg)
    say(f"[apply small] {name} n={cfg['nx']}x{cfg['ny']}x{cfg['nz']} k={cfg['degree']} op={cfg['op']}")
    pb = Problem.from_config(cfg, V)
    op = Operator.from_config(cfg, V).bind(with_solver=False)
    x = W.uniform_vector(cfg["x_seed"], pb.ndof)
    xt = torch.from_numpy(x).cuda()
    for parts, pname in ((PART_CELL, ("cell",)), (PART_INTERIOR, ("interior",)),
                         (PART_BOUNDARY, ("boundary",)), (7, ("cell", "interior", "boundary"))):
        ref = oracle_apply(pb, x, pname)
        if not np.any(ref):
            continue
        y = op.apply(xt, parts=parts).cpu().numpy()
        e = rel_err(y, ref)
        say(f"   parts={pname} fp64 err={e:.3e}")
        assert e <= TOL64, (name, pname, e)
    x32 = xt.float()
    ref32 = oracle_apply(pb, x32.double().cpu().numpy())
    y32 = op.apply(x32).double().cpu().numpy()
    e32 = rel_err(y32, ref32)
    say(f"   fp32 err={e32:.3e}")
    assert e32 <= TOL32


def test_apply_matches_assembled_matrix_c1():
    cfg = W.config("c1")
    pb = Problem.from_config(cfg)
    A = assemble(pb)
    op = Operator.from_config(cfg).bind(with_solver=False)
    x = W.uniform_vector(11, pb.ndof)
    y = op.apply(torch.from_numpy(x).cuda()).cpu().numpy()
    assert rel_err(y, A @ x) <= TOL64


@pytest.mark.parametrize("name,cfg", small_cases()[:5], ids=[c[0] for c in small_cases()[:5]])
def test_diagonal_matches_oracle(name, cfg):
    V = mixed_vertices(cfg)
    say(f"[diagonal] {name}")
    pb = Problem.from_config(cfg, V)
    op = Operator.from_config(cfg, V).bind(with_solver=False)
    ref = oracle_diagonal(pb)
    d = op.diagonal(torch.float64).cpu().numpy()
    assert rel_err(d, ref) <= TOL64
    dinv = op.diagonal(torch.float64, inverse=True).cpu().numpy()
    assert rel_err(dinv, 1.0 / ref) <= TOL64
    d32 = op.diagonal(torch.float32).double().cpu().numpy()
    assert rel_err(d32, ref) <= 1e-7


@pytest.mark.parametrize("name", ["c1", "c2@5", "c3@3"])
def test_viscosity_at_quadrature_points(name):
    cfg = dict(small_cases())[name]
    V = mixed_vertices(cfg)
    say(f"[viscosity] {name}")
    pb = Problem.from_config(cfg, V)
    op = Operator.from_config(cfg, V).bind(with_solver=False)
    mc, mf = (t.cpu().numpy() for t in op.viscosity_values())
    xq, _, _ = _cell_geo(pb, np.arange(pb.mesh.ncells))
    ref_c = oracle_viscosity(cfg["law"], xq).reshape(-1)
    assert np.abs(mc - ref_c).max() <= 1e-12 * np.abs(ref_c).max()
    # faces: x-faces, then y-faces, then z-faces (library numbering); the
    # points are taken from the lower cell where it exists
    m, n, nx, ny, nz = pb.mesh, pb.n, cfg["nx"], cfg["ny"], cfg["nz"]
    ref_f = []
    cell = lambda ex, ey, ez: (ez * ny + ey) * nx + ex
    faces = [(0, ex, ey, ez) for ez in range(nz) for ey in range(ny) for ex in range(nx + 1)]
    faces += [(1, ex, ey, ez) for ez in range(nz) for ey in range(ny + 1) for ex in range(nx)]
    faces += [(2, ex, ey, ez) for ez in range(nz + 1) for ey in range(ny) for ex in range(nx)]
    for d, ex, ey, ez in faces:
        pos = (ex, ey, ez)[d]
        lo = pos > 0
        ijk = [ex, ey, ez]
        if lo:
            ijk[d] -= 1
        pts, _ = face_points(n, d, 1 if lo else 0)
        ref_f.append(oracle_viscosity(cfg["law"], m.map(np.array([cell(*ijk)]), pts)[0]))
    ref_f = np.concatenate(ref_f)
    assert mf.shape == ref_f.shape
    assert np.abs(mf - ref_f).max() <= 1e-12 * np.abs(ref_f).max()


def test_apply_is_deterministic():
    cfg = W.config("c2", 6)
    V = vertices_of(cfg)
    op = Operator.from_config(cfg, V).bind(with_solver=False)
    x = torch.from_numpy(W.uniform_vector(3, op.ndof)).cuda()
    y1 = op.apply(x)
    y2 = op.apply(x)
    assert torch.equal(y1, y2)


FULL = ["c1", "c2", "c3", "c4p", "c4v"]


@pytest.mark.parametrize("name", FULL)
def test_full_size_sampled_cells(name):
    """Full workload size, the launch the bench times; 48 sampled cells
    (corners, edges and interior) evaluated by the oracle one by one."""
    cfg = W.config(name)
    V = vertices_of(cfg)
    say(f"[full size] {name} ndof={W.ndofs(cfg)}")
    pb = Problem.from_config(cfg, V)
    op = Operator.from_config(cfg, V).bind(with_solver=False)
    x = W.uniform_vector(cfg["x_seed"], pb.ndof)
    xt = torch.from_numpy(x).cuda()
    y = op.apply(xt).cpu().numpy().reshape(pb.mesh.ncells, -1)
    y32 = op.apply(xt.float()).double().cpu().numpy().reshape(pb.mesh.ncells, -1)
    rng = np.random.default_rng(0)
    nc = pb.mesh.ncells
    cells = np.unique(np.concatenate([[0, nc - 1, cfg["nx"] - 1, nc // 2], rng.integers(0, nc, 44)]))
    ref = oracle_apply(pb, x, cells=cells).reshape(nc, -1)[cells]
    e = rel_err(y[cells], ref)
    say(f"   fp64 sampled err={e:.3e}")
    assert e <= TOL64
    x32 = xt.float().double().cpu().numpy()
    ref32 = oracle_apply(pb, x32, cells=cells).reshape(nc, -1)[cells]
    e32 = rel_err(y32[cells], ref32)
    say(f"   fp32 sampled err={e32:.3e}")
    assert e32 <= TOL32


@pytest.mark.parametrize("name", ["c2", "c4p"])
def test_full_size_properties(name):
    """Symmetry u.Av = v.Au at full size; A 1 = 0 for the pure-Neumann Poisson."""
    cfg = W.config(name)
    V = vertices_of(cfg)
    op = Operator.from_config(cfg, V).bind(with_solver=False)
    u = torch.from_numpy(W.uniform_vector(21, op.ndof)).cuda()
    v = torch.from_numpy(W.uniform_vector(22, op.ndof)).cuda()
    Au, Av = op.apply(u), op.apply(v)
    a, b = float(v @ Au), float(u @ Av)
    scale = float(u.norm() * Av.norm())
    assert abs(a - b) <= 1e-12 * scale
    if name == "c4p":
        one = torch.ones(op.ndof, dtype=torch.float64, device="cuda")
        A1 = op.apply(one)
        assert float(A1.abs().max()) <= 1e-12 * float(Au.abs().max())


def test_max_size_sampled_cells():
    """Near the library's indexing limit (ndof < 2^31): 192^3 curved cells
    at k = 3, 1,358,954,496 unknowns (10.9 GB per FP64 vector), 32 sampled
    cells (corners, the last cell, random) evaluated by the oracle one by
    one, FP64 and FP32."""
    n = 192
    cfg = W.config("c2", n)
    V = W.box_vertices(n, n, n, cfg["perturb"])
    ndof = W.ndofs(cfg)
    assert 2 ** 30 < ndof < 2 ** 31 - 1
    free, _ = torch.cuda.mem_get_info()
    if free < 80 * 2 ** 30:
        pytest.skip(f"needs ~60 GB of device memory, {free / 2 ** 30:.0f} GB free")
    say(f"[max size] {n}^3 k=3: {ndof} DoFs")
    op = Operator.from_config(cfg, V).bind(with_solver=False)
    x = W.uniform_vector(cfg["x_seed"], ndof)
    xt = torch.from_numpy(x).cuda()
    y = op.apply(xt).cpu().numpy()
    y32 = op.apply(xt.float()).cpu().numpy()
    torch.cuda.synchronize()
    say("   applied")
    pb = Problem.from_config(cfg, V)
    nc = pb.mesh.ncells
    rng = np.random.default_rng(3)
    cells = np.unique(np.concatenate([[0, n - 1, nc - n, nc - 1, nc // 2], rng.integers(0, nc, 27)]))
    nl = pb.nloc
    ref = oracle_apply(pb, x, cells=cells).reshape(nc, nl)[cells]
    e = rel_err(y.reshape(nc, nl)[cells], ref)
    say(f"   fp64 sampled err={e:.3e}")
    assert e <= TOL64
    x32 = x.astype(np.float32).astype(np.float64)
    ref32 = oracle_apply(pb, x32, cells=cells).reshape(nc, nl)[cells]
    e32 = rel_err(y32.astype(np.float64).reshape(nc, nl)[cells], ref32)
    say(f"   fp32 sampled err={e32:.3e}")
    assert e32 <= TOL32
