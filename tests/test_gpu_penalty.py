"""GPU parity of the penalty-step operator (Sec. 4.3, "Consistent
Stabilization", eq. penalty_step) with the oracle: operator parts and whole,
diagonal, multigrid transfers of the penalty factors through V-cycles, and
preconditioned solves; full size on sampled cells and by a property that
holds at any size.

Bars as for the SIPG operators: FP64 within 1e-12 relative, FP32 within 1e-5.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import multigrid as MG
from oracle.forms import Problem, apply as oracle_apply, diagonal as oracle_diagonal, interpolate
from oracle.solvers import solve as oracle_solve

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2506_14424_amd import Operator, SolveOptions, PART_CELL, PART_INTERIOR, PART_BOUNDARY  # noqa: E402

TOL64, TOL32 = 1e-12, 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_err(y, ref):
    y, ref = np.asarray(y, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    scale = np.abs(ref).max()
    return max(np.abs(y - ref).max() / scale, np.linalg.norm(y - ref) / np.linalg.norm(ref))


def pen_case(nx, ny, nz, deg, perturb=0.1, bc=("D",) * 6, alpha=1.0, seed=6):
    """Penalty-step configuration with the workload's factor recipe on a
    smaller (possibly non-cubic) mesh."""
    V = W.box_vertices(nx, ny, nz, perturb) if perturb > 0 else None
    td, tc = W.penalty_parameters(nx, ny, nz, deg, V, seed)
    cfg = W.config("c6", 4)
    cfg.update(nx=nx, ny=ny, nz=nz, degree=deg, bc=tuple(bc), alpha=alpha, perturb=perturb,
               tau_div=td, tau_cont=tc, name=f"pen{nx}x{ny}x{nz}k{deg}")
    return cfg, V


CASES = {
    "c6@3": lambda: pen_case(3, 3, 3, 3),
    "k1-mixed": lambda: pen_case(3, 4, 2, 1, bc=("D", "N", "N", "D", "D", "N")),
    "k2-mixed": lambda: pen_case(2, 3, 5, 2, bc=("N", "D", "D", "N", "N", "D"), alpha=0.3),
    "k4-straight": lambda: pen_case(3, 2, 2, 4, perturb=0.0),
    "k5-curved": lambda: pen_case(2, 2, 3, 5, bc=("D", "D", "N", "N", "D", "D")),
}


@pytest.mark.parametrize("name", list(CASES))
def test_penalty_apply_matches_oracle(name):
    cfg, V = CASES[name]()
    say(f"[penalty apply] {name} ({cfg['nx']}x{cfg['ny']}x{cfg['nz']}, k={cfg['degree']}, bc={cfg['bc']})")
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
    e32 = rel_err(op.apply(x32).double().cpu().numpy(), ref32)
    say(f"   fp32 err={e32:.3e}")
    assert e32 <= TOL32


@pytest.mark.parametrize("name", ["c6@3", "k2-mixed", "k5-curved"])
def test_penalty_diagonal_matches_oracle(name):
    cfg, V = CASES[name]()
    say(f"[penalty diagonal] {name}")
    pb = Problem.from_config(cfg, V)
    op = Operator.from_config(cfg, V).bind(with_solver=False)
    ref = oracle_diagonal(pb)
    assert rel_err(op.diagonal(torch.float64).cpu().numpy(), ref) <= TOL64
    assert rel_err(op.diagonal(torch.float64, inverse=True).cpu().numpy(), 1.0 / ref) <= TOL64
    assert rel_err(op.diagonal(torch.float32).double().cpu().numpy(), ref) <= 1e-7


def test_penalty_rejects_bad_factors():
    cfg, V = pen_case(2, 2, 2, 2)
    bad = np.array(cfg["tau_div"])
    bad[3] = -1.0
    with pytest.raises(RuntimeError):
        Operator(2, 2, 2, 2, "penalty", 1.0, 1.0, None, V, cfg["bc"], bad, cfg["tau_cont"])
    with pytest.raises(ValueError):
        Operator(2, 2, 2, 2, "penalty", 1.0, 1.0, None, V, cfg["bc"], cfg["tau_div"][:5], cfg["tau_cont"])
    with pytest.raises(ValueError):
        Operator(2, 2, 2, 2, "penalty", 1.0, 1.0, None, V, cfg["bc"])


def test_penalty_alpha_zero_solve_is_refused():
    cfg, V = pen_case(2, 2, 2, 2, alpha=0.0)
    op = Operator.from_config(cfg, V).bind(with_solver=True)
    b = torch.ones(op.ndof, dtype=torch.float64, device="cuda")
    with pytest.raises(RuntimeError, match="singular"):
        op.solve(b)


def test_penalty_vcycle_and_solve_match_oracle():
    """Level factors are the means of the children's (mesh steps); the
    V-cycle and the preconditioned solve follow the oracle's."""
    cfg, V = pen_case(4, 4, 4, 3)
    pb = Problem.from_config(cfg, V)
    H = MG.Hierarchy(pb, smooth_degree=3, coarse_degree=12, min_cells=1)
    op = Operator.from_config(cfg, V).set_multigrid(coarse_degree=12, min_cells=1, continuous=False).bind(with_solver=True)
    ref_levels = [(p.degree, p.mesh.nx, p.mesh.ny, p.mesh.nz) for p in H.levels]
    say(f"[penalty mg] levels {op.multigrid_levels()}")
    assert op.multigrid_levels() == ref_levels
    r = W.uniform_vector(11, pb.ndof)
    z = op.precondition(torch.from_numpy(r).cuda(), opts=SolveOptions(
        precond_precision="f64", cheb_degree=3, precond="multigrid")).cpu().numpy()
    ref = H.vcycle(r)
    err = float(np.linalg.norm(z - ref) / np.linalg.norm(ref))
    say(f"   V-cycle rel. diff {err:.2e}")
    assert err <= 1e-8
    b = W.uniform_vector(5, pb.ndof)
    A = lambda v: oracle_apply(pb, v)
    _, info_ref = oracle_solve(A, 1.0 / H.dinv[0], b, tol=1e-10, precond=H.vcycle)
    for prec in ("f64", "f32"):
        x, info = op.solve(torch.from_numpy(b).cuda(), opts=SolveOptions(
            rel_tol=1e-10, precond_precision=prec, cheb_degree=3, precond="multigrid"))
        res = float(np.linalg.norm(b - A(x.cpu().numpy())) / np.linalg.norm(b))
        say(f"   solve {prec}: {info}; oracle {info_ref['iterations']} its; oracle residual {res:.2e}")
        assert info["status"] == "SIPG_OK" and res <= 1.0001e-10
        assert abs(info["iterations"] - info_ref["iterations"]) <= (1 if prec == "f64" else 3)
    xc, infoc = op.solve(torch.from_numpy(b).cuda(), opts=SolveOptions(rel_tol=1e-10))
    say(f"   one-level Chebyshev: {infoc}")
    assert infoc["status"] == "SIPG_OK"
    assert float(np.linalg.norm(b - A(xc.cpu().numpy())) / np.linalg.norm(b)) <= 1.0001e-10


def test_full_size_c6_sampled_cells_and_solve():
    """Full workload size, 48 sampled cells by the oracle, then the
    multigrid-preconditioned mixed-precision solve."""
    cfg = W.config("c6")
    V = W.box_vertices(cfg["nx"], cfg["ny"], cfg["nz"], cfg["perturb"])
    say(f"[penalty full size] c6 ndof={W.ndofs(cfg)}")
    pb = Problem.from_config(cfg, V)
    op = Operator.from_config(cfg, V).set_multigrid().bind(with_solver=True)
    x = W.uniform_vector(cfg["x_seed"], pb.ndof)
    xt = torch.from_numpy(x).cuda()
    nc = pb.mesh.ncells
    y = op.apply(xt).cpu().numpy().reshape(nc, -1)
    y32 = op.apply(xt.float()).double().cpu().numpy().reshape(nc, -1)
    rng = np.random.default_rng(0)
    cells = np.unique(np.concatenate([[0, nc - 1, cfg["nx"] - 1, nc // 2], rng.integers(0, nc, 44)]))
    ref = oracle_apply(pb, x, cells=cells).reshape(nc, -1)[cells]
    e = rel_err(y[cells], ref)
    say(f"   fp64 sampled err={e:.3e}")
    assert e <= TOL64
    ref32 = oracle_apply(pb, xt.float().double().cpu().numpy(), cells=cells).reshape(nc, -1)[cells]
    e32 = rel_err(y32[cells], ref32)
    say(f"   fp32 sampled err={e32:.3e}")
    assert e32 <= TOL32
    b = xt
    sol, info = op.solve(b, opts=SolveOptions(rel_tol=1e-8, precond="multigrid", cheb_degree=3))
    say(f"   solve: levels {op.multigrid_levels()}: {info}")
    assert info["status"] == "SIPG_OK" and info["iterations"] < 60
    assert float((b - op.apply(sol)).norm() / b.norm()) <= 1.0001e-8


def test_full_size_divergence_free_field_feels_only_the_mass():
    """u = (x^2, -2xy, 0) is continuous and divergence-free and lies in the
    space on trilinear cells for k >= 2, so with Neumann sides A u = alpha M u
    at any size (M from the diagonal of the operator with zero factors)."""
    cfg = W.config("c6")
    n = cfg["nx"]
    V = W.box_vertices(n, n, n, cfg["perturb"])
    bc = ("N",) * 6
    op = Operator(n, n, n, 3, "penalty", 1.0, 1.0, None, V, bc, cfg["tau_div"], cfg["tau_cont"]).bind(False)
    zero = np.zeros(n ** 3)
    mass = Operator(n, n, n, 3, "penalty", 1.0, 1.0, None, V, bc, zero, zero).bind(False)
    pb = Problem.from_config(dict(cfg, bc=bc), V)
    u = interpolate(pb, lambda X: np.stack([X[:, 0] ** 2, -2 * X[:, 0] * X[:, 1], 0 * X[:, 0]], axis=1))
    ut = torch.from_numpy(u).cuda()
    Au = op.apply(ut)
    Mu = mass.diagonal(torch.float64) * ut
    e = float((Au - Mu).abs().max() / Mu.abs().max())
    say(f"[penalty full size] divergence-free field: |Au - Mu| / |Mu| = {e:.2e}")
    assert e <= 1e-11
