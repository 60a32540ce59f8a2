"""GPU hp-multigrid (Sec. 5.3) against the oracle: the level hierarchy, the
transfer kernels (restriction and prolongation, degree and mesh steps), one
V-cycle application, and multigrid-preconditioned solves."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle import multigrid as MG  # noqa: E402
from oracle.forms import Problem, apply as oracle_apply  # noqa: E402
from oracle.solvers import chebyshev_jacobi, lanczos_max, solve as oracle_solve  # noqa: E402
from oracle.forms import diagonal as oracle_diagonal  # noqa: E402
from paper_2506_14424_amd import Operator, SolveOptions  # noqa: E402


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def small_curved(nx, ny, nz, deg, op="viscous"):
    cfg = W.config("c2")
    cfg.update(nx=nx, ny=ny, nz=nz, degree=deg, op=op)
    if op == "poisson":
        cfg.update(alpha=1.0)
    return cfg, W.box_vertices(nx, ny, nz, cfg["perturb"])


def test_hierarchy_matches_oracle_levels():
    for cfg, V, mc in ((W.config("c1"), None, 2), (*small_curved(4, 2, 6, 3), 1)):
        op = Operator.from_config(cfg, V).set_multigrid(min_cells=mc)
        pb = Problem.from_config(cfg, V)
        ref = [(p.degree, p.mesh.nx, p.mesh.ny, p.mesh.nz) for p in MG.level_problems(pb, min_cells=mc)]
        print(f"[mg] levels {op.multigrid_levels()}", flush=True)
        assert op.multigrid_levels() == ref


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-13), (torch.float32, 2e-6)])
@pytest.mark.parametrize("op_kind", ["viscous", "poisson"])
def test_transfers_match_oracle(dtype, tol, op_kind):
    cfg, V = small_curved(4, 2, 6, 3, op_kind)
    op = Operator.from_config(cfg, V).set_multigrid(min_cells=1).bind(with_solver=True)
    pb = Problem.from_config(cfg, V)
    levels = MG.level_problems(pb, min_cells=1)
    rng = np.random.default_rng(7)
    for l in range(len(levels) - 1):
        P = MG.prolongation(levels[l], levels[l + 1])
        vf = rng.uniform(-1, 1, levels[l].ndof)
        vc = rng.uniform(-1, 1, levels[l + 1].ndof)
        print(f"[mg] {op_kind} {dtype} level {l} -> {l + 1}: {levels[l].ndof} -> {levels[l + 1].ndof}", flush=True)
        rc = torch.zeros(levels[l + 1].ndof, dtype=dtype, device="cuda")
        op.multigrid_transfer(l, torch.from_numpy(vf).to("cuda", dtype), True, out=rc)
        assert rel(rc.double().cpu().numpy(), P.T @ vf) <= tol
        zf = torch.from_numpy(vf).to("cuda", dtype)                  # prolongation adds into the output
        op.multigrid_transfer(l, torch.from_numpy(vc).to("cuda", dtype), False, out=zf)
        assert rel(zf.double().cpu().numpy(), vf + P @ vc) <= tol


@pytest.mark.parametrize("case", ["c1", "curved"])
def test_vcycle_matches_oracle(case):
    if case == "c1":
        cfg, V = W.config("c1"), None
    else:
        cfg, V = small_curved(4, 4, 4, 3)
    pb = Problem.from_config(cfg, V)
    H = MG.Hierarchy(pb, smooth_degree=3, coarse_degree=12)
    op = Operator.from_config(cfg, V).set_multigrid(coarse_degree=12, continuous=False).bind(with_solver=True)
    r = W.uniform_vector(11, pb.ndof)
    opts = SolveOptions(precond_precision="f64", cheb_degree=3, precond="multigrid")
    z = op.precondition(torch.from_numpy(r).cuda(), opts=opts).cpu().numpy()
    ref = H.vcycle(r)
    err = float(np.linalg.norm(z - ref) / np.linalg.norm(ref))
    print(f"[mg] {case}: V-cycle rel. diff {err:.2e}", flush=True)
    assert err <= 1e-12
    # the one-level Chebyshev-Jacobi preconditioner through the same entry point
    zc = op.precondition(torch.from_numpy(r).cuda(),
                         opts=SolveOptions(precond_precision="f64", cheb_degree=5)).cpu().numpy()
    dinv = H.dinv[0]
    lam = lanczos_max(lambda v: oracle_apply(pb, v), dinv)
    refc = chebyshev_jacobi(lambda v: oracle_apply(pb, v), dinv, r, 5, 1.2 * lam, 1.2 * lam / 20)
    errc = float(np.linalg.norm(zc - refc) / np.linalg.norm(refc))
    # the same one-level polynomial with the operator applied in FP32 (the
    # mixed-precision preconditioner as the solves use it)
    zc32 = op.precondition(torch.from_numpy(r).cuda(),
                           opts=SolveOptions(precond_precision="f32", cheb_degree=5)).cpu().numpy()
    errc32 = float(np.linalg.norm(zc32 - refc) / np.linalg.norm(refc))
    errc32m = float(np.abs(zc32 - refc).max() / np.abs(refc).max())
    # FP32 V-cycle: the same operator up to single-precision rounding
    z32 = op.precondition(torch.from_numpy(r).cuda(), opts=SolveOptions(
        precond_precision="f32", cheb_degree=3, precond="multigrid")).cpu().numpy()
    err32 = float(np.linalg.norm(z32 - ref) / np.linalg.norm(ref))
    print(f"[mg] {case}: one-level FP64 {errc:.2e}, one-level FP32 {errc32:.2e} (max {errc32m:.2e}), "
          f"V-cycle FP32 {err32:.2e}", flush=True)
    assert errc <= 1e-12
    assert errc32 <= 1e-5 and errc32m <= 1e-5
    assert err32 <= 1e-4


def test_multigrid_solve_matches_oracle_solver():
    cfg, V = small_curved(4, 4, 4, 3)
    pb = Problem.from_config(cfg, V)
    H = MG.Hierarchy(pb, smooth_degree=3, coarse_degree=12)
    b = W.uniform_vector(5, pb.ndof)
    A = lambda v: oracle_apply(pb, v)
    _, ref = oracle_solve(A, 1.0 / H.dinv[0], b, tol=1e-10, precond=H.vcycle)
    _, cheb = oracle_solve(A, 1.0 / H.dinv[0], b, tol=1e-10)
    op = Operator.from_config(cfg, V).set_multigrid(coarse_degree=12, continuous=False).bind(with_solver=True)
    for prec in ("f64", "f32"):
        x, info = op.solve(torch.from_numpy(b).cuda(), opts=SolveOptions(
            rel_tol=1e-10, precond_precision=prec, cheb_degree=3, precond="multigrid"))
        xr = x.cpu().numpy()
        res = float(np.linalg.norm(b - A(xr)) / np.linalg.norm(b))
        print(f"[mg] solve {prec}: {info}; oracle MG {ref['iterations']} its, one-level {cheb['iterations']} its; "
              f"oracle residual {res:.2e}", flush=True)
        assert info["status"] == "SIPG_OK" and res <= 1.0001e-10
        assert abs(info["iterations"] - ref["iterations"]) <= (1 if prec == "f64" else 3)
        assert info["iterations"] < cheb["iterations"] / 2


def test_multigrid_neumann_poisson_solve():
    cfg = W.config("c4p", 8)
    op = Operator.from_config(cfg).set_multigrid().bind(with_solver=True)
    b = torch.from_numpy(W.uniform_vector(4, op.ndof)).cuda()
    print(f"[mg] c4p 8^3 levels {op.multigrid_levels()}", flush=True)
    x, info = op.solve(b, opts=SolveOptions(rel_tol=1e-8, precond="multigrid", cheb_degree=3))
    xc, infoc = op.solve(b, opts=SolveOptions(rel_tol=1e-8))
    print(f"[mg] multigrid {info}; chebyshev {infoc}", flush=True)
    assert info["status"] == "SIPG_OK" and info["iterations"] < infoc["iterations"] / 2
    bm = b - b.mean()
    assert float((bm - op.apply(x)).norm() / bm.norm()) <= 1.0001e-8
    assert abs(float(x.mean())) <= 1e-12 * float(x.abs().max())


def test_multigrid_full_size_c3_mixed_solve():
    cfg = W.config("c3")
    V = W.box_vertices(cfg["nx"], cfg["ny"], cfg["nz"], cfg["perturb"])
    op = Operator.from_config(cfg, V).set_multigrid().bind(with_solver=True)
    b = torch.from_numpy(W.uniform_vector(cfg["x_seed"], op.ndof)).cuda()
    x, info = op.solve(b, opts=SolveOptions(rel_tol=1e-8, precond="multigrid", cheb_degree=3))
    print(f"[mg] c3 levels {op.multigrid_levels()}: {info}", flush=True)
    assert info["status"] == "SIPG_OK" and info["iterations"] < 100
    assert float((b - op.apply(x)).norm() / b.norm()) <= 1.0001e-8
