"""The no-allocation Picard entry point, sipg_picard_solve_noalloc (work
area in the library's static device array), against sipg_picard_solve with
a caller buffer: two calls in a row, the second on a smaller problem (the
array keeps the first call's contents), each bitwise equal to the
caller-buffer solve of the same problem with the same iteration history;
plans beyond the array's size and graph replay are refused before any work."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2506_14424_amd import Operator, SolveOptions  # noqa: E402
from paper_2506_14424_amd import _ffi as F  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def problem(n, deg):
    cfg = W.config("c7", n)
    cfg["degree"] = deg
    cfg["b_scale"] = 100.0 * cfg["alpha"] / (n ** 3 * (deg + 1) ** 3)
    return cfg, W.box_vertices(n, n, n, cfg["perturb"])


def solve(cfg, V, noalloc):
    op = Operator.from_config(cfg, V).set_multigrid().bind(with_solver=True)
    b = torch.from_numpy(W.uniform_vector(cfg["x_seed"], op.ndof) * cfg["b_scale"]).cuda()
    lin = SolveOptions(rel_tol=1e-3, precond="multigrid", cheb_degree=4)
    fn = op.picard_solve_noalloc if noalloc else op.picard_solve
    x, info = fn(b, opts=lin, rel_tol=1e-8, max_iter=60)
    torch.cuda.synchronize()
    return op, b, x, info


def test_noalloc_picard_equals_caller_buffer_picard():
    cases = [("8^3 k=4", problem(8, 4)), ("4^3 k=3", problem(4, 3))]
    ref = {}
    for name, (cfg, V) in cases:
        say(f"[noalloc] caller-buffer Picard solve {name}")
        ref[name] = solve(cfg, V, False)
    for name, (cfg, V) in cases:          # two no-allocation calls in a row, the second smaller
        say(f"[noalloc] static-array Picard solve {name}")
        op, b, x, info = solve(cfg, V, True)
        _, _, xr, ir = ref[name]
        say(f"   {op.ndof} DoFs: {info['iterations']} Picard its ({info['linear_iterations']} CG), "
            f"reference {ir['iterations']} ({ir['linear_iterations']})")
        assert info["status"] == ir["status"] == "SIPG_OK"
        assert info["iterations"] == ir["iterations"] and info["linear_iterations"] == ir["linear_iterations"]
        assert info["residual_norms"] == ir["residual_norms"] and info["omegas"] == ir["omegas"]
        assert torch.equal(x, xr)
        op.update_viscosity(x)                       # the result solves the nonlinear problem
        assert float((b - op.apply(x)).norm()) <= 1.0001e-8 * info["residual_initial"]


def test_noalloc_picard_refuses_oversize_plans_and_graphs():
    cfg, V = problem(20, 4)
    op = Operator.from_config(cfg, V).bind(with_solver=True)
    assert op.ndof > F.PICARD_NOALLOC_MAX_DOF
    b = torch.ones(op.ndof, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    with pytest.raises(RuntimeError, match="static work area"):
        op.picard_solve_noalloc(b, x=x)
    assert float(x.abs().max()) == 0.0                # refused before any work
    cfg, V = problem(3, 2)
    op = Operator.from_config(cfg, V).bind(with_solver=True)
    b = torch.ones(op.ndof, dtype=torch.float64, device="cuda")
    with pytest.raises(RuntimeError, match="use_graph"):
        op.picard_solve_noalloc(b, opts=SolveOptions(rel_tol=1e-3, use_graph=True))
