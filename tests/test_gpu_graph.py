"""Solves whose iteration chunks are captured once into a HIP graph and
replayed (SolveOptions.use_graph) give the same result, bit for bit, as the
eager enqueue: same kernels in the same order.  Each graph is replayed
several times with eager work and synchronisations in between, for the
one-level and multigrid preconditioners, FP32 and FP64 preconditioning, an
odd chunk length (the ping-pong parity alternates between two cached
graphs), the mean-zero Poisson solve and the asynchronous entry points."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2506_14424_amd import Operator, SolveOptions  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def small(name, n):
    cfg = W.config(name, n)
    V = W.box_vertices(n, n, n, cfg["perturb"]) if cfg["perturb"] else None
    return cfg, V


CASES = [
    ("c1 chebyshev f32", "c1", 4, dict(precond_precision="f32"), False),
    ("c1 chebyshev f64, odd chunks", "c1", 4, dict(precond_precision="f64", check_every=3), False),
    ("c6@6 penalty chebyshev", "c6", 6, dict(precond_precision="f32"), False),
    ("c3@6 multigrid f32", "c3", 6, dict(precond_precision="f32", precond="multigrid", cheb_degree=3), True),
    ("c4p@4 mean-zero multigrid", "c4p", 4, dict(precond_precision="f32", precond="multigrid", cheb_degree=3), True),
]


@pytest.mark.parametrize("label,name,n,kw,mg", CASES, ids=[c[0] for c in CASES])
def test_graph_solve_equals_eager(label, name, n, kw, mg):
    cfg, V = small(name, n)
    op = Operator.from_config(cfg, V)
    if mg:
        op.set_multigrid()
    op.bind(with_solver=True)
    b = torch.from_numpy(W.uniform_vector(5, op.ndof)).cuda()
    eager = SolveOptions(rel_tol=1e-10, **kw)
    x_ref, info_ref = op.solve(b, opts=eager)
    say(f"[graph] {label}: eager {info_ref}")
    graph = SolveOptions(rel_tol=1e-10, use_graph=True, **kw)
    probe = torch.from_numpy(W.uniform_vector(6, op.ndof)).cuda()
    for rep in range(3):
        x, info = op.solve(b, opts=graph)
        torch.cuda.synchronize()
        assert info["status"] == info_ref["status"] == "SIPG_OK"
        assert info["iterations"] == info_ref["iterations"]
        assert torch.equal(x, x_ref), (label, rep, float((x - x_ref).abs().max()))
        op.apply(probe)                      # eager work between the replays
        torch.cuda.synchronize()
    x2, info2 = op.solve(b, opts=eager)      # and eager again afterwards
    assert torch.equal(x2, x_ref) and info2["iterations"] == info_ref["iterations"]


def test_graph_async_entry_points():
    cfg, V = small("c2", 4)
    op = Operator.from_config(cfg, V).bind(with_solver=True)
    b = torch.from_numpy(W.uniform_vector(9, op.ndof)).cuda()
    x_ref, info_ref = op.solve(b, opts=SolveOptions(rel_tol=1e-9))
    x = torch.empty_like(b)
    op.solve_begin(b, x, opts=SolveOptions(rel_tol=1e-9, use_graph=True))
    for _ in range(10000):
        op.solve_advance(4)
        torch.cuda.synchronize()
        done, info = op.solve_poll()
        if done:
            break
    assert done and info["status"] == "SIPG_OK" and info["iterations"] == info_ref["iterations"]
    assert torch.equal(x, x_ref)
