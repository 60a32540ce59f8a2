"""Continuous batching on the GPU: every result of a mixed batch equals the
same request solved alone (the kernels are deterministic and each solve only
touches its own buffers), and every solve reaches its tolerance.  The
executor's default preconditioner is the FP32 hp-multigrid V-cycle; one test
also runs the one-level Chebyshev-Jacobi variant."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2506_14424_amd import Operator, SolveOptions  # noqa: E402
from paper_2506_14424_amd.serve import GpuExecutor, Request, Server  # noqa: E402


def test_mixed_batch_equals_solo_solves():
    stream = W.serving_requests(seed=11, count=12, rate=200.0, nmin=2, nmax=6)
    reqs = []
    for r in stream:
        cfg = r["cfg"]
        reqs.append(Request(r["id"], r["arrival"], cfg, W.uniform_vector(cfg["x_seed"], W.ndofs(cfg)),
                            None, 1e-8))
    print(f"[serve] {len(reqs)} requests, ndof {[W.ndofs(r.cfg) for r in reqs]}", flush=True)
    out = Server(GpuExecutor(keep_solutions=True), hbm_budget=256 << 20, max_active=6,
                 iters_per_round=3).run(reqs)
    print(f"   {out}", flush=True)
    for r in reqs:
        print(f"   req {r.id}: N={r.cfg['nx']} k={r.cfg['degree']} law={r.cfg['law']['kind']} "
              f"alpha={r.cfg['alpha']:.2f} -> {r.info}", flush=True)
    assert out["requests"] == 12
    assert out["peak_reserved"] <= 256 << 20
    for r in reqs:
        op = Operator.from_config(r.cfg).set_multigrid().bind()
        b = torch.from_numpy(r.rhs).cuda()
        x, info = op.solve(b, opts=SolveOptions(rel_tol=1e-8, precond="multigrid", cheb_degree=4),
                           raise_on_error=False)
        assert info["status"] == r.info["status"] and info["iterations"] == r.info["iterations"], r.id
        assert torch.equal(x, r.x), r.id
        if info["status"] == "SIPG_OK":
            assert float((b - op.apply(x)).norm() / b.norm()) <= 1.2e-8
    assert out["converged"] == 12 and not out["failed"]


def test_mixed_batch_with_chebyshev_preconditioner():
    stream = W.serving_requests(seed=12, count=6, rate=200.0, nmin=2, nmax=6)
    reqs = [Request(r["id"], r["arrival"], r["cfg"], W.uniform_vector(r["cfg"]["x_seed"], W.ndofs(r["cfg"])),
                    None, 1e-8) for r in stream]
    out = Server(GpuExecutor(keep_solutions=True, multigrid=False), hbm_budget=256 << 20, max_active=4,
                 iters_per_round=3).run(reqs)
    print(f"   {out}", flush=True)
    for r in reqs:
        op = Operator.from_config(r.cfg).bind()
        x, info = op.solve(torch.from_numpy(r.rhs).cuda(), opts=SolveOptions(rel_tol=1e-8), raise_on_error=False)
        assert info["status"] == r.info["status"] and info["iterations"] == r.info["iterations"], r.id
        assert torch.equal(x, r.x), r.id
    assert out["converged"] == 6 and not out["failed"]
