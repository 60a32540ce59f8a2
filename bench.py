"""Benchmark of the matrix-free SIPG viscous operator on one MI355X.

One step = one FP64 application y = A x of the viscous operator on the
headline workload (32^3 trilinear cells with perturbed vertices, k = 3,
mu = 10^(3 s(x)), 6,291,456 unknowns); inputs resident in device memory,
(x, y) rotated over enough buffers that they do not stay in the 256 MB
last-level cache.  Besides the headline DoF/s the line reports the FP32
(preconditioner precision) apply, the setup including the inverse diagonal,
FP64- vs FP32-preconditioned solves (one-level Chebyshev-Jacobi and
hp-multigrid) of the 24^3 k = 4 Carreau workload to 1e-8, the penalty-step
operator (applies and solves), the Picard-Aitken nonlinear viscous step, one
dual-splitting time step, the continuous-batching request loop (solves/s, p50/p99), the
roofline of the apply kernel and the CPU oracle timed on this host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
                       [--no-solve] [--no-serve] [--copy-probe] [--hot-cache]
                       [--split-only] [--apply-only c2|c3|c4v|c4p|c6]
The CPU leg (skipped by --no-cpu) times the oracle on the host and checks
the line's GPU results against it (sampled cells of every apply, the
oracle-measured residual of the solutions).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, published
FP64_PEAK_TFLOPS = 78.6          # MI355X FP64 vector, published
METRIC = "operator DoF/s FP64 vs mixed; solves/s and p50/p99 latency at 1e-8 rel. res."
KERNEL_SRC = [os.path.join(ROOT, "paper_2506_14424_amd", "csrc", f) for f in ("apply_kernel.h", "apply.hip")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_apply_c2.json")
CHECKS = []                      # GPU results the oracle leg checks


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(cfg, elem: int) -> dict:
    """Bytes an apply must move at least: x in, y out, the viscosity at cell
    and face quadrature points (stored pointwise; viscous operator) or the two
    penalty factors per cell (penalty step), the mesh vertices."""
    n = cfg["degree"] + 1
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    ncell = nx * ny * nz
    C = 1 if cfg["op"] == "poisson" else 3
    ndof = ncell * C * n ** 3
    nface = (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1)
    vec = 2 * ndof * elem
    if cfg["op"] == "viscous":
        mu = (ncell * n ** 3 + nface * n * n) * elem
    elif cfg["op"] == "penalty":
        mu = 2 * ncell * elem
    else:
        mu = 0
    verts = (nx + 1) * (ny + 1) * (nz + 1) * 3 * elem if cfg["perturb"] else 0
    return {"vectors": vec, "coefficients": mu, "vertices": verts, "total": vec + mu + verts,
            "per_dof": (vec + mu + verts) / ndof}


def kernel_hash() -> str:
    return hashlib.sha256(b"".join(open(f, "rb").read() for f in KERNEL_SRC)).hexdigest()[:16]


def time_applies(op, dtype, steps, warmup, rotate_bytes=640e6, hot=False, seed=2):
    """HIP events over `steps` applies on the torch stream, (x, y) rotated over
    pairs totalling more than the 256 MB last-level cache; with `hot`, also
    the same pair over and over (cache-resident rate)."""
    import torch
    import workloads as W
    npairs = max(1, math.ceil(rotate_bytes / (2 * op.ndof * (8 if dtype == torch.float64 else 4))))
    base = torch.from_numpy(W.uniform_vector(seed, op.ndof)).cuda().to(dtype)
    xs = [base.roll(i * 7919) for i in range(npairs)]
    ys = [torch.empty_like(base) for _ in range(npairs)]
    for i in range(warmup):
        op.apply(xs[i % npairs], ys[i % npairs])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for i in range(steps):
        op.apply(xs[i % npairs], ys[i % npairs])
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    hot_ms = None
    if hot:
        # cache-resident ("hot") rate for reference: the same pair over and over
        e2, e3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e2.record()
        for i in range(steps):
            op.apply(xs[0], ys[0])
        e3.record()
        torch.cuda.synchronize()
        hot_ms = e2.elapsed_time(e3)
    del xs, ys
    return {"wall_s": wall, "event_ms": ev_ms, "hot_event_ms": hot_ms, "pairs": npairs}


def sampled_cells(cfg, count=64, seed=9):
    """Corner cells plus seeded random cells: where the oracle checks a result."""
    import numpy as np
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    nc = nx * ny * nz
    corners = [0, nx - 1, nx * ny - 1, nc - 1]
    rnd = np.random.default_rng(seed).choice(nc, size=min(count, nc), replace=False)
    return np.unique(np.concatenate([corners, rnd]))


def rows_of(v, cfg, cells):
    """Host copy of the rows of `cells` of a device vector (cell-major layout)."""
    nc = cfg["nx"] * cfg["ny"] * cfg["nz"]
    return v.reshape(nc, -1)[cells].double().cpu().numpy()


def apply_rows(op, cfg, cells, seed):
    """FP64 and FP32 applies of the seeded input, the rows of `cells`."""
    import torch
    import workloads as W
    x = torch.from_numpy(W.uniform_vector(seed, op.ndof)).cuda()
    return {"seed": seed, "cells": cells, "f64": rows_of(op.apply(x), cfg, cells),
            "f32": rows_of(op.apply(x.float()), cfg, cells)}


def copy_probe(nbytes=1 << 30, reps=5):
    """A plain device copy of known size, for scaling HBM counters."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    return {"bytes_read": nbytes, "bytes_written": nbytes, "reps": reps}


def cpu_baseline(cfg, V):
    """The oracle's direct quadrature apply of the whole workload, once."""
    import numpy as np
    import workloads as W
    from oracle.forms import Problem, apply as oracle_apply
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    pb = Problem.from_config(cfg, V)
    x = W.uniform_vector(cfg["x_seed"], pb.ndof)
    reps, dt = 0, 0.0
    while reps < 3 and (reps == 0 or dt < 10.0):   # bounded: about 10-20 s of CPU work
        t0 = time.perf_counter()
        oracle_apply(pb, x)
        dt += time.perf_counter() - t0
        reps += 1
    return {"value": reps * pb.ndof / dt, "unit": "DoF/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{reps} full FP64 applies of the same workload by the oracle's direct quadrature "
                      f"evaluation ({pb.ndof} unknowns each, {dt:.1f} s in total, numpy/BLAS threads={threads})"}


def solve_compare(tol=1e-8):
    """c3 solved to `tol` four ways: one-level Chebyshev-Jacobi (degree 5) and
    cph-multigrid V-cycles (Chebyshev-Jacobi degree 4 on the DG level and on
    every continuous level, FP64 direct coarse solve), each with the
    preconditioner in FP64 and in FP32 (outer CG always FP64); and the FP32
    V-cycle of the all-DG hierarchy."""
    import torch
    import workloads as W
    from paper_2506_14424_amd import Operator, SolveOptions
    cfg = W.config("c3")
    V = W.box_vertices(cfg["nx"], cfg["ny"], cfg["nz"], cfg["perturb"])
    op = Operator.from_config(cfg, V).set_multigrid().bind(with_solver=True)
    b = torch.from_numpy(W.uniform_vector(cfg["x_seed"], op.ndof)).cuda()
    out = {"workload": "c3: viscous k=4, 24^3 perturbed, Carreau of a seeded velocity, "
                       f"{op.ndof} DoFs, rel. tol {tol:g}",
           "multigrid_levels": op.multigrid_levels()}
    sols = {}
    for key, prec, kind, deg, graph in (("f64_precond", "f64", "chebyshev", 5, False),
                                        ("f32_precond", "f32", "chebyshev", 5, False),
                                        ("mg_f64_precond", "f64", "multigrid", 4, False),
                                        ("mg_f32_precond", "f32", "multigrid", 4, False),
                                        ("mg_f32_precond_graph", "f32", "multigrid", 4, True)):
        opts = SolveOptions(rel_tol=tol, precond_precision=prec, precond=kind, cheb_degree=deg,
                            check_every=25 if kind == "chebyshev" else 5, use_graph=graph)
        op.solve(b, opts=opts)                       # warm (eigenvalue estimates cached after the first)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = op.solve(b, opts=opts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        sols[key] = x
        out[key] = {"seconds": dt, "iterations": info["iterations"], "rel_residual": info["rel_residual"],
                    "status": info["status"], "preconditioner": kind, "degree": deg, "hip_graph": graph}
    # the same solve with the all-DG hierarchy (no continuous levels), for comparison
    opdg = Operator.from_config(cfg, V).set_multigrid(continuous=False).bind(with_solver=True)
    opts = SolveOptions(rel_tol=tol, precond_precision="f32", precond="multigrid", cheb_degree=4, check_every=5)
    opdg.solve(b, opts=opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xdg, info = opdg.solve(b, opts=opts)
    torch.cuda.synchronize()
    out["mg_dg_f32_precond"] = {"seconds": time.perf_counter() - t0, "iterations": info["iterations"],
                                "rel_residual": info["rel_residual"], "status": info["status"],
                                "preconditioner": "multigrid, all levels DG", "degree": 4}
    del opdg, xdg
    out["speedup_mixed_over_fp64"] = out["f64_precond"]["seconds"] / out["f32_precond"]["seconds"]
    out["speedup_mg_mixed_over_mg_fp64"] = out["mg_f64_precond"]["seconds"] / out["mg_f32_precond"]["seconds"]
    out["speedup_mg_mixed_over_chebyshev_mixed"] = out["f32_precond"]["seconds"] / out["mg_f32_precond"]["seconds"]
    out["rel_diff_solutions"] = float((sols["f32_precond"] - sols["f64_precond"]).norm() / sols["f64_precond"].norm())
    out["rel_diff_solutions_mg"] = float((sols["mg_f32_precond"] - sols["f64_precond"]).norm()
                                         / sols["f64_precond"].norm())
    # for the oracle leg: the applies' rows on sampled cells and the solutions
    cells = sampled_cells(cfg)
    CHECKS.append({"section": ("solve",), "cfg": cfg, "V": V, "applies": apply_rows(op, cfg, cells, 31),
                   "solutions": {k: sols[k].cpu().numpy() for k in ("f32_precond", "mg_f32_precond",
                                                                      "mg_f64_precond")},
                   "b_seed": cfg["x_seed"], "tol": tol})
    return out


def c4_mixed(steps, warmup, tol=1e-8):
    """c4: the pressure-step Poisson operator at k = 5 (20^3 affine cells,
    all Neumann, mean-zero) solved to `tol` with FP32- and FP64-applied
    preconditioners (hp-multigrid and one-level Chebyshev-Jacobi; outer CG,
    dot products and the true-residual check in FP64), and the viscous
    operator at k = 5 on the same mesh applied in FP64 and FP32."""
    import torch
    import workloads as W
    from paper_2506_14424_amd import Operator, SolveOptions
    out = {}
    cfgp = W.config("c4p")
    op = Operator.from_config(cfgp).set_multigrid().bind(with_solver=True)
    r64 = time_applies(op, torch.float64, steps, warmup, seed=4)
    r32 = time_applies(op, torch.float32, steps, warmup, seed=4)
    b = torch.from_numpy(W.uniform_vector(cfgp["x_seed"], op.ndof)).cuda()
    bm = b - b.mean()
    res = {"workload": f"c4p: SIPG Poisson (pressure step), k=5, 20^3 affine cells, all Neumann, {op.ndof} DoFs, "
                       f"b ~ U(-1,1) seed {cfgp['x_seed']} with its mean removed, rel. tol {tol:g}",
           "multigrid_levels": op.multigrid_levels()}
    res.update(apply_entry(cfgp, op.ndof, r64, r32, steps))
    sols = {}
    for key, prec, kind, deg in (("mg_f32_precond", "f32", "multigrid", 4), ("mg_f64_precond", "f64", "multigrid", 4),
                                 ("chebyshev_f32_precond", "f32", "chebyshev", 5),
                                 ("chebyshev_f64_precond", "f64", "chebyshev", 5)):
        opts = SolveOptions(rel_tol=tol, precond_precision=prec, precond=kind, cheb_degree=deg,
                            check_every=25 if kind == "chebyshev" else 5)
        op.solve(b, opts=opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = op.solve(b, opts=opts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        sols[key] = x
        res[key] = {"seconds": dt, "iterations": info["iterations"], "status": info["status"],
                    "rel_residual": float((bm - op.apply(x)).norm() / bm.norm()),
                    "solution_mean": float(x.mean()), "solution_max_abs": float(x.abs().max())}
    res["speedup_mixed_over_fp64_mg"] = res["mg_f64_precond"]["seconds"] / res["mg_f32_precond"]["seconds"]
    res["speedup_mixed_over_fp64_chebyshev"] = (res["chebyshev_f64_precond"]["seconds"]
                                                / res["chebyshev_f32_precond"]["seconds"])
    res["rel_diff_mixed_fp64_mg"] = float((sols["mg_f32_precond"] - sols["mg_f64_precond"]).norm()
                                          / sols["mg_f64_precond"].norm())
    cells = sampled_cells(cfgp)
    CHECKS.append({"section": ("c4", "c4p"), "cfg": cfgp, "V": None, "applies": apply_rows(op, cfgp, cells, 41),
                   "solutions": {k: sols[k].cpu().numpy() for k in ("mg_f32_precond", "mg_f64_precond")},
                   "b_seed": cfgp["x_seed"], "tol": tol, "mean_zero": True})
    out["c4p"] = res
    del op, sols, b, bm
    torch.cuda.empty_cache()

    cfgv = W.config("c4v")
    op = Operator.from_config(cfgv).bind(with_solver=False)
    r64 = time_applies(op, torch.float64, steps, warmup, seed=4)
    r32 = time_applies(op, torch.float32, steps, warmup, seed=4)
    res = {"workload": f"c4v: SIPG viscous operator, k=5, 20^3 affine cells, mu = 1 + 0.5 sin sin sin, "
                       f"all-Dirichlet, alpha/dt = 10, {op.ndof} DoFs"}
    res.update(apply_entry(cfgv, op.ndof, r64, r32, steps))
    cells = sampled_cells(cfgv)
    CHECKS.append({"section": ("c4", "c4v"), "cfg": cfgv, "V": None, "applies": apply_rows(op, cfgv, cells, 42)})
    out["c4v"] = res
    del op
    torch.cuda.empty_cache()
    return out


def apply_entry(cfg, ndof, r64, r32, steps):
    """DoF/s, launch time and HBM fraction of timed FP64 and FP32 applies."""
    b64, b32 = algorithmic_bytes(cfg, 8), algorithmic_bytes(cfg, 4)
    ms64, ms32 = r64["event_ms"] / steps, r32["event_ms"] / steps
    ent = lambda ms, b: {"dof_per_s": ndof / (ms * 1e-3), "avg_launch_ms": ms,
                         "achieved_GBs": b["total"] / (ms * 1e-3) / 1e9,
                         "hbm_frac": b["total"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "algorithmic_bytes_per_dof": b["per_dof"]}
    return {"apply_f64": ent(ms64, b64), "apply_f32": ent(ms32, b32),
            "speedup_f32_over_f64": ms64 / ms32, "rotating_buffer_pairs": r64["pairs"]}


def oracle_checks(line, checks):
    """Oracle leg: every GPU result of the line against the CPU FP64 oracle.
    Applies: the rows of sampled cells (the oracle evaluates only those
    cells), max-abs error over the max-abs reference and 2-norm ratio.
    Solves: the relative residual |b - A x| / |b| of the returned solution,
    measured with the oracle's whole-operator apply."""
    import numpy as np
    import workloads as W
    from oracle.forms import Problem, apply as oracle_apply
    for c in checks:
        cfg, V = c["cfg"], c["V"]
        pb = Problem.from_config(cfg, V)
        nc = pb.mesh.ncells
        sec = line
        for k in c["section"]:
            sec = sec[k]
        out = {}
        a = c["applies"]
        x = W.uniform_vector(a["seed"], pb.ndof)
        ref = oracle_apply(pb, x, cells=a["cells"]).reshape(nc, -1)[a["cells"]]
        x32 = x.astype(np.float32).astype(np.float64)      # the FP32 apply's input, exactly
        ref32 = oracle_apply(pb, x32, cells=a["cells"]).reshape(nc, -1)[a["cells"]]
        for prec, r in (("f64", ref), ("f32", ref32)):
            d = a[prec] - r
            out[f"apply_{prec}"] = {"max_err_over_max_ref": float(np.abs(d).max() / np.abs(r).max()),
                                    "rel_l2_err": float(np.linalg.norm(d) / np.linalg.norm(r)),
                                    "cells": int(len(a["cells"]))}
        for key, xs in c.get("solutions", {}).items():
            b = W.uniform_vector(c["b_seed"], pb.ndof)
            if c.get("mean_zero"):
                b = b - b.mean()
            r = b - oracle_apply(pb, xs)
            out[f"solve_{key}_rel_residual"] = float(np.linalg.norm(r) / np.linalg.norm(b))
        sec["error_vs_oracle"] = out
        log(f"oracle check {'/'.join(c['section'])}: {json.dumps(out)}")


def penalty_step(steps, warmup, tol=1e-8):
    """c6: the penalty-step operator (mass + divergence and normal-continuity
    penalties), FP64 and FP32 applies, and mixed-precision solves with the
    one-level Chebyshev-Jacobi and the hp-multigrid preconditioners, each
    with eager kernel launches and with the iteration chunks replayed from
    captured HIP graphs (a small, launch-bound problem)."""
    import torch
    import workloads as W
    from paper_2506_14424_amd import Operator, SolveOptions
    cfg = W.config("c6")
    V = W.box_vertices(cfg["nx"], cfg["ny"], cfg["nz"], cfg["perturb"])
    op = Operator.from_config(cfg, V).set_multigrid().bind(with_solver=True)
    r64 = time_applies(op, torch.float64, steps, warmup)
    r32 = time_applies(op, torch.float32, steps, warmup)
    ms64, ms32 = r64["event_ms"] / steps, r32["event_ms"] / steps
    b64, b32 = algorithmic_bytes(cfg, 8), algorithmic_bytes(cfg, 4)
    out = {"workload": f"c6: penalty step, k=3, 16^3 perturbed, per-cell factors of a seeded velocity, "
                       f"{op.ndof} DoFs",
           "apply_f64": {"dof_per_s": op.ndof / (ms64 * 1e-3), "avg_launch_ms": ms64,
                         "achieved_GBs": b64["total"] / (ms64 * 1e-3) / 1e9,
                         "hbm_frac": b64["total"] / (ms64 * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "algorithmic_bytes_per_dof": b64["per_dof"]},
           "apply_f32": {"dof_per_s": op.ndof / (ms32 * 1e-3), "avg_launch_ms": ms32,
                         "achieved_GBs": b32["total"] / (ms32 * 1e-3) / 1e9},
           "multigrid_levels": op.multigrid_levels()}
    b = torch.from_numpy(W.uniform_vector(cfg["x_seed"], op.ndof)).cuda()
    for key, kind, deg, graph in (("chebyshev_f32_precond", "chebyshev", 5, False),
                                  ("chebyshev_f32_precond_graph", "chebyshev", 5, True),
                                  ("mg_f32_precond", "multigrid", 3, False),
                                  ("mg_f32_precond_graph", "multigrid", 3, True)):
        opts = SolveOptions(rel_tol=tol, precond_precision="f32", precond=kind, cheb_degree=deg, check_every=5,
                            use_graph=graph)
        op.solve(b, opts=opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = op.solve(b, opts=opts)
        torch.cuda.synchronize()
        out[key] = {"seconds": time.perf_counter() - t0, "iterations": info["iterations"],
                    "rel_residual": info["rel_residual"], "status": info["status"], "degree": deg,
                    "hip_graph": graph}
    return out


def picard_step(tol=1e-8):
    """c7: the nonlinear viscous step (viscosity from the velocity, Picard
    iterations) with and without Aitken relaxation, linear solves to 1e-3 with
    FP32 hp-multigrid, re-estimating the smoothers' eigenvalues after every
    viscosity update or (aitken_reuse_eigs) keeping the estimates the plan
    already holds (here: from the warm-up run), or (aitken_lanczos10)
    re-estimating them with 10 Lanczos steps instead of 20; plus the
    viscosity update alone (all levels and their diagonals)."""
    import torch
    import workloads as W
    from paper_2506_14424_amd import Operator, SolveOptions
    cfg = W.config("c7")
    V = W.box_vertices(cfg["nx"], cfg["ny"], cfg["nz"], cfg["perturb"])
    op = Operator.from_config(cfg, V).set_multigrid().bind(with_solver=True)
    b = torch.from_numpy(W.uniform_vector(cfg["x_seed"], op.ndof) * cfg["b_scale"]).cuda()
    lin = SolveOptions(rel_tol=1e-3, precond="multigrid", cheb_degree=4)
    work = torch.empty(op.picard_work_bytes() + 256, dtype=torch.uint8, device="cuda")
    out = {"workload": f"c7: nonlinear viscous step, k=4, 24^3 perturbed, Carreau law of the velocity, "
                       f"{op.ndof} DoFs, x0 = 0, rel. tol {tol:g} of the nonlinear residual"}
    reuse = SolveOptions(rel_tol=1e-3, precond="multigrid", cheb_degree=4, reuse_eigs=True)
    lz10 = SolveOptions(rel_tol=1e-3, precond="multigrid", cheb_degree=4, lanczos_steps=10)
    for key, aitken, lo in (("aitken", True, lin), ("plain", False, lin), ("aitken_reuse_eigs", True, reuse),
                            ("aitken_lanczos10", True, lz10)):
        op.picard_solve(b, opts=lo, rel_tol=tol, max_iter=60, aitken=aitken, work=work)   # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = op.picard_solve(b, opts=lo, rel_tol=tol, max_iter=60, aitken=aitken, work=work)
        torch.cuda.synchronize()
        out[key] = {"seconds": time.perf_counter() - t0, "picard_iterations": info["iterations"],
                    "cg_iterations": info["linear_iterations"], "status": info["status"],
                    "residual_reduction": info["residual_final"] / info["residual_initial"]}
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    s0.record()
    for _ in range(reps):
        op.update_viscosity(x)
    s1.record()
    torch.cuda.synchronize()
    out["update_viscosity_ms"] = s0.elapsed_time(s1) / reps
    out["speedup_aitken"] = out["plain"]["seconds"] / out["aitken"]["seconds"]
    return out


def split_step(reps=5, tol=1e-8):
    """c8: one dual-splitting time step (BDF1, lid-driven box) and a BDF2
    step from its result (also with kept eigenvalue estimates, with warm
    starts, and with the library's general 20 Lanczos steps instead of the
    split step's 10): the whole step
    (convective step, pressure right-hand side, pressure Poisson solve,
    projection, viscosity update, viscous solve, penalty factors, penalty
    solve) and each part alone; the three non-solve operators with their
    algorithmic bytes."""
    import torch
    import workloads as W
    from paper_2506_14424_amd import SolveOptions, SplitOptions, SplitStep
    cfg = W.config("c8")
    m, deg, dt = cfg["nx"], cfg["degree"], cfg["dt"]
    V = W.box_vertices(m, m, m, cfg["perturb"])
    st = SplitStep(m, m, m, deg, dt, cfg["law"], V).set_multigrid().bind()
    u0, b0 = W.split_inputs(cfg, V)
    u, b = torch.from_numpy(u0).cuda(), torch.from_numpy(b0).cuda()
    gw = torch.from_numpy(W.lid_data(cfg)).cuda()
    # the split step's default solve settings: 10-step Lanczos estimates
    mg = SolveOptions(rel_tol=tol, precond="multigrid", cheb_degree=4, lanczos_steps=10)
    opts = SplitOptions(pressure=mg, viscous=mg, penalty=SolveOptions(rel_tol=tol, lanczos_steps=10), zeta=1.0)
    un, p, info = st.step(u, b, opts=opts, g_wall=gw)              # warm: eigenvalue estimates, code paths
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        un, p, info = st.step(u, b, u_new=un, p=p, opts=opts, g_wall=gw)
    torch.cuda.synchronize()
    step_s = (time.perf_counter() - t0) / reps
    mgr = SolveOptions(rel_tol=tol, precond="multigrid", cheb_degree=4, reuse_eigs=True, lanczos_steps=10)
    ropts = SplitOptions(pressure=mg, viscous=mgr, penalty=SolveOptions(rel_tol=tol, reuse_eigs=True, lanczos_steps=10),
                         zeta=1.0)
    un_r, p_r, info_r = st.step(u, b, opts=ropts, g_wall=gw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        un_r, p_r, info_r = st.step(u, b, u_new=un_r, p=p_r, opts=ropts, g_wall=gw)
    torch.cuda.synchronize()
    step_reuse_s = (time.perf_counter() - t0) / reps
    reuse_diff = float((un_r - un).norm() / un.norm())
    wopts = SplitOptions(pressure=mg, viscous=mgr, penalty=SolveOptions(rel_tol=tol, reuse_eigs=True, lanczos_steps=10),
                         zeta=1.0, warm_start=True)
    un_w, p_w, info_w = st.step(u, b, opts=wopts, g_wall=gw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        un_w, p_w, info_w = st.step(u, b, u_new=un_w, p=p_w, opts=wopts, g_wall=gw)
    torch.cuda.synchronize()
    step_warm_s = (time.perf_counter() - t0) / reps
    warm_diff = float((un_w - un).norm() / un.norm())
    mg20 = SolveOptions(rel_tol=tol, precond="multigrid", cheb_degree=4, lanczos_steps=20)
    lopts = SplitOptions(pressure=mg20, viscous=mg20, penalty=SolveOptions(rel_tol=tol, lanczos_steps=20), zeta=1.0)
    un_l, p_l, info_l = st.step(u, b, opts=lopts, g_wall=gw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        un_l, p_l, info_l = st.step(u, b, u_new=un_l, p=p_l, opts=lopts, g_wall=gw)
    torch.cuda.synchronize()
    step_lz20_s = (time.perf_counter() - t0) / reps
    lz20_diff = float((un_l - un).norm() / un.norm())
    # BDF2 steps (u^{n-1} = the BDF1 step's input, u^n = its result): plans with gamma_0 = 3/2
    st2 = SplitStep(m, m, m, deg, dt, cfg["law"], V, order=2).set_multigrid().bind()
    un2, p2, info2 = st2.step(un, b, opts=opts, g_wall=gw, u_prev=u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        un2, p2, info2 = st2.step(un, b, u_new=un2, p=p2, opts=opts, g_wall=gw, u_prev=u)
    torch.cuda.synchronize()
    step2_s = (time.perf_counter() - t0) / reps
    del st2
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed(fn, n=20):
        fn()
        ev[0].record()
        for _ in range(n):
            fn()
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / n

    uhat = st.convective_step(u, b, g_wall=gw)
    f = st.pressure_rhs(uhat, u, b, g_wall=gw)
    uhh, rhs = st.projection(uhat, p)
    ms_conv = timed(lambda: st.convective_step(u, b, uhat=uhat, g_wall=gw))
    ms_rhs = timed(lambda: st.pressure_rhs(uhat, u, b, f=f, g_wall=gw))
    ms_proj = timed(lambda: st.projection(uhat, p))
    ms_pen = timed(lambda: st.update_penalty_factors(u))
    ms_visc = timed(lambda: st.vel.update_viscosity(u), 5)
    ms_load = timed(lambda: st.wall_load(st.vel, gw, rhs))

    def wall(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t, r

    t_p, (_, ip) = wall(lambda: st.pres.solve(f, opts=mg))
    st.vel.update_viscosity(u)
    t_v, (uv, iv) = wall(lambda: st.vel.solve(rhs, opts=mg))
    t_vc, _ = wall(lambda: st.vel.solve(rhs, opts=mg))              # eigenvalue estimates cached
    st.update_penalty_factors(u)
    t_q, (_, iq) = wall(lambda: st.pen.solve(rhs, opts=opts.penalty))
    nu, npr = st.ndof_u, st.ndof_p
    ncell = m ** 3
    nb = m ** 3 - (m - 2) ** 3                                     # cells on a wall
    verts = (m + 1) ** 3 * 3 * 8
    bytes_conv = 3 * 8 * nu + verts                                # u, b in; uhat out
    bytes_rhs = 8 * nu + 8 * npr + 2 * 8 * nb * 3 * (deg + 1) ** 3 + verts   # uhat; f; u, b of the wall cells
    bytes_proj = 3 * 8 * nu + 8 * npr + verts                      # uhat, p in; uhh, rhs out

    def kern(ms, nbytes):
        return {"avg_launch_ms": ms, "algorithmic_bytes": nbytes, "achieved_GBs": nbytes / (ms * 1e-3) / 1e9,
                "hbm_frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}

    return {"workload": f"c8: one BDF1 dual-splitting step of a lid-driven box, 24^3 perturbed cells, velocity k={deg} "
                        f"({nu} DoFs), pressure k={deg - 1} ({npr} DoFs), Carreau viscosity of u^n, dt={dt:g}, "
                        f"lid (1, 0, 0) on +z, no-slip elsewhere, solves to {tol:g} (FP32 multigrid with "
                        f"degree-4 Chebyshev-Jacobi smoothing for pressure and viscous, one-level "
                        f"Chebyshev-Jacobi for the penalty step; 10-step Lanczos estimates, the split "
                        f"step's default)",
            "step_seconds": step_s,
            "step_seconds_reuse_eigs": step_reuse_s,
            "step_seconds_reuse_eigs_warm_start": step_warm_s,
            "warm_start_iterations": {k: v["iterations"] for k, v in info_w.items()},
            "warm_start_rel_diff_u": warm_diff,
            "lanczos_steps": 10,
            "step_seconds_lanczos20": step_lz20_s,
            "lanczos20_iterations": {k: v["iterations"] for k, v in info_l.items()},
            "lanczos20_rel_diff_u": lz20_diff,
            "bdf2_step_seconds": step2_s,
            "bdf2_iterations": {k: v["iterations"] for k, v in info2.items()},
            "reuse_eigs_note": "viscous and penalty solves keep the eigenvalue estimates of an earlier "
                               "step (the preconditioner refreshed less often than the operator); every "
                               "timed step starts from the same u^n, so here the kept estimates are those "
                               "of the same operator",
            "reuse_eigs_rel_diff_u": reuse_diff,
            "iterations": {k: v["iterations"] for k, v in info.items()},
            "status": {k: v["status"] for k, v in info.items()},
            "convective_step": kern(ms_conv, bytes_conv),
            "pressure_rhs": kern(ms_rhs, bytes_rhs),
            "projection": kern(ms_proj, bytes_proj),
            "penalty_factors_ms": ms_pen,
            "viscous_wall_load_ms": ms_load,
            "viscosity_update_ms": ms_visc,
            "pressure_solve_s": t_p, "pressure_iterations": ip["iterations"],
            "viscous_solve_s": t_v, "viscous_solve_cached_eigs_s": t_vc, "viscous_iterations": iv["iterations"],
            "penalty_solve_s": t_q, "penalty_iterations": iq["iterations"]}


def split_step_32(reps=3, tol=1e-8):
    """The c8 step at the size of the paper's cavity runs (32^3 cells,
    velocity k = 4, pressure k = 3: 14.3 M unknowns): whole steps with
    fresh and with kept eigenvalue estimates, as unknowns per second and
    time step (velocity + pressure), the paper's throughput unit."""
    import torch
    import workloads as W
    from paper_2506_14424_amd import SolveOptions, SplitOptions, SplitStep
    cfg = W.config("c8", 32)
    m, deg, dt = cfg["nx"], cfg["degree"], cfg["dt"]
    V = W.box_vertices(m, m, m, cfg["perturb"])
    st = SplitStep(m, m, m, deg, dt, cfg["law"], V).set_multigrid().bind()
    u0, b0 = W.split_inputs(cfg, V)
    u, b = torch.from_numpy(u0).cuda(), torch.from_numpy(b0).cuda()
    gw = torch.from_numpy(W.lid_data(cfg)).cuda()
    out = {"workload": f"c8 family at 32^3 cells (lid-driven box): velocity k={deg} ({st.ndof_u} DoFs), pressure k={deg - 1} "
                       f"({st.ndof_p} DoFs), solves to {tol:g}",
           "unknowns": st.ndof_u + st.ndof_p}
    for key, reuse in (("fresh_eigs", False), ("reuse_eigs", True)):
        mg = SolveOptions(rel_tol=tol, precond="multigrid", cheb_degree=4, lanczos_steps=10)
        mgv = SolveOptions(rel_tol=tol, precond="multigrid", cheb_degree=4, reuse_eigs=reuse, lanczos_steps=10)
        opts = SplitOptions(pressure=mg, viscous=mgv,
                            penalty=SolveOptions(rel_tol=tol, reuse_eigs=reuse, lanczos_steps=10))
        un, p, info = st.step(u, b, opts=opts, g_wall=gw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            un, p, info = st.step(u, b, u_new=un, p=p, opts=opts, g_wall=gw)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / reps
        out[key] = {"step_seconds": sec, "unknowns_per_s_per_step": out["unknowns"] / sec,
                    "iterations": {k: v["iterations"] for k, v in info.items()}}
    out["paper_context"] = ("splitting scheme on 2x EPYC 9254 (48 cores), cavity 32^3 cells k_u=4/k_p=3, "
                            "14.4e6 unknowns, BDF2: 31.2-56.3e4 unknowns/s/core/step with constant viscosity, "
                            "12.4-36.3e4 with linearised variable viscosity, i.e. 1.5-2.7e7 and 0.6-1.7e7 "
                            "unknowns/s/step for the node; context only (different time integrator, flow and "
                            "solver settings)")
    return out


def serving(count=256, rate=20.0, budget=8 << 30):
    """c5: the seeded request stream through the continuous-batching loop."""
    import workloads as W
    from paper_2506_14424_amd.serve import GpuExecutor, Request, Server
    reqs = []
    for r in W.serving_requests(5, count, rate):
        cfg = r["cfg"]
        rhs = (lambda s=cfg["x_seed"], n=W.ndofs(cfg): W.uniform_vector(s, n))
        reqs.append(Request(r["id"], r["arrival"], cfg, rhs, None, cfg["tol"]))
    out = Server(GpuExecutor(), hbm_budget=budget).run(reqs)
    out["workload"] = (f"c5: {count} viscous-step solves, Poisson arrivals {rate:g}/s, N~U{{4..24}}, "
                       "k~U{2..5}, contrast~U{1,1e2,1e4}, alpha/dt~U[1,100], FP64 CG with FP32 hp-multigrid "
                       "V-cycles to 1e-8, HBM budget %d GiB" % (budget >> 30))
    return out


def apply_only(name, steps, warmup):
    """The timed FP64 and FP32 applies of one workload and nothing else."""
    import torch
    import workloads as W
    from paper_2506_14424_amd import Operator
    cfg = W.config(name)
    V = W.box_vertices(cfg["nx"], cfg["ny"], cfg["nz"], cfg["perturb"]) if cfg["perturb"] else None
    op = Operator.from_config(cfg, V).bind(with_solver=False)
    r64 = time_applies(op, torch.float64, steps, warmup)
    r32 = time_applies(op, torch.float32, steps, warmup)
    out = {"workload": name, "ndof": op.ndof, "steps": steps, "warmup": warmup}
    out.update(apply_entry(cfg, op.ndof, r64, r32, steps))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--copy-probe", action="store_true", help="also run a plain copy of known size")
    ap.add_argument("--split-only", action="store_true", help="only the dual-splitting step section")
    ap.add_argument("--hot-cache", action="store_true",
                    help="also time the headline apply on one (x, y) pair (last-level-cache resident)")
    ap.add_argument("--apply-only", choices=("c2", "c3", "c4v", "c4p", "c6"),
                    help="only the timed FP64 and FP32 applies of one workload (for counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the operator path has no "
                                   "multi-GPU mode (it would shard by blocks of cells with one face-trace "
                                   "exchange per apply)",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.split_only:
        print(json.dumps({"split_step": split_step(), "split_step_32": split_step_32()}), flush=True)
        return
    if args.apply_only:
        out = apply_only(args.apply_only, args.steps, args.warmup)
        if args.copy_probe:
            out["copy_probe"] = copy_probe()
        print(json.dumps(out), flush=True)
        return

    import torch
    import workloads as W
    from paper_2506_14424_amd import Operator

    cfg = W.config("c2")
    V = W.box_vertices(cfg["nx"], cfg["ny"], cfg["nz"], cfg["perturb"])
    op = Operator.from_config(cfg, V)
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ws = torch.empty(op.workspace_bytes(False) + 256, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    s0.record()
    op.bind(with_solver=False, workspace=ws)
    s1.record()
    torch.cuda.synchronize()
    setup_ms = s0.elapsed_time(s1)
    log(f"c2 bound: {op.ndof} DoFs, setup {setup_ms:.2f} ms")

    r64 = time_applies(op, torch.float64, args.steps, args.warmup, hot=args.hot_cache)
    r32 = time_applies(op, torch.float32, args.steps, args.warmup)
    CHECKS.append({"section": (), "cfg": cfg, "V": V, "applies": apply_rows(op, cfg, sampled_cells(cfg), 21)})
    k = args.steps
    ms64 = r64["event_ms"] / k
    value = op.ndof * k / r64["wall_s"]
    b64 = algorithmic_bytes(cfg, 8)
    b32 = algorithmic_bytes(cfg, 4)
    achieved = b64["total"] / (ms64 * 1e-3) / 1e9
    # HBM bytes and FP64 operations per launch measured with rocprofv3 counters
    # (FETCH_SIZE, WRITE_SIZE scaled by a plain copy of known size; SQ FP64
    # instruction counts); only used while the kernel source is unchanged
    traffic, counters = None, None
    if os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        if tr.get("kernel_hash") == kernel_hash():
            counters = tr
            traffic = tr["fetch_bytes_per_launch"] + tr["write_bytes_per_launch"]
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": k,
        "warmup": args.warmup,
        "ms_per_step": r64["wall_s"] * 1e3 / k,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "c2: SIPG viscous operator (alpha/dt) M - div(2 mu eps(u)), k=3, "
                               "32^3 hex cells with vertices perturbed by 0.1h sin sin sin (trilinear), "
                               "mu = 10^(3 s(x)) seeded smooth field, all-Dirichlet, "
                               f"{op.ndof} DoFs, FP64 apply y = A x",
                   "ndof": op.ndof, "degree": 3, "cells": 32 ** 3, "rotating_buffer_pairs": r64["pairs"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_apply<n=4,C=3,double,curved>",
                     "algorithmic_bytes_per_launch": b64["total"],
                     "algorithmic_bytes_per_dof": b64["per_dof"],
                     "avg_launch_ms": ms64,
                     "traffic_detail": None if counters is None else {
                         "fetch_bytes": counters["fetch_bytes_per_launch"],
                         "write_bytes": counters["write_bytes_per_launch"],
                         "fetch_over_algorithmic_reads": counters["fetch_bytes_per_launch"] / (b64["total"] - b64["vectors"] / 2),
                         "source": os.path.relpath(TRAFFIC_FILE, ROOT)},
                     "fp64_alu": None if counters is None else {
                         "flops_per_launch": counters["fp64_flops_per_launch"],
                         "vector_flops_per_launch": counters.get("fp64_vector_flops_per_launch"),
                         "matrix_flops_per_launch": counters.get("fp64_matrix_flops_per_launch"),
                         "flops_per_dof": counters["fp64_flops_per_launch"] / op.ndof,
                         "achieved_tflops": counters["fp64_flops_per_launch"] / (ms64 * 1e-3) / 1e12,
                         "peak_tflops": FP64_PEAK_TFLOPS,
                         "frac": counters["fp64_flops_per_launch"] / (ms64 * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                         "note": "executed FP64 operations from SQ counters (vector FMA counted twice, plus "
                                 "the 4x4x4 matrix-core products of the 1D sweeps), divided by the "
                                 "event-timed launch; the kernel reaches neither this roof nor the HBM "
                                 "roof: its VALU issue floor is 42-47 % of the launch, the rest is latency "
                                 "at 2 wavefronts per SIMD"}},
        "fp32_apply": {"dof_per_s": op.ndof * k / (r32["event_ms"] * 1e-3),
                       "avg_launch_ms": r32["event_ms"] / k,
                       "achieved_GBs": b32["total"] / (r32["event_ms"] / k * 1e-3) / 1e9,
                       "algorithmic_bytes_per_launch": b32["total"],
                       "speedup_over_fp64": r64["event_ms"] / r32["event_ms"]},
        "hot_cache": None if r64["hot_event_ms"] is None else {
            "dof_per_s": op.ndof * k / (r64["hot_event_ms"] * 1e-3),
            "note": "same (x, y) pair every step: inputs served from the 256 MB last-level cache"},
        "setup_ms": setup_ms,
        "setup_note": "plan bind: cell sizes, penalty factors, viscosity at all quadrature points, "
                      "diagonal and inverse diagonal (FP64 + FP32)",
    }
    log(f"apply f64: {ms64:.3f} ms/launch, {value:.3e} DoF/s, {achieved:.0f} GB/s algorithmic; "
        f"f32 {r32['event_ms'] / k:.3f} ms")
    if args.copy_probe:
        line["copy_probe"] = copy_probe()
    del op, ws
    torch.cuda.empty_cache()

    if not args.no_solve:
        log("solve comparison (c3) ...")
        line["solve"] = solve_compare()
        log(json.dumps(line["solve"]))
        log("mixed precision at k = 5 (c4) ...")
        line["c4"] = c4_mixed(args.steps, args.warmup)
        log(json.dumps(line["c4"]))
        log("penalty step (c6) ...")
        line["penalty_step"] = penalty_step(args.steps, args.warmup)
        log(json.dumps(line["penalty_step"]))
        log("nonlinear viscous step (c7) ...")
        line["picard"] = picard_step()
        log(json.dumps(line["picard"]))
        log("dual-splitting step (c8) ...")
        line["split_step"] = split_step()
        log(json.dumps(line["split_step"]))
        line["split_step_32"] = split_step_32()
        log(json.dumps(line["split_step_32"]))
    if not args.no_serve:
        log("serving loop (c5) ...")
        line["serving"] = serving()
        log(json.dumps(line["serving"]))
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        line["cpu_baseline"] = cpu_baseline(cfg, V)
        log(json.dumps(line["cpu_baseline"]))
        log("oracle checks of the GPU results ...")
        oracle_checks(line, CHECKS)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
