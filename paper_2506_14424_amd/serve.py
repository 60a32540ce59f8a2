"""Continuous batching of heterogeneous viscous-step solves on one GPU.

Requests (mesh size, degree, viscosity field, alpha/dt, right-hand side)
arrive over time.  The loop admits a waiting request as soon as an active
slot and enough of the device-memory budget are free (admission by the
plan's exact footprint: its workspace plus the request's b and x), binds its
plan on one of a pool of HIP streams, and then interleaves all active solves:
every round enqueues a few CG iterations of each active solve on its own
stream without any host synchronisation, so the kernels of different
requests overlap on the device, and polls each solve's asynchronous status
read-back.  Finished requests release their memory immediately, which lets
queued ones in.  Each solve is the library's deterministic sequence of
kernels on its own data, so its result does not depend on what else runs.

The device work sits behind a small executor interface (footprint, start,
advance, poll, release) so the scheduling logic can be exercised without a
GPU.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    id: int
    arrival: float              # seconds after the start of the run
    cfg: dict                   # operator description (nx, ny, nz, degree, op, alpha, penalty, law, bc)
    rhs: object                 # host FP64 right-hand side, or a callable producing it
    vertices: np.ndarray | None = None
    tol: float = 1e-8
    # filled in by the server
    admitted: float | None = None
    finished: float | None = None
    info: dict | None = None
    footprint: int = 0
    x: object = None


class GpuExecutor:
    """Runs each request as one libsipg plan on a pool of HIP streams, by
    default preconditioned by FP32 hp-multigrid V-cycles."""

    def __init__(self, n_streams: int = 8, precond: str = "f32", keep_solutions: bool = False,
                 depth: int = 2, multigrid: bool = True, smooth_degree: int = 4):
        import torch
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]   # default priority
        self.precond = precond
        self.keep = keep_solutions
        self.depth = depth
        self.multigrid = multigrid
        self.smooth_degree = smooth_degree
        self._rr = 0

    def prepare(self, req: Request):
        from .operator import Operator
        op = Operator.from_config(req.cfg, req.vertices)
        if self.multigrid:
            op.set_multigrid()
        return op, op.workspace_bytes(True) + 256 + 2 * 8 * op.ndof

    def start(self, req: Request, op):
        import torch
        from .operator import SolveOptions
        stream = self.streams[self._rr % len(self.streams)]
        self._rr += 1
        with torch.cuda.stream(stream):
            rhs = req.rhs() if callable(req.rhs) else req.rhs
            b = torch.from_numpy(np.ascontiguousarray(rhs, dtype=np.float64)).to("cuda")
            x = torch.empty_like(b)
            op.bind(with_solver=True, stream=stream)
            opts = (SolveOptions(rel_tol=req.tol, precond_precision=self.precond, precond="multigrid",
                                 cheb_degree=self.smooth_degree) if self.multigrid
                    else SolveOptions(rel_tol=req.tol, precond_precision=self.precond))
            op.solve_begin(b, x, opts, stream=stream)
        return (op, b, x, stream, [])

    def advance(self, handle, iters: int):
        """Enqueue `iters` more iterations, keeping at most `depth` rounds in
        flight per request: a request whose earlier rounds are still queued
        on its stream gets no new work this round, so a solve that has
        converged on the device is seen by poll() after at most that many
        rounds instead of after an ever-growing queue of skipped kernels."""
        import torch
        inflight = handle[4]
        while inflight and inflight[0].query():
            inflight.pop(0)
        if len(inflight) >= self.depth:
            return
        handle[0].solve_advance(iters)
        ev = torch.cuda.Event()
        ev.record(handle[3])
        inflight.append(ev)

    def poll(self, handle):
        return handle[0].solve_poll()

    def release(self, req: Request, handle):
        if self.keep:
            req.x = handle[2].detach().clone()


class ServingStall(RuntimeError):
    """No active request finished for `stall_timeout` seconds."""


class Server:
    def __init__(self, executor, hbm_budget: int = 8 << 30, max_active: int = 32,
                 iters_per_round: int = 4, stall_timeout: float = 120.0):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_active = max_active
        self.iters = iters_per_round
        self.stall_timeout = stall_timeout
        self.used = 0
        self.peak_used = 0
        self.peak_active = 0

    def run(self, requests: list[Request], clock=time.perf_counter, sleep=time.sleep) -> dict:
        pending = sorted(requests, key=lambda r: r.arrival)
        waiting: list = []            # (request, prepared op)
        active: list = []             # (request, handle)
        completed: list[Request] = []
        t0 = clock()
        i = 0
        last_progress = 0.0           # time of the last completion (or of the run's start)
        while i < len(pending) or waiting or active:
            now = clock() - t0
            if active and now - last_progress > self.stall_timeout:
                # the loop only enqueues and polls; with requests on the
                # device and none finishing, the device queues have stopped
                # retiring work: report what is in flight instead of spinning
                raise ServingStall(
                    f"no request finished for {now - last_progress:.1f} s; in flight: "
                    + ", ".join(f"{r.id} (admitted {r.admitted:.2f} s)" for r, _ in active))
            while i < len(pending) and pending[i].arrival <= now:
                req = pending[i]
                op, req.footprint = self.ex.prepare(req)
                waiting.append((req, op))
                i += 1
            # admission: first come first served, by footprint and free slots
            while waiting and len(active) < self.max_active:
                req, op = waiting[0]
                if req.footprint > self.budget:
                    req.info = {"status": "SIPG_ERR_OOM", "iterations": 0}
                    req.admitted = req.finished = now
                    completed.append(req)
                    waiting.pop(0)
                    continue
                if self.used + req.footprint > self.budget:
                    break
                waiting.pop(0)
                try:
                    handle = self.ex.start(req, op)
                except Exception as exc:          # isolate a failing request
                    req.info = {"status": f"failed: {exc}", "iterations": 0}
                    req.admitted = req.finished = now
                    completed.append(req)
                    continue
                self.used += req.footprint
                self.peak_used = max(self.peak_used, self.used)
                req.admitted = now
                active.append((req, handle))
            self.peak_active = max(self.peak_active, len(active))
            if not active:
                if i < len(pending) and not waiting:
                    sleep(max(0.0, min(pending[i].arrival - (clock() - t0), 0.01)))
                continue
            for _, h in active:           # enqueue: no host synchronisation
                self.ex.advance(h, self.iters)
            still = []
            for req, h in active:
                try:
                    done, info = self.ex.poll(h)
                except Exception as exc:
                    done, info = True, {"status": f"failed: {exc}", "iterations": -1}
                if done:
                    req.finished = clock() - t0
                    last_progress = req.finished
                    req.info = info
                    self.ex.release(req, h)
                    self.used -= req.footprint
                    completed.append(req)
                else:
                    still.append((req, h))
            active = still
        t_end = clock() - t0
        return summarize(completed, min((r.arrival for r in requests), default=0.0), t_end,
                         peak_reserved=self.peak_used, budget=self.budget, peak_active=self.peak_active)


def _ndof(cfg):
    n = cfg["degree"] + 1
    return cfg["nx"] * cfg["ny"] * cfg["nz"] * (3 if cfg["op"] == "viscous" else 1) * n ** 3


def summarize(completed, t_start, t_end, **extra) -> dict:
    good = [r for r in completed if r.info.get("status") == "SIPG_OK"]
    lat = np.array([r.finished - r.arrival for r in good])
    wait = np.array([r.admitted - r.arrival for r in completed])
    its = np.array([r.info.get("iterations", 0) for r in completed])
    span = max(t_end - t_start, 1e-9)
    pct = lambda a, q: float(np.percentile(a, q)) if len(a) else None
    out = {
        # throughput and latency count converged solves only; the others are listed
        "requests": len(completed), "converged": len(good),
        "failed": {str(r.id): r.info.get("status") for r in completed if r not in good},
        "solves_per_s": len(good) / span,
        "latency_p50_s": pct(lat, 50), "latency_p99_s": pct(lat, 99),
        "queue_wait_p50_s": pct(wait, 50), "queue_wait_p99_s": pct(wait, 99),
        "iterations_mean": float(its.mean()) if len(its) else None,
        "iterations_max": int(its.max()) if len(its) else None,
        "dofs_total": int(sum(_ndof(r.cfg) for r in completed)),
        "span_s": span,
    }
    out.update(extra)
    return out
