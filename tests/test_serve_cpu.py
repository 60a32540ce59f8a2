"""The continuous-batching scheduler without a GPU: a stand-in executor that
only counts iterations exercises admission by footprint, queueing, slots,
rejection of oversized requests and isolation of a failing request."""
import numpy as np

from paper_2506_14424_amd.serve import Request, Server


class FakeClock:
    def __init__(self, dt=0.001):
        self.t, self.dt = 0.0, dt

    def __call__(self):
        self.t += self.dt
        return self.t

    def sleep(self, s):
        self.t += s


class FakeExecutor:
    """footprint = cfg['bytes']; a solve finishes after cfg['iters'] iterations;
    cfg['fail'] makes start() raise."""

    def __init__(self):
        self.started, self.live, self.max_live_bytes, self.live_bytes = [], 0, 0, 0

    def prepare(self, req):
        return None, req.cfg["bytes"]

    def start(self, req, op):
        if req.cfg.get("fail"):
            raise RuntimeError("device error")
        self.started.append(req.id)
        self.live_bytes += req.footprint
        self.max_live_bytes = max(self.max_live_bytes, self.live_bytes)
        return {"left": req.cfg["iters"], "done": 0, "req": req}

    def advance(self, h, iters):
        step = min(iters, h["left"])
        h["left"] -= step
        h["done"] += step

    def poll(self, h):
        if h["left"] == 0:
            return True, {"status": "SIPG_OK", "iterations": h["done"]}
        return False, None

    def release(self, req, h):
        self.live_bytes -= req.footprint


def make(i, t, nbytes, iters, **kw):
    cfg = {"nx": 2, "ny": 2, "nz": 2, "degree": 2, "op": "viscous", "bytes": nbytes, "iters": iters}
    cfg.update(kw)
    return Request(i, t, cfg, np.zeros(1))


def test_admission_respects_budget_and_fifo():
    ex = FakeExecutor()
    reqs = [make(i, 0.001 * i, 300, 20) for i in range(10)]
    clk = FakeClock()
    out = Server(ex, hbm_budget=1000, max_active=8, iters_per_round=4).run(reqs, clock=clk, sleep=clk.sleep)
    assert out["requests"] == 10 and out["converged"] == 10
    assert ex.max_live_bytes <= 1000 and out["peak_reserved"] <= 1000
    assert out["peak_active"] == 3                  # 3 x 300 fits, 4 does not
    assert ex.started == list(range(10))            # first come, first served
    assert out["queue_wait_p99_s"] > 0              # later requests had to wait


def test_slots_limit_concurrency():
    ex = FakeExecutor()
    reqs = [make(i, 0.0, 1, 8) for i in range(12)]
    clk = FakeClock()
    out = Server(ex, hbm_budget=10 ** 9, max_active=5, iters_per_round=2).run(reqs, clock=clk, sleep=clk.sleep)
    assert out["peak_active"] == 5 and out["requests"] == 12


def test_oversized_request_is_rejected_and_others_proceed():
    ex = FakeExecutor()
    reqs = [make(0, 0.0, 50, 4), make(1, 0.0, 5000, 4), make(2, 0.0, 50, 4)]
    clk = FakeClock()
    out = Server(ex, hbm_budget=1000).run(reqs, clock=clk, sleep=clk.sleep)
    st = {r.id: r.info["status"] for r in reqs}
    assert st == {0: "SIPG_OK", 1: "SIPG_ERR_OOM", 2: "SIPG_OK"}
    assert out["converged"] == 2 and out["failed"] == {"1": "SIPG_ERR_OOM"}
    assert out["solves_per_s"] == 2 / out["span_s"]     # only converged solves count


def test_failing_request_is_isolated():
    ex = FakeExecutor()
    reqs = [make(0, 0.0, 10, 6), make(1, 0.0, 10, 6, fail=True), make(2, 0.01, 10, 6)]
    clk = FakeClock()
    out = Server(ex, hbm_budget=100).run(reqs, clock=clk, sleep=clk.sleep)
    assert reqs[1].info["status"].startswith("failed")
    assert reqs[0].info["status"] == reqs[2].info["status"] == "SIPG_OK"
    assert ex.live_bytes == 0 and out["requests"] == 3
    assert list(out["failed"]) == ["1"] and out["converged"] == 2


def test_latency_accounts_for_arrival_times():
    ex = FakeExecutor()
    reqs = [make(0, 0.5, 10, 4), make(1, 1.0, 10, 4)]
    clk = FakeClock(dt=0.01)
    Server(ex, hbm_budget=100, iters_per_round=1).run(reqs, clock=clk, sleep=clk.sleep)
    for r in reqs:
        assert r.admitted >= r.arrival and r.finished > r.admitted
        assert r.finished - r.arrival < 0.5


class OutOfOrderExecutor(FakeExecutor):
    """Each solve needs a seeded random number of polls before its status
    read-back shows it done (device work of different streams finishing in
    any order, polls that find nothing new)."""

    def __init__(self, seed):
        super().__init__()
        self.rng = np.random.default_rng(seed)

    def start(self, req, op):
        h = super().start(req, op)
        h["polls"] = int(self.rng.integers(1, 40))
        return h

    def poll(self, h):
        h["polls"] -= 1
        if h["left"] == 0 and h["polls"] <= 0:
            return True, {"status": "SIPG_OK", "iterations": h["done"]}
        return False, None


def test_out_of_order_completion_drains_every_request():
    for seed in range(5):
        ex = OutOfOrderExecutor(seed)
        reqs = [make(i, 0.002 * i, 100 + 37 * (i % 5), 3 + i % 7) for i in range(40)]
        clk = FakeClock()
        out = Server(ex, hbm_budget=600, max_active=6, iters_per_round=2).run(reqs, clock=clk, sleep=clk.sleep)
        assert out["requests"] == 40 and out["converged"] == 40 and not out["failed"]
        assert ex.live_bytes == 0 and out["peak_reserved"] <= 600


class StuckExecutor(FakeExecutor):
    """Request 1 never finishes (its device queue stops retiring work)."""

    def poll(self, h):
        if h["req"].id == 1:
            return False, None
        return super().poll(h)


def test_stalled_device_work_is_reported_not_spun_on():
    import pytest
    from paper_2506_14424_amd.serve import ServingStall
    ex = StuckExecutor()
    reqs = [make(i, 0.0, 10, 4) for i in range(4)]
    clk = FakeClock(dt=0.01)
    with pytest.raises(ServingStall, match="in flight: 1"):
        Server(ex, hbm_budget=100, stall_timeout=5.0).run(reqs, clock=clk, sleep=clk.sleep)
