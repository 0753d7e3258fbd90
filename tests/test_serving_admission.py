"""CPU checks of the serving scheduler (no GPU), with stand-ins for the
set-up, batch step and finish of a request: FIFO admission within the
memory budget, every request runs exactly its steps, each batch step holds
requests of one precision and at most max_batch of them, requests join and
leave the batches while others run, and failures are reported, not fatal."""
import threading
import time

import numpy as np
import pytest

from paper_1802_00704_amd.serving import Request, Server, estimate_footprint


class FakeMesh:
    def __init__(self, nt):
        self.tri = np.zeros((nt, 3), dtype=np.int32)


class Log:
    def __init__(self):
        self.lock = threading.Lock()
        self.bytes = 0
        self.max_bytes = 0
        self.batches = []          # (precision set, size, {rid: step index})
        self.setup_order = []


def parts(log, fail_setup=(), fail_step=()):
    def build(req):
        if req.rid in fail_setup:
            raise RuntimeError("setup boom")
        with log.lock:
            log.bytes += req.footprint
            log.max_bytes = max(log.max_bytes, log.bytes)
            log.setup_order.append(req.rid)
        time.sleep(0.001)
        req.state = {"steps": 0}

    class Stepper:
        def __call__(self, reqs):
            with log.lock:
                log.batches.append(({r.precision for r in reqs}, len(reqs), {r.rid: r.state["steps"] for r in reqs}))
            time.sleep(0.0005 * len(reqs))
            out = []
            for r in reqs:
                r.state["steps"] += 1
                out.append((-5 if r.rid in fail_step else 0, 1.0, 0.5))
            return out

    def finish(req):
        with log.lock:
            log.bytes -= req.footprint
        if req.error is None:
            req.W = np.full(1, req.state["steps"])
        req.state = None

    return build, Stepper, finish


def requests(n, seed=0):
    rng = np.random.default_rng(seed)
    return [Request(rid=i, mesh=FakeMesh(int(rng.integers(100, 1000))), W0=None, steps=int(rng.integers(1, 8)),
                    params={"precision": int(rng.integers(0, 2))}, arrival=0.002 * i,
                    footprint=int(rng.integers(10, 60)))
            for i in range(n)]


def test_budget_fifo_batches_and_steps():
    log = Log()
    build, Stepper, finish = parts(log)
    reqs = requests(80)
    srv = Server(hbm_budget=200, max_batch=5, setup_threads=3, build=build, stepper=Stepper, finish=finish)
    stats = srv.run(reqs, realtime=True)
    assert stats["completed"] == 80 and stats["failed"] == 0
    assert log.max_bytes <= 200 and srv.peak_bytes <= 200
    admits = [r.t_admit for r in sorted(reqs, key=lambda r: r.rid)]
    assert admits == sorted(admits)                                   # FIFO admission
    for r in reqs:
        assert r.W[0] == r.steps and len(r.step_ms) == r.steps         # exactly its steps
    assert all(len(p) == 1 for p, _, _ in log.batches)               # one precision per batch
    assert max(n for _, n, _ in log.batches) <= 5 and srv.peak_batch >= 2
    # continuous batching: some batch holds requests at different steps
    assert any(len(set(steps.values())) > 1 for _, _, steps in log.batches)


def test_oversized_request_is_rejected():
    log = Log()
    build, Stepper, finish = parts(log)
    srv = Server(hbm_budget=10, build=build, stepper=Stepper, finish=finish)
    with pytest.raises(ValueError):
        srv.submit(Request(rid=0, mesh=FakeMesh(10), W0=None, steps=1, footprint=11))


def test_failures_are_reported_not_fatal():
    log = Log()
    build, Stepper, finish = parts(log, fail_setup={1}, fail_step={4})
    reqs = requests(8, seed=3)
    srv = Server(hbm_budget=1000, max_batch=4, build=build, stepper=Stepper, finish=finish)
    stats = srv.run(reqs, realtime=False)
    assert stats["completed"] == 6 and stats["failed"] == 2
    assert "setup boom" in reqs[1].error and reqs[4].error is not None
    assert log.bytes == 0 and srv._in_use == 0 and srv._admitted == 0   # everything released


def test_footprint_estimate_grows_with_size_and_mixed_form():
    assert estimate_footprint(20000, 1) > estimate_footprint(20000, 0) > estimate_footprint(10000, 0)
