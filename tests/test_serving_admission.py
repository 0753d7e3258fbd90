"""CPU checks of the serving scheduler (no GPU): FIFO admission, the memory
budget and the slot count are never exceeded, and every request runs."""
import threading
import time

import numpy as np
import pytest

from paper_1802_00704_amd.serving import Request, Server, estimate_footprint


class FakeMesh:
    def __init__(self, nt):
        self.tri = np.zeros((nt, 3), dtype=np.int32)


def test_budget_slots_and_fifo():
    lock = threading.Lock()
    state = {"bytes": 0, "active": 0, "max_bytes": 0, "max_active": 0, "order": []}

    def runner(req, stream):
        with lock:
            state["bytes"] += req.footprint
            state["active"] += 1
            state["max_bytes"] = max(state["max_bytes"], state["bytes"])
            state["max_active"] = max(state["max_active"], state["active"])
            state["order"].append(req.rid)
        time.sleep(0.002 * (1 + req.rid % 3))
        req.W = np.zeros(1)
        with lock:
            state["bytes"] -= req.footprint
            state["active"] -= 1

    rng = np.random.default_rng(0)
    reqs = [Request(rid=i, mesh=FakeMesh(int(rng.integers(100, 1000))), W0=None, steps=1, footprint=int(rng.integers(10, 60)))
            for i in range(60)]
    srv = Server(slots=4, hbm_budget=100, runner=runner)
    stats = srv.run(reqs, realtime=False)
    assert stats["completed"] == 60 and stats["failed"] == 0
    assert state["max_bytes"] <= 100 and srv.peak_bytes <= 100
    assert state["max_active"] <= 4
    assert state["order"] == sorted(state["order"])        # FIFO admission
    assert srv.peak_active >= 2


def test_oversized_request_is_rejected():
    srv = Server(slots=1, hbm_budget=10, runner=lambda r, s: None)
    with pytest.raises(ValueError):
        srv.submit(Request(rid=0, mesh=FakeMesh(10), W0=None, steps=1, footprint=11))


def test_failed_request_is_reported_not_fatal():
    def runner(req, stream):
        if req.rid == 1:
            raise RuntimeError("boom")
        req.W = np.zeros(1)
    reqs = [Request(rid=i, mesh=FakeMesh(10), W0=None, steps=1, footprint=1) for i in range(3)]
    stats = Server(slots=2, hbm_budget=10, runner=runner).run(reqs, realtime=False)
    assert stats["completed"] == 2 and stats["failed"] == 1
    assert "boom" in reqs[1].error


def test_footprint_estimate_grows_with_size_and_mixed_form():
    assert estimate_footprint(20000, 1) > estimate_footprint(20000, 0) > estimate_footprint(10000, 0)
