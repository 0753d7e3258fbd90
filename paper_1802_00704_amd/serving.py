"""Continuous-batching server: many simulation requests on one GPU at once.

A request is a mesh, its initial cell averages, scheme parameters and a
number of steps.  Requests wait in a FIFO queue and are admitted as soon as
a worker slot is free and their device-memory footprint fits the budget
beside the requests already running.  Each admitted request gets its own
library handle (per-mesh setup, state, CLS factors and Krylov basis stay
resident in HBM until it finishes) on its own HIP stream, driven by its own
host thread; library calls release the GIL, so the kernels of concurrent
requests overlap on the device.  When a request finishes, its memory and
slot are released and the next queued request is admitted.

Every request's arithmetic is independent of the others (own handle, own
stream, fixed-order reductions), so its result is bitwise the same alone and
in the mix.

Reported: per-step and per-solve latency percentiles (host wall time of
``gks_step`` and of its reconstruction solve), per-request queueing and end
to end latency, and throughput in cell-steps/s over the makespan.
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from ._lib import GKS_MIXED, default_params


@dataclass
class Request:
    rid: int
    mesh: object                 # gks_inputs.Mesh-like (xy, tri, edge_tag, periodic, L, bc_table)
    W0: np.ndarray               # [4, nt] initial cell averages
    steps: int
    params: dict = field(default_factory=dict)   # gks_params overrides
    arrival: float = 0.0         # seconds after the start of the stream
    # filled in by the server
    footprint: int = 0
    t_admit: float = float("nan")
    t_done: float = float("nan")
    setup_ms: float = float("nan")
    step_ms: list = field(default_factory=list)
    solve_ms: list = field(default_factory=list)
    W: np.ndarray | None = None
    error: str | None = None
    graph_steps: int = 0         # steps replayed through captured graphs
    capture_failures: int = 0    # captures that fell back to eager launches

    @property
    def nt(self) -> int:
        return int(self.mesh.tri.shape[0])


def estimate_footprint(nt: int, precision: int = 0, restart: int = 30) -> int:
    """Device bytes one handle holds for nt cells (upper estimate of the
    allocations of gks_mesh_create): FP64 matrix, factors and geometry,
    solver vectors and the Krylov basis, FP32 copies and the FP32 basis in
    the mixed form."""
    per_cell = 2300 + 380 + (7 + restart) * 160 + 400
    if precision == GKS_MIXED:
        per_cell += 1100 + (restart + 2) * 80
    return int(nt * per_cell * 1.05) + (1 << 20)


class Server:
    """FIFO queue, footprint-based admission and `slots` concurrent workers.

    runner(request, stream) does the work of one admitted request; the
    default runs it on the GPU through the library.  A different runner can
    be given (tests use one that needs no GPU)."""

    def __init__(self, slots: int = 8, hbm_budget: int | None = None, runner=None):
        self.slots = int(slots)
        if hbm_budget is None:
            import torch
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = int(free * 0.8)
        self.budget = int(hbm_budget)
        self.runner = runner or gpu_runner
        self._cv = threading.Condition()
        self._queue = collections.deque()
        self._in_use = 0
        self._active = 0
        self._closed = False
        self.peak_bytes = 0
        self.peak_active = 0
        self.completed = []

    # ----------------------------------------------------------- admission
    def submit(self, req: Request):
        if not req.footprint:
            req.footprint = estimate_footprint(req.nt, req.params.get("precision", 0),
                                               req.params.get("restart", 30))
        if req.footprint > self.budget:
            raise ValueError("request %d needs %d bytes, over the budget %d" % (req.rid, req.footprint, self.budget))
        with self._cv:
            self._queue.append(req)
            self._cv.notify_all()

    def _admit(self):
        """Next request once a slot is free and its footprint fits (FIFO)."""
        with self._cv:
            while True:
                if self._queue:
                    head = self._queue[0]
                    if self._in_use + head.footprint <= self.budget:
                        self._queue.popleft()
                        self._in_use += head.footprint
                        self._active += 1
                        self.peak_bytes = max(self.peak_bytes, self._in_use)
                        self.peak_active = max(self.peak_active, self._active)
                        return head
                elif self._closed:
                    return None
                self._cv.wait()

    def _release(self, req: Request):
        with self._cv:
            self._in_use -= req.footprint
            self._active -= 1
            self.completed.append(req)
            self._cv.notify_all()

    # ----------------------------------------------------------- running
    def _worker(self, t0: float):
        stream = None
        try:
            import torch
            if torch.cuda.is_available():
                stream = torch.cuda.Stream()
        except ImportError:
            pass
        while True:
            req = self._admit()
            if req is None:
                return
            req.t_admit = time.perf_counter() - t0
            try:
                self.runner(req, stream)
            except Exception as e:  # a failed request is reported, not fatal
                req.error = "%s: %s" % (type(e).__name__, e)
            req.t_done = time.perf_counter() - t0
            self._release(req)

    def run(self, requests, realtime: bool = True) -> dict:
        """Feed requests at their arrival times (or all at once when
        realtime is False), serve them, and return the statistics."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        self._closed = False
        t0 = time.perf_counter()
        workers = [threading.Thread(target=self._worker, args=(t0,), daemon=True) for _ in range(self.slots)]
        for w in workers:
            w.start()
        for r in reqs:
            if realtime:
                delay = r.arrival - (time.perf_counter() - t0)
                if delay > 0:
                    time.sleep(delay)
            self.submit(r)
        with self._cv:
            self._closed = True
            self._cv.notify_all()
        for w in workers:
            w.join()
        makespan = time.perf_counter() - t0
        return summarize(reqs, makespan, self)


def gpu_runner(req: Request, stream):
    """Run one request through the library on its own stream."""
    import torch
    from ._lib import GksMesh
    with torch.cuda.stream(stream):
        t = time.perf_counter()
        prm = default_params(**req.params)
        gm = GksMesh(req.mesh, prm, stream=stream)
        W = torch.tensor(np.ascontiguousarray(req.W0), dtype=torch.float64, device="cuda")
        req.setup_ms = (time.perf_counter() - t) * 1e3
        try:
            for _ in range(req.steps):
                _, info = gm.step(W)
                req.step_ms.append(info["call_ms"])
                req.solve_ms.append(info["solve_ms"])
            req.W = W.cpu().numpy()
            st = gm.stats()
            req.graph_steps, req.capture_failures = st["graph_steps"], st["capture_failures"]
        finally:
            gm.close()


def _pct(x, q):
    return float(np.percentile(np.asarray(x), q)) if len(x) else float("nan")


def summarize(reqs, makespan: float, server: Server | None = None) -> dict:
    ok = [r for r in reqs if r.error is None and r.W is not None]
    steps = [s for r in ok for s in r.step_ms]
    solves = [s for r in ok for s in r.solve_ms]
    e2e = [(r.t_done - r.arrival) * 1e3 for r in ok]
    wait = [(r.t_admit - r.arrival) * 1e3 for r in ok]
    cell_steps = sum(r.nt * r.steps for r in ok)
    span = max(r.arrival for r in reqs) if reqs else 0.0
    offered = sum(r.nt * r.steps for r in reqs) / span if span > 0 else float("nan")
    out = {
        "requests": len(reqs), "completed": len(ok), "failed": len(reqs) - len(ok),
        "makespan_s": makespan, "cell_steps": cell_steps, "throughput_cell_steps_per_s": cell_steps / makespan,
        "offered_cell_steps_per_s": offered,
        "step_ms_p50": _pct(steps, 50), "step_ms_p99": _pct(steps, 99),
        "solve_ms_p50": _pct(solves, 50), "solve_ms_p99": _pct(solves, 99),
        "request_ms_p50": _pct(e2e, 50), "request_ms_p99": _pct(e2e, 99),
        "queue_wait_ms_p50": _pct(wait, 50), "queue_wait_ms_p99": _pct(wait, 99),
        "graph_steps": sum(r.graph_steps for r in ok), "capture_failures": sum(r.capture_failures for r in reqs),
    }
    if server is not None:
        out.update({"slots": server.slots, "hbm_budget": server.budget, "peak_admitted_bytes": server.peak_bytes,
                    "peak_concurrent": server.peak_active})
    return out
