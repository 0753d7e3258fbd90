"""Continuous-batching server: many simulation requests on one GPU at once.

A request is a mesh, its initial cell averages, scheme parameters and a
number of steps.  Requests wait in a FIFO queue and are admitted as soon as
their device-memory footprint fits the budget beside the requests already
admitted.  Set-up threads build each admitted request's library handle
(per-mesh set-up, factors, Krylov basis and solution history stay resident
in HBM until it finishes) and hand it to the driver of its precision.  Each
driver (one host thread and one HIP stream per precision, FP64 and mixed)
repeatedly takes every ready request into its active set and advances all of
them by one step with gks_batch_step: every kernel of the step is one
grouped launch over the concatenated meshes of the active requests, each at
its own offset.  Requests join and leave the active set at step boundaries:
a finished request's memory is released and the next queued request is
admitted.

Each request's arithmetic is exactly that of its own eager step (the batch
runs the same kernels with each request's own arguments and grids), so its
result is bitwise the same alone and in the mix.

Reported: per-step and per-solve latency percentiles (host wall time of the
batch steps a request took part in, and of their reconstruction solves),
per-request queueing, set-up and end-to-end latency, and throughput in
cell-steps/s over the makespan.

The scheduling is independent of the GPU: `build`, `step` and `finish` can be
replaced (the CPU tests do).
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
    mesh: object                 # gks_inputs.Mesh-like (xy, tri, edge_tag, periodic, L, bc_table), or None
    W0: np.ndarray               # [4, nt] initial cell averages (None with `make`)
    steps: int
    params: dict = field(default_factory=dict)   # gks_params overrides
    arrival: float = 0.0         # seconds after the start of the stream
    make: object = None          # callable returning (mesh, W0), run at set-up when mesh is None
    nt_hint: int = 0             # cells, for admission when mesh is None
    # filled in by the server
    footprint: int = 0
    t_admit: float = float("nan")
    t_ready: float = float("nan")
    t_done: float = float("nan")
    setup_ms: float = float("nan")
    step_ms: list = field(default_factory=list)
    solve_ms: list = field(default_factory=list)
    done_steps: int = 0
    W: np.ndarray | None = None
    error: str | None = None
    state: object = None         # device state while admitted (handle, W)

    @property
    def nt(self) -> int:
        return int(self.mesh.tri.shape[0]) if self.mesh is not None else int(self.nt_hint)

    @property
    def precision(self) -> int:
        return int(self.params.get("precision", 0))


def estimate_footprint(nt: int, precision: int = 0, restart: int = 30) -> int:
    """Device bytes one request holds for nt cells (upper estimate of the
    allocations of gks_mesh_create plus its state W): FP64 matrix, factors
    and geometry, solver vectors and the Krylov basis, FP32 copies and the
    FP32 basis in the mixed form, and up to five earlier solutions for the
    extrapolated start."""
    per_cell = 2300 + 380 + (7 + restart) * 160 + 400 + 32 + 640
    if precision == GKS_MIXED:
        per_cell += 1100 + (restart + 2) * 80
    return int(nt * per_cell * 1.05) + (1 << 20)


# ------------------------------------------------------------------ GPU parts
def gpu_build(req: Request):
    """Set-up of one request (runs on a set-up thread, on its own stream)."""
    import torch
    from ._lib import GksMesh
    if req.mesh is None:
        req.mesh, req.W0 = req.make()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        gm = GksMesh(req.mesh, default_params(**dict(req.params, graphs=0)), stream=stream)
        W = torch.tensor(np.ascontiguousarray(req.W0), dtype=torch.float64, device="cuda")
    stream.synchronize()
    req.state = (gm, W)


class GpuBatchStepper:
    """One batch context (stream) per driver thread."""

    def __init__(self):
        import torch
        from ._lib import GksBatch
        self.stream = torch.cuda.Stream()
        self.batch = GksBatch(stream=self.stream)

    def __call__(self, reqs):
        res = self.batch.step([r.state[0] for r in reqs], [r.state[1] for r in reqs])
        return [(code, info["call_ms"], info["solve_ms"]) for code, _, info in res]

    def close(self):
        self.batch.close()


def gpu_finish(req: Request):
    gm, W = req.state
    if req.error is None:
        req.W = W.cpu().numpy()
    gm.close()
    req.state = None


class Server:
    """FIFO queue, footprint-based admission, set-up threads and one batch
    driver per precision.

    build(req) sets up an admitted request (req.state); stepper() makes a
    callable that advances a list of ready requests by one step together and
    returns per request (status code, step ms, solve ms); finish(req)
    collects the result and frees the request's state."""

    def __init__(self, hbm_budget: int | None = None, max_batch: int = 64, setup_threads: int = 4,
                 build=None, stepper=None, finish=None, log_every: int = 0):
        if hbm_budget is None:
            import torch
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = int(free * 0.8)
        self.budget = int(hbm_budget)
        self.max_batch = int(max_batch)
        self.setup_threads = int(setup_threads)
        self.build = build or gpu_build
        self.make_stepper = stepper or GpuBatchStepper
        self.finish = finish or gpu_finish
        self._cv = threading.Condition()
        self._queue = collections.deque()        # waiting for admission
        self._setup = collections.deque()        # admitted, waiting for set-up
        self._ready = {0: [], 1: []}             # set up, waiting to join a driver's batch
        self._in_use = 0
        self._admitted = 0                        # admitted and not yet finished
        self._closed = False
        self.peak_bytes = 0
        self.peak_admitted = 0
        self.peak_batch = 0
        self.batch_steps = 0
        self.completed = []
        self.log_every = int(log_every)   # > 0: a line on stderr every log_every finished requests

    # ----------------------------------------------------------- admission
    def submit(self, req: Request):
        if not req.footprint:
            req.footprint = estimate_footprint(req.nt, req.precision, req.params.get("restart", 30))
        if req.footprint > self.budget:
            raise ValueError("request %d needs %d bytes, over the budget %d" % (req.rid, req.footprint, self.budget))
        with self._cv:
            self._queue.append(req)
            self._admit_locked()

    def _admit_locked(self):
        """Admit queue heads while their footprints fit (FIFO; the lock is held)."""
        while self._queue and self._in_use + self._queue[0].footprint <= self.budget:
            req = self._queue.popleft()
            req.t_admit = time.perf_counter() - self._t0
            self._in_use += req.footprint
            self._admitted += 1
            self.peak_bytes = max(self.peak_bytes, self._in_use)
            self.peak_admitted = max(self.peak_admitted, self._admitted)
            self._setup.append(req)
        self._cv.notify_all()

    def _release(self, req: Request):
        req.t_done = time.perf_counter() - self._t0
        with self._cv:
            self._in_use -= req.footprint
            self._admitted -= 1
            self.completed.append(req)
            self._admit_locked()
            done = len(self.completed)
        if self.log_every > 0 and done % self.log_every == 0:
            import sys
            print("# serving: %d requests finished at %.1f s" % (done, req.t_done), file=sys.stderr, flush=True)

    def _idle_locked(self) -> bool:
        return self._closed and not self._queue and not self._setup and self._admitted == 0

    # ----------------------------------------------------------- set-up threads
    def _setup_worker(self):
        while True:
            with self._cv:
                while not self._setup and not self._idle_locked():
                    self._cv.wait()
                if not self._setup:
                    return
                req = self._setup.popleft()
            t = time.perf_counter()
            try:
                self.build(req)
            except Exception as e:  # a failed request is reported, not fatal
                req.error = "%s: %s" % (type(e).__name__, e)
            req.setup_ms = (time.perf_counter() - t) * 1e3
            req.t_ready = time.perf_counter() - self._t0
            if req.error is not None:
                if req.state is not None:
                    self.finish(req)
                self._release(req)
                continue
            with self._cv:
                self._ready[1 if req.precision == GKS_MIXED else 0].append(req)
                self._cv.notify_all()

    # ----------------------------------------------------------- batch drivers
    def _driver(self, group: int):
        stepper = self.make_stepper()
        active = []
        try:
            while True:
                with self._cv:
                    while not active and not self._ready[group] and not self._idle_locked():
                        self._cv.wait()
                    active += self._ready[group]
                    self._ready[group] = []
                    if not active:
                        return
                for q in range(0, len(active), self.max_batch):
                    chunk = active[q:q + self.max_batch]
                    self.peak_batch = max(self.peak_batch, len(chunk))
                    self.batch_steps += 1
                    try:
                        res = stepper(chunk)
                    except Exception as e:
                        res = [(None, 0.0, 0.0, "%s: %s" % (type(e).__name__, e))] * len(chunk)
                    for req, out in zip(chunk, res):
                        code, step_ms, solve_ms = out[:3]
                        if code == 0:
                            req.step_ms.append(step_ms)
                            req.solve_ms.append(solve_ms)
                            req.done_steps += 1
                        else:
                            req.error = out[3] if len(out) > 3 else "step failed with status %s" % code
                still = []
                for req in active:
                    if req.error is not None or req.done_steps >= req.steps:
                        self.finish(req)
                        self._release(req)
                    else:
                        still.append(req)
                active = still
        finally:
            close = getattr(stepper, "close", None)
            if close:
                close()

    # ----------------------------------------------------------- running
    def run(self, requests, realtime: bool = True) -> dict:
        """Feed requests at their arrival times (or all at once when
        realtime is False), serve them, and return the statistics."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        self._closed = False
        self._t0 = t0 = time.perf_counter()
        threads = [threading.Thread(target=self._setup_worker, daemon=True) for _ in range(self.setup_threads)]
        threads += [threading.Thread(target=self._driver, args=(grp,), daemon=True) for grp in (0, 1)]
        for t in threads:
            t.start()
        for r in reqs:
            if realtime:
                delay = r.arrival - (time.perf_counter() - t0)
                if delay > 0:
                    time.sleep(delay)
            self.submit(r)
        with self._cv:
            self._closed = True
            self._cv.notify_all()
        for t in threads:
            t.join()
        makespan = time.perf_counter() - t0
        return summarize(reqs, makespan, self)


def _pct(x, q):
    return float(np.percentile(np.asarray(x), q)) if len(x) else float("nan")


def summarize(reqs, makespan: float, server: Server | None = None) -> dict:
    ok = [r for r in reqs if r.error is None and r.W is not None]
    steps = [s for r in ok for s in r.step_ms]
    solves = [s for r in ok for s in r.solve_ms]
    e2e = [(r.t_done - r.arrival) * 1e3 for r in ok]
    wait = [(r.t_admit - r.arrival) * 1e3 for r in ok]
    setup = [r.setup_ms for r in ok]
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
        "setup_ms_p50": _pct(setup, 50), "setup_ms_p99": _pct(setup, 99),
    }
    if server is not None:
        out.update({"hbm_budget": server.budget, "peak_admitted_bytes": server.peak_bytes,
                    "peak_admitted": server.peak_admitted, "peak_batch": server.peak_batch,
                    "batch_steps": server.batch_steps, "max_batch": server.max_batch})
    return out
