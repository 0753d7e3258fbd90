"""Captured step graphs against eager launches, on the GPU.

gks_step with graphs on replays two captured HIP graphs per step (the solve
with its first GMRES cycle unrolled to a step budget, and copy-out, flux and
update) and continues on the host when a solve needs more.  The kernels and
their order are the same as in eager mode, with the unused steps of the
budget gated off on the device, so every step must agree BITWISE with the
eager path: state, time step and solver statistics.

Each case replays the graphs over several steps, alternates the caller's W
buffer between two allocations (the graphs must not capture it), and puts
eager library work and host synchronisations between the replays.  The
budgets and restart lengths are chosen to reach every continuation: the
whole solve in the graph, resumption inside the first cycle (budget 1 and 2),
and resumption at the start of a second cycle (restart 2 and 3).
"""
import numpy as np
import pytest

import gks_inputs as gi

torch = pytest.importorskip("torch")
import paper_1802_00704_amd as g  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda"
STEPS = 5


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def adv_case():
    m = gi.jss_mesh(20, 20, 1)
    return m, gi.density_advection_ic(m)


def sv_case():
    left, _ = gi.shock_vortex_states()
    m = gi.jss_mesh(16, 8, 3, Lx=2.0, Ly=1.0, periodic=False,
                    walls=((gi.BC_INFLOW, left), (gi.BC_OUTFLOW, None), (gi.BC_SLIP, None), (gi.BC_SLIP, None)))
    return m, gi.shock_vortex_ic(m)


def run(mesh, W0, interleave, **prm):
    """STEPS steps; returns [(W, dt, info)] after each.

    interleave: between steps, eager work on a second handle of the same
    mesh (a reconstruction solve) and on this handle (a flux evaluation,
    which leaves the solver state alone), then a device synchronisation.
    The solver warm-starts from the previous solution, so a reconstruction
    on the stepping handle itself would change the next solve."""
    gm = g.GksMesh(mesh, **prm)
    other = g.GksMesh(mesh, graphs=0) if interleave else None
    bufs = [dev(W0), torch.empty((4, W0.shape[1]), dtype=torch.float64, device=DEV)]
    cur = 0
    out = []
    try:
        for _ in range(STEPS):
            nxt = 1 - cur
            bufs[nxt].copy_(bufs[cur])
            dt, info = gm.step(bufs[nxt])
            cur = nxt
            out.append((bufs[cur].cpu().numpy().copy(), dt, info))
            if interleave:
                X, _ = other.reconstruct(bufs[cur])
                F = gm.flux(bufs[cur], X, 0.5 * dt)
                assert bool(torch.isfinite(F).all())
                torch.cuda.synchronize()
        st = gm.stats()
        assert st["capture_failures"] == 0
        assert st["graph_steps"] == (STEPS if prm.get("graphs", 1) else 0)
    finally:
        gm.close()
        if other is not None:
            other.close()
    return out


def assert_same(a, b):
    assert len(a) == len(b)
    for k, ((Wa, dta, ia), (Wb, dtb, ib)) in enumerate(zip(a, b)):
        assert dta == dtb, k
        assert np.array_equal(Wa, Wb), (k, float(np.abs(Wa - Wb).max()))
        assert ia["iters"] == ib["iters"], (k, ia["iters"], ib["iters"])
        assert ia["restarts"] == ib["restarts"], k
        assert ia["rel_resid"] == ib["rel_resid"], k
        assert ia["nonphys"] == ib["nonphys"], k


CASES = [
    # (case, precision, graph_budget, restart)
    ("adv", "fp64", 0, 30),
    ("adv", "mixed", 0, 30),
    ("adv", "fp64", 1, 30),
    ("adv", "mixed", 2, 30),
    ("adv", "fp64", 0, 3),
    ("sv", "mixed", 0, 2),
    ("sv", "fp64", 2, 30),
]


@pytest.mark.parametrize("case,precision,budget,restart", CASES)
def test_graph_steps_equal_eager(case, precision, budget, restart):
    mesh, W0 = adv_case() if case == "adv" else sv_case()
    prec = g.GKS_MIXED if precision == "mixed" else g.GKS_FP64
    kw = dict(precision=prec, restart=restart, max_iter=400)
    print("graph parity case", case, precision, "budget", budget, "restart", restart, flush=True)
    eager = run(mesh, W0, False, graphs=0, **kw)
    graphed = run(mesh, W0, True, graphs=1, graph_budget=budget, **kw)
    assert_same(graphed, eager)
    if restart <= 3:   # the second-cycle continuation was reached
        assert max(max(info["restarts"]) for _, _, info in graphed) >= 2


def test_graph_nonconvergence_matches_eager():
    mesh, W0 = adv_case()
    kw = dict(precision=g.GKS_FP64, max_iter=2, tol=1e-15)
    for graphs in (0, 1):
        gm = g.GksMesh(mesh, graphs=graphs, **kw)
        W = dev(W0)
        with pytest.raises(g.NonConvergence):
            gm.step(W)
        assert np.array_equal(W.cpu().numpy(), W0)
        gm.close()


def test_graph_path_off_while_profiling():
    """With the event profiler on, gks_step launches eagerly (every kernel is
    timed) and still gives the graph path's result."""
    mesh, W0 = adv_case()
    a = run(mesh, W0, False, graphs=1)
    gm = g.GksMesh(mesh, graphs=1)
    gm.profile(True)
    W = dev(W0)
    b = []
    bufs = [W, torch.empty_like(W)]
    cur = 0
    for _ in range(STEPS):
        nxt = 1 - cur
        bufs[nxt].copy_(bufs[cur])
        dt, info = gm.step(bufs[nxt])
        cur = nxt
        b.append((bufs[cur].cpu().numpy().copy(), dt, info))
    prof = gm.profile_get()
    gm.close()
    assert_same(a, b)
    assert prof["spmv"]["launches"] > 0
