"""gks_batch_step: several meshes stepped in shared grouped launches, each
with exactly the arithmetic of its own step.

Every case steps each request alone (its own handle, eager launches and the
default captured graphs, which are bitwise the same) and the same request,
from the same state, inside a batch, and compares W, the time step and the
iteration counts bitwise:
  * density-advection and shock-vortex meshes of uneven sizes, FP64 and
    mixed batches (sections 4.1 and 4.6 workloads);
  * requests joining and leaving the batch between steps (continuous
    batching), including a request joining with no history;
  * more requests than one grouped launch holds (split launches);
  * solves longer than the fused Gram-Schmidt passes hold, with restarts;
  * one request failing (a step far beyond the CFL limit with the fallback
    off: GKS_ENONPHYS, its W unchanged) beside requests that succeed;
  * argument errors: mixed precisions, a handle twice, a mixed-form handle
    without the split-form sweeps.
"""
import numpy as np
import pytest

import gks_inputs as gi
from mesh_variants import split_some_triangles

torch = pytest.importorskip("torch")
import paper_1802_00704_amd as g  # noqa: E402

pytestmark = pytest.mark.gpu


def sv(nx, ny, seed=3):
    left, _ = gi.shock_vortex_states()
    walls = ((gi.BC_INFLOW, left), (gi.BC_OUTFLOW, None), (gi.BC_SLIP, None), (gi.BC_SLIP, None))
    m = gi.jss_mesh(nx, ny, seed, Lx=2.0, Ly=1.0, periodic=False, walls=walls)
    return m, gi.shock_vortex_ic(m)


def adv(n, seed=2):
    m = gi.jss_mesh(n, n, seed)
    return m, gi.density_advection_ic(m)


CASES = [lambda: adv(12), lambda: sv(30, 15), lambda: adv(40, 5), lambda: sv(16, 8, 9), lambda: adv(7, 11)]


def handle(mesh, precision, **kw):
    return g.GksMesh(mesh, precision=precision, nonphys_fallback=1, tol=1e-10, **kw)


def dev(W):
    return torch.tensor(np.ascontiguousarray(W), dtype=torch.float64, device="cuda")


def alone(case, precision, steps, graphs):
    m, W0 = case()
    gm = handle(m, precision, graphs=graphs)
    W = dev(W0)
    out = []
    for _ in range(steps):
        dt, info = gm.step(W)
        out.append((W.cpu().numpy().copy(), dt, info["iters"]))
    gm.close()
    return out


@pytest.mark.parametrize("precision", [g.GKS_FP64, g.GKS_MIXED])
def test_batch_equals_alone(precision):
    steps = 4
    print("batch of", len(CASES), "requests, precision", precision, flush=True)
    ref = [alone(c, precision, steps, graphs=0) for c in CASES]
    ref_graphs = [alone(c, precision, steps, graphs=1) for c in CASES]
    hs, Ws = [], []
    for c in CASES:
        m, W0 = c()
        hs.append(handle(m, precision, graphs=0))
        Ws.append(dev(W0))
    b = g.GksBatch()
    for k in range(steps):
        res = b.step(hs, Ws)
        for r, (code, dt, info) in enumerate(res):
            assert code == 0
            Wr, dtr, itr = ref[r][k]
            assert dt == dtr
            assert info["iters"] == itr
            assert np.array_equal(Ws[r].cpu().numpy(), Wr), (r, k)
            assert np.array_equal(ref_graphs[r][k][0], Wr)
    b.close()
    for h in hs:
        h.close()


@pytest.mark.parametrize("precision", [g.GKS_FP64, g.GKS_MIXED])
def test_requests_join_and_leave(precision):
    """Membership by step: request 0 steps 0-5, request 1 joins at step 2,
    request 2 steps 1-3, request 3 only at step 4.  Each request's states
    equal its own run's, step for step."""
    plan = {0: range(0, 6), 1: range(2, 6), 2: range(1, 4), 3: range(4, 5)}
    cases = CASES[:4]
    ref = {r: alone(cases[r], precision, len(plan[r]), graphs=1) for r in plan}
    hs, Ws, done = {}, {}, {r: 0 for r in plan}
    b = g.GksBatch()
    for step in range(6):
        members = [r for r in plan if step in plan[r]]
        for r in members:
            if r not in hs:
                m, W0 = cases[r]()
                hs[r], Ws[r] = handle(m, precision, graphs=0), dev(W0)
        print("step", step, "members", members, flush=True)
        res = b.step([hs[r] for r in members], [Ws[r] for r in members])
        for r, (code, dt, info) in zip(members, res):
            assert code == 0
            Wr, dtr, itr = ref[r][done[r]]
            assert dt == dtr and info["iters"] == itr
            assert np.array_equal(Ws[r].cpu().numpy(), Wr), (r, step)
            done[r] += 1
        for r in list(hs):
            if step + 1 not in plan[r]:
                hs.pop(r).close()
    b.close()


def test_more_requests_than_one_launch_holds():
    cases = [lambda s=s: adv(4 + s % 5, 20 + s) for s in range(20)]
    ref = [alone(c, g.GKS_MIXED, 2, graphs=0) for c in cases]
    hs, Ws = [], []
    for c in cases:
        m, W0 = c()
        hs.append(handle(m, g.GKS_MIXED, graphs=0))
        Ws.append(dev(W0))
    b = g.GksBatch()
    for k in range(2):
        res = b.step(hs, Ws)
        assert all(code == 0 for code, _, _ in res)
        for r in range(len(cases)):
            assert np.array_equal(Ws[r].cpu().numpy(), ref[r][k][0])
    b.close()
    for h in hs:
        h.close()


def cav(n=24, seed=4):
    walls = ((gi.BC_NOSLIP, (0.0, 0.0, 0.0, 0.0)),) * 3 + ((gi.BC_NOSLIP, (0.0, 1.0, 0.0, 0.0)),)
    m = gi.jss_mesh(n, n, seed, Lx=1.0, Ly=1.0, periodic=False, stretch=1.5, walls=walls)
    return m, gi.cavity_ic(m)


@pytest.mark.parametrize("precision", [g.GKS_FP64, g.GKS_MIXED])
def test_long_solves_and_restarts_in_a_batch(precision):
    """Viscous cavity meshes (section 4.7) whose FP64 solves take more Arnoldi
    steps than the fused Gram-Schmidt passes hold (8) and, with restart 12,
    several cycles: batch and alone bitwise equal, with the second pass
    taken selectively on both paths."""
    cases = [lambda: cav(24), lambda: cav(16, 9), lambda: adv(10)]
    kw = dict(mu=1e-3, restart=12, tol=1e-12)

    def mk(c):
        m, W0 = c()
        return g.GksMesh(m, precision=precision, nonphys_fallback=1, graphs=0, **kw), dev(W0)

    ref = []
    for c in cases:
        h, W = mk(c)
        out = []
        for _ in range(3):
            dt, info = h.step(W)
            out.append((W.cpu().numpy().copy(), dt, info["iters"], info["restarts"], info["reorth"]))
        h.close()
        ref.append(out)
    if precision == g.GKS_FP64:
        assert max(max(r[2]) for r in ref[0]) > 12 and max(max(r[3]) for r in ref[0]) >= 2
    pairs = [mk(c) for c in cases]
    b = g.GksBatch()
    for k in range(3):
        res = b.step([p[0] for p in pairs], [p[1] for p in pairs])
        for r, (code, dt, info) in enumerate(res):
            assert code == 0
            Wr, dtr, itr, rsr, ror = ref[r][k]
            print("request", r, "step", k, "iters", itr, "restarts", rsr, "second passes", ror, flush=True)
            assert dt == dtr and info["iters"] == itr and info["restarts"] == rsr and info["reorth"] == ror
            assert np.array_equal(pairs[r][1].cpu().numpy(), Wr), (r, k)
    b.close()
    for h, _ in pairs:
        h.close()


def test_one_failing_request_leaves_the_others():
    (m0, W0), (m1, W1) = adv(12), sv(30, 15)
    ref = alone(lambda: (m1, W1), g.GKS_FP64, 1, graphs=0)
    h0 = g.GksMesh(m0, nonphys_fallback=0, graphs=0)
    h1 = handle(m1, g.GKS_FP64, graphs=0)
    Wa, Wb = dev(W0), dev(W1)
    b = g.GksBatch()
    res = b.step([h0, h1], [Wa, Wb], dt=[50.0, 0.0])
    assert res[0][0] == g._lib.GKS_ENONPHYS
    assert np.array_equal(Wa.cpu().numpy(), W0)
    assert res[1][0] == 0
    assert np.array_equal(Wb.cpu().numpy(), ref[0][0])
    b.close()
    h0.close()
    h1.close()


def test_batch_argument_errors():
    (m0, W0), (m1, W1) = adv(8), sv(12, 6)
    h0 = handle(m0, g.GKS_FP64)
    h1 = handle(m1, g.GKS_MIXED)
    Wa, Wb = dev(W0), dev(W1)
    b = g.GksBatch()
    with pytest.raises(g.GksError):
        b.step([h0, h1], [Wa, Wb])            # mixed precisions
    with pytest.raises(g.GksError):
        b.step([h0, h0], [Wa, Wa])            # a handle twice
    m2 = split_some_triangles(sv(12, 6)[0])
    h2 = handle(m2, g.GKS_MIXED)
    assert h2.stats()["split_form"] == 0
    W2 = dev(gi.shock_vortex_ic(m2))
    with pytest.raises(g.GksError):
        b.step([h1, h2], [Wb, W2])            # no split-form sweeps
    assert np.array_equal(Wa.cpu().numpy(), W0) and np.array_equal(Wb.cpu().numpy(), W1)
    b.close()
    for h in (h0, h1, h2):
        h.close()
