"""The extrapolated start of each step's solve (gks_params.extrap_points).

On a 100x50 shock-vortex mesh (10,000 triangles, section 4.6 workload), both
forms, 12 steps with 1 to 5 extrapolation points:
  * every solve meets the tolerance 1e-10, and the states agree with those
    of the 3-point start to 1e-9 (the start changes only where the solve
    begins);
  * the starting residual (gks_solve_info.start_resid) over the steps with a
    full history shrinks with each point added up to 3, and 5 points beat 3
    (the CPU study of this workload: about 100 times);
  * the default (0) takes 5 points, and 3 with the limiter on.
A reconstruction outside the step sequence clears the step sizes, so the
steps after it extrapolate only from solutions of the sequence (finite,
converged starts).
"""
import numpy as np
import pytest

import gks_inputs as gi

torch = pytest.importorskip("torch")
import paper_1802_00704_amd as g  # noqa: E402

pytestmark = pytest.mark.gpu
STEPS = 12


def sv(nx=100, ny=50, seed=3):
    left, _ = gi.shock_vortex_states()
    walls = ((gi.BC_INFLOW, left), (gi.BC_OUTFLOW, None), (gi.BC_SLIP, None), (gi.BC_SLIP, None))
    m = gi.jss_mesh(nx, ny, seed, Lx=2.0, Ly=1.0, periodic=False, walls=walls)
    return m, gi.shock_vortex_ic(m)


def run(precision, points, **kw):
    m, W0 = sv()
    gm = g.GksMesh(m, precision=precision, tol=1e-10, extrap_points=points, **kw)
    W = torch.tensor(W0, device="cuda")
    r0 = []
    for _ in range(STEPS):
        _, info = gm.step(W)
        assert max(info["rel_resid"]) <= 1e-10
        r0.append(info["start_resid"])
    gm.close()
    return W.cpu().numpy(), r0


@pytest.mark.parametrize("precision", [g.GKS_FP64, g.GKS_MIXED])
def test_more_points_start_closer(precision):
    runs = {p: run(precision, p) for p in (1, 2, 3, 4, 5)}
    ref = runs[3][0]
    scale = np.abs(ref).max(axis=1, keepdims=True)
    bar = 1e-9   # both forms solve to 1e-10
    med = {}
    for p, (W, r0) in runs.items():
        assert (np.abs(W - ref) / scale).max() <= bar, p
        med[p] = float(np.median(r0[6:]))
    print("precision", precision, "median starting residual by points", med, flush=True)
    assert med[1] > med[2] > med[3]
    assert med[5] < 0.2 * med[3]
    Wd, r0d = run(precision, 0)
    assert np.array_equal(Wd, runs[5][0]) and r0d == runs[5][1]


def test_limiter_default_takes_three_points():
    Wd, r0d = run(g.GKS_MIXED, 0, limiter=g.LIMIT_CHARACTERISTIC, nonphys_fallback=1)
    W3, r03 = run(g.GKS_MIXED, 3, limiter=g.LIMIT_CHARACTERISTIC, nonphys_fallback=1)
    assert np.array_equal(Wd, W3) and r0d == r03


def test_steps_after_a_reconstruction():
    m, W0 = sv(40, 20)
    gm = g.GksMesh(m, precision=g.GKS_MIXED, tol=1e-10, extrap_points=5)
    W = torch.tensor(W0, device="cuda")
    for _ in range(6):
        gm.step(W)
    gm.reconstruct(W)
    for _ in range(6):
        _, info = gm.step(W)
        assert np.isfinite(info["start_resid"]) and max(info["rel_resid"]) <= 1e-10
    assert np.isfinite(W.cpu().numpy()).all()
    gm.close()
