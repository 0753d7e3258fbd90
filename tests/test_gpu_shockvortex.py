"""The benchmark's workload run forward: 500 steps of the shock-vortex
interaction (section 4.6) on 1,000,000 walled triangles, mixed form, with and
without the DWBAP limiter.  The paper's figures for this case are missing,
so these are property checks: the run stays physical without a single
Gauss-point fallback; the vortex (the pressure minimum upstream of the
shock) travels with the pre-shock speed Ma sqrt(gamma); and limiting keeps
the density overshoot at the shock, which grows without it, smaller."""
import math

import numpy as np
import pytest

import gks_inputs as gi

torch = pytest.importorskip("torch")
import paper_1802_00704_amd as g  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sv1m():
    left, _ = gi.shock_vortex_states()
    walls = ((gi.BC_INFLOW, left), (gi.BC_OUTFLOW, None), (gi.BC_SLIP, None), (gi.BC_SLIP, None))
    m = gi.jss_mesh(1000, 500, 3, Lx=2.0, Ly=1.0, periodic=False, walls=walls)
    return m, gi.shock_vortex_ic(m), m.unwrapped_vertices().mean(axis=1)


def run(m, W0, limiter, steps=500):
    gm = g.GksMesh(m, tol=1e-10, precision=g.GKS_MIXED, nonphys_fallback=1, limiter=limiter)
    W = torch.tensor(W0, device="cuda")
    t, nonphys = 0.0, 0
    for _ in range(steps):
        dt, info = gm.step(W)
        t += dt
        nonphys += info["nonphys"]
    gm.close()
    return W.cpu().numpy(), t, nonphys


def test_shock_vortex_500_steps(sv1m):
    m, W0, cen = sv1m
    Wl, t, nonphys = run(m, W0, g.LIMIT_CHARACTERISTIC)
    print("limited: t %.5f rho [%.4f, %.4f], fallbacks %d" % (t, Wl[0].min(), Wl[0].max(), nonphys), flush=True)
    assert nonphys == 0
    rho_post = gi.shock_vortex_states()[1][0]
    assert Wl[0].min() > 0.85 and Wl[0].max() < rho_post + 0.08
    p = 0.4 * (Wl[3] - 0.5 * (Wl[1] ** 2 + Wl[2] ** 2) / Wl[0])
    upstream = cen[:, 0] < 0.45
    i = np.argmin(np.where(upstream, p, np.inf))
    x_expect = 0.25 + 1.1 * math.sqrt(1.4) * t
    print("vortex centre (%.4f, %.4f), expected x %.4f" % (cen[i, 0], cen[i, 1], x_expect), flush=True)
    assert abs(cen[i, 0] - x_expect) < 0.006 and abs(cen[i, 1] - 0.5) < 0.006
    Wu, _, _ = run(m, W0, 0)
    print("unlimited: rho max %.4f" % Wu[0].max(), flush=True)
    assert Wu[0].max() > Wl[0].max()
