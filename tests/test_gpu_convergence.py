"""Third-order accuracy of the whole GPU scheme on the density-advection
exact solution (section 4.1, in its diagonal periodic form on [0, 2]^2):
JSS meshes of 64, 128, 256 and 512 squares per side, common final time
T = 0.05 with dt = T / ceil(T / dt_CFL), GMRES tolerance 1e-12, for the
collision-time coefficient 0.01 of Eq. tauIns and for 0.  Errors are
area-weighted L1 and L2 of the cell-average density against the exact
cell averages.

Measured orders level off near 2.84 (L1, 256 to 512).  Halving the time
step changes the errors by about 1% (the temporal error is negligible at
these CFL steps), and the same study on unjittered meshes gives 2.87, so
the shortfall from 3 is spatial and not the jitter's: the pre-asymptotic
range of the third-order reconstruction.  The bars: every L1 order and the
L2 orders of the two finer pairs above 2.7, the finest pair's L1 order above
2.8, and halving the time step moving the
256^2 error by less than 3%."""
import math

import numpy as np
import pytest

import gks_inputs as gi

torch = pytest.importorskip("torch")
import paper_1802_00704_amd as g  # noqa: E402

pytestmark = pytest.mark.gpu
T_FINAL = 0.05


def errors(N, eps, dt_div=1):
    m = gi.jss_mesh(N, N, 2)
    W0 = gi.density_advection_ic(m)
    gm = g.GksMesh(m, tol=1e-12, tau_eps=eps)
    probe = torch.tensor(W0, device="cuda")
    dt_cfl, _ = gm.step(probe)
    nst = math.ceil(T_FINAL / dt_cfl) * dt_div
    dt = T_FINAL / nst
    gm.close()
    gm = g.GksMesh(m, tol=1e-12, tau_eps=eps)
    W = torch.tensor(W0, device="cuda")
    for _ in range(nst):
        gm.step(W, dt)
    area = g.host_inspect(m)["area"]
    e = np.abs(W[0].cpu().numpy() - gi.density_advection_exact(m, T_FINAL)[0])
    return (e * area).sum() / area.sum(), math.sqrt((e * e * area).sum() / area.sum()), nst


@pytest.mark.parametrize("eps", [0.01, 0.0])
def test_third_order_convergence_64_to_512(eps):
    res = [errors(N, eps) for N in (64, 128, 256, 512)]
    o1 = [math.log2(res[k][0] / res[k + 1][0]) for k in range(3)]
    o2 = [math.log2(res[k][1] / res[k + 1][1]) for k in range(3)]
    print("eps", eps, "L1", [r[0] for r in res], "L2", [r[1] for r in res], "steps", [r[2] for r in res])
    print("orders L1", o1, "L2", o2)
    assert min(o1) > 2.7 and min(o2[1:]) > 2.7
    assert o1[2] > 2.8


def test_time_step_error_is_negligible():
    e1 = errors(256, 0.0)
    e2 = errors(256, 0.0, dt_div=2)
    print("256^2 L1 at dt and dt/2:", e1[0], e2[0], "steps", e1[2], e2[2])
    assert abs(e2[0] - e1[0]) < 0.03 * e1[0]
