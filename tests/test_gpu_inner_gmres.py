"""The mixed form with inner GMRES as each outer step's preconditioner
(gks_params.inner_solver = GKS_INNER_GMRES): inner_iters GMRES steps on
K z = v, right-preconditioned by one FP32 BILU(0) application, with the FP64
matrix and an FP64 Arnoldi process.

  * Steps of the density-advection and shock-vortex workloads (sections 4.1
    and 4.6) within 1e-9 of the oracle with the true residual at 1e-10, with
    eager launches and with the captured graphs (bitwise the same).
  * The preconditioner alone (gks_apply_precond) on unit columns: the inner
    GMRES residual |v - K z| on the oracle's matrix is no larger than that of
    a single BILU(0) application (the first Krylov direction), and shrinks as
    the step count grows (GMRES minimises over nested spaces).
  * gks_batch_step refuses such handles.
"""
import numpy as np
import pytest

import gks_inputs as gi
from oracle import scheme

torch = pytest.importorskip("torch")
import paper_1802_00704_amd as g  # noqa: E402

pytestmark = pytest.mark.gpu


def relinf(a, ref):
    scale = np.abs(ref).max(axis=1, keepdims=True)
    return float((np.abs(a - ref) / scale).max())


def sv_mesh(nx=24, ny=12, seed=3):
    left, _ = gi.shock_vortex_states()
    walls = ((gi.BC_INFLOW, left), (gi.BC_OUTFLOW, None), (gi.BC_SLIP, None), (gi.BC_SLIP, None))
    return gi.jss_mesh(nx, ny, seed, Lx=2.0, Ly=1.0, periodic=False, walls=walls)


def case(name):
    if name == "advection":
        m = gi.jss_mesh(24, 24, 7)
        return m, gi.density_advection_ic(m)
    m = sv_mesh()
    return m, gi.shock_vortex_ic(m)


@pytest.mark.parametrize("inner_iters", [2, 4])
@pytest.mark.parametrize("name", ["advection", "shock_vortex"])
def test_inner_gmres_step_parity(name, inner_iters):
    m, W = case(name)
    s = scheme.Solver(m)
    runs = {}
    for graphs in (0, 1):
        gm = g.GksMesh(m, tol=1e-10, precision=g.GKS_MIXED, inner_solver=g.GKS_INNER_GMRES,
                       inner_iters=inner_iters, graphs=graphs)
        Wt = torch.tensor(W, device="cuda")
        Wr = W.copy()
        iters = []
        for _ in range(3):
            used, info = gm.step(Wt)
            assert max(info["rel_resid"]) <= 1e-10
            iters.append(max(info["iters"]))
            Wr, _ = s.step(Wr, used)
        gm.close()
        runs[graphs] = Wt.cpu().numpy()
        err = relinf(runs[graphs], Wr)
        print(name, "inner GMRES steps", inner_iters, "graphs", graphs, "outer iterations", iters, "vs oracle", err,
              flush=True)
        assert err <= 1e-9
    assert np.array_equal(runs[0], runs[1])


def test_inner_gmres_minimises_the_residual():
    m = sv_mesh(40, 20)
    K = scheme.Solver(m).K
    from oracle import cls as ocls
    rng = np.random.default_rng(17)
    V = rng.normal(size=(4, 5, m.nt))
    V /= np.sqrt((V * V).sum(axis=(1, 2), keepdims=True))   # unit columns
    Vt = torch.tensor(V, device="cuda")

    def resid(Z):
        return ocls.residual(K, np.ascontiguousarray(V.transpose(0, 2, 1)), Z.cpu().numpy())

    one = g.GksMesh(m, precision=g.GKS_MIXED, inner_iters=1)
    r1 = resid(one.apply_precond(Vt, form=g.GKS_MIXED))
    one.close()
    prev = None
    for mi in (1, 2, 4, 6):
        gm = g.GksMesh(m, precision=g.GKS_MIXED, inner_solver=g.GKS_INNER_GMRES, inner_iters=mi)
        r = resid(gm.apply_precond(Vt, form=g.GKS_MIXED))
        gm.close()
        print("inner GMRES steps", mi, "residual", r, "one BILU(0) application", r1, flush=True)
        assert np.all(r <= r1 * (1 + 1e-6))
        if prev is not None:
            assert np.all(r <= prev * (1 + 1e-6))
        prev = r
    assert np.all(prev < 0.5 * r1)


def test_batch_refuses_inner_gmres():
    m, W = case("advection")
    h = g.GksMesh(m, precision=g.GKS_MIXED, inner_solver=g.GKS_INNER_GMRES, inner_iters=3)
    Wt = torch.tensor(W, device="cuda")
    b = g.GksBatch()
    with pytest.raises(g.GksError):
        b.step([h], [Wt])
    assert np.array_equal(Wt.cpu().numpy(), W)
    b.close()
    h.close()


def test_inner_gmres_parameter_checks():
    m, _ = case("advection")
    with pytest.raises(g.GksError):
        g.GksMesh(m, precision=g.GKS_MIXED, inner_solver=g.GKS_INNER_GMRES, inner_iters=9)
    with pytest.raises(g.GksError):
        g.GksMesh(m, precision=g.GKS_MIXED, inner_solver=2)
