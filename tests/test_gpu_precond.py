"""The preconditioner the solver applies, on the GPU, against block
substitutions in NumPy on the factors the host builds (gks_host_inspect).

This pins the device storage of the BILU(0) factors (sliced per level, rows
sorted by neighbour count) and the sweep kernels directly: a wrong or
missing block would only slow GMRES down and pass every parity test of the
converged solution.  FP64 form: one forward and one backward substitution,
to rounding (<= 1e-12 relative).  Mixed form: inner_iters Richardson sweeps
with FP32 storage, against the same sweeps in FP64 (<= 1e-4 relative, far
below the O(1) error of a structural mistake).
"""
import numpy as np
import pytest

import gks_inputs as gi
from mesh_variants import split_some_triangles

torch = pytest.importorskip("torch")
import paper_1802_00704_amd as g  # noqa: E402

pytestmark = pytest.mark.gpu


def sv_mesh():
    left, _ = gi.shock_vortex_states()
    return gi.jss_mesh(16, 8, 3, Lx=2.0, Ly=1.0, periodic=False,
                       walls=((gi.BC_INFLOW, left), (gi.BC_OUTFLOW, None), (gi.BC_SLIP, None), (gi.BC_SLIP, None)))


class Factors:
    """M = (I + L)(D + U) and K in solver order, from gks_host_inspect."""

    def __init__(self, hs):
        self.n = n = hs["nt"]
        self.perm = hs["perm"]
        blocks = lambda val, col, slots: [[(int(col[s, i]), val[s, :, i].reshape(5, 5))
                                           for s in range(slots) if col[s, i] != n] for i in range(n)]
        self.L = blocks(hs["lval"], hs["lcol"], 3)
        self.U = blocks(hs["uval"], hs["ucol"], 3)
        self.K = blocks(hs["kval"], hs["kcol"], 4)
        self.Dinv = [hs["dinv"][:, i].reshape(5, 5) for i in range(n)]

    def to_solver(self, V):          # [4][5][nt] caller order -> [n][5][4]
        return np.transpose(V, (2, 1, 0))[self.perm].copy()

    def to_caller(self, Z):
        out = np.empty_like(Z)
        out[self.perm] = Z
        return np.transpose(out, (2, 1, 0))

    def msolve(self, v):
        y = np.empty_like(v)
        for i in range(self.n):
            acc = v[i].copy()
            for k, B in self.L[i]:
                acc -= B @ y[k]
            y[i] = acc
        z = np.empty_like(v)
        for i in range(self.n - 1, -1, -1):
            acc = y[i].copy()
            for j, B in self.U[i]:
                acc -= B @ z[j]
            z[i] = self.Dinv[i] @ acc
        return z

    def kmul(self, x):
        out = np.zeros_like(x)
        for i in range(self.n):
            for j, B in self.K[i]:
                out[i] += B @ x[j]
        return out


def relerr(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("case,ordering", [("adv", g.GKS_ORDER_MULTICOLOR), ("sv", g.GKS_ORDER_MULTICOLOR),
                                           ("adv", g.GKS_ORDER_RCM), ("sv", g.GKS_ORDER_RCM),
                                           ("split", g.GKS_ORDER_MULTICOLOR), ("split", g.GKS_ORDER_RCM)])
def test_preconditioner_matches_host_factors(case, ordering):
    """JSS meshes have no 3-cycles in their cell graph, so the mixed inner
    sweeps run in the split form; the "split" case inserts centroid
    vertices, whose three cells are mutually adjacent, and so runs the
    general fused sweeps.  Both must equal plain Richardson on the factors."""
    mesh = {"adv": lambda: gi.jss_mesh(20, 20, 1), "sv": sv_mesh,
            "split": lambda: split_some_triangles(sv_mesh())}[case]()
    print("preconditioner case", case, "ordering", ordering, flush=True)
    hs = g.host_inspect(mesh, ordering=ordering)
    F = Factors(hs)
    rng = np.random.default_rng(7)
    V = rng.standard_normal((4, 5, F.n))
    Vd = torch.tensor(V, device="cuda")

    gm = g.GksMesh(mesh, ordering=ordering, precision=g.GKS_MIXED)
    assert gm.stats()["split_form"] == (0 if case == "split" else 1)
    z64 = gm.apply_precond(Vd, g.GKS_FP64).cpu().numpy()
    v = F.to_solver(V)
    ref = F.to_caller(F.msolve(v))
    assert relerr(z64, ref) <= 1e-12

    q = gm.params.inner_iters
    zmx = gm.apply_precond(Vd, g.GKS_MIXED).cpu().numpy()
    z = F.msolve(v)
    for _ in range(q - 1):
        z = z + F.msolve(v - F.kmul(z))
    ref_mx = F.to_caller(z)
    assert relerr(zmx, ref_mx) <= 1e-4
    # the sweeps do reduce the residual of K z = v relative to one BILU solve
    r1 = np.abs(v - F.kmul(F.to_solver(z64))).max()
    rq = np.abs(v - F.kmul(F.to_solver(zmx))).max()
    assert rq < r1
    gm.close()


def test_apply_precond_rejects_bad_arguments():
    mesh = gi.jss_mesh(6, 6, 1)
    gm = g.GksMesh(mesh)          # FP64 handle: no FP32 factors
    V = torch.zeros((4, 5, gm.nt), dtype=torch.float64, device="cuda")
    with pytest.raises(g.GksError):
        gm.apply_precond(V, g.GKS_MIXED)
    with pytest.raises(g.GksError):
        gm.apply_precond(V, g.GKS_FP64, Z=V)
    gm.close()


@pytest.mark.parametrize("precision", [g.GKS_FP64, g.GKS_MIXED])
def test_extrapolated_start_cuts_iterations(precision):
    """gks_step starts each solve from the extrapolation in time of the last
    solutions (order 0, 1, then 2 as history accumulates).  On smooth
    advection that start is orders of magnitude closer, so later steps need
    fewer iterations; a reconstruction call in between restarts the history
    without changing the converged result beyond the tolerance."""
    mesh = gi.jss_mesh(64, 64, 2)
    W0 = gi.density_advection_ic(mesh)
    gm = g.GksMesh(mesh, precision=precision, tol=1e-10)
    W = torch.tensor(W0, device="cuda")
    its = []
    for _ in range(6):
        _, info = gm.step(W)
        its.append(max(info["iters"]))
    print("iterations per step", its, flush=True)
    assert max(its[3:]) < its[1]
    # same W, fresh handle: the reconstruction agrees to the solver tolerance
    X1, _ = gm.reconstruct(W)
    X2, _ = g.GksMesh(mesh, precision=precision, tol=1e-10).reconstruct(W)
    assert float((X1 - X2).abs().max() / X2.abs().max()) < 1e-8
    _, info = gm.step(W)   # order 0 again after the reconstruction
    assert max(info["iters"]) <= its[1]
    gm.close()
