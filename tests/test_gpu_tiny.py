"""Tiny walled meshes against the oracle: dependency levels of one to a few
rows (every wave of every kernel is partial, some launches cover a single
row), cells with one or two neighbours, and the degenerate two-triangle
mesh, whose CLS matrix is singular (each cell's gradient along the shared
edge is bound only to the other's), which must be refused cleanly."""
import numpy as np
import pytest

import gks_inputs as gi
from oracle import cls, limiter, scheme
from oracle.mesh import build_geometry
from parity import state_relinf

torch = pytest.importorskip("torch")
import paper_1802_00704_amd as g  # noqa: E402

pytestmark = pytest.mark.gpu
SIZES = [(2, 1), (2, 2), (3, 2), (4, 3)]


def mesh(nx, ny):
    return gi.jss_mesh(nx, ny, 1, Lx=float(nx), Ly=float(ny), periodic=False)   # slip walls


def state(m):
    c = m.unwrapped_vertices().mean(axis=1)
    rho = 1.0 + 0.1 * np.sin(c[:, 0]) * np.cos(c[:, 1])
    return gi.prim_to_cons(rho, 0.1, -0.05, 1.0 + 0.05 * np.cos(c[:, 0] + c[:, 1]), 1.4)


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("precision", [g.GKS_FP64, g.GKS_MIXED])
@pytest.mark.parametrize("nx,ny", SIZES)
def test_tiny_step_parity(nx, ny, precision):
    m = mesh(nx, ny)
    print("tiny mesh", nx, ny, m.nt, "precision", precision, flush=True)
    W0 = state(m)
    s = scheme.Solver(m)
    gm = g.GksMesh(m, precision=precision, tol=1e-13 if precision == g.GKS_FP64 else 1e-12)
    W = dev(W0)
    Wr = W0.copy()
    for _ in range(3):
        dt, _ = gm.step(W)
        Wr, _ = s.step(Wr, dt)
    rel = state_relinf(W.cpu().numpy(), Wr, per_component=True)
    print("relative L-inf per component", rel, flush=True)
    assert rel.max() <= (1e-12 if precision == g.GKS_FP64 else 1e-9), rel
    gm.close()


@pytest.mark.parametrize("variables", [g.LIMIT_CONSERVATIVE, g.LIMIT_CHARACTERISTIC])
@pytest.mark.parametrize("nx,ny", SIZES)
def test_tiny_limit_parity(nx, ny, variables):
    m = mesh(nx, ny)
    geo = build_geometry(m)
    W = state(m)
    X = cls.reconstruct(geo, W, cls.cell_orders(geo))
    name = {g.LIMIT_CONSERVATIVE: "conservative", g.LIMIT_CHARACTERISTIC: "characteristic"}[variables]
    Xo, mask = limiter.limit(geo, W, X, m, threshold=-1.0, variables=name)
    gm = g.GksMesh(m)
    Xl, n = gm.limit(dev(W), dev(X), -1.0, variables)
    assert n == int(mask.sum()) == geo.nt
    assert np.abs(Xl.cpu().numpy() - Xo).max() <= 1e-11 * max(np.abs(X).max(), 1e-300)
    gm.close()


def test_two_triangles_are_refused():
    with pytest.raises(g.GksError):
        g.GksMesh(mesh(1, 1))
