"""The preconditioner on the benchmark's 1,000,000-cell mesh, element by
element against block substitutions on the host-built factors.

Levels of at least 131,072 rows (every level of this mesh) launch the sweep
kernels in 256-thread blocks, smaller levels (the meshes of
test_gpu_precond.py) in one-wave blocks, so this is the check of the wide
launch shape.  Each multicolour level holds rows with no dependencies among
them, so the host substitution runs level by level with vectorised 5 x 5
block products instead of row by row: forward y_i = v_i - sum_k L_ik y_k over
the levels in order, backward z_i = D_i^-1 (y_i - sum_j U_ij z_j) in reverse
(section 3.2, BILU(0) with M = (I + L)(D + U)).
FP64 form: one substitution pair, <= 1e-12 relative.  Mixed form: the
inner Richardson sweeps with FP32 storage against the same sweeps in FP64,
<= 1e-4 relative.
"""
import numpy as np
import pytest

import gks_inputs as gi

torch = pytest.importorskip("torch")
import paper_1802_00704_amd as g  # noqa: E402

pytestmark = pytest.mark.gpu


def bench_mesh():
    left, _ = gi.shock_vortex_states()
    walls = ((gi.BC_INFLOW, left), (gi.BC_OUTFLOW, None), (gi.BC_SLIP, None), (gi.BC_SLIP, None))
    return gi.jss_mesh(1000, 500, 3, Lx=2.0, Ly=1.0, periodic=False, walls=walls)


class LevelFactors:
    """K, L, U and D^-1 in solver order from gks_host_inspect, applied one
    dependency level at a time.  Vectors are [n + 1, 5, 4] with a zero row n
    that empty slots point at."""

    def __init__(self, hs):
        self.n = hs["nt"]
        self.perm = hs["perm"]
        self.lev = hs["lev_ptr"]
        tr = lambda v: np.ascontiguousarray(np.transpose(v.reshape(v.shape[0], 5, 5, -1), (0, 3, 1, 2)))
        self.L, self.lcol = tr(hs["lval"]), hs["lcol"]
        self.U, self.ucol = tr(hs["uval"]), hs["ucol"]
        self.K, self.kcol = tr(hs["kval"]), hs["kcol"]
        self.Dinv = np.ascontiguousarray(np.transpose(hs["dinv"].reshape(5, 5, -1), (2, 0, 1)))

    def to_solver(self, V):
        out = np.zeros((self.n + 1, 5, 4))
        out[:self.n] = np.transpose(V, (2, 1, 0))[self.perm]
        return out

    def to_caller(self, Z):
        out = np.empty((self.n, 5, 4))
        out[self.perm] = Z[:self.n]
        return np.transpose(out, (2, 1, 0))

    def msolve(self, v):
        y = np.zeros_like(v)
        for l in range(len(self.lev) - 1):
            r = slice(self.lev[l], self.lev[l + 1])
            acc = v[r].copy()
            for s in range(self.lcol.shape[0]):
                acc -= np.einsum("rab,rbc->rac", self.L[s, r], y[self.lcol[s, r]])
            y[r] = acc
        z = np.zeros_like(v)
        for l in range(len(self.lev) - 2, -1, -1):
            r = slice(self.lev[l], self.lev[l + 1])
            acc = y[r].copy()
            for s in range(self.ucol.shape[0]):
                acc -= np.einsum("rab,rbc->rac", self.U[s, r], z[self.ucol[s, r]])
            z[r] = np.einsum("rab,rbc->rac", self.Dinv[r], acc)
        return z

    def kmul(self, x):
        out = np.zeros_like(x)
        for s in range(self.kcol.shape[0]):
            out[:self.n] += np.einsum("rab,rbc->rac", self.K[s], x[self.kcol[s]])
        return out


def relerr(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_wide_sweeps_match_host_factors():
    mesh = bench_mesh()
    hs = g.host_inspect(mesh, precision=g.GKS_MIXED)
    lev = hs["lev_ptr"]
    sizes = np.diff(lev)
    print("levels", sizes.tolist(), flush=True)
    assert sizes.min() >= 131072          # every level takes the 256-thread launch
    F = LevelFactors(hs)
    del hs
    rng = np.random.default_rng(17)
    V = rng.standard_normal((4, 5, F.n))
    gm = g.GksMesh(mesh, precision=g.GKS_MIXED)
    assert gm.stats()["split_form"] == 1
    Vd = torch.tensor(V, device="cuda")
    z64 = gm.apply_precond(Vd, g.GKS_FP64).cpu().numpy()
    zmx = gm.apply_precond(Vd, g.GKS_MIXED).cpu().numpy()
    q = gm.params.inner_iters
    gm.close()
    v = F.to_solver(V)
    z = F.msolve(v)
    e64 = relerr(z64, F.to_caller(z))
    for _ in range(q - 1):
        z = z + F.msolve(v - F.kmul(z))
    emx = relerr(zmx, F.to_caller(z))
    print("FP64 sweep pair %.3e, mixed inner sweeps %.3e" % (e64, emx), flush=True)
    assert e64 <= 1e-12
    assert emx <= 1e-4
