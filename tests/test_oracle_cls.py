"""Pins of the oracle's CLS reconstruction (section 3).

* Block entries equal brute-force cell-j means of the weighted basis
  derivatives (Eqs. A:B:b, A:B:b:3), by adaptive quadrature.
* The assembled normal equations give the same solution as a library
  least-squares solve of the explicitly stacked over-determined system
  (Eqs. spdConserved:4-5).
* Exactness: cell averages of a global quadratic are reproduced exactly when
  every cell is quadratic; with linear boundary cells (Eq. k_i) global linear
  fields are reproduced exactly.
* Under the global reading the matrix is symmetric positive definite.
* Dense LU and sparse LU agree.
"""
import numpy as np
import pytest

import gks_inputs as gi
from oracle import cls
from oracle.mesh import build_geometry
from tests.test_oracle_geometry import tri_quad


def quad_avg(mesh, fn):
    """Exact averages of the polynomial fn over every cell (Duffy rule of the
    input generator, exact for polynomials of degree <= 14)."""
    return gi.cell_average(mesh, lambda x, y: fn(x, y)[None])[0]


def test_blocks_match_quadrature():
    m = gi.jss_mesh(4, 4, 9, Lx=1.0, Ly=1.0, periodic=False)
    geo = build_geometry(m)
    k = cls.cell_orders(geo, all_quadratic=True)
    i, j = cls.interior_pairs(geo)
    A, B, a0 = cls.pair_blocks(geo, i, j, k)
    v = m.unwrapped_vertices()
    w = cls.CLS_W
    for p in range(0, i.size, 9):
        ci, cj = i[p], j[p]
        hi, hj = geo.h[ci], geo.h[cj]
        Aj = geo.area[cj]

        def mean_j(fn):
            return tri_quad(v[cj], fn) / Aj

        cx, cy = geo.cen[ci]
        phi_i = [
            lambda x, y: (x - cx) / hi,
            lambda x, y: (y - cy) / hi,
            lambda x, y: 0.5 * (((x - cx) / hi) ** 2 - geo.Ixx[ci] / hi ** 2),
            lambda x, y: (x - cx) * (y - cy) / hi ** 2 - geo.Ixy[ci] / hi ** 2,
            lambda x, y: 0.5 * (((y - cy) / hi) ** 2 - geo.Iyy[ci] / hi ** 2),
        ]
        # row p = 0: means over cell j of the basis of cell i
        for l in range(5):
            assert A[p, 0, l] == pytest.approx(mean_j(phi_i[l]), rel=1e-10, abs=1e-12)
        # rows p = 1: weight (w h_i) times the mean of the x / y derivatives
        dphidx = [lambda x, y: 1 / hi, lambda x, y: 0.0, lambda x, y: (x - cx) / hi ** 2,
                  lambda x, y: (y - cy) / hi ** 2, lambda x, y: 0.0]
        dphidy = [lambda x, y: 0.0, lambda x, y: 1 / hi, lambda x, y: 0.0,
                  lambda x, y: (x - cx) / hi ** 2, lambda x, y: (y - cy) / hi ** 2]
        for l in range(5):
            assert A[p, 1, l] == pytest.approx(w * hi * mean_j(dphidx[l]), rel=1e-10, abs=1e-12)
            assert A[p, 2, l] == pytest.approx(w * hi * mean_j(dphidy[l]), rel=1e-10, abs=1e-12)
        # rows p = 2 (constant second derivatives) and the neighbour's basis
        assert np.allclose(A[p, 3:, 2:], (w * hi) ** 2 * np.eye(3) / hi ** 2, rtol=1e-14)
        assert np.allclose(B[p, 1:3, :2], w * hi * np.eye(2) / hj, rtol=1e-14)
        assert np.allclose(B[p, 3:, 2:], (w * hi) ** 2 * np.eye(3) / hj ** 2, rtol=1e-14)
        assert np.all(B[p, 0] == 0.0)


def stacked_lstsq(geo, k, W):
    """Least-squares solution of the explicitly stacked system C u = b."""
    i, j = cls.interior_pairs(geo)
    A, B, a0 = cls.pair_blocks(geo, i, j, k)
    n = 5 * geo.nt
    rows = []
    rhs = []
    for p in range(i.size):
        for r in range(6):
            if not (A[p, r].any() or B[p, r].any()):
                continue
            row = np.zeros(n)
            row[5 * i[p]: 5 * i[p] + 5] += A[p, r]
            row[5 * j[p]: 5 * j[p] + 5] -= B[p, r]
            rows.append(row)
            rhs.append((W[:, j[p]] - W[:, i[p]]) if r == 0 else np.zeros(4))
    lin = np.nonzero(k == 1)[0]
    for c in lin:              # unused quadratic unknowns of linear cells
        for l in range(2, 5):
            row = np.zeros(n)
            row[5 * c + l] = 1.0
            rows.append(row)
            rhs.append(np.zeros(4))
    C = np.array(rows)
    b = np.array(rhs)
    sol = np.linalg.lstsq(C, b, rcond=None)[0]         # [n, 4]
    return sol.T.reshape(4, geo.nt, 5).transpose(0, 2, 1)


@pytest.mark.parametrize("periodic", [True, False])
def test_normal_equations_equal_stacked_lstsq(periodic):
    m = gi.jss_mesh(4, 4, 21, Lx=1.0, Ly=1.0, periodic=periodic)
    geo = build_geometry(m)
    k = cls.cell_orders(geo)
    rng = np.random.default_rng(3)
    W = rng.uniform(0.5, 1.5, (4, geo.nt))
    X = cls.reconstruct(geo, W, k)
    Xs = stacked_lstsq(geo, k, W)
    assert np.abs(X - Xs).max() < 1e-11 * max(1.0, np.abs(Xs).max())


def test_quadratic_fields_are_exact():
    m = gi.jss_mesh(7, 6, 4, Lx=1.3, Ly=1.1, periodic=False)
    geo = build_geometry(m)
    k = cls.cell_orders(geo, all_quadratic=True)
    c = np.array([0.3, -1.2, 0.7, 2.1, -0.9, 1.6])
    q = lambda x, y: c[0] + c[1] * x + c[2] * y + c[3] * x * x + c[4] * x * y + c[5] * y * y
    ubar = quad_avg(m, q)
    W = np.stack([ubar, 2 * ubar, -ubar, ubar + 1.0])
    X = cls.reconstruct(geo, W, k)
    cx, cy = geo.cen[:, 0], geo.cen[:, 1]
    h = geo.h
    qx = c[1] + 2 * c[3] * cx + c[4] * cy
    qy = c[2] + c[4] * cx + 2 * c[5] * cy
    expect = np.stack([h * qx, h * qy, h * h * 2 * c[3], h * h * c[4], h * h * 2 * c[5]])
    for v, s in enumerate((1.0, 2.0, -1.0, 1.0)):
        assert np.abs(X[v] - s * expect).max() < 1e-11


def test_linear_fields_exact_with_linear_boundary_cells():
    m = gi.jss_mesh(7, 6, 8, Lx=1.0, Ly=1.0, periodic=False)
    geo = build_geometry(m)
    k = cls.cell_orders(geo)
    assert (k == 1).sum() > 0
    q = lambda x, y: 0.4 - 1.7 * x + 0.6 * y
    ubar = quad_avg(m, q)
    W = np.stack([ubar] * 4)
    X = cls.reconstruct(geo, W, k)
    expect = np.stack([geo.h * -1.7, geo.h * 0.6] + [np.zeros(geo.nt)] * 3)
    assert np.abs(X[0] - expect).max() < 1e-12


def test_global_reading_is_spd_and_solvers_agree():
    m = gi.jss_mesh(5, 4, 2, Lx=1.0, Ly=1.0, periodic=True)
    geo = build_geometry(m)
    K, pairs = cls.assemble(geo)
    Kd = K.toarray()
    assert np.abs(Kd - Kd.T).max() < 1e-15 * np.abs(Kd).max()
    assert np.linalg.eigvalsh(Kd).min() > 1e-3
    W = gi.density_advection_ic(m)
    R = cls.rhs(geo, pairs, W)
    Xd = cls.solve(K, R)
    import scipy.sparse.linalg as spla
    Xs = spla.splu(K.tocsc()).solve(R.reshape(4, -1).T).T.reshape(4, geo.nt, 5).transpose(0, 2, 1)
    assert np.abs(Xd - Xs).max() < 1e-13
    assert cls.residual(K, R, Xd).max() < 1e-13


def test_per_cell_reading_shares_rhs_and_pattern():
    m = gi.jss_mesh(4, 4, 2)
    geo = build_geometry(m)
    KG, pG = cls.assemble(geo, reading="G")
    KP, pP = cls.assemble(geo, reading="P")
    W = gi.density_advection_ic(m)
    assert np.array_equal(cls.rhs(geo, pG, W), cls.rhs(geo, pP, W))
    assert np.array_equal((abs(KG) > 0).toarray().astype(int) @ np.ones(KG.shape[0]) > 0,
                          (abs(KP) > 0).toarray().astype(int) @ np.ones(KP.shape[0]) > 0)


@pytest.mark.parametrize("walled", [True, False])
def test_cg_solve_equals_direct_solve(walled):
    """Beyond SciPy's SuperLU range the oracle solves the normal equations
    by block-Jacobi conjugate gradients (K is SPD under reading G): on a mesh
    where both run, CG to a relative residual of 1e-14 gives the direct
    solution to 1e-12 and its true residual is at most 2e-14."""
    if walled:
        left, _ = gi.shock_vortex_states()
        walls = ((gi.BC_INFLOW, left), (gi.BC_OUTFLOW, None), (gi.BC_SLIP, None), (gi.BC_SLIP, None))
        m = gi.jss_mesh(40, 20, 3, Lx=2.0, Ly=1.0, periodic=False, walls=walls)
        W = gi.shock_vortex_ic(m)
    else:
        m = gi.jss_mesh(24, 24, 2)
        W = gi.density_advection_ic(m)
    geo = build_geometry(m)
    k = cls.cell_orders(geo)
    K, pairs = cls.assemble(geo, k)
    R = cls.rhs(geo, pairs, W)
    Xd = cls.solve(K, R)
    Xc = cls.solve_cg(K, R)
    assert np.abs(Xc - Xd).max() <= 1e-12 * np.abs(Xd).max()
    assert cls.residual(K, R, Xc).max() <= 2e-14
    # the step's solve mode selects it
    from oracle import scheme
    a = scheme.Solver(m, scheme.Params(solve="cg")).reconstruct(W)
    assert np.array_equal(a, Xc)
