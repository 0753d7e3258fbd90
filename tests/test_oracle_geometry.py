"""Pins of the oracle's geometry and basis against brute-force integration.

Pins: triangle moments by adaptive 2-D quadrature; closed cells
(sum of S n over a cell's faces is zero); the circumradius by the
perpendicular-bisector construction; the zero mean of the basis of
Eq. quadRCP over its own cell (the cell-average condition, Eq.
cellAVGCond); the two-point Gauss rule of each face integrating cubics.
"""
import numpy as np
import pytest
from scipy import integrate

import gks_inputs as gi
from oracle.mesh import build_geometry, triangle_geometry


def tri_quad(v, fn):
    """Adaptive quadrature of fn over the triangle v [3, 2] (dblquad on the
    reference triangle, independent of the oracle)."""
    a, b, c = v
    J = abs((b[0] - a[0]) * (c[1] - a[1]) - (c[0] - a[0]) * (b[1] - a[1]))

    def g(t, s):
        p = a + s * (b - a) + t * (c - a)
        return fn(p[0], p[1]) * J

    val, _ = integrate.dblquad(g, 0.0, 1.0, lambda s: 0.0, lambda s: 1.0 - s, epsabs=1e-14, epsrel=1e-13)
    return val


@pytest.fixture(scope="module")
def tris():
    rng = np.random.default_rng(7)
    out = []
    for _ in range(4):
        v = rng.uniform(-1, 1, (3, 2))
        area2 = (v[1, 0] - v[0, 0]) * (v[2, 1] - v[0, 1]) - (v[2, 0] - v[0, 0]) * (v[1, 1] - v[0, 1])
        if area2 < 0:
            v = v[[0, 2, 1]]
        out.append(v)
    return np.array(out)


def test_triangle_moments_brute_force(tris):
    area, cen, Ixx, Ixy, Iyy, rad = triangle_geometry(tris)
    for t, v in enumerate(tris):
        A = tri_quad(v, lambda x, y: 1.0)
        cx = tri_quad(v, lambda x, y: x) / A
        cy = tri_quad(v, lambda x, y: y) / A
        assert area[t] == pytest.approx(A, rel=1e-12)
        assert cen[t, 0] == pytest.approx(cx, rel=1e-11, abs=1e-13)
        assert cen[t, 1] == pytest.approx(cy, rel=1e-11, abs=1e-13)
        assert Ixx[t] == pytest.approx(tri_quad(v, lambda x, y: (x - cx) ** 2) / A, rel=1e-10)
        assert Ixy[t] == pytest.approx(tri_quad(v, lambda x, y: (x - cx) * (y - cy)) / A, rel=1e-9, abs=1e-13)
        assert Iyy[t] == pytest.approx(tri_quad(v, lambda x, y: (y - cy) ** 2) / A, rel=1e-10)


def test_circumradius_bisectors(tris):
    *_, rad = triangle_geometry(tris)
    for t, (a, b, c) in enumerate(tris):
        # centre O solves |O - a| = |O - b| = |O - c|
        M = 2.0 * np.array([b - a, c - a])
        rhs = np.array([b @ b - a @ a, c @ c - a @ a])
        O = np.linalg.solve(M, rhs)
        assert rad[t] == pytest.approx(np.linalg.norm(O - a), rel=1e-12)


@pytest.mark.parametrize("periodic", [True, False])
def test_cells_are_closed_and_faces_unique(periodic):
    m = gi.jss_mesh(6, 5, 11, Lx=2.0, Ly=1.5, periodic=periodic)
    geo = build_geometry(m)
    acc = np.zeros((geo.nt, 2))
    sn = geo.normal * geo.S[:, None]
    np.add.at(acc, geo.own, sn)
    inner = geo.nbr >= 0
    np.add.at(acc, geo.nbr[inner], -sn[inner])
    assert np.abs(acc).max() < 1e-14
    # Euler characteristic: every cell has three faces
    cnt = np.bincount(geo.own, minlength=geo.nt) + np.bincount(geo.nbr[inner], minlength=geo.nt)
    assert np.all(cnt == 3)
    assert geo.nf == (3 * geo.nt + (~inner).sum()) // 2
    if periodic:
        assert inner.all()
    # faces are emitted in (owner, local edge) order
    assert np.all(np.diff(geo.own) >= 0)


def test_basis_zero_mean_and_h():
    m = gi.jss_mesh(4, 3, 5, Lx=1.0, Ly=1.0, periodic=False)
    geo = build_geometry(m)
    v = m.unwrapped_vertices()
    for t in range(0, geo.nt, 5):
        h = geo.h[t]
        cx, cy = geo.cen[t]
        A = geo.area[t]
        phis = [
            lambda x, y: (x - cx) / h,
            lambda x, y: (y - cy) / h,
            lambda x, y: 0.5 * (((x - cx) / h) ** 2 - geo.Ixx[t] / h ** 2),
            lambda x, y: (x - cx) * (y - cy) / h ** 2 - geo.Ixy[t] / h ** 2,
            lambda x, y: 0.5 * (((y - cy) / h) ** 2 - geo.Iyy[t] / h ** 2),
        ]
        for phi in phis:
            assert abs(tri_quad(v[t], phi) / A) < 1e-12
        a, b, c = v[t]
        R = np.linalg.norm(a - b) * np.linalg.norm(b - c) * np.linalg.norm(c - a) / (4 * A)
        assert h == pytest.approx(max(R, np.sqrt(A)), rel=1e-14)


def test_face_gauss_rule_integrates_cubics():
    m = gi.jss_mesh(4, 4, 3)
    geo = build_geometry(m)
    rng = np.random.default_rng(1)
    c = rng.normal(size=4)
    for f in range(0, geo.nf, 7):
        g0, g1 = geo.gp[f]
        mid = 0.5 * (g0 + g1)
        d = (g1 - g0) / np.linalg.norm(g1 - g0)
        S = geo.S[f]
        p = lambda s: c[0] + c[1] * s + c[2] * s ** 2 + c[3] * s ** 3
        exact = integrate.quad(p, -S / 2, S / 2, epsabs=1e-15)[0]
        s0 = (g0 - mid) @ d
        s1 = (g1 - mid) @ d
        assert 0.5 * S * (p(s0) + p(s1)) == pytest.approx(exact, rel=1e-13, abs=1e-15)
