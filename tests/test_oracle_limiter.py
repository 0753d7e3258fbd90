"""Pins of the oracle's DWBAP limiter and shock detector (section 3.3).

Nothing here retypes the limiter's formulas.  The checks are properties the
method must have whatever the reading of its open points:
  * the biased averaging reproduces equal candidates, stays within the
    candidates' range, and compresses an outlying candidate;
  * the weights form a convex combination that, in a region of uniform
    pressure, all but selects the cell's own candidate (accuracy keeping);
  * on fields the reconstruction reproduces exactly (global quadratics in the
    all-quadratic mode, global linears with linear boundary cells) every
    neighbour's polynomial is the cell's own, so the indicator is zero and
    even limiting forced onto every cell changes nothing in cells with three
    neighbours: this pins the remainder averages, the h scalings and the
    periodic images; in wall cells, whose candidates are directional, every
    limited slope component stays within the gradient's length;
  * the indicator fires at a density jump and not away from it, and on a
    smooth wave it falls as h^1.5 as the mesh is refined (Eq. ISD1 with
    k = 2 and a third-order reconstruction);
  * limiting removes at least 40% of the reconstruction's overshoot at a jump of
    density and pressure, and moves the coefficients far less across a pure
    contact (the smoothness measure reads the pressure);
  * characteristic variables (reading L9): the basis diagonalises the
    Jacobian of the Euler flux, found by finite differences of the flux
    itself, with eigenvalues u_n - c, u_n, u_n, u_n + c; exactness holds in
    this mode too; and across a moving contact, whose data vary along the
    entropy eigenvector alone, the limited polynomials keep velocity and
    pressure uniform at every Gauss point, which limiting the conserved
    variables one by one (arctan is not linear) cannot; and a quarter turn
    of the whole problem turns the limited polynomials with it (the
    direction of the decomposition follows the data, not the axes).
"""
import numpy as np
import pytest

import gks_inputs as gi
from oracle import cls, limiter
from oracle.mesh import build_geometry
from oracle import scheme


def quad_avg(m, q):
    return gi.cell_average(m, lambda x, y: q(x, y)[None])[0]


def test_biased_average_identities():
    rng = np.random.default_rng(0)
    for _ in range(50):
        J = rng.integers(1, 4)
        w = rng.random(J + 1)
        w /= w.sum()
        U = 10 ** rng.uniform(-3, 3)
        u = rng.normal() * U
        assert limiter.dwbap(np.full(J + 1, u), w) == pytest.approx(u, rel=1e-12)
        c = rng.normal(size=J + 1) * U
        L = limiter.dwbap(c, w)
        assert c.min() * (1 + 1e-12) - 1e-300 <= L <= c.max() * (1 + 1e-12) + 1e-300 or \
            c.min() - 1e-12 * abs(c.min()) <= L <= c.max() + 1e-12 * abs(c.max())
    # arctan compresses an outlier: one huge candidate moves the result far
    # less than an arithmetic mean would
    w = np.array([0.5, 0.25, 0.25])
    L = limiter.dwbap(np.array([1.0, 1.0, 1e6]), w)
    assert 1.0 < L < 10.0


def test_smoothness_exponent():
    S0 = limiter.smoothness_exponent(0.0)
    assert S0 == pytest.approx(1.0 / (1e-4 + 0.05), rel=1e-12)
    chis = np.array([0.0, 1e-6, 1e-3, 0.1, 1.0, 10.0])
    S = limiter.smoothness_exponent(chis)
    assert np.all(np.diff(S) < 0) and S[-1] > 0


def test_weights_convex_and_keep_own_value_where_pressure_is_uniform():
    m = gi.jss_mesh(8, 8, 3, Lx=1.0, Ly=1.0, periodic=True)
    geo = build_geometry(m)
    W = gi.prim_to_cons(np.ones(geo.nt), np.full(geo.nt, 0.3), np.full(geo.nt, -0.2), np.ones(geo.nt), 1.4)
    st = limiter.cell_stencils(geo, m)
    for i in range(0, geo.nt, 7):
        w = limiter.limiter_weights(geo, W, i, st[i], 1.4)
        assert np.all(w > 0) and w.sum() == pytest.approx(1.0, rel=1e-14)
        assert w[0] > 0.99


def _three_neighbours(geo, m):
    return np.array([len(st) == 3 for st in limiter.cell_stencils(geo, m)])


def _force_all(m, geo, W, X, k, variables="conservative"):
    return limiter.limit(geo, W, X, m, threshold=-1.0, k=k, variables=variables)


@pytest.mark.parametrize("variables", ["conservative", "characteristic"])
def test_quadratic_fields_unchanged_even_when_every_cell_is_limited(variables):
    m = gi.jss_mesh(7, 6, 4, Lx=1.3, Ly=1.1, periodic=False)
    geo = build_geometry(m)
    c = np.array([0.3, -1.2, 0.7, 2.1, -0.9, 1.6])
    q = lambda x, y: c[0] + c[1] * x + c[2] * y + c[3] * x * x + c[4] * x * y + c[5] * y * y
    k = cls.cell_orders(geo, all_quadratic=True)
    ubar = quad_avg(m, q) + 3.0   # positive density
    W = np.stack([ubar, 2 * ubar, -ubar, 4 * ubar + 10.0])
    X = cls.reconstruct(geo, W, k)
    IS = limiter.shock_indicator(geo, W, X, m, k=k)
    assert np.abs(IS).max() < 1e-10
    Xl, mask = _force_all(m, geo, W, X, k, variables)
    assert mask.all()
    inner = _three_neighbours(geo, m)
    assert np.abs(Xl[:, :, inner] - X[:, :, inner]).max() <= 1e-10 * np.abs(X).max()


@pytest.mark.parametrize("variables", ["conservative", "characteristic"])
def test_linear_fields_unchanged_with_linear_boundary_cells(variables):
    m = gi.jss_mesh(7, 6, 8, Lx=1.0, Ly=1.0, periodic=False)
    geo = build_geometry(m)
    k = cls.cell_orders(geo)
    assert (k == 1).sum() > 0
    q = lambda x, y: 2.4 - 1.7 * x + 0.6 * y
    ubar = quad_avg(m, q)
    W = np.stack([ubar, 0.5 * ubar, -0.25 * ubar, 3 * ubar])
    X = cls.reconstruct(geo, W, k)
    assert np.abs(limiter.shock_indicator(geo, W, X, m, k=k)).max() < 1e-10
    Xl, _ = _force_all(m, geo, W, X, k, variables)
    inner = _three_neighbours(geo, m)
    assert inner.sum() > 0 and (~inner).sum() > 0
    assert np.abs(Xl[:, :, inner] - X[:, :, inner]).max() <= 1e-11 * np.abs(X).max()
    if variables == "characteristic":
        return   # the wall bound below is per conserved variable
    # wall cells take directional candidates, the projections of the exact
    # gradient on the neighbour directions, none longer than the gradient;
    # each limited component lies within its candidates' range, so it is
    # bounded by the gradient's length
    wall = ~inner
    glen = np.linalg.norm(X[:, 0:2, wall], axis=1)
    assert np.all(np.abs(Xl[:, 0:2, wall]) <= glen[:, None, :] * (1 + 1e-12))


def test_candidates_are_exact_for_linear_data():
    """For u = a + g.x the remainder differences are g.(r_j - r_i): cells
    with three neighbours get g itself from every pair, wall cells get the
    projections (g.e_j) e_j of g on the neighbour directions."""
    m = gi.jss_mesh(7, 6, 8, Lx=1.0, Ly=1.0, periodic=False)
    geo = build_geometry(m)
    k = cls.cell_orders(geo)
    gx, gy = -1.7, 0.6
    ubar = quad_avg(m, lambda x, y: 2.4 + gx * x + gy * y)
    W = np.stack([ubar] * 4)
    X = cls.reconstruct(geo, W, k)
    st = limiter.cell_stencils(geo, m)
    g = np.array([gx, gy])
    for i in range(geo.nt):
        c1, _ = limiter.first_derivative_candidates(geo, W, X, X, i, st[i], np.full(len(st[i]) + 1, 1.0))
        for n, (j, _f) in enumerate(st[i], start=1):
            if len(st[i]) == 3:
                expect = g
            else:
                e = geo.cen[j] - geo.cen[i]
                e = e / np.linalg.norm(e)
                expect = (g @ e) * e
            assert np.abs(c1[n, 0] - expect).max() <= 1e-10 * np.abs(g).max()


def _jump_case(nx=24, ny=4):
    """Sod-like states (density and pressure jump) on a periodic strip.  A
    pure contact would not do: the smoothness measure of Eq. DWBAP_S reads
    the pressure, so across a contact the weights keep each cell's own
    value."""
    m = gi.jss_mesh(nx, ny, 5, Lx=2.0, Ly=1.0 / 3.0, periodic=True)
    geo = build_geometry(m)
    inner = lambda x: np.abs(x - 1.0) < 0.5
    rho = quad_avg(m, lambda x, y: np.where(inner(x), 1.0, 0.125))
    p = quad_avg(m, lambda x, y: np.where(inner(x), 1.0, 0.1))
    W = gi.prim_to_cons(rho, np.zeros(geo.nt), np.zeros(geo.nt), p, 1.4)
    s = scheme.Solver(m)
    X = s.reconstruct(W)
    return m, geo, W, X


def test_indicator_fires_at_a_jump_only():
    m, geo, W, X = _jump_case()
    IS = limiter.shock_indicator(geo, W, X, m)
    x = geo.cen[:, 0]
    near = (np.abs(x - 0.5) < 0.1) | (np.abs(x - 1.5) < 0.1)
    far = (np.abs(x - 0.5) > 0.3) & (np.abs(x - 1.5) > 0.3)
    assert IS[near].max() >= 1.0
    assert IS[far].max() < 1.0


def test_limiting_removes_most_of_the_overshoot():
    m, geo, W, X = _jump_case()
    Xl, mask = limiter.limit(geo, W, X, m)
    assert mask.any()
    pts = geo.gp.reshape(-1, 2)
    cells = np.repeat(geo.own, 2)

    def overshoot(XX):
        Q = scheme.gp_states(geo, W, XX, cells, pts)[0][0]
        return max(Q.max() - W[0].max(), W[0].min() - Q.min())

    o0, o1 = overshoot(X), overshoot(Xl)
    assert o0 > 0.02
    assert o1 < 0.6 * o0   # a one-pass averaging limiter is not strictly bounded


def test_a_pure_contact_is_limited_far_less_than_a_shock_like_jump():
    """The smoothness measure reads the pressure: across a contact (uniform
    pressure) chi = 0 and the weights all but keep each cell's own values,
    so the coefficients move an order of magnitude less than across a
    jump of density and pressure of the same size."""
    m = gi.jss_mesh(24, 4, 5, Lx=2.0, Ly=1.0 / 3.0, periodic=True)
    geo = build_geometry(m)
    rho = quad_avg(m, lambda x, y: np.where(np.abs(x - 1.0) < 0.5, 1.0, 0.125))
    W = gi.prim_to_cons(rho, np.zeros(geo.nt), np.zeros(geo.nt), np.ones(geo.nt), 1.4)
    X = scheme.Solver(m).reconstruct(W)
    Xl, mask = limiter.limit(geo, W, X, m)
    assert mask.any()                     # the density indicator fires at the contact
    _, _, W2, X2 = _jump_case()
    Xl2, _ = limiter.limit(geo, W2, X2, m)
    assert np.abs(Xl - X).max() < 0.2 * np.abs(Xl2 - X2).max()


def test_indicator_decays_like_h_to_the_1_5_on_smooth_data():
    peaks = []
    for n in (16, 32, 64):
        m = gi.jss_mesh(n, n, 2)
        W = gi.density_advection_ic(m)
        geo = build_geometry(m)
        X = scheme.Solver(m).reconstruct(W)
        peaks.append(limiter.shock_indicator(geo, W, X, m).max())
    r1, r2 = peaks[0] / peaks[1], peaks[1] / peaks[2]
    assert peaks[0] < 1.0
    assert 2.0 < r1 and 2.0 < r2 < 4.0   # 2^1.5 = 2.83


def _euler_flux_n(W, n, gamma):
    rho, mx, my, E = W
    u, v = mx / rho, my / rho
    p = (gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v))
    un = u * n[0] + v * n[1]
    return np.array([rho * un, mx * un + p * n[0], my * un + p * n[1], (E + p) * un])


def test_characteristic_basis_diagonalises_the_euler_flux_jacobian():
    rng = np.random.default_rng(3)
    G = 1.4
    for _ in range(20):
        rho, p = rng.uniform(0.1, 3.0), rng.uniform(0.1, 5.0)
        u, v = rng.normal(size=2)
        W = gi.prim_to_cons(np.array([rho]), u, v, p, G)[:, 0]
        th = rng.uniform(0, 2 * np.pi)
        n = np.array([np.cos(th), np.sin(th)])
        A = np.zeros((4, 4))
        for q in range(4):
            e = np.zeros(4)
            e[q] = 1e-6 * max(1.0, abs(W[q]))
            A[:, q] = (_euler_flux_n(W + e, n, G) - _euler_flux_n(W - e, n, G)) / (2 * e[q])
        R = limiter.characteristic_basis(W, G, n)
        c = np.sqrt(G * p / rho)
        un = u * n[0] + v * n[1]
        lam = np.array([un - c, un, un, un + c])
        scale = np.abs(A).max() * np.abs(R).max()
        assert np.abs(A @ R - R * lam[None, :]).max() <= 1e-7 * scale
        assert np.linalg.cond(R) < 1e4


def test_characteristic_limiting_keeps_a_moving_contact_pure():
    m = gi.jss_mesh(24, 4, 5, Lx=2.0, Ly=1.0 / 3.0, periodic=True)
    geo = build_geometry(m)
    u0, v0, p0 = 0.7, -0.3, 1.0
    rho = quad_avg(m, lambda x, y: np.where(np.abs(x - 1.0) < 0.5, 1.0, 0.125))
    W = gi.prim_to_cons(rho, u0, v0, p0, 1.4)
    X = scheme.Solver(m).reconstruct(W)
    pts = geo.gp.reshape(-1, 2)
    cells = np.repeat(geo.own, 2)
    dev = {}
    for variables in ("conservative", "characteristic"):
        Xl, mask = limiter.limit(geo, W, X, m, variables=variables)
        assert mask.any()
        Q = scheme.gp_states(geo, W, Xl, cells, pts)[0]
        vel = np.abs(Q[1] / Q[0] - u0).max() + np.abs(Q[2] / Q[0] - v0).max()
        prs = np.abs(0.4 * (Q[3] - 0.5 * (Q[1] ** 2 + Q[2] ** 2) / Q[0]) - p0).max()
        dev[variables] = max(vel, prs)
    assert dev["characteristic"] <= 1e-12
    assert dev["conservative"] > 1e-4


@pytest.mark.parametrize("variables", ["conservative", "characteristic"])
def test_limiting_commutes_with_a_quarter_turn(variables):
    from test_oracle_scheme import rotate_coefficients, rotate_mesh
    m = gi.jss_mesh(10, 8, 11, Lx=1.0, Ly=0.8, periodic=False, walls=((gi.BC_SLIP, None),) * 4)
    geo = build_geometry(m)
    # an oblique shock-like jump: density, pressure and the normal velocity
    # jump (with uniform velocity the characteristic coordinates of a jump
    # in density and pressure would not depend on the direction at all)
    nu = np.array([1.0, 0.6]) / np.hypot(1.0, 0.6)
    side = lambda x, y: (x + 0.6 * y < 0.55).astype(float)
    rho = quad_avg(m, lambda x, y: 0.2 + 0.8 * side(x, y))
    p = quad_avg(m, lambda x, y: 0.3 + 0.7 * side(x, y))
    mx = quad_avg(m, lambda x, y: (0.2 + 0.8 * side(x, y)) * (0.3 + 0.5 * nu[0] * side(x, y)))
    my = quad_avg(m, lambda x, y: (0.2 + 0.8 * side(x, y)) * (-0.2 + 0.5 * nu[1] * side(x, y)))
    W = gi.prim_to_cons(rho, mx / rho, my / rho, p, 1.4)
    X = scheme.Solver(m).reconstruct(W)
    Xl, mask = limiter.limit(geo, W, X, m, variables=variables)
    assert 0 < mask.sum() < geo.nt
    mr, R = rotate_mesh(m, np.pi / 2)
    Wr = W.copy()
    Wr[1:3] = R @ W[1:3]
    Xlr, maskr = limiter.limit(build_geometry(mr), Wr, rotate_coefficients(X, R), mr, variables=variables)
    assert np.array_equal(mask, maskr)
    assert np.abs(Xlr - rotate_coefficients(Xl, R)).max() <= 1e-12 * np.abs(X).max()
