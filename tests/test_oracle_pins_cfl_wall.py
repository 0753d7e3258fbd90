"""Pins of the oracle's time-step rule and of its moving no-slip wall ghost.

Time step (reading R14, the paper gives none):
  dt = CFL min_i |Omega_i| / sum_{f in i} S_f (|U_i . n_f| + c_i).
  * One equilateral triangle of side a with walls on every edge, fluid
    moving along x: the three outward normals are (0, -1), (sqrt3/2, 1/2),
    (-sqrt3/2, 1/2), so sum_f S_f |U . n_f| = sqrt3 a |u| and
    dt = CFL (sqrt3/4 a^2) / (a (sqrt3 |u| + 3 c)), written out by hand.
  * A periodic lattice of right triangles (legs h, no jitter), uniform flow
    (u, v): a cell split along the diagonal (1, 1) has faces of length h with
    normals along x and y and one of length sqrt2 h with normal (1, -1)/sqrt2,
    so sum_f S_f |U . n_f| = h (|u| + |v| + |u - v|) and sum_f S_f =
    (2 + sqrt2) h; along the other diagonal |u + v| replaces |u - v|.  Every
    interior face counts for both of its cells: counting it only for its
    owner, or |U| in place of |U . n|, changes the minimum.

Moving no-slip wall (section 4.7's lid; ghost reading R9):
  * Galilean covariance of the ghost map.  A boost by V maps conserved
    variables linearly, B(V) (rho, m, E) = (rho, m - rho V, E - m.V +
    rho |V|^2 / 2), and derivatives with the same matrix.  Seen from the
    wall's frame the moving wall is at rest, so the ghost of a wall moving
    with V must equal B(-V) applied to the resting wall's ghost of
    B(V) W, for every state and derivative set and any V.
  * Galilean covariance of the wall flux for a tangential wall velocity and
    a state uniform along the wall: the kinetic flux of the boosted problem
    maps back by F_rho' = F_rho, F_m' = F_m + V F_rho,
    F_E' = F_E + V.F_m + |V|^2 F_rho / 2.  (With variation along the wall the
    two fluxes are not comparable: the lab frame's Gauss point is fixed,
    while the boosted frame's moves along the face by V t during the step.)
  * A Couette state (variation normal to the wall only) next to a resting
    no-slip wall is symmetric under x -> -x, (u, v) -> (-u, -v), so no mass
    and no energy cross the wall; next to a wall moving with V_t (the lid)
    the mass flux stays zero and the energy flux is V_t times the tangential
    momentum flux (the work of the wall's shear).
"""
import math

import numpy as np
import pytest

import gks_inputs as gi
from oracle import kinetic, scheme
from oracle.mesh import build_geometry


# ------------------------------------------------------------------ time step
def one_triangle(a):
    xy = np.array([[0.0, 0.0], [a, 0.0], [0.5 * a, 0.5 * math.sqrt(3.0) * a]])
    return gi.Mesh(xy=xy, tri=np.array([[0, 1, 2]], dtype=np.int32), edge_tag=np.ones((1, 3), dtype=np.int32),
                   periodic=(False, False), L=(1.0, 1.0), bc_table=[(gi.BC_SLIP, None)])


@pytest.mark.parametrize("a,u", [(1.0, 0.0), (0.3, 0.7), (2.0, -1.9)])
def test_cfl_on_one_equilateral_triangle(a, u):
    rho, p, gamma, cfl = 1.2, 0.9, 1.4, 0.5
    m = one_triangle(a)
    W = gi.prim_to_cons(np.array([rho]), u, 0.0, p, gamma)
    c = math.sqrt(gamma * p / rho)
    expect = cfl * (math.sqrt(3.0) / 4.0 * a * a) / (a * (math.sqrt(3.0) * abs(u) + 3.0 * c))
    got = scheme.cfl_dt(build_geometry(m), W, scheme.Params(cfl=cfl, gamma=gamma))
    assert got == pytest.approx(expect, rel=1e-14)


@pytest.mark.parametrize("u,v", [(1.0, 1.0), (2.0, -0.5), (-0.3, 0.8)])
def test_cfl_on_a_right_triangle_lattice(u, v):
    n, L = 6, 1.5
    h = L / n
    m = gi.jss_mesh(n, n, 11, Lx=L, Ly=L, jitter=0.0)
    rho, p, gamma, cfl = 0.8, 1.1, 1.4, 0.5
    W = gi.prim_to_cons(np.full(m.nt, rho), u, v, p, gamma)
    c = math.sqrt(gamma * p / rho)
    # the lattice's cells are split along (1, 1) or along (-1, 1); the seeded
    # mesh has both kinds, and the minimum comes from the larger sum
    diag_sum = max(abs(u - v), abs(u + v))
    den = h * (abs(u) + abs(v) + diag_sum) + (2.0 + math.sqrt(2.0)) * h * c
    expect = cfl * (0.5 * h * h) / den
    v_ = m.unwrapped_vertices()
    kinds = set()
    for t in range(m.nt):
        e = v_[t, [1, 2, 0]] - v_[t]
        kinds.update(int(round(np.sign(d[0] * d[1]))) for d in e if abs(d[0]) > 1e-12 and abs(d[1]) > 1e-12)
    assert kinds == {-1, 1}, "the seeded lattice must hold both diagonals"
    got = scheme.cfl_dt(build_geometry(m), W, scheme.Params(cfl=cfl, gamma=gamma))
    assert got == pytest.approx(expect, rel=1e-13)


# ------------------------------------------------------------------ moving no-slip wall
def boost(V):
    """B(V) for face-frame momentum (n, t), V = (Vn, Vt)."""
    Vn, Vt = V
    return np.array([[1.0, 0.0, 0.0, 0.0],
                     [-Vn, 1.0, 0.0, 0.0],
                     [-Vt, 0.0, 1.0, 0.0],
                     [0.5 * (Vn * Vn + Vt * Vt), -Vn, -Vt, 1.0]])


def random_side(rng, m, couette=False):
    rho = rng.uniform(0.8, 1.3, m)
    u = rng.uniform(-0.4, 0.4, m)
    v = rng.uniform(-0.4, 0.4, m)
    p = rng.uniform(0.8, 1.2, m)
    W = gi.prim_to_cons(rho, u, v, p, 1.4)
    d = {k: 0.05 * rng.normal(size=(4, m)) * np.array([1.0, 1.0, 1.0, 3.0])[:, None]
         for k in ("n", "t", "nn", "nt", "tt")}
    if couette:
        for k in ("t", "nt", "tt"):
            d[k][:] = 0.0
    return W, d


def wall_state(nx, ny, Vn, Vt):
    """(rho, u, v, p) row of a wall moving with face-frame velocity (Vn, Vt)
    in x-y components."""
    tx, ty = -ny, nx
    return (1.0, Vn * nx + Vt * tx, Vn * ny + Vt * ty, 1.0)


def test_noslip_ghost_is_galilean_covariant():
    rng = np.random.default_rng(7)
    m = 16
    for _ in range(20):
        th = rng.uniform(0, 2 * np.pi)
        nx, ny = np.full(m, np.cos(th)), np.full(m, np.sin(th))
        V = rng.uniform(-0.7, 0.7, 2)
        W, d = random_side(rng, m)
        Wg, dg = scheme.ghost(W, d, scheme.BC_NOSLIP, wall_state(nx[0], ny[0], *V), 1.4, nx, ny, None)
        B = boost(V)
        Binv = boost(-V)
        W0g, d0g = scheme.ghost(B @ W, {k: B @ x for k, x in d.items()}, scheme.BC_NOSLIP,
                                wall_state(nx[0], ny[0], 0.0, 0.0), 1.4, nx, ny, None)
        assert np.abs(Wg - Binv @ W0g).max() < 1e-14 * np.abs(Wg).max()
        for k in d:
            assert np.abs(dg[k] - Binv @ d0g[k]).max() < 1e-14 * max(1.0, np.abs(dg[k]).max())


def wall_flux(W, d, nx, ny, V, dt=2e-3, mu=0.0):
    Wg, dg = scheme.ghost(W, d, scheme.BC_NOSLIP, wall_state(nx[0], ny[0], *V), 1.4, nx, ny, None)
    return kinetic.gp_flux(W, d, Wg, dg, dt, 1.4, mu, 0.01)


@pytest.mark.parametrize("mu", [0.0, 2e-3])
def test_lid_flux_is_galilean_covariant(mu):
    rng = np.random.default_rng(11)
    m = 12
    for _ in range(6):
        nx, ny = np.full(m, 0.6), np.full(m, 0.8)
        Vt = rng.uniform(-1.0, 1.0)
        W, d = random_side(rng, m, couette=True)
        F = wall_flux(W, d, nx, ny, (0.0, Vt), mu=mu)
        B = boost((0.0, Vt))
        F0 = wall_flux(B @ W, {k: B @ x for k, x in d.items()}, nx, ny, (0.0, 0.0), mu=mu)
        expect = np.stack([F0[0], F0[1], F0[2] + Vt * F0[0], F0[3] + Vt * F0[2] + 0.5 * Vt * Vt * F0[0]])
        scale = np.abs(F).max(axis=1, keepdims=True)
        assert np.abs(F - expect).max() < 1e-14 * scale.max(), np.abs(F - expect).max() / scale.max()


@pytest.mark.parametrize("mu", [0.0, 2e-3])
def test_couette_state_at_a_moving_wall(mu):
    rng = np.random.default_rng(5)
    m = 12
    nx, ny = np.full(m, 0.0), np.full(m, 1.0)
    W, d = random_side(rng, m, couette=True)
    F_rest = wall_flux(W, d, nx, ny, (0.0, 0.0), mu=mu)
    big = np.abs(F_rest).max()
    assert np.abs(F_rest[0]).max() < 1e-14 * big
    assert np.abs(F_rest[3]).max() < 1e-14 * big
    Vt = 0.9
    F = wall_flux(W, d, nx, ny, (0.0, Vt), mu=mu)
    big = np.abs(F).max()
    assert np.abs(F[0]).max() < 1e-14 * big
    assert np.abs(F[3] - Vt * F[2]).max() < 1e-13 * big
    assert np.abs(F[2]).max() > 1e-3 * big     # the wall's shear is not zero
