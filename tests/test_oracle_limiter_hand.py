"""A hand-computed case of the DWBAP limiter (section 3.3, Eqs. DWBAP,
DWBAP_w, DWBAP_S; readings L1-L5 of the oracle's header).

Four congruent right isosceles triangles (legs 2, so h = sqrt2 for every
cell, Eq. h): the central cell C = (0,0), (2,0), (0,2) and its mirror images
across its three edges, B (bottom), D (across the hypotenuse) and L (left).
Every other edge is a slip wall, so C has three neighbours in local-edge
order B, D, L and is quadratic; the others are linear.

Geometry, worked out by hand:
  centroids C (2/3, 2/3), B (2/3, -2/3), D (4/3, 4/3), L (-2/3, 2/3);
  midpoints of C's faces (1, 0), (1, 1), (0, 1);
  mean distance from each centroid to those midpoints (reading L4; the
  common factor 1/h cancels in the normalised weights):
    D_C = (2 sqrt5 + sqrt2) / 9,  D_B = D_L = (sqrt5 + sqrt26 + sqrt29) / 9,
    D_D = (2 sqrt17 + sqrt2) / 9.
Neighbour pressures 1, 2, 3 give chi = sqrt(2/3) / 2 (population standard
deviation over the mean, reading L5), S = 1 / (sqrt(chi + 1e-8) + 0.05) and
omega_j = D_j^-S / sum_k D_k^-S.

Second derivatives (variable rho u, whose cell averages are zero so the
pressures above stand): C's own (u_xx, u_xy, u_yy) = (1, 0, -1); the
neighbours' u_xx = (B 0, D 0.5, L 2), u_xy = (1, 2, 3), u_yy = 0, so
  u_xx = tan(w_C pi/4 + w_D atan(1/2) + w_L atan 2),
  u_xy = tan(w_B atan 1 + w_D atan 2 + w_L atan 3),
  u_yy = tan(-w_C pi/4).
First derivatives (variable rho, no second derivatives anywhere, so the
remainder differences are the plain differences of the averages): rho = 2 in
C, 2/3 in B and L, 4 in D.  The planes through C and a neighbour pair, with
centroid offsets B (0, -4/3), D (2/3, 2/3), L (-4/3, 0), have gradients
  (B, D): (2, 1),  (D, L): (1, 2),  (L, B): (1, 1),
and carry the pair weights (w_B + w_D)/2, (w_D + w_L)/2, (w_L + w_B)/2; C's
own gradient is (3, 0):
  u_x = tan(w_C atan 3 + (w_B+w_D)/2 atan 2 + (w_D+w_L)/2 atan 1 + (w_L+w_B)/2 atan 1),
  u_y = tan((w_B+w_D)/2 atan 1 + (w_D+w_L)/2 atan 2 + (w_L+w_B)/2 atan 1).
Wall cell B (one neighbour, C): both centroids lie at the same distance
sqrt5/3 from the shared face's midpoint (1, 0), so the weights are 1/2 and
1/2; its directional candidate is
(rho_C - rho_B) d / |d|^2 with d = (0, 4/3), i.e. (0, 1); with B's own
gradient (0.5, -1):  u_x = tan(atan(0.5) / 2),  u_y = tan((atan(-1) + atan 1) / 2) = 0.
"""
import math

import numpy as np
import pytest

import gks_inputs as gi
from oracle import limiter
from oracle.mesh import build_geometry

R2 = math.sqrt(2.0)


def four_cells():
    xy = np.array([[0, 0], [2, 0], [0, 2], [0, -2], [-2, 0], [2, 2]], dtype=np.float64)
    tri = np.array([[0, 1, 2],     # C
                    [0, 3, 1],     # B
                    [0, 2, 4],     # L
                    [1, 5, 2]],    # D
                   dtype=np.int32)
    tag = np.array([[0, 0, 0], [1, 1, 0], [0, 1, 1], [1, 1, 0]], dtype=np.int32)
    return gi.Mesh(xy=xy, tri=tri, edge_tag=tag, periodic=(False, False), L=(1.0, 1.0),
                   bc_table=[(gi.BC_SLIP, None)])


C, B, L, D = 0, 1, 2, 3


def weights():
    chi = math.sqrt(2.0 / 3.0) / 2.0
    S = 1.0 / (math.sqrt(chi + 1e-8) + 0.05)
    dist = {C: (2 * math.sqrt(5) + R2) / 9, B: (math.sqrt(5) + math.sqrt(26) + math.sqrt(29)) / 9,
            L: (math.sqrt(5) + math.sqrt(26) + math.sqrt(29)) / 9, D: (2 * math.sqrt(17) + R2) / 9}
    beta = {k: v ** -S for k, v in dist.items()}
    tot = sum(beta.values())
    return {k: v / tot for k, v in beta.items()}


def state_and_coefficients():
    h = R2
    gamma = 1.4
    W = np.zeros((4, 4))
    W[0] = [2.0, 2.0 / 3.0, 2.0 / 3.0, 4.0]            # C, B, L, D
    p = {C: 1.0, B: 1.0, D: 2.0, L: 3.0}
    W[3] = [p[c] / (gamma - 1.0) for c in range(4)]
    X = np.zeros((4, 5, 4))
    X[0, 0, C], X[0, 1, C] = 3.0 * h, 0.0              # rho: own gradient (3, 0)
    X[0, 0, B], X[0, 1, B] = 0.5 * h, -1.0 * h         # wall cell B: own gradient (0.5, -1)
    X[0, 0, D], X[0, 1, D] = 0.2 * h, 0.1 * h          # (not limited here)
    X[0, 0, L], X[0, 1, L] = -0.3 * h, 0.4 * h
    hh = h * h
    X[1, 2:5, C] = np.array([1.0, 0.0, -1.0]) * hh      # rho u: second derivatives
    X[1, 2:5, B] = np.array([0.0, 1.0, 0.0]) * hh
    X[1, 2:5, D] = np.array([0.5, 2.0, 0.0]) * hh
    X[1, 2:5, L] = np.array([2.0, 3.0, 0.0]) * hh
    return W, X


def test_geometry_of_the_case():
    geo = build_geometry(four_cells())
    assert np.allclose(geo.h, R2, rtol=0, atol=1e-15)
    assert np.allclose(geo.cen, [[2 / 3, 2 / 3], [2 / 3, -2 / 3], [-2 / 3, 2 / 3], [4 / 3, 4 / 3]], atol=1e-15)
    st = limiter.cell_stencils(geo, four_cells())
    assert [j for j, _ in st[C]] == [B, D, L]


def test_weights_by_hand():
    m = four_cells()
    geo = build_geometry(m)
    W, _ = state_and_coefficients()
    st = limiter.cell_stencils(geo, m)
    w = limiter.limiter_weights(geo, W, C, st[C], 1.4)
    wh = weights()
    assert w == pytest.approx([wh[C], wh[B], wh[D], wh[L]], rel=1e-13)
    assert wh[B] != pytest.approx(wh[D], rel=1e-3)   # unequal: a misplaced pair weight shows


def test_limited_coefficients_by_hand():
    m = four_cells()
    geo = build_geometry(m)
    W, X = state_and_coefficients()
    Xl, mask = limiter.limit(geo, W, X, m, threshold=-1.0)
    assert mask.all()
    w = weights()
    h2 = 2.0
    at = math.atan
    uxx = math.tan(w[C] * math.pi / 4 + w[D] * at(0.5) + w[L] * at(2.0))
    uxy = math.tan(w[B] * at(1.0) + w[D] * at(2.0) + w[L] * at(3.0))
    uyy = math.tan(-w[C] * math.pi / 4)
    assert Xl[1, 2:5, C] / h2 == pytest.approx([uxx, uxy, uyy], rel=1e-13)
    pBD, pDL, pLB = 0.5 * (w[B] + w[D]), 0.5 * (w[D] + w[L]), 0.5 * (w[L] + w[B])
    ux = math.tan(w[C] * at(3.0) + pBD * at(2.0) + pDL * at(1.0) + pLB * at(1.0))
    uy = math.tan(pBD * at(1.0) + pDL * at(2.0) + pLB * at(1.0))
    assert Xl[0, 0:2, C] / R2 == pytest.approx([ux, uy], rel=1e-13)
    assert Xl[0, 2:5, C] == pytest.approx([0.0, 0.0, 0.0], abs=1e-15)
    # wall cell B: weights 1/2, 1/2; directional candidate (0, 1)
    assert Xl[0, 0, B] / R2 == pytest.approx(math.tan(0.5 * at(0.5)), rel=1e-13)
    assert Xl[0, 1, B] / R2 == pytest.approx(0.0, abs=1e-15)
