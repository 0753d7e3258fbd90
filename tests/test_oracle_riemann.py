"""Pins of the oracle's exact Riemann solver (used for the Sod and Lax tubes,
sections 4.2-4.3), by the conservation laws themselves rather than by
printed numbers:
  * across the shock the Rankine-Hugoniot relations hold for mass, momentum
    and energy with the sampled shock speed;
  * through a rarefaction the entropy p / rho^gamma and the Riemann
    invariant u +- 2c / (gamma - 1) are constant;
  * velocity and pressure are continuous across the contact;
  * the integrals of the conserved variables over the tube do not change;
  * equal states give the uniform state, and mirroring the problem mirrors
    the solution.
"""
import numpy as np
import pytest

from oracle import riemann

G = 1.4
SOD = ((1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
LAX = ((0.445, 0.698, 3.528), (0.5, 0.0, 0.571))


def cons(rho, u, p):
    return np.array([rho, rho * u, p / (G - 1) + 0.5 * rho * u * u])


def flux(rho, u, p):
    E = p / (G - 1) + 0.5 * rho * u * u
    return np.array([rho * u, rho * u * u + p, u * (E + p)])


def jumps(left, right):
    """Sample densely and locate the discontinuities (indices of jumps)."""
    s = np.linspace(-4.0, 4.0, 400001)
    r, u, p = riemann.sample(left, right, s, G)
    return s, r, u, p


@pytest.mark.parametrize("case", [SOD, LAX])
def test_rankine_hugoniot_at_the_shock(case):
    s, r, u, p = jumps(*case)
    dp = np.abs(np.diff(p))
    k = int(np.argmax(dp))            # the largest pressure jump is the shock
    a, b = k - 1, k + 2
    Ua, Ub = cons(r[a], u[a], p[a]), cons(r[b], u[b], p[b])
    Fa, Fb = flux(r[a], u[a], p[a]), flux(r[b], u[b], p[b])
    S = (Fb[0] - Fa[0]) / (Ub[0] - Ua[0])
    assert np.allclose(Fb - Fa, S * (Ub - Ua), rtol=1e-9, atol=1e-9)
    assert abs(S - s[k]) < 1e-4


@pytest.mark.parametrize("case", [SOD, LAX])
def test_contact_and_rarefaction(case):
    left, right = case
    ps, us = riemann.star_state(left, right, G)
    s, r, u, p = jumps(left, right)
    # contact: rho jumps, u and p do not
    k = int(np.argmin(np.abs(s - us)))
    assert abs(p[k - 2] - p[k + 2]) < 1e-12 and abs(u[k - 2] - u[k + 2]) < 1e-12
    assert abs(r[k - 2] - r[k + 2]) > 1e-3
    # left rarefaction (both cases have one): entropy and u + 2c/(g-1) constant
    cl = np.sqrt(G * left[2] / left[0])
    fan = (s > left[1] - cl + 1e-6) & (s < us - np.sqrt(G * ps / (left[0] * (ps / left[2]) ** (1 / G))) - 1e-6)
    assert fan.sum() > 100
    c = np.sqrt(G * p[fan] / r[fan])
    assert np.abs(p[fan] / r[fan] ** G - left[2] / left[0] ** G).max() < 1e-12
    assert np.abs(u[fan] + 2 * c / (G - 1) - (left[1] + 2 * cl / (G - 1))).max() < 1e-12


@pytest.mark.parametrize("case,t", [(SOD, 0.2), (LAX, 0.14)])
def test_conservation_over_the_tube(case, t):
    left, right = case
    x = np.linspace(0.0, 1.0, 400001)
    r, u, p = riemann.sample(left, right, (x - 0.5) / t, G)
    U = cons(r, u, p)
    left_c, right_c = cons(*left), cons(*right)
    init = 0.5 * left_c + 0.5 * right_c
    # boundary fluxes of the undisturbed end states over [0, t]
    bnd = t * (flux(*left) - flux(*right))
    tot = np.trapezoid(U, x, axis=1)
    assert np.allclose(tot, init + bnd, rtol=2e-5, atol=2e-5)


def test_uniform_and_mirror():
    st = (0.7, 0.3, 1.9)
    r, u, p = riemann.sample(st, st, np.linspace(-2, 2, 11), G)
    assert np.allclose(r, 0.7) and np.allclose(u, 0.3) and np.allclose(p, 1.9)
    s = np.linspace(-3, 3, 1201)
    left, right = LAX
    r1, u1, p1 = riemann.sample(left, right, s, G)
    ml, mr = (right[0], -right[1], right[2]), (left[0], -left[1], left[2])
    r2, u2, p2 = riemann.sample(ml, mr, -s, G)
    keep = np.abs(np.diff(r1, prepend=r1[0])) < 1e-9   # away from jumps
    assert np.allclose(r1[keep], r2[keep]) and np.allclose(u1[keep], -u2[keep]) and np.allclose(p1[keep], p2[keep])
