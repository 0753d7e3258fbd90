"""Oracle: exact solution of the one-dimensional Riemann problem for the
Euler equations of a polytropic gas (used for the Sod and Lax shock tubes of
sections 4.2 and 4.3).

TEST INFRASTRUCTURE ONLY: imported by tests/, never by the library.

Across each nonlinear wave the star pressure p* fixes the state: a shock
(p* > p_K) obeys the Rankine-Hugoniot relations, a rarefaction (p* <= p_K)
the isentropic relations with a constant Riemann invariant.  The velocity
jump f_L(p) + f_R(p) + (u_R - u_L) = 0, with the branch functions below, is
solved for p* by Newton's method; the solution at x/t is then sampled from
the wave pattern.
"""
from __future__ import annotations

import math

import numpy as np


def _branch(p, rho, pk, gamma):
    """f_K(p) and its derivative: the velocity change across the wave
    connecting state K (rho, pk) with pressure p."""
    c = math.sqrt(gamma * pk / rho)
    if p > pk:   # shock
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        q = math.sqrt(A / (p + B))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (p + B))
    # rarefaction
    e = (gamma - 1.0) / (2.0 * gamma)
    r = p / pk
    return 2.0 * c / (gamma - 1.0) * (r ** e - 1.0), 1.0 / (rho * c) * r ** (-(gamma + 1.0) / (2.0 * gamma))


def star_state(left, right, gamma=1.4):
    """(p*, u*) for primitive states left = (rho, u, p), right likewise."""
    rl, ul, pl = left
    rr, ur, pr = right
    p = max(1e-12, 0.5 * (pl + pr))
    for _ in range(100):
        fl, dl = _branch(p, rl, pl, gamma)
        fr, dr = _branch(p, rr, pr, gamma)
        g = fl + fr + (ur - ul)
        pn = max(1e-14, p - g / (dl + dr))
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _branch(p, rl, pl, gamma)
    fr, _ = _branch(p, rr, pr, gamma)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(left, right, s, gamma=1.4):
    """Primitive (rho, u, p) at similarity coordinates s = (x - x0) / t."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = star_state(left, right, gamma)
    s = np.asarray(s, dtype=np.float64)
    rho = np.empty_like(s)
    u = np.empty_like(s)
    p = np.empty_like(s)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    for k, sk in np.ndenumerate(s):
        if sk <= us:   # left of the contact
            rho_k, u_k, p_k, sign = rl, ul, pl, -1.0
        else:
            rho_k, u_k, p_k, sign = rr, ur, pr, 1.0
        c_k = math.sqrt(gamma * p_k / rho_k)
        if ps > p_k:   # shock on this side
            rho_s = rho_k * (ps / p_k + g1) / (g1 * ps / p_k + 1.0)
            speed = u_k + sign * c_k * math.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / p_k + (gamma - 1.0) / (2.0 * gamma))
            behind = sk < speed if sign > 0 else sk > speed
            rho[k], u[k], p[k] = (rho_s, us, ps) if behind else (rho_k, u_k, p_k)
        else:          # rarefaction on this side
            rho_s = rho_k * (ps / p_k) ** (1.0 / gamma)
            c_s = c_k * (ps / p_k) ** ((gamma - 1.0) / (2.0 * gamma))
            head = u_k + sign * c_k
            tail = us + sign * c_s
            outside = sk > head if sign > 0 else sk < head
            inside_star = sk < tail if sign > 0 else sk > tail
            if outside:
                rho[k], u[k], p[k] = rho_k, u_k, p_k
            elif inside_star:
                rho[k], u[k], p[k] = rho_s, us, ps
            else:      # inside the fan
                uu = 2.0 / (gamma + 1.0) * (-sign * c_k + (gamma - 1.0) / 2.0 * u_k + sk)
                cc = 2.0 / (gamma + 1.0) * (c_k - sign * (gamma - 1.0) / 2.0 * (u_k - sk))
                rho[k] = rho_k * (cc / c_k) ** (2.0 / (gamma - 1.0))
                u[k] = uu
                p[k] = p_k * (cc / c_k) ** (2.0 * gamma / (gamma - 1.0))
    return rho, u, p


def tube_cell_averages(mesh, left, right, x0, t, gamma=1.4):
    """Conserved cell averages [4, nt] of the exact shock-tube solution at
    time t (the 8 x 8 collapsed Gauss rule of the input generator)."""
    import gks_inputs as gi

    def fn(x, y):
        rho, u, p = sample(left, right, (x - x0) / t, gamma)
        return np.stack([rho, rho * u, np.zeros_like(rho), p / (gamma - 1.0) + 0.5 * rho * u * u])

    return gi.cell_average(mesh, fn)
