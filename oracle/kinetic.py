"""Oracle third-order BGK flux at a Gauss point, section 2.

Everything is written in a local frame at the Gauss point: x along the unit
normal (from the left state L to the right state R), y along the tangent, the
origin at the Gauss point, so y = 0 there.  Conserved states are
W = (rho, rho U, rho V, E) with U normal and V tangential.

Particle-velocity polynomials are dictionaries {(a, b, c): coeff} for the
monomial u^a v^b (xi^2)^c, coefficients being arrays over Gauss points.
Moments of a Maxwellian factorise, <u^a v^b xi^2c> = <u^a><v^b><xi^2c>, with
<.> the integral against g / rho over the full velocity space or over one
half (u > 0 or u < 0) for the u factor.

Flux (Eq. generalSolution integrated over [0, dt]): the equilibrium part is
the time integral of Eq. 3orderg:2 and the initial non-equilibrium part that
of Eq. 3orderf0:2, both at y = 0; the second uses the half-space moments of
the left (u > 0) and right (u < 0) Maxwellians.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.special import erfc

# ---------------------------------------------------------------- polynomials


def poly_add(*ps):
    out = {}
    for p in ps:
        for key, c in p.items():
            out[key] = out.get(key, 0.0) + c
    return out


def poly_scale(p, s):
    return {key: c * s for key, c in p.items()}


def poly_mul(p, q):
    out = {}
    for (a1, b1, c1), x in p.items():
        for (a2, b2, c2), y in q.items():
            key = (a1 + a2, b1 + b2, c1 + c2)
            out[key] = out.get(key, 0.0) + x * y
    return out


ONE = {(0, 0, 0): 1.0}
U = {(1, 0, 0): 1.0}
V = {(0, 1, 0): 1.0}
# psi = (1, u, v, (u^2 + v^2 + xi^2) / 2), Eq. macroVar
PSI = [ONE, U, V, {(2, 0, 0): 0.5, (0, 2, 0): 0.5, (0, 0, 1): 0.5}]


def slope_poly(a):
    """a . psi for a = [4, ng] (the velocity polynomial a^0 + a^1 u + a^2 v
    + a^3 (u^2 + v^2 + xi^2) / 2 of Eq. Nomenclature1's a_1, a_2, A, ...)."""
    return poly_add(*[poly_scale(PSI[q], a[q]) for q in range(4)])


# ---------------------------------------------------------------- moments

@dataclass
class Moments:
    u: list   # <u^a>, a = 0..deg (full space or a half space)
    v: list   # <v^b>, full space
    x: list   # <(xi^2)^c>, c = 0..3


def full_u_moments(Uc, lam, deg):
    """<u^n> over the full line for the 1-D Gaussian of mean Uc and variance
    1/(2 lam): <u^0> = 1, <u> = Uc, <u^{n+2}> = Uc <u^{n+1}> + (n+1)/(2 lam) <u^n>."""
    m = [np.ones_like(Uc), Uc.copy()]
    for n in range(deg - 1):
        m.append(Uc * m[n + 1] + (n + 1) / (2.0 * lam) * m[n])
    return m[: deg + 1]


def half_u_moments(Uc, lam, deg, sign):
    """<u^n> over u > 0 (sign = +1) or u < 0 (sign = -1): the zeroth is
    erfc(-+ sqrt(lam) Uc) / 2, the first adds +- exp(-lam Uc^2) / (2 sqrt(pi lam)),
    and higher ones follow the same recursion as the full line."""
    m0 = 0.5 * erfc(-sign * np.sqrt(lam) * Uc)
    m1 = Uc * m0 + sign * np.exp(-lam * Uc * Uc) / (2.0 * np.sqrt(np.pi * lam))
    m = [m0, m1]
    for n in range(deg - 1):
        m.append(Uc * m[n + 1] + (n + 1) / (2.0 * lam) * m[n])
    return m[: deg + 1]


def xi_moments(lam, K):
    """<(xi^2)^c> for K internal degrees of freedom, each of variance 1/(2 lam)."""
    one = np.ones_like(lam)
    return [one, K / (2.0 * lam) * one, K * (K + 2.0) / (4.0 * lam ** 2),
            K * (K + 2.0) * (K + 4.0) / (8.0 * lam ** 3)]


def expect(p, mom: Moments):
    """<p> for a velocity polynomial p."""
    out = 0.0
    for (a, b, c), coef in p.items():
        out = out + coef * mom.u[a] * mom.v[b] * mom.x[c]
    return out


def psi_moments(p, mom: Moments):
    """[<psi_alpha p>]_alpha, shape [4, ng]."""
    return np.stack([np.broadcast_to(expect(poly_mul(PSI[q], p), mom), mom.u[0].shape) for q in range(4)])


# ---------------------------------------------------------------- states

def primitives(W, K):
    """rho, U, V, lambda of Eq. lambda (D = 2) from conserved W [4, ng]."""
    rho = W[0]
    Uc = W[1] / rho
    Vc = W[2] / rho
    lam = (K + 2.0) * rho / (4.0 * (W[3] - 0.5 * rho * (Uc * Uc + Vc * Vc)))
    return rho, Uc, Vc, lam


def maxwell_moments(W, K, deg_u=10, deg_v=10, half=0):
    rho, Uc, Vc, lam = primitives(W, K)
    if half == 0:
        mu = full_u_moments(Uc, lam, deg_u)
    else:
        mu = half_u_moments(Uc, lam, deg_u, half)
    return Moments(mu, full_u_moments(Vc, lam, deg_v), xi_moments(lam, K))


def slope(W, mom_full: Moments, D):
    """Solve rho <psi (a . psi)> = D for a (the inverse moment problem that
    turns a macroscopic derivative D into the coefficients of (dg/dx)/g);
    returns a [4, ng]."""
    rho = W[0]
    M = np.empty(D.shape[1:] + (4, 4))
    for al in range(4):
        for be in range(4):
            M[..., al, be] = rho * expect(poly_mul(PSI[al], PSI[be]), mom_full)
    return np.linalg.solve(M, np.moveaxis(D, 0, -1)[..., None])[..., 0].T


# ---------------------------------------------------------------- time integrals

def time_integrals(dt, tau, exact=False):
    """Integrals over [0, dt] of the coefficients c_1..c_8 of Eq.
    Nomenclature2, plus T9 = integral of c_7 t^2 / 2 (the coefficient of the
    second-order spatial term of Eq. 3orderf0:2 along x = -u t).

    With exact=True, c_4, c_5 and c_6 are replaced by the exact time
    integrals of the second-order terms of Eq. 3orderg:1, which add
    2 tau^2 c_1 to each."""
    e = np.exp(-dt / tau)
    T1 = dt - tau * (1.0 - e)
    T2 = 2.0 * tau * tau * (1.0 - e) - tau * dt * (1.0 + e)
    T3 = 0.5 * dt * dt - tau * dt + tau * tau * (1.0 - e)
    T4 = -4.0 * tau ** 3 + e * tau * (dt * dt + 4.0 * tau * dt + 4.0 * tau * tau)
    T5 = dt ** 3 / 3.0 - tau * dt * dt
    T6 = -0.5 * tau * dt * dt - tau ** 3 * (1.0 - e) + e * dt * tau * tau
    T7 = tau * (1.0 - e)
    T8 = -tau * tau + e * tau * (tau + dt)
    T9 = tau ** 3 - 0.5 * e * tau * (dt * dt + 2.0 * dt * tau + 2.0 * tau * tau)
    if exact:
        T4 = T4 + 2.0 * tau * tau * T1
        T5 = T5 + 2.0 * tau * tau * T1
        T6 = T6 + 2.0 * tau * tau * T1
    return T1, T2, T3, T4, T5, T6, T7, T8, T9


# ---------------------------------------------------------------- slopes

@dataclass
class Slopes:
    a1: np.ndarray
    a2: np.ndarray
    a11: np.ndarray
    a12: np.ndarray
    a22: np.ndarray
    A: np.ndarray
    A1: np.ndarray
    A2: np.ndarray
    At: np.ndarray | None = None


def side_slopes(W, Wn, Wt, Wnn, Wnt, Wtt, mom_full, with_At=False):
    """Slopes of Eq. Nomenclature1 for one Maxwellian with the given
    macroscopic first (n, t) and second (nn, nt, tt) derivatives.

    a1, a2: moments of dg/dx, dg/dy reproduce W_x, W_y.
    a11, a12, a22: d^2 g = g (a a + a_ij) reproduces the second derivatives.
    A (= dg/dt / g) and its derivatives A1 = a_1t, A2 = a_2t, A_t follow
    from the Euler-level compatibility <psi (u a1 + v a2 + A)> = 0 and its
    x-, y- and t-derivatives.
    """
    rho = W[0]
    a1 = slope(W, mom_full, Wn)
    a2 = slope(W, mom_full, Wt)
    p1 = slope_poly(a1)
    p2 = slope_poly(a2)
    a11 = slope(W, mom_full, Wnn - rho * psi_moments(poly_mul(p1, p1), mom_full))
    a12 = slope(W, mom_full, Wnt - rho * psi_moments(poly_mul(p1, p2), mom_full))
    a22 = slope(W, mom_full, Wtt - rho * psi_moments(poly_mul(p2, p2), mom_full))
    adv = poly_add(poly_mul(p1, U), poly_mul(p2, V))            # u a1 + v a2
    A = slope(W, mom_full, -rho * psi_moments(adv, mom_full))
    q = poly_add(adv, slope_poly(A))                              # u a1 + v a2 + A
    p11, p12, p22 = slope_poly(a11), slope_poly(a12), slope_poly(a22)
    A1 = slope(W, mom_full, -rho * psi_moments(
        poly_add(poly_mul(p11, U), poly_mul(p12, V), poly_mul(p1, q)), mom_full))
    A2 = slope(W, mom_full, -rho * psi_moments(
        poly_add(poly_mul(p12, U), poly_mul(p22, V), poly_mul(p2, q)), mom_full))
    At = None
    if with_At:
        pA = slope_poly(A)
        At = slope(W, mom_full, -rho * psi_moments(
            poly_add(poly_mul(slope_poly(A1), U), poly_mul(slope_poly(A2), V), poly_mul(pA, q)), mom_full))
    return Slopes(a1, a2, a11, a12, a22, A, A1, A2, At)


# ---------------------------------------------------------------- flux

def collision_time(pL, pR, p0, dt, mu, eps):
    """Eq. tauIns (mu = 0) or Eq. tauVis (mu > 0); the pressure-jump term is
    multiplied by dt (as printed it has no time unit, so it is read as a
    fraction of the step)."""
    jump = np.abs(pL - pR) / np.abs(pL + pR) * dt
    if mu > 0.0:
        return mu / p0 + jump
    return eps * dt + jump


def pressure(W, gamma):
    return (gamma - 1.0) * (W[3] - 0.5 * (W[1] ** 2 + W[2] ** 2) / W[0])


def gp_flux(WL, dL, WR, dR, dt, gamma, mu=0.0, eps=0.01, exact_time=False, return_parts=False):
    """Time-integrated flux per unit length over [0, dt] at Gauss points.

    WL, WR  [4, ng] local-frame conserved states of both sides
    dL, dR  dicts with keys 'n', 't', 'nn', 'nt', 'tt' -> [4, ng] derivatives
    Returns F [4, ng] = integral over [0, dt] of the moments
    (u psi f) dXi (Eq. fluxes) with f from Eq. generalSolution.
    """
    K = 2.0 / (gamma - 1.0) - 2.0
    momL = maxwell_moments(WL, K)
    momR = maxwell_moments(WR, K)
    momLp = maxwell_moments(WL, K, half=+1)
    momRm = maxwell_moments(WR, K, half=-1)

    # equilibrium state at the interface: collision of the two half streams
    W0 = WL[0] * psi_moments(ONE, momLp) + WR[0] * psi_moments(ONE, momRm)
    mom0 = maxwell_moments(W0, K)

    pL = pressure(WL, gamma)
    pR = pressure(WR, gamma)
    p0 = pressure(W0, gamma)
    tau = collision_time(pL, pR, p0, dt, mu, eps)

    sL = side_slopes(WL, dL["n"], dL["t"], dL["nn"], dL["nt"], dL["tt"], momL)
    sR = side_slopes(WR, dR["n"], dR["t"], dR["nn"], dR["nt"], dR["tt"], momR)
    d0 = {key: 0.5 * (dL[key] + dR[key]) for key in dL}
    s0 = side_slopes(W0, d0["n"], d0["t"], d0["nn"], d0["nt"], d0["tt"], mom0, with_At=True)

    T1, T2, T3, T4, T5, T6, T7, T8, T9 = time_integrals(dt, tau, exact_time)

    # equilibrium part, time integral of Eq. 3orderg:2 at y = 0
    b1, b2 = slope_poly(s0.a1), slope_poly(s0.a2)
    bA = slope_poly(s0.A)
    sq11 = poly_add(poly_mul(b1, b1), slope_poly(s0.a11))          # a1^2 + a11
    sq12 = poly_add(poly_mul(b1, b2), slope_poly(s0.a12))          # a1 a2 + a12
    sq22 = poly_add(poly_mul(b2, b2), slope_poly(s0.a22))          # a2^2 + a22
    Peq = poly_add(
        poly_scale(ONE, T1),
        poly_scale(poly_add(poly_mul(b1, U), poly_mul(b2, V)), T2),
        poly_scale(bA, T3),
        poly_scale(poly_add(poly_mul(sq11, poly_mul(U, U)),
                            poly_scale(poly_mul(sq12, poly_mul(U, V)), 2.0),
                            poly_mul(sq22, poly_mul(V, V))), 0.5 * T4),
        poly_scale(poly_add(poly_mul(poly_add(poly_mul(bA, b1), slope_poly(s0.A1)), U),
                            poly_mul(poly_add(poly_mul(bA, b2), slope_poly(s0.A2)), V)), T6),
        poly_scale(poly_add(poly_mul(bA, bA), slope_poly(s0.At)), 0.5 * T5),
    )

    def nonequilibrium(s: Slopes):
        """Time integral of Eq. 3orderf0:2 at y = 0 (as the factor of g_k)."""
        p1, p2 = slope_poly(s.a1), slope_poly(s.a2)
        pA = slope_poly(s.A)
        q = poly_add(poly_mul(p1, U), poly_mul(p2, V), pA)         # a1 u + a2 v + A
        zero = poly_add(ONE, poly_scale(q, -tau))
        xpart = poly_mul(U, poly_add(p1, poly_scale(poly_add(
            poly_mul(p1, q), poly_mul(slope_poly(s.a11), U), poly_mul(slope_poly(s.a12), V),
            slope_poly(s.A1)), -tau)))
        ypart = poly_mul(V, poly_add(p2, poly_scale(poly_add(
            poly_mul(p2, q), poly_mul(slope_poly(s.a12), U), poly_mul(slope_poly(s.a22), V),
            slope_poly(s.A2)), -tau)))
        s11 = poly_add(poly_mul(p1, p1), slope_poly(s.a11))
        s12 = poly_add(poly_mul(p1, p2), slope_poly(s.a12))
        s22 = poly_add(poly_mul(p2, p2), slope_poly(s.a22))
        second = poly_add(poly_mul(s11, poly_mul(U, U)), poly_scale(poly_mul(s12, poly_mul(U, V)), 2.0),
                          poly_mul(s22, poly_mul(V, V)))
        return poly_add(poly_scale(zero, T7), poly_scale(poly_add(xpart, ypart), T8),
                        poly_scale(second, T9))

    PL = nonequilibrium(sL)
    PR = nonequilibrium(sR)
    F_eq = W0[0] * psi_moments(poly_mul(U, Peq), mom0)
    F_L = WL[0] * psi_moments(poly_mul(U, PL), momLp)
    F_R = WR[0] * psi_moments(poly_mul(U, PR), momRm)
    F = F_eq + F_L + F_R
    if return_parts:
        return F, dict(W0=W0, tau=tau, sL=sL, sR=sR, s0=s0, F_eq=F_eq, F_L=F_L, F_R=F_R)
    return F
