"""Pins of the oracle's kinetic flux (section 2) against what mathematics fixes.

* Full- and half-space Maxwellian moments against adaptive 1-D quadrature
  and a 5-D Gauss-Hermite product rule (u, v and K = 3 internal variables).
* Moments of psi reproduce W (Eq. macroVar); the two half spaces add up to
  the full space.
* Slope inversion: residual of the moment equations and the compatibility
  condition.
* Time integrals against direct integration of the printed c_k(t) of Eq.
  Nomenclature2, and c_1 + c_7 = 1.  The exact variant against numerical
  integration of the BGK integral solution (Eq. generalSolution) of each
  Taylor monomial of Eq. 3orderg:1 along the characteristic.
* Uniform equilibrium flow: the flux is dt times the Euler flux for any tau.
* Mirror symmetries in the normal and tangential directions.
* tau = 0 smooth advection: the time-integrated mass flux matches the exact
  one to O(dt^4).
"""
import itertools

import numpy as np
import pytest
from scipy import integrate
from scipy.special import roots_hermite

from oracle import kinetic as kn

GAMMA = 1.4
K = 2.0 / (GAMMA - 1.0) - 2.0


def cons(rho, u, v, p):
    return np.array([rho, rho * u, rho * v, p / (GAMMA - 1.0) + 0.5 * rho * (u * u + v * v)], dtype=float)


def test_half_space_moments_quadrature():
    for Uc, lam in ((0.7, 1.3), (-1.1, 0.4), (0.0, 2.0)):
        Ua, la = np.array([Uc]), np.array([lam])
        for sign in (+1, -1):
            mom = kn.half_u_moments(Ua, la, 9, sign)
            lo, hi = (0.0, np.inf) if sign > 0 else (-np.inf, 0.0)
            for n in range(10):
                ref = integrate.quad(lambda u: u ** n * np.sqrt(lam / np.pi) * np.exp(-lam * (u - Uc) ** 2),
                                     lo, hi, epsabs=1e-15, epsrel=1e-14)[0]
                assert mom[n][0] == pytest.approx(ref, rel=1e-12, abs=1e-14)
        full = kn.full_u_moments(Ua, la, 9)
        plus = kn.half_u_moments(Ua, la, 9, +1)
        minus = kn.half_u_moments(Ua, la, 9, -1)
        for n in range(10):
            assert plus[n][0] + minus[n][0] == pytest.approx(full[n][0], rel=1e-13, abs=1e-14)


def hermite_expect(W, fn, npts=12):
    """rho-normalised expectation of fn(u, v, xi2) over the Maxwellian of W by a
    Gauss-Hermite product rule in (u, v, xi_1, xi_2, xi_3)."""
    rho, Uc, Vc, lam = [float(q[0]) for q in kn.primitives(W[:, None], K)]
    x, w = roots_hermite(npts)
    s = 1.0 / np.sqrt(lam)
    w = w / np.sqrt(np.pi)
    tot = 0.0
    for (i, xu), (j, xv) in itertools.product(enumerate(x), enumerate(x)):
        u = Uc + s * xu
        v = Vc + s * xv
        xi = s * x
        xi2 = (xi[:, None, None] ** 2 + xi[None, :, None] ** 2 + xi[None, None, :] ** 2)
        wx = w[:, None, None] * w[None, :, None] * w[None, None, :]
        tot += w[i] * w[j] * np.sum(wx * fn(u, v, xi2))
    return tot


def test_factorised_moments_against_5d_hermite():
    W = cons(1.3, 0.4, -0.7, 0.9)
    mom = kn.maxwell_moments(W[:, None], K)
    for a, b, c in ((0, 0, 0), (3, 1, 0), (2, 2, 1), (1, 0, 2), (0, 3, 3), (4, 2, 1)):
        got = kn.expect({(a, b, c): 1.0}, mom)[0]
        ref = hermite_expect(W, lambda u, v, x2: u ** a * v ** b * x2 ** c)
        assert got == pytest.approx(ref, rel=1e-11)


def test_psi_moments_reproduce_W():
    W = cons(0.8, -0.3, 1.2, 2.0)[:, None]
    mom = kn.maxwell_moments(W, K)
    assert np.allclose(W[0] * kn.psi_moments(kn.ONE, mom), W, rtol=1e-14)


def test_slope_inversion_residual_and_compatibility():
    rng = np.random.default_rng(4)
    W = np.stack([cons(1.1, 0.5, -0.2, 0.8), cons(0.6, -1.3, 0.9, 1.7)], axis=1)
    mom = kn.maxwell_moments(W, K)
    D = rng.normal(size=(4, 2))
    a = kn.slope(W, mom, D)
    back = W[0] * kn.psi_moments(kn.slope_poly(a), mom)
    assert np.abs(back - D).max() < 1e-13 * np.abs(D).max()
    # against quadrature, independent of the factorised moments
    for g in range(2):
        Wg = W[:, g]
        psi = lambda u, v, x2: [np.ones_like(x2), u + 0 * x2, v + 0 * x2, 0.5 * (u * u + v * v + x2)]
        aps = lambda u, v, x2: a[0, g] + a[1, g] * u + a[2, g] * v + a[3, g] * 0.5 * (u * u + v * v + x2)
        for al in range(4):
            val = Wg[0] * hermite_expect(Wg, lambda u, v, x2: psi(u, v, x2)[al] * aps(u, v, x2))
            assert val == pytest.approx(D[al, g], rel=1e-10, abs=1e-12)
    # Euler-level compatibility: <psi (u a1 + v a2 + A)> = 0
    s = kn.side_slopes(W, D, 0.5 * D, 0.1 * D, -0.2 * D, 0.3 * D, mom)
    q = kn.poly_add(kn.poly_mul(kn.slope_poly(s.a1), kn.U), kn.poly_mul(kn.slope_poly(s.a2), kn.V),
                    kn.slope_poly(s.A))
    assert np.abs(kn.psi_moments(q, mom)).max() < 1e-12


PRINTED_C = {  # the coefficients c_1..c_8 as printed in Eq. Nomenclature2
    1: lambda t, tau: 1 - np.exp(-t / tau),
    2: lambda t, tau: (t + tau) * np.exp(-t / tau) - tau,
    3: lambda t, tau: t - tau + tau * np.exp(-t / tau),
    4: lambda t, tau: -np.exp(-t / tau) * (t * t + 2 * t * tau),
    5: lambda t, tau: t * t - 2 * tau * t,
    6: lambda t, tau: -t * tau - np.exp(-t / tau) * t * tau,
    7: lambda t, tau: np.exp(-t / tau),
    8: lambda t, tau: -t * np.exp(-t / tau),
}


@pytest.mark.parametrize("dt,tau", [(1e-3, 1e-5), (0.01, 0.004), (0.2, 0.5)])
def test_time_integrals_of_printed_coefficients(dt, tau):
    T = kn.time_integrals(dt, tau)
    for k in range(1, 9):
        ref = integrate.quad(lambda t: PRINTED_C[k](t, tau), 0.0, dt, epsabs=0, epsrel=1e-13, limit=200)[0]
        assert T[k - 1] == pytest.approx(ref, rel=1e-9, abs=1e-22)
    ref9 = integrate.quad(lambda t: 0.5 * t * t * np.exp(-t / tau), 0.0, dt, epsabs=0, epsrel=1e-13)[0]
    assert T[8] == pytest.approx(ref9, rel=1e-9, abs=1e-24)
    assert T[0] + T[6] == pytest.approx(dt, rel=1e-14)
    assert PRINTED_C[1](0.3, 0.1) + PRINTED_C[7](0.3, 0.1) == pytest.approx(1.0)


@pytest.mark.parametrize("dt,tau", [(0.01, 0.004), (0.2, 0.5)])
def test_exact_time_integrals_from_the_integral_solution(dt, tau):
    """Integrate (1/tau) int_0^t m(s) e^{-s/tau} ds over t in [0, dt] for each
    monomial of Eq. 3orderg:1 written along x' = -u s, t' = t - s (per unit u)."""
    def kernel(mono):
        inner = lambda t: integrate.quad(lambda s: mono(s, t) * np.exp(-s / tau) / tau, 0.0, t,
                                         epsabs=0, epsrel=1e-13)[0]
        return integrate.quad(inner, 0.0, dt, epsabs=0, epsrel=1e-12)[0]

    T = kn.time_integrals(dt, tau, exact=True)
    assert T[0] == pytest.approx(kernel(lambda s, t: 1.0), rel=1e-9)
    assert T[1] == pytest.approx(kernel(lambda s, t: -s), rel=1e-9)              # x
    assert T[2] == pytest.approx(kernel(lambda s, t: t - s), rel=1e-9)           # t
    assert T[3] == pytest.approx(kernel(lambda s, t: s * s), rel=1e-9)           # x^2
    assert T[4] == pytest.approx(kernel(lambda s, t: (t - s) ** 2), rel=1e-9)    # t^2
    assert T[5] == pytest.approx(kernel(lambda s, t: -s * (t - s)), rel=1e-9)    # x t


def zero_derivs(m):
    return {key: np.zeros((4, m)) for key in ("n", "t", "nn", "nt", "tt")}


@pytest.mark.parametrize("eps,mu", [(0.01, 0.0), (0.0, 0.0), (0.01, 2e-3)])
def test_uniform_flow_gives_euler_flux(eps, mu):
    W = np.stack([cons(1.2, 0.7, -0.4, 1.1), cons(0.9, -1.5, 0.2, 0.6), cons(1.0, 0.0, 0.0, 1.0)], axis=1)
    dt = 0.013
    with np.errstate(divide="ignore"):
        F = kn.gp_flux(W, zero_derivs(3), W, zero_derivs(3), dt, GAMMA, mu=mu, eps=eps)
    rho, u, v = W[0], W[1] / W[0], W[2] / W[0]
    p = (GAMMA - 1) * (W[3] - 0.5 * rho * (u * u + v * v))
    euler = np.stack([rho * u, rho * u * u + p, rho * u * v, u * (W[3] + p)])
    assert np.abs(F - dt * euler).max() < 1e-14 * np.abs(dt * euler).max() * 10


def random_side(rng, m):
    W = np.stack([cons(rng.uniform(0.7, 1.3), rng.uniform(-0.8, 0.8), rng.uniform(-0.8, 0.8),
                       rng.uniform(0.7, 1.3)) for _ in range(m)], axis=1)
    d = {key: 0.05 * rng.normal(size=(4, m)) for key in ("n", "t", "nn", "nt", "tt")}
    return W, d


def test_normal_mirror_symmetry():
    rng = np.random.default_rng(12)
    WL, dL = random_side(rng, 5)
    WR, dR = random_side(rng, 5)
    dt = 0.01
    F = kn.gp_flux(WL, dL, WR, dR, dt, GAMMA)
    P = np.array([1.0, -1.0, 1.0, 1.0])[:, None]
    odd = {"n": -1.0, "t": 1.0, "nn": 1.0, "nt": -1.0, "tt": 1.0}
    mir = lambda d: {key: odd[key] * P * val for key, val in d.items()}
    Fm = kn.gp_flux(P * WR, mir(dR), P * WL, mir(dL), dt, GAMMA)
    expect = np.array([-1.0, 1.0, -1.0, -1.0])[:, None] * F
    assert np.abs(Fm - expect).max() < 1e-13 * np.abs(F).max()


def test_tangential_mirror_symmetry():
    rng = np.random.default_rng(13)
    WL, dL = random_side(rng, 5)
    WR, dR = random_side(rng, 5)
    dt = 0.01
    F = kn.gp_flux(WL, dL, WR, dR, dt, GAMMA)
    Q = np.array([1.0, 1.0, -1.0, 1.0])[:, None]
    odd = {"n": 1.0, "t": -1.0, "nn": 1.0, "nt": -1.0, "tt": 1.0}
    mir = lambda d: {key: odd[key] * Q * val for key, val in d.items()}
    Fm = kn.gp_flux(Q * WL, mir(dL), Q * WR, mir(dR), dt, GAMMA)
    assert np.abs(Fm - Q * F).max() < 1e-13 * np.abs(F).max()


def test_smooth_advection_flux_is_fourth_order_in_dt():
    """Identical sides, tau = 0, rho(x) = 1 + 0.2 sin(k x + 0.3), u = 1, p = 1:
    the exact time-integrated mass flux through x = 0 is the integral of
    rho(-t) over [0, dt]; the error must fall as dt^4."""
    kk, ph, Uc, p = 2.0, 0.3, 1.0, 1.0
    rho = lambda x: 1 + 0.2 * np.sin(kk * x + ph)
    rx = lambda x: 0.2 * kk * np.cos(kk * x + ph)
    rxx = lambda x: -0.2 * kk * kk * np.sin(kk * x + ph)
    W = cons(rho(0.0), Uc, 0.0, p)[:, None]
    def dcons(d):
        return np.array([d, d * Uc, 0.0, 0.5 * d * Uc * Uc])[:, None]
    dd = {"n": dcons(rx(0.0)), "t": np.zeros((4, 1)), "nn": dcons(rxx(0.0)),
          "nt": np.zeros((4, 1)), "tt": np.zeros((4, 1))}
    errs = []
    for dt in (0.04, 0.02, 0.01):
        with np.errstate(divide="ignore"):
            F = kn.gp_flux(W, dd, W, dd, dt, GAMMA, eps=0.0)
        exact = integrate.quad(lambda t: rho(-Uc * t) * Uc, 0.0, dt, epsabs=1e-17, epsrel=1e-14)[0]
        errs.append(abs(F[0, 0] - exact))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 13.0 < r1 < 19.0 and 13.0 < r2 < 19.0, errs


# ------------------------------------------------------------------ slopes by definition

def log_g_coeffs(Wv):
    """ln g = b0 + b1 u + b2 v + b3 (u^2 + v^2 + xi^2) / 2 for the Maxwellian of
    conserved W (Eq. maxwellian); returns b [4]."""
    rho, Uc, Vc = Wv[0], Wv[1] / Wv[0], Wv[2] / Wv[0]
    lam = (K + 2.0) * rho / (4.0 * (Wv[3] - 0.5 * rho * (Uc * Uc + Vc * Vc)))
    return np.array([np.log(rho) + 0.5 * (K + 2.0) * np.log(lam / np.pi) - lam * (Uc * Uc + Vc * Vc),
                     2.0 * lam * Uc, 2.0 * lam * Vc, -2.0 * lam])


def euler_flux_x(Wv):
    rho, Uc, Vc = Wv[0], Wv[1] / Wv[0], Wv[2] / Wv[0]
    p = (GAMMA - 1.0) * (Wv[3] - 0.5 * rho * (Uc * Uc + Vc * Vc))
    return np.array([rho * Uc, rho * Uc * Uc + p, rho * Uc * Vc, Uc * (Wv[3] + p)])


def test_slopes_match_derivatives_of_log_g():
    """a1 = d(ln g)/dx, a11 = da1/dx (Eq. Nomenclature1) along a quadratic
    macroscopic field W(x); A = d(ln g)/dt, A1 = dA/dx and A_t = dA/dt with
    W_t, W_tt from the one-dimensional Euler equations.  Derivatives are taken
    by finite differences, independently of the moment inversion."""
    W0 = cons(1.1, 0.4, -0.3, 0.9)
    W1 = np.array([0.07, -0.05, 0.03, 0.11])
    W2 = np.array([-0.09, 0.04, 0.06, -0.08])
    Wof = lambda x: W0 + W1 * x + 0.5 * W2 * x * x
    d = 1e-3
    fd1 = lambda f: (-f(2 * d) + 8 * f(d) - 8 * f(-d) + f(-2 * d)) / (12 * d)
    fd2 = lambda f: (-f(2 * d) + 16 * f(d) - 30 * f(0.0) + 16 * f(-d) - f(-2 * d)) / (12 * d * d)
    Wt = lambda x: -fd1(lambda s: euler_flux_x(Wof(x + s)))                  # W_t(x)
    jac = lambda Wv, dW: (euler_flux_x(Wv + 1e-6 * dW) - euler_flux_x(Wv - 1e-6 * dW)) / 2e-6
    Wtt0 = -fd1(lambda s: jac(Wof(s), Wt(s)))                                # W_tt(0)
    lg = lambda Wv: log_g_coeffs(Wv)
    a1_ref = fd1(lambda s: lg(Wof(s)))
    a11_ref = fd2(lambda s: lg(Wof(s)))
    dlg = lambda Wv, dW: (lg(Wv + 1e-6 * dW) - lg(Wv - 1e-6 * dW)) / 2e-6    # d(ln g)/dW . dW
    A_ref = dlg(W0, Wt(0.0))
    A1_ref = fd1(lambda s: dlg(Wof(s), Wt(s)))
    # d2(ln g)/dt2 = D2 lg[W_t, W_t] + D lg[W_tt]
    h = 1e-4
    Wt0 = Wt(0.0)
    At_ref = (lg(W0 + h * Wt0) - 2 * lg(W0) + lg(W0 - h * Wt0)) / h ** 2 + dlg(W0, Wtt0)

    mom = kn.maxwell_moments(W0[:, None], K)
    z = np.zeros((4, 1))
    s = kn.side_slopes(W0[:, None], W1[:, None], z, W2[:, None], z, z, mom, with_At=True)
    # a . psi has coefficients (a0, a1, a2, a3) on (1, u, v, (u^2+v^2+xi^2)/2): same as b
    for got, ref, tol in ((s.a1, a1_ref, 1e-9), (s.a11, a11_ref, 1e-6), (s.A, A_ref, 1e-8),
                          (s.A1, A1_ref, 1e-6), (s.At, At_ref, 1e-5)):
        assert np.abs(got[:, 0] - ref).max() < tol * max(1.0, np.abs(ref).max()), (got[:, 0], ref)
    assert np.abs(s.a2).max() == 0.0


# ------------------------------------------------------------------ flux by direct quadrature

def velocity_rules(Wv, half):
    """Quadrature nodes/weights for the Maxwellian of W: u over the full line
    (Gauss-Hermite) or one half line (Gauss-Legendre on a truncated range), v
    by Gauss-Hermite, xi^2 by generalised Gauss-Laguerre (K = 3)."""
    from scipy.special import roots_genlaguerre
    rho, Uc, Vc = Wv[0], Wv[1] / Wv[0], Wv[2] / Wv[0]
    lam = (K + 2.0) * rho / (4.0 * (Wv[3] - 0.5 * rho * (Uc * Uc + Vc * Vc)))
    sd = 1.0 / np.sqrt(2.0 * lam)
    if half == 0:
        x, w = roots_hermite(30)
        u, wu = Uc + np.sqrt(2.0) * sd * x, w / np.sqrt(np.pi)
    else:
        lo, hi = (0.0, max(Uc, 0.0) + 14 * sd) if half > 0 else (min(Uc, 0.0) - 14 * sd, 0.0)
        x, w = np.polynomial.legendre.leggauss(200)
        u = 0.5 * (hi - lo) * x + 0.5 * (hi + lo)
        wu = 0.5 * (hi - lo) * w * np.sqrt(lam / np.pi) * np.exp(-lam * (u - Uc) ** 2)
    x, w = roots_hermite(30)
    v, wv = Vc + np.sqrt(2.0) * sd * x, w / np.sqrt(np.pi)
    r, wr = roots_genlaguerre(10, K / 2.0 - 1.0)       # xi^2 = r / lam
    from math import gamma as G
    return u, wu, v, wv, r / lam, wr / G(K / 2.0)


def test_flux_equals_direct_quadrature_of_the_expansions():
    """Integrate u psi f over velocity and t in [0, dt], with f written term by
    term from Eqs. generalSolution, 3orderg:2 and 3orderf0:2 (y = 0) and the
    printed c_k(t), using the oracle's slopes, W0 and tau."""
    rng = np.random.default_rng(21)
    WL, dL = random_side(rng, 1)
    WR, dR = random_side(rng, 1)
    dL = {k: 4 * v for k, v in dL.items()}
    dR = {k: 4 * v for k, v in dR.items()}
    dt = 0.02
    F, parts = kn.gp_flux(WL, dL, WR, dR, dt, GAMMA, eps=0.3, return_parts=True)
    tau = float(parts["tau"][0])
    assert tau > 0.1 * dt           # the non-equilibrium part matters here
    tq, tw = np.polynomial.legendre.leggauss(24)
    tq, tw = 0.5 * dt * (tq + 1), 0.5 * dt * tw
    c = {k: PRINTED_C[k](tq, tau) for k in PRINTED_C}

    def sp(a, u, v, x2):            # a . psi at velocity points
        return a[0, 0] + a[1, 0] * u + a[2, 0] * v + a[3, 0] * 0.5 * (u * u + v * v + x2)

    def integrate_side(Wv, half, integrand):
        u, wu, v, wv, x2, wx = velocity_rules(Wv, half)
        U_, V_, X_ = np.meshgrid(u, v, x2, indexing="ij")
        Wt = wu[:, None, None] * wv[None, :, None] * wx[None, None, :]
        psi = [np.ones_like(U_), U_, V_, 0.5 * (U_ * U_ + V_ * V_ + X_)]
        out = np.zeros(4)
        for it in range(tq.size):
            fval = integrand(U_, V_, X_, it)
            for al in range(4):
                out[al] += tw[it] * Wv[0] * np.sum(Wt * U_ * psi[al] * fval)
        return out

    s0 = parts["s0"]

    def eq(u, v, x2, it):
        b1, b2, bA = sp(s0.a1, u, v, x2), sp(s0.a2, u, v, x2), sp(s0.A, u, v, x2)
        return (c[1][it] + c[2][it] * (b1 * u + b2 * v) + c[3][it] * bA
                + 0.5 * c[4][it] * ((b1 * b1 + sp(s0.a11, u, v, x2)) * u * u
                                    + 2 * (b1 * b2 + sp(s0.a12, u, v, x2)) * u * v
                                    + (b2 * b2 + sp(s0.a22, u, v, x2)) * v * v)
                + c[6][it] * ((bA * b1 + sp(s0.A1, u, v, x2)) * u + (bA * b2 + sp(s0.A2, u, v, x2)) * v)
                + 0.5 * c[5][it] * (bA * bA + sp(s0.At, u, v, x2)))

    def noneq(s):
        def fn(u, v, x2, it):
            t = tq[it]
            a1, a2, A = sp(s.a1, u, v, x2), sp(s.a2, u, v, x2), sp(s.A, u, v, x2)
            a11, a12, a22 = sp(s.a11, u, v, x2), sp(s.a12, u, v, x2), sp(s.a22, u, v, x2)
            A1, A2 = sp(s.A1, u, v, x2), sp(s.A2, u, v, x2)
            return (c[7][it] * (1 - tau * (a1 * u + a2 * v + A))
                    + c[8][it] * (a1 * u - tau * ((a1 * a1 + a11) * u * u + (a1 * a2 + a12) * u * v + (A * a1 + A1) * u))
                    + c[8][it] * (a2 * v - tau * ((a1 * a2 + a12) * u * v + (a2 * a2 + a22) * v * v + (A * a2 + A2) * v))
                    + 0.5 * c[7][it] * ((a1 * a1 + a11) * (u * t) ** 2 + 2 * (a1 * a2 + a12) * (u * t) * (v * t)
                                        + (a2 * a2 + a22) * (v * t) ** 2))
        return fn

    ref = (integrate_side(parts["W0"][:, 0], 0, eq) + integrate_side(WL[:, 0], +1, noneq(parts["sL"]))
           + integrate_side(WR[:, 0], -1, noneq(parts["sR"])))
    assert np.abs(F[:, 0] - ref).max() < 1e-11 * np.abs(ref).max(), (F[:, 0], ref)
    # the pieces are individually significant, so a dropped term would show
    assert np.abs(parts["F_L"]).max() > 1e-3 * np.abs(F).max()


@pytest.mark.parametrize("mu", [0.0, 3e-3])
def test_flux_is_invariant_under_a_change_of_time_unit(mu):
    """With t' = s t the BGK model maps onto itself when velocities scale by
    1/s, pressure and energy by 1/s^2, mu by 1/s and tau by s; the
    time-integrated fluxes then scale as (1, 1/s, 1/s, 1/s^2).  This fixes the
    dimensions of every term, including the collision time."""
    rng = np.random.default_rng(31)
    WL, dL = random_side(rng, 4)
    WR, dR = random_side(rng, 4)
    dt = 0.01
    F = kn.gp_flux(WL, dL, WR, dR, dt, GAMMA, mu=mu)
    s = 3.0
    sc = np.array([1.0, 1 / s, 1 / s, 1 / s ** 2])[:, None]
    Fs = kn.gp_flux(sc * WL, {k: sc * v for k, v in dL.items()}, sc * WR,
                    {k: sc * v for k, v in dR.items()}, s * dt, GAMMA, mu=mu / s)
    assert np.abs(Fs - sc * F).max() < 1e-13 * np.abs(sc * F).max()


def test_viscous_shear_stress_is_navier_stokes():
    """Smooth shear U_t = s x_n across the face (same polynomial on both
    sides), tau = mu / p (Eq. tauVis with no pressure jump): the
    time-integrated tangential momentum flux is the Navier-Stokes shear
    stress -mu s dt up to O(tau / dt)."""
    rho, p, s, mu, dt = 1.0, 30.0, 0.8, 1e-3, 2e-3
    W = cons(rho, 0.0, 0.0, p)[:, None]
    d = {key: np.zeros((4, 1)) for key in ("n", "t", "nn", "nt", "tt")}
    d["n"][2, 0] = rho * s
    F = kn.gp_flux(W, d, W, d, dt, GAMMA, mu=mu)
    ref = -mu * s * dt
    assert F[2, 0] == pytest.approx(ref, rel=2e-3)
    assert abs(F[0, 0]) < 1e-15 and abs(F[3, 0]) < 1e-15
