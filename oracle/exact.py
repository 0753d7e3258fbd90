"""Oracle: exact solutions used to measure the whole scheme's accuracy.

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and
bench.py's CPU-baseline leg, never by the library.

Acoustic pressure pulse (section 4.4, Eq. cirPulseSolution): the linear
acoustics solution of a Gaussian pressure perturbation at rest,
    p - p_inf = eps / (2 alpha) * int_0^inf exp(-xi^2 / (4 alpha))
                cos(c xi t) J0(xi eta) xi d xi,
with c the sound speed of the uniform state, evaluated by adaptive
quadrature (the J0 integral of the paper) on a table of radii and
interpolated with a cubic spline.  It is the solution of the linearised
Euler equations; the scheme solves the nonlinear ones, which differ at
O(eps^2).
"""
from __future__ import annotations

import math
import warnings

import numpy as np
from scipy import integrate, interpolate, special


def acoustic_pulse_radial(eta, t, amp=0.01, half_width=0.04, gamma=1.4, p_inf=1.0, rho_inf=1.0):
    """p - p_inf at radii eta (array) and time t, by quadrature per radius."""
    alpha = math.log(2.0) / half_width ** 2
    c = math.sqrt(gamma * p_inf / rho_inf)
    xmax = math.sqrt(4.0 * alpha * 40.0)      # exp(-40) cuts the Gaussian
    out = np.empty(np.shape(eta))
    flat = np.ravel(eta)
    res = np.empty(flat.shape)
    with warnings.catch_warnings():
        # far from the pulse the integral is ~1e-19 and quad reports round-off
        warnings.simplefilter("ignore", integrate.IntegrationWarning)
        for k, r in enumerate(flat):
            f = lambda xi: math.exp(-xi * xi / (4.0 * alpha)) * math.cos(c * xi * t) * special.j0(xi * r) * xi
            val, _ = integrate.quad(f, 0.0, xmax, limit=800, epsabs=1e-15, epsrel=1e-12)
            res[k] = amp / (2.0 * alpha) * val
    out[...] = res.reshape(np.shape(eta))
    return out


def acoustic_pulse_table(t, eta_max=0.75, n=1501, **kw):
    """Cubic spline of p - p_inf over [0, eta_max] at time t."""
    eta = np.linspace(0.0, eta_max, n)
    return interpolate.CubicSpline(eta, acoustic_pulse_radial(eta, t, **kw))


def acoustic_pulse_cell_pressure(mesh, t, center=(0.5, 0.5), p_inf=1.0, **kw):
    """Exact cell averages of the pressure at time t (8 x 8 collapsed Gauss
    rule of the input generator on the tabulated radial solution)."""
    import gks_inputs as gi
    spl = acoustic_pulse_table(t, **kw)
    cx, cy = center

    def p_fn(x, y):
        return (p_inf + spl(np.hypot(x - cx, y - cy)))[None]

    return gi.cell_average(mesh, p_fn)[0]
