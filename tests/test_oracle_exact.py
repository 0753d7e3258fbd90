"""Pins of the oracle's exact acoustic-pulse solution (section 4.4, Eq.
cirPulseSolution, a J0 integral evaluated by quadrature):
  * at t = 0 it is the initial Gaussian (Hankel transform of a Gaussian);
  * the plane integral of the pressure perturbation stays eps pi / alpha
    (linear acoustics with zero initial velocity conserves it);
  * it satisfies the radial wave equation p_tt = c^2 (p_rr + p_r / r) with
    c = sqrt(gamma p / rho), by central differences;
  * the tabulated spline reproduces the quadrature.
"""
import math

import numpy as np
from scipy import integrate

from oracle import exact

AMP, HW, GAMMA = 0.01, 0.04, 1.4
ALPHA = math.log(2.0) / HW ** 2


def test_initial_gaussian():
    eta = np.linspace(0.0, 0.3, 31)
    p = exact.acoustic_pulse_radial(eta, 0.0)
    assert np.abs(p - AMP * np.exp(-ALPHA * eta ** 2)).max() <= 1e-14


def test_plane_integral_is_conserved():
    eta = np.linspace(0.0, 0.75, 6001)
    for t in (0.1, 0.2):
        spl = exact.acoustic_pulse_table(t)
        val = integrate.simpson(spl(eta) * 2.0 * np.pi * eta, x=eta)
        assert abs(val - AMP * math.pi / ALPHA) <= 1e-6 * AMP * math.pi / ALPHA


def test_radial_wave_equation():
    c2 = GAMMA
    d = 2e-4
    for r, t in ((0.12, 0.08), (0.2, 0.12), (0.25, 0.15)):
        f = lambda rr, tt: exact.acoustic_pulse_radial(np.array([rr]), tt)[0]
        ptt = (f(r, t + d) - 2 * f(r, t) + f(r, t - d)) / d ** 2
        prr = (f(r + d, t) - 2 * f(r, t) + f(r - d, t)) / d ** 2
        pr = (f(r + d, t) - f(r - d, t)) / (2 * d)
        res = ptt - c2 * (prr + pr / r)
        assert abs(res) <= 2e-3 * abs(ptt) + 1e-6


def test_table_matches_quadrature():
    spl = exact.acoustic_pulse_table(0.15)
    eta = np.array([0.0, 0.033, 0.1, 0.177, 0.2501, 0.31])
    assert np.abs(spl(eta) - exact.acoustic_pulse_radial(eta, 0.15)).max() <= 1e-9 * AMP
