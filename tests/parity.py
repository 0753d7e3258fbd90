"""Relative L-inf error of conserved states: the parity measure of the tests.

For each conserved component q the error is max_i |a_qi - ref_qi| / d_q,
with d_q the largest |ref_qi| over the cells (or the given full-field
maxima, when only a sample of cells is compared).  The two momentum
components use as d_q at least 1% of the larger of their two maxima, so a
component that the reference holds at zero up to rounding (rho v in a
one-dimensional problem) is measured against the flow's momentum scale
rather than against its own rounding noise.  The result is the maximum over
the four components.
"""
import numpy as np

MOMENTUM_FLOOR = 0.01


def denominators(ref, wmax=None):
    d = np.abs(np.asarray(ref)).reshape(4, -1).max(axis=1) if wmax is None else np.asarray(wmax, dtype=float).copy()
    mom = max(d[1], d[2])
    d[1] = max(d[1], MOMENTUM_FLOOR * mom)
    d[2] = max(d[2], MOMENTUM_FLOOR * mom)
    return d


def state_relinf(a, ref, wmax=None, per_component=False):
    a = np.asarray(a).reshape(4, -1)
    ref = np.asarray(ref).reshape(4, -1)
    d = denominators(ref, wmax)
    errs = np.array([np.abs(a[q] - ref[q]).max() / d[q] if d[q] > 0 else np.abs(a[q] - ref[q]).max()
                     for q in range(4)])
    return errs if per_component else float(errs.max())
