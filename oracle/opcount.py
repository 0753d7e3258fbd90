"""Operation count of the oracle's third-order flux at one Gauss point.

TEST AND MEASUREMENT INFRASTRUCTURE ONLY: run by hand to fix the flux's
algorithmic FLOP count F_G (the FP64 operations the method performs per
Gauss point as the oracle writes it out, section 2.2: moments, slope
inversions, time integrals, polynomial contractions); the library never
imports it.  The figure is stored, with the command that produced it, in
profiles/gks_flux_opcount.txt, and the benchmark reads it from there.

Method: the oracle's gp_flux runs on arrays of a counting ndarray subclass.
Every numpy ufunc it calls (arithmetic, sqrt, exp, scipy's erfc, and the
4 x 4 solve gufunc of its slope inversions) is intercepted and charged per
output element:
  * add, subtract, multiply, divide, sqrt, absolute, hypot, maximum,
    minimum: 1 FLOP each; power by 2 or 3: 1 or 2 FLOPs;
  * exp, erfc: counted apart as transcendentals;
  * each slope inversion (kinetic.slope, the 4 x 4 moment system): its
    right-hand side as the oracle forms it, the moment matrix of its
    Maxwellian once per Maxwellian (the oracle rebuilds it on every call:
    three Maxwellians serve the 25 inversions of a Gauss point), and 62
    FLOPs for the solve with one right-hand side (LU without pivoting 34,
    forward substitution 12, back substitution 16);
  * operations the dictionary form of the velocity polynomials adds but the
    method does not have are free: multiplying or dividing by a literal 1
    or -1, multiplying by a literal 0, adding or subtracting a literal 0,
    negation.
Usage: python -m oracle.opcount
"""
from __future__ import annotations

import numpy as np
from . import kinetic

FREE_SCALARS_MUL = (1.0, -1.0)


class Tally:
    flops = 0
    trans = 0
    solves = 0
    by_ufunc: dict = {}


def _is_literal(x, values):
    if isinstance(x, np.ndarray) and x.ndim > 0:
        return False
    try:
        v = float(np.asarray(x))
    except (TypeError, ValueError):
        return False
    return v in values


class Counted(np.ndarray):
    """ndarray whose ufunc calls are charged to Tally."""

    def __array_ufunc__(self, ufunc, method, *inputs, **kwargs):
        raw = [np.asarray(x).view(np.ndarray) if isinstance(x, Counted) else x for x in inputs]
        if "out" in kwargs:
            kwargs["out"] = tuple(np.asarray(o).view(np.ndarray) if isinstance(o, Counted) else o
                                  for o in kwargs["out"])
        res = getattr(ufunc, method)(*raw, **kwargs)
        size = int(np.size(res[0] if isinstance(res, tuple) else res))
        name = ufunc.__name__
        cost, trans = 0, 0
        if name in ("add", "subtract"):
            cost = 0 if any(_is_literal(x, (0.0,)) for x in raw) else 1
        elif name == "multiply":
            cost = 0 if any(_is_literal(x, FREE_SCALARS_MUL + (0.0,)) for x in raw) else 1
        elif name in ("divide", "true_divide"):
            cost = 0 if _is_literal(raw[1], FREE_SCALARS_MUL) else 1
        elif name in ("sqrt", "absolute", "hypot", "maximum", "minimum", "square", "reciprocal"):
            cost = 1
        elif name == "power":
            e = float(np.asarray(raw[1]))
            cost = {1.0: 0, 2.0: 1, 3.0: 2}.get(e, 1)
        elif name in ("exp", "erfc"):
            trans = 1
        elif name in ("negative", "positive"):
            cost = 0
        elif name.startswith("solve"):
            # gufunc over [..., 4, 4] x [..., 4, 1]: size counts the outputs
            n_sys = size // 4
            cost = 62
            size = n_sys
            Tally.solves += n_sys
        else:
            raise NotImplementedError("uncounted ufunc %s" % name)
        Tally.flops += cost * size
        Tally.trans += trans * size
        Tally.by_ufunc[name] = Tally.by_ufunc.get(name, 0) + (cost + trans) * size
        if isinstance(res, tuple):
            return tuple(np.asarray(r).view(Counted) for r in res)
        return np.asarray(res).view(Counted)


def count(ng: int = 16, seed: int = 3, mu: float = 0.0):
    """(FLOPs, transcendentals, 4x4 solves) per Gauss point of kinetic.gp_flux
    on ng random physical Gauss-point pairs."""
    rng = np.random.default_rng(seed)

    def state():
        rho = rng.uniform(0.8, 1.2, ng)
        u = rng.uniform(-0.5, 0.5, ng)
        v = rng.uniform(-0.5, 0.5, ng)
        p = rng.uniform(0.8, 1.2, ng)
        return np.stack([rho, rho * u, rho * v, p / 0.4 + 0.5 * rho * (u * u + v * v)])

    def derivs():
        return {k: 0.05 * rng.standard_normal((4, ng)) for k in ("n", "t", "nn", "nt", "tt")}

    WL, WR, dL, dR = state(), state(), derivs(), derivs()
    c = lambda a: np.asarray(a).view(Counted)
    Tally.flops = Tally.trans = Tally.solves = 0
    Tally.by_ufunc = {}
    matrices = {}

    def slope_once(W, mom_full, D):
        # the oracle's kinetic.slope with its moment matrix built once per
        # Maxwellian (the same numbers; the counted solve is charged below)
        key = id(mom_full)
        if key not in matrices:
            rho = W[0]
            M = np.empty(D.shape[1:] + (4, 4))
            for al in range(4):
                for be in range(4):
                    M[..., al, be] = np.asarray(rho * kinetic.expect(kinetic.poly_mul(kinetic.PSI[al],
                                                                                      kinetic.PSI[be]), mom_full))
            matrices[key] = (mom_full, M)
        M = matrices[key][1]
        Tally.solves += ng
        Tally.flops += 62 * ng
        Tally.by_ufunc["solve4x4"] = Tally.by_ufunc.get("solve4x4", 0) + 62 * ng
        rhs = np.moveaxis(np.asarray(D).view(np.ndarray), 0, -1)[..., None]
        return np.linalg.solve(M, rhs)[..., 0].T.view(Counted)

    orig = kinetic.slope
    kinetic.slope = slope_once
    try:
        F = kinetic.gp_flux(c(WL), {k: c(v) for k, v in dL.items()}, c(WR), {k: c(v) for k, v in dR.items()},
                            c(np.full(ng, 1e-3)), 1.4, mu, 0.01)
    finally:
        kinetic.slope = orig
    ref = kinetic.gp_flux(WL, dL, WR, dR, np.full(ng, 1e-3), 1.4, mu, 0.01)
    assert np.array_equal(np.asarray(F), ref), "the counting run must compute the same flux"
    return Tally.flops / ng, Tally.trans / ng, Tally.solves / ng, {k: v / ng for k, v in Tally.by_ufunc.items()}


if __name__ == "__main__":
    for mu in (0.0, 1e-3):
        fl, tr, sv, by = count(mu=mu)
        print("mu=%g: %.0f FP64 FLOP per Gauss point, %.0f transcendentals (exp, erfc), %.0f 4x4 solves"
              % (mu, fl, tr, sv))
        print("   by operation:", {k: round(v) for k, v in sorted(by.items(), key=lambda kv: -kv[1])})
