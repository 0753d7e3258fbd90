"""Write the stored oracle results of the full-size multi-step parity tests.

Calls only the oracle (``oracle/``) and the seeded input generators
(``gks_inputs``): each workload is run from its initial state with the
oracle's direct CLS solve, its CFL time step and its flux, for the stated
number of steps, and the result is stored as

    idx      cells whose final state is kept (all cells, or a seeded sample
             joined with the cells that changed most)
    W        [4, len(idx)] final cell averages at those cells
    dts      [steps] the oracle's time steps
    wmax     [4] max |W_final| over every cell, per component
    total    [4] sum over every cell of area * W_final
    nonphys  Gauss-point fallbacks (reading R18) met over the run

Usage: python tests/golden/make_fullsize.py NAME [NAME ...]
       (NAME in advection_512, shock_vortex_1m, shock_vortex_250x125, cavity_256)
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import gks_inputs as gi  # noqa: E402
from oracle import scheme  # noqa: E402

SAMPLE = 32768       # cells kept when the mesh is larger than this
ACTIVE = 8192        # of which the cells whose state changed most


def shock_vortex(nx, ny):
    left, _ = gi.shock_vortex_states()
    walls = ((gi.BC_INFLOW, left), (gi.BC_OUTFLOW, None), (gi.BC_SLIP, None), (gi.BC_SLIP, None))
    m = gi.jss_mesh(nx, ny, 3, Lx=2.0, Ly=1.0, periodic=False, walls=walls)
    return m, gi.shock_vortex_ic(m)


def cavity(n):
    walls = ((gi.BC_NOSLIP, (0.0, 0.0, 0.0, 0.0)),) * 3 + ((gi.BC_NOSLIP, (0.0, 1.0, 0.0, 0.0)),)
    m = gi.jss_mesh(n, n, 4, Lx=1.0, Ly=1.0, periodic=False, stretch=1.5, walls=walls)
    return m, gi.cavity_ic(m)


def advection(n):
    m = gi.jss_mesh(n, n, 2)
    return m, gi.density_advection_ic(m)


# name -> (mesh and initial state, oracle parameters, steps)
CASES = {
    "advection_512": (lambda: advection(512), dict(), 10),
    "shock_vortex_1m": (lambda: shock_vortex(1000, 500), dict(fallback=True), 10),
    "shock_vortex_250x125": (lambda: shock_vortex(250, 125), dict(fallback=True), 500),
    "cavity_256": (lambda: cavity(256), dict(mu=1e-3), 200),
}


def path(name):
    return os.path.join(HERE, "fullsize_%s.npz" % name)


def make(name):
    build, prm, steps = CASES[name]
    m, W0 = build()
    t0 = time.perf_counter()
    s = scheme.Solver(m, scheme.Params(**prm))
    W = W0
    dts = []
    for k in range(steps):
        W, dt = s.step(W)
        dts.append(dt)
        if k % 10 == 0 or k == steps - 1:
            print("%s: step %d/%d, dt %.6e, %.0f s" % (name, k + 1, steps, dt, time.perf_counter() - t0),
                  flush=True)
    nt = m.nt
    if nt <= SAMPLE:
        idx = np.arange(nt)
    else:
        wmax0 = np.abs(W0).max(axis=1)
        change = (np.abs(W - W0) / wmax0[:, None]).max(axis=0)
        active = np.argsort(-change, kind="stable")[:ACTIVE]
        rng = np.random.Generator(np.random.PCG64(2024))
        rest = np.setdiff1d(np.arange(nt), active)
        idx = np.sort(np.concatenate([active, rng.choice(rest, SAMPLE - ACTIVE, replace=False)]))
    np.savez_compressed(path(name), idx=idx.astype(np.int32), W=W[:, idx], dts=np.array(dts),
                        wmax=np.abs(W).max(axis=1), total=(s.geo.area[None] * W).sum(axis=1),
                        nonphys=np.int64(s.counters.get("nonphys", 0)), steps=np.int64(steps), nt=np.int64(nt))
    print("%s: wrote %s (%d cells kept) in %.0f s" % (name, path(name), idx.size, time.perf_counter() - t0),
          flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or list(CASES)
    for n in names:
        if n not in CASES:
            raise SystemExit("unknown case %r" % n)
        make(n)
