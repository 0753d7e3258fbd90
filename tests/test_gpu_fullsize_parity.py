"""Multi-step parity with the oracle at the workloads' full sizes.

Each case runs the library from the workload's seeded initial state, in the
launch configuration of the benchmark (captured step graphs, multicolour
BILU(0), CFL time steps), and compares the state after the last step with
the oracle's run of the same workload.  The oracle's result (a direct CLS
solve each step) is stored in tests/golden/ by make_fullsize.py, which calls
only the oracle and the input generators; the file keeps the final state at
a seeded sample of cells joined with the cells that changed most, the full
field's maxima and area-weighted totals, and the oracle's time steps.

Cases (section 4.1 density advection, 4.6 shock-vortex, 4.7 cavity):
  512^2 density advection, 524,288 cells, 10 steps;
  1000 x 500 shock-vortex, 1,000,000 cells, 10 steps;
  250 x 125 shock-vortex (same generator and seed), 62,500 cells, 500 steps;
  256^2 lid-driven cavity, 131,072 cells, 200 steps.
Bars (relative L-inf per conserved component, tests/parity.py): FP64 form
<= 1e-12 with the GMRES tolerance at 1e-12; mixed form <= 1e-9 at the
benchmark's tolerance 1e-10.  Time steps agree to 1e-12 relative; the
area-weighted totals to 1e-12 of their scale.
"""
import os

import numpy as np
import pytest

import gks_inputs as gi
from parity import state_relinf

torch = pytest.importorskip("torch")
import paper_1802_00704_amd as g  # noqa: E402

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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


CASES = {
    "advection_512": (lambda: advection(512), {}),
    "shock_vortex_1m": (lambda: shock_vortex(1000, 500), {"nonphys_fallback": 1}),
    "shock_vortex_250x125": (lambda: shock_vortex(250, 125), {"nonphys_fallback": 1}),
    "cavity_256": (lambda: cavity(256), {"mu": 1e-3}),
}


def area(m):
    v = m.unwrapped_vertices()
    return 0.5 * ((v[:, 1, 0] - v[:, 0, 0]) * (v[:, 2, 1] - v[:, 0, 1])
                  - (v[:, 2, 0] - v[:, 0, 0]) * (v[:, 1, 1] - v[:, 0, 1]))


@pytest.mark.parametrize("form", ["fp64", "mixed"])
@pytest.mark.parametrize("name", list(CASES))
def test_fullsize_parity(name, form):
    path = os.path.join(GOLDEN, "fullsize_%s.npz" % name)
    if not os.path.exists(path):
        pytest.skip("stored oracle result %s not generated" % os.path.basename(path))
    ref = np.load(path)
    build, kw = CASES[name]
    m, W0 = build()
    assert m.nt == int(ref["nt"])
    steps = int(ref["steps"])
    print("full-size parity", name, form, m.nt, "cells", steps, "steps", flush=True)
    prec = g.GKS_FP64 if form == "fp64" else g.GKS_MIXED
    tol = 1e-12 if form == "fp64" else 1e-10
    gm = g.GksMesh(m, precision=prec, tol=tol, **kw)
    W = torch.tensor(W0, dtype=torch.float64, device="cuda")
    dts, nonphys = [], 0
    for _ in range(steps):
        dt, info = gm.step(W)
        dts.append(dt)
        nonphys += info["nonphys"]
    Wg = W.cpu().numpy()
    gm.close()
    idx = ref["idx"]
    rel = state_relinf(Wg[:, idx], ref["W"], wmax=ref["wmax"], per_component=True)
    dt_rel = float(np.max(np.abs(np.array(dts) - ref["dts"]) / ref["dts"]))
    tot = (area(m)[None] * Wg).sum(axis=1)
    scale = (area(m)[None] * np.abs(Wg)).sum(axis=1)
    tot_rel = float(np.max(np.abs(tot - ref["total"]) / scale))
    print("  relative L-inf per component", rel, "dt", dt_rel, "totals", tot_rel,
          "fallbacks", nonphys, "oracle", int(ref["nonphys"]), flush=True)
    bar = 1e-12 if form == "fp64" else 1e-9
    assert rel.max() <= bar
    assert dt_rel <= (1e-12 if form == "fp64" else 1e-9)
    assert tot_rel <= (1e-12 if form == "fp64" else 1e-9)
    assert nonphys == int(ref["nonphys"])
