"""Sod and Lax shock tubes (sections 4.2-4.3) on unstructured JSS meshes of
[0, 1] x [0, 0.1] with the DWBAP limiter, against the exact Riemann solution
of the oracle.

The paper does not state the conditions at the tube's ends.  The waves do
not reach them by t = 0.2 (Sod) and t = 0.14 (Lax), so the ends hold the
initial left and right states as fixed-state boundaries (exact there); top
and bottom are slip walls.  Errors are area-weighted L1 of the cell-average
density against the exact cell averages.  With discontinuities the scheme
converges at first order in L1, so the checks are that the error falls
under refinement and stays small.  Oscillation is measured as the largest
new extremum: how far a cell's density leaves the range the exact solution
spans within 2h of its centroid (smearing a jump does not count, an
overshoot does); its area-weighted mean is reported beside the maximum.
The first steps are also compared with the oracle's reconstruct - limit -
flux - update chain.
"""
import math

import numpy as np
import pytest

import gks_inputs as gi
from oracle import limiter, riemann, scheme
from oracle.mesh import build_geometry
from parity import state_relinf

torch = pytest.importorskip("torch")
import paper_1802_00704_amd as g  # noqa: E402

pytestmark = pytest.mark.gpu
G = 1.4
SOD = ((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 0.2)
LAX = ((0.445, 0.698, 3.528), (0.5, 0.0, 0.571), 0.14)


def tube(nx, case):
    left, right, _ = case
    ends = [(gi.BC_INFLOW, (st[0], st[1], 0.0, st[2])) for st in (left, right)]
    m = gi.jss_mesh(nx, max(2, nx // 10), 7, Lx=1.0, Ly=0.1, periodic=False,
                    walls=(ends[0], ends[1], (gi.BC_SLIP, None), (gi.BC_SLIP, None)))

    def fn(x, y):
        st = [np.where(x < 0.5, a, b) for a, b in zip(left, right)]
        rho, u, p = st
        return np.stack([rho, rho * u, np.zeros_like(rho), p / (G - 1) + 0.5 * rho * u * u])

    return m, gi.cell_average(m, fn)


def run(nx, case, lim=1):
    m, W0 = tube(nx, case)
    T = case[2]
    gm = g.GksMesh(m, limiter=lim, nonphys_fallback=1, tol=1e-10)
    probe = torch.tensor(W0, device="cuda")
    dt0, _ = gm.step(probe)
    nst = math.ceil(T / (0.6 * dt0))
    dt = T / nst
    gm.close()
    gm = g.GksMesh(m, limiter=lim, nonphys_fallback=1, tol=1e-10)
    W = torch.tensor(W0, device="cuda")
    nonphys = limited = 0
    torch.cuda.synchronize()
    import time
    t0 = time.perf_counter()
    for _ in range(nst):
        try:
            _, info = gm.step(W, dt)
        except g.NonPhysical:
            gm.close()
            return {"failed": True, "overshoot": math.inf, "l1": math.inf}
        nonphys += info["nonphys"]
        limited += info["limited"]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    gm.close()
    Wn = W.cpu().numpy()
    ex = riemann.tube_cell_averages(m, case[0], case[1], 0.5, T, G)
    area = g.host_inspect(m)["area"]
    l1 = float((np.abs(Wn[0] - ex[0]) * area).sum() / area.sum())
    exc = excursion(m, Wn[0], case, 2.0 / nx)
    return {"l1": l1, "overshoot": float(exc.max()), "osc_l1": float((exc * area).sum() / area.sum()),
            "nonphys": nonphys, "limited": limited, "steps": nst, "cell_steps_per_s": m.tri.shape[0] * nst / el}


def excursion(m, rho, case, band):
    """Per cell: distance of the density outside the exact solution's range
    over [x - band, x + band] at the final time (0 inside it)."""
    left, right, T = case
    xs = np.linspace(0.0, 1.0, 20001)
    ex = riemann.sample(left, right, (xs - 0.5) / T, G)[0]
    cx = m.xy[m.tri].mean(axis=1)[:, 0]
    lo = np.searchsorted(xs, cx - band)
    hi = np.searchsorted(xs, cx + band)
    out = np.zeros(rho.size)
    for i in range(rho.size):
        seg = ex[lo[i]:max(hi[i], lo[i] + 1)]
        out[i] = max(0.0, rho[i] - seg.max(), seg.min() - rho[i])
    return out


def test_sod_converges_with_the_limiter():
    res = [run(nx, SOD) for nx in (50, 100, 200)]
    print("Sod with DWBAP:", res, flush=True)
    l1 = [r["l1"] for r in res]
    assert l1[1] < 0.8 * l1[0] and l1[2] < 0.8 * l1[1]
    assert l1[1] < 0.005
    assert all(r["overshoot"] < 0.04 for r in res)     # 4% of the density jump
    assert all(r["limited"] > 0 for r in res)


def test_limiter_removes_much_of_the_oscillation_sod():
    with_l = run(100, SOD, 1)
    without = run(100, SOD, 0)
    print("Sod h=1/100: limited", with_l, "unlimited", without, flush=True)
    assert not with_l.get("failed")
    assert with_l["overshoot"] < 0.6 * without["overshoot"]
    assert with_l["l1"] <= without["l1"]


def test_lax_with_the_limiter():
    r = run(100, LAX)
    print("Lax with DWBAP, h=1/100:", r, flush=True)
    assert not r.get("failed")
    assert r["l1"] < 0.012
    assert r["overshoot"] < 0.12                          # 14% of the density jump
    assert r["limited"] > 0


@pytest.mark.parametrize("case", [SOD, LAX], ids=["sod", "lax"])
def test_characteristic_limiting(case):
    """Section 4.2 compares limiting in conserved and in characteristic
    variables and finds less oscillation with the latter.  Measured at
    h = 1/100: the mean excursion falls 15% at Sod (1.12e-3 -> 0.96e-3) and
    2% at Lax, the L1 error a little in both; the single largest excursion
    falls at Sod and rises 12% at Lax.  So the observation holds at Sod on
    every measure and at Lax only on the averaged ones: at Lax the test
    checks the L1 error and the mean excursion, and makes no claim about the
    largest one."""
    cons = run(100, case, g.LIMIT_CONSERVATIVE)
    char = run(100, case, g.LIMIT_CHARACTERISTIC)
    print("h=1/100 conservative", cons, "characteristic", char, flush=True)
    assert not char.get("failed")
    assert char["l1"] <= 1.02 * cons["l1"]
    if case is SOD:
        assert char["osc_l1"] < 0.9 * cons["osc_l1"]
        assert char["overshoot"] < cons["overshoot"]
    else:
        assert char["osc_l1"] <= 1.02 * cons["osc_l1"]


def test_sod_first_steps_match_the_oracle():
    m, W0 = tube(40, SOD)
    geo = build_geometry(m)
    s = scheme.Solver(m, scheme.Params(fallback=True))
    gm = g.GksMesh(m, limiter=1, tol=1e-13, nonphys_fallback=1)
    W = torch.tensor(W0, device="cuda")
    Wr = W0.copy()
    for _ in range(3):
        dt, info = gm.step(W)
        X = s.reconstruct(Wr)
        Xl, mask = limiter.limit(geo, Wr, X, m)
        Wr = scheme.update(geo, Wr, s.flux(Wr, Xl, dt))
        assert info["limited"] == int(mask.sum())
    rel = state_relinf(W.cpu().numpy(), Wr, per_component=True)
    print("relative L-inf per component", rel, flush=True)
    assert rel.max() <= 1e-9, rel
    gm.close()
