"""Serving on the GPU: the same requests run alone (one at a time) and in
the mix (admitted concurrently on separate streams) give the same states;
each result also matches a plain single-handle run; and the handle's real
device memory stays within the admission estimate."""
import numpy as np
import pytest

import gks_inputs as gi

torch = pytest.importorskip("torch")
import paper_1802_00704_amd as g  # noqa: E402
from paper_1802_00704_amd.serving import Request, Server, estimate_footprint  # noqa: E402

pytestmark = pytest.mark.gpu


def make_requests():
    specs = gi.serving_specs(6, rate=1000.0, seed=11, nt_range=(2e3, 8e3), steps_range=(4, 9))
    reqs = []
    for sp in specs:
        m, W0 = gi.serving_case(sp)
        prm = {"precision": g.GKS_MIXED if sp["mixed"] else g.GKS_FP64, "nonphys_fallback": 1}
        reqs.append(Request(rid=sp["rid"], mesh=m, W0=W0, steps=sp["steps"], params=prm, arrival=sp["arrival"]))
    return reqs


def test_alone_equals_mix():
    alone = make_requests()
    Server(slots=1, hbm_budget=1 << 36).run(alone, realtime=False)
    mix = make_requests()
    stats = Server(slots=6, hbm_budget=1 << 36).run(mix, realtime=True)
    assert stats["completed"] == len(mix)
    assert stats["peak_concurrent"] >= 2
    # every step of the concurrent mix replayed its captured graphs
    assert stats["capture_failures"] == 0
    assert stats["graph_steps"] == sum(r.steps for r in mix)
    for a, b in zip(alone, mix):
        assert a.error is None and b.error is None, (a.error, b.error)
        assert np.array_equal(a.W, b.W), a.rid


def test_served_result_matches_direct_run():
    req = make_requests()[0]
    Server(slots=2, hbm_budget=1 << 36).run([req], realtime=False)
    gm = g.GksMesh(req.mesh, g.default_params(**req.params))
    W = torch.tensor(req.W0, device="cuda")
    for _ in range(req.steps):
        gm.step(W)
    assert np.array_equal(W.cpu().numpy(), req.W)


@pytest.mark.parametrize("precision", [0, 1])
def test_footprint_estimate_bounds_real_allocation(precision):
    m, _ = gi.serving_case({"kind": "shock_vortex", "nt": 20000, "seed": 3})
    gm = g.GksMesh(m, precision=precision)
    real = gm.stats()["device_bytes"]
    est = estimate_footprint(m.nt, precision)
    assert real <= est <= 1.6 * real
