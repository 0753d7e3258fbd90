"""Host-side pieces of bench.py (no GPU): the one-GPU guard, the parsing of
the committed counter summaries under profiles/, and the roofline
arithmetic on a synthetic event profile."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    return b


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one MI355X" in r.stderr


def test_committed_summaries_parse():
    from paper_1802_00704_amd.profiling import read_summary
    b = load_bench()
    sha, traffic = read_summary(b.TRAFFIC_SUMMARY)
    assert len(sha) == 64 and traffic["ilu_fwd32"] > 0 and traffic["flux"] > 0
    sha2, flops = read_summary(b.FP64_SUMMARY, column=2, ncols=8)
    assert len(sha2) == 64
    # one thread per Gauss point: 10^3..10^5 FP64 FLOPs each at 3,003,000 points
    assert 3.003e9 < flops["flux"] < 3.003e11


def test_stale_summaries_are_not_used(monkeypatch):
    import paper_1802_00704_amd.profiling as prof
    b = load_bench()
    monkeypatch.setattr(prof, "kernel_sources_sha256", lambda: "0" * 64)
    assert b.measured_traffic("ilu_fwd32") is None
    assert b.measured_flops("flux") is None


def test_roofline_arithmetic(monkeypatch):
    b = load_bench()
    monkeypatch.setattr(b, "measured_traffic", lambda cls: None)
    monkeypatch.setattr(b, "measured_flops", lambda cls: 3.2e10)
    prof = {"ilu_fwd32": {"ms": 6.0, "launches": 100, "bytes": 100 * 2.4e8},
            "flux": {"ms": 2.4, "launches": 3, "bytes": 3 * 9e8}}
    r = b.roofline(prof, 0.01, 3_000_000)
    assert r["kernel"] == "ilu_fwd32" and r["unit"] == "GB/s" and r["bound"] == "hbm"
    assert r["achieved"] == pytest.approx(2.4e8 / 60e-6 / 1e9, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, rel=1e-3)
    assert r["traffic"] is None
    f = b.flux_fp64(prof, 3_000_000)
    assert f["achieved"] == pytest.approx(3.2e10 / 0.8e-3 / 1e12, rel=1e-3)
    assert f["frac"] == pytest.approx(f["achieved"] / 78.6, rel=1e-3)
    assert f["executed_flop_per_gauss_point"] == pytest.approx(3.2e10 / 3e6, rel=1e-3)
    fg = b.algorithmic_flux_flops()
    assert fg and f["algorithmic_rate_TFLOPs"] == pytest.approx(fg * 3e6 / 0.8e-3 / 1e12, rel=1e-3)


def test_roofline_of_the_flux_when_it_dominates(monkeypatch):
    """The FP64-bound flux is priced on its executed FP64 FLOPs against the
    FP64 vector peak, with the method's term-by-term count beside them; with
    a stale counter summary it reports no fraction."""
    b = load_bench()
    monkeypatch.setattr(b, "measured_flops", lambda cls: 3.2e10)
    prof = {"ilu_fwd32": {"ms": 2.0, "launches": 100, "bytes": 100 * 2.4e8},
            "flux": {"ms": 2.4, "launches": 3, "bytes": 3 * 9e8}}
    r = b.roofline(prof, 0.01, 3_000_000)
    fg = b.algorithmic_flux_flops()
    assert r["kernel"] == "flux" and r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == 78.6
    assert r["achieved"] == pytest.approx(3.2e10 / 0.8e-3 / 1e12, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / 78.6, rel=1e-3)
    assert r["method_rate_TFLOPs"] == pytest.approx(fg * 3e6 / 0.8e-3 / 1e12, rel=1e-3)
    monkeypatch.setattr(b, "measured_flops", lambda cls: None)
    r = b.roofline(prof, 0.01, 3_000_000)
    assert r["achieved"] is None and r["frac"] is None
