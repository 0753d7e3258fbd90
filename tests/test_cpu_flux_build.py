"""The library's Gauss-point flux code compiled for the CPU (with address and
undefined-behaviour sanitizers) against the oracle, on seeded states: catches
indexing and formula errors in the device code without a GPU."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import kinetic as kn

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cpu_build", "gp_flux_cpu.cpp")
EXE = os.path.join(HERE, "cpu_build", "_gp_flux_cpu")
CLANG = "/opt/rocm/llvm/bin/clang++"


@pytest.fixture(scope="module")
def exe():
    if not os.path.exists(CLANG):
        pytest.skip("clang++ of ROCm not available")
    dep = os.path.join(HERE, "..", "paper_1802_00704_amd", "csrc", "gks_flux_device.h")
    if (not os.path.exists(EXE) or os.path.getmtime(EXE) < max(os.path.getmtime(SRC), os.path.getmtime(dep))):
        san = "-fsanitize=" + "address,undefined"
        cmd = [CLANG, "-x", "c++", "-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
               san, "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", SRC, "-o", EXE + ".tmp%d" % os.getpid()]
        subprocess.run(cmd, check=True)
        shutil.move(EXE + ".tmp%d" % os.getpid(), EXE)
    return EXE


def cons(rho, u, v, p, gamma=1.4):
    return np.array([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


def sides(rng, m, scale):
    W = np.stack([cons(rng.uniform(0.6, 1.4), rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0.6, 1.4))
                  for _ in range(m)], axis=1)
    d = {k: scale * rng.normal(size=(4, m)) for k in ("n", "t", "nn", "nt", "tt")}
    return W, d


def run_cpu(exe, WL, dL, WR, dR, dt, gamma=1.4, mu=0.0, eps=0.01, exact=0):
    m = WL.shape[1]
    keys = ("n", "t", "nn", "nt", "tt")
    rows = [np.concatenate([WL[:, i]] + [dL[k][:, i] for k in keys] + [WR[:, i]] + [dR[k][:, i] for k in keys])
            for i in range(m)]
    payload = (np.array([m, exact], dtype="<i4").tobytes() + np.array([gamma, mu, eps, dt], dtype="<f8").tobytes()
               + np.array(rows, dtype="<f8").tobytes())
    out = subprocess.run([exe], input=payload, capture_output=True, check=True).stdout
    return np.frombuffer(out, dtype="<f8").reshape(m, 4).T


@pytest.mark.parametrize("mu,eps,exact,scale", [(0.0, 0.01, 0, 0.05), (0.0, 0.3, 0, 0.5), (2e-3, 0.01, 1, 0.2),
                                                (0.0, 0.01, 1, 1.0)])
def test_cpu_build_of_device_flux_matches_oracle(exe, mu, eps, exact, scale):
    rng = np.random.default_rng(int(1000 * scale) + exact)
    m = 64
    WL, dL = sides(rng, m, scale)
    WR, dR = sides(rng, m, scale)
    dt = 0.01
    ref = kn.gp_flux(WL, dL, WR, dR, dt, 1.4, mu=mu, eps=eps, exact_time=bool(exact))
    got = run_cpu(exe, WL, dL, WR, dR, dt, mu=mu, eps=eps, exact=exact)
    for q in range(4):
        assert np.abs(got[q] - ref[q]).max() <= 1e-13 * np.abs(ref[q]).max(), q
