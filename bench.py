"""Throughput benchmark of the third-order gas-kinetic step on one MI355X.

One step = CFL time step + CLS reconstruction solve (to relative residual
1e-10) + Gauss-point BGK fluxes + finite-volume update, i.e. one pass of
the whole hot path, on seeded synthetic input already resident in HBM.

Default workload: the shock-vortex interaction on the jittered split-square
mesh of 1000 x 500 squares on [0, 2] x [0, 1] (1,000,000 triangles), run in
the mixed form (FP64 flexible GMRES with FP32 inner BILU(0)/SpMV sweeps) and
in the plain FP64 form.  The headline value is the mixed form's
cell-steps/s; the FP64 form is reported beside it.

Prints ONE JSON line.  The value is timed over the K steps without
instrumentation.  The roofline entry is for the kernel class with the
largest share of kernel time, whose launch durations are measured with HIP
event pairs on the library's stream over K further steps of the same run;
its traffic comes from the committed counter summary when the kernel sources
still match it.  The CPU baseline is the oracle on a bounded sample of the
same workload family.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-steps/s at 1M tris, mixed vs FP64 at resid 1e-10; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector peak
FP64_VALU_PEAK_TFLOPS = 78.6


def workload(name: str):
    import gks_inputs as gi
    if name == "shock_vortex_1m":
        left, _ = gi.shock_vortex_states()
        walls = ((gi.BC_INFLOW, left), (gi.BC_OUTFLOW, None), (gi.BC_SLIP, None), (gi.BC_SLIP, None))
        m = gi.jss_mesh(1000, 500, 3, Lx=2.0, Ly=1.0, periodic=False, walls=walls)
        W = gi.shock_vortex_ic(m)
        desc = ("shock-vortex (Ma 1.1 stationary shock, vortex 0.3/0.05), JSS 1000x500 on [0,2]x[0,1], "
                "1,000,000 triangles, inviscid, CFL 0.5, CLS tol 1e-10")
        return m, W, desc, {}
    if name == "advection_512":
        m = gi.jss_mesh(512, 512, 2)
        W = gi.density_advection_ic(m)
        desc = "density advection, periodic JSS 512x512 on [0,2]^2, 524,288 triangles, CFL 0.5, CLS tol 1e-10"
        return m, W, desc, {}
    if name == "acoustic_pulse_1m":
        m = gi.jss_mesh(708, 708, 6, Lx=1.0, Ly=1.0)
        W = gi.acoustic_pulse_ic(m)
        desc = ("acoustic pressure pulse (amplitude 0.01, half width 0.04), periodic JSS 708x708 on [0,1]^2, "
                "1,002,528 triangles, CFL 0.5, CLS tol 1e-10")
        return m, W, desc, {}
    if name == "cavity_256":
        walls = ((gi.BC_NOSLIP, (0.0, 0.0, 0.0, 0.0)),) * 3 + ((gi.BC_NOSLIP, (0.0, 1.0, 0.0, 0.0)),)
        m = gi.jss_mesh(256, 256, 4, Lx=1.0, Ly=1.0, periodic=False, stretch=1.5, walls=walls)
        W = gi.cavity_ic(m)
        desc = ("lid-driven cavity (lid u = 1, Ma 0.15, Re 1000: mu 1e-3, viscous collision time), JSS 256x256 "
                "tanh-clustered (1.5) on [0,1]^2, 131,072 triangles, CFL 0.5, CLS tol 1e-10")
        return m, W, desc, {"mu": 1e-3}
    raise SystemExit("unknown workload %r" % name)


def host_cpu() -> dict:
    """Host CPU model and the cores this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        usable = os.cpu_count()
    return {"model": model, "nproc": usable, "os_cpu_count": os.cpu_count()}


def _oracle_sample(name: str):
    import gks_inputs as gi
    from oracle import scheme
    if name == "shock_vortex_1m":
        left, _ = gi.shock_vortex_states()
        walls = ((gi.BC_INFLOW, left), (gi.BC_OUTFLOW, None), (gi.BC_SLIP, None), (gi.BC_SLIP, None))
        m = gi.jss_mesh(100, 50, 3, Lx=2.0, Ly=1.0, periodic=False, walls=walls)
        W = gi.shock_vortex_ic(m)
        sample = "shock-vortex JSS 100x50 (10,000 triangles), same family at 10x coarser h"
        prm = scheme.Params(fallback=True)
    elif name == "acoustic_pulse_1m":
        m = gi.jss_mesh(71, 71, 6, Lx=1.0, Ly=1.0)
        W = gi.acoustic_pulse_ic(m)
        sample = "acoustic pulse JSS 71x71 (10,082 triangles), same family at 10x coarser h"
        prm = scheme.Params()
    elif name == "cavity_256":
        walls = ((gi.BC_NOSLIP, (0.0, 0.0, 0.0, 0.0)),) * 3 + ((gi.BC_NOSLIP, (0.0, 1.0, 0.0, 0.0)),)
        m = gi.jss_mesh(64, 64, 4, Lx=1.0, Ly=1.0, periodic=False, stretch=1.5, walls=walls)
        W = gi.cavity_ic(m)
        sample = "lid-driven cavity JSS 64x64 tanh-clustered (8,192 triangles), same family at 4x coarser h"
        prm = scheme.Params(mu=1e-3)
    else:
        m = gi.jss_mesh(64, 64, 2)
        W = gi.density_advection_ic(m)
        sample = "density advection JSS 64x64 (8,192 triangles)"
        prm = scheme.Params()
    return m, W, sample, prm


def oracle_worker(name: str, budget_s: float):
    """One single-threaded oracle run on the bounded sample: (cells, steps,
    seconds, sample text).  Runs in the parent or in a pool worker."""
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    from oracle import scheme
    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    m, W, sample, prm = _oracle_sample(name)
    s = scheme.Solver(m, prm)
    s.step(W)  # factorisation of the CLS matrix (setup, not timed)
    steps = 0
    t0 = time.perf_counter()
    while True:
        W, _ = s.step(W)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= 200:
            break
    del ctx
    return m.nt, steps, el, sample


def cpu_baseline(name: str, budget_s: float = 12.0) -> dict:
    """The oracle (plain FP64 NumPy/SciPy) on a bounded sample: the same
    workload family on a smaller mesh, timed over whole steps, on one core
    and on every usable host core (one single-threaded oracle process per
    core, each on its own copy of the sample; the aggregate is reported).
    Runs before the GPU is touched."""
    import concurrent.futures as cf
    import multiprocessing as mp
    cpu = host_cpu()
    nt, steps, el, sample = oracle_worker(name, budget_s)
    one = nt * steps / el
    workers = max(1, min(16, cpu["nproc"] or 1))
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        res = list(ex.map(oracle_worker, [name] * workers, [budget_s] * workers))
    allc = sum(r[0] * r[1] / r[2] for r in res)
    return {"value": one, "unit": "cell-steps/s", "cores": 1, "kind": "oracle",
            "sample": "%s, %d steps in %.1f s on one core" % (sample, steps, el),
            "all_cores": {"value": allc, "unit": "cell-steps/s", "cores": workers,
                          "sample": "%d single-threaded oracle processes, one per core, each on the same sample"
                                    % workers},
            "host_cpu": cpu}


def run_form(m, W0, precision: int, steps: int, warmup: int, profile: bool, graphs: int = 1, limiter: int = 0,
             extra: dict | None = None, late_at: int = 0):
    import torch
    import paper_1802_00704_amd as g
    t0 = time.perf_counter()
    gm = g.GksMesh(m, tol=1e-10, precision=precision, nonphys_fallback=1, graphs=graphs, limiter=limiter,
                   **(extra or {}))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    W = torch.tensor(W0, dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        gm.step(W)
    torch.cuda.synchronize()
    lat = []
    iters = []
    first = []
    r0 = []
    limited = []
    nonphys = []
    pts = []
    st0 = gm.stats()
    # as timeit does, no garbage collection inside the timed steps
    gc.collect()
    gc.disable()
    t_start = time.perf_counter()
    for _ in range(steps):
        t = time.perf_counter()
        used, info = gm.step(W)
        lat.append(time.perf_counter() - t)
        pts.append(info["start_points"])
        iters.append(max(info["iters"]))
        first.append(info["first_sweeps"])
        r0.append(info["start_resid"])
        limited.append(info["limited"])
        nonphys.append(info["nonphys"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    gc.enable()
    st1 = gm.stats()
    slow = int(np.argmax(lat))
    window = {"graph_captures": st1["graph_captures"] - st0["graph_captures"],
              "capture_ms": st1["capture_ms"] - st0["capture_ms"],
              "slowest_step": {"index": warmup + 1 + slow, "ms": lat[slow] * 1e3, "outer": iters[slow],
                               "first_sweeps": first[slow], "start_points": pts[slow]}}
    done = warmup + steps
    # Kernel durations: the same number of steps again, right after the timed
    # ones (so that they solve alike), with a HIP event pair around every
    # launch on the library's stream (events add host latency between
    # launches, so these steps are not part of the timed value).
    prof, prof_elapsed = {}, 0.0
    if profile:
        gm.profile(True)
        t_p = time.perf_counter()
        for _ in range(steps):
            gm.step(W)
        torch.cuda.synchronize()
        prof_elapsed = time.perf_counter() - t_p
        prof = gm.profile_get()
        gm.profile(False)
    # a second timed window late in the run (steps late_at + 1 .. late_at +
    # steps), where the flow has developed, after untimed steps up to it
    late = None
    done += steps if profile else 0
    if late_at >= done:
        for _ in range(late_at - done):
            gm.step(W)
        torch.cuda.synchronize()
        l_iters, l_np, l_first, l_lat, l_r0, l_pts = [], [], [], [], [], []
        st0 = gm.stats()
        gc.collect()
        gc.disable()
        t_l = time.perf_counter()
        for _ in range(steps):
            t = time.perf_counter()
            _, info = gm.step(W)
            l_lat.append(time.perf_counter() - t)
            l_iters.append(max(info["iters"]))
            l_np.append(info["nonphys"])
            l_first.append(info["first_sweeps"])
            l_r0.append(info["start_resid"])
            l_pts.append(info["start_points"])
        torch.cuda.synchronize()
        el_l = time.perf_counter() - t_l
        gc.enable()
        st1 = gm.stats()
        slow = int(np.argmax(l_lat))
        late = {"steps": "%d-%d" % (late_at + 1, late_at + steps), "value": m.nt * steps / el_l,
                "ms_per_step": el_l * 1e3 / steps, "krylov_iters_per_step": float(np.mean(l_iters)),
                "step_ms_p50": float(np.percentile(np.array(l_lat) * 1e3, 50)),
                "step_ms_max": float(np.max(l_lat) * 1e3),
                "first_step_sweeps": float(np.mean(l_first)),
                "start_resid_median": float(np.median(l_r0)),
                "start_points": float(np.mean(l_pts)),
                "graph_captures": st1["graph_captures"] - st0["graph_captures"],
                "capture_ms": st1["capture_ms"] - st0["capture_ms"],
                "slowest_step": {"index": late_at + 1 + slow, "ms": l_lat[slow] * 1e3, "outer": l_iters[slow],
                                 "first_sweeps": l_first[slow], "start_points": l_pts[slow]},
                "gauss_point_fallbacks_per_step": float(np.mean(l_np))}
    stats = gm.stats()
    gm.close()
    lat_ms = np.array(lat) * 1e3
    return {
        "value": m.nt * steps / elapsed,
        "ms_per_step": elapsed * 1e3 / steps,
        "step_ms_p50": float(np.percentile(lat_ms, 50)),
        "step_ms_p99": float(np.percentile(lat_ms, 99)),
        "krylov_iters_per_step": float(np.mean(iters)),
        "first_step_sweeps": float(np.mean(first)),
        "start_resid_median": float(np.median(r0)),
        "limited_cells_per_step": float(np.mean(limited)),
        "gauss_point_fallbacks_per_step": float(np.mean(nonphys)),
        "late_window": late,
        "window": window,
        "setup_s": setup_s,
        "stats": stats,
        "profile": prof,
        "elapsed_s": elapsed,
        "profiled_elapsed_s": prof_elapsed,
    }


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "gks_solver_hbm_traffic_shock_vortex_1m.txt")
FP64_SUMMARY = os.path.join(ROOT, "profiles", "gks_fp64_flops_shock_vortex_1m.txt")


def measured_traffic(kernel_class: str):
    """HBM bytes per launch of a kernel class from the committed counter
    summary, or None when the kernels changed since the counters were taken."""
    try:
        from paper_1802_00704_amd.profiling import kernel_sources_sha256, read_summary
        sha, table = read_summary(TRAFFIC_SUMMARY)
    except (OSError, ImportError):
        return None
    if sha != kernel_sources_sha256():
        return None
    return table.get(kernel_class)


def measured_flops(kernel_class: str):
    """FP64 FLOPs per launch of a kernel class from the committed counter
    summary, or None when the kernels changed since the counters were taken."""
    try:
        from paper_1802_00704_amd.profiling import kernel_sources_sha256, read_summary
        sha, table = read_summary(FP64_SUMMARY, column=2, ncols=8)
    except (OSError, ImportError):
        return None
    if sha != kernel_sources_sha256():
        return None
    return table.get(kernel_class)


OPCOUNT_SUMMARY = os.path.join(ROOT, "profiles", "gks_flux_opcount.txt")


def algorithmic_flux_flops():
    """FP64 FLOPs per Gauss point of the method as the oracle writes it out
    (operation count of its flux, profiles/gks_flux_opcount.txt)."""
    try:
        with open(OPCOUNT_SUMMARY) as f:
            for line in f:
                if line.startswith("flop_per_gauss_point"):
                    return float(line.split()[1])
    except OSError:
        return None
    return None


def flux_fp64(prof: dict, n_gauss: int):
    """FP64 VALU roofline of the flux kernel: FP64 FLOPs executed per launch
    (the counters) over the live average launch duration; beside it the
    method's FLOPs (the oracle's operation count) at the same duration."""
    d = prof.get("flux") if prof else None
    fl = measured_flops("flux")
    if not d or d["ms"] <= 0 or not fl:
        return None
    us = d["ms"] * 1e3 / max(1, d["launches"])
    achieved = fl / (us * 1e-6) / 1e12
    out = {"bound": "fp64_valu", "kernel": "flux", "achieved": round(achieved, 2), "peak": FP64_PEAK_TFLOPS,
           "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "avg_launch_us": round(us, 2),
           "flop_per_launch": fl, "executed_flop_per_gauss_point": round(fl / n_gauss, 1)}
    fg = algorithmic_flux_flops()
    if fg:
        out["algorithmic_flop_per_gauss_point"] = fg
        out["algorithmic_rate_TFLOPs"] = round(fg * n_gauss / (us * 1e-6) / 1e12, 2)
    return out


def roofline(prof: dict, elapsed_s: float, n_gauss: int):
    """Roofline entry of the kernel class with the largest share of kernel
    time.  The memory-bound classes are priced on their algorithmic bytes
    against the HBM peak.  The flux kernel is FP64-arithmetic bound and is
    priced against the FP64 vector peak on the FP64 FLOPs it executes (the
    committed counter summary, while it matches the kernel sources).  The
    method's FLOPs as the oracle writes them out (its operation count per
    Gauss point) are reported beside them but not used for the fraction:
    the kernel's coefficient-combined contraction does that work in about
    half the operations, so on that count it would exceed the peak."""
    if not prof:
        return None
    tot = sum(v["ms"] for v in prof.values())
    name, d = max(prof.items(), key=lambda kv: kv[1]["ms"])
    shares = {k: round(v["ms"] / tot, 4) for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["ms"]) if v["ms"] > 0}
    us = d["ms"] * 1e3 / max(1, d["launches"])
    common = {"avg_launch_us": round(us, 2), "time_share": shares,
              "kernel_time_fraction_of_steps": round(tot * 1e-3 / elapsed_s, 4)}
    if name == "flux":
        fg = algorithmic_flux_flops()
        fl = measured_flops("flux")
        if d["ms"] <= 0:
            return None
        out = {"bound": "alu", "kernel": name, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
               "traffic": measured_traffic(name)}
        if fl:
            ex = fl / (us * 1e-6) / 1e12
            out.update({"achieved": round(ex, 2), "frac": round(ex / FP64_PEAK_TFLOPS, 4),
                        "flop_basis": "FP64 FLOPs executed (counters)", "flop_per_launch": fl})
        else:
            out.update({"achieved": None, "frac": None,
                        "flop_basis": "counter summary older than the kernel sources"})
        if fg:
            out.update({"method_flop_per_gauss_point": fg, "gauss_points_per_launch": n_gauss,
                        "method_rate_TFLOPs": round(fg * n_gauss / (us * 1e-6) / 1e12, 2)})
        out.update(common)
        return out
    if d["ms"] <= 0 or d["bytes"] <= 0:
        return None
    achieved = d["bytes"] / (d["ms"] * 1e-3) / 1e9
    out = {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(name),
           "bytes_per_launch": d["bytes"] / max(1, d["launches"])}
    out.update(common)
    return out


SAME_WORK_CLASSES = ("rhs", "cfl", "update", "copyout", "spmv_resid", "ilu_fwd32", "ilu_bwd32",
                     "ilu_fwd", "ilu_bwd")


def kernel_table(prof: dict) -> dict:
    """Every kernel class that moves memory: live average launch duration,
    algorithmic GB/s and its fraction of the HBM peak, share of kernel time,
    and, while the kernel sources match the committed counter summary, the
    counted HBM traffic per launch and the GB/s it implies."""
    if not prof:
        return {}
    tot = sum(v["ms"] for v in prof.values())
    out = {}
    for k, d in sorted(prof.items(), key=lambda kv: -kv[1]["ms"]):
        if d["ms"] <= 0 or d["bytes"] <= 0 or k in ("flux", "limit_apply"):
            continue
        gbs = d["bytes"] / (d["ms"] * 1e-3) / 1e9
        us = d["ms"] * 1e3 / max(1, d["launches"])
        row = {"launches": d["launches"], "avg_launch_us": round(us, 2), "achieved_GBs": round(gbs, 1),
               "frac": round(gbs / HBM_PEAK_GBS, 4), "time_share": round(d["ms"] / tot, 4)}
        # the counter summary averages each class over both forms' launches;
        # only classes whose launches do the same work in either form use it
        tr = measured_traffic(k) if k in SAME_WORK_CLASSES else None
        if tr:
            row["traffic_GBs"] = round(tr / (us * 1e-6) / 1e9, 1)
        out[k] = row
    return out


def serving_leg(n_requests: int, max_batch: int) -> dict:
    """The first n_requests of the seeded serving stream of 2,000 requests
    (Poisson arrivals at 40/s; advection or shock-vortex, 2e3-2e5 triangles
    log-uniform, 50-500 steps, FP64 or mixed), served with continuous
    batching: each request's mesh and initial state are generated by the
    server's set-up threads after admission."""
    import gks_inputs as gi
    import paper_1802_00704_amd as g
    from paper_1802_00704_amd.serving import Request, Server
    reqs = []
    for sp in gi.serving_specs(2000)[:n_requests]:
        prm = {"precision": g.GKS_MIXED if sp["mixed"] else g.GKS_FP64, "nonphys_fallback": 1}
        reqs.append(Request(rid=sp["rid"], mesh=None, W0=None, make=lambda sp=sp: gi.serving_case(sp),
                            nt_hint=gi.serving_cells(sp), steps=sp["steps"], params=prm, arrival=sp["arrival"]))
    stats = Server(max_batch=max_batch, log_every=50).run(reqs, realtime=True)
    stats["stream"] = ("first %d of the 2000 seeded requests, Poisson 40/s, 2e3-2e5 triangles, 50-500 steps, "
                       "50/50 FP64/mixed" % n_requests)
    return stats


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="shock_vortex_1m",
                    choices=["shock_vortex_1m", "advection_512", "acoustic_pulse_1m", "cavity_256"])
    ap.add_argument("--forms", default="mixed,fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--graphs", type=int, default=1, choices=[0, 1],
                    help="1: steps replay captured HIP graphs; 0: eager launches (counter runs use 0 so that "
                         "every traced launch does work)")
    ap.add_argument("--serving-requests", type=int, default=200,
                    help="requests of the serving stream to run after the throughput legs (0: skip)")
    ap.add_argument("--serving-max-batch", type=int, default=64,
                    help="requests per batched step (gks_batch_step) of each precision's driver")
    ap.add_argument("--late-window", type=int, default=480,
                    help="shock-vortex workload: also time steps late_window+1 .. late_window+steps of the "
                         "500-step run (0: skip)")
    ap.add_argument("--no-limiter-leg", action="store_true",
                    help="skip the extra runs of the mixed form with the DWBAP limiter on")
    ap.add_argument("--other-workloads", default="advection_512,cavity_256",
                    help="also time both forms on these workloads (steps and warm-up as above, no event "
                         "profile); empty to skip")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one MI355X only; multi-GPU runs are not part of this build "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    # the oracle's CPU baseline runs first, before anything touches the GPU
    cpu = None if args.no_cpu_baseline else cpu_baseline(args.workload)
    import torch
    import paper_1802_00704_amd as g
    m, W0, desc, extra = workload(args.workload)
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    late_at = args.late_window if args.workload == "shock_vortex_1m" else 0
    res = {}
    for f in forms:
        prec = g.GKS_MIXED if f == "mixed" else g.GKS_FP64
        res[f] = run_form(m, W0, prec, args.steps, args.warmup, not args.no_profile, args.graphs, extra=extra,
                          late_at=late_at)
        print("# %s: %.4g cell-steps/s, %.3f ms/step, %.1f Krylov iterations/step" %
              (f, res[f]["value"], res[f]["ms_per_step"], res[f]["krylov_iters_per_step"]), file=sys.stderr,
              flush=True)
    head = forms[0]
    r = res[head]
    # the DWBAP limiter (section 3.3) on the same workload, mixed form, in
    # conserved and in characteristic variables (section 4.2)
    lim = None
    if not args.no_limiter_leg:
        lim = {}
        for name, variables in (("conservative", g.LIMIT_CONSERVATIVE), ("characteristic", g.LIMIT_CHARACTERISTIC)):
            rl = run_form(m, W0, g.GKS_MIXED, args.steps, args.warmup, not args.no_profile, args.graphs,
                          limiter=variables, extra=extra)
            pl = rl["profile"].get("limit") if rl["profile"] else None
            pa = rl["profile"].get("limit_apply") if rl["profile"] else None
            leg = {"ms_per_step": rl["ms_per_step"], "value": rl["value"],
                   "limited_cells_per_step": rl["limited_cells_per_step"],
                   "krylov_iters_per_step": rl["krylov_iters_per_step"]}
            if pl and pl["ms"] > 0:
                # indicator pass over every cell (memory-bound)
                leg["mark_kernel"] = {"avg_launch_us": round(pl["ms"] * 1e3 / max(1, pl["launches"]), 2),
                                      "achieved_GBs": round(pl["bytes"] / (pl["ms"] * 1e-3) / 1e9, 1),
                                      "frac_of_hbm_peak": round(pl["bytes"] / (pl["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                      "traffic": measured_traffic("limit") if name == "conservative" else None}
            if pa and pa["ms"] > 0:
                # limiting of the listed cells and the scatter (arithmetic on a few cells)
                leg["apply_us_per_step"] = round(pa["ms"] * 1e3 / max(1, pa["launches"] // 2), 2)
            lim[name] = leg
            print("# mixed + limiter (%s variables): %.4g cell-steps/s, %.3f ms/step, %.0f cells limited per step" %
                  (name, rl["value"], rl["ms_per_step"], rl["limited_cells_per_step"]), file=sys.stderr, flush=True)
    # the other workloads of the paper's test set (sections 4.1 and 4.7), both forms
    others = {}
    for name in [w.strip() for w in args.other_workloads.split(",") if w.strip() and w.strip() != args.workload]:
        mo, Wo, desc_o, extra_o = workload(name)
        leg = {"workload": desc_o, "cells": mo.nt}
        for f in ("mixed", "fp64"):
            prec = g.GKS_MIXED if f == "mixed" else g.GKS_FP64
            ro = run_form(mo, Wo, prec, args.steps, args.warmup, False, args.graphs, extra=extra_o)
            leg[f] = {k: ro[k] for k in ("value", "ms_per_step", "krylov_iters_per_step", "first_step_sweeps",
                                         "start_resid_median", "gauss_point_fallbacks_per_step")}
            print("# %s, %s: %.4g cell-steps/s, %.3f ms/step, %.1f Krylov iterations/step" %
                  (name, f, ro["value"], ro["ms_per_step"], ro["krylov_iters_per_step"]), file=sys.stderr, flush=True)
        others[name] = leg
    serving = serving_leg(args.serving_requests, args.serving_max_batch) if args.serving_requests > 0 else None
    if serving:
        print("# serving: %.4g cell-steps/s, step p50/p99 %.2f/%.2f ms, solve p50/p99 %.2f/%.2f ms" %
              (serving["throughput_cell_steps_per_s"], serving["step_ms_p50"], serving["step_ms_p99"],
               serving["solve_ms_p50"], serving["solve_ms_p99"]), file=sys.stderr, flush=True)
    out = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": desc, "form": head,
                   "solver": ("multicolour BILU(0); FP64 FGMRES(30) preconditioned by FP32 BILU(0)-Richardson sweeps (7 in the first outer step, adapted down while one outer step suffices; 4 after)"
                              + (" (split form)" if r["stats"].get("split_form") else "")
                              + "; start extrapolated from up to six past solutions") if head == "mixed"
                   else "multicolour BILU(0); FP64 GMRES(30); start extrapolated from up to six past solutions",
                   "cells": m.nt},
        "roofline": roofline(r["profile"], r["profiled_elapsed_s"], 2 * int(r["stats"]["nf"])),
        "flux_fp64": flux_fp64(r["profile"], 2 * int(r["stats"]["nf"])),
        "cpu_baseline": cpu,
        "forms": {f: dict({k: v for k, v in res[f].items() if k not in ("profile", "stats", "elapsed_s", "profiled_elapsed_s")},
                          hbm_kernels=kernel_table(res[f]["profile"]))
                  for f in forms},
        "latency_ms": {"step_p50": r["step_ms_p50"], "step_p99": r["step_ms_p99"],
                       "serving_step_p50": serving["step_ms_p50"] if serving else None,
                       "serving_step_p99": serving["step_ms_p99"] if serving else None,
                       "serving_solve_p50": serving["solve_ms_p50"] if serving else None,
                       "serving_solve_p99": serving["solve_ms_p99"] if serving else None},
        "serving": serving,
        "limiter": lim,
        "other_workloads": others or None,
        "device": torch.cuda.get_device_name(0),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
