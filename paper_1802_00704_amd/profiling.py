"""Turn rocprofv3 counter traces of libgks into per-kernel-class HBM traffic.

Usage (after two counter runs of the same command, FETCH_SIZE then
WRITE_SIZE, each converted with ``rocpd2csv -i <db> -d <dir>``):

    python -m paper_1802_00704_amd.profiling <fetch_csv_dir> <write_csv_dir>

prints, per kernel class of the library's event profiler, the mean HBM
bytes per launch.  Counter values (KiB per dispatch) are scaled by what
the same counter reads for the library's plain copy kernel ``k_copy``, whose
bytes are known exactly (8 bytes read and 8 written per element of its
grid).  The output also carries a SHA-256 of the kernel sources, so a reader
can tell whether the figures still describe the current kernels.

    python -m paper_1802_00704_amd.profiling --fp64 <csv_dir>

does the same for one counter run of SQ_INSTS_VALU_FLOPS_FP64,
SQ_INSTS_VALU_{FMA,ADD,MUL,TRANS}_F64 and SQ_INSTS_VALU: per kernel class,
FP64 FLOPs per launch.  The FLOPS counter adds 2 per FMA and 1 per other
FP64 instruction of a wave; times 64 lanes it gives the FLOPs of full
waves (an upper bound where lanes are inactive).

    python -m paper_1802_00704_amd.profiling --gathers

prints, for the sweeps of the 1M-triangle shock-vortex mesh, the bytes of
the neighbour rows that each level's launch must read from memory at least
once: a sweep gathers the rows of its lower (forward) or upper (backward)
neighbours, which other levels' launches produced, so every distinct
neighbour row is one compulsory read per launch beside the launch's
algorithmic bytes (host set-up only, no GPU).
"""
from __future__ import annotations

import collections
import csv
import glob
import hashlib
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/gks_kernels.hip", "csrc/gks_flux_device.h", "csrc/gks_char_basis.h", "csrc/gks_internal.h")

# rocprof kernel symbol (without arguments) -> event-profiler class name
CLASS_OF = [
    (r"k_mx_fwd", "ilu_fwd32"), (r"k_mx_bwd", "ilu_bwd32"),
    (r"k_ilu_fwd", "ilu_fwd"), (r"k_ilu_bwd", "ilu_bwd"),
    (r"k_spmv<double, double, true>", "spmv_resid"), (r"k_spmv", "spmv"),
    (r"k_dots", "dots"), (r"k_axpy", "axpy_dots"), (r"k_combine", "combine"), (r"k_acc", "axpy"),
    (r"k_sum_partials", "finalize"), (r"k_gmres_ctl", "misc"), (r"k_mask_cols", "misc"),
    (r"k_copyout", "copyout"), (r"k_rhs", "rhs"), (r"k_flux", "flux"), (r"k_update", "update"),
    (r"k_cfl", "cfl"), (r"k_copyout", "copyout"), (r"k_copyin", "misc"), (r"k_copy", "copy"), (r"k_extrap", "extrap"),
    (r"k_limit_mark", "limit"), (r"k_limit_apply", "limit_apply"), (r"k_limit_scatter", "limit_apply"),
    (r"k_es_fwd", "ilu_fwd32"), (r"k_es_bwd", "ilu_bwd32"),
]


def kernel_sources_sha256() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def kernel_class(name: str) -> str | None:
    base = re.sub(r"\(.*", "", name).replace("void ", "").replace("gks::", "").strip()
    if base.startswith("kg_"):          # grouped launches (batched steps) count with their kernel
        base = "k_" + base[3:]
    for pat, cls in CLASS_OF:
        if base.startswith(pat):
            return cls
    return None


def _load(path_dir: str, counter: str):
    files = glob.glob(os.path.join(path_dir, "*counter_collection*.csv"))
    if not files:
        raise FileNotFoundError("no counter_collection csv in %s" % path_dir)
    rows = []
    for r in csv.DictReader(open(files[0])):
        if r["Counter_Name"] == counter:
            rows.append((r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"])))
    return rows


def traffic(fetch_dir: str, write_dir: str) -> dict:
    f = _load(fetch_dir, "FETCH_SIZE")
    w = _load(write_dir, "WRITE_SIZE")

    def calib(rows):
        cp = [(g, v) for n, g, v in rows if kernel_class(n) == "copy"]
        if not cp:
            raise ValueError("the copy kernel is missing from the trace")
        return sum(8.0 * g for g, _ in cp) / sum(1024.0 * v for _, v in cp)

    cf, cw = calib(f), calib(w)
    out = collections.OrderedDict()
    for rows, key, c in ((f, "fetch", cf), (w, "write", cw)):
        acc = collections.defaultdict(list)
        for n, _, v in rows:
            cls = kernel_class(n)
            if cls:
                acc[cls].append(1024.0 * v * c)
        for cls, vals in acc.items():
            out.setdefault(cls, {})[key] = sum(vals) / len(vals)
            out[cls]["launches"] = len(vals)
    return {"calibration": {"fetch": cf, "write": cw}, "classes": out}


FP64_COUNTERS = ("SQ_INSTS_VALU_FLOPS_FP64", "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_ADD_F64",
                 "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_TRANS_F64", "SQ_INSTS_VALU")


def fp64(csv_dir: str) -> dict:
    """{class: {counter: mean value per launch, "launches": n}}"""
    out = collections.OrderedDict()
    for counter in FP64_COUNTERS:
        acc = collections.defaultdict(list)
        for n, _, v in _load(csv_dir, counter):
            cls = kernel_class(n)
            if cls:
                acc[cls].append(v)
        for cls, vals in acc.items():
            out.setdefault(cls, {})[counter] = sum(vals) / len(vals)
            out[cls]["launches"] = len(vals)
    return out


def main_fp64(csv_dir: str) -> int:
    t = fp64(csv_dir)
    print("kernel_sources_sha256 %s" % kernel_sources_sha256())
    print("%-12s %8s %16s %13s %13s %13s %11s %13s" % ("class", "launches", "fp64_flop/launch", "fma_f64",
                                                        "add_f64", "mul_f64", "trans_f64", "valu_insts"))
    for cls, d in t.items():
        if d.get("SQ_INSTS_VALU_FLOPS_FP64", 0.0) <= 0.0:
            continue
        print("%-12s %8d %16.0f %13.0f %13.0f %13.0f %11.0f %13.0f" % (
            cls, d["launches"], 64.0 * d["SQ_INSTS_VALU_FLOPS_FP64"], d.get("SQ_INSTS_VALU_FMA_F64", 0.0),
            d.get("SQ_INSTS_VALU_ADD_F64", 0.0), d.get("SQ_INSTS_VALU_MUL_F64", 0.0),
            d.get("SQ_INSTS_VALU_TRANS_F64", 0.0), d.get("SQ_INSTS_VALU", 0.0)))
    return 0


def gathers(mesh, applications=(7, 4)) -> dict:
    """Distinct neighbour rows per level and the mean compulsory gather bytes
    per launch of each sweep class, for the launch pattern of preconditioner
    applications of the given sweep counts (default: one solve of two outer
    steps, 7 then 4 sweeps): split-form FP32 sweeps (80-byte rows; the first
    sweep of an application covers every level in its forward pass, the
    later ones skip level 0; every sweep's backward pass covers all but the
    last level) and the FP64 BILU(0) solve (160-byte rows; forward levels
    1.., backward all but the last)."""
    import numpy as np
    from ._lib import host_inspect
    h = host_inspect(mesh)
    lp, nt = h["lev_ptr"], h["nt"]
    nl = len(lp) - 1
    lo, up = [], []
    for l in range(nl):
        lc = h["lcol"][:, lp[l]:lp[l + 1]]
        uc = h["ucol"][:, lp[l]:lp[l + 1]]
        lo.append(int(np.unique(lc[lc < nt]).size))
        up.append(int(np.unique(uc[uc < nt]).size))
    fwd32, bwd32 = [], []
    for q in applications:
        fwd32 += [lo[l] for l in range(nl)] + [lo[l] for _ in range(q - 1) for l in range(1, nl)]
        bwd32 += [up[l] for _ in range(q) for l in range(nl - 2, -1, -1)]
    fwd64 = [lo[l] for l in range(1, nl)]
    bwd64 = [up[l] for l in range(nl - 2, -1, -1)]
    mean = lambda rows, b: b * float(np.mean(rows)) if rows else 0.0
    return {"levels": [int(lp[l + 1] - lp[l]) for l in range(nl)], "lower_rows": lo, "upper_rows": up,
            "ilu_fwd32": mean(fwd32, 80), "ilu_bwd32": mean(bwd32, 80),
            "ilu_fwd": mean(fwd64, 160), "ilu_bwd": mean(bwd64, 160)}


def main_gathers() -> int:
    import gks_inputs as gi
    left, _ = gi.shock_vortex_states()
    walls = ((gi.BC_INFLOW, left), (gi.BC_OUTFLOW, None), (gi.BC_SLIP, None), (gi.BC_SLIP, None))
    m = gi.jss_mesh(1000, 500, 3, Lx=2.0, Ly=1.0, periodic=False, walls=walls)
    g = gathers(m)
    print("levels (rows)          %s" % " ".join(str(r) for r in g["levels"]))
    print("distinct lower rows    %s" % " ".join(str(r) for r in g["lower_rows"]))
    print("distinct upper rows    %s" % " ".join(str(r) for r in g["upper_rows"]))
    print("%-12s %22s" % ("class", "gather_B/launch"))
    for cls in ("ilu_fwd32", "ilu_bwd32", "ilu_fwd", "ilu_bwd"):
        print("%-12s %22.0f" % (cls, g[cls]))
    return 0


def main(argv):
    if len(argv) == 2 and argv[1] == "--gathers":
        return main_gathers()
    if len(argv) == 3 and argv[1] == "--fp64":
        return main_fp64(argv[2])
    if len(argv) != 3:
        print(__doc__)
        return 2
    t = traffic(argv[1], argv[2])
    print("kernel_sources_sha256 %s" % kernel_sources_sha256())
    print("calibration fetch %.6f write %.6f" % (t["calibration"]["fetch"], t["calibration"]["write"]))
    print("%-12s %8s %16s %16s %16s" % ("class", "launches", "fetch_B/launch", "write_B/launch", "traffic_B/launch"))
    for cls, d in t["classes"].items():
        fe, wr = d.get("fetch", 0.0), d.get("write", 0.0)
        print("%-12s %8d %16.0f %16.0f %16.0f" % (cls, d["launches"], fe, wr, fe + wr))
    return 0


def read_summary(path: str, column: int = 4, ncols: int = 5) -> tuple[str, dict]:
    """(sha256, {class: value}) from a committed summary: the traffic bytes
    per launch (defaults), or with column=2, ncols=8 the FP64 FLOPs per
    launch of the --fp64 table."""
    sha, table = "", {}
    for line in open(path):
        parts = line.split()
        if len(parts) == 2 and parts[0] == "kernel_sources_sha256":
            sha = parts[1]
        elif len(parts) == ncols and not line.startswith("#") and parts[0] != "class":
            try:
                table[parts[0]] = float(parts[column])
            except ValueError:
                pass
    return sha, table


if __name__ == "__main__":
    sys.exit(main(sys.argv))
