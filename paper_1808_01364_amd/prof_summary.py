"""Summaries of rocprofv3 output for profiles/ (short text files with the figures used).

    python -m paper_1808_01364_amd.prof_summary stats  <run_kernel_stats.csv> <out.txt> "<command>"
    python -m paper_1808_01364_amd.prof_summary traffic <fetch counter csv> <write counter csv> <out.txt> \
        "<command>" [kernel ...]
    python -m paper_1808_01364_amd.prof_summary mfma <counter csv> <out.txt> "<command>"

The mfma summary gives, per kernel, the matrix-core busy fraction
SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE x SIMDs) over its dispatches (1024 SIMDs: 256 CUs of
4) and the FP64 / FP32 matrix flops (SQ_INSTS_VALU_MFMA_MOPS_* x 512).
The traffic summary scales FETCH_SIZE and WRITE_SIZE (KiB per dispatch) by what the same
counters read for the library's plain copy kernel (k_copy, 2 x 8 x N bytes per dispatch),
and records the SHA-256 of the kernel source so that stale figures can be recognized.
"""
from __future__ import annotations

import collections
import csv
import hashlib
import os
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = os.path.join(HERE, "csrc", "kernels.hip")

# kernel-class name used by bench.py -> the device kernels launched under it
CLASS_KERNEL = {"front_csr": ("k_front_csr", "k_leaf_dofs"), "front_extend": ("k_front_extend",),
                "elim_leaf": ("k_leaf_elim", "k_potrf_batch"),
                "elim_upper": ("k_chol_lead", "k_trsm_rows", "k_syrk_schur", "k_potrf_batch"),
                "root": ("k_potrf_batch",), "precond_chol": ("k_precond_groups",),
                "precond_scale": ("k_precond_scale",), "skeletonize": ("k_skeletonize",),
                "apply_up": ("k_apply_trsv_up", "k_apply_gemv_up", "k_apply_up"),
                "apply_down": ("k_apply_trsv_dn", "k_apply_gemv_dn", "k_apply_down"),
                "apply_gather": ("k_apply_group_up", "k_apply_group_dn", "k_sep_gather"),
                "spmv": ("k_spmv_dot",)}


def kernel_source_sha() -> str:
    with open(KERNEL_SOURCE, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def _short(name: str) -> str:
    """The kernel's base name: no namespace, return type or template arguments (the forms of
    one kernel template are counted together)."""
    base = name.split("(")[0].replace("rhif::", "")
    if base.startswith("void "):
        base = base[5:]
    return base.split("<")[0]


def stats(csv_path: str, out: str, command: str, top: int = 20) -> None:
    rows = list(csv.DictReader(open(csv_path)))
    lines = [f"# rocprofv3 --kernel-trace --stats summary", f"command: {command}",
             f"kernels_hip_sha256: {kernel_source_sha()}", "",
             f"{'kernel':<28} {'calls':>6} {'total_us':>11} {'avg_us':>9} {'min_us':>9} {'max_us':>9} {'pct':>6}"]
    agg = {}
    for r in rows:
        a = agg.setdefault(_short(r["Name"]), [0, 0.0, float("inf"), 0.0, 0.0])
        a[0] += int(r["Calls"])
        a[1] += float(r["TotalDurationNs"])
        a[2] = min(a[2], float(r["MinNs"]))
        a[3] = max(a[3], float(r["MaxNs"]))
        a[4] += float(r["Percentage"])
    for name, (calls, tot, mn, mx, pct) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:top]:
        lines.append(f"{name[:28]:<28} {calls:>6} {tot/1e3:>11.1f} {tot/calls/1e3:>9.2f} {mn/1e3:>9.2f} "
                     f"{mx/1e3:>9.2f} {pct:>6.2f}")
    open(out, "w").write("\n".join(lines) + "\n")


def _counter(path: str, counter: str):
    d = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") == counter:
            d[_short(r["Kernel_Name"])].append((float(r["Counter_Value"]), int(r["Grid_Size"])))
    return d


def traffic(fetch_csv: str, write_csv: str, out: str, command: str, kernels=None, N: int = 262144) -> None:
    f = _counter(fetch_csv, "FETCH_SIZE")
    w = _counter(write_csv, "WRITE_SIZE")
    known_kib = 8.0 * N / 1024.0
    fs = known_kib / statistics.mean(v for v, _ in f["k_copy"])
    ws = known_kib / statistics.mean(v for v, _ in w["k_copy"])
    kernels = kernels or sorted(f, key=lambda k: -sum(v for v, _ in f[k]))[:20]
    lines = ["# HBM traffic per dispatch from rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE (two runs)",
             f"command: {command}", f"kernels_hip_sha256: {kernel_source_sha()}",
             f"copy_kernel: k_copy, {int(known_kib)} KiB read + {int(known_kib)} KiB written per dispatch",
             f"copy_fetch_scale: {fs:.4f}", f"copy_write_scale: {ws:.4f}", "",
             f"{'kernel':<22} {'dispatches':>10} {'fetch_KiB':>11} {'write_KiB':>11} {'traffic_bytes':>14}"]
    for k in kernels:
        if k not in f:
            continue
        fk = statistics.mean(v for v, _ in f[k])
        wk = statistics.mean(v for v, _ in w.get(k, [(0.0, 0)]))
        tb = 1024.0 * (fk * fs + wk * ws)
        lines.append(f"{k:<22} {len(f[k]):>10} {fk:>11.1f} {wk:>11.1f} {tb:>14.0f}")
    open(out, "w").write("\n".join(lines) + "\n")


SIMDS = 1024


def mfma(csv_path: str, out: str, command: str, top: int = 24) -> None:
    vals = collections.defaultdict(lambda: collections.defaultdict(float))
    disp = collections.defaultdict(set)
    for r in csv.DictReader(open(csv_path)):
        k = _short(r["Kernel_Name"])
        vals[k][r["Counter_Name"]] += float(r["Counter_Value"])
        disp[k].add(r.get("Dispatch_Id", ""))
    lines = ["# matrix-core use per kernel from rocprofv3 --pmc SQ_VALU_MFMA_BUSY_CYCLES "
             "SQ_INSTS_VALU_MFMA_MOPS_F64 SQ_INSTS_VALU_MFMA_MOPS_F32 SQ_BUSY_CYCLES GRBM_GUI_ACTIVE",
             f"command: {command}", f"kernels_hip_sha256: {kernel_source_sha()}",
             "mfma_busy = sum SQ_VALU_MFMA_BUSY_CYCLES / (sum GRBM_GUI_ACTIVE x 1024 SIMDs) over the dispatches", "",
             f"{'kernel':<22} {'dispatches':>10} {'mfma_busy':>10} {'f64_mfma_GFLOP':>15} {'f32_mfma_GFLOP':>15}"]
    rows = []
    for k, v in vals.items():
        gui = v.get("GRBM_GUI_ACTIVE", 0.0)
        busy = v.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) / (gui * SIMDS) if gui > 0 else 0.0
        rows.append((k, len(disp[k]), busy, 512.0 * v.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) / 1e9,
                     512.0 * v.get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0) / 1e9, gui))
    rows.sort(key=lambda t: -t[5])
    for k, nd, busy, g64, g32, _ in rows[:top]:
        lines.append(f"{k[:22]:<22} {nd:>10} {busy:>10.4f} {g64:>15.3f} {g32:>15.3f}")
    open(out, "w").write("\n".join(lines) + "\n")


def read_traffic(path: str, kernels):
    """Scaled HBM bytes per dispatch over `kernels` (a name or a tuple of names; dispatch-weighted
    mean) from a traffic summary, or None if the summary is missing, lists none of them, or was
    taken on other kernel source."""
    if isinstance(kernels, str):
        kernels = (kernels,)
    if not os.path.exists(path):
        return None
    sha = None
    tot = 0.0
    nd = 0
    for ln in open(path):
        if ln.startswith("kernels_hip_sha256:"):
            sha = ln.split(":", 1)[1].strip()
        parts = ln.split()
        if len(parts) == 5 and parts[0] in kernels:
            tot += int(parts[1]) * float(parts[4])
            nd += int(parts[1])
    if sha != kernel_source_sha() or nd == 0:
        return None
    return tot / nd


if __name__ == "__main__":
    mode = sys.argv[1]
    if mode == "stats":
        stats(sys.argv[2], sys.argv[3], sys.argv[4])
    elif mode == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], sys.argv[6:] or None)
    elif mode == "mfma":
        mfma(sys.argv[2], sys.argv[3], sys.argv[4])
    else:
        raise SystemExit(__doc__)
