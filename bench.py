#!/usr/bin/env python3
"""Benchmark: factor + PCG solve throughput of the RHIF library on one MI355X.

One step = rhif_factor of the assembled matrix (planning, every level's elimination,
block-Jacobi preconditioning, skeletonization, root) followed by rhif_pcg_solve to a
relative residual of 1e-12 with F^-1 as the preconditioner. The matrix and right-hand side
are resident in HBM before the timed region. Workload: 2D 5-point FD on a 512 x 512 grid,
a = exp(3 g) with g a standardized Gaussian random field (correlation length 8 cells,
seed 1), b = 0, f ~ N(0,1), leaf 16, eps 1e-6, FP64.

Prints one JSON line (see the fields below). --gpus N > 1 is refused: the library runs on
one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--eps", type=float, default=1e-6)
    ap.add_argument("--side", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the FP32-mixed leg, the uneven batch and the 2048^2 point")
    ap.add_argument("--cpu-sample-side", type=int, default=512,
                    help="side of the (corner) window of the same field timed with the CPU oracle")
    ap.add_argument("--profile-3d", action="store_true",
                    help="profiling aid: only factor and solve the 3D 64^3 problem --warmup + --steps "
                         "times (FP64) and print their times; no benchmark line")
    return ap.parse_args()


def profile_3d(args):
    """The 3D 64^3 two-valued problem (the 3D leg of the extras), factored and solved
    --warmup + --steps times, for kernel traces and counters."""
    import torch
    from paper_1808_01364_amd import rhif
    from workloads.fields import CONFIGS
    torch.cuda.set_device(0)
    C = CONFIGS["cfg3"]()
    dev = "cuda:0"
    a = torch.tensor(C.a_cells.ravel(), dtype=torch.float64, device=dev)
    b = torch.tensor(C.b, dtype=torch.float64, device=dev)
    csr = rhif.assemble_fd(3, C.s, a, b)
    f = torch.tensor(C.f, dtype=torch.float64, device=dev)
    for k in range(args.warmup + args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F = rhif.Factor(3, C.s, csr, C.leaf, C.eps, 1)
        t1 = time.perf_counter()
        u, it, rr = F.pcg(f, 1e-12, 500)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        F.close()
        print(f"{C.name} step {k}: factor {1e3 * (t1 - t0):.1f} ms, pcg {1e3 * (t2 - t1):.1f} ms, "
              f"{it} iterations, relres {rr:.2e}", flush=True)


def make_workload(side: int, eps: float):
    from workloads import make_problem
    return make_problem("lognormal", 2, side, seed=1, leaf=16, eps=eps, sigma=3.0, corr_len=8.0,
                        name=f"2d-{side}-lognormal-s3-eps{eps:g}")


def cpu_baseline(P, sample_side: int):
    """The oracle (plain FP64 NumPy/SciPy) on a window of the same coefficient field: the
    (sample_side+1)^2 cells in the corner of the field, the matching slice of f."""
    import numpy as np
    import oracle as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
    except Exception:
        threads = 1
    s = sample_side
    what = "the full workload" if s == P.s else f"the {s}x{s} corner window of the same field"
    a = np.ascontiguousarray(P.a_cells[: s + 1, : s + 1])
    f = np.ascontiguousarray(P.f.reshape(P.s, P.s)[:s, :s]).ravel()
    A = O.assemble_fd(2, s, a, None)
    t0 = time.perf_counter()
    F = O.factor(A, 2, s, P.leaf, P.eps, 1)
    t1 = time.perf_counter()
    res = O.pcg(A, f, lambda v: O.apply_inverse(F, v), 1e-12, 500)
    t2 = time.perf_counter()
    return {"value": s * s / (t2 - t0), "unit": "DOFs/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle factor+PCG on {what} "
                      f"(N={s*s}, leaf {P.leaf}, eps {P.eps:g}); t_factor {t1-t0:.2f} s, "
                      f"t_pcg {t2-t1:.2f} s, {res.iters} iterations, host threads {threads} "
                      f"of {os.cpu_count()} cores"}


HBM_CLASSES = ("apply_up", "apply_down", "apply_gather", "spmv", "vector", "front_csr", "front_extend")
MFMA_CLASSES = ("elim_leaf", "elim_upper", "root")


def class_rows(kernels):
    """Per kernel class: device time, launches, algorithmic work and the fraction of the
    roofline that bounds it (HBM bytes for the memory-bound classes, FP64 flops otherwise)."""
    rows = {}
    for name, kv in kernels.items():
        ms = kv["ms"]
        if ms <= 0:
            continue
        if name in HBM_CLASSES:
            ach = kv["bytes"] / (ms * 1e-3) / 1e9
            rows[name] = {"ms": round(ms, 4), "launches": kv["launches"], "bound": "hbm", "alg_bytes": kv["bytes"],
                          "achieved_GBs": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4)}
        else:
            ach = kv["flops"] / (ms * 1e-3) / 1e12
            rows[name] = {"ms": round(ms, 4), "launches": kv["launches"],
                          "bound": "mfma" if name in MFMA_CLASSES else "alu", "alg_flops": kv["flops"],
                          "achieved_TFLOPs": round(ach, 4), "frac": round(ach / FP64_PEAK_TFLOPS, 5)}
    return rows


def timed_solve(rhif, torch, P, csr, f, precision=0, reps=3):
    """Median factor and PCG times (ms) of `reps` factor+solve steps after one warm-up."""
    tf, tp, it = [], [], 0
    for k in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F = rhif.Factor(P.d, P.s, csr, P.leaf, P.eps, 1, precision=precision)
        t1 = time.perf_counter()
        u, it, rr = F.pcg(f, 1e-12, 500)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        F.close()
        if k > 0:
            tf.append(1e3 * (t1 - t0))
            tp.append(1e3 * (t2 - t1))
    import numpy as np
    return float(np.median(tf)), float(np.median(tp)), it, rr


def extras(rhif, torch, P, csr, f):
    """The FP32-mixed factor on the same workload; the uneven batch (64 problems, sides from
    {128, 192, 256, 384, 512}, a = exp(2 g), eps 1e-4): plain FP64 one by one against the
    FP32-mixed autotuned batch; and a problem too large for the on-chip caches (2048^2, the
    same field recipe, seed 7) with the per-class roofline of its kernels; the 512^2 system at
    eps 1e-3; and the 3D 64^3 two-valued problem in FP64 and FP32-mixed."""
    import dataclasses
    import numpy as np
    from paper_1808_01364_amd import batch
    from workloads import make_problem
    from workloads.fields import CONFIGS, batch_problem
    out = {}
    f64 = timed_solve(rhif, torch, P, csr, f, 0)
    f32 = timed_solve(rhif, torch, P, csr, f, 1)
    out["fp32_mixed"] = {
        "workload": P.name, "fp64": {"t_factor_ms": f64[0], "t_pcg_ms": f64[1], "pcg_iters": f64[2],
                                     "dofs_per_s": P.N / ((f64[0] + f64[1]) * 1e-3)},
        "fp32_mixed": {"t_factor_ms": f32[0], "t_pcg_ms": f32[1], "pcg_iters": f32[2], "relres": f32[3],
                       "dofs_per_s": P.N / ((f32[0] + f32[1]) * 1e-3)}}
    # the uneven batch
    probs = [batch_problem(k, 1e-4) for k in range(64)]
    dofs = sum(q.N for q in probs)
    dev = "cuda:0"
    items64 = [batch.BatchItem(2, q.s, torch.tensor(q.a_cells.ravel(), dtype=torch.float64, device=dev),
                               torch.tensor(q.f, dtype=torch.float64, device=dev), None, q.leaf, q.eps, 0)
               for q in probs]
    items32 = [batch.BatchItem(it.dim, it.n, it.a_cells, it.f, None, it.leaf, it.eps, 1) for it in items64]
    for it in items64[:4]:
        batch.solve_one(it)                                   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq = [batch.solve_one(it) for it in items64]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ns, order, group = batch.autotune(items32)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    bat = batch.solve_many(items32, ns, order, group=group)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    out["batch"] = {"problems": len(probs), "dofs": dofs,
                    "fp64_one_by_one_dofs_per_s": dofs / (t1 - t0),
                    "fp32_mixed_autotuned_batch_dofs_per_s": dofs / (t3 - t2),
                    "speedup": (t1 - t0) / (t3 - t2), "autotuned": {"streams": ns, "order": order, "problems_per_factor_call": group},
                    "max_iters": {"fp64": max(r[1] for r in seq), "fp32_batch": max(r[1] for r in bat)},
                    "worst_relres_fp32_batch": max(r[2] for r in bat)}
    del items64, items32, seq, bat
    # out of the on-chip caches: 2048^2
    Q = make_problem("lognormal", 2, 2048, seed=7, leaf=16, eps=P.eps, sigma=3.0, corr_len=8.0,
                     name=f"2d-2048-lognormal-s3-eps{P.eps:g}-seed7")
    aq = torch.tensor(Q.a_cells.ravel(), dtype=torch.float64, device=dev)
    cq = rhif.assemble_fd(2, Q.s, aq, None)
    fq = torch.tensor(Q.f, dtype=torch.float64, device=dev)
    tq = timed_solve(rhif, torch, Q, cq, fq, 0, reps=2)
    F = rhif.Factor(2, Q.s, cq, Q.leaf, Q.eps, 1, flags=rhif.FLAG_KERNEL_TIMES)
    F.pcg(fq, 1e-12, 500)
    rows = class_rows(F.stats()["kernels"])
    F.close()
    out["out_of_cache_2048"] = {"workload": Q.name, "N": Q.N, "t_factor_ms": tq[0], "t_pcg_ms": tq[1],
                                "pcg_iters": tq[2], "dofs_per_s": Q.N / ((tq[0] + tq[1]) * 1e-3),
                                "classes": rows}
    del aq, cq, fq
    # the same 512^2 system with a coarser ID tolerance (a cheaper, weaker preconditioner)
    P3 = dataclasses.replace(P, eps=1e-3, name=P.name.replace(f"eps{P.eps:g}", "eps0.001"))
    t3 = timed_solve(rhif, torch, P3, csr, f, 0)
    out["eps_1e-3"] = {"workload": P3.name, "t_factor_ms": t3[0], "t_pcg_ms": t3[1], "pcg_iters": t3[2],
                       "relres": t3[3], "dofs_per_s": P3.N / ((t3[0] + t3[1]) * 1e-3)}
    # 3D: 64^3 two-valued coefficients (1e-3 / 1e3), b = 1e-2, leaf 4, eps 1e-3; FP64 and
    # FP32-mixed, and the per-class rows of the FP64 factor and solve
    C = CONFIGS["cfg3"]()
    a3 = torch.tensor(C.a_cells.ravel(), dtype=torch.float64, device=dev)
    b3 = torch.tensor(C.b, dtype=torch.float64, device=dev)
    c3 = rhif.assemble_fd(3, C.s, a3, b3)
    f3 = torch.tensor(C.f, dtype=torch.float64, device=dev)
    d64 = timed_solve(rhif, torch, C, c3, f3, 0, reps=2)
    d32 = timed_solve(rhif, torch, C, c3, f3, 1, reps=2)
    F = rhif.Factor(3, C.s, c3, C.leaf, C.eps, 1, flags=rhif.FLAG_KERNEL_TIMES)
    F.pcg(f3, 1e-12, 500)
    rows3 = class_rows(F.stats()["kernels"])
    F.close()
    out["3d_64"] = {"workload": C.name, "N": C.N,
                    "fp64": {"t_factor_ms": d64[0], "t_pcg_ms": d64[1], "pcg_iters": d64[2], "relres": d64[3],
                             "dofs_per_s": C.N / ((d64[0] + d64[1]) * 1e-3)},
                    "fp32_mixed": {"t_factor_ms": d32[0], "t_pcg_ms": d32[1], "pcg_iters": d32[2],
                                   "relres": d32[3], "dofs_per_s": C.N / ((d32[0] + d32[1]) * 1e-3)},
                    "classes_fp64": rows3}
    return out


def main():
    args = _args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the RHIF library runs one problem on one GPU; multi-GPU runs are not "
              "part of this build (how the path would shard is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    if args.profile_3d:
        profile_3d(args)
        return
    import numpy as np
    import torch
    from paper_1808_01364_amd import rhif

    torch.cuda.set_device(0)
    P = make_workload(args.side, args.eps)
    dev = "cuda:0"
    a = torch.tensor(P.a_cells.ravel(), dtype=torch.float64, device=dev)
    csr = rhif.assemble_fd(2, P.s, a, None)
    f = torch.tensor(P.f, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    def step(flags):
        F = rhif.Factor(2, P.s, csr, P.leaf, P.eps, 1, flags=flags)
        u, it, rr = F.pcg(f, 1e-12, 500)
        return F, u, it, rr

    # warm-up steps time every kernel class with HIP events to find the dominant kernel
    per_class = {}
    warm_kernels = {}
    for _ in range(max(args.warmup, 1)):
        F, u, it, rr = step(rhif.FLAG_KERNEL_TIMES)
        for name, kv in F.stats()["kernels"].items():
            per_class[name] = per_class.get(name, 0.0) + kv["ms"]
            acc = warm_kernels.setdefault(name, {"ms": 0.0, "launches": 0, "flops": 0.0, "bytes": 0.0})
            for key in acc:
                acc[key] += kv[key]
        F.close()
    torch.cuda.synchronize()
    dom = max(per_class, key=per_class.get)
    dom_id = rhif.KCLASS_NAMES.index(dom)
    # the timed steps bracket only the dominant kernel's launches with events
    flags = rhif.FLAG_KERNEL_TIMES | ((1 << dom_id) << rhif.KERNEL_MASK_SHIFT)
    # every step factors, solves and frees its factor, so that the next step reuses its
    # device memory (the steady state of a solver that serves one system after another)
    kvs = []
    t_fac, t_pcg = [], []
    F = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ta = time.perf_counter()
        F = rhif.Factor(2, P.s, csr, P.leaf, P.eps, 1, flags=flags)
        tb = time.perf_counter()
        u, it, rr = F.pcg(f, 1e-12, 500)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        t_fac.append(tb - ta)
        t_pcg.append(tc - tb)
        kvs.append(F.kernel_class(dom))
        if k + 1 < args.steps:
            F.close()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    total = t1 - t0
    st = F.stats()
    kms = kfl = kby = 0.0
    kl = 0
    for kv in kvs:
        if kv:
            kms += kv["ms"]
            kfl += kv["flops"]
            kby += kv["bytes"]
            kl += kv["launches"]
    from paper_1808_01364_amd.prof_summary import CLASS_KERNEL, read_traffic
    eps_tag = f"{P.eps:g}".replace("e-0", "e-")   # 1e-06 -> 1e-6, as the profile files are named
    traffic = read_traffic(os.path.join(ROOT, "profiles", f"traffic_2d{P.s}_eps{eps_tag}.txt"),
                           CLASS_KERNEL.get(dom, ()))
    hbm_bound = dom in ("apply_up", "apply_down", "apply_gather", "spmv", "vector", "front_csr", "front_extend")
    if hbm_bound:
        achieved = kby / (kms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic}
    else:
        achieved = kfl / (kms * 1e-3) / 1e12
        roof = {"bound": "mfma" if dom.startswith("elim") or dom == "root" else "alu",
                "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic}
    roof.update({"kernel": dom, "launches": kl, "avg_launch_us": 1e3 * kms / max(kl, 1),
                 "alg_per_launch": (kby if hbm_bound else kfl) / max(kl, 1),
                 "share_of_device_time_warmup": per_class[dom] / sum(per_class.values())})
    Au = F.matvec(u)
    true_rel = float(torch.linalg.norm(f - Au) / torch.linalg.norm(f))
    ms = 1e3 * total / args.steps
    out = {
        "metric": "factor+solve DOFs/s (PCG to rel. residual 1e-12)",
        "value": P.N * args.steps / total,
        "unit": "DOFs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": P.name, "grid": f"{P.s}x{P.s}", "N": P.N, "leaf": P.leaf, "eps": P.eps,
                   "precond": 1, "pcg_iters": it, "relres": rr, "true_relres": true_rel,
                   "t_factor_ms": 1e3 * float(np.median(t_fac)), "t_pcg_ms": 1e3 * float(np.median(t_pcg)),
                   "levels": st["levels"], "root_size": st["root_size"],
                   "factor_MB": st["factor_bytes"] / 1e6},
    }
    out["roofline"] = roof
    out["kernel_ms_warmup"] = {k: round(v, 4) for k, v in sorted(per_class.items(), key=lambda kv: -kv[1])}
    out["classes"] = class_rows(warm_kernels)
    F.close()
    if not args.no_extras:
        out["extras"] = extras(rhif, torch, P, csr, f)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(P, min(args.cpu_sample_side, P.s))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
