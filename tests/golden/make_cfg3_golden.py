"""Writes tests/golden/cfg3_oracle.npz: what the CPU oracle computes on the 3D 64^3 two-valued
problem (a = 1e-3 / 1e3 per voxel, b = 1e-2, leaf 4, eps 1e-3, seed 2), for the full-size
GPU test, which cannot run the oracle itself in its time limit.

Calls only the oracle and the shared input generator:
    python tests/golden/make_cfg3_golden.py     (about an hour on 8 cores)

Stored: every ID's choices (first unknown, size, rank, pivot order), the ratios that decide
them (|R_jj|/|R_11| of the steps taken and at the failing step; per pivot step the relative
gap between the two largest trailing norms), the largest condition number of a triangular
factor, |S_L|, the PCG iteration count and residual history, and at 4096 sampled unknowns
(plus the 2-norm of the whole vector) the PCG solution and F^-1 r for a seeded r."""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from workloads import CONFIGS  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg3_oracle.npz")


def main():
    P = CONFIGS["cfg3"]()
    A = O.assemble_fd(P.d, P.s, P.a_cells, P.b)
    t0 = time.perf_counter()
    F = O.factor(A, P.d, P.s, P.leaf, P.eps, P.precond)
    t1 = time.perf_counter()
    print(f"factor {t1 - t0:.1f} s, root {F.root_size}", flush=True)
    lv_, fd_, sz_, rk_, perm_, ratio_, gap_, ratio_ptr, gap_ptr = [], [], [], [], [], [], [], [0], [0]
    for lv in F.levels:
        for sk in lv.skels:
            lv_.append(lv.level)
            fd_.append(int(sk.group[0]))
            sz_.append(len(sk.group))
            rk_.append(len(sk.hat))
            perm_.append(np.asarray(sk.perm, dtype=np.int32))
            r11 = float(sk.rdiag[0]) if len(sk.rdiag) else 0.0
            ratios = list(np.asarray(sk.rdiag) / r11) if r11 > 0 else []
            ratios.append(sk.trace["stop_norm"] / r11 if r11 > 0 else np.nan)
            ratio_ += ratios
            ratio_ptr.append(len(ratio_))
            for nj in sk.trace["norms"]:
                v = np.sort(nj[np.isfinite(nj)])[::-1]
                gap_.append((v[0] - v[1]) / v[0] if len(v) > 1 and v[0] > 0 else 1.0)
            gap_ptr.append(len(gap_))
    kappa = 1.0
    mats = [F.root_L]
    for lv in F.levels:
        mats += [c.L for c in lv.cells] + [g.L for g in lv.groups] + [sk.Lt for sk in lv.skels]
    for M in mats:
        if M.size:
            kappa = max(kappa, float(np.linalg.cond(M)))
    t2 = time.perf_counter()
    print(f"choices and kappa {t2 - t1:.1f} s, kappa {kappa:.3e}", flush=True)
    res = O.pcg(A, P.f, lambda v: O.apply_inverse(F, v), 1e-12, 100)
    r = np.random.default_rng(12).standard_normal(P.N)
    z = O.apply_inverse(F, r)
    t3 = time.perf_counter()
    print(f"pcg {res.iters} iterations, relres {res.relres:.2e}, true {res.true_relres:.2e}, {t3 - t2:.1f} s",
          flush=True)
    idx = np.sort(np.random.default_rng(13).choice(P.N, 4096, replace=False))
    np.savez_compressed(
        OUT, level=np.array(lv_, np.int32), first_dof=np.array(fd_, np.int32), size=np.array(sz_, np.int32),
        rank=np.array(rk_, np.int32), perm=np.concatenate(perm_) if perm_ else np.zeros(0, np.int32),
        ratio=np.array(ratio_), ratio_ptr=np.array(ratio_ptr, np.int64), gap=np.array(gap_),
        gap_ptr=np.array(gap_ptr, np.int64), kappa=np.array(kappa), root_size=np.array(F.root_size),
        iters=np.array(res.iters), history=np.array(res.history), idx=idx.astype(np.int64),
        u_samples=res.u[idx], u_norm=np.array(np.linalg.norm(res.u)), z_samples=z[idx],
        z_norm=np.array(np.linalg.norm(z)), r_seed=np.array(12), eps=np.array(P.eps))
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
