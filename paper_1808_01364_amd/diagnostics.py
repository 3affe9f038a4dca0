"""Quality measures of a factorization, as the paper reports them (Sec. 4, Tables 1-2): the
root size |S_L|, the apply error e_a = ||A - F|| / ||A|| and the solve error
e_s = ||I - G^-1 A G^-T|| (power iteration on the GPU: rhif_estimate_ea, rhif_estimate_es) and
the PCG iteration count n_i to a relative residual of 1e-12, for the recursively preconditioned
factorization (PHIF) against plain HIF on the same problem.

    python -m paper_1808_01364_amd.diagnostics 2 1023 8 1e-4 1e-6     # dim side leaf eps...

prints one line per (eps, method). A loss of positive definiteness (HIF at loose eps) is
reported as such, as in the paper's tables.
"""
from __future__ import annotations

import sys
import time

from . import rhif


def trend_row(P, precond: int, seed: int = 0, maxit: int = 500) -> dict:
    """|S_L|, e_a, e_s, n_i and the factor / solve times of one problem (a workloads.Problem) with
    block-Jacobi preconditioning on (PHIF) or off (HIF)."""
    import torch
    dev = "cuda"
    a = torch.tensor(P.a_cells.ravel(), dtype=torch.float64, device=dev)
    b = None if P.b is None else torch.tensor(P.b, dtype=torch.float64, device=dev)
    csr = rhif.assemble_fd(P.d, P.s, a, b)
    f = torch.tensor(P.f, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    try:
        F = rhif.Factor(P.d, P.s, csr, P.leaf, P.eps, precond)
    except rhif.NotSPD as e:
        return {"N": P.N, "eps": P.eps, "method": "PHIF" if precond else "HIF", "not_spd": str(e)}
    t1 = time.perf_counter()
    st = F.stats()
    ea, ea_it = F.estimate_ea(seed=seed)
    es, es_it = F.estimate_es(seed=seed)
    try:
        u, it, rr = F.pcg(f, 1e-12, maxit)
    except rhif.NoConvergence as e:
        it, rr = e.iters, e.relres
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    F.close()
    return {"N": P.N, "eps": P.eps, "method": "PHIF" if precond else "HIF", "S_L": st["root_size"], "e_a": ea,
            "e_s": es, "e_a_iters": ea_it, "e_s_iters": es_it, "n_i": it, "relres": rr, "t_factor_ms": 1e3 * (t1 - t0)}


def main(argv):
    from workloads import make_problem
    dim, side, leaf = int(argv[0]), int(argv[1]), int(argv[2])
    for eps in (float(e) for e in argv[3:]):
        P = make_problem("paper", dim, side, 0, leaf, eps, lo=1e-2, hi=1e2)
        for precond in (0, 1):
            print(trend_row(P, precond), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
