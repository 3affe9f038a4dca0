"""Helpers shared by the GPU tests: run a seeded problem through the HIP library and
through the CPU oracle on the same inputs."""
import numpy as np

U = np.finfo(np.float64).eps

import oracle as O
from workloads import make_problem


def _host(t):
    return t.detach().cpu().numpy()


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def to_dev(x):
    torch = torch_cuda()
    return None if x is None else torch.tensor(np.ascontiguousarray(x).ravel(), dtype=torch.float64, device="cuda")


def gpu_csr(P):
    from paper_1808_01364_amd import rhif
    return rhif.assemble_fd(P.d, P.s, to_dev(P.a_cells), to_dev(P.b))


def gpu_factor(P, csr=None, eps=None, precond=None, flags=0):
    from paper_1808_01364_amd import rhif
    csr = csr if csr is not None else gpu_csr(P)
    return rhif.Factor(P.d, P.s, csr, P.leaf, P.eps if eps is None else eps,
                       P.precond if precond is None else precond, flags=flags)


def gpu_choices(F, L):
    """(level, smallest unknown) -> (k, pivot order) of every ID the GPU took; L is the
    number of skeletonization levels."""
    out = {}
    for lvl in range(L):
        sk = F.skeletons(lvl)
        for fd, n, k, perm in zip(sk.first_dof, sk.size, sk.rank, sk.perm):
            out[(lvl, fd)] = (k, np.array(perm))
    return out


def _certify(sk, k_g, perm_g, eps, tie_rel):
    """Why the GPU's (k_g, perm_g) may differ from the oracle's ID of group sk: "pivot" if at
    the first step where the pivot orders part the oracle's trailing norm of the GPU's column
    is within tie_rel of the largest one (several columns tie, Sec. 2.2: the skeleton is not
    unique), "rank" if the pivot orders agree up to the smaller rank and the deciding ratio
    |R_jj|/|R_11| is within tie_rel (relative) of eps; None if neither holds."""
    perm_o = np.asarray(sk.perm)
    k_o = len(sk.hat)
    tr = sk.trace or {}
    norms = tr.get("norms", [])
    kk = min(k_g, k_o)
    for j in range(kk):
        if perm_g[j] != perm_o[j]:
            if j >= len(norms):
                return None
            nj = norms[j]
            mx = float(np.nanmax(nj))
            ng = float(nj[perm_g[j]])
            return "pivot" if np.isfinite(ng) and mx - ng <= tie_rel * mx else None
    if k_g == k_o:
        return "same"
    if len(sk.rdiag) == 0 or sk.rdiag[0] <= 0:
        return None
    r11 = float(sk.rdiag[0])
    if kk < len(sk.rdiag):
        deciding = float(sk.rdiag[kk])       # the oracle took step kk, the GPU stopped there
    else:
        deciding = float(tr.get("stop_norm", np.nan))   # the oracle stopped at step kk
    if not np.isfinite(deciding) or eps <= 0:
        return None
    return "rank" if abs(deciding / r11 - eps) <= tie_rel * eps else None


def compare_choices(gpu, orc_factor, eps=None, tie_rel=1e-10):
    """Compare every ID of the GPU with the oracle's on the same matrix (both sides see the
    same groups). Returns counts: total, same (equal rank and skeleton set), tie_pivot and
    tie_rank (differences certified as ties of the pivot norms or of the rank test, within
    tie_rel), bad (differences that are not ties), missing (oracle groups the GPU lacks) and
    extra (GPU groups the oracle lacks); `bad_keys` lists the first offending groups."""
    eps = orc_factor.eps if eps is None else eps
    out = dict(total=0, same=0, tie_pivot=0, tie_rank=0, bad=0, missing=0, extra=0, bad_keys=[])
    seen = set()
    for lv in orc_factor.levels:
        for sk in lv.skels:
            key = (lv.level, int(sk.group[0]))
            seen.add(key)
            out["total"] += 1
            if key not in gpu:
                out["missing"] += 1
                continue
            k, perm = gpu[key]
            perm = np.asarray(perm)
            if k == len(sk.hat) and set(perm[:k].tolist()) == set(np.asarray(sk.perm)[:k].tolist()):
                out["same"] += 1
                continue
            why = _certify(sk, k, perm, eps, tie_rel)
            if why == "pivot":
                out["tie_pivot"] += 1
            elif why == "rank":
                out["tie_rank"] += 1
            elif why == "same":
                out["same"] += 1
            else:
                out["bad"] += 1
                if len(out["bad_keys"]) < 8:
                    out["bad_keys"].append((key, k, len(sk.hat)))
    out["extra"] = sum(1 for key in gpu if key not in seen)
    return out


def assert_choices(c):
    """Every difference must be a certified tie, and both sides must have the same groups."""
    assert c["bad"] == 0 and c["missing"] == 0 and c["extra"] == 0, c


def parity_check(P, A, n_rhs=3, well_conditioned=False, sol_tol=1e-10, flags=0, c_kappa=100.0, seed=11, F=None):
    """GPU against the oracle on the same matrix (the parity protocol of the ID's possible
    ties, Sec. 2.2):
    * every ID takes the oracle's rank and skeleton set, or differs only where the oracle's
      pivot norms or rank test tie (within 1e-10 relative), and both sides have the same groups;
    * the oracle then replays the GPU's choices; applies to n_rhs seeded vectors agree with
      the replayed oracle's, normwise and elementwise, to 100 u on well-conditioned inputs and
      otherwise to c u kappa, kappa the largest condition number of a triangular factor the
      apply solves with (the forward error of the solves);
    * PCG takes the oracle's number of iterations and the solutions agree to sol_tol.
    F: a factor of P made elsewhere (for example by a batched call); closed at the end."""
    F = gpu_factor(P, flags=flags) if F is None else F
    st = F.stats()
    ch = gpu_choices(F, st["levels"] - st["sublevels"])
    orc = O.factor(A, P.d, P.s, P.leaf, P.eps, P.precond)
    assert st["levels"] - st["sublevels"] == orc.L
    c = compare_choices(ch, orc)
    assert_choices(c)
    # replay the GPU's choices in the oracle (the same computation when every choice agrees)
    rep = orc if c["same"] == c["total"] else O.factor(A, P.d, P.s, P.leaf, P.eps, P.precond, replay=ch)
    assert rep.root_size == st["root_size"]
    kappa = max_block_cond(rep)
    bound = 100 * U if well_conditioned else max(100 * U, c_kappa * U * kappa)
    rng = np.random.default_rng(seed)
    worst = worst_max = 0.0
    for _ in range(n_rhs):
        r = rng.standard_normal(P.N)
        zg = _host(F.apply(to_dev(r)))
        zo = O.apply_inverse(rep, r)
        worst = max(worst, rel(zg, zo))
        worst_max = max(worst_max, rel_max(zg, zo))
    print(f"apply: normwise {worst:.2e} elementwise {worst_max:.2e} bound {bound:.2e} "
          f"(kappa {kappa:.2e}, u kappa {U * kappa:.2e})")
    assert worst <= bound and worst_max <= bound, (worst, worst_max, bound)
    # PCG: same iteration count as the replayed oracle, solutions agree
    f = to_dev(P.f)
    ug, itg, rrg = F.pcg(f, 1e-12, 300)
    res = O.pcg(A, P.f, lambda v: O.apply_inverse(rep, v), 1e-12, 300)
    assert res.converged and rrg <= 1e-12
    assert itg == res.iters, (itg, res.iters)
    u = _host(ug)
    assert rel(u, res.u) < sol_tol and rel_max(u, res.u) < sol_tol, (rel(u, res.u), rel_max(u, res.u))
    F.close()
    return dict(choices={k: v for k, v in c.items() if k != "bad_keys"}, apply_err=worst,
                apply_err_max=worst_max, kappa=kappa, iters=itg, sol_err=rel(u, res.u))


def problem(kind, d, s, leaf, eps, seed=0, precond=1, **kw):
    P = make_problem(kind, d, s, seed, leaf, eps, precond=precond, **kw)
    A = O.assemble_fd(d, s, P.a_cells, P.b)
    return P, A


def rel(a, b):
    """Normwise relative difference ||a - b||_2 / ||b||_2."""
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def rel_max(a, b):
    """Elementwise check: max_i |a_i - b_i| / max_i |b_i|."""
    a = np.asarray(a)
    b = np.asarray(b)
    nb = float(np.max(np.abs(b))) if b.size else 0.0
    return float(np.max(np.abs(a - b)) / (nb if nb > 0 else 1.0)) if b.size else 0.0


def max_block_cond(orc_factor):
    """Largest 2-norm condition number over the triangular factors the apply solves with
    (cells' L, block-Jacobi L_g, skeleton L~, root): the forward error of an apply is of the
    order u times this."""
    worst = 1.0
    mats = [orc_factor.root_L]
    for lv in orc_factor.levels:
        mats += [c.L for c in lv.cells] + [g.L for g in lv.groups] + [sk.Lt for sk in lv.skels]
    for M in mats:
        if M.size:
            worst = max(worst, float(np.linalg.cond(M)))
    return worst
