"""Helpers shared by the GPU tests: run a seeded problem through the HIP library and
through the CPU oracle on the same inputs."""
import numpy as np

import oracle as O
from workloads import make_problem


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


def compare_choices(gpu, orc_factor):
    """Count groups whose rank or skeleton set differ between the GPU and the oracle."""
    diff_rank = diff_set = total = 0
    for lv in orc_factor.levels:
        for sk in lv.skels:
            key = (lv.level, int(sk.group[0]))
            total += 1
            if key not in gpu:
                diff_rank += 1
                continue
            k, perm = gpu[key]
            if k != len(sk.hat):
                diff_rank += 1
            elif set(perm[:k].tolist()) != set(sk.perm[:k].tolist()):
                diff_set += 1
    return total, diff_rank, diff_set


def problem(kind, d, s, leaf, eps, seed=0, precond=1, **kw):
    P = make_problem(kind, d, s, seed, leaf, eps, precond=precond, **kw)
    A = O.assemble_fd(d, s, P.a_cells, P.b)
    return P, A


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))
