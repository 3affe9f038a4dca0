"""Host-side checks (no GPU): the Python binding refuses tensors whose dtype, size, layout or
device would make a kernel read or write out of bounds, before any device work; and the
tie certification the GPU parity tests use tells a tie of the ID's pivot norms or rank test
from a wrong choice."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1808_01364_amd import rhif
from tests.gpu_common import _certify, compare_choices


def test_assemble_rejects_bad_tensors():
    n = 8
    good_cpu = torch.ones((n + 1) ** 2, dtype=torch.float64)
    with pytest.raises(ValueError, match="float64"):
        rhif.assemble_fd(2, n, torch.ones((n + 1) ** 2, dtype=torch.float32))
    with pytest.raises(ValueError, match="elements"):
        rhif.assemble_fd(2, n, torch.ones(n * n, dtype=torch.float64))
    with pytest.raises(ValueError, match="contiguous"):
        rhif.assemble_fd(2, n, torch.ones(2 * (n + 1) ** 2, dtype=torch.float64)[::2])
    with pytest.raises(ValueError, match="GPU"):
        rhif.assemble_fd(2, n, good_cpu)


def test_gradient_and_factor_reject_bad_tensors():
    n = 6
    a = torch.ones((n + 1) ** 2, dtype=torch.float64)
    with pytest.raises(ValueError, match="u must have"):
        rhif.grad_log_a(2, n, a, torch.zeros(n * n + 1, dtype=torch.float64), torch.zeros(n * n, dtype=torch.float64))
    with pytest.raises(ValueError, match="row_ptr"):
        rhif.Factor(2, n, (torch.zeros(n * n, dtype=torch.int32), torch.zeros(1, dtype=torch.int32),
                           torch.zeros(1, dtype=torch.float64)), 4, 1e-3)
    with pytest.raises(ValueError, match="col must have"):
        rhif.Factor(2, n, (torch.zeros(n * n + 1, dtype=torch.int32), torch.zeros(7, dtype=torch.int32),
                           torch.zeros(7, dtype=torch.float64)), 4, 1e-3)


def test_factor_methods_check_before_launch():
    F = object.__new__(rhif.Factor)       # no handle: a check that passed would fail later
    F._h, F.N = None, 64
    with pytest.raises(ValueError, match="shape"):
        F.apply(torch.zeros(63, dtype=torch.float64))
    with pytest.raises(ValueError, match="float64"):
        F.apply(torch.zeros(64, dtype=torch.float32))
    with pytest.raises(ValueError, match="out must have the shape"):
        F.apply(torch.zeros(2, 64, dtype=torch.float64), out=torch.zeros(64, dtype=torch.float64))
    with pytest.raises(ValueError, match="float64"):
        F.pcg(torch.zeros(64, dtype=torch.float32))
    with pytest.raises(ValueError, match="out must have"):
        F.pcg(torch.zeros(64, dtype=torch.float64), out=torch.zeros(32, dtype=torch.float64))
    with pytest.raises(ValueError, match="x must have"):
        F.matvec(torch.zeros(65, dtype=torch.float64))


def _one_skel(M, eps):
    """A stand-in for an oracle skeleton record of the ID of M."""
    tr = {}
    k, perm, T, rdiag = O.cpqr_id(M, eps, trace=tr)

    class Sk:
        pass
    sk = Sk()
    sk.perm, sk.hat, sk.rdiag, sk.trace = perm, perm[:k], rdiag, tr
    return sk


def test_tie_certification():
    rng = np.random.default_rng(0)
    M = rng.standard_normal((12, 5))
    M[:, 3] = M[:, 1]                    # columns 1 and 3 have equal norms throughout
    M[:, 1] *= 10.0
    M[:, 3] *= 10.0
    sk = _one_skel(M, 1e-3)
    assert sk.perm[0] == 1               # the first of the two largest columns
    other = np.array([3, 1] + [c for c in sk.perm if c not in (1, 3)])
    assert _certify(sk, len(sk.hat), other, 1e-3, 1e-10) == "pivot"
    wrong = np.array([0] + [c for c in sk.perm if c != 0])
    assert _certify(sk, len(sk.hat), wrong, 1e-3, 1e-10) is None
    # a rank that differs where the rank test is not a tie is refused
    assert _certify(sk, len(sk.hat) - 1, sk.perm, 1e-3, 1e-10) is None
    # eps set exactly at a ratio |R_jj|/|R_11|: a rank one lower is a tie of the rank test
    eps = float(sk.rdiag[2] / sk.rdiag[0])
    sk2 = _one_skel(M, eps)
    assert len(sk2.hat) == 2
    assert _certify(sk2, 3, sk2.perm, eps, 1e-10) == "rank"


def test_compare_choices_counts_one_sided_groups():
    from workloads import make_problem
    P = make_problem("two_valued", 2, 16, 0, 4, 1e-3)
    A = O.assemble_fd(2, 16, P.a_cells, P.b)
    F = O.factor(A, 2, 16, 4, 1e-3)
    gpu = {(lv.level, int(sk.group[0])): (len(sk.hat), np.asarray(sk.perm)) for lv in F.levels for sk in lv.skels}
    c = compare_choices(gpu, F)
    assert c["same"] == c["total"] and c["bad"] == 0 and c["missing"] == 0 and c["extra"] == 0
    key = next(iter(gpu))
    gpu2 = dict(gpu)
    del gpu2[key]
    gpu2[(99, 0)] = (1, np.arange(3))
    c2 = compare_choices(gpu2, F)
    assert c2["missing"] == 1 and c2["extra"] == 1
