"""Pins of the oracle's accuracy measures (Sec. 4: e_a = ||A - F|| / ||A|| and
e_s = ||I - G^-1 A G^-T||, by power iteration to 1e-2) and of the pieces they use: the two
halves G^-1 and G^-T of F^-1 (eq. (3.2), (3.3)) and the forward product F x = G G^T x.
Each is pinned by something other than itself: the composition of the halves, exactness at
eps = 0 (F = A), the inverse of the dense F^-1, dense 2-norms, and Proposition 1.1."""
import numpy as np
import pytest

import oracle as O
from workloads import make_problem


def _prob(d, s, leaf, eps, precond=1, kind="two_valued", seed=0):
    P = make_problem(kind, d, s, seed, leaf, eps, lo=1e-2, hi=1e2)
    A = O.assemble_fd(d, s, P.a_cells, P.b)
    return P, A, O.factor(A, d, s, leaf, eps, precond)


def _dense(op, n):
    return np.column_stack([op(e) for e in np.eye(n)])


@pytest.mark.parametrize("d,s,leaf,eps,precond", [(2, 24, 4, 1e-3, 1), (3, 8, 2, 1e-2, 1), (2, 20, 4, 1e-2, 0)])
def test_halves_compose_to_the_apply(d, s, leaf, eps, precond):
    P, A, F = _prob(d, s, leaf, eps, precond)
    r = np.random.default_rng(1).standard_normal(P.N)
    assert np.array_equal(O.apply_ginv_t(F, O.apply_ginv(F, r)), O.apply_inverse(F, r))


@pytest.mark.parametrize("d,s,leaf,precond", [(2, 24, 4, 1), (2, 19, 4, 0), (3, 9, 2, 1)])
def test_forward_at_eps0_is_A(d, s, leaf, precond):
    """eps = 0 is exact nested dissection, so F = A."""
    P, A, F = _prob(d, s, leaf, 0.0, precond)
    x = np.random.default_rng(2).standard_normal(P.N)
    assert np.linalg.norm(O.apply_forward(F, x) - A @ x) <= 1e-13 * np.linalg.norm(A @ x)


def test_forward_is_the_inverse_of_the_dense_apply():
    """F from apply_forward equals the inverse of the dense F^-1 (whose columns come from the
    apply, itself pinned against the product of the paper's operators), and is symmetric."""
    P, A, F = _prob(2, 10, 2, 1e-2)
    Finv = _dense(lambda v: O.apply_inverse(F, v), P.N)
    Fd = _dense(lambda v: O.apply_forward(F, v), P.N)
    ref = np.linalg.inv(Finv)
    assert np.linalg.norm(Fd - ref) <= 1e-10 * np.linalg.norm(ref)
    assert np.linalg.norm(Fd - Fd.T) <= 1e-12 * np.linalg.norm(Fd)
    x = np.random.default_rng(3).standard_normal(P.N)
    assert np.linalg.norm(O.apply_inverse(F, O.apply_forward(F, x)) - x) <= 1e-12 * np.linalg.norm(x)


def test_power_norm_of_an_indefinite_matrix():
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(rng.standard_normal((60, 60)))
    lam = np.concatenate([[-5.0, 3.0], rng.uniform(-1, 1, 58)])
    M = (Q * lam) @ Q.T
    est = O.rhif_oracle._power_norm(lambda v: M @ v, 60)
    assert abs(est - 5.0) <= 0.02 * 5.0


@pytest.mark.parametrize("precond", [1, 0])
def test_estimates_match_dense_norms(precond):
    """e_a and e_s from power iteration agree with the dense 2-norms of their definitions."""
    P, A, F = _prob(2, 12, 4, 1e-2, precond)
    n = P.N
    Ad = A.toarray()
    Fd = _dense(lambda v: O.apply_forward(F, v), n)
    Gi = _dense(lambda v: O.apply_ginv(F, v), n)
    Git = _dense(lambda v: O.apply_ginv_t(F, v), n)
    assert np.linalg.norm(Git - Gi.T) <= 1e-12 * np.linalg.norm(Gi)
    ea = np.linalg.norm(Ad - Fd, 2) / np.linalg.norm(Ad, 2)
    es = np.linalg.norm(np.eye(n) - Gi @ Ad @ Git, 2)
    ea_est, es_est = O.estimate_ea(A, F), O.estimate_es(A, F)
    assert abs(ea_est - ea) <= 0.05 * ea
    assert abs(es_est - es) <= 0.05 * es


def test_proposition_1_1():
    """Block Jacobi before compression (Proposition 1.1): for an SPD A = C [[I, B^T], [B, I]] C^T
    and F built with the truncated SVD of B, ||I - G^-1 A G^-T|| <= ||B - B~|| = eps; the
    estimator finds that norm."""
    rng = np.random.default_rng(5)
    n1, n2, k = 30, 24, 6
    U, _ = np.linalg.qr(rng.standard_normal((n2, n2)))
    V, _ = np.linalg.qr(rng.standard_normal((n1, n1)))
    sv = np.sort(rng.uniform(0.0, 0.9, n2))[::-1]
    B = (U * sv) @ V[:n2, :]
    Bt = (U[:, :k] * sv[:k]) @ V[:k, :]
    eps = np.linalg.norm(B - Bt, 2)
    C1 = np.linalg.cholesky(np.cov(rng.standard_normal((n1, 3 * n1))) + 0.1 * np.eye(n1))
    C2 = np.linalg.cholesky(np.cov(rng.standard_normal((n2, 3 * n2))) + 0.1 * np.eye(n2))
    C = np.block([[C1, np.zeros((n1, n2))], [np.zeros((n2, n1)), C2]])
    Amid = np.block([[np.eye(n1), B.T], [B, np.eye(n2)]])
    Fmid = np.block([[np.eye(n1), Bt.T], [Bt, np.eye(n2)]])
    A = C @ Amid @ C.T
    G = np.linalg.cholesky(C @ Fmid @ C.T)
    S = np.linalg.solve(G, np.linalg.solve(G, A).T).T      # G^-1 A G^-T
    es = np.linalg.norm(np.eye(n1 + n2) - S, 2)
    assert es <= eps * (1 + 1e-10)
    assert np.linalg.cond(S) <= (1 + eps) / (1 - eps) * (1 + 1e-10)
    est = O.rhif_oracle._power_norm(lambda v: v - S @ v, n1 + n2)
    assert abs(est - es) <= 0.02 * es


def test_block_jacobi_improves_the_solve_error():
    """The trend of Sec. 4: PHIF improves e_s over HIF by orders of magnitude at comparable
    e_a = O(eps) (high-contrast medium, eps 1e-3)."""
    P, A, Fp = _prob(2, 32, 4, 1e-3, 1)
    Fh = O.factor(A, 2, 32, 4, 1e-3, 0)
    es_p, es_h = O.estimate_es(A, Fp), O.estimate_es(A, Fh)
    ea_p, ea_h = O.estimate_ea(A, Fp), O.estimate_ea(A, Fh)
    assert es_p * 10 < es_h
    assert ea_p < 1e-1 and ea_h < 1e-1
