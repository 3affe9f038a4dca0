"""Pins of the CPU oracle against facts fixed by the paper and by mathematics, independent
of the oracle's own formulas (closed forms, library routines, brute force, invariants).

Which mistake each test is meant to catch is stated in its docstring."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle as O
from workloads import make_problem

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


# ---------------------------------------------------------------- assembly (eq. 1.1-1.2)

@pytest.mark.parametrize("d,s", [(2, 7), (3, 4)])
def test_laplacian_spectrum_closed_form(d, s):
    """a = 1, b = 0 gives the textbook 5/7-point Laplacian, whose eigenvalues are
    4 h^-2 sum_k sin^2(pi j_k h / 2), j_k = 1..s. Catches a wrong stencil weight, a wrong
    h, or a wrong neighbour index."""
    A = O.assemble_fd(d, s, np.ones((s + 1,) * d))
    h = 1.0 / (s + 1)
    lam1 = 4.0 / h**2 * np.sin(np.pi * np.arange(1, s + 1) * h / 2) ** 2
    grids = np.meshgrid(*([lam1] * d), indexing="ij")
    expect = np.sort(sum(g.ravel() for g in grids))
    got = np.sort(np.linalg.eigvalsh(A.toarray()))
    assert np.allclose(got, expect, rtol=1e-12, atol=0)


@pytest.mark.parametrize("d,s", [(2, 9), (3, 5)])
def test_energy_identity_cellwise(d, s):
    """u^T A u equals the cell-by-cell energy sum_c a_c 2^(1-d) sum_{e in c} (du_e)^2/h^2
    + sum b u^2. Catches a wrong face-averaging of the cell coefficient or a transposed
    axis in the coefficient array."""
    rng = np.random.default_rng(5)
    a = np.where(rng.random((s + 1,) * d) < 0.5, 1e-2, 1e2) * rng.uniform(0.5, 2.0, (s + 1,) * d)
    b = rng.uniform(0.0, 3.0, s**d)
    A = O.assemble_fd(d, s, a, b)
    for _ in range(3):
        u = rng.standard_normal(s**d)
        assert np.isclose(u @ (A @ u), O.fd_energy(d, s, a, b, u), rtol=1e-12)


@pytest.mark.parametrize("d,s", [(2, 6), (3, 4)])
def test_assembly_structure(d, s):
    """Symmetric, positive diagonal, non-positive couplings only between grid neighbours,
    and nnz = N + 2 d s^(d-1) (s-1)."""
    rng = np.random.default_rng(1)
    a = np.exp(rng.standard_normal((s + 1,) * d))
    A = O.assemble_fd(d, s, a)
    assert abs(A - A.T).max() == 0
    assert A.nnz == s**d + 2 * d * s ** (d - 1) * (s - 1)
    assert np.all(A.diagonal() > 0)
    C = O.dof_coords(d, s)
    Acoo = A.tocoo()
    off = Acoo.row != Acoo.col
    dist = np.abs(C[Acoo.row[off]] - C[Acoo.col[off]]).sum(axis=1)
    assert np.all(dist == 1) and np.all(Acoo.data[off] < 0)


# ------------------------------------------------------------- tree and groups (Sec. 3)

def test_levels():
    assert O.num_levels(64, 8) == 4
    assert O.num_levels(63, 8) == 3
    assert O.num_levels(512, 16) == 6
    assert O.num_levels(64, 4) == 5
    assert O.num_levels(7, 8) == 0


@pytest.mark.parametrize("d,L,m", [(2, 3, 4), (3, 2, 4)])
def test_group_counts_match_paper(d, L, m):
    """With n = 2^L m (s = n - 1) every level-l cell has (2^l m - 1)^d interior points,
    every edge (2D) / face (3D) has (2^l m - 1)^(d-1) points, 3D edges 2^l m - 1 and
    corners 1 (Sec. 3.1 and 3.2); there are 2^(d(L-l)) cells."""
    s = (m << L) - 1
    C = O.dof_coords(d, s)
    allidx = np.arange(s**d)
    for lvl in range(L):
        w = m << lvl
        groups, gclass = O.classify(C, allidx, w)
        ncell = (2 ** (L - lvl)) ** d
        sizes = {c: sorted(len(groups[k]) for k in groups if gclass[k] == c) for c in range(d + 1)}
        assert len(sizes[0]) == ncell and set(sizes[0]) == {(w - 1) ** d}
        assert set(sizes[1]) == {(w - 1) ** (d - 1)}
        if d == 3:
            assert set(sizes[2]) == {w - 1}
        assert set(sizes[d]) == {1}
        # every cell has 3^d - 1 boundary groups inside the domain except at its border
        for k in groups:
            if gclass[k] == 0:
                bks = [bk for bk in O.closure_keys(k) if bk in groups]
                assert len(bks) <= 3**d - 1


# ----------------------------------------------------------------------- ID (Sec. 2.2)

def _lowrank(rng, r, n, decay):
    U, _ = np.linalg.qr(rng.standard_normal((r, r)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    sv = decay ** np.arange(min(r, n))
    return (U[:, : len(sv)] * sv) @ V[: len(sv)]


@pytest.mark.parametrize("r,n", [(40, 12), (12, 30), (96, 15)])
def test_cpqr_matches_lapack_geqp3(r, n):
    """On generic matrices the pivot order and |R_jj| agree with LAPACK's column-pivoted
    QR (scipy.linalg.qr(pivoting=True)). Catches a wrong norm, a wrong reflector, or a
    pivot that is not the largest trailing column."""
    rng = np.random.default_rng(r * 100 + n)
    M = _lowrank(rng, r, n, 0.7) + 1e-3 * rng.standard_normal((r, n))
    k, perm, T, rdiag = O.cpqr_id(M, 0.0)
    _, R, P = sla.qr(M, pivoting=True, mode="economic")
    assert k == min(r, n)
    assert np.array_equal(perm[:k], P[:k])
    assert np.allclose(rdiag, np.abs(np.diag(R))[:k], rtol=1e-10)


@pytest.mark.parametrize("eps", [1e-2, 1e-4, 1e-6, 1e-9])
def test_cpqr_id_error_and_monotone_rank(eps):
    """||M[:, redundant] - M[:, skeleton] T|| is O(eps |R_11|) and the rank does not grow
    as eps grows (Sec. 2.2)."""
    rng = np.random.default_rng(7)
    M = _lowrank(rng, 80, 20, 0.5)
    k, perm, T, rdiag = O.cpqr_id(M, eps)
    err = np.linalg.norm(M[:, perm[k:]] - M[:, perm[:k]] @ T, 2) if k < 20 else 0.0
    assert err <= 10 * np.sqrt(20) * eps * rdiag[0]
    assert np.all(rdiag[:k] > eps * rdiag[0])
    k_looser, *_ = O.cpqr_id(M, eps * 10)
    assert k_looser <= k


def test_cpqr_exact_and_degenerate():
    """eps = 0 reconstructs exactly; a zero matrix has rank 0; forced replay of the
    oracle's own choices reproduces T; fewer rows than columns caps the rank."""
    rng = np.random.default_rng(3)
    M = rng.standard_normal((10, 6)) @ rng.standard_normal((6, 9))
    k, perm, T, _ = O.cpqr_id(M, 0.0)
    assert np.allclose(M[:, perm[k:]], M[:, perm[:k]] @ T, atol=1e-10 * np.abs(M).max())
    k0, _, T0, _ = O.cpqr_id(np.zeros((5, 4)), 1e-3)
    assert k0 == 0 and T0.shape == (0, 4)
    k1, p1, T1, _ = O.cpqr_id(M, 1e-3)
    k2, p2, T2, _ = O.cpqr_id(M, 1e-3, forced=(k1, p1))
    assert k2 == k1 and np.array_equal(p1, p2) and np.allclose(T1, T2, rtol=1e-12, atol=1e-14)
    k3, *_ = O.cpqr_id(rng.standard_normal((3, 8)), 1e-12)
    assert k3 == 3


# ------------------------------------------------- factorization end to end (Sec. 3)

def _prob(d, s, leaf, eps, precond=1, kind="two_valued", seed=0, **kw):
    P = make_problem(kind, d, s, seed, leaf, eps, precond=precond, **kw)
    A = O.assemble_fd(d, s, P.a_cells, P.b)
    return P, A


@pytest.mark.parametrize("d,s,leaf,precond", [
    (2, 16, 4, 1), (2, 13, 4, 1), (2, 20, 4, 0), (2, 31, 8, 1), (3, 7, 2, 1), (3, 10, 4, 1), (3, 9, 2, 0)])
def test_eps0_is_exact_nested_dissection(d, s, leaf, precond):
    """eps = 0 keeps every column, so F = A up to roundoff: F^-1 f agrees with a dense
    Cholesky solve and PCG stops after one product (ND reduction of the method).
    Catches any error in E, C, K, the root or the apply order."""
    P, A = _prob(d, s, leaf, 0.0, precond, lo=0.5, hi=2.0)
    F = O.factor(A, d, s, leaf, 0.0, precond)
    u = O.dense_solve(A, P.f)
    z = O.apply_inverse(F, P.f)
    assert np.linalg.norm(z - u) / np.linalg.norm(u) < 1e-12
    res = O.pcg(A, P.f, lambda v: O.apply_inverse(F, v), 1e-12, 5)
    assert res.iters == 1 and res.converged


def test_degenerate_tree_is_dense_cholesky():
    """s < m: no levels, the root is all of A and F^-1 is the dense solve."""
    P, A = _prob(2, 7, 8, 1e-3)
    F = O.factor(A, 2, 7, 8, 1e-3)
    assert F.L == 0 and F.root_size == 49
    assert np.allclose(F.root_L @ F.root_L.T, A.toarray(), rtol=1e-13, atol=1e-9)
    u = O.dense_solve(A, P.f)
    assert np.linalg.norm(O.apply_inverse(F, P.f) - u) / np.linalg.norm(u) < 1e-13


def _dense_R(F, lv, N):
    """R_l = E_l C_l K_l as dense N x N matrices built directly from the paper's
    definitions: E_I from eq. (2.1), C_I from eq. (2.3), K_I = Z_I E_Itilde
    with Z_I from eq. (2.2); E_l, C_l, K_l are the products over their index sets."""
    def elim(I, B, L, W):
        Em = np.eye(N)
        Linv_T = sla.solve_triangular(L, np.eye(len(I)), lower=True).T      # L^-T
        Em[np.ix_(I, I)] = Linv_T
        if len(B):
            Em[np.ix_(I, B)] = -Linv_T @ W                                    # -A_II^-1 A_BI^T
        return Em
    E = np.eye(N)
    for c in lv.cells:
        E = E @ elim(c.I, c.B, c.L, c.W)
    C = np.eye(N)
    for g in lv.groups:
        Cg = np.eye(N)
        Cg[np.ix_(g.idx, g.idx)] = sla.solve_triangular(g.L, np.eye(len(g.idx)), lower=True).T
        C = C @ Cg
    K = np.eye(N)
    for sk in lv.skels:
        if len(sk.tilde) == 0:
            continue
        Z = np.eye(N)
        Z[np.ix_(sk.hat, sk.tilde)] = -sk.T
        K = K @ Z @ elim(sk.tilde, sk.hat, sk.Lt, sk.Wt)
    return E @ C @ K


@pytest.mark.parametrize("d,s,leaf,eps,precond", [(2, 12, 3, 1e-2, 1), (2, 12, 3, 1e-2, 0), (3, 6, 2, 1e-2, 1)])
def test_apply_equals_paper_operator_product(d, s, leaf, eps, precond):
    """The sweep apply equals R_0 ... R_{L-1} A_L^-1 R_{L-1}^T ... R_0^T (eq. (3.2)) with
    every R_l assembled densely from the paper's matrix definitions, and R^T A R equals
    the identity outside S_L and A_L = B_L B_L^T on S_L up to the dropped ID error
    (eq. (3.1)). Catches a swapped sweep order, a missing transpose or a wrong T sign."""
    P, A = _prob(d, s, leaf, eps, precond)
    F = O.factor(A, d, s, leaf, eps, precond)
    N = P.N
    Rs = [_dense_R(F, lv, N) for lv in F.levels]
    Rall = np.eye(N)
    for R in Rs:
        Rall = Rall @ R
    ALinv = np.eye(N)
    root = F.root_idx
    ALinv[np.ix_(root, root)] = np.linalg.inv(F.root_L @ F.root_L.T)
    Finv = Rall @ ALinv @ Rall.T
    rng = np.random.default_rng(0)
    for _ in range(2):
        r = rng.standard_normal(N)
        z = O.apply_inverse(F, r)
        assert np.linalg.norm(z - Finv @ r) <= 1e-10 * np.linalg.norm(z)
    # eq. (3.1): R^T A R ~ blockdiag(I, A_L) with an O(eps) defect in the scaled norm
    RAR = Rall.T @ A.toarray() @ Rall
    target = np.eye(N)
    target[np.ix_(root, root)] = F.root_L @ F.root_L.T
    defect = np.linalg.norm(RAR - target, 2)
    assert defect < 50 * eps * np.linalg.norm(target, 2) + 1e-9


def test_eps0_operator_product_is_exact():
    """At eps = 0 the congruence R^T A R is exactly blockdiag(I, A_L) (eq. (3.1))."""
    P, A = _prob(2, 12, 3, 0.0, 1)
    F = O.factor(A, 2, 12, 3, 0.0, 1)
    Rall = np.eye(P.N)
    for lv in F.levels:
        Rall = Rall @ _dense_R(F, lv, P.N)
    RAR = Rall.T @ A.toarray() @ Rall
    target = np.eye(P.N)
    target[np.ix_(F.root_idx, F.root_idx)] = F.root_L @ F.root_L.T
    assert np.abs(RAR - target).max() < 1e-9 * np.abs(target).max()


def test_phif_skeleton_closed_form():
    """After block Jacobi the group's diagonal block is I, so the skeleton elimination
    sees [[I + T^T T, -T^T], [-T, I]] and leaves (I + T T^T)^-1 on the skeleton
    (closed form of the error-analysis section; Woodbury)."""
    P, A = _prob(2, 31, 8, 1e-3, 1)
    F = O.factor(A, 2, 31, 8, 1e-3, 1)
    checked = 0
    for lv in F.levels:
        for sk in lv.skels:
            k, n = len(sk.hat), len(sk.group)
            if k == 0 or k == n:
                continue
            T = sk.T
            assert np.allclose(sk.Lt @ sk.Lt.T, np.eye(n - k) + T.T @ T, rtol=1e-12, atol=1e-12)
            assert np.allclose(sk.Lt @ sk.Wt, -T.T, rtol=1e-12, atol=1e-12)
            schur = np.eye(k) - sk.Wt.T @ sk.Wt
            assert np.allclose(schur, np.linalg.inv(np.eye(k) + T @ T.T), rtol=1e-10, atol=1e-12)
            checked += 1
    assert checked > 10


def test_schur_complements_spd_and_Finv_symmetric():
    """Cell Schur complements stay SPD and F^-1 is symmetric positive definite
    (generalized Cholesky, eq. (3.3))."""
    P, A = _prob(2, 24, 4, 1e-2, 1, lo=1e-2, hi=1e2)
    F = O.factor(A, 2, 24, 4, 1e-2, 1, check_spd=True)
    assert len(F.schur_min_eig) > 0 and min(F.schur_min_eig) > 0
    rng = np.random.default_rng(2)
    x, y = rng.standard_normal(P.N), rng.standard_normal(P.N)
    fx, fy = O.apply_inverse(F, x), O.apply_inverse(F, y)
    assert abs(x @ fy - y @ fx) <= 1e-12 * np.linalg.norm(fx) * np.linalg.norm(y)
    assert x @ fx > 0


def _solve_error(A, F, iters=40, seed=0):
    """||I - F^-1 A||_2 by power iteration (the solve error e_s of Sec. 4 up to similarity)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(A.shape[0])
    v /= np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        wv = v - O.apply_inverse(F, A @ v)
        lam = np.linalg.norm(wv)
        if lam == 0:
            return 0.0
        v = wv / lam
    return lam


def test_preconditioning_improves_solve_error_and_iterations():
    """Qualitative claim of Tables 1-2: on a high-contrast medium PHIF has a much smaller
    solve error and needs fewer CG iterations than HIF at the same eps (parity unpinned
    numerically: the paper's draws, sizes and leaf size differ)."""
    P, A = _prob(2, 47, 6, 1e-3, 1, kind="paper", seed=4)
    Fp = O.factor(A, 2, 47, 6, 1e-3, 1)
    Fh = O.factor(A, 2, 47, 6, 1e-3, 0)
    es_p, es_h = _solve_error(A, Fp), _solve_error(A, Fh)
    assert es_p < es_h
    it_p = O.pcg(A, P.f, lambda v: O.apply_inverse(Fp, v), 1e-12, 300).iters
    it_h = O.pcg(A, P.f, lambda v: O.apply_inverse(Fh, v), 1e-12, 300).iters
    assert it_p <= it_h


def test_error_decreases_with_eps():
    """A tighter ID tolerance gives a smaller solve error and at least as many skeletons."""
    P, A = _prob(2, 31, 4, 1e-2, 1, kind="lognormal", seed=1, sigma=2.0)
    prev_es, prev_root = None, None
    for eps in (1e-1, 1e-3, 1e-6):
        F = O.factor(A, 2, 31, 4, eps, 1)
        es = _solve_error(A, F)
        if prev_es is not None:
            assert es < prev_es
            assert F.root_size >= prev_root
        prev_es, prev_root = es, F.root_size


def test_not_spd_is_reported():
    """A strongly negative reaction term makes the first interior block indefinite: the
    factorization stops with a located loss-of-positive-definiteness error."""
    P, A = _prob(2, 16, 4, 1e-3, 1, lo=1.0, hi=1.0)
    A = (A - 1e6 * sp.eye(P.N)).tocsr()
    with pytest.raises(O.NotSPDError) as ei:
        O.factor(A, 2, 16, 4, 1e-3, 1)
    assert ei.value.level == 0 and ei.value.step == "E"


# ------------------------------------------------------------------------- CG (Sec. 4)

def test_unpreconditioned_cg_matches_scipy():
    """With M = I the iterates are textbook CG: identical to scipy.sparse.linalg.cg after
    the same number of iterations."""
    P, A = _prob(2, 20, 4, 1e-3, 1, lo=0.5, hi=2.0)
    for it in (3, 12):
        ours = O.pcg(A, P.f, None, rtol=1e-300, maxit=it)
        ref, _ = spla.cg(A, P.f, x0=np.zeros(P.N), rtol=1e-300, atol=0.0, maxiter=it)
        assert ours.iters == it
        assert np.linalg.norm(ours.u - ref) <= 1e-11 * np.linalg.norm(ref)


def test_pcg_converges_with_factor():
    P, A = _prob(2, 64, 8, 1e-3, 1)
    F = O.factor(A, 2, 64, 8, 1e-3, 1)
    res = O.pcg(A, P.f, lambda v: O.apply_inverse(F, v), 1e-12, 100)
    assert res.converged and res.iters < 20 and res.true_relres < 1e-10


# ---------------------------------------------------------------------------------------
# Adjoint gradient with respect to theta = log a
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("d,s", [(2, 7), (3, 4)])
def test_grad_cell_form_sums_to_the_matrix(d, s):
    """sum_c -grad_c(x, y) = sum_c a_c x^T (dA/da_c) y = x^T K(a) y: the per-cell edge form of
    grad_log_a, summed over the cells, reproduces the assembled operator (without b)."""
    rng = np.random.default_rng(5)
    a = np.exp(rng.standard_normal((s + 1,) * d))
    A = O.assemble_fd(d, s, a, None)
    x = rng.standard_normal(s ** d)
    y = rng.standard_normal(s ** d)
    g = O.grad_log_a(d, s, a, y, x)
    ref = float(x @ (A @ y))
    assert abs(-g.sum() - ref) <= 1e-12 * abs(ref)


def test_grad_matches_central_differences():
    """dL/dtheta of L = 0.5 |u - u_obs|^2, A(exp theta) u = f, from the adjoint solution
    (dense solves on a 6 x 6 grid) equals central differences of L in every theta_c."""
    d, s = 2, 6
    rng = np.random.default_rng(6)
    theta = rng.standard_normal((s + 1,) * d)
    f = rng.standard_normal(s * s)
    u_obs = rng.standard_normal(s * s)

    def loss(th):
        A = O.assemble_fd(d, s, np.exp(th), None)
        u = O.dense_solve(A, f)
        return 0.5 * float(np.sum((u - u_obs) ** 2)), A, u

    L0, A, u = loss(theta)
    lam = O.dense_solve(A, u - u_obs)
    g = O.grad_log_a(d, s, np.exp(theta), u, lam)
    fd = np.zeros_like(theta)
    delta = 1e-5
    for idx in np.ndindex(theta.shape):
        tp = theta.copy()
        tm = theta.copy()
        tp[idx] += delta
        tm[idx] -= delta
        fd[idx] = (loss(tp)[0] - loss(tm)[0]) / (2 * delta)
    assert np.linalg.norm(g - fd) <= 1e-7 * np.linalg.norm(fd)
