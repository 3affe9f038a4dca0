"""Independent problems factored in one call (rhif_factor_batch): the problems advance level
by level together and every elimination, block-Jacobi and skeletonization kernel of a level
is one launch over the blocks of all problems; their applies and PCG solves run jointly too
(rhif_apply_batch, rhif_pcg_solve_batch). Each problem is checked against the oracle (the
full parity protocol) and against what rhif_factor, rhif_apply and rhif_pcg_solve give for it
alone."""
import numpy as np
import pytest

from tests.gpu_common import gpu_choices, gpu_csr, parity_check, problem, rel, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _batch(probs, precision=0, flags=0):
    from paper_1808_01364_amd import rhif
    P0 = probs[0]
    csrs = [gpu_csr(P) for P in probs]
    Fs = rhif.factor_batch([(P.d, P.s, c) for P, c in zip(probs, csrs)], P0.leaf, P0.eps, P0.precond,
                           precision, flags)
    return csrs, Fs


def _against_single(probs, precision=0, flags=0, seed=5):
    """Every problem of the batch against its lone factorization: the same ranks and pivot
    orders at every level, the same root, and bitwise the same applies and PCG solutions, both
    problem by problem on the batch's handles and in the joint apply and joint PCG over all
    of them (rhif_apply_batch, rhif_pcg_solve_batch). The handles are destroyed in another
    order than made."""
    from paper_1808_01364_amd import rhif
    torch = torch_cuda()
    csrs, Fs = _batch(probs, precision, flags)
    rng = np.random.default_rng(seed)
    singles, rs, z1s, sols = [], [], [], []
    for P, c, Fb in zip(probs, csrs, Fs):
        F1 = rhif.Factor(P.d, P.s, c, P.leaf, P.eps, P.precond, precision=precision, flags=flags)
        singles.append(F1)
        s1, sb = F1.stats(), Fb.stats()
        for key in ("levels", "root_size", "n_active", "n_skel", "sum_rank", "max_rank", "factor_bytes"):
            assert s1[key] == sb[key], (P.name, key, s1[key], sb[key])
        ch1, chb = gpu_choices(F1, s1["levels"]), gpu_choices(Fb, sb["levels"])
        assert ch1.keys() == chb.keys()
        for key in ch1:
            assert ch1[key][0] == chb[key][0] and np.array_equal(ch1[key][1], chb[key][1]), (P.name, key)
        r = to_dev(rng.standard_normal(P.N))
        rs.append(r)
        z1 = F1.apply(r)
        z1s.append(z1)
        assert torch.equal(z1, Fb.apply(r)), P.name
        f = to_dev(P.f)
        u1, i1, r1 = F1.pcg(f, 1e-12, 300)
        ub, ib, rb = Fb.pcg(f, 1e-12, 300)
        assert i1 == ib and r1 == rb and torch.equal(u1, ub), P.name
        sols.append((f, u1, i1, r1))
    zb = rhif.apply_batch(Fs, rs)
    for P, z1, z in zip(probs, z1s, zb):
        assert torch.equal(z1, z), (P.name, rel(z.cpu().numpy(), z1.cpu().numpy()))
    out = rhif.pcg_batch(Fs, [f for f, _, _, _ in sols], 1e-12, 300)
    for P, (f, u1, i1, r1), (u, it, rr) in zip(probs, sols, out):
        print(f"{P.name}: iterations {it} (alone {i1}), "
              f"relres {rr:.2e}, joint solution vs alone {rel(u.cpu().numpy(), u1.cpu().numpy()):.1e}", flush=True)
        assert it == i1 and rr == r1 and rr <= 1e-12 and torch.equal(u, u1), P.name
    for F1 in singles:
        F1.close()
    for Fb in reversed(Fs):
        Fb.close()


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_batch_2d_uneven_sides(precision):
    """Five 2D problems with sides 64, 96, 40, 33, 128 (ragged cells, 2 to 4 levels, so the
    roots fall on different levels) and different fields."""
    probs = [problem("lognormal", 2, s, 8, 1e-6, seed=k, sigma=2.0)[0]
             for k, s in enumerate((64, 96, 40, 33, 128))]
    _against_single(probs, precision)


@pytest.mark.parametrize("flags", [0, 16, 32], ids=["default", "global_staging", "skel_multi"])
def test_batch_3d(flags):
    """Three 3D problems (sides 12, 16, 9; leaf 4; two-valued 1e-3/1e3 field, b = 1e-2), also
    with the global-memory forms and the multi-workgroup ID forced."""
    probs = [problem("two_valued", 3, s, 4, 1e-3, seed=k, lo=1e-3, hi=1e3, b_const=1e-2)[0]
             for k, s in enumerate((12, 16, 9))]
    _against_single(probs, 0, flags)


def test_batch_many_groups():
    """Twelve 64^2 problems (leaf 8): 1344 level-0 edges in one launch, which takes the
    many-groups form of the skeletonization that none of them takes alone."""
    probs = [problem("two_valued", 2, 64, 8, 1e-3, seed=k)[0] for k in range(12)]
    _against_single(probs)


@pytest.mark.timeout(300)
def test_batch_against_oracle():
    """Each problem of a batch (2D 64^2 two-valued, 2D 48^2 log-normal, 2D 33^2 constant; leaf
    8, eps 1e-6 for all, as the options are shared) against the oracle: the parity protocol of
    the lone factorization (identical choices or certified ties, applies within c u kappa of
    the replayed oracle, same PCG iteration count, solutions within 1e-10)."""
    pa = [problem("two_valued", 2, 64, 8, 1e-6, seed=0),
          problem("lognormal", 2, 48, 8, 1e-6, seed=1, sigma=2.0),
          problem("constant", 2, 33, 8, 1e-6, seed=2)]
    probs = [P for P, _ in pa]
    _, Fs = _batch(probs)
    # the joint PCG against the oracle's own solve of each problem
    from paper_1808_01364_amd import rhif
    import oracle as O
    out = rhif.pcg_batch(Fs, [to_dev(P.f) for P in probs], 1e-12, 300)
    for (P, A), (u, it, rr) in zip(pa, out):
        ref = O.pcg(A, P.f, lambda v, F=O.factor(A, P.d, P.s, P.leaf, P.eps, P.precond): O.apply_inverse(F, v),
                    1e-12, 300)
        e = rel(u.cpu().numpy(), ref.u)
        print(f"{P.name}: joint PCG {it} iterations (oracle {ref.iters}), error vs oracle {e:.1e}", flush=True)
        assert rr <= 1e-12 and e <= 1e-10
    for (P, A), F in zip(pa, Fs):
        out = parity_check(P, A, F=F, well_conditioned=P.meta["kind"] == "constant")
        print(P.name, out, flush=True)


def test_batch_one_equals_factor():
    """A batch of one is rhif_factor itself: bitwise the same apply."""
    from paper_1808_01364_amd import rhif
    torch = torch_cuda()
    P, _ = problem("lognormal", 2, 96, 8, 1e-6, seed=3, sigma=2.0)
    c = gpu_csr(P)
    (Fb,) = rhif.factor_batch([(2, P.s, c)], P.leaf, P.eps)
    F1 = rhif.Factor(2, P.s, c, P.leaf, P.eps)
    r = to_dev(np.random.default_rng(0).standard_normal(P.N))
    assert torch.equal(F1.apply(r), Fb.apply(r))
    F1.close()
    Fb.close()


def test_batch_not_spd_fails_whole_call():
    """A problem that loses positive definiteness (negative coefficients) fails the whole call
    with ENOTSPD and returns no handle; the next call works."""
    from paper_1808_01364_amd import rhif
    torch_cuda()
    good, _ = problem("two_valued", 2, 32, 8, 1e-3, seed=0)
    bad, _ = problem("constant", 2, 32, 8, 1e-3, seed=1)
    bad.a_cells[:] = -1.0
    c1, c2 = gpu_csr(good), gpu_csr(bad)
    with pytest.raises(rhif.NotSPD, match="batch"):
        rhif.factor_batch([(2, 32, c1), (2, 32, c2)], 8, 1e-3)
    (F,) = rhif.factor_batch([(2, 32, c1)], 8, 1e-3)
    F.close()


def test_joint_calls_need_the_whole_batch():
    """The joint apply and PCG take exactly the handles of one factor_batch call, in its order,
    while all of them live; anything else is refused before any device work."""
    from paper_1808_01364_amd import rhif
    torch_cuda()
    probs = [problem("two_valued", 2, 32, 8, 1e-3, seed=k)[0] for k in range(3)]
    csrs, Fs = _batch(probs)
    rs = [to_dev(P.f) for P in probs]
    with pytest.raises(rhif.RhifError, match="every handle"):
        rhif.apply_batch(Fs[:2], rs[:2])
    with pytest.raises(rhif.RhifError, match="every handle"):
        rhif.apply_batch(Fs[::-1], rs[::-1])
    F1 = rhif.Factor(2, 32, csrs[0], 8, 1e-3)
    with pytest.raises(rhif.RhifError, match="rhif_factor_batch"):
        rhif.pcg_batch([F1, Fs[1], Fs[2]], rs)
    F1.close()
    rhif.apply_batch(Fs, rs)
    Fs[1].close()
    with pytest.raises(RuntimeError):
        rhif.apply_batch(Fs, rs)
    Fs[0].close()
    Fs[2].close()
