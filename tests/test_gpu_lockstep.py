"""Independent problems factored in one call (rhif_factor_batch): the problems advance level
by level together and every elimination, block-Jacobi and skeletonization kernel of a level
is one launch over the blocks of all problems. Each problem's factor is checked against the
oracle (the full parity protocol) and against the factor rhif_factor makes of it alone."""
import numpy as np
import pytest

from tests.gpu_common import U, gpu_choices, gpu_csr, parity_check, problem, rel, rel_max, to_dev, torch_cuda

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
    orders at every level, the same root, applies and solutions equal to rounding (bitwise
    where the level's kernels take the same storage form alone and in the batch), the same
    PCG iteration counts. The handles are destroyed in another order than made."""
    from paper_1808_01364_amd import rhif
    torch = torch_cuda()
    csrs, Fs = _batch(probs, precision, flags)
    rng = np.random.default_rng(seed)
    nbit = 0
    for P, c, Fb in zip(probs, csrs, Fs):
        F1 = rhif.Factor(P.d, P.s, c, P.leaf, P.eps, P.precond, precision=precision, flags=flags)
        s1, sb = F1.stats(), Fb.stats()
        for key in ("levels", "root_size", "n_active", "n_skel", "sum_rank", "max_rank", "factor_bytes"):
            assert s1[key] == sb[key], (P.name, key, s1[key], sb[key])
        ch1, chb = gpu_choices(F1, s1["levels"]), gpu_choices(Fb, sb["levels"])
        assert ch1.keys() == chb.keys()
        for key in ch1:
            assert ch1[key][0] == chb[key][0] and np.array_equal(ch1[key][1], chb[key][1]), (P.name, key)
        r = to_dev(rng.standard_normal(P.N))
        z1, zb = F1.apply(r), Fb.apply(r)
        same = bool(torch.equal(z1, zb))
        nbit += same
        e = rel(zb.cpu().numpy(), z1.cpu().numpy())
        f = to_dev(P.f)
        u1, i1, r1 = F1.pcg(f, 1e-12, 300)
        ub, ib, rb = Fb.pcg(f, 1e-12, 300)
        es = rel(ub.cpu().numpy(), u1.cpu().numpy())
        print(f"{P.name}: levels {sb['levels']}, root {sb['root_size']}, apply {'bitwise' if same else f'{e:.1e}'}, "
              f"iterations {ib}, solution {es:.1e}", flush=True)
        assert e <= 100 * U and i1 == ib and rb <= 1e-12 and es <= 1e-12
        F1.close()
    for Fb in reversed(Fs):
        Fb.close()
    return nbit


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_batch_2d_uneven_sides(precision):
    """Five 2D problems with sides 64, 96, 40, 33, 128 (ragged cells, 2 to 4 levels, so the
    roots fall on different levels) and different fields."""
    probs = [problem("lognormal", 2, s, 8, 1e-6, seed=k, sigma=2.0)[0]
             for k, s in enumerate((64, 96, 40, 33, 128))]
    nbit = _against_single(probs, precision)
    assert nbit == len(probs)


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
