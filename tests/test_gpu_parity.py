"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on the same seeded
inputs. Where the interpolative decompositions could legitimately choose differently
(pivot ties), the oracle replays the GPU's choices and the choices are checked apart."""
import numpy as np
import pytest

import oracle as O
from tests.gpu_common import (gpu_choices, gpu_csr, gpu_factor, parity_check, problem, rel, rel_max, to_dev,
                              torch_cuda)

pytestmark = pytest.mark.gpu

U = np.finfo(np.float64).eps


def _host(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("d,s", [(2, 13), (3, 6), (2, 64)])
def test_assembly_bitwise(d, s):
    """The device assembly reproduces the oracle's CSR exactly (same operation order)."""
    P, A = problem("two_valued", d, s, 4, 1e-3, seed=3, lo=1e-2, hi=1e2, b_const=0.25 if d == 3 else 0.0)
    rp, col, val = gpu_csr(P)
    assert np.array_equal(_host(rp), A.indptr)
    assert np.array_equal(_host(col), A.indices)
    assert np.array_equal(_host(val), A.data)


@pytest.mark.parametrize("d,s,leaf,precond", [(2, 16, 4, 1), (2, 20, 8, 1), (2, 13, 4, 0), (3, 7, 2, 1),
                                              (3, 10, 4, 1), (2, 5, 8, 1)])
def test_eps0_apply_is_dense_solve(d, s, leaf, precond):
    """eps = 0: F^-1 on the GPU is the exact inverse (nested dissection), so it matches a
    dense Cholesky solve; PCG stops after one product."""
    P, A = problem("two_valued", d, s, leaf, 0.0, precond=precond, lo=0.5, hi=2.0)
    F = gpu_factor(P)
    f = to_dev(P.f)
    z = _host(F.apply(f))
    u = O.dense_solve(A, P.f)
    assert rel(z, u) < 1e-12
    uu, it, rr = F.pcg(f, 1e-12, 5)
    assert it == 1 and rr <= 1e-12
    F.close()


def _parity(P, A, **kw):
    return parity_check(P, A, **kw)


@pytest.mark.parametrize("d,s,leaf,eps,kind,hi", [
    (2, 64, 8, 1e-3, "constant", 1.0),       # a = 1 on the 64^2 geometry
    (2, 64, 8, 1e-3, "two_valued", 10.0),    # the 64^2 geometry at contrast 10
    (2, 64, 8, 1e-6, "two_valued", 10.0),
    (3, 12, 4, 1e-3, "constant", 1.0)])
def test_well_conditioned_apply_100u(d, s, leaf, eps, kind, hi):
    """On well-conditioned inputs the applies agree with the replayed oracle to 100 u."""
    P, A = problem(kind, d, s, leaf, eps, seed=0, lo=1.0, hi=hi)
    out = _parity(P, A, well_conditioned=True)
    print((d, s, leaf, eps, kind, hi), out)


def test_cfg1_parity():
    """2D 64^2, iid two-valued 1e-2/1e2, leaf 8, eps 1e-3 (the small configuration)."""
    from workloads import CONFIGS
    P = CONFIGS["cfg1"]()
    A = O.assemble_fd(P.d, P.s, P.a_cells, P.b)
    out = _parity(P, A)
    print("cfg1", out)


@pytest.mark.parametrize("d,s,leaf,eps,kind,precond", [
    (2, 31, 4, 1e-6, "lognormal", 1), (2, 40, 8, 1e-3, "two_valued", 0), (2, 13, 4, 1e-2, "two_valued", 1),
    (3, 9, 2, 1e-3, "two_valued", 1), (3, 12, 4, 1e-3, "two_valued", 1),
    # interiors and a root larger than one elimination panel (128 columns)
    (3, 20, 4, 1e-3, "two_valued", 1)])
def test_small_parity(d, s, leaf, eps, kind, precond):
    P, A = problem(kind, d, s, leaf, eps, seed=2, precond=precond, sigma=2.0, lo=1e-2, hi=1e2)
    out = _parity(P, A)
    print((d, s, leaf, eps, kind, precond), out)


@pytest.mark.parametrize("d,s,leaf,eps,precision", [(2, 31, 4, 1e-6, 0), (2, 64, 16, 1e-3, 0), (3, 12, 4, 1e-3, 0),
                                                     (3, 16, 4, 1e-3, 0), (2, 40, 8, 1e-6, 1)])
def test_multi_workgroup_id_parity(d, s, leaf, eps, precision):
    """RHIF_FLAG_SKEL_MULTI: the interpolative decompositions of every level taken by the form
    that spreads each group's column-pivoted QR over row blocks (one launch per step), which
    the large faces of the upper 3D levels take by default; it agrees with the oracle like the
    one-workgroup forms (FP64), and converges in the FP32-mixed form."""
    from paper_1808_01364_amd import rhif
    P, A = problem("two_valued", d, s, leaf, eps, seed=7, lo=1e-2, hi=1e2)
    if precision == 0:
        out = _parity(P, A, flags=rhif.FLAG_SKEL_MULTI)
        print((d, s, leaf, eps), out)
        return
    csr = gpu_csr(P)
    F = rhif.Factor(P.d, P.s, csr, P.leaf, P.eps, 1, precision=precision, flags=rhif.FLAG_SKEL_MULTI)
    u, it, rr = F.pcg(to_dev(P.f), 1e-12, 300)
    ref = O.dense_solve(A, P.f)
    print((d, s, leaf, eps, precision), it, rr, rel(_host(u), ref))
    assert rr <= 1e-12 and rel(_host(u), ref) <= 1e-10
    F.close()


@pytest.mark.parametrize("d,s,leaf,eps", [(2, 31, 4, 1e-6), (3, 12, 4, 1e-3)])
def test_global_staging_parity(d, s, leaf, eps):
    """The paths that groups too large for LDS take (block-Jacobi scaling and ID operands in
    global memory), forced on small problems, agree with the oracle like the LDS paths."""
    from paper_1808_01364_amd import rhif
    P, A = problem("two_valued", d, s, leaf, eps, seed=4, lo=1e-2, hi=1e2)
    out = _parity(P, A, flags=rhif.FLAG_GLOBAL_STAGING)
    print((d, s, leaf, eps), out)


@pytest.mark.parametrize("d,s,leaf,eps,kind,precond,b", [
    (2, 1, 8, 1e-6, "two_valued", 1, 0.0),     # one unknown: the root is the whole problem
    (3, 1, 4, 1e-3, "two_valued", 1, 0.0),
    (2, 2, 2, 1e-6, "two_valued", 1, 0.0),     # the smallest grid with a level
    (2, 24, 4, 1e-6, "lognormal", 1, 1.0),     # reaction term b > 0
    (3, 9, 2, 1e-3, "two_valued", 0, 0.0),     # HIF (no block Jacobi) in 3D
    (2, 33, 4, 1e-6, "paper", 1, 0.0),         # the paper's quantized field, ragged side
])
def test_edge_cases(d, s, leaf, eps, kind, precond, b):
    P, A = problem(kind, d, s, leaf, eps, seed=8, precond=precond, sigma=2.0, lo=1e-2, hi=1e2, b_const=b)
    out = _parity(P, A)
    print((d, s, leaf, eps, kind, precond, b), out)


def test_not_spd_is_reported():
    """A strongly negative reaction term: the device Cholesky of the first cells fails and
    the library reports loss of positive definiteness at level 0, step E."""
    from paper_1808_01364_amd import rhif
    P, A = problem("constant", 2, 16, 4, 1e-3)
    P.b = np.full(P.N, -1e6)
    with pytest.raises(rhif.NotSPD) as ei:
        gpu_factor(P)
    assert "level 0" in str(ei.value) and "E" in str(ei.value)


def test_repeatable_bitwise():
    """No floating-point atomics: two factorizations and applies give identical bits."""
    P, A = problem("two_valued", 2, 48, 8, 1e-3, seed=5)
    csr = gpu_csr(P)
    r = to_dev(np.random.default_rng(1).standard_normal(P.N))
    F1 = gpu_factor(P, csr)
    F2 = gpu_factor(P, csr)
    z1, z2 = _host(F1.apply(r)), _host(F2.apply(r))
    assert np.array_equal(z1, z2)
    F1.close()
    F2.close()


def test_solve_graphs_parity():
    """RHIF_FLAG_SOLVE_GRAPHS: the applies and PCG iterations replayed as HIP graphs give the
    same bits as direct launches, also after a second solve into another output buffer
    (the graphs are captured again for it), and agree with the replayed oracle."""
    from paper_1808_01364_amd import rhif
    torch = torch_cuda()
    P, A = problem("two_valued", 2, 64, 8, 1e-3, seed=0, lo=1e-2, hi=1e2)
    csr = gpu_csr(P)
    Fg = gpu_factor(P, csr, flags=rhif.FLAG_SOLVE_GRAPHS)
    Fd = gpu_factor(P, csr)
    r = to_dev(np.random.default_rng(3).standard_normal(P.N))
    zg1, zg2, zd = _host(Fg.apply(r)), _host(Fg.apply(r)), _host(Fd.apply(r))
    assert np.array_equal(zg1, zd) and np.array_equal(zg2, zd)
    f = to_dev(P.f)
    out1 = torch.empty_like(f)
    out2 = torch.empty_like(f)
    u1, it1, _ = Fg.pcg(f, 1e-12, 300, out=out1)
    u2, it2, _ = Fg.pcg(f, 1e-12, 300, out=out2)
    u3, it3, _ = Fg.pcg(f, 1e-12, 300, out=out1)
    ud, itd, _ = Fd.pcg(f, 1e-12, 300)
    assert it1 == it2 == it3 == itd
    for uu in (u1, u2, u3):
        assert np.array_equal(_host(uu), _host(ud))
    st = Fg.stats()
    ch = gpu_choices(Fg, st["levels"])
    rep = O.factor(A, P.d, P.s, P.leaf, P.eps, P.precond, replay=ch)
    res = O.pcg(A, P.f, lambda v: O.apply_inverse(rep, v), 1e-12, 300)
    assert res.iters == it1 and rel(_host(u2), res.u) < 1e-10
    Fg.close()
    Fd.close()


def test_apply_several_rhs():
    """rhif_apply with nrhs = 3 (right-hand sides one after another), into a separate output
    and in place (r == z), against the replayed oracle at 100 u (a = 1)."""
    torch = torch_cuda()
    P, A = problem("constant", 2, 64, 8, 1e-3)
    F = gpu_factor(P)
    st = F.stats()
    rep = O.factor(A, P.d, P.s, P.leaf, P.eps, P.precond, replay=gpu_choices(F, st["levels"]))
    R = np.random.default_rng(5).standard_normal((3, P.N))
    Rd = torch.tensor(R, dtype=torch.float64, device="cuda")
    Z = _host(F.apply(Rd))
    F.apply(Rd, out=Rd)          # in place
    Zi = _host(Rd)
    assert np.array_equal(Z, Zi)
    for j in range(3):
        zo = O.apply_inverse(rep, R[j])
        assert rel(Z[j], zo) <= 100 * U and rel_max(Z[j], zo) <= 100 * U, (j, rel(Z[j], zo))
    F.close()


def test_removed_flag_is_rejected():
    """Option bit 2 (the former leaf sublevels) is refused before any device work."""
    from paper_1808_01364_amd import rhif
    P, A = problem("constant", 2, 16, 4, 1e-3)
    with pytest.raises(rhif.RhifError, match="not supported"):
        gpu_factor(P, flags=4)
