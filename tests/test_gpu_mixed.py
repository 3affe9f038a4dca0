"""The FP32-mixed factorizations (precision 1: the interpolative decompositions in FP32;
precision 2: also the Schur products of the cell eliminations on the FP32 matrix cores; every
Cholesky factor and the apply in FP64) with the flexible PCG, through the C ABI. PCG refines the solution to the
same 1e-12 relative residual as with the FP64 factor; the error against the FP64 oracle is
stated for every result, and asserted where the conditioning allows."""
import os

import numpy as np
import pytest

import oracle as O
from tests.gpu_common import U, gpu_choices, gpu_csr, problem, rel, rel_max, to_dev

pytestmark = pytest.mark.gpu

U32 = float(np.finfo(np.float32).eps)


def _host(t):
    return t.detach().cpu().numpy()


def _factor(P, csr, precision, flags=0):
    from paper_1808_01364_amd import rhif
    return rhif.Factor(P.d, P.s, csr, P.leaf, P.eps, P.precond, precision=precision, flags=flags)


def _residual_floor(A, f, u):
    return float(np.linalg.norm(abs(A) @ abs(u)) * U * 8 / np.linalg.norm(f))


@pytest.mark.parametrize("precision", [1, 2])
@pytest.mark.parametrize("d,s,leaf,eps,kind,hi", [
    (2, 64, 8, 1e-3, "two_valued", 1e2),      # the 64^2 configuration (contrast 1e4)
    (2, 64, 8, 1e-6, "two_valued", 10.0),
    (2, 48, 16, 1e-6, "lognormal", 1e2),
    (3, 16, 4, 1e-3, "two_valued", 1e2)])
def test_mixed_small_against_oracle(d, s, leaf, eps, kind, hi, precision):
    """Small problems: the FP32-mixed solve reaches 1e-12 and its solution agrees with the
    oracle's dense FP64 solve to 1e-10 (these are well enough conditioned); the apply differs
    from the FP64 oracle's (replaying the GPU's choices) by no more than the FP32 rounding
    of the ID and the Schur products allows."""
    P, A = problem(kind, d, s, leaf, eps, seed=1, lo=1e-2, hi=hi, sigma=3.0)
    csr = gpu_csr(P)
    F32 = _factor(P, csr, precision)
    F64 = _factor(P, csr, 0)
    f = to_dev(P.f)
    u32, it32, rr32 = F32.pcg(f, 1e-12, 300)
    u64, it64, rr64 = F64.pcg(f, 1e-12, 300)
    ud = O.dense_solve(A, P.f)
    e32, e64 = rel(_host(u32), ud), rel(_host(u64), ud)
    st = F32.stats()
    rep = O.factor(A, P.d, P.s, P.leaf, P.eps, P.precond, replay=gpu_choices(F32, st["levels"]))
    r = np.random.default_rng(4).standard_normal(P.N)
    ea = rel(_host(F32.apply(to_dev(r))), O.apply_inverse(rep, r))
    print(f"{(d, s, leaf, eps, kind, hi)} precision {precision}: iters {it32} (FP64 {it64}); solution error vs dense FP64 solve "
          f"FP32-mixed {e32:.2e}, FP64 {e64:.2e}; apply vs FP64 oracle {ea:.2e}", flush=True)
    assert rr32 <= 1e-12 and it32 <= 2 * it64 + 2
    assert e32 <= 1e-10
    assert ea <= max(1e-3, 1e4 * U32 * eps ** 0)   # FP32 ID and Schur products: a perturbed preconditioner
    F32.close()
    F64.close()


@pytest.mark.timeout(300)
@pytest.mark.parametrize("cfg,eps,precision", [("cfg2", 1e-6, 1), ("cfg2", 1e-6, 2), ("cfg2", 1e-3, 1),
                                               ("cfg3", None, 1), ("cfg3", None, 2)])
def test_mixed_fullsize(cfg, eps, precision):
    """512^2 (eps 1e-6, 1e-3) and 3D 64^3 with the FP32-mixed factor: PCG reaches 1e-12, the
    true residual is at the FP64 rounding floor, and the solution is compared with the FP64
    factor's (which agrees with the oracle to 1e-10 in the FP64 parity tests)."""
    from workloads import CONFIGS
    P = CONFIGS[cfg](eps) if eps is not None else CONFIGS[cfg]()
    A = O.assemble_fd(P.d, P.s, P.a_cells, P.b)
    csr = gpu_csr(P)
    f = to_dev(P.f)
    F32 = _factor(P, csr, precision)
    u32, it32, rr32 = F32.pcg(f, 1e-12, 300)
    F32.close()
    F64 = _factor(P, csr, 0)
    u64, it64, rr64 = F64.pcg(f, 1e-12, 300)
    F64.close()
    a, b = _host(u32), _host(u64)
    tr = float(np.linalg.norm(P.f - A @ a) / np.linalg.norm(P.f))
    print(f"{cfg} {eps} precision {precision}: iters {it32} (FP64 {it64}), relres {rr32:.2e}, true {tr:.2e}, "
          f"solution vs FP64 {rel(a, b):.2e} (max {rel_max(a, b):.2e})", flush=True)
    assert rr32 <= 1e-12
    assert tr <= 10 * _residual_floor(A, P.f, a) + 1e-12
    assert rel(a, b) <= 1e-8


def test_bad_precision_is_rejected():
    from paper_1808_01364_amd import rhif
    P, A = problem("constant", 2, 16, 4, 1e-3)
    with pytest.raises(rhif.RhifError, match="precision"):
        _factor(P, gpu_csr(P), 3)
