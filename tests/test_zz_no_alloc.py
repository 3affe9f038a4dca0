"""rhif_pcg_solve_noalloc (the entry point for callers that cannot allocate) against
rhif_pcg_solve on the same handle: two calls in a row, the second on a smaller problem (the
shared workspace keeps the first call's contents), and the size limit."""
import numpy as np
import pytest

from tests.gpu_common import gpu_csr, gpu_factor, problem, rel, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _host(t):
    return t.detach().cpu().numpy()


def _check(P):
    torch = torch_cuda()
    F = gpu_factor(P)
    f = to_dev(P.f)
    u_ref, it_ref, rr_ref = F.pcg(f, 1e-12, 300)
    u = torch.full_like(f, float("nan"))
    u, it, rr = F.pcg(f, 1e-12, 300, out=u, noalloc=True)
    torch.cuda.synchronize()
    a, b = _host(u), _host(u_ref)
    print(P.name, "iters", it, it_ref, "relres", rr, rr_ref, "bitwise", np.array_equal(a, b), flush=True)
    assert it == it_ref and rr <= 1e-12
    assert rel(a, b) <= 1e-10 and np.max(np.abs(a - b)) <= 1e-10 * np.max(np.abs(b))
    F.close()


def test_noalloc_pcg_two_calls_second_smaller():
    P1, _ = problem("two_valued", 2, 96, 8, 1e-3, seed=1, lo=1e-2, hi=1e2)
    P2, _ = problem("lognormal", 2, 40, 8, 1e-6, seed=2, sigma=2.0)
    _check(P1)
    _check(P2)


def test_noalloc_rejects_too_large():
    from paper_1808_01364_amd import rhif
    torch = torch_cuda()
    P, _ = problem("constant", 2, 1025, 16, 1e-3)
    assert P.N > rhif.NOALLOC_MAX_N
    F = gpu_factor(P)
    f = to_dev(P.f)
    with pytest.raises(rhif.RhifError, match="RHIF_NOALLOC_MAX_N"):
        F.pcg(f, 1e-12, 10, out=torch.empty_like(f), noalloc=True)
    F.close()
