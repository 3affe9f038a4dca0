"""Full-size workloads through the C ABI, in the launch configuration the benchmark times:
* the 512^2 log-normal problem (sigma 3, leaf 16) at eps 1e-6 and 1e-3 against the CPU
  oracle on the same inputs;
* a 3D 32^3 two-valued problem (1e-3 / 1e3, b = 1e-2, leaf 4, eps 1e-3) against the oracle:
  more than 512 faces at level 0 (the many-group form of the skeletonization) and faces of
  hundreds of unknowns at the top;
* the 3D 64^3 two-valued problem against the oracle's results stored in tests/golden (the
  oracle takes about an hour there), and by properties that hold at any size (convergence to
  1e-12, the true residual, consistent statistics, symmetry of F^-1)."""
import os

import numpy as np
import pytest

import oracle as O
from tests.gpu_common import U, gpu_choices, gpu_csr, gpu_factor, parity_check, problem, rel, rel_max, to_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cfg3_oracle.npz")


def _host(t):
    return t.detach().cpu().numpy()


def _true_relres(A, f, u):
    return float(np.linalg.norm(f - A @ u) / np.linalg.norm(f))


def _residual_floor(A, f, u):
    """Rounding floor of ||f - A u|| / ||f||: the sum of |A||u| in FP64 (forward error of a
    sparse matrix-vector product, at most 2d+1 terms per row)."""
    return float(np.linalg.norm(abs(A) @ abs(u)) * U * 8 / np.linalg.norm(f))


@pytest.mark.timeout(600)
@pytest.mark.parametrize("eps", [1e-6, 1e-3])
def test_cfg2_full_parity(eps):
    """512^2 (the benchmark's workload): every ID agrees with the oracle's (or is a certified
    tie), applies agree with the replayed oracle to c u kappa, and PCG takes the same number
    of iterations to the same solution (1e-10)."""
    from workloads import CONFIGS
    P = CONFIGS["cfg2"](eps)
    A = O.assemble_fd(P.d, P.s, P.a_cells, P.b)
    out = parity_check(P, A, n_rhs=2, seed=12)
    print("cfg2", eps, out, flush=True)


@pytest.mark.timeout(600)
def test_3d_32_parity():
    """3D 32^3, leaf 4, eps 1e-3, a = 1e-3 / 1e3 per voxel, b = 1e-2: 1344 faces at level 0
    and faces of several hundred unknowns at the top levels, against the oracle."""
    P, A = problem("two_valued", 3, 32, 4, 1e-3, seed=2, lo=1e-3, hi=1e3, b_const=1e-2)
    out = parity_check(P, A, n_rhs=2, seed=12)
    print("3d-32", out, flush=True)


def _golden_choices_ok(G, gpu):
    """Every ID of the GPU against the stored oracle choices; a difference passes only if the
    stored ratios show a tie (pivot-norm gap or rank ratio within 1e-10 of eps). Returns
    (identical, n_ties)."""
    eps = float(G["eps"])
    perm_ptr = np.concatenate([[0], np.cumsum(G["size"])])
    keys = set()
    ties = 0
    for i in range(len(G["level"])):
        key = (int(G["level"][i]), int(G["first_dof"][i]))
        keys.add(key)
        assert key in gpu, ("group missing on the GPU", key)
        k_o = int(G["rank"][i])
        perm_o = G["perm"][perm_ptr[i]:perm_ptr[i + 1]]
        k_g, perm_g = gpu[key]
        if k_g == k_o and set(perm_g[:k_g].tolist()) == set(perm_o[:k_o].tolist()):
            continue
        ratios = G["ratio"][G["ratio_ptr"][i]:G["ratio_ptr"][i + 1]]
        gaps = G["gap"][G["gap_ptr"][i]:G["gap_ptr"][i + 1]]
        kk = min(k_g, k_o)
        j = next((j for j in range(kk) if perm_g[j] != perm_o[j]), None)
        if j is not None:
            assert j < len(gaps) and gaps[j] <= 1e-10, ("pivot differs without a tie", key, j)
        else:
            assert abs(ratios[kk] - eps) <= 1e-10 * eps, ("rank differs without a tie", key, k_g, k_o)
        ties += 1
    assert not (set(gpu) - keys), "the GPU has groups the oracle lacks"
    return ties == 0, ties


@pytest.mark.timeout(300)
def test_cfg3_against_stored_oracle():
    """3D 64^3 (a = 1e-3 / 1e3 per voxel, b = 1e-2, leaf 4, eps 1e-3) against what the oracle
    computed on the same inputs (tests/golden/make_cfg3_golden.py): the same IDs, |S_L| and
    PCG iteration count; F^-1 r and the PCG solution at 4096 sampled unknowns (and in norm)."""
    if not os.path.exists(GOLDEN):
        pytest.skip("tests/golden/cfg3_oracle.npz has not been written")
    from workloads import CONFIGS
    G = np.load(GOLDEN)
    P = CONFIGS["cfg3"]()
    F = gpu_factor(P)
    st = F.stats()
    identical, ties = _golden_choices_ok(G, gpu_choices(F, st["levels"] - st["sublevels"]))
    print("cfg3 choices identical", identical, "certified ties", ties, flush=True)
    f = to_dev(P.f)
    ug, it, rr = F.pcg(f, 1e-12, 100)
    u = _host(ug)
    r = np.random.default_rng(int(G["r_seed"])).standard_normal(P.N)
    z = _host(F.apply(to_dev(r)))
    idx = G["idx"]
    bound = 10 * U * float(G["kappa"])
    ez = max(abs(np.linalg.norm(z) - float(G["z_norm"])) / float(G["z_norm"]),
             rel_max(z[idx], G["z_samples"]))
    eu = max(abs(np.linalg.norm(u) - float(G["u_norm"])) / float(G["u_norm"]), rel_max(u[idx], G["u_samples"]))
    print(f"cfg3 apply {ez:.2e} (bound {bound:.2e}), pcg {it} vs {int(G['iters'])}, solution {eu:.2e}",
          flush=True)
    assert rr <= 1e-12
    if identical:
        assert st["root_size"] == int(G["root_size"])
        assert ez <= bound, (ez, bound)
        assert it == int(G["iters"])
        assert eu <= 1e-10, eu
    F.close()


@pytest.mark.timeout(300)
@pytest.mark.parametrize("cfg,eps,maxit", [("cfg2", 1e-3, 100), ("cfg3", None, 50)])
def test_fullsize_properties(cfg, eps, maxit):
    """PCG with the GPU factor converges to 1e-12; the true residual of the returned solution
    is at the rounding floor; the statistics are consistent with the grid."""
    from workloads import CONFIGS
    P = CONFIGS[cfg](eps) if eps is not None else CONFIGS[cfg]()
    A = O.assemble_fd(P.d, P.s, P.a_cells, P.b)
    csr = gpu_csr(P)
    F = gpu_factor(P, csr)
    st = F.stats()
    f = to_dev(P.f)
    ug, it, rr = F.pcg(f, 1e-12, maxit)
    u = _host(ug)
    tr = _true_relres(A, P.f, u)
    print(cfg, eps, "iters", it, "relres", rr, "true", tr, "root", st["root_size"], flush=True)
    assert rr <= 1e-12 and it < maxit
    assert tr <= 10 * _residual_floor(A, P.f, u) + 1e-12
    assert st["n_active"][0] == P.N
    assert all(st["n_active"][l + 1] <= st["n_active"][l] for l in range(st["levels"]))
    assert st["n_active"][st["levels"]] == st["root_size"]
    # F^-1 is symmetric: <x, F^-1 y> = <F^-1 x, y>
    rng = np.random.default_rng(3)
    x, y = rng.standard_normal(P.N), rng.standard_normal(P.N)
    fx, fy = _host(F.apply(to_dev(x))), _host(F.apply(to_dev(y)))
    assert abs(x @ fy - fx @ y) <= 1e-10 * np.linalg.norm(x) * np.linalg.norm(fy)
    F.close()
