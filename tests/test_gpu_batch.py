"""Batches of uneven problems solved concurrently on several streams (the batched-solver
extension): with one problem per factorization call the solutions, iteration counts and
residuals equal those of solving the problems one by one, bit for bit, since no kernel's
arithmetic depends on the interleaving; with groups of problems per call (rhif_factor_batch)
they agree to rounding; the FP32-mixed, autotuned batch agrees with the oracle problem by
problem."""
import time

import numpy as np
import pytest

from tests.gpu_common import to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def test_batch_equals_one_by_one():
    torch = torch_cuda()
    from paper_1808_01364_amd.batch import BatchItem, solve_many, solve_one
    from workloads.fields import batch_problem
    probs = [batch_problem(k) for k in range(8)]
    items = [BatchItem(2, P.s, to_dev(P.a_cells), to_dev(P.f), None, P.leaf, P.eps) for P in probs]
    torch.cuda.synchronize()
    solve_many(items, nstreams=4, order="given", group=1)   # warm-up (kernel loading, memory cache)
    solve_many(items, nstreams=2, order="given", group=4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq = [solve_one(it) for it in items]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    bat = solve_many(items, nstreams=4, order="given", group=1)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    bat2 = solve_many(items, nstreams=2, order="given", group=1)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    grp = solve_many(items, nstreams=2, order="largest_first", group=4)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    dofs = sum(P.s * P.s for P in probs)
    print(f"sides {[P.s for P in probs]}: one by one {dofs / (t1 - t0) / 1e6:.1f} M DOFs/s, "
          f"4 streams {dofs / (t2 - t1) / 1e6:.1f}, 2 streams {dofs / (t3 - t2) / 1e6:.1f}, "
          f"2 streams with groups of 4 {dofs / (t4 - t3) / 1e6:.1f}", flush=True)
    bat3 = solve_many(items, nstreams=3, order="largest_first", group=1)
    for (u1, i1, r1), (u2, i2, r2) in zip(seq, grp):
        e = float(torch.linalg.norm(u1 - u2) / torch.linalg.norm(u1))
        assert i1 == i2 and r2 <= 1e-12 and e <= 1e-12, (i1, i2, r2, e)
    for (u1, i1, r1), (u2, i2, r2) in zip(seq, bat3):
        assert i1 == i2 and r1 == r2 and torch.equal(u1, u2)
    for (u1, i1, r1), (u2, i2, r2) in zip(seq, bat2):
        assert i1 == i2 and r1 == r2 and torch.equal(u1, u2)
    for (u1, i1, r1), (u2, i2, r2) in zip(seq, bat):
        assert i1 == i2 and r1 == r2 and r1 <= 1e-12
        assert torch.equal(u1, u2)


@pytest.mark.timeout(300)
def test_mixed_autotuned_batch_against_oracle():
    """Problems 11, 14, 1, 6 of the uneven batch (sides 128, 128, 256, 256; a = exp(2 g),
    eps 1e-4) solved as one FP32-mixed, autotuned batch: every solution agrees with the
    oracle's (its own FP64 factorization and PCG to 1e-12) to 1e-9, and every residual
    reaches 1e-12."""
    import oracle as O
    from paper_1808_01364_amd import batch
    from workloads.fields import batch_problem
    torch_cuda()
    probs = [batch_problem(k) for k in (11, 14, 1, 6)]
    items = [batch.BatchItem(2, P.s, to_dev(P.a_cells), to_dev(P.f), None, P.leaf, P.eps, precision=1)
             for P in probs]
    ns, order, group = batch.autotune(items, sample=4, verbose=True)
    out = batch.solve_many(items)
    for P, (u, it, rr) in zip(probs, out):
        A = O.assemble_fd(2, P.s, P.a_cells, None)
        F = O.factor(A, 2, P.s, P.leaf, P.eps, 1)
        ref = O.pcg(A, P.f, lambda v: O.apply_inverse(F, v), 1e-12, 300)
        e = float(np.linalg.norm(u.cpu().numpy() - ref.u) / np.linalg.norm(ref.u))
        print(f"side {P.s}: iterations {it} (oracle {ref.iters}), relres {rr:.1e}, error vs oracle {e:.2e}",
              flush=True)
        assert rr <= 1e-12 and e <= 1e-9
    print("autotuned:", ns, order, group)
