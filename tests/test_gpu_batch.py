"""Batches of uneven problems solved concurrently on several streams (the batched-solver
extension): the solutions, iteration counts and residuals equal those of solving the
problems one by one, bit for bit, since no kernel's arithmetic depends on the interleaving."""
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
    solve_many(items, nstreams=4)             # warm-up (kernel loading, device memory cache)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq = [solve_one(it) for it in items]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    bat = solve_many(items, nstreams=4)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    bat2 = solve_many(items, nstreams=2)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    dofs = sum(P.s * P.s for P in probs)
    print(f"sides {[P.s for P in probs]}: one by one {dofs / (t1 - t0) / 1e6:.1f} M DOFs/s, "
          f"4 streams {dofs / (t2 - t1) / 1e6:.1f}, 2 streams {dofs / (t3 - t2) / 1e6:.1f}", flush=True)
    for (u1, i1, r1), (u2, i2, r2) in zip(seq, bat2):
        assert i1 == i2 and r1 == r2 and torch.equal(u1, u2)
    for (u1, i1, r1), (u2, i2, r2) in zip(seq, bat):
        assert i1 == i2 and r1 == r2 and r1 <= 1e-12
        assert torch.equal(u1, u2)
