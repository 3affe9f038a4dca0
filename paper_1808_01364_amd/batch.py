"""Many independent problems solved concurrently on one GPU (the batched form of the solver).

Each worker thread owns a HIP stream and takes problems from a shared queue: assembly,
factorization, PCG and release of the factor, all stream-ordered on its own stream. A
factorization waits for its ranks once per level; while one problem's host plans its next
level, the kernels of the others keep the GPU busy, and the small upper levels of several
problems run side by side. Results do not depend on the interleaving (every kernel's
arithmetic order is fixed), so a batch reproduces the one-by-one solutions bit for bit.

The batch shape (how many streams, and whether the queue takes the largest problems first)
is picked by a small autotuner that times the candidates on a sample of the batch and
remembers the choice for batches of the same size mix.
"""
from __future__ import annotations

import concurrent.futures as cf
import threading
import time
from dataclasses import dataclass

from . import rhif


@dataclass
class BatchItem:
    dim: int
    n: int
    a_cells: object          # device float64 tensor, (n+1)^dim cell coefficients
    f: object                # device float64 tensor, N values
    b: object = None         # device float64 tensor or None
    leaf: int = 16
    eps: float = 1e-6
    precision: int = 0       # 0: FP64 factor; 1: FP32-mixed factor (flexible PCG)


def solve_one(item: BatchItem, rtol: float = 1e-12, maxit: int = 500, stream=None):
    """(u, iterations, relative residual) for one problem on `stream` (the current stream if
    None); the factor is released before returning."""
    csr = rhif.assemble_fd(item.dim, item.n, item.a_cells, item.b, stream=stream)
    F = rhif.Factor(item.dim, item.n, csr, item.leaf, item.eps, 1, precision=item.precision, stream=stream)
    try:
        u, it, rr = F.pcg(item.f, rtol, maxit, stream=stream)
    finally:
        F.close()
    return u, it, rr


def _order(items, order: str):
    idx = list(range(len(items)))
    if order == "largest_first":
        idx.sort(key=lambda i: -(items[i].n ** items[i].dim))
    return idx


def _run(items, nstreams: int, order: str, rtol: float, maxit: int):
    import torch
    out = [None] * len(items)
    queue = _order(items, order)
    nxt = [0]
    lock = threading.Lock()

    def worker():
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            while True:
                with lock:
                    q = nxt[0]
                    nxt[0] += 1
                if q >= len(queue):
                    break
                i = queue[q]
                out[i] = solve_one(items[i], rtol, maxit)
        st.synchronize()

    nw = max(1, min(nstreams, len(items)))
    with cf.ThreadPoolExecutor(max_workers=nw) as ex:
        for fut in [ex.submit(worker) for _ in range(nw)]:
            fut.result()
    return out


# batch signature -> (nstreams, order) chosen by autotune
_TUNED = {}
STREAM_CANDIDATES = (1, 2, 4, 8)
ORDER_CANDIDATES = ("given", "largest_first")


def _signature(items):
    """Size mix of a batch: the number of problems per (dim, side, precision), bucketed."""
    mix = {}
    for it in items:
        key = (it.dim, it.n, it.precision)
        mix[key] = mix.get(key, 0) + 1
    return tuple(sorted((k, (v + 3) // 4) for k, v in mix.items()))


def autotune(items, sample: int = 12, rtol: float = 1e-12, maxit: int = 500, verbose: bool = False):
    """Pick (nstreams, order) for this batch: each candidate solves the same sample of the batch
    (every len/sample-th problem), after one warm-up pass; the highest DOFs/s wins. The
    choice is remembered for batches with the same size mix."""
    import torch
    key = _signature(items)
    if key in _TUNED:
        return _TUNED[key]
    step = max(1, len(items) // max(1, sample))
    samp = items[::step][:sample]
    dofs = sum(it.n ** it.dim for it in samp)
    _run(samp, 4, "given", rtol, maxit)      # warm-up: kernel loading, device memory cache
    best, best_rate = (4, "given"), -1.0
    for ns in STREAM_CANDIDATES:
        for order in ORDER_CANDIDATES:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _run(samp, ns, order, rtol, maxit)
            torch.cuda.synchronize()
            rate = dofs / (time.perf_counter() - t0)
            if verbose:
                print(f"autotune: {ns} streams, {order}: {rate / 1e6:.1f} M DOFs/s", flush=True)
            if rate > best_rate:
                best, best_rate = (ns, order), rate
    _TUNED[key] = best
    return best


def solve_many(items, nstreams: int = None, order: str = None, rtol: float = 1e-12, maxit: int = 500):
    """Solve every item; returns [(u, iterations, relative residual)] in the items' order.
    nstreams worker threads, one default-priority HIP stream each; order "given" or
    "largest_first". Either left None is taken from autotune()."""
    if nstreams is None or order is None:
        ns, od = autotune(items, rtol=rtol, maxit=maxit)
        nstreams = ns if nstreams is None else nstreams
        order = od if order is None else order
    return _run(items, nstreams, order, rtol, maxit)
