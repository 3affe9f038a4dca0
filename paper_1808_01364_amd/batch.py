"""Many independent problems solved concurrently on one GPU (the batched form of the solver).

Worker threads, each with its own HIP stream, take work from a shared queue. A unit of work
is a group of problems factored in one call (rhif_factor_batch: the group advances level by
level together, every elimination, block-Jacobi and skeletonization kernel of a level is one
launch over the blocks of all the group's problems, and one read-back per level brings all
their ranks), then solved in one joint PCG (rhif_pcg_solve_batch: every apply and vector
kernel one launch over all of them, one residual read-back per iteration), then released,
all stream-ordered on the worker's stream. Groups of one problem are plain rhif_factor calls.
While one worker's host plans its group's next level, the kernels of the others keep the GPU
busy. Results do not depend on the interleaving (every kernel's arithmetic order is fixed),
so a batch reproduces the one-by-one solutions; grouping changes at most the storage form a
kernel takes for a level, which leaves its arithmetic as it is.

The batch shape (group size, number of streams, and whether the queue takes the largest
problems first) is picked by a small autotuner that times the candidates on a sample of the
batch and remembers the choice for batches of the same size mix.
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


def solve_group(items, rtol: float = 1e-12, maxit: int = 500, stream=None):
    """[(u, iterations, relative residual)] of problems with the same dim, leaf, eps and
    precision, factored in one rhif_factor_batch call and solved in one joint PCG
    (rhif_pcg_solve_batch) on `stream` (the current stream if None); the factors are released
    before returning."""
    it0 = items[0]
    csrs = [rhif.assemble_fd(it.dim, it.n, it.a_cells, it.b, stream=stream) for it in items]
    Fs = rhif.factor_batch([(it.dim, it.n, c) for it, c in zip(items, csrs)], it0.leaf, it0.eps, 1,
                           it0.precision, stream=stream)
    try:
        if len(Fs) == 1:
            return [Fs[0].pcg(items[0].f, rtol, maxit, stream=stream)]
        return rhif.pcg_batch(Fs, [it.f for it in items], rtol, maxit, stream=stream)
    finally:
        for F in Fs:
            F.close()


def _order(items, order: str):
    idx = list(range(len(items)))
    if order == "largest_first":
        idx.sort(key=lambda i: -(items[i].n ** items[i].dim))
    return idx


def _groups(items, order: str, group: int):
    """The queue: consecutive problems (in the given order) with the same dim, leaf, eps and
    precision, in groups of at most `group`."""
    out = []
    for i in _order(items, order):
        it = items[i]
        key = (it.dim, it.leaf, it.eps, it.precision)
        if out and len(out[-1][1]) < group and out[-1][0] == key:
            out[-1][1].append(i)
        else:
            out.append((key, [i]))
    return [g for _, g in out]


# Worker threads and their streams live for the life of the process: the library keeps
# per-thread host state (pinned staging buffers, planner scratch, the level-0 plan of the last
# geometry) that a fresh thread would have to build again.
_POOL = None
_TLS = threading.local()


def _executor():
    global _POOL
    if _POOL is None:
        _POOL = cf.ThreadPoolExecutor(max_workers=max(STREAM_CANDIDATES))
    return _POOL


def _thread_stream():
    import torch
    st = getattr(_TLS, "stream", None)
    if st is None:
        st = _TLS.stream = torch.cuda.Stream()
    return st


def _run(items, nstreams: int, order: str, rtol: float, maxit: int, group: int = 1):
    import torch
    out = [None] * len(items)
    queue = _groups(items, order, max(1, group))
    nxt = [0]
    lock = threading.Lock()

    def worker():
        st = _thread_stream()
        with torch.cuda.stream(st):
            while True:
                with lock:
                    q = nxt[0]
                    nxt[0] += 1
                if q >= len(queue):
                    break
                idx = queue[q]
                if len(idx) == 1:
                    out[idx[0]] = solve_one(items[idx[0]], rtol, maxit)
                else:
                    for i, r in zip(idx, solve_group([items[i] for i in idx], rtol, maxit)):
                        out[i] = r
        st.synchronize()

    nw = max(1, min(nstreams, len(queue), max(STREAM_CANDIDATES)))
    for fut in [_executor().submit(worker) for _ in range(nw)]:
        fut.result()
    return out


# batch signature -> (nstreams, order, group) chosen by autotune
_TUNED = {}
STREAM_CANDIDATES = (1, 2, 4, 8)
ORDER_CANDIDATES = ("given", "largest_first")
GROUP_CANDIDATES = (4, 8, 16)


def _signature(items):
    """Size mix of a batch: the number of problems per (dim, side, precision), bucketed."""
    mix = {}
    for it in items:
        key = (it.dim, it.n, it.precision)
        mix[key] = mix.get(key, 0) + 1
    return tuple(sorted((k, (v + 3) // 4) for k, v in mix.items()))


def autotune(items, sample: int = 64, rtol: float = 1e-12, maxit: int = 500, verbose: bool = False):
    """Pick (nstreams, order, group) for this batch. Every candidate solves the same sample of the
    batch (every len/sample-th problem; the whole batch up to `sample` problems, since the group
    sizes and stream counts only show their effect on as many problems as they spread over)
    after one warm-up pass, and the highest DOFs/s wins: first
    (nstreams, order) with one problem per factorization call, then (group, nstreams) with
    that order. The choice is remembered for batches with the same size mix."""
    import torch
    key = _signature(items)
    if key in _TUNED:
        return _TUNED[key]
    step = max(1, len(items) // max(1, sample))
    samp = items[::step][:sample]
    dofs = sum(it.n ** it.dim for it in samp)
    _run(samp, 4, "given", rtol, maxit)              # warm-up: kernel loading, device memory cache
    _run(samp, 2, "given", rtol, maxit, group=max(GROUP_CANDIDATES))

    def rate(ns, order, group):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _run(samp, ns, order, rtol, maxit, group)
        torch.cuda.synchronize()
        r = dofs / (time.perf_counter() - t0)
        if verbose:
            print(f"autotune: {ns} streams, {order}, groups of {group}: {r / 1e6:.1f} M DOFs/s", flush=True)
        return r

    best, best_rate = (4, "given", 1), -1.0
    for ns in STREAM_CANDIDATES:
        for order in ORDER_CANDIDATES:
            r = rate(ns, order, 1)
            if r > best_rate:
                best, best_rate = (ns, order, 1), r
    order = best[1]
    for group in GROUP_CANDIDATES:
        for ns in (2, 4, 8):
            r = rate(ns, order, group)
            if r > best_rate:
                best, best_rate = (ns, order, group), r
    _TUNED[key] = best
    return best


def solve_many(items, nstreams: int = None, order: str = None, rtol: float = 1e-12, maxit: int = 500,
               group: int = None):
    """Solve every item; returns [(u, iterations, relative residual)] in the items' order.
    nstreams worker threads, one default-priority HIP stream each; order "given" or
    "largest_first"; group: problems factored per rhif_factor_batch call. Any left None is
    taken from autotune()."""
    if nstreams is None or order is None or group is None:
        ns, od, gr = autotune(items, rtol=rtol, maxit=maxit)
        nstreams = ns if nstreams is None else nstreams
        order = od if order is None else order
        group = gr if group is None else group
    return _run(items, nstreams, order, rtol, maxit, group)
