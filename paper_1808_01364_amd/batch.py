"""Many independent problems solved concurrently on one GPU.

Each worker thread owns a HIP stream and takes problems from a shared list: assembly,
factorization, PCG and release of the factor, all stream-ordered on its own stream. A
factorization waits for its ranks once per level; while one problem's host plans its next
level, the kernels of the others keep the GPU busy, and the small upper levels of several
problems run side by side. Results do not depend on the interleaving (every kernel's
arithmetic order is fixed), so a batch reproduces the one-by-one solutions bit for bit.
"""
from __future__ import annotations

import concurrent.futures as cf
import threading
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


def solve_one(item: BatchItem, rtol: float = 1e-12, maxit: int = 500, stream=None):
    """(u, iterations, relative residual) for one problem on `stream` (the current stream if
    None); the factor is released before returning."""
    csr = rhif.assemble_fd(item.dim, item.n, item.a_cells, item.b, stream=stream)
    F = rhif.Factor(item.dim, item.n, csr, item.leaf, item.eps, 1, stream=stream)
    try:
        u, it, rr = F.pcg(item.f, rtol, maxit, stream=stream)
    finally:
        F.close()
    return u, it, rr


def solve_many(items, nstreams: int = 4, rtol: float = 1e-12, maxit: int = 500):
    """Solve every item; returns [(u, iterations, relative residual)] in the items' order.
    nstreams worker threads, one default-priority HIP stream each."""
    import torch
    out = [None] * len(items)
    nxt = [0]
    lock = threading.Lock()

    def worker():
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            while True:
                with lock:
                    i = nxt[0]
                    nxt[0] += 1
                if i >= len(items):
                    break
                out[i] = solve_one(items[i], rtol, maxit)
        st.synchronize()

    with cf.ThreadPoolExecutor(max_workers=max(1, nstreams)) as ex:
        for fut in [ex.submit(worker) for _ in range(max(1, nstreams))]:
            fut.result()
    return out
