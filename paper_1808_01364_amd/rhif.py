"""Python binding of librhif.so (the C ABI in include/rhif.h).

Argument marshalling only: torch tensors supply device memory and the current HIP
stream; every step of the factorization, the apply and the solve runs in the library's
HIP kernels. There is no fallback: without the built library, or without a GPU, the
calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Tuple

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librhif.so")

RHIF_OK, RHIF_EINVAL, RHIF_ENOTSPD, RHIF_ENOMEM, RHIF_EDEVICE, RHIF_ENOCONV = range(6)
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOTSPD", 3: "ENOMEM", 4: "EDEVICE", 5: "ENOCONV"}
MAX_LEVELS = 32
FLAG_PHASE_TIMES = 1
FLAG_KERNEL_TIMES = 2
KERNEL_MASK_SHIFT = 8
FLAG_SOLVE_GRAPHS = 8
FLAG_GLOBAL_STAGING = 16
FLAG_SKEL_MULTI = 32
NUM_KCLASS = 16
NOALLOC_MAX_N = 1 << 20
KCLASS_NAMES = ["front_csr", "front_extend", "elim_leaf", "elim_upper", "root", "precond_chol",
                "precond_scale", "skeletonize", "apply_up", "apply_down", "apply_gather", "spmv",
                "vector", "-", "-", "-"]

# every function declared in include/rhif.h
EXPORTED = ["rhif_fd_nnz", "rhif_assemble_fd", "rhif_factor", "rhif_factor_batch", "rhif_apply", "rhif_pcg_solve",
            "rhif_apply_batch", "rhif_pcg_solve_batch",
            "rhif_pcg_solve_noalloc", "rhif_apply_half", "rhif_estimate_es",
            "rhif_apply_forward", "rhif_estimate_ea", "rhif_matvec", "rhif_grad_log_a", "rhif_stats", "rhif_skeletons", "rhif_destroy",
            "rhif_last_error", "rhif_version"]


class RhifError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class NotSPD(RhifError):
    pass


class NoConvergence(RhifError):
    def __init__(self, status, msg, iters, relres):
        super().__init__(status, msg)
        self.iters, self.relres = iters, relres


class Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 3)]


class Opts(ctypes.Structure):
    _fields_ = [("leaf", ctypes.c_int32), ("eps", ctypes.c_double), ("precond", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("root_size", ctypes.c_int32),
                ("factor_bytes", ctypes.c_int64),
                ("n_active", ctypes.c_int64 * (MAX_LEVELS + 1)),
                ("n_cells", ctypes.c_int32 * (MAX_LEVELS + 1)),
                ("max_front", ctypes.c_int32 * (MAX_LEVELS + 1)),
                ("n_groups", ctypes.c_int32 * MAX_LEVELS),
                ("n_skel", ctypes.c_int32 * MAX_LEVELS),
                ("sum_skel_n", ctypes.c_int64 * MAX_LEVELS),
                ("sum_rank", ctypes.c_int64 * MAX_LEVELS),
                ("max_rank", ctypes.c_int32 * MAX_LEVELS),
                ("flops", ctypes.c_double * (MAX_LEVELS + 1)),
                ("t_total_ms", ctypes.c_double),
                ("t_phase_ms", ctypes.c_double * 8),
                ("kernel_ms", ctypes.c_double * NUM_KCLASS),
                ("kernel_launches", ctypes.c_int64 * NUM_KCLASS),
                ("kernel_flops", ctypes.c_double * NUM_KCLASS),
                ("kernel_bytes", ctypes.c_double * NUM_KCLASS),
                ("sublevels", ctypes.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load librhif.so; raises if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1808_01364_amd.build`")
    lib = ctypes.CDLL(path)
    c_i32p = ctypes.POINTER(ctypes.c_int32)
    vp = ctypes.c_void_p
    lib.rhif_fd_nnz.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(ctypes.c_int64)]
    lib.rhif_assemble_fd.argtypes = [ctypes.POINTER(Grid), vp, vp, vp, vp, vp, vp]
    lib.rhif_factor.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Opts), vp, vp, vp, vp, ctypes.POINTER(vp)]
    lib.rhif_factor_batch.argtypes = [ctypes.c_int32, ctypes.POINTER(Grid), ctypes.POINTER(Opts),
                                      ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), vp,
                                      ctypes.POINTER(vp)]
    lib.rhif_apply.argtypes = [vp, vp, vp, ctypes.c_int32, vp]
    lib.rhif_apply_batch.argtypes = [ctypes.c_int32, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
    lib.rhif_pcg_solve_batch.argtypes = [ctypes.c_int32, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                         ctypes.c_double, ctypes.c_int32, c_i32p, ctypes.POINTER(ctypes.c_double), vp]
    lib.rhif_pcg_solve.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.c_int32, c_i32p,
                                   ctypes.POINTER(ctypes.c_double), vp]
    lib.rhif_pcg_solve_noalloc.argtypes = lib.rhif_pcg_solve.argtypes
    lib.rhif_matvec.argtypes = [vp, vp, vp, vp]
    lib.rhif_apply_half.argtypes = [vp, vp, vp, ctypes.c_int32, vp]
    lib.rhif_apply_forward.argtypes = [vp, vp, vp, vp]
    lib.rhif_estimate_ea.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                     c_i32p, vp]
    lib.rhif_estimate_es.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                     c_i32p, vp]
    lib.rhif_grad_log_a.argtypes = [ctypes.POINTER(Grid), vp, vp, vp, vp, vp]
    lib.rhif_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    lib.rhif_skeletons.argtypes = [vp, ctypes.c_int32, c_i32p, ctypes.POINTER(ctypes.c_int64), c_i32p, c_i32p,
                                   c_i32p, c_i32p]
    lib.rhif_destroy.argtypes = [vp]
    lib.rhif_destroy.restype = None
    lib.rhif_last_error.restype = ctypes.c_char_p
    lib.rhif_version.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name not in ("rhif_destroy", "rhif_last_error", "rhif_version"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(st: int):
    if st != RHIF_OK:
        msg = load_library().rhif_last_error().decode()
        if st == RHIF_ENOTSPD:
            raise NotSPD(st, msg)
        raise RhifError(st, msg)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("librhif needs a GPU; torch.cuda is not available")
    return torch


def _stream(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t) -> int:
    return int(t.data_ptr()) if t is not None else 0


def _need(*specs):
    """Check tensors handed to the library before any device work. Each spec is
    (tensor, name, numel) or (tensor, name, numel, dtype); dtype defaults to float64. First
    every tensor's dtype, size (the kernels read and write exactly `numel` elements through
    its pointer) and contiguity, then that every one lives on a GPU. Raises ValueError."""
    for spec in specs:
        t, name, numel = spec[:3]
        dtype = spec[3] if len(spec) > 3 else "float64"
        if t is None or not hasattr(t, "data_ptr"):
            raise ValueError(f"{name} must be a torch tensor")
        if str(t.dtype) != f"torch.{dtype}":
            raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
        if t.numel() != numel:
            raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
    for spec in specs:
        t, name = spec[:2]
        if t.device.type != "cuda":
            raise ValueError(f"{name} must be a GPU (cuda) tensor, got device {t.device}")


def make_grid(dim: int, n: int) -> Grid:
    g = Grid()
    g.dim = dim
    g.n[0] = n
    g.n[1] = n
    g.n[2] = n if dim == 3 else 0
    return g


def fd_nnz(dim: int, n: int) -> int:
    out = ctypes.c_int64()
    _check(load_library().rhif_fd_nnz(ctypes.byref(make_grid(dim, n)), ctypes.byref(out)))
    return out.value


def assemble_fd(dim: int, n: int, a_cells, b=None, stream=None):
    """CSR (row_ptr, col, val) of the FD matrix, as device tensors (int32, int32, float64).
    a_cells: (n+1)^dim cell coefficients on the device, c_1 fastest; b: N values or None."""
    N = n ** dim
    _need((a_cells, "a_cells", (n + 1) ** dim), *([(b, "b", N)] if b is not None else []))
    torch = _torch()
    dev = a_cells.device
    nnz = fd_nnz(dim, n)
    rp = torch.empty(N + 1, dtype=torch.int32, device=dev)
    col = torch.empty(nnz, dtype=torch.int32, device=dev)
    val = torch.empty(nnz, dtype=torch.float64, device=dev)
    _check(load_library().rhif_assemble_fd(ctypes.byref(make_grid(dim, n)), _ptr(a_cells), _ptr(b),
                                           _ptr(rp), _ptr(col), _ptr(val), _stream(stream)))
    return rp, col, val


def grad_log_a(dim: int, n: int, a_cells, u, lam, stream=None):
    """Per-cell -a_c lam^T (dA/da_c) u as a device tensor of (n+1)^dim values (c_1 fastest):
    the gradient with respect to log a of a loss of the solution u when A lam = dL/du."""
    N = n ** dim
    _need((a_cells, "a_cells", (n + 1) ** dim), (u, "u", N), (lam, "lam", N))
    torch = _torch()
    g = torch.empty_like(a_cells)
    _check(load_library().rhif_grad_log_a(ctypes.byref(make_grid(dim, n)), _ptr(a_cells), _ptr(u), _ptr(lam),
                                          _ptr(g), _stream(stream)))
    return g


@dataclass
class Skeletons:
    first_dof: List[int]
    size: List[int]
    rank: List[int]
    perm: List[List[int]]


class Factor:
    """An RHIF factorization held by the library (rhif_factor / rhif_destroy)."""

    def __init__(self, dim: int, n: int, csr, leaf: int, eps: float, precond: int = 1,
                 precision: int = 0, flags: int = 0, stream=None):
        self._h = None
        self.dim, self.n, self.N = dim, n, n ** dim
        rp, col, val = csr
        nnz = fd_nnz(dim, n)
        _need((rp, "row_ptr", self.N + 1, "int32"), (col, "col", nnz, "int32"), (val, "val", nnz))
        self._lib = load_library()
        o = Opts()
        o.leaf, o.eps, o.precond, o.precision, o.flags = leaf, eps, precond, precision, flags
        h = ctypes.c_void_p()
        _check(self._lib.rhif_factor(ctypes.byref(make_grid(dim, n)), ctypes.byref(o), _ptr(rp), _ptr(col),
                                     _ptr(val), _stream(stream), ctypes.byref(h)))
        self._h = h

    @classmethod
    def _adopt(cls, dim: int, n: int, h: ctypes.c_void_p) -> "Factor":
        self = cls.__new__(cls)
        self.dim, self.n, self.N = dim, n, n ** dim
        self._lib = load_library()
        self._h = h
        return self

    @property
    def handle(self):
        if self._h is None or not self._h.value:
            raise RuntimeError("factor has been destroyed")
        return self._h

    def apply(self, r, out=None, stream=None):
        """z = F^-1 r for r of shape (N,) or (nrhs, N) (rows are right-hand sides)."""
        if r is None or r.dim() not in (1, 2) or r.shape[-1] != self.N:
            raise ValueError(f"r must have shape ({self.N},) or (nrhs, {self.N})")
        nrhs = 1 if r.dim() == 1 else r.shape[0]
        if out is not None and tuple(out.shape) != tuple(r.shape):
            raise ValueError(f"out must have the shape of r, {tuple(r.shape)}")
        _need((r, "r", nrhs * self.N), *([(out, "out", nrhs * self.N)] if out is not None else []))
        torch = _torch()
        z = out if out is not None else torch.empty_like(r)
        _check(self._lib.rhif_apply(self.handle, _ptr(r), _ptr(z), nrhs, _stream(stream)))
        return z

    def apply_half(self, r, transpose: bool = False, out=None, stream=None):
        """z = G^-1 r (transpose=False) or G^-T r (transpose=True), F = G G^T."""
        _need((r, "r", self.N), *([(out, "out", self.N)] if out is not None else []))
        torch = _torch()
        z = out if out is not None else torch.empty_like(r)
        _check(self._lib.rhif_apply_half(self.handle, _ptr(r), _ptr(z), 1 if transpose else 0, _stream(stream)))
        return z

    def apply_forward(self, x, out=None, stream=None):
        """y = F x = G G^T x (the forward product of the factorization)."""
        _need((x, "x", self.N), *([(out, "out", self.N)] if out is not None else []))
        torch = _torch()
        y = out if out is not None else torch.empty_like(x)
        _check(self._lib.rhif_apply_forward(self.handle, _ptr(x), _ptr(y), _stream(stream)))
        return y

    def _start(self, v0, seed):
        torch = _torch()
        if v0 is None:
            import numpy as np
            v0 = torch.tensor(np.random.default_rng(seed).standard_normal(self.N), dtype=torch.float64,
                              device="cuda")
        _need((v0, "v0", self.N))
        return v0

    def estimate_ea(self, v0=None, seed: int = 0, maxit: int = 50, rtol: float = 1e-2, stream=None):
        """(e_a, iterations): ||A - F||_2 / ||A||_2 by power iteration (Sec. 4); start vector as
        for estimate_es."""
        v0 = self._start(v0, seed)
        ea = ctypes.c_double()
        it = ctypes.c_int32()
        _check(self._lib.rhif_estimate_ea(self.handle, _ptr(v0), maxit, rtol, ctypes.byref(ea), ctypes.byref(it),
                                          _stream(stream)))
        return ea.value, it.value

    def estimate_es(self, v0=None, seed: int = 0, maxit: int = 50, rtol: float = 1e-2, stream=None):
        """(e_s, iterations): ||I - G^-1 A G^-T||_2 by power iteration (Sec. 4). The start vector
        is v0 (device, N values) or, if None, numpy.random.default_rng(seed).standard_normal(N)."""
        v0 = self._start(v0, seed)
        es = ctypes.c_double()
        it = ctypes.c_int32()
        _check(self._lib.rhif_estimate_es(self.handle, _ptr(v0), maxit, rtol, ctypes.byref(es), ctypes.byref(it),
                                          _stream(stream)))
        return es.value, it.value

    def matvec(self, x, out=None, stream=None):
        _need((x, "x", self.N), *([(out, "out", self.N)] if out is not None else []))
        torch = _torch()
        y = out if out is not None else torch.empty_like(x)
        _check(self._lib.rhif_matvec(self.handle, _ptr(x), _ptr(y), _stream(stream)))
        return y

    def pcg(self, f, rtol: float = 1e-12, maxit: int = 500, out=None, stream=None,
            raise_on_noconv: bool = True, noalloc: bool = False) -> Tuple[object, int, float]:
        """(u, iterations, final relative residual) of the PCG solve A u = f. noalloc=True calls
        rhif_pcg_solve_noalloc (workspace in the library's device array; needs `out`)."""
        _need((f, "f", self.N), *([(out, "out", self.N)] if out is not None else []))
        torch = _torch()
        u = out if out is not None else torch.empty_like(f)
        it = ctypes.c_int32()
        rel = ctypes.c_double()
        fn = self._lib.rhif_pcg_solve_noalloc if noalloc else self._lib.rhif_pcg_solve
        st = fn(self.handle, _ptr(f), _ptr(u), rtol, maxit, ctypes.byref(it), ctypes.byref(rel), _stream(stream))
        if st == RHIF_ENOCONV:
            if raise_on_noconv:
                raise NoConvergence(st, self._lib.rhif_last_error().decode(), it.value, rel.value)
        else:
            _check(st)
        return u, it.value, rel.value

    def stats(self) -> dict:
        s = Stats()
        _check(self._lib.rhif_stats(self.handle, ctypes.byref(s)))
        L = s.levels
        return dict(levels=L, sublevels=s.sublevels, root_size=s.root_size, factor_bytes=s.factor_bytes,
                    n_active=list(s.n_active[: L + 1]), n_cells=list(s.n_cells[: L + 1]),
                    max_front=list(s.max_front[: L + 1]), n_groups=list(s.n_groups[:L]),
                    n_skel=list(s.n_skel[:L]), sum_skel_n=list(s.sum_skel_n[:L]),
                    sum_rank=list(s.sum_rank[:L]), max_rank=list(s.max_rank[:L]),
                    flops=list(s.flops[: L + 1]), t_total_ms=s.t_total_ms,
                    t_phase_ms=list(s.t_phase_ms),
                    kernels={KCLASS_NAMES[c]: dict(ms=s.kernel_ms[c], launches=s.kernel_launches[c],
                                                   flops=s.kernel_flops[c], bytes=s.kernel_bytes[c])
                             for c in range(NUM_KCLASS) if s.kernel_launches[c] > 0})

    def kernel_class(self, name: str):
        """The HIP-event timing of one kernel class (dict of ms, launches, flops, bytes, or None):
        the part of stats() a timing loop needs, without building the whole dictionary."""
        s = getattr(self, "_stats_buf", None)
        if s is None:
            s = self._stats_buf = Stats()
        _check(self._lib.rhif_stats(self.handle, ctypes.byref(s)))
        c = KCLASS_NAMES.index(name)
        if s.kernel_launches[c] <= 0:
            return None
        return dict(ms=s.kernel_ms[c], launches=s.kernel_launches[c], flops=s.kernel_flops[c],
                    bytes=s.kernel_bytes[c])

    def skeletons(self, level: int) -> Skeletons:
        ng = ctypes.c_int32()
        tot = ctypes.c_int64()
        _check(self._lib.rhif_skeletons(self.handle, level, ctypes.byref(ng), ctypes.byref(tot),
                                        None, None, None, None))
        n = ng.value
        A = ctypes.c_int32 * max(n, 1)
        fd, sz, rk = A(), A(), A()
        pm = (ctypes.c_int32 * max(tot.value, 1))()
        _check(self._lib.rhif_skeletons(self.handle, level, ctypes.byref(ng), ctypes.byref(tot), fd, sz, rk, pm))
        perms, off = [], 0
        for e in range(n):
            perms.append(list(pm[off: off + sz[e]]))
            off += sz[e]
        return Skeletons(list(fd[:n]), list(sz[:n]), list(rk[:n]), perms)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.rhif_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def factor_batch(problems, leaf: int, eps: float, precond: int = 1, precision: int = 0, flags: int = 0,
                 stream=None) -> List[Factor]:
    """Factor independent problems together (rhif_factor_batch): problems is a list of
    (dim, n, csr) with csr = (row_ptr, col, val) device tensors as for Factor. Returns one
    Factor per problem, each bitwise the one Factor(dim, n, csr, ...) would give."""
    if not problems:
        return []
    lib = load_library()
    count = len(problems)
    grids = (Grid * count)()
    rps, cols, vals = ((ctypes.c_void_p * count)() for _ in range(3))
    for i, (dim, n, csr) in enumerate(problems):
        rp, col, val = csr
        nnz = fd_nnz(dim, n)
        _need((rp, f"row_ptr[{i}]", n ** dim + 1, "int32"), (col, f"col[{i}]", nnz, "int32"),
              (val, f"val[{i}]", nnz))
        grids[i] = make_grid(dim, n)
        rps[i], cols[i], vals[i] = _ptr(rp), _ptr(col), _ptr(val)
    o = Opts()
    o.leaf, o.eps, o.precond, o.precision, o.flags = leaf, eps, precond, precision, flags
    hs = (ctypes.c_void_p * count)()
    _check(lib.rhif_factor_batch(count, grids, ctypes.byref(o), rps, cols, vals, _stream(stream), hs))
    return [Factor._adopt(dim, n, ctypes.c_void_p(hs[i])) for i, (dim, n, _) in enumerate(problems)]


def _batch_handles(factors):
    hs = (ctypes.c_void_p * len(factors))()
    for i, F in enumerate(factors):
        hs[i] = F.handle.value
    return hs


def apply_batch(factors, rs, out=None, stream=None):
    """[F_i^-1 r_i] for the factors of one factor_batch call (all of them, in order), in one
    joint apply (rhif_apply_batch)."""
    if len(rs) != len(factors):
        raise ValueError("one right-hand side per factor")
    _need(*[(r, f"r[{i}]", F.N) for i, (F, r) in enumerate(zip(factors, rs))])
    torch = _torch()
    zs = out if out is not None else [torch.empty_like(r) for r in rs]
    _need(*[(z, f"out[{i}]", F.N) for i, (F, z) in enumerate(zip(factors, zs))])
    n = len(factors)
    rp, zp = (ctypes.c_void_p * n)(*[_ptr(r) for r in rs]), (ctypes.c_void_p * n)(*[_ptr(z) for z in zs])
    _check(load_library().rhif_apply_batch(n, _batch_handles(factors), rp, zp, _stream(stream)))
    return zs


def pcg_batch(factors, fs, rtol: float = 1e-12, maxit: int = 500, out=None, stream=None,
              raise_on_noconv: bool = True):
    """[(u_i, iterations_i, relative residual_i)] of A_i u_i = f_i for the factors of one
    factor_batch call (all of them, in order), solved together (rhif_pcg_solve_batch)."""
    if len(fs) != len(factors):
        raise ValueError("one right-hand side per factor")
    _need(*[(f, f"f[{i}]", F.N) for i, (F, f) in enumerate(zip(factors, fs))])
    torch = _torch()
    us = out if out is not None else [torch.empty_like(f) for f in fs]
    _need(*[(u, f"out[{i}]", F.N) for i, (F, u) in enumerate(zip(factors, us))])
    n = len(factors)
    fp, up = (ctypes.c_void_p * n)(*[_ptr(f) for f in fs]), (ctypes.c_void_p * n)(*[_ptr(u) for u in us])
    it = (ctypes.c_int32 * n)()
    rel = (ctypes.c_double * n)()
    lib = load_library()
    st = lib.rhif_pcg_solve_batch(n, _batch_handles(factors), fp, up, rtol, maxit, it, rel, _stream(stream))
    if st == RHIF_ENOCONV:
        if raise_on_noconv:
            raise NoConvergence(st, lib.rhif_last_error().decode(), list(it), list(rel))
    else:
        _check(st)
    return [(u, it[i], rel[i]) for i, u in enumerate(us)]


def version() -> str:
    return load_library().rhif_version().decode()


# ---------------------------------------------------------------- host-only planner check

_ID_FN = ctypes.CFUNCTYPE(ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                          ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32))
_CELL_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                            ctypes.c_int32, ctypes.POINTER(ctypes.c_int32))


def plan_dry_run(dim: int, n: int, leaf: int, choose, on_cell=None) -> int:
    """Run the library's level planner on the host (no GPU) with ID choices from
    ``choose(level, first_dof, size) -> (k, perm)``; ``on_cell(level, cell, interior,
    boundary)`` sees every cell with interior unknowns. Returns |S_L|."""
    lib = load_library()
    lib.rhif_plan_dry_run.argtypes = [ctypes.POINTER(Grid), ctypes.c_int32, _ID_FN, ctypes.c_void_p, _CELL_FN,
                                      ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]
    lib.rhif_plan_dry_run.restype = ctypes.c_int
    lib.rhif_plan_last_error.restype = ctypes.c_char_p
    errors = []

    def _id(ctx, level, first, size, kp, pp):
        try:
            k, perm = choose(level, first, size)
            kp[0] = int(k)
            for q in range(size):
                pp[q] = int(perm[q])
            return 0
        except Exception as e:  # reported after the run
            errors.append(e)
            return 1

    def _cell(ctx, level, cell, nI, nB, dofs):
        if on_cell is not None:
            arr = [dofs[q] for q in range(nI + nB)]
            on_cell(level, cell, arr[:nI], arr[nI:])

    idf, cellf = _ID_FN(_id), _CELL_FN(_cell)
    root = ctypes.c_int64()
    st = lib.rhif_plan_dry_run(ctypes.byref(make_grid(dim, n)), leaf, idf, None, cellf, None, ctypes.byref(root))
    if errors:
        raise errors[0]
    if st != RHIF_OK:
        raise RhifError(st, lib.rhif_plan_last_error().decode())
    return root.value
