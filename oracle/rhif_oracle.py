"""Plain, slow, FP64 CPU oracle of the recursively preconditioned hierarchical interpolative
factorization (called PHIF in the paper, RHIF here) and of the preconditioned CG solve
that uses it.

THIS IS TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import or run it. The product path (the HIP library and its
Python binding) never calls it and shares no code with it; the only thing both sides
share is the seeded input generator in ``workloads``.

Every step keeps the whole current matrix A_l as one global scipy.sparse matrix over the
original N unknowns and works on dense submatrices pulled out of it, so each formula can
be read against the paper directly:

* assembly .................. eq. (1.1)-(1.2), 5-/7-point stencils of Sec. 3.1 / 3.2
* DOF grouping .............. Sec. 3.1 (interior / edge / corner), Sec. 3.2 (+ faces)
* cell elimination E_l ...... Sec. 2.1, eq. (2.1) and the Schur complement after it
* block Jacobi C_l .......... Sec. 2.3, eq. (2.3)
* skeletonization K_l ....... Sec. 2.2 (ID, eq. (2.2), redundant elimination), done
                               "simultaneously": every ID first, then every Z and E
* root and F^{-1} ........... Sec. 3.1, eqs. (3.1)-(3.3)
* CG with F^{-1} ............ Sec. 4 (relative residual 1e-12)

Readings where the paper leaves a choice open (each is restated where it is used):

R1  grid: unknowns at x in {1..s}^d, h = 1/(s+1); level-l separators are the unknowns
    with some x_k divisible by w = 2^l m; levels run while w <= s, and the root is what
    is left (this is the paper's tree exactly when s = 2^L m - 1).
R2  a is constant per grid cell; the coefficient on a grid edge is the mean over the
    2^(d-1) cells that contain that edge; A = h^-2 (diffusion) + diag(b).
R3  ID: Householder QR with column pivoting on the recomputed 2-norms of the trailing
    columns (ties to the lowest column); rank k = number of leading |R_jj| > eps |R_11|,
    stopping at the first failure; T = R11^-1 R12.
R4  the block-Jacobi step treats every separator group (edges and corners in 2D; faces,
    edges and corners in 3D); only edges (2D) / faces (3D) are skeletonized.
R5  DOFs inside any group are kept in ascending linear index; cell boundaries B are the
    active separator unknowns on the closed cell.
R6  a Cholesky pivot that is <= 0 or not finite is a loss of positive definiteness and
    stops the factorization (NotSPDError); nothing is shifted or regularized.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from itertools import product
from typing import Dict, List, Optional, Tuple

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


class NotSPDError(RuntimeError):
    """A Cholesky pivot was <= 0 or not finite (loss of positive definiteness)."""

    def __init__(self, level: int, step: str, block: int, detail: str = ""):
        super().__init__(f"not SPD at level {level}, step {step}, block {block} {detail}")
        self.level, self.step, self.block = level, step, block


# ----------------------------------------------------------------------------------------
# Grid and assembly (eq. (1.1), (1.2); five-point stencil of Sec. 3.1, seven-point of 3.2)
# ----------------------------------------------------------------------------------------

def dof_coords(d: int, s: int) -> np.ndarray:
    """(N, d) integer grid coordinates x_k in 1..s of every DOF (x_1 fastest)."""
    idx = np.arange(s ** d, dtype=np.int64)
    return np.stack([(idx // s ** k) % s + 1 for k in range(d)], axis=1)


def _edge_coefficient(a_cells: np.ndarray, d: int, s: int, k: int) -> np.ndarray:
    """Coefficient of every grid edge from x to x + e_k, for x with x_k in 0..s and the
    other coordinates in 1..s (reading R2): the mean of the 2^(d-1) cells containing it.

    Returned with shape (s+1 along axis k, s along the others), indexed like a_cells
    ([x_d, ..., x_1] with the ghost-inclusive range along k)."""
    # a_cells is indexed [c_d, ..., c_1]; numpy axis for coordinate k is d-1-k.
    ax_k = d - 1 - k
    acc = np.zeros(tuple((s + 1) if (d - 1 - ax) == k else s for ax in range(d)))
    count = 0
    # cells containing the edge: c_k = x_k, and c_j in {x_j - 1, x_j} for j != k
    others = [j for j in range(d) if j != k]
    for shifts in product((0, 1), repeat=len(others)):
        sl = [slice(None)] * d
        for j, sh in zip(others, shifts):
            ax = d - 1 - j
            # x_j in 1..s and c_j = x_j - 1 + sh  -> slice [sh, sh + s)
            sl[ax] = slice(sh, sh + s)
        sl[ax_k] = slice(0, s + 1)
        acc += a_cells[tuple(sl)]
        count += 1
    return acc / count


def assemble_fd(d: int, s: int, a_cells: np.ndarray, b: Optional[np.ndarray] = None) -> sp.csr_matrix:
    """Finite-difference matrix of -div(a grad u) + b u on the interior grid with zero
    Dirichlet ghosts (eq. (1.1)-(1.2), Sec. 3.1 / 3.2; readings R1, R2).

    For every grid edge (x, x+e_k) with coefficient alpha: both endpoints that are
    unknowns get +alpha/h^2 on the diagonal, and if both are unknowns they are coupled
    by -alpha/h^2. b is added to the diagonal (not scaled by h^2)."""
    a_cells = np.asarray(a_cells, dtype=np.float64)
    assert a_cells.shape == (s + 1,) * d
    N = s ** d
    h = 1.0 / (s + 1)
    inv_h2 = 1.0 / (h * h)
    diag = np.zeros((s,) * d)
    rows, cols, vals = [], [], []
    lin = np.arange(N).reshape((s,) * d)
    for k in range(d):
        ax = d - 1 - k
        alpha = _edge_coefficient(a_cells, d, s, k) * inv_h2   # edges x_k = 0..s -> x_k+1
        # endpoint x (x_k in 1..s) owns edges to x - e_k (index x_k-1) and x + e_k (index x_k)
        lo = [slice(None)] * d
        hi = [slice(None)] * d
        lo[ax] = slice(0, s)        # edge from x - e_k to x
        hi[ax] = slice(1, s + 1)    # edge from x to x + e_k
        diag += alpha[tuple(lo)] + alpha[tuple(hi)]
        # couplings between interior neighbours: edges with x_k in 1..s-1
        mid = [slice(None)] * d
        mid[ax] = slice(1, s)
        a_in = alpha[tuple(mid)]
        left = [slice(None)] * d
        right = [slice(None)] * d
        left[ax] = slice(0, s - 1)
        right[ax] = slice(1, s)
        i = lin[tuple(left)].ravel()
        j = lin[tuple(right)].ravel()
        v = -a_in.ravel()
        rows += [i, j]
        cols += [j, i]
        vals += [v, v]
    dvec = diag.ravel()
    if b is not None:
        dvec = dvec + np.asarray(b, dtype=np.float64)
    rows.append(np.arange(N))
    cols.append(np.arange(N))
    vals.append(dvec)
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A


def fd_energy(d: int, s: int, a_cells: np.ndarray, b: Optional[np.ndarray], u: np.ndarray) -> float:
    """u^T A u written cell by cell: every cell c adds a_c * 2^(1-d) * (u(p)-u(q))^2 / h^2
    for each of its grid edges (p, q), plus sum b u^2 (ghost values are zero). Used only
    to pin the assembly from an independent direction."""
    h = 1.0 / (s + 1)
    ug = np.zeros((s + 2,) * d)
    ug[(slice(1, s + 1),) * d] = np.asarray(u).reshape((s,) * d)
    total = 0.0
    w = 2.0 ** (1 - d)
    for k in range(d):
        ax = d - 1 - k
        # difference along k for every edge (x_k = 0..s) at every transverse grid point 0..s+1
        sl_hi = [slice(None)] * d
        sl_lo = [slice(None)] * d
        sl_hi[ax] = slice(1, s + 2)
        sl_lo[ax] = slice(0, s + 1)
        diff2 = (ug[tuple(sl_hi)] - ug[tuple(sl_lo)]) ** 2   # shape: s+1 along k, s+2 others
        # a cell (c) contains the edges whose transverse coordinates are c_j or c_j+1
        others = [j for j in range(d) if j != k]
        for shifts in product((0, 1), repeat=len(others)):
            sl = [slice(None)] * d
            for j, sh in zip(others, shifts):
                sl[d - 1 - j] = slice(sh, sh + s + 1)
            sl[ax] = slice(0, s + 1)
            total += w * float(np.sum(a_cells * diff2[tuple(sl)]))
    total /= h * h
    if b is not None:
        total += float(np.sum(np.asarray(b) * np.asarray(u) ** 2))
    return total


# ----------------------------------------------------------------------------------------
# Tree and DOF groups (Sec. 3.1 and 3.2; reading R1)
# ----------------------------------------------------------------------------------------

def num_levels(s: int, leaf: int) -> int:
    """Number L of elimination/skeletonization levels: all l >= 0 with 2^l m <= s."""
    L = 0
    while (leaf << L) <= s:
        L += 1
    return L


def classify(coords: np.ndarray, active: np.ndarray, w: int):
    """Group the active DOFs at cell width w.

    Each coordinate gets key_k = 2*(x_k // w) + (x_k % w != 0): even keys are separator
    planes x_k = (key_k/2) w, odd keys the open slab of cell index key_k // 2. DOFs with
    equal key tuples form one group; the group's class is the number of even components
    (0 = cell interior, 1 = edge in 2D / face in 3D, 2 = corner in 2D / edge in 3D,
    3 = corner in 3D).

    Returns a dict key_tuple -> ascending array of global DOF indices (reading R5) and a
    dict key_tuple -> class."""
    x = coords[active]
    key = 2 * (x // w) + (x % w != 0)
    cls = (x % w == 0).sum(axis=1)
    groups: Dict[tuple, np.ndarray] = {}
    gclass: Dict[tuple, int] = {}
    if len(active) == 0:
        return groups, gclass
    order = np.lexsort(key.T[::-1])  # deterministic order of the groups
    ks = key[order]
    brk = np.ones(len(order), dtype=bool)
    brk[1:] = np.any(ks[1:] != ks[:-1], axis=1)
    starts = np.flatnonzero(brk)
    ends = np.append(starts[1:], len(order))
    for a0, a1 in zip(starts, ends):
        kt = tuple(int(v) for v in ks[a0])
        members = np.sort(active[order[a0:a1]])
        groups[kt] = members
        gclass[kt] = int(cls[order[a0]])
    return groups, gclass


def closure_keys(cell_key: tuple) -> List[tuple]:
    """Keys of the separator groups on the closed boundary of a cell (3^d - 1 of them)."""
    out = []
    for off in product((-1, 0, 1), repeat=len(cell_key)):
        if all(o == 0 for o in off):
            continue
        out.append(tuple(c + o for c, o in zip(cell_key, off)))
    return out


# ----------------------------------------------------------------------------------------
# Dense primitives
# ----------------------------------------------------------------------------------------

def chol(Ablk: np.ndarray, level: int, step: str, block: int) -> np.ndarray:
    """Lower Cholesky factor; any pivot <= 0 or non-finite raises NotSPDError (R6)."""
    n = Ablk.shape[0]
    if n == 0:
        return np.zeros((0, 0))
    if not np.all(np.isfinite(Ablk)):
        raise NotSPDError(level, step, block, "(non-finite entries)")
    try:
        Lf = np.linalg.cholesky(Ablk)
    except np.linalg.LinAlgError as e:
        raise NotSPDError(level, step, block, str(e)) from None
    if not np.all(np.isfinite(Lf)) or np.any(np.diag(Lf) <= 0):
        raise NotSPDError(level, step, block, "(non-positive pivot)")
    return Lf


def cpqr_id(M: np.ndarray, eps: float, forced: Optional[Tuple[int, np.ndarray]] = None,
            trace: Optional[dict] = None):
    """Interpolative decomposition of the columns of M (Sec. 2.2, reading R3).

    Householder QR with column pivoting: at step j the pivot is the trailing column of
    largest recomputed 2-norm over rows j.. (ties -> lowest column). The rank k is the
    number of leading steps with |R_jj| > eps |R_11|, stopping at the first failure
    (eps = 0 keeps every step with |R_jj| > 0). With P the column permutation,
    M[:, P[k:]] ~= M[:, P[:k]] T,  T = R11^{-1} R12  (k x (n-k)).

    forced = (k, perm) replays a given rank and pivot order (QR of M[:, perm] without
    pivot search) so that arithmetic can be compared apart from discrete choices.

    Returns (k, perm, T, rdiag) with rdiag the |R_jj| of the steps taken.

    trace, if a dict, receives what decides the discrete choices (for telling a legitimate
    tie from a wrong choice; the arithmetic is unchanged): "norms", per pivot step, the
    trailing column norms indexed by original column (NaN for columns already chosen), and
    "stop_norm", the largest trailing norm at the step where the rank test failed (NaN if
    every step passed)."""
    M = np.array(M, dtype=np.float64, copy=True)
    r, n = M.shape
    perm = np.arange(n)
    if forced is not None:
        kf, pf = forced
        perm = np.asarray(pf, dtype=np.int64).copy()
        M = M[:, perm]
    kmax = min(r, n)
    rdiag = []
    r11 = 0.0
    k = 0
    if trace is not None:
        trace["norms"] = []
        trace["stop_norm"] = float("nan")
    for j in range(kmax):
        if forced is None:
            norms = np.sqrt(np.sum(M[j:, j:] ** 2, axis=0))
            if trace is not None:
                byc = np.full(n, np.nan)
                byc[perm[j:]] = norms
                trace["norms"].append(byc)
            p = j + int(np.argmax(norms))          # argmax returns the first maximum
            if p != j:
                M[:, [j, p]] = M[:, [p, j]]
                perm[[j, p]] = perm[[p, j]]
            nrm = float(norms[p - j])
        else:
            if j >= forced[0]:
                break
            nrm = float(np.sqrt(np.sum(M[j:, j] ** 2)))
        if j == 0:
            r11 = nrm
        if forced is None and not (nrm > eps * r11):
            if trace is not None:
                trace["stop_norm"] = nrm
            break
        x0 = M[j, j]
        alpha = -math.copysign(nrm, x0) if nrm > 0 else 0.0
        v = M[j:, j].copy()
        v[0] -= alpha
        vtv = float(v @ v)
        if vtv > 0.0:
            M[j:, j + 1:] -= np.outer(v, (2.0 / vtv) * (v @ M[j:, j + 1:]))
        M[j, j] = alpha
        M[j + 1:, j] = 0.0
        rdiag.append(abs(alpha))
        k = j + 1
    if forced is not None:
        k = int(forced[0])
    R11 = np.triu(M[:k, :k])
    R12 = M[:k, k:]
    T = sla.solve_triangular(R11, R12, lower=False) if k > 0 else np.zeros((0, n - k))
    return k, perm, T, np.array(rdiag)


# ----------------------------------------------------------------------------------------
# Factorization
# ----------------------------------------------------------------------------------------

@dataclass
class CellFactor:            # one E_I (eq. (2.1)): L = chol(A_II), W = L^-1 A_BI^T
    I: np.ndarray
    B: np.ndarray
    L: np.ndarray
    W: np.ndarray


@dataclass
class GroupFactor:           # one C_I (eq. (2.3)): L_g = chol(A_gg)
    idx: np.ndarray
    L: np.ndarray


@dataclass
class SkelFactor:            # one K_I = Z_I E_Itilde (eq. (2.2) and the elimination after it)
    key: tuple
    group: np.ndarray        # group DOFs, ascending
    hat: np.ndarray          # skeleton DOFs (pivot order)
    tilde: np.ndarray        # redundant DOFs (pivot order)
    perm: np.ndarray         # local pivot order of the group
    T: np.ndarray            # k x (n-k)
    Lt: np.ndarray           # chol of A~_{Itilde,Itilde}
    Wt: np.ndarray           # Lt^-1 A~_{Ihat,Itilde}^T
    rdiag: np.ndarray
    trace: Optional[dict] = None   # cpqr_id's record of the pivot norms (not replayed IDs)


@dataclass
class LevelFactor:
    level: int
    w: int
    cells: List[CellFactor] = field(default_factory=list)
    groups: List[GroupFactor] = field(default_factory=list)
    skels: List[SkelFactor] = field(default_factory=list)
    n_active: int = 0


@dataclass
class Factorization:
    d: int
    s: int
    leaf: int
    eps: float
    precond: int
    L: int
    N: int
    levels: List[LevelFactor]
    root_idx: np.ndarray
    root_L: np.ndarray
    schur_min_eig: List[float] = field(default_factory=list)

    @property
    def root_size(self) -> int:
        return len(self.root_idx)

    def ranks(self):
        """Per level: list of (group key, group size n, rank k)."""
        return [[(sk.key, len(sk.group), len(sk.hat)) for sk in lv.skels] for lv in self.levels]


def _sub(A: sp.csr_matrix, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    if len(rows) == 0 or len(cols) == 0:
        return np.zeros((len(rows), len(cols)))
    return A[rows][:, cols].toarray()


def _coo(N, rows, cols, vals):
    if not rows:
        return sp.csr_matrix((N, N))
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, N)).tocsr()


def _keep_only(A: sp.csr_matrix, active_mask: np.ndarray) -> sp.csr_matrix:
    """Zero every row and column of an eliminated DOF (they are decoupled identities)."""
    D = sp.diags(active_mask.astype(np.float64))
    A = (D @ A @ D).tocsr()
    A.eliminate_zeros()
    return A


def _assign_blocks(A: sp.csr_matrix, blocks) -> sp.csr_matrix:
    """Overwrite dense blocks: A[r, c] := V for each (r, c, V). Implemented as subtracting
    the old entries (exactly zero afterwards) and then adding the new ones."""
    N = A.shape[0]
    r_old, c_old, v_old, r_new, c_new, v_new = [], [], [], [], [], []
    for r, c, V in blocks:
        if len(r) == 0 or len(c) == 0:
            continue
        rr, cc = np.meshgrid(r, c, indexing="ij")
        r_old.append(rr.ravel()); c_old.append(cc.ravel())
        v_old.append(-_sub(A, r, c).ravel())
        r_new.append(rr.ravel()); c_new.append(cc.ravel())
        v_new.append(np.asarray(V, dtype=np.float64).ravel())
    A = (A + _coo(N, r_old, c_old, v_old)).tocsr()
    A = (A + _coo(N, r_new, c_new, v_new)).tocsr()
    A.eliminate_zeros()
    return A


def factor(A0: sp.csr_matrix, d: int, s: int, leaf: int, eps: float, precond: int = 1,
           replay: Optional[Dict[Tuple[int, int], Tuple[int, np.ndarray]]] = None,
           check_spd: bool = False) -> Factorization:
    """Recursively preconditioned HIF of the SPD matrix A0 (Sec. 3.1 / 3.2).

    For l = 0 .. L-1 (L = num_levels): cell elimination, block-Jacobi preconditioning of
    every separator group (skipped when precond = 0, i.e. plain HIF), and simultaneous
    skeletonization of every edge (2D) / face (3D). The remaining matrix A_L is factored
    densely (root). replay maps (level, smallest DOF of the group) -> (k, perm) to force
    the ID's discrete choices. check_spd additionally records the smallest eigenvalue of
    every Schur complement block (tiny problems only)."""
    if leaf < 2:
        raise ValueError("leaf must be >= 2")
    N = s ** d
    A = sp.csr_matrix(A0, dtype=np.float64, copy=True)
    coords = dof_coords(d, s)
    active_mask = np.ones(N, dtype=bool)
    L = num_levels(s, leaf)
    levels: List[LevelFactor] = []
    min_eigs: List[float] = []

    for lvl in range(L):
        w = leaf << lvl
        lv = LevelFactor(level=lvl, w=w, n_active=int(active_mask.sum()))
        active = np.flatnonzero(active_mask)
        groups, gclass = classify(coords, active, w)

        # ---- (1) cell elimination: E_l = prod_i E_{I_i}  (Sec. 2.1, eq. (2.1)) ----
        upd_r, upd_c, upd_v = [], [], []
        for key in sorted(k for k in groups if gclass[k] == 0):
            I = groups[key]
            B = np.sort(np.concatenate([groups[bk] for bk in closure_keys(key) if bk in groups]
                                       + [np.zeros(0, dtype=np.int64)])).astype(np.int64)
            A_II = _sub(A, I, I)
            A_BI = _sub(A, B, I)
            Lc = chol(A_II, lvl, "E", int(I[0]))
            W = sla.solve_triangular(Lc, A_BI.T, lower=True) if len(B) else np.zeros((len(I), 0))
            lv.cells.append(CellFactor(I=I, B=B, L=Lc, W=W))
            if len(B):
                S = -(W.T @ W)                       # A_BB <- A_BB - A_BI A_II^-1 A_BI^T
                rr, cc = np.meshgrid(B, B, indexing="ij")
                upd_r.append(rr.ravel()); upd_c.append(cc.ravel()); upd_v.append(S.ravel())
            active_mask[I] = False
        A = (A + _coo(N, upd_r, upd_c, upd_v)).tocsr()
        A = _keep_only(A, active_mask)
        if check_spd:
            for cf in lv.cells:
                if len(cf.B):
                    min_eigs.append(float(np.linalg.eigvalsh(_sub(A, cf.B, cf.B)).min()))

        seps = sorted(k for k in groups if gclass[k] >= 1)

        # ---- (2) block Jacobi: A'' = C^T A' C, C = blockdiag(L_g^-T)  (Sec. 2.3) ----
        if precond:
            blocks = []
            for key in seps:
                g = groups[key]
                Lg = chol(_sub(A, g, g), lvl, "C", int(g[0]))
                lv.groups.append(GroupFactor(idx=g, L=Lg))
                blocks.append((g, sla.solve_triangular(Lg, np.eye(len(g)), lower=True)))
            # sparse block diagonal D = blockdiag(L_g^-1) in global numbering: A'' = D A' D^T
            dr, dc, dv = [], [], []
            for g, Linv in blocks:
                rr, cc = np.meshgrid(g, g, indexing="ij")
                dr.append(rr.ravel()); dc.append(cc.ravel()); dv.append(Linv.ravel())
            D = _coo(N, dr, dc, dv)
            A = (D @ A @ D.T).tocsr()
            # the diagonal blocks are the identity (unit block diagonal, Sec. 2.3)
            A = _assign_blocks(A, [(g, g, np.eye(len(g))) for g, _ in blocks])

        # ---- (3) skeletonization of edges (2D) / faces (3D), simultaneously (Sec. 2.2) ----
        Acsc = A.tocsc()
        ids = []
        for key in seps:
            if gclass[key] != 1:
                continue
            g = groups[key]
            col = Acsc[:, g].toarray()
            rowmask = np.any(col != 0.0, axis=1)
            rowmask[g] = False                       # R = every other active DOF
            M = col[rowmask]
            forced = None if replay is None else replay.get((lvl, int(g[0])))
            tr = {} if forced is None else None
            k, perm, T, rdiag = cpqr_id(M, eps, forced, trace=tr)
            ids.append((key, g, k, perm, T, rdiag, tr))
        assign = []
        for key, g, k, perm, T, rdiag, tr in ids:
            n = len(g)
            hat = g[perm[:k]]
            tilde = g[perm[k:]]
            Ahh = _sub(A, hat, hat)
            Aht = _sub(A, hat, tilde)                # A_{Ihat, Itilde}
            Att = _sub(A, tilde, tilde)
            # A~ blocks after zeroing with Z = [[I, 0], [-T, I]] (eq. (2.2) and below)
            Att_t = Att - T.T @ Aht - Aht.T @ T + T.T @ Ahh @ T
            Aht_t = Aht - Ahh @ T
            Lt = chol(Att_t, lvl, "K", int(g[0]))
            Wt = sla.solve_triangular(Lt, Aht_t.T, lower=True) if n - k > 0 else np.zeros((0, k))
            Ahh_new = Ahh - Wt.T @ Wt
            lv.skels.append(SkelFactor(key=key, group=g, hat=hat, tilde=tilde, perm=perm, T=T,
                                       Lt=Lt, Wt=Wt, rdiag=rdiag, trace=tr))
            assign.append((hat, hat, Ahh_new))
            active_mask[tilde] = False
        A = _assign_blocks(A, assign)
        A = _keep_only(A, active_mask)               # drops A_{R, Itilde} and eliminated rows
        levels.append(lv)

    # ---- root: A_L = B_L B_L^T on the remaining active DOFs (eq. (3.3)) ----
    root = np.flatnonzero(active_mask)
    RL = chol(_sub(A, root, root), L, "root", int(root[0]) if len(root) else 0)
    return Factorization(d=d, s=s, leaf=leaf, eps=eps, precond=precond, L=L, N=N,
                         levels=levels, root_idx=root, root_L=RL, schur_min_eig=min_eigs)


# ----------------------------------------------------------------------------------------
# Apply F^-1 = R_0 ... R_{L-1} A_L^-1 R_{L-1}^T ... R_0^T,  R_l = E_l C_l K_l  (eq. (3.2))
# ----------------------------------------------------------------------------------------

def apply_inverse(F: Factorization, r: np.ndarray) -> np.ndarray:
    """z = F^{-1} r. The up-sweep applies R_l^T = K_l^T C_l^T E_l^T for l = 0..L-1, the
    root applies A_L^{-1}, and the down-sweep applies R_l = E_l C_l K_l for l = L-1..0."""
    z = np.array(r, dtype=np.float64, copy=True)
    tri = sla.solve_triangular
    for lv in F.levels:
        # E^T: z_I <- L^-1 z_I ; z_B <- z_B - W^T z_I   (E_I^T from eq. (2.1))
        for c in lv.cells:
            zi = tri(c.L, z[c.I], lower=True)
            z[c.I] = zi
            if len(c.B):
                z[c.B] -= c.W.T @ zi
        # C^T: z_g <- L_g^-1 z_g
        for g in lv.groups:
            z[g.idx] = tri(g.L, z[g.idx], lower=True)
        # K^T = E_Itilde^T Z^T: z_tilde -= T^T z_hat ; z_tilde <- Lt^-1 z_tilde ; z_hat -= Wt^T z_tilde
        for sk in lv.skels:
            if len(sk.tilde) == 0:
                continue
            zt = z[sk.tilde] - sk.T.T @ z[sk.hat]
            zt = tri(sk.Lt, zt, lower=True)
            z[sk.tilde] = zt
            if len(sk.hat):
                z[sk.hat] -= sk.Wt.T @ zt
    if len(F.root_idx):
        y = tri(F.root_L, z[F.root_idx], lower=True)
        z[F.root_idx] = tri(F.root_L.T, y, lower=False)
    for lv in reversed(F.levels):
        # K = Z E_Itilde: z_tilde <- Lt^-T (z_tilde - Wt z_hat) ; z_hat -= T z_tilde
        for sk in lv.skels:
            if len(sk.tilde) == 0:
                continue
            zt = z[sk.tilde] - (sk.Wt @ z[sk.hat] if len(sk.hat) else 0.0)
            zt = tri(sk.Lt.T, zt, lower=False)
            z[sk.tilde] = zt
            if len(sk.hat):
                z[sk.hat] -= sk.T @ zt
        # C: z_g <- L_g^-T z_g
        for g in lv.groups:
            z[g.idx] = tri(g.L.T, z[g.idx], lower=False)
        # E: z_I <- L^-T (z_I - W z_B)
        for c in lv.cells:
            zi = z[c.I] - (c.W @ z[c.B] if len(c.B) else 0.0)
            z[c.I] = tri(c.L.T, zi, lower=False)
    return z


# ----------------------------------------------------------------------------------------
# The two halves of F^-1 = G^-T G^-1, the forward product F x = G G^T x, and the paper's
# accuracy measures e_a = ||A - F|| / ||A|| and e_s = ||I - G^-1 A G^-T|| (Sec. 3.1, eq. (3.3);
# Sec. 4), estimated by power iteration.
# ----------------------------------------------------------------------------------------

def apply_ginv(F: Factorization, r: np.ndarray) -> np.ndarray:
    """G^-1 r: the up-sweep R_0^T .. R_{L-1}^T of eq. (3.2), then the forward solve with the
    root factor B_L (A_L = B_L B_L^T), so that apply_ginv_t(apply_ginv(r)) = F^-1 r."""
    z = np.array(r, dtype=np.float64, copy=True)
    tri = sla.solve_triangular
    for lv in F.levels:
        for c in lv.cells:
            zi = tri(c.L, z[c.I], lower=True)
            z[c.I] = zi
            if len(c.B):
                z[c.B] -= c.W.T @ zi
        for g in lv.groups:
            z[g.idx] = tri(g.L, z[g.idx], lower=True)
        for sk in lv.skels:
            if len(sk.tilde) == 0:
                continue
            zt = tri(sk.Lt, z[sk.tilde] - sk.T.T @ z[sk.hat], lower=True)
            z[sk.tilde] = zt
            if len(sk.hat):
                z[sk.hat] -= sk.Wt.T @ zt
    if len(F.root_idx):
        z[F.root_idx] = tri(F.root_L, z[F.root_idx], lower=True)
    return z


def apply_ginv_t(F: Factorization, y: np.ndarray) -> np.ndarray:
    """G^-T y: the backward solve with B_L^T, then the down-sweep R_{L-1} .. R_0."""
    z = np.array(y, dtype=np.float64, copy=True)
    tri = sla.solve_triangular
    if len(F.root_idx):
        z[F.root_idx] = tri(F.root_L.T, z[F.root_idx], lower=False)
    for lv in reversed(F.levels):
        for sk in lv.skels:
            if len(sk.tilde) == 0:
                continue
            zt = tri(sk.Lt.T, z[sk.tilde] - (sk.Wt @ z[sk.hat] if len(sk.hat) else 0.0), lower=False)
            z[sk.tilde] = zt
            if len(sk.hat):
                z[sk.hat] -= sk.T @ zt
        for g in lv.groups:
            z[g.idx] = tri(g.L.T, z[g.idx], lower=False)
        for c in lv.cells:
            z[c.I] = tri(c.L.T, z[c.I] - (c.W @ z[c.B] if len(c.B) else 0.0), lower=False)
    return z


def apply_forward(F: Factorization, x: np.ndarray) -> np.ndarray:
    """F x = G G^T x, the generalized Cholesky form of eq. (3.3), by undoing each step of the
    two sweeps in reverse order: G^T x undoes the down-sweep (level 0 first: E_0, then C_0,
    then K_0, ...) and the backward root solve; G y undoes the forward root solve and the
    up-sweep (level L-1 first: K^T, C^T, E^T)."""
    z = np.array(x, dtype=np.float64, copy=True)
    # G^T x: inverse of the down-sweep, E then C then K at every level, levels 0 .. L-1
    for lv in F.levels:
        for c in lv.cells:                 # z_I <- L^T z_I + W z_B  (undoes z_I <- L^-T (z_I - W z_B))
            z[c.I] = c.L.T @ z[c.I] + (c.W @ z[c.B] if len(c.B) else 0.0)
        for g in lv.groups:                # z_g <- L_g^T z_g
            z[g.idx] = g.L.T @ z[g.idx]
        for sk in lv.skels:                # z_h += T z_t ; z_t <- L~^T z_t + W~ z_h
            if len(sk.tilde) == 0:
                continue
            if len(sk.hat):
                z[sk.hat] += sk.T @ z[sk.tilde]
            z[sk.tilde] = sk.Lt.T @ z[sk.tilde] + (sk.Wt @ z[sk.hat] if len(sk.hat) else 0.0)
    if len(F.root_idx):                    # B_L^T undoes the backward root solve
        z[F.root_idx] = F.root_L.T @ z[F.root_idx]
    # G y: the forward root solve, then the up-sweep undone from level L-1 down to 0
    if len(F.root_idx):
        z[F.root_idx] = F.root_L @ z[F.root_idx]
    for lv in reversed(F.levels):
        for sk in lv.skels:                # z_h += W~^T z_t ; z_t <- L~ z_t + T^T z_h
            if len(sk.tilde) == 0:
                continue
            if len(sk.hat):
                z[sk.hat] += sk.Wt.T @ z[sk.tilde]
            z[sk.tilde] = sk.Lt @ z[sk.tilde] + sk.T.T @ z[sk.hat]
        for g in lv.groups:                # z_g <- L_g z_g
            z[g.idx] = g.L @ z[g.idx]
        for c in lv.cells:                 # z_B += W^T z_I ; z_I <- L z_I
            if len(c.B):
                z[c.B] += c.W.T @ z[c.I]
            z[c.I] = c.L @ z[c.I]
    return z


def _power_norm(op, n: int, seed: int = 0, rtol: float = 1e-2, maxit: int = 50) -> float:
    """||M||_2 of a symmetric operator M = op by power iteration on M^2 (so the dominant
    eigenvalue in magnitude is found even when M is indefinite): Gaussian start (seed),
    stop when the estimate changes by less than rtol (relative), at most maxit products."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(n)
    v /= np.linalg.norm(v)
    est = 0.0
    for _ in range(maxit):
        w = op(op(v))
        nw = float(np.linalg.norm(w))
        new = np.sqrt(nw)
        if nw == 0.0:
            return 0.0
        v = w / nw
        if est > 0.0 and abs(new - est) <= rtol * new:
            return new
        est = new
    return est


def estimate_ea(A: sp.csr_matrix, F: Factorization, seed: int = 0, rtol: float = 1e-2, maxit: int = 50) -> float:
    """e_a = ||A - F||_2 / ||A||_2 (Sec. 4), both norms by power iteration."""
    na = _power_norm(lambda x: A @ x, A.shape[0], seed, rtol, maxit)
    nd = _power_norm(lambda x: A @ x - apply_forward(F, x), A.shape[0], seed, rtol, maxit)
    return nd / na if na > 0 else 0.0


def estimate_es(A: sp.csr_matrix, F: Factorization, seed: int = 0, rtol: float = 1e-2, maxit: int = 50) -> float:
    """e_s = ||I - G^-1 A G^-T||_2 (Sec. 4) by power iteration on the symmetric operator."""
    return _power_norm(lambda x: x - apply_ginv(F, A @ apply_ginv_t(F, x)), A.shape[0], seed, rtol, maxit)


# ----------------------------------------------------------------------------------------
# Preconditioned CG (Sec. 4: CG with F^-1 to relative residual 1e-12)
# ----------------------------------------------------------------------------------------

@dataclass
class PCGResult:
    u: np.ndarray
    iters: int
    relres: float           # recursively updated residual ||r_k|| / ||f||
    true_relres: float      # ||f - A u|| / ||f||
    converged: bool
    history: List[float]


def pcg(A: sp.csr_matrix, f: np.ndarray, precond=None, rtol: float = 1e-12, maxit: int = 500) -> PCGResult:
    """Textbook preconditioned CG from u_0 = 0. iters counts the products A p taken when
    ||r_k||/||f|| <= rtol first holds (on the recursively updated residual)."""
    f = np.asarray(f, dtype=np.float64)
    nf = float(np.linalg.norm(f))
    u = np.zeros_like(f)
    if nf == 0.0:
        return PCGResult(u, 0, 0.0, 0.0, True, [0.0])
    Minv = precond if precond is not None else (lambda v: v.copy())
    r = f.copy()
    z = Minv(r)
    p = z.copy()
    rho = float(r @ z)
    hist = [1.0]
    it = 0
    converged = False
    while it < maxit:
        q = A @ p
        alpha = rho / float(p @ q)
        u += alpha * p
        r -= alpha * q
        it += 1
        rel = float(np.linalg.norm(r)) / nf
        hist.append(rel)
        if rel <= rtol:
            converged = True
            break
        z = Minv(r)
        rho_new = float(r @ z)
        beta = rho_new / rho
        p = z + beta * p
        rho = rho_new
    true_rel = float(np.linalg.norm(f - A @ u)) / nf
    return PCGResult(u, it, hist[-1], true_rel, converged, hist)


def grad_log_a(d: int, s: int, a_cells: np.ndarray, u: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """Gradient with respect to theta = log a of a loss L(u) of the solution of A u = f,
    given the adjoint solution lam = A^-1 dL/du (A is symmetric):
        dL/dtheta_c = -a_c * lam^T (dA/da_c) u.
    With the cell-wise form of the operator (eq. (1.1) with reading R2, the bilinear version
    of fd_energy), lam^T (dA/da_c) u is 2^(1-d) / h^2 times the sum, over the grid edges
    (p, p + e_k) of cell c, of (lam(p + e_k) - lam(p)) * (u(p + e_k) - u(p)), with the values
    at the Dirichlet ghosts 0. Cell c = (c_1..c_d), c_k in 0..s, has the grid points with
    x_k in {c_k, c_k + 1} as corners. Plain loops over cells and edges."""
    h = 1.0 / (s + 1)
    a_cells = np.asarray(a_cells, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64).ravel()
    lam = np.asarray(lam, dtype=np.float64).ravel()

    def val(v, x):
        if any(xk < 1 or xk > s for xk in x):
            return 0.0
        return v[sum((xk - 1) * s ** k for k, xk in enumerate(x))]

    a_flat = a_cells.ravel()   # indexed [c_d, ..., c_1]: c_1 fastest
    g = np.zeros((s + 1) ** d)
    for c in range((s + 1) ** d):
        cc = [(c // (s + 1) ** k) % (s + 1) for k in range(d)]
        acc = 0.0
        for k in range(d):
            others = [j for j in range(d) if j != k]
            for shifts in product((0, 1), repeat=d - 1):
                p = list(cc)
                for j, sh in zip(others, shifts):
                    p[j] = cc[j] + sh
                q = list(p)
                q[k] += 1
                acc += (val(lam, q) - val(lam, p)) * (val(u, q) - val(u, p))
        g[c] = -a_flat[c] * acc * 2.0 ** (1 - d) / (h * h)
    return g.reshape(a_cells.shape)


def dense_solve(A: sp.csr_matrix, f: np.ndarray) -> np.ndarray:
    """Brute force: dense Cholesky solve (small problems only)."""
    Ad = A.toarray()
    Lc = np.linalg.cholesky(Ad)
    y = sla.solve_triangular(Lc, f, lower=True)
    return sla.solve_triangular(Lc.T, y, lower=False)
