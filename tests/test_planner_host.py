"""Host-side checks of the library: it loads, exports every declared entry point, and its
level planner (integers only, run without a GPU) reproduces the oracle's grouping of the
unknowns level by level when given the oracle's ID choices."""
import re
import os

import numpy as np
import pytest

import oracle as O
from paper_1808_01364_amd import rhif
from workloads import make_problem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    return sorted(set(re.findall(r"\b(rhif_[a-z_]+)\s*\(", text)) - {"rhif_id_choice_fn", "rhif_cell_fn"})


def test_library_exports_every_declared_symbol():
    lib = rhif.load_library()
    names = _declared("rhif.h") + _declared("rhif_plan.h")
    assert "rhif_factor" in names and "rhif_apply" in names and "rhif_pcg_solve" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(rhif.EXPORTED) <= set(names)
    assert "gfx950" in rhif.version()


def test_factor_batch_rejects_bad_calls_before_device_work():
    """rhif_factor_batch checks its arguments before touching the device (the CSR pointers
    here are never dereferenced): no problem, timing flags with several problems, grids of
    different dimension; every out[i] is NULL afterwards."""
    import ctypes
    lib = rhif.load_library()
    o = rhif.Opts()
    o.leaf, o.eps, o.precond, o.precision, o.flags = 8, 1e-3, 1, 0, 0
    grids = (rhif.Grid * 2)(rhif.make_grid(2, 16), rhif.make_grid(2, 24))
    fake = (ctypes.c_void_p * 2)(16, 16)
    out = (ctypes.c_void_p * 2)(1, 1)
    assert lib.rhif_factor_batch(0, grids, ctypes.byref(o), fake, fake, fake, None, out) == rhif.RHIF_EINVAL
    assert "count" in lib.rhif_last_error().decode()
    o.flags = rhif.FLAG_KERNEL_TIMES
    assert lib.rhif_factor_batch(2, grids, ctypes.byref(o), fake, fake, fake, None, out) == rhif.RHIF_EINVAL
    assert "single" in lib.rhif_last_error().decode() and not out[0] and not out[1]
    o.flags = 0
    grids[1] = rhif.make_grid(3, 8)
    out[0] = out[1] = 1
    assert lib.rhif_factor_batch(2, grids, ctypes.byref(o), fake, fake, fake, None, out) == rhif.RHIF_EINVAL
    assert "same dim" in lib.rhif_last_error().decode() and not out[0] and not out[1]


def test_fd_nnz_host():
    assert rhif.fd_nnz(2, 64) == 64 * 64 + 2 * 2 * 64 * 63
    assert rhif.fd_nnz(3, 5) == 125 + 2 * 3 * 25 * 4
    with pytest.raises(rhif.RhifError):
        rhif.fd_nnz(4, 3)


def _oracle_replay(d, s, leaf, eps, kind="two_valued", seed=0, **kw):
    P = make_problem(kind, d, s, seed, leaf, eps, **kw)
    A = O.assemble_fd(d, s, P.a_cells, P.b)
    F = O.factor(A, d, s, leaf, eps, 1)
    choices = {}
    for lv in F.levels:
        for sk in lv.skels:
            choices[(lv.level, int(sk.group[0]))] = (len(sk.hat), list(sk.perm), len(sk.group))
    cells = {}
    for lv in F.levels:
        for c in lv.cells:
            cells[(lv.level, int(c.I[0]))] = (sorted(c.I.tolist()), sorted(c.B.tolist()))
    cells[(F.L, int(F.root_idx[0]))] = (sorted(F.root_idx.tolist()), [])
    return F, choices, cells


@pytest.mark.parametrize("d,s,leaf", [(2, 16, 4), (2, 13, 4), (2, 33, 8), (2, 64, 8), (2, 40, 6),
                                      (3, 7, 2), (3, 10, 4), (3, 9, 2)])
def test_planner_matches_oracle_grouping(d, s, leaf):
    """Given the oracle's ranks and pivots, the planner's cells at every level have the
    oracle's interior and boundary sets, and the same root size."""
    F, choices, cells = _oracle_replay(d, s, leaf, 1e-3)
    used = set()

    def choose(level, first, size):
        k, perm, n = choices[(level, first)]
        assert n == size
        used.add((level, first))
        return k, perm

    seen = {}

    def on_cell(level, cell, interior, boundary):
        seen[(level, interior[0])] = (sorted(interior), sorted(boundary))

    root = rhif.plan_dry_run(d, s, leaf, choose, on_cell)
    assert root == F.root_size
    assert used == set(choices)
    assert set(seen) == set(cells)
    for key in cells:
        assert seen[key] == cells[key], key


@pytest.mark.parametrize("d,s,leaf", [(2, 1, 2), (2, 2, 2), (2, 5, 8), (2, 8, 8), (2, 15, 8), (2, 17, 4),
                                      (2, 192, 16), (3, 3, 2), (3, 4, 4), (3, 11, 3), (3, 16, 4)])
@pytest.mark.parametrize("mode", ["random", "none", "all"])
def test_planner_tables_in_bounds(d, s, leaf, mode):
    """Every device table passes the bounds validator for arbitrary (random, all-redundant,
    all-skeleton) ID choices, including ragged sides and trees without levels."""
    rng = np.random.default_rng(s * 7 + leaf)

    def choose(level, first, size):
        perm = rng.permutation(size)
        k = {"random": int(rng.integers(0, size + 1)), "none": 0, "all": size}[mode]
        return k, perm

    root = rhif.plan_dry_run(d, s, leaf, choose)
    assert 0 <= root <= s ** d


def test_planner_rejects_bad_choice():
    with pytest.raises(rhif.RhifError):
        rhif.plan_dry_run(2, 16, 4, lambda lvl, first, n: (n + 1, list(range(n))))
    with pytest.raises(rhif.RhifError):
        rhif.plan_dry_run(2, 16, 4, lambda lvl, first, n: (0, [0] * n) if n > 1 else (0, [0]))
