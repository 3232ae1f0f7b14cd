"""The oracle's pins catch plausible mistakes.

Each case copies hk_oracle.c, plants one mistake (a wrong index, a dropped
term, a flipped test), compiles the copy into a temporary library and runs
the same pins the real oracle passes (exhaustive search, closed forms,
Konig certificate).  At least one must fail.  Everything runs on the CPU.
"""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle as O
from paper_1303_1379_amd import graphgen as gg

SRC = os.path.join(os.path.dirname(O.__file__), "hk_oracle.c")

MUTANTS = {
    # greedy takes a row that is already matched
    "cheap_init_wrong_test": ("if (rmatch[r] == -1) {\n                cmatch[c] = r;",
                              "if (rmatch[r] != -2) {\n                cmatch[c] = r;"),
    # layered DFS descends on the wrong layer
    "dfs_wrong_layer": ("dist[m] == dist[u] + 1", "dist[m] == dist[u]"),
    # augmentation forgets to move to the previous mate
    "augment_drops_prev": ("        row = prev;\n", "\n"),
    # BFS forgets to record the distance of a newly reached column
    "bfs_no_distance": ("dist[m] = dist[c] + 1;", "dist[m] = dist[c];"),
    # augmenting-path length off by one
    "limit_off_by_one": ("limit = dist[c] + 1;", "limit = dist[c] + 2;"),
    # Konig cover takes the reached matched columns instead of the unreached
    "konig_transposed": ("(cmatch[c] != -1 && !zc[c])", "(cmatch[c] != -1 && zc[c])"),
    # verifier accepts an uncovered edge
    "verify_weak_cover": ("if (!col_in_cover[c] && !row_in_cover[rowind[j]]) return 2;",
                          "if (!col_in_cover[c] && !row_in_cover[rowind[j]] && 0) return 2;"),
    # brute force lets a column take a used row
    "brute_reuses_row": ("if (mask & bit) continue;", "(void)0;"),
    # input check: colptr need not start at 0
    "csc_no_start_check": ("if (colptr[0] != 0) return -1;", "(void)0;"),
    # input check: a decreasing colptr passes
    "csc_accepts_decrease": ("if (colptr[c + 1] < colptr[c]) return -1;", "(void)0;"),
    # input check: row index nr passes (off by one)
    "csc_row_bound_off_by_one": ("rowind[j] >= nr", "rowind[j] > nr"),
    # bounded run: the DFS reads are not counted
    "hk_edges_skip_dfs": ("                ++nedges;\n", "\n"),
    # bounded run: the phase bound is ignored
    "hk_phase_bound_ignored": ("if (nph >= max_phases) break;", "(void)0;"),
}

# (nc, nr, colptr, rowind, well formed)
CSC_CASES = [(3, 3, [0, 1, 2, 3], [0, 1, 2], True), (2, 2, [0, 2, 2], [1, 1], True),
             (3, 3, [1, 1, 2, 3], [0, 1, 2, 0], False), (3, 3, [0, 2, 1, 3], [0, 1, 2], False),
             (3, 3, [0, 1, 2, 3], [0, 1, 3], False), (3, 3, [0, 1, 2, 3], [0, -1, 2], False)]


class _Raw:
    def __init__(self, nc, nr, colptr, rowind):
        self.nc, self.nr = nc, nr
        self.colptr = np.asarray(colptr, np.int32)
        self.rowind = np.asarray(rowind, np.int32)


def _build_mutant(name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert old in src, f"mutation anchor for {name} not found"
    d = tempfile.mkdtemp(prefix="orcmut_")
    c = os.path.join(d, "m.c")
    so = os.path.join(d, "m.so")
    with open(c, "w") as f:
        f.write(src.replace(old, new, 1))
    subprocess.run(["gcc", "-O1", "-fPIC", "-shared", "-std=c11", "-w", "-o", so, c], check=True)
    return so


def _pins_hold(so):
    """The real oracle's pins, run against library `so`; False if any fails."""
    saved = O._lib
    O._lib = None
    real = O._LIB
    try:
        O._LIB = so
        O._load()
        cases = [gg.random_small(8, 9, 0.35, s) for s in range(25)]
        cases += [gg.complete(5, 7), gg.path(9), gg.permutation_plus_noise(200, 2, 1), gg.grid5(12, 5, 6, 3)]
        for g in cases:
            cm, rm = O.cheap_init(g)
            if O.check_matching(g, cm, rm) is None:
                return False
            card, cm, rm, _ = O.hopcroft_karp(g, cm, rm)
            if O.check_matching(g, cm, rm) != card:
                return False
            if g.nr <= 20 and card != O.brute_force(g):
                return False
            if g.nnz <= 24 and card != O.brute_force_subsets(g):
                return False
            k, cc, rc = O.konig_cover(g, cm, rm)
            if k != card or O.verify_cover(g, cm, rm, cc, rc) != 0:
                return False
            # verifier must reject an uncovered edge
            cols, rows = g.edges()
            idx = np.flatnonzero((cc[cols] == 0) & (rc[rows] == 1))
            if len(idx):
                rc2 = rc.copy()
                rc2[rows[idx[0]]] = 0
                if O.verify_cover(g, cm, rm, cc, rc2) != 2:
                    return False
        for m, n in [(3, 5), (6, 6)]:
            if O.hopcroft_karp(gg.complete(m, n))[0] != min(m, n):
                return False
        for nc, nr, cp, ri, ok in CSC_CASES:
            if O.check_csc(_Raw(nc, nr, cp, ri)) != ok:
                return False
        # the hand-worked two-phase instance of test_oracle (counts derived there)
        g = gg.from_edges(3, 3, [(0, 0), (1, 1), (2, 1), (2, 2)])
        cm0, rm0 = np.array([-1, -1, 1], np.int32), np.array([-1, 2, -1], np.int32)
        card, _, _, ph, ed = O.hopcroft_karp_ex(g, cm0, rm0, max_phases=1)
        if (card, ph, ed) != (2, 1, 6):
            return False
        card, _, _, ph, ed = O.hopcroft_karp_ex(g, cm0, rm0)
        if (card, ph, ed) != (3, 2, 12):
            return False
        return True
    finally:
        O._LIB = real
        O._lib = saved


def test_real_oracle_passes_the_mutant_pins():
    assert _pins_hold(O._LIB if os.path.exists(O._LIB) else O.build())


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    so = _build_mutant(name)
    assert not _pins_hold(so), f"planted mistake {name} was not detected"
