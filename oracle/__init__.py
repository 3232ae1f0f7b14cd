"""CPU reference ("oracle") for maximum-cardinality bipartite matching.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check in
``__graft_entry__.py`` and by the CPU-baseline leg of ``bench.py``; never by
the matching library.  It shares no code with the GPU path: the arithmetic
is in ``hk_oracle.c`` (plain C, single thread), this module only marshals
numpy arrays.

What it computes (paper, section 2 and section 3):
  * cheap_init      -- the greedy initial matching every run starts from
                       (section 4, experimental setup);
  * check_csc       -- the input is well formed (step 0 of every run);
  * hopcroft_karp   -- maximum matching from a given matching (section 2);
    hopcroft_karp_ex and hopcroft_karp_sample run it phase-bounded and
    count the adjacency entries read (the CPU baseline);
  * konig_cover     -- a vertex cover of size |M| from the final alternating
                       BFS (Berge / Konig: certifies maximality);
  * verify_cover    -- an independent weak-duality certificate check;
  * brute_force*    -- exhaustive maximum for tiny graphs;
  * alt_bfs_levels  -- the level sets of the alternating BFS from all
                       unmatched columns (what one BFS pass of the paper's
                       Algorithm 2 computes level by level).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hk_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build() -> str:
    """Compile hk_oracle.c into liboracle.so (plain gcc, portable -O3)."""
    cmd = ["gcc", "-O3", "-fPIC", "-shared", "-std=c11", "-Wall", "-Wextra", "-o", _LIB + ".tmp", _SRC]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        vp, i32 = ctypes.c_void_p, ctypes.c_int32
        lib.orc_check_csc.argtypes = [i32, i32, vp, vp]
        lib.orc_check_csc.restype = ctypes.c_int
        lib.orc_check_matching.argtypes = [i32, i32, vp, vp, vp, vp, vp]
        lib.orc_check_matching.restype = ctypes.c_int
        lib.orc_cheap_init.argtypes = [i32, i32, vp, vp, vp, vp]
        lib.orc_cheap_init.restype = None
        lib.orc_hopcroft_karp.argtypes = [i32, i32, vp, vp, vp, vp, vp]
        lib.orc_hopcroft_karp.restype = ctypes.c_int64
        lib.orc_hopcroft_karp_ex.argtypes = [i32, i32, vp, vp, vp, vp, ctypes.c_int64, vp, vp]
        lib.orc_hopcroft_karp_ex.restype = ctypes.c_int64
        lib.orc_konig_cover.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp]
        lib.orc_konig_cover.restype = ctypes.c_int64
        lib.orc_verify_cover.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp]
        lib.orc_verify_cover.restype = ctypes.c_int
        lib.orc_brute_force.argtypes = [i32, i32, vp, vp]
        lib.orc_brute_force.restype = ctypes.c_int64
        lib.orc_brute_force_subsets.argtypes = [i32, i32, vp, vp]
        lib.orc_brute_force_subsets.restype = ctypes.c_int64
        lib.orc_alt_bfs_levels.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp]
        lib.orc_alt_bfs_levels.restype = ctypes.c_int64
        _lib = lib
    return _lib


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a if a.size else np.zeros(1, np.int32)


def _g(g):
    return g.nc, g.nr, _i32(g.colptr), _i32(g.rowind)


def check_csc(g) -> bool:
    nc, nr, cp, ri = _g(g)
    return _load().orc_check_csc(nc, nr, cp.ctypes.data, ri.ctypes.data) == 0


def check_matching(g, cmatch, rmatch):
    """Return |M| if (cmatch, rmatch) is a matching of g, else None."""
    nc, nr, cp, ri = _g(g)
    cm, rm = _i32(cmatch), _i32(rmatch)
    card = ctypes.c_int64(0)
    rc = _load().orc_check_matching(nc, nr, cp.ctypes.data, ri.ctypes.data, cm.ctypes.data, rm.ctypes.data,
                                    ctypes.addressof(card))
    return int(card.value) if rc == 0 else None


def cheap_init(g):
    """Greedy initial matching (columns in order, first free row in stored order)."""
    nc, nr, cp, ri = _g(g)
    cm = np.empty(max(nc, 1), np.int32)
    rm = np.empty(max(nr, 1), np.int32)
    _load().orc_cheap_init(nc, nr, cp.ctypes.data, ri.ctypes.data, cm.ctypes.data, rm.ctypes.data)
    return cm[:nc].copy(), rm[:nr].copy()


def hopcroft_karp(g, cmatch=None, rmatch=None, timed: bool = False):
    """Maximum matching from (cmatch, rmatch) (empty if None).

    Returns (card, cmatch, rmatch, phases[, seconds]) where seconds covers
    the Hopcroft-Karp phases only (not the copy of the initial matching)."""
    nc, nr, cp, ri = _g(g)
    cm = np.full(max(nc, 1), -1, np.int32)
    rm = np.full(max(nr, 1), -1, np.int32)
    if cmatch is not None:
        cm[:nc] = cmatch
        rm[:nr] = rmatch
    ph = ctypes.c_int64(0)
    t0 = time.perf_counter()
    card = _load().orc_hopcroft_karp(nc, nr, cp.ctypes.data, ri.ctypes.data, cm.ctypes.data, rm.ctypes.data,
                                     ctypes.addressof(ph))
    dt = time.perf_counter() - t0
    if card < 0:
        raise MemoryError("orc_hopcroft_karp failed")
    out = (int(card), cm[:nc].copy(), rm[:nr].copy(), int(ph.value))
    return out + (dt,) if timed else out


def hopcroft_karp_ex(g, cmatch, rmatch, max_phases: int | None = None):
    """Hopcroft-Karp from (cmatch, rmatch), at most `max_phases` augmenting
    phases (None: until maximum).  Returns (card, cmatch, rmatch, phases,
    edges_scanned), edges_scanned counting the adjacency entries read by the
    BFS and DFS steps of every phase run, including the last BFS."""
    nc, nr, cp, ri = _g(g)
    cm = np.full(max(nc, 1), -1, np.int32)
    rm = np.full(max(nr, 1), -1, np.int32)
    cm[:nc] = cmatch
    rm[:nr] = rmatch
    ph = ctypes.c_int64(0)
    ed = ctypes.c_int64(0)
    lim = (1 << 63) - 1 if max_phases is None else int(max_phases)
    card = _load().orc_hopcroft_karp_ex(nc, nr, cp.ctypes.data, ri.ctypes.data, cm.ctypes.data, rm.ctypes.data, lim,
                                        ctypes.addressof(ph), ctypes.addressof(ed))
    if card < 0:
        raise MemoryError("orc_hopcroft_karp_ex failed")
    return int(card), cm[:nc].copy(), rm[:nr].copy(), int(ph.value), int(ed.value)


def hopcroft_karp_sample(g, cmatch, rmatch, budget_s: float = 15.0):
    """Bounded CPU sample: Hopcroft-Karp phases, one call per phase, from
    (cmatch, rmatch) until `budget_s` seconds of phase time have been spent
    or the matching is maximum.  Returns dict(seconds, phases, edges, card,
    done).  Single thread."""
    nc, nr, cp, ri = _g(g)
    cm = np.full(max(nc, 1), -1, np.int32)
    rm = np.full(max(nr, 1), -1, np.int32)
    cm[:nc] = cmatch
    rm[:nr] = rmatch
    lib = _load()
    total_t, total_e, total_p, done, card = 0.0, 0, 0, False, int((cm[:nc] >= 0).sum())
    while total_t < budget_s:
        ph = ctypes.c_int64(0)
        ed = ctypes.c_int64(0)
        t0 = time.perf_counter()
        card = lib.orc_hopcroft_karp_ex(nc, nr, cp.ctypes.data, ri.ctypes.data, cm.ctypes.data, rm.ctypes.data, 1,
                                        ctypes.addressof(ph), ctypes.addressof(ed))
        total_t += time.perf_counter() - t0
        total_e += int(ed.value)
        if ph.value == 0:
            done = True
            break
        total_p += int(ph.value)
    return {"seconds": total_t, "phases": total_p, "edges": total_e, "card": int(card), "done": done}


def konig_cover(g, cmatch, rmatch):
    """(|K|, col_in_cover, row_in_cover); |K| = -3 if the matching is not maximum."""
    nc, nr, cp, ri = _g(g)
    cm, rm = _i32(cmatch), _i32(rmatch)
    cc = np.zeros(max(nc, 1), np.uint8)
    rc = np.zeros(max(nr, 1), np.uint8)
    k = _load().orc_konig_cover(nc, nr, cp.ctypes.data, ri.ctypes.data, cm.ctypes.data, rm.ctypes.data,
                                cc.ctypes.data, rc.ctypes.data)
    return int(k), cc[:nc].copy(), rc[:nr].copy()


def verify_cover(g, cmatch, rmatch, col_in_cover, row_in_cover) -> int:
    """0 if (M, K) certifies a maximum matching; 1: not a matching,
    2: an edge is uncovered, 3: |K| != |M|."""
    nc, nr, cp, ri = _g(g)
    cm, rm = _i32(cmatch), _i32(rmatch)
    cc = np.ascontiguousarray(col_in_cover, dtype=np.uint8)
    rc = np.ascontiguousarray(row_in_cover, dtype=np.uint8)
    cc = cc if cc.size else np.zeros(1, np.uint8)
    rc = rc if rc.size else np.zeros(1, np.uint8)
    return int(_load().orc_verify_cover(nc, nr, cp.ctypes.data, ri.ctypes.data, cm.ctypes.data, rm.ctypes.data,
                                        cc.ctypes.data, rc.ctypes.data))


def brute_force(g) -> int:
    """Maximum matching size by a DP over used-row subsets (nr <= 20)."""
    nc, nr, cp, ri = _g(g)
    v = _load().orc_brute_force(nc, nr, cp.ctypes.data, ri.ctypes.data)
    if v < 0:
        raise ValueError("brute_force: graph too large")
    return int(v)


def brute_force_subsets(g) -> int:
    """Maximum matching size by enumerating every edge subset (nnz <= 24)."""
    nc, nr, cp, ri = _g(g)
    v = _load().orc_brute_force_subsets(nc, nr, cp.ctypes.data, ri.ctypes.data)
    if v < 0:
        raise ValueError("brute_force_subsets: graph too large")
    return int(v)


def alt_bfs_levels(g, cmatch, rmatch):
    """(clevel[nc], rlevel[nr], free_rows_reached) of the alternating BFS
    from all unmatched columns, without early stop."""
    nc, nr, cp, ri = _g(g)
    cm, rm = _i32(cmatch), _i32(rmatch)
    cl = np.zeros(max(nc, 1), np.int32)
    rl = np.zeros(max(nr, 1), np.int32)
    f = _load().orc_alt_bfs_levels(nc, nr, cp.ctypes.data, ri.ctypes.data, cm.ctypes.data, rm.ctypes.data,
                                   cl.ctypes.data, rl.ctypes.data)
    return cl[:nc].copy(), rl[:nr].copy(), int(f)


def solve(g, init: str = "cheap"):
    """Convenience: greedy init (or empty) then Hopcroft-Karp; returns dict."""
    if init == "cheap":
        cm0, rm0 = cheap_init(g)
    else:
        cm0 = np.full(g.nc, -1, np.int32)
        rm0 = np.full(g.nr, -1, np.int32)
    card, cm, rm, ph, dt = hopcroft_karp(g, cm0, rm0, timed=True)
    return {"card": card, "cmatch": cm, "rmatch": rm, "phases": ph, "seconds": dt,
            "init_card": int((cm0 >= 0).sum())}
