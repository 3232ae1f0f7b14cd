"""Seeded synthetic bipartite graphs (int32 CSC) for tests and benchmarks.

Holds no matching arithmetic.  The large generators are C (``libmcmgen.so``,
built from ``csrc/graphgen.c``); the tiny closed-form families are plain
numpy.  Every graph is returned as a :class:`Graph` with ``colptr`` and
``rowind`` numpy int32 arrays, rows of each column sorted ascending and
without duplicates.

The workload recipes mirror the sparse-matrix classes of the paper's
experiments (section 4: mesh/road-like and Kronecker/social-like matrices
and their random row/column permutations); the matrices themselves are not
used.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmcmgen.so")


class _GG(ctypes.Structure):
    _fields_ = [
        ("nc", ctypes.c_int32),
        ("nr", ctypes.c_int32),
        ("nnz", ctypes.c_int64),
        ("colptr", ctypes.POINTER(ctypes.c_int32)),
        ("rowind", ctypes.POINTER(ctypes.c_int32)),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is missing: run __graft_entry__.build() first")
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER
        lib.gg_uniform.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int,
                                   ctypes.c_uint64, P(_GG)]
        lib.gg_grid5.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
                                 P(_GG), ctypes.c_void_p, ctypes.c_void_p]
        lib.gg_rmat.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_int32, ctypes.c_int, ctypes.c_uint64, P(_GG)]
        lib.gg_batch_member.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                        P(_GG)]
        lib.gg_transpose.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p]
        lib.gg_fnv1a.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
        lib.gg_fnv1a.restype = ctypes.c_uint64
        lib.gg_seed_mix.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.gg_seed_mix.restype = ctypes.c_uint64
        lib.gg_request_trace.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_double, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_int32, ctypes.c_int32] + [ctypes.c_void_p] * 5
        lib.gg_permute.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                   P(_GG)]
        lib.gg_free.argtypes = [P(_GG)]
        for f in ("gg_uniform", "gg_grid5", "gg_rmat", "gg_batch_member", "gg_transpose", "gg_request_trace",
                  "gg_permute"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclass
class Graph:
    """A bipartite graph in CSC: column c holds rows rowind[colptr[c]:colptr[c+1]]."""
    nc: int
    nr: int
    colptr: np.ndarray
    rowind: np.ndarray
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.colptr[-1]) if len(self.colptr) else 0

    def fnv1a(self) -> int:
        lib = _load()
        cp = np.ascontiguousarray(self.colptr, dtype=np.int32)
        ri = np.ascontiguousarray(self.rowind, dtype=np.int32)
        if ri.size == 0:
            ri = np.zeros(1, np.int32)
        return int(lib.gg_fnv1a(self.nc, cp.ctypes.data, ri.ctypes.data))

    def csr(self):
        """(rowptr[nr+1], colind[nnz]) of the same pattern, columns ascending per row."""
        lib = _load()
        rp = np.zeros(self.nr + 1, np.int32)
        ci = np.zeros(max(self.nnz, 1), np.int32)
        cp = np.ascontiguousarray(self.colptr, dtype=np.int32)
        ri = np.ascontiguousarray(self.rowind, dtype=np.int32)
        if ri.size == 0:
            ri = np.zeros(1, np.int32)
        rc = lib.gg_transpose(self.nc, self.nr, cp.ctypes.data, ri.ctypes.data, rp.ctypes.data, ci.ctypes.data)
        if rc != 0:
            raise MemoryError("gg_transpose failed")
        return rp, ci[: self.nnz]

    def edges(self):
        """(col, row) pairs as two int64 arrays."""
        cols = np.repeat(np.arange(self.nc, dtype=np.int64), np.diff(self.colptr).astype(np.int64))
        return cols, self.rowind.astype(np.int64)


def _take(g: _GG, name: str) -> Graph:
    lib = _load()
    nc, nr, nnz = g.nc, g.nr, g.nnz
    cp = np.ctypeslib.as_array(g.colptr, shape=(nc + 1,)).copy()
    ri = np.ctypeslib.as_array(g.rowind, shape=(max(nnz, 1),))[:nnz].copy() if nnz > 0 else np.zeros(0, np.int32)
    lib.gg_free(ctypes.byref(g))
    return Graph(nc, nr, cp.astype(np.int32, copy=False), ri.astype(np.int32, copy=False), name)


def _check(rc: int, what: str):
    if rc == -2:
        raise MemoryError(f"{what}: allocation failed")
    if rc != 0:
        raise ValueError(f"{what}: bad arguments (rc={rc})")


def seed_mix(a: int, b: int) -> int:
    return int(_load().gg_seed_mix(a, b))


# ---------------------------------------------------------------- generators
def uniform(nc: int, nr: int, deg: int, seed: int, replace: bool = True) -> Graph:
    """Every column draws `deg` rows uniformly (with replacement, deduplicated,
    unless replace=False, which draws min(deg, nr) distinct rows)."""
    g = _GG()
    _check(_load().gg_uniform(nc, nr, deg, 1 if replace else 0, seed, ctypes.byref(g)), "uniform")
    return _take(g, f"uniform_{nc}x{nr}_d{deg}_s{seed}")


def grid5(k: int, ndel_cols: int, ndel_rows: int, seed: int, return_masks: bool = False):
    """5-point stencil pattern on a k x k grid with deleted columns and rows."""
    g = _GG()
    n = k * k
    dc = np.zeros(max(n, 1), np.uint8)
    dr = np.zeros(max(n, 1), np.uint8)
    _check(_load().gg_grid5(k, ndel_cols, ndel_rows, seed, ctypes.byref(g), dc.ctypes.data, dr.ctypes.data),
           "grid5")
    out = _take(g, f"grid5_{k}_dc{ndel_cols}_dr{ndel_rows}_s{seed}")
    if return_masks:
        return out, dc[:n].astype(bool), dr[:n].astype(bool)
    return out


def rmat(scale: int, nsamples: int, seed: int, a=0.57, b=0.19, c=0.19, n_limit: int = 0,
         permute: bool = False) -> Graph:
    """R-MAT pattern, duplicates removed, optional random row/column permutation."""
    g = _GG()
    _check(_load().gg_rmat(scale, nsamples, a, b, c, n_limit, 1 if permute else 0, seed, ctypes.byref(g)), "rmat")
    return _take(g, f"rmat_s{scale}_m{nsamples}_seed{seed}{'_perm' if permute else ''}")


def permute(g: Graph, seed: int) -> Graph:
    """Random row and column permutation of g (the RCP transform; rows
    sorted within columns).  |M| is invariant; the BFS structure is not."""
    out = _GG()
    cp = np.ascontiguousarray(g.colptr, dtype=np.int32)
    ri = np.ascontiguousarray(g.rowind, dtype=np.int32)
    if ri.size == 0:
        ri = np.zeros(1, np.int32)
    _check(_load().gg_permute(g.nc, g.nr, cp.ctypes.data, ri.ctypes.data, ctypes.c_uint64(seed), ctypes.byref(out)),
           "permute")
    return _take(out, f"{g.name}_rcp{seed}")


def batch_member(seed: int, gidx: int, lo: int = 64, hi: int = 65536, dmin: int = 2, dmax: int = 12,
                 halfband: int = 5, empty_frac: float = 0.02) -> Graph:
    """Graph `gidx` of an uneven batch (even: uniform rows, odd: banded)."""
    g = _GG()
    _check(_load().gg_batch_member(seed, gidx, lo, hi, dmin, dmax, halfband, empty_frac, ctypes.byref(g)),
           "batch_member")
    return _take(g, f"batch_s{seed}_g{gidx}")


def request_trace(seed: int, count: int, lam: float = 2000.0, lo: int = 1000, hi: int = 1000000,
                  dmin: int = 4, dmax: int = 16):
    """Arrival gaps (s), sizes, degrees, kinds (0 uniform, 1 R-MAT) and seeds of a request stream."""
    gap = np.zeros(count, np.float64)
    n = np.zeros(count, np.int32)
    deg = np.zeros(count, np.int32)
    kind = np.zeros(count, np.int32)
    rseed = np.zeros(count, np.uint64)
    _check(_load().gg_request_trace(seed, count, lam, lo, hi, dmin, dmax, gap.ctypes.data, n.ctypes.data,
                                    deg.ctypes.data, kind.ctypes.data, rseed.ctypes.data), "request_trace")
    return gap, n, deg, kind, rseed


def request_graph(n: int, deg: int, kind: int, rseed: int) -> Graph:
    """One serving request: uniform (deg distinct rows per column) or R-MAT
    (scale ceil(log2 n), deg*n samples, ids >= n rejected)."""
    if kind == 0:
        return uniform(n, n, deg, int(rseed), replace=False)
    scale = max(1, math.ceil(math.log2(n)))
    return rmat(scale, deg * n, int(rseed), n_limit=n)


# ------------------------------------------------- the named workloads
def workload(name: str) -> Graph:
    """The named single-graph workloads.

    uniform2000 : 2000 x 2000, each column draws 4 rows uniformly (seed 1).
    grid2048    : 5-point grid, 2048 x 2048, 3 % of columns and 3 % of rows
                  emptied (seed 2).
    rmat23      : R-MAT scale 23, 16 * 2^23 samples, (.57,.19,.19,.05),
                  duplicates removed, random row/column permutation (seed 3).
    grid2048p   : grid2048 under a random row and column permutation (seed 7),
                  the paper's RCP transform.
    Reduced-size variants for tests: grid<k>, grid<k>p, rmat<scale>.
    """
    if name == "uniform2000":
        return uniform(2000, 2000, 4, 1)
    if name.startswith("grid"):
        perm = name.endswith("p")
        k = int(name[4:-1] if perm else name[4:])
        nd = int(math.floor(0.03 * k * k))
        g = grid5(k, nd, nd, 2)
        return permute(g, 7) if perm else g
    if name.startswith("rmat"):
        s = int(name[4:])
        return rmat(s, 16 * (1 << s), 3, permute=True)
    raise KeyError(name)


# ------------------------------------------------- tiny closed-form families
def from_edges(nc: int, nr: int, edges, name: str = "") -> Graph:
    """CSC from (col, row) pairs; duplicates removed, rows sorted per column."""
    e = sorted(set((int(c), int(r)) for c, r in edges))
    colptr = np.zeros(nc + 1, np.int32)
    for c, _ in e:
        colptr[c + 1] += 1
    colptr = np.cumsum(colptr).astype(np.int32)
    rowind = np.array([r for _, r in e], dtype=np.int32)
    return Graph(nc, nr, colptr, rowind, name)


def complete(m: int, n: int) -> Graph:
    """K_{m,n}: m columns, n rows, every pair adjacent."""
    return from_edges(m, n, [(c, r) for c in range(m) for r in range(n)], f"K{m},{n}")


def star(k: int) -> Graph:
    """K_{1,k}: one column adjacent to k rows."""
    return from_edges(1, k, [(0, r) for r in range(k)], f"star{k}")


def path(k: int) -> Graph:
    """Path on k vertices alternating column, row, column, ... (c0-r0-c1-r1-...)."""
    nc = (k + 1) // 2
    nr = k // 2
    edges = []
    for v in range(k - 1):
        if v % 2 == 0:
            edges.append((v // 2, v // 2))          # c_{v/2} - r_{v/2}
        else:
            edges.append(((v + 1) // 2, v // 2))    # r_{(v-1)/2} - c_{(v+1)/2}
    return from_edges(nc, nr, edges, f"path{k}")


def permutation_plus_noise(n: int, extra: int, seed: int) -> Graph:
    """A random permutation pattern (one entry per column and row) plus
    `extra` uniformly random extra entries per column."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    edges = [(c, int(perm[c])) for c in range(n)]
    for c in range(n):
        for r in rng.integers(0, n, size=extra):
            edges.append((c, int(r)))
    return from_edges(n, n, edges, f"permnoise{n}_{extra}_s{seed}")


def disjoint_union(a: Graph, b: Graph) -> Graph:
    """Block-diagonal union: b's columns and rows are shifted past a's."""
    cp = np.concatenate([a.colptr, b.colptr[1:] + a.nnz]).astype(np.int32)
    ri = np.concatenate([a.rowind, b.rowind + a.nr]).astype(np.int32)
    return Graph(a.nc + b.nc, a.nr + b.nr, cp, ri, f"({a.name})+({b.name})")


def random_small(nc: int, nr: int, p: float, seed: int) -> Graph:
    """Erdos-Renyi bipartite pattern: each (c, r) present with probability p."""
    rng = np.random.default_rng(seed)
    m = rng.random((nc, nr)) < p
    return from_edges(nc, nr, [(c, r) for c in range(nc) for r in range(nr) if m[c, r]], f"er{nc}x{nr}_p{p}_s{seed}")


def empty(nc: int, nr: int) -> Graph:
    return Graph(nc, nr, np.zeros(nc + 1, np.int32), np.zeros(0, np.int32), f"empty{nc}x{nr}")
