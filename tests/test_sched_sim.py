"""The correctness arguments of the GPU phase, checked on the CPU under
adversarial schedules (tests/sched_sim.py re-enacts the kernels' BFS,
Alternate and FixMatching with random, lock-step and sequential
interleavings of their memory accesses).

After every phase, whatever the schedule:
  I1  cmatch and rmatch describe a matching of the graph (symmetric, on edges);
  I2  a matched column stays matched;
  I3  |M| grows by exactly the number of BFS trees that reached an unmatched
      row (every such tree's root gets matched, and nothing else changes
      size) -- for the classic walk with its predecessor check and for the
      recorded-row walk that has none, with several ends per tree sharing
      their way to the root;
  I4  no row is left marked -2.
FixMatching runs over every row, only over the rows the walks report
(each row a walk writes, and the row a classic walk stops at), or only over
the rows claimed in the phase (the kernel's full scan gathers a row's column
only for those: I5 below).
Phases repeat until a BFS finds no end; the result then equals the
oracle's maximum.  A planted mistake in FixMatching must break I1 or I4."""
import random
import zlib

import numpy as np
import pytest

import oracle as O
from paper_1303_1379_amd import graphgen as gg
import sched_sim as S


def _graphs():
    out = []
    for s in range(6):
        out.append(gg.uniform(40, 40, 2, 900 + s))
        out.append(gg.uniform(60, 45, 3, 950 + s))
    out += [gg.grid5(8, 3, 3, 5), gg.grid5(10, 4, 2, 6), gg.workload("rmat8"), gg.workload("grid12p")]
    return out


def _valid(g, cm, rm):
    return O.check_matching(g, cm, rm)


def _run(g, init, rng, **kw):
    cm = np.full(g.nc, -1, np.int64)
    rm = np.full(g.nr, -1, np.int64)
    if init == "cheap":
        c0, r0 = O.cheap_init(g)
        cm[:], rm[:] = c0, r0
    phases = 0
    while True:
        before = cm >= 0
        card0 = int(before.sum())
        f, trees = S.phase(g.colptr, g.rowind, cm, rm, rng, **kw)
        phases += 1
        assert not (rm == -2).any(), "I4: a row is left marked"
        assert _valid(g, cm.astype(np.int32), rm.astype(np.int32)) is not None, "I1: not a matching"
        assert (cm[before] >= 0).all(), "I2: a matched column lost its row"
        assert int((cm >= 0).sum()) == card0 + trees, "I3: |M| did not grow by the trees with an end"
        if not f.ends:
            return int((cm >= 0).sum()), phases
        assert phases <= g.nc + 1


KW = [dict(walk=w, schedule=s, order=o, wr=wr, one_end=oe, local_p=lp, fix=fx)
      for w in ("recorded", "classic") for s in ("random", "lockstep", "sequential")
      for o, lp in (("levels", 0.0), ("levels", 0.5), ("lockstep", 0.0), ("pool", 0.0))
      for wr, oe in ((True, False), (True, True), (False, False))
      for fx in ("scan", "list", "reached")]


@pytest.mark.parametrize("kw", KW, ids=lambda d: "-".join(f"{k}={v}" for k, v in d.items()))
def test_phase_invariants_and_final_maximum(kw):
    rng = random.Random(zlib.crc32(repr(sorted(kw.items())).encode()))
    for i, g in enumerate(_graphs()):
        ref = O.hopcroft_karp(g, *O.cheap_init(g))[0]
        for init in ("empty", "cheap"):
            card, _ = _run(g, init, rng, **kw)
            assert card == ref, (i, g.name, init)


def test_several_ends_share_ways_to_the_root():
    """The interesting case for the recorded-row walk is present: trees
    with several ends whose walks meet before the root."""
    rng = random.Random(3)
    shared = 0
    for g in _graphs():
        c0, r0 = O.cheap_init(g)
        cm, rm = c0.astype(np.int64), r0.astype(np.int64)
        f = S.bfs_phase(g.colptr, g.rowind, cm, rm, rng, wr=True)
        # walk columns of each end; count columns visited by two walks
        seen = {}
        for e in f.ends:
            r = e
            while r != -1:
                c = int(f.pred[r])
                seen[c] = seen.get(c, 0) + 1
                r = int(f.prow[r])
        shared += sum(1 for v in seen.values() if v > 1)
    assert shared > 0


def test_planted_fix_mistake_is_caught():
    """FixMatching that skips the 'column points elsewhere' reset leaves a
    row matched to a column that took another row: I1 must fail on some
    schedule of the recorded-row walk."""
    real = S.fix_matching

    def broken(cmatch, rmatch, marked, rows=None):
        for r in range(len(rmatch)):
            if rmatch[r] < -1:
                rmatch[r] = -1

    S.fix_matching = broken
    try:
        caught = False
        rng = random.Random(5)
        for g in _graphs():
            for _ in range(3):
                try:
                    _run(g, "empty", rng, walk="recorded", schedule="random", wr=False)
                except AssertionError:
                    caught = True
                    break
            if caught:
                break
        assert caught
    finally:
        S.fix_matching = real


def test_listed_fix_needs_the_stop_rows():
    """With FixMatching over the reported rows only, a classic walk that does
    not report the row it stops at leaves that row pointing at a column
    that took another row: I1 must fail on some schedule."""
    real = S._walk_classic

    def no_stop_report(f, cmatch, rmatch, e, touched):
        sink = []
        for x in real(f, cmatch, rmatch, e, sink):
            yield x
        # report every row but a stop row: the last reported one if it was
        # not written by this walk (its column points elsewhere)
        for r in sink:
            if rmatch[r] >= 0 and cmatch[rmatch[r]] == r or r != sink[-1]:
                touched.append(r)

    S._walk_classic = no_stop_report
    try:
        caught = False
        rng = random.Random(9)
        for g in _graphs():
            for _ in range(4):
                try:
                    _run(g, "cheap", rng, walk="classic", schedule="random", wr=False, fix="list")
                except AssertionError:
                    caught = True
                    break
            if caught:
                break
        assert caught
    finally:
        S._walk_classic = real


@pytest.mark.parametrize("walk", ["recorded", "classic"])
@pytest.mark.parametrize("one_end", [False, True])
@pytest.mark.parametrize("order", ["levels", "pool"])
def test_rows_outside_the_forest_stay_consistent(walk, one_end, order):
    """I5: after Alternate, every row the phase's BFS did not claim is still
    unmatched or matched to a column that points back, under every schedule:
    a walk writes, stops at or leaves behind only claimed rows (the old mate
    of a flipped column is the walk's next row, whose claim brought that
    column into the tree).  So FixMatching may skip the other rows, and
    matching with it to the end gives the maximum."""
    rng = random.Random(zlib.crc32(f"{walk}{one_end}{order}".encode()))
    for i, g in enumerate(_graphs()):
        ref = O.hopcroft_karp(g, *O.cheap_init(g))[0]
        for init in ("empty", "cheap"):
            cm = np.full(g.nc, -1, np.int64)
            rm = np.full(g.nr, -1, np.int64)
            if init == "cheap":
                c0, r0 = O.cheap_init(g)
                cm[:], rm[:] = c0, r0
            for _ in range(g.nc + 2):
                f = S.bfs_phase(g.colptr, g.rowind, cm, rm, rng, order=order, one_end=one_end)
                for r in np.flatnonzero(f.marked):
                    rm[r] = -2
                S.alternate(f, cm, rm, rng, walk=walk, schedule="random")
                out = np.flatnonzero(f.pred < 0)
                m = rm[out]
                assert ((m == -1) | ((m >= 0) & (cm[np.maximum(m, 0)] == out))).all(), (i, init)
                S.fix_matching(cm, rm, f.marked, np.flatnonzero(f.pred >= 0))
                assert not (rm == -2).any()
                assert _valid(g, cm.astype(np.int32), rm.astype(np.int32)) is not None
                if not f.ends:
                    break
            assert int((cm >= 0).sum()) == ref, (i, g.name, init)
