"""A CPU schedule simulator of one phase of the GPU matching path.

It re-enacts, on small graphs and in plain Python, what the gfx950 kernels do
in a phase, with the schedule (the order in which concurrent lanes touch
memory) drawn at random or in lock-step, so that the arguments the kernels'
correctness rests on can be checked under adversarial interleavings:

  BFS (Algorithm 2 GPUBFS / Algorithm 4 GPUBFS-WR, APFB): frontier entries
      carry their root; a row is claimed once per phase (the atomic on the
      row word), its mate column joins the claimer's tree; an unmatched row
      becomes an augmenting-path end and, with WR, marks its root done,
      after which the tree's entries expand nothing.  Orders modelled:
      level-synchronous with edge visits of a level interleaved at random,
      "local levels" (a lane expands a column it just claimed before the
      level ends), and no levels at all (one phase-long pool of entries
      taken in random order).
  Alternate (Algorithm 3): one walk per end, each memory access a separate
      scheduling point; the classic walk (reads cmatch, stops where the
      predecessor check finds another walk's flip) or the recorded-row walk
      (follows the row each claim recorded, no check).
  FixMatching: rows whose column points elsewhere, and rows still marked
      -2, are unmatched.

Test infrastructure only; it shares no code with the library or the oracle.
"""
from __future__ import annotations

import random
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Forest:
    pred: np.ndarray          # [nr] column that claimed the row, -1
    prow: np.ndarray          # [nr] mate of the claiming column during the BFS (-1 for a root)
    root: np.ndarray          # [nc] root of the column's tree, -1 if not reached
    ends: list = field(default_factory=list)  # unmatched rows reached, in the order found
    marked: np.ndarray = None  # [nr] True for rows marked -2 (ends, and with one end per root the others)


def bfs_phase(colptr, rowind, cmatch, rmatch, rng: random.Random, wr=True, order="levels", one_end=False,
              local_p=0.0, stale_p=0.5):
    """One APFB BFS phase from every unmatched column with edges.

    order: "levels" (level-synchronous, edge visits of a level shuffled),
           "lockstep" (level-synchronous, entries visited in index order),
           "pool" (no levels: the next entry is drawn at random from all
           pending ones).
    local_p: with "levels", chance that a lane expands a column it just
           claimed before the level ends (local levels).
    stale_p: chance that a visit reads its root's done mark as it was when
           the level began ("pool": when the entry was queued), not as it is
           now: another lane's mark may not have reached it yet, so a tree
           can find several ends in one level."""
    nc, nr = len(cmatch), len(rmatch)
    visited = np.zeros(nr, bool)
    pred = np.full(nr, -1, np.int64)
    prow = np.full(nr, -1, np.int64)
    root = np.full(nc, -1, np.int64)
    done = np.zeros(nc, bool)
    marked = np.zeros(nr, bool)
    ends = []
    frontier = []
    for c in range(nc):
        if cmatch[c] == -1:
            root[c] = c
            if colptr[c + 1] > colptr[c]:
                frontier.append(c)

    snap = done.copy()

    def visit(c, r, push, seen=None):
        """One edge visit of entry c; its root's done mark read now, or
        (stale) as `seen` / the level's snapshot holds it."""
        R = root[c]
        stale = snap[R] if seen is None else seen
        if wr and (stale if rng.random() < stale_p else done[R]):
            return
        if visited[r]:
            return
        visited[r] = True                      # the claim: exactly one visitor per phase
        pred[r] = c
        prow[r] = cmatch[c]
        m = rmatch[r]
        if m >= 0:
            root[m] = R
            push(m)
        else:
            if one_end:
                # one end per root: a row reached after the first is left
                # unmatched at once (its claim keeps it out of the phase)
                if not done[R]:
                    ends.append(r)
                    marked[r] = True
            else:
                ends.append(r)
                marked[r] = True
            if wr:
                done[R] = True

    if order == "pool":
        pool = [(c, False) for c in frontier]
        while pool:
            c, seen = pool.pop(rng.randrange(len(pool)))
            rows = list(rowind[colptr[c]:colptr[c + 1]])
            for r in rows:
                visit(c, int(r), lambda m: pool.append((m, bool(done[root[m]]))), seen)
        return Forest(pred, prow, root, ends, marked)

    while frontier:
        snap[:] = done
        nxt = []
        if order == "lockstep":
            # entries side by side, one edge each per step (lanes of a wavefront)
            width = max(int(colptr[c + 1] - colptr[c]) for c in frontier)
            for k in range(width):
                for c in frontier:
                    if colptr[c] + k < colptr[c + 1]:
                        visit(c, int(rowind[colptr[c] + k]), nxt.append)
        else:
            work = [(c, int(r)) for c in frontier for r in rowind[colptr[c]:colptr[c + 1]]]
            rng.shuffle(work)
            while work:
                c, r = work.pop()
                newcols = []
                visit(c, r, newcols.append)
                for m in newcols:
                    if local_p and rng.random() < local_p:
                        # a local level: this lane expands its new column now
                        work.extend((m, int(x)) for x in rowind[colptr[m]:colptr[m + 1]])
                        rng.shuffle(work)
                    else:
                        nxt.append(m)
        frontier = nxt
    return Forest(pred, prow, root, ends, marked)


def _walk_classic(f: Forest, cmatch, rmatch, e, touched):
    """Algorithm 3 from end e, one memory access per yield; every row it
    writes, and the row it stops at, is reported to `touched`."""
    r = e
    c = f.pred[r]
    yield
    while True:
        r2 = cmatch[c]
        yield
        c2 = -1
        if r2 != -1:
            c2 = f.pred[r2]
            yield
            if c2 == c:
                touched.append(r)             # r keeps its old column
                return                        # c was already flipped by another walk
        cmatch[c] = r
        yield
        rmatch[r] = c
        touched.append(r)
        yield
        if r2 == -1:
            return                            # reached the root
        r, c = r2, c2


def _walk_recorded(f: Forest, cmatch, rmatch, e, touched):
    """The recorded-row walk from end e: pred and the recorded row, no check."""
    r = e
    while True:
        c = f.pred[r]
        yield
        r2 = f.prow[r]
        yield
        cmatch[c] = r
        yield
        rmatch[r] = c
        touched.append(r)
        yield
        if r2 == -1:
            return
        r = r2


def alternate(f: Forest, cmatch, rmatch, rng: random.Random, walk="recorded", schedule="random"):
    """Runs every walk to its end under the given schedule: "random" (the
    next access of a randomly chosen walk), "lockstep" (round robin, one
    access each, as lanes of a wavefront) or "sequential" (one walk after
    the other, in a random order)."""
    mk = _walk_recorded if walk == "recorded" else _walk_classic
    touched = []
    walks = [mk(f, cmatch, rmatch, e, touched) for e in f.ends]
    if schedule == "sequential":
        rng.shuffle(walks)
        for w in walks:
            for _ in w:
                pass
        return touched
    live = list(walks)
    while live:
        if schedule == "lockstep":
            nxt = []
            for w in live:
                try:
                    next(w)
                    nxt.append(w)
                except StopIteration:
                    pass
            live = nxt
        else:
            i = rng.randrange(len(live))
            try:
                next(live[i])
            except StopIteration:
                live.pop(i)
    return touched


def fix_matching(cmatch, rmatch, marked, rows=None):
    """Rows still marked -2 and rows whose column points elsewhere become
    unmatched; cmatch is not touched.  `rows`: only these rows (the rows
    the walks reported), else every row."""
    for r in (range(len(rmatch)) if rows is None else rows):
        if rmatch[r] < -1:
            rmatch[r] = -1
        elif rmatch[r] >= 0 and cmatch[rmatch[r]] != r:
            rmatch[r] = -1


def phase(colptr, rowind, cmatch, rmatch, rng, **kw):
    """One full phase; returns (forest, number of trees with an end)."""
    bkw = {k: kw[k] for k in ("wr", "order", "one_end", "local_p", "stale_p") if k in kw}
    f = bfs_phase(colptr, rowind, cmatch, rmatch, rng, **bkw)
    # rows reached as ends carry -2 until Alternate or FixMatching settles them
    for r in np.flatnonzero(f.marked):
        rmatch[r] = -2
    touched = alternate(f, cmatch, rmatch, rng, walk=kw.get("walk", "recorded"), schedule=kw.get("schedule", "random"))
    fix = kw.get("fix", "scan")
    # "list": the rows the walks reported; "reached": the rows claimed in the
    # phase (what the kernel's full scan gathers columns for); "scan": all
    rows = touched if fix == "list" else (np.flatnonzero(f.pred >= 0) if fix == "reached" else None)
    fix_matching(cmatch, rmatch, f.marked, rows)
    trees = len({int(f.root[f.pred[e]]) for e in f.ends})
    return f, trees
