"""The forest of one BFS phase as the GPU grows it (mcm_bfs_forest), checked
against what the paper's BFS kernels guarantee.

GPUBFS (Algorithm 2) is level-synchronous and its level sets do not depend
on the schedule: they must equal the oracle's alternating-BFS levels
exactly.  GPUBFS-WR (Algorithm 4) reads the root's done mark while the level
runs, so its sets depend on the schedule; what it guarantees, and what is
checked here under every claim, flush, end and root-test form:
  * a subset of GPUBFS: every column it reaches is reached by GPUBFS, never
    at a lower level;
  * tree structure: a non-root column m is reached through its matched row
    r, whose predecessor p (a column adjacent to r) is one level lower and
    in the same tree: root[m] = root[pred[cmatch[m]]];
  * early exit: a tree stops growing one level after its root first reached
    an unmatched row (the done mark is set during that level and read at the
    next);
  * with one end per root, no root has two ends; every end is an unmatched
    row reached from a column of its tree, and ends are distinct."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_1303_1379_amd import graphgen as gg, mcm  # noqa: E402

DEFAULTS = dict(bfs="wr", endpoints="auto", claim="auto", flush="auto", wr_check="auto", mapping="auto",
                loop="auto", barrier="counter")


@pytest.fixture(autouse=True)
def _reset():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    yield
    for k, v in DEFAULTS.items():
        mcm.set_option(k, v)


def _forest(g, cm, rm):
    dg = mcm.to_device(g)
    ends, cl, cr, rp = mcm.bfs_forest(dg, torch.from_numpy(cm).cuda(), torch.from_numpy(rm).cuda())
    return ends.cpu().numpy(), cl.cpu().numpy(), cr.cpu().numpy(), rp.cpu().numpy()


def _is_edge(g, c, r):
    """Whether each (c[i], r[i]) is an edge of g (vectorised)."""
    cols, rows = g.edges()
    keys = np.unique(cols * g.nr + rows)
    q = np.asarray(c, np.int64) * g.nr + np.asarray(r, np.int64)
    return np.isin(q, keys)


def _check_structure(g, cm, rm, ends, cl, cr, rp):
    un = cm == -1
    assert (cl[un] == 0).all() and (cr[un] == np.flatnonzero(un)).all()
    reached = cl >= 0
    assert ((cr >= 0) == reached).all()
    m = np.flatnonzero(reached & ~un)          # non-root columns: reached through their matched row
    r = cm[m]
    p = rp[r]
    assert (p >= 0).all()
    assert (cl[p] >= 0).all() and (cl[m] == cl[p] + 1).all() and (cr[m] == cr[p]).all()
    assert _is_edge(g, p, r).all()
    rr = np.flatnonzero(rp >= 0)               # reached rows: claimed from an adjacent reached column
    pp = rp[rr]
    assert (cl[pp] >= 0).all() and _is_edge(g, pp, rr).all()
    mr = rm[rr] >= 0                           # a matched row brings its column into the claimer's tree
    assert (cl[rm[rr][mr]] == cl[pp[mr]] + 1).all() and (cr[rm[rr][mr]] == cr[pp[mr]]).all()
    assert len(np.unique(ends)) == len(ends)
    assert (rm[ends] == -1).all() and (rp[ends] >= 0).all()


@pytest.mark.parametrize("name", ["grid128", "grid256p", "rmat13", "uniform2000"])
def test_gpubfs_forest_equals_oracle_levels(name):
    g = gg.workload(name)
    cm, rm = O.cheap_init(g)
    mcm.set_option("bfs", "plain")
    ends, cl, cr, rp = _forest(g, cm, rm)
    ocl, orl, nfree = O.alt_bfs_levels(g, cm, rm)
    assert (cl == ocl).all()
    assert ((rp >= 0) == (orl >= 0)).all()
    assert len(ends) == nfree
    _check_structure(g, cm, rm, ends, cl, cr, rp)


FORMS = [dict(claim=c, flush=f, endpoints=e, wr_check=w) for c in ("probe", "max") for f in ("atomic", "defer")
         for e in ("all", "one") for w in ("early", "late")]


@pytest.mark.parametrize("name", ["grid128", "grid256p", "rmat13", "uniform2000"])
def test_gpubfs_wr_invariants(name):
    g = gg.workload(name)
    cm, rm = O.cheap_init(g)
    ocl, _, _ = O.alt_bfs_levels(g, cm, rm)
    for form in FORMS:
        for k, v in form.items():
            mcm.set_option(k, v)
        mcm.set_option("bfs", "wr")
        ends, cl, cr, rp = _forest(g, cm, rm)
        _check_structure(g, cm, rm, ends, cl, cr, rp)
        reached = cl >= 0
        assert (ocl[reached] >= 0).all(), form                  # subset of GPUBFS
        assert (cl[reached] >= ocl[reached]).all(), form        # never earlier
        # early exit: a tree stops one level after its root's first end
        end_root = cr[rp[ends]]
        end_level = cl[rp[ends]]
        first = {}
        for R, L in zip(end_root.tolist(), end_level.tolist()):
            first[R] = min(first.get(R, L), L)
        for R, L in first.items():
            assert cl[cr == R].max() <= L + 1, (form, R, L)
        if form["endpoints"] == "one":
            assert len(np.unique(end_root)) == len(end_root), form
        # every root with an end was stopped: fewer columns than GPUBFS reaches overall, or equal
        assert reached.sum() <= (ocl >= 0).sum()
