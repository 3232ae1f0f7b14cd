"""Pins of the CPU oracle against facts that do not come from the oracle itself:
exhaustive search, closed forms, independent library routines, Konig's
theorem, and the paper's Fig. 1 worked example.  No GPU needed."""
import itertools

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle as O
from paper_1303_1379_amd import graphgen as gg
from conftest import load_golden


def _empty_match(g):
    return np.full(g.nc, -1, np.int32), np.full(g.nr, -1, np.int32)


def _hk(g, init="empty"):
    if init == "cheap":
        cm, rm = O.cheap_init(g)
    else:
        cm, rm = _empty_match(g)
    card, cm, rm, _ = O.hopcroft_karp(g, cm, rm)
    return card, cm, rm


def _certify(g, cm, rm):
    k, cc, rc = O.konig_cover(g, cm, rm)
    assert k >= 0
    assert O.verify_cover(g, cm, rm, cc, rc) == 0
    return k


# ------------------------------------------------------------ brute force
def _py_subsets(g):
    """The definition, in Python: largest edge subset with no shared vertex."""
    cols, rows = g.edges()
    e = list(zip(cols.tolist(), rows.tolist()))
    best = 0
    for k in range(len(e), 0, -1):
        for sub in itertools.combinations(e, k):
            cs = {c for c, _ in sub}
            rs = {r for _, r in sub}
            if len(cs) == k and len(rs) == k:
                return k
    return best


@pytest.mark.parametrize("seed", range(12))
def test_brute_force_variants_agree_with_definition(seed):
    rng = np.random.default_rng(seed)
    nc, nr = int(rng.integers(1, 6)), int(rng.integers(1, 6))
    g = gg.random_small(nc, nr, 0.45, seed)
    if g.nnz > 12:
        pytest.skip("python definition limited to 12 edges")
    v = _py_subsets(g)
    assert O.brute_force(g) == v
    assert O.brute_force_subsets(g) == v


@pytest.mark.parametrize("seed", range(60))
def test_hk_equals_brute_force_random_tiny(seed):
    rng = np.random.default_rng(1000 + seed)
    nc, nr = int(rng.integers(1, 13)), int(rng.integers(1, 13))
    p = float(rng.choice([0.1, 0.2, 0.35, 0.6]))
    g = gg.random_small(nc, nr, p, seed)
    bf = O.brute_force(g)
    for init in ("empty", "cheap"):
        card, cm, rm = _hk(g, init)
        assert card == bf
        assert O.check_matching(g, cm, rm) == card
        assert _certify(g, cm, rm) == card


@settings(max_examples=80, deadline=None)
@given(st.integers(1, 10), st.integers(1, 10), st.lists(st.tuples(st.integers(0, 9), st.integers(0, 9)), max_size=40))
def test_hk_equals_brute_force_hypothesis(nc, nr, edges):
    edges = [(c % nc, r % nr) for c, r in edges]
    g = gg.from_edges(nc, nr, edges)
    card, cm, rm = _hk(g, "cheap")
    assert card == O.brute_force(g)
    assert _certify(g, cm, rm) == card


# ------------------------------------------------------------ closed forms
@pytest.mark.parametrize("m,n", [(1, 1), (1, 7), (7, 1), (3, 5), (6, 6), (9, 4), (20, 13)])
def test_complete_bipartite(m, n):
    g = gg.complete(m, n)
    assert _hk(g, "cheap")[0] == min(m, n)
    assert _hk(g, "empty")[0] == min(m, n)


@pytest.mark.parametrize("k", [1, 2, 5, 40])
def test_star(k):
    assert _hk(gg.star(k))[0] == 1


@pytest.mark.parametrize("k", range(1, 16))
def test_path(k):
    g = gg.path(k)
    assert _hk(g)[0] == k // 2
    assert _hk(g, "cheap")[0] == k // 2


@pytest.mark.parametrize("n,extra,seed", [(10, 0, 0), (100, 2, 1), (1000, 3, 2), (5000, 5, 3)])
def test_permutation_plus_noise(n, extra, seed):
    g = gg.permutation_plus_noise(n, extra, seed)
    card, cm, rm = _hk(g, "cheap")
    assert card == n
    assert _certify(g, cm, rm) == n


def test_disjoint_union_adds():
    parts = [gg.complete(3, 5), gg.path(7), gg.star(4), gg.random_small(8, 9, 0.3, 5)]
    total = sum(_hk(p)[0] for p in parts)
    u = parts[0]
    for p in parts[1:]:
        u = gg.disjoint_union(u, p)
    assert _hk(u, "cheap")[0] == total


def test_empty_graphs():
    for nc, nr in [(0, 0), (0, 5), (5, 0), (4, 4)]:
        g = gg.empty(nc, nr)
        card, cm, rm = _hk(g, "cheap")
        assert card == 0
        assert (cm == -1).all() and (rm == -1).all()


@pytest.mark.parametrize("k", [1, 2, 5, 32, 64])
def test_full_grid_has_perfect_matching(k):
    g = gg.grid5(k, 0, 0, 7)
    assert g.nnz == 5 * k * k - 4 * k
    assert _hk(g, "cheap")[0] == k * k


@pytest.mark.parametrize("k,ndel", [(16, 3), (40, 50), (64, 100)])
def test_grid_with_emptied_columns_only(k, ndel):
    """Deleting only columns: the remaining diagonal stays intact, so nu = n - ndel."""
    g = gg.grid5(k, ndel, 0, 11)
    card, cm, rm = _hk(g, "cheap")
    assert card == k * k - ndel
    assert _certify(g, cm, rm) == card


@pytest.mark.parametrize("k,ndel", [(16, 3), (64, 100)])
def test_grid_with_emptied_rows_only(k, ndel):
    g = gg.grid5(k, 0, ndel, 13)
    assert _hk(g)[0] == k * k - ndel


@pytest.mark.parametrize("k,frac,seed", [(32, 0.03, 2), (128, 0.03, 2), (256, 0.05, 9)])
def test_grid_with_both_deletions_in_window(k, frac, seed):
    n = k * k
    nd = int(np.floor(frac * n))
    g, dc, dr = gg.grid5(k, nd, nd, seed, return_masks=True)
    card, cm, rm = _hk(g, "cheap")
    assert n - int((dc | dr).sum()) <= card <= n - nd
    assert _certify(g, cm, rm) == card


@pytest.mark.parametrize("seed", range(5))
def test_upper_bound_nonempty_vertices(seed):
    g = gg.uniform(300, 200, 2, seed)
    nonempty_cols = int((np.diff(g.colptr) > 0).sum())
    nonempty_rows = len(np.unique(g.rowind))
    assert _hk(g)[0] <= min(nonempty_cols, nonempty_rows)


# ------------------------------------------------------------ library cross-checks
@pytest.mark.parametrize("name", ["uniform2000", "grid64", "rmat12", "rmat14"])
def test_against_scipy(name):
    import scipy.sparse as sp
    from scipy.sparse.csgraph import maximum_bipartite_matching
    g = gg.workload(name)
    a = sp.csc_matrix((np.ones(g.nnz), g.rowind, g.colptr), shape=(g.nr, g.nc))
    perm = maximum_bipartite_matching(a.tocsr(), perm_type="column")
    ref = int((perm >= 0).sum())
    assert _hk(g, "cheap")[0] == ref
    assert _hk(g, "empty")[0] == ref


@pytest.mark.parametrize("seed", range(4))
def test_against_networkx(seed):
    import networkx as nx
    g = gg.uniform(150, 170, 3, seed)
    G = nx.Graph()
    G.add_nodes_from(("c", c) for c in range(g.nc))
    G.add_nodes_from(("r", r) for r in range(g.nr))
    cols, rows = g.edges()
    G.add_edges_from((("c", int(c)), ("r", int(r))) for c, r in zip(cols, rows))
    m = nx.bipartite.hopcroft_karp_matching(G, top_nodes=[("c", c) for c in range(g.nc)])
    assert _hk(g, "cheap")[0] == len(m) // 2


# ------------------------------------------------------------ cheap init
def test_cheap_init_rule_hand_example():
    # rows of a column are stored ascending: column 0 (rows 0, 2) takes 0;
    # column 1 (rows 0, 1) takes 1; column 2 (rows 0, 1) finds none free;
    # column 3 (row 2) takes 2.
    g = gg.from_edges(4, 3, [(0, 0), (0, 2), (1, 0), (1, 1), (2, 0), (2, 1), (3, 2)])
    cm, rm = O.cheap_init(g)
    assert cm.tolist() == [0, 1, -1, 2]
    assert rm.tolist() == [0, 1, 3]


@pytest.mark.parametrize("seed", range(6))
def test_cheap_init_is_maximal(seed):
    g = gg.uniform(400, 300, 3, seed)
    cm, rm = O.cheap_init(g)
    assert O.check_matching(g, cm, rm) is not None
    cols, rows = g.edges()
    # greedy leaves no edge with both endpoints unmatched
    assert not np.any((cm[cols] == -1) & (rm[rows] == -1))


# ------------------------------------------------------------ Konig certificate
def test_cover_detects_non_maximum_matching():
    g = gg.path(4)                           # c0-r0-c1-r1: nu = 2
    cm = np.array([-1, 0], np.int32)         # c1-r0 only: augmenting path c0-r0-c1-r1
    rm = np.array([1, -1], np.int32)
    k, _, _ = O.konig_cover(g, cm, rm)
    assert k == -3


def test_verifier_rejects_planted_errors():
    g = gg.uniform(200, 200, 3, 4)
    card, cm, rm = _hk(g, "cheap")
    k, cc, rc = O.konig_cover(g, cm, rm)
    assert k == card and O.verify_cover(g, cm, rm, cc, rc) == 0
    # (1) not a matching: break symmetry
    c = int(np.flatnonzero(cm >= 0)[0])
    cm2 = cm.copy(); cm2[c] = (cm[c] + 1) % g.nr
    assert O.verify_cover(g, cm2, rm, cc, rc) == 1
    # (2) an uncovered edge: drop a covered row whose edge has an uncovered column
    cols, rows = g.edges()
    idx = np.flatnonzero((cc[cols] == 0) & (rc[rows] == 1))
    rc2 = rc.copy(); rc2[rows[idx[0]]] = 0
    assert O.verify_cover(g, cm, rm, cc, rc2) == 2
    # (3) cover larger than the matching
    cc3 = cc.copy(); cc3[np.flatnonzero(cc == 0)[0]] = 1
    assert O.verify_cover(g, cm, rm, cc3, rc) == 3
    # a maximal but non-maximum matching cannot be certified
    cm0, rm0 = O.cheap_init(g)
    if (cm0 >= 0).sum() < card:
        assert O.konig_cover(g, cm0, rm0)[0] == -3


def test_check_matching_rejects_off_edge_pair():
    g = gg.from_edges(2, 2, [(0, 0), (1, 1)])
    assert O.check_matching(g, np.array([1, -1], np.int32), np.array([-1, 0], np.int32)) is None


# ------------------------------------------------------------ alternating BFS levels
def _nx_levels(g, cm, rm):
    """Independent: networkx BFS on the explicit alternating digraph."""
    import networkx as nx
    D = nx.DiGraph()
    D.add_node("src")
    cols, rows = g.edges()
    for c, r in zip(cols.tolist(), rows.tolist()):
        if cm[c] != r:
            D.add_edge(("c", c), ("r", r))
    for r in range(g.nr):
        if rm[r] >= 0:
            D.add_edge(("r", r), ("c", int(rm[r])))
    for c in range(g.nc):
        if cm[c] == -1:
            D.add_edge("src", ("c", c))
    dist = nx.single_source_shortest_path_length(D, "src")
    cl = np.full(g.nc, -1, np.int64)
    rl = np.full(g.nr, -1, np.int64)
    for v, d in dist.items():
        if v == "src":
            continue
        if v[0] == "c":
            cl[v[1]] = (d - 1) // 2
        else:
            rl[v[1]] = (d - 2) // 2
    return cl, rl


@pytest.mark.parametrize("seed", range(6))
def test_alt_bfs_levels_against_networkx(seed):
    g = gg.uniform(120, 130, 3, 50 + seed)
    cm, rm = O.cheap_init(g)
    cl, rl, nfree = O.alt_bfs_levels(g, cm, rm)
    ncl, nrl = _nx_levels(g, cm, rm)
    assert (cl == ncl).all()
    assert (rl == nrl).all()
    assert nfree == int(((rl >= 0) & (rm == -1)).sum())


# ------------------------------------------------------------ the paper's Fig. 1
def test_fig1_worked_example():
    d = load_golden("fig1.txt")
    g = gg.from_edges(d["nc"], d["nr"], d["edges"])
    cm = np.full(g.nc, -1, np.int32)
    rm = np.full(g.nr, -1, np.int32)
    for c, r in d["match"]:
        cm[c], rm[r] = r, c
    cl, rl, nfree = O.alt_bfs_levels(g, cm, rm)
    assert cl.tolist() == d["expect_clevel"]
    assert rl.tolist() == d["expect_rlevel"]
    assert nfree == d["expect_free_reached"]
    card, cm2, rm2, phases = O.hopcroft_karp(g, cm, rm)
    assert card == d["expect_card"] and phases == 1
    assert O.brute_force(g) == d["expect_card"]
    assert _certify(g, cm2, rm2) == d["expect_card"]


# ------------------------------------------------------------ input check (O0)
class _Raw:
    """A CSC pattern as given, without the generators' normalisation."""

    def __init__(self, nc, nr, colptr, rowind):
        self.nc, self.nr = nc, nr
        self.colptr = np.asarray(colptr, np.int32)
        self.rowind = np.asarray(rowind, np.int32)


def _scipy_accepts(g):
    """Independent decision: scipy's full structural check of a CSC matrix
    (index pointer starts at 0 and never decreases, indices in range)."""
    import scipy.sparse as sp
    try:
        a = sp.csc_matrix((np.ones(len(g.rowind)), g.rowind, g.colptr), shape=(g.nr, g.nc))
        a.check_format(full_check=True)
        return True
    except ValueError:
        return False


@pytest.mark.parametrize("nc,nr,colptr,rowind,ok", [
    (3, 3, [0, 1, 2, 3], [0, 1, 2], True),
    (0, 0, [0], [], True),
    (0, 4, [0], [], True),
    (2, 2, [0, 2, 2], [1, 1], True),             # duplicates and an empty column are well formed
    (2, 3, [0, 2, 3], [2, 0, 1], True),          # rows of a column in any order
    (3, 3, [1, 1, 2, 3], [0, 1, 2, 0], False),   # colptr[0] != 0
    (3, 3, [0, 2, 1, 3], [0, 1, 2], False),      # colptr decreases
    (3, 3, [0, 1, 2, 3], [0, 1, 3], False),      # row index = nr
    (3, 3, [0, 1, 2, 3], [0, -1, 2], False),     # negative row index
    (1, 0, [0, 1], [0], False),                  # an edge in a graph without rows
])
def test_check_csc_hand_cases(nc, nr, colptr, rowind, ok):
    g = _Raw(nc, nr, colptr, rowind)
    assert O.check_csc(g) == ok
    assert _scipy_accepts(g) == ok


def test_check_csc_rejects_negative_sizes():
    assert not O.check_csc(_Raw(-1, 3, [0], []))
    assert not O.check_csc(_Raw(2, -1, [0, 0, 0], []))


@pytest.mark.parametrize("seed", range(40))
def test_check_csc_agrees_with_scipy_on_planted_faults(seed):
    """A well-formed random pattern with at most one planted fault (colptr
    start, a decrease inside colptr, a row index out of range on either
    side): the oracle's verdict equals scipy's."""
    rng = np.random.default_rng(7000 + seed)
    g0 = gg.uniform(int(rng.integers(1, 40)), int(rng.integers(1, 40)), 3, seed)
    cp, ri = g0.colptr.copy(), g0.rowind.copy()
    fault = seed % 5
    if fault == 1:
        cp[0] = 1
    elif fault == 2 and g0.nc >= 2:
        c = int(rng.integers(1, g0.nc))
        cp[c] = cp[c + 1] + 1                    # cp[c] > cp[c + 1]: decreasing
    elif fault == 3 and len(ri):
        ri[int(rng.integers(0, len(ri)))] = g0.nr
    elif fault == 4 and len(ri):
        ri[int(rng.integers(0, len(ri)))] = -1 - int(rng.integers(0, 5))
    g = _Raw(g0.nc, g0.nr, cp, ri)
    assert O.check_csc(g) == _scipy_accepts(g)


def test_generated_workloads_are_well_formed():
    for name in ("uniform2000", "grid64", "rmat12"):
        g = gg.workload(name)
        assert O.check_csc(g) and _scipy_accepts(g)


# ------------------------------------------------------------ bounded Hopcroft-Karp (the CPU-baseline sample)
def _two_phase_graph():
    """Hand-worked instance.  Columns c0, c1, c2; rows r0, r1, r2; edges
    c0-r0, c1-r1, c2-r1, c2-r2 (rows of c2 stored r1 then r2); initial
    matching {c2-r1}.  Phase 1: the BFS layers c0, c1 (distance 0) and c2
    (distance 1, the mate of r1); r0 is free next to c0, so the shortest
    augmenting path has one column and only c0-r0 is augmented; the path
    c1-r1-c2-r2 (two columns) is left for phase 2.  Edges read, phase 1:
    BFS c0 (1) + c1 (1), c2 is not scanned (its distance reaches the limit);
    DFS from c0 reads r0 (1), from c1 reads r1 (1) and descends to c2, which
    reads r1 and r2 (2) before it is exhausted: 6 in all.  Phase 2: BFS
    c1 (1) + c2 (2), DFS c1 reads r1 (1), c2 reads r1, r2 (2) and augments:
    6 again.  A third BFS starts from no unmatched column: 0."""
    g = gg.from_edges(3, 3, [(0, 0), (1, 1), (2, 1), (2, 2)])
    cm = np.array([-1, -1, 1], np.int32)
    rm = np.array([-1, 2, -1], np.int32)
    return g, cm, rm


def test_bounded_hk_one_phase_is_valid_and_not_maximum():
    g, cm0, rm0 = _two_phase_graph()
    assert O.brute_force(g) == 3
    card, cm, rm, phases, edges = O.hopcroft_karp_ex(g, cm0, rm0, max_phases=1)
    assert (card, phases, edges) == (2, 1, 6)
    assert O.check_matching(g, cm, rm) == 2
    assert cm.tolist() == [0, -1, 1] and rm.tolist() == [0, 2, -1]
    assert O.konig_cover(g, cm, rm)[0] == -3          # not maximum: an augmenting path is left
    card, cm, rm, phases, edges = O.hopcroft_karp_ex(g, cm0, rm0)
    assert (card, phases, edges) == (3, 2, 12)
    assert _certify(g, cm, rm) == 3


def test_bounded_hk_sample_adds_up_to_the_complete_run():
    g, cm0, rm0 = _two_phase_graph()
    s = O.hopcroft_karp_sample(g, cm0, rm0, budget_s=60.0)
    assert s == {**s, "phases": 2, "edges": 12, "card": 3, "done": True}
    # on a larger input: phase by phase, the same phases, edges and result as one complete run
    g = gg.workload("grid64")
    cm0, rm0 = O.cheap_init(g)
    card, _, _, phases, edges = O.hopcroft_karp_ex(g, cm0, rm0)
    s = O.hopcroft_karp_sample(g, cm0, rm0, budget_s=60.0)
    assert s["done"] and (s["card"], s["phases"], s["edges"]) == (card, phases, edges)
    import scipy.sparse as sp
    from scipy.sparse.csgraph import maximum_bipartite_matching
    a = sp.csc_matrix((np.ones(g.nnz), g.rowind, g.colptr), shape=(g.nr, g.nc))
    assert card == int((maximum_bipartite_matching(a.tocsr(), perm_type="column") >= 0).sum())
    # a budget of zero runs no phase
    s0 = O.hopcroft_karp_sample(g, cm0, rm0, budget_s=0.0)
    assert s0["phases"] == 0 and s0["edges"] == 0 and not s0["done"]
