"""GPU path vs the CPU oracle, through the C ABI.

Cardinality must equal the oracle's exactly; the returned arrays must form a
matching of the input; maximality is certified by a Konig cover exported by
the GPU and checked by the oracle's independent verifier.  The matching
arrays themselves are not compared: maximum matchings are not unique and the
GPU's depends on the schedule of the concurrent flips."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_1303_1379_amd import graphgen as gg, mcm  # noqa: E402
from conftest import load_golden  # noqa: E402

DRIVER_COMBOS = [
    dict(driver="apfb", bfs="wr", mapping="wave", loop="device"),
    dict(driver="apfb", bfs="wr", mapping="thread", loop="device"),
    dict(driver="apfb", bfs="plain", mapping="wave", loop="device"),
    dict(driver="apsb", bfs="wr", mapping="wave", loop="device"),
    dict(driver="apsb", bfs="plain", mapping="thread", loop="device"),
    dict(driver="apfb", bfs="wr", mapping="wave", loop="host"),
    dict(driver="apsb", bfs="wr", mapping="thread", loop="host"),
    dict(driver="apfb", bfs="wr", mapping="wave", loop="device", endpoints="one"),
    dict(driver="apsb", bfs="wr", mapping="wave", loop="device", endpoints="all"),
    dict(driver="apsb", bfs="wr", mapping="thread", loop="host", endpoints="one"),
    # level-free BFS (no grid barrier between levels)
    dict(driver="apfb", bfs="wr", mapping="wave", loop="device", schedule="async"),
    dict(driver="apfb", bfs="wr", mapping="thread", loop="device", schedule="async"),
    dict(driver="apfb", bfs="plain", mapping="wave", loop="device", schedule="async"),
    dict(driver="apfb", bfs="wr", mapping="wave", loop="device", endpoints="one", schedule="async"),
]

DEFAULTS = dict(driver="apfb", bfs="wr", mapping="auto", loop="auto", validate=0, stats=0, wg_threshold=16384,
                level_entries=128, idle_sleep=8, wr_check="auto", small_max=256, endpoints="auto", barrier="counter", claim="auto", flush="auto", local_levels="auto", local_edges=1024, wg_lds="on", fuse="on",
                alternate="auto", schedule="levels", fix="auto", roots="auto")


@pytest.fixture(autouse=True)
def _reset_options():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    for k, v in DEFAULTS.items():
        mcm.set_option(k, v)
    yield
    for k, v in DEFAULTS.items():
        mcm.set_option(k, v)


def _set(**kw):
    for k, v in kw.items():
        mcm.set_option(k, v)


def _oracle_card(g, init="cheap"):
    if init == "cheap":
        cm, rm = O.cheap_init(g)
    else:
        cm, rm = np.full(g.nc, -1, np.int32), np.full(g.nr, -1, np.int32)
    return O.hopcroft_karp(g, cm, rm)[0]


def _gpu(g, init="cheap", certify=True):
    dg = mcm.to_device(g)
    if init == "cheap":
        _, cm0, rm0 = mcm.cheap_init_host(g.colptr, g.rowind, g.nr)
        card, cm, rm = mcm.match(dg, torch.from_numpy(cm0).cuda(), torch.from_numpy(rm0).cuda())
    else:
        card, cm, rm = mcm.match(dg)
    cmh, rmh = cm.cpu().numpy(), rm.cpu().numpy()
    assert O.check_matching(g, cmh, rmh) == card, f"{g.name}: not a matching of size {card}"
    if certify:
        k, cc, rc = mcm.konig_cover(dg, cm, rm)
        assert k == card
        assert O.verify_cover(g, cmh, rmh, cc.cpu().numpy(), rc.cpu().numpy()) == 0
    return card, cmh, rmh


# ------------------------------------------------------------------ the paper's Fig. 1
def test_fig1_worked_example():
    d = load_golden("fig1.txt")
    g = gg.from_edges(d["nc"], d["nr"], d["edges"])
    cm = np.full(g.nc, -1, np.int32)
    rm = np.full(g.nr, -1, np.int32)
    for c, r in d["match"]:
        cm[c], rm[r] = r, c
    dg = mcm.to_device(g)
    cmt, rmt = torch.from_numpy(cm).cuda(), torch.from_numpy(rm).cuda()
    nfree, cl, rp = mcm.bfs_levels(dg, cmt, rmt)
    assert nfree == d["expect_free_reached"]
    assert cl.cpu().tolist() == d["expect_clevel"]
    # r2 and r3 are both reached from c2 (the second walk must stop at c2)
    assert rp.cpu().tolist() == [0, 1, 1]
    for combo in DRIVER_COMBOS:
        for thr in (16384, 0):
            _set(wg_threshold=thr, **combo)
            card, cmo, rmo = mcm.match(dg, cmt.clone(), rmt.clone())
            assert card == d["expect_card"], (combo, thr)
            assert O.check_matching(g, cmo.cpu().numpy(), rmo.cpu().numpy()) == card


# ------------------------------------------------------------------ tiny graphs, every path
@pytest.mark.parametrize("path", ["wg", "device", "host"])
def test_random_tiny_graphs(path):
    rng = np.random.default_rng(7)
    if path == "wg":
        _set(wg_threshold=1 << 30)
    else:
        _set(wg_threshold=0, loop=path)
    for i in range(60):
        nc, nr = int(rng.integers(1, 14)), int(rng.integers(1, 14))
        g = gg.random_small(nc, nr, float(rng.choice([0.1, 0.25, 0.5])), 100 + i)
        bf = O.brute_force(g)
        for init in ("cheap", "empty"):
            card, _, _ = _gpu(g, init)
            assert card == bf, (path, i, init)


# ------------------------------------------------------------------ closed forms and edge cases
@pytest.mark.parametrize("thr", [1 << 30, 0])
def test_closed_forms(thr):
    _set(wg_threshold=thr)
    assert _gpu(gg.complete(7, 5))[0] == 5
    assert _gpu(gg.complete(5, 9), "empty")[0] == 5
    assert _gpu(gg.star(30))[0] == 1
    for k in (2, 7, 64, 513):
        assert _gpu(gg.path(k), "empty")[0] == k // 2
    assert _gpu(gg.permutation_plus_noise(3000, 3, 4))[0] == 3000
    assert _gpu(gg.grid5(64, 0, 0, 1), "empty")[0] == 64 * 64
    assert _gpu(gg.grid5(64, 200, 0, 3))[0] == 64 * 64 - 200


def test_empty_inputs():
    for nc, nr in [(0, 0), (0, 5), (5, 0), (6, 4)]:
        g = gg.empty(nc, nr)
        dg = mcm.to_device(g)
        card, cm, rm = mcm.match(dg)
        assert card == 0
        assert (cm.cpu().numpy() == -1).all() and (rm.cpu().numpy() == -1).all()
        k, cc, rc = mcm.konig_cover(dg, cm, rm)
        assert k == 0


def test_outputs_may_alias_init():
    g = gg.workload("grid64")
    _, cm0, rm0 = mcm.cheap_init_host(g.colptr, g.rowind, g.nr)
    dg = mcm.to_device(g)
    for thr in (1 << 30, 0):
        _set(wg_threshold=thr)
        cm = torch.from_numpy(cm0).cuda()
        rm = torch.from_numpy(rm0).cuda()
        card, cmo, rmo = mcm.match(dg, cm, rm, out_cmatch=cm, out_rmatch=rm)
        assert cmo.data_ptr() == cm.data_ptr()
        assert card == _oracle_card(g)
        assert O.check_matching(g, cm.cpu().numpy(), rm.cpu().numpy()) == card


def test_maximum_init_is_kept():
    g = gg.workload("uniform2000")
    card, cm, rm, _ = O.hopcroft_karp(g, *O.cheap_init(g))
    dg = mcm.to_device(g)
    c2, cmo, rmo = mcm.match(dg, torch.from_numpy(cm).cuda(), torch.from_numpy(rm).cuda())
    assert c2 == card
    assert mcm.last_stats()["phases"] == 1


# ------------------------------------------------------------------ level sets of one BFS (GPUBFS mode)
@pytest.mark.parametrize("name", ["uniform2000", "grid96", "rmat12"])
@pytest.mark.parametrize("mapping", ["wave", "thread"])
@pytest.mark.parametrize("loop", ["device", "host"])
def test_bfs_levels_exact(name, mapping, loop):
    _set(mapping=mapping, loop=loop)
    g = gg.workload(name)
    cm, rm = O.cheap_init(g)
    ocl, orl, ofree = O.alt_bfs_levels(g, cm, rm)
    dg = mcm.to_device(g)
    nfree, cl, rp = mcm.bfs_levels(dg, torch.from_numpy(cm).cuda(), torch.from_numpy(rm).cuda())
    cl, rp = cl.cpu().numpy(), rp.cpu().numpy()
    assert nfree == ofree
    assert (cl == ocl).all()
    reached = rp >= 0
    assert (reached == (orl >= 0)).all()
    # pred[r] is a column adjacent to r at the level that reaches r
    rows = np.flatnonzero(reached)
    pc = rp[rows]
    assert (cl[pc] == orl[rows]).all()
    for r, c in zip(rows[:4000], pc[:4000]):
        assert r in g.rowind[g.colptr[c]:g.colptr[c + 1]]


# ------------------------------------------------------------------ driver variants
@pytest.mark.parametrize("combo", DRIVER_COMBOS, ids=lambda c: "-".join(c.values()))
@pytest.mark.parametrize("name", ["uniform2000", "grid128", "rmat13"])
def test_driver_variants(combo, name):
    g = gg.workload(name)
    ref = _oracle_card(g)
    for thr in (1 << 30, 0):
        _set(wg_threshold=thr, **combo)
        card, _, _ = _gpu(g)
        assert card == ref, (combo, thr)


# Both ways of claiming a row, forced on graphs of either degree profile
# (auto picks the atomic maximum for the grids and uniform graphs and the
# probe for R-MAT): drivers, mappings, both level loops, both end rules,
# single-workgroup runs of small levels on and off, cheap and empty starts.
CLAIM_COMBOS = [dict(driver="apfb", mapping="wave", loop="device", endpoints="auto", small_max=256),
                dict(driver="apfb", mapping="wave", loop="device", endpoints="auto", schedule="async"),
                dict(driver="apfb", mapping="thread", loop="device", endpoints="one", small_max=0),
                dict(driver="apsb", mapping="wave", loop="device", endpoints="auto", small_max=0),
                dict(driver="apsb", mapping="thread", loop="host", endpoints="all", small_max=256),
                dict(driver="apfb", mapping="wave", loop="host", endpoints="auto", small_max=256)]


@pytest.mark.parametrize("claim", ["max", "probe"])
@pytest.mark.parametrize("combo", CLAIM_COMBOS, ids=lambda c: "-".join(str(v) for v in c.values()))
@pytest.mark.parametrize("name", ["uniform2000", "grid128", "grid256p", "rmat13"])
def test_claim_modes(claim, combo, name):
    g = gg.workload(name)
    _set(wg_threshold=0, claim=claim, **combo)
    assert _gpu(g)[0] == _oracle_card(g), (claim, combo)
    assert _gpu(g, "empty", certify=False)[0] == _oracle_card(g, "empty"), (claim, combo)


# Both ways of reserving a grid level's next frontier: a queue atomic per
# workgroup, or the counter barrier's own addition with the entries written
# after arriving (deferred).  Cases: APsB stops that leave a frontier behind
# in a grid level (small_max 0) and in a single-workgroup run; every level
# on all blocks; one block per entry; few blocks; R-MAT levels large enough
# that wavefronts drain their stage during the level; cheap and empty starts.
FLUSH_COMBOS = [dict(driver="apfb", mapping="wave", level_entries=128, small_max=256),
                dict(driver="apsb", mapping="wave", level_entries=1, small_max=0),
                dict(driver="apsb", mapping="thread", level_entries=128, small_max=256),
                dict(driver="apfb", mapping="thread", level_entries=0, small_max=0),
                dict(driver="apsb", mapping="wave", level_entries=4096, small_max=0, endpoints="all")]


@pytest.mark.parametrize("flush", ["defer", "atomic"])
@pytest.mark.parametrize("combo", FLUSH_COMBOS, ids=lambda c: "-".join(str(v) for v in c.values()))
@pytest.mark.parametrize("name", ["uniform2000", "grid256p", "rmat15"])
def test_flush_modes(flush, combo, name):
    g = gg.workload(name)
    _set(wg_threshold=0, loop="device", flush=flush, **combo)
    assert _gpu(g)[0] == _oracle_card(g), (flush, combo)
    assert _gpu(g, "empty", certify=False)[0] == _oracle_card(g, "empty"), (flush, combo)


# Local levels: a wavefront expands the entries it just claimed before the
# grid level ends (the trees are no longer level-exact, the cardinality is
# still the oracle's).  Both mappings and drivers, both flush forms, both
# claims, APsB stops in a local level.
LOCAL_COMBOS = [dict(driver="apfb", mapping="wave", flush="defer", claim="max"),
                dict(driver="apsb", mapping="wave", flush="defer", claim="probe"),
                dict(driver="apfb", mapping="thread", flush="atomic", claim="probe"),
                dict(driver="apsb", mapping="thread", flush="atomic", claim="max", endpoints="all")]


@pytest.mark.parametrize("local", [0, 1, 3, 16])
@pytest.mark.parametrize("combo", LOCAL_COMBOS, ids=lambda c: "-".join(str(v) for v in c.values()))
@pytest.mark.parametrize("name", ["uniform2000", "grid256p", "rmat15"])
def test_local_levels(local, combo, name):
    g = gg.workload(name)
    _set(wg_threshold=0, loop="device", small_max=0, local_levels=local, **combo)
    assert _gpu(g)[0] == _oracle_card(g), (local, combo)
    assert _gpu(g, "empty", certify=False)[0] == _oracle_card(g, "empty"), (local, combo)


# A local level takes only the newest staged entries whose edges fit the
# local_edges budget (at least one entry), leaving the older ones staged for
# the next grid level: budgets of one edge (one entry per local level), of a
# few entries, the default and none; both claims, both drivers.
@pytest.mark.parametrize("edges", [1, 40, 1024, 0])
@pytest.mark.parametrize("combo", [dict(driver="apfb", claim="probe"), dict(driver="apsb", claim="max"),
                                   dict(driver="apfb", claim="max", endpoints="all")],
                         ids=lambda c: "-".join(str(v) for v in c.values()))
@pytest.mark.parametrize("name", ["rmat15", "grid256p", "uniform2000"])
def test_local_edge_budget(edges, combo, name):
    g = gg.workload(name)
    _set(wg_threshold=0, loop="device", small_max=0, local_levels=16, local_edges=edges, **combo)
    assert _gpu(g)[0] == _oracle_card(g), (edges, combo)
    assert _gpu(g, "empty", certify=False)[0] == _oracle_card(g, "empty"), (edges, combo)


@pytest.mark.parametrize("name,low", [("grid256p", True), ("uniform2000", True), ("rmat15", False)])
def test_auto_claim_and_flush(name, low):
    """claim, flush, wr_check and alternate on auto pick the atomic maximum,
    deferred levels, the root test beside the edge visit and the recorded-row
    Alternate for graphs with at most 8 edges per row on average, the probe,
    the queue atomic, the root test before the scan and the classic Alternate
    otherwise; deferred levels need the device loop and the counter
    barrier."""
    g = gg.workload(name)
    ref = _oracle_card(g)
    _set(wg_threshold=0, local_levels="auto")
    assert _gpu(g, certify=False)[0] == ref
    s = mcm.last_stats()
    assert (s["claim"], s["flush"], s["wr_check"], s["alternate"]) == ((1, 1, 1, 1) if low else (0, 0, 0, 0))
    assert s["local_levels"] == (6 if low else 16)
    _set(loop="host")
    assert _gpu(g, certify=False)[0] == ref
    assert mcm.last_stats()["flush"] == 0
    _set(loop="device", barrier="flags")
    assert _gpu(g, certify=False)[0] == ref
    assert mcm.last_stats()["flush"] == 0


# Alternate following the rows recorded at the claims (fast) or reading
# cmatch at each step (classic): several ends per root (APFB, shared ways to
# the root, junction conflicts), one end per root (APsB), both mappings (the
# wave mapping hands each edge its entry's recorded row across lanes, also in
# rounds where the owner lane has no edge of its own), both level loops, and
# local levels on and off.  grid128 and rmat13 are where a lane-shuffle
# mistake once recorded wrong rows.
ALT_COMBOS = [dict(driver="apfb", mapping="wave", loop="device", endpoints="all"),
              dict(driver="apfb", mapping="thread", loop="device", endpoints="all", local_levels=0),
              dict(driver="apsb", mapping="wave", loop="device", endpoints="one"),
              dict(driver="apfb", mapping="wave", loop="host", endpoints="all"),
              dict(driver="apsb", mapping="thread", loop="host", endpoints="all"),
              dict(driver="apfb", bfs="plain", mapping="wave", loop="device", endpoints="all"),
              dict(driver="apfb", mapping="wave", loop="device", endpoints="all", schedule="async"),
              dict(driver="apfb", bfs="plain", mapping="thread", loop="device", endpoints="all", schedule="async")]


@pytest.mark.parametrize("alt", ["fast", "classic"])
@pytest.mark.parametrize("combo", ALT_COMBOS, ids=lambda c: "-".join(str(v) for v in c.values()))
@pytest.mark.parametrize("name", ["grid128", "rmat13", "uniform2000", "grid256p"])
def test_alternate_forms(alt, combo, name):
    g = gg.workload(name)
    _set(wg_threshold=0, alternate=alt, **combo)
    assert _gpu(g)[0] == _oracle_card(g), (alt, combo)
    assert _gpu(g, "empty", certify=False)[0] == _oracle_card(g, "empty"), (alt, combo)


# FixMatching over every row or over the rows the walks reported, the root
# scan over every column or over the previous phase's roots, with both
# schedules and both walks; one end per root leaves the other unmatched rows
# it reaches unmatched at once (no row is left marked for FixMatching).
@pytest.mark.parametrize("fix", ["scan", "list", "auto"])
@pytest.mark.parametrize("roots", ["scan", "list", "auto"])
@pytest.mark.parametrize("form", [dict(schedule="levels", alternate="fast"), dict(schedule="levels", alternate="classic"),
                                  dict(schedule="async", alternate="fast"), dict(schedule="async", alternate="classic"),
                                  dict(schedule="levels", alternate="classic", endpoints="one"),
                                  dict(schedule="async", alternate="fast", endpoints="one", bfs="wr")],
                         ids=lambda d: "-".join(str(v) for v in d.values()))
@pytest.mark.parametrize("name", ["grid128", "rmat13", "grid256p"])
def test_listed_passes(fix, roots, form, name):
    g = gg.workload(name)
    _set(wg_threshold=0, fix=fix, roots=roots, **form)
    assert _gpu(g)[0] == _oracle_card(g), (fix, roots, form)
    assert _gpu(g, "empty", certify=False)[0] == _oracle_card(g, "empty"), (fix, roots, form)


# The one-workgroup path (ncols + nrows at most wg_threshold) with the graph
# in the workgroup's LDS where it fits (uniform2000, grid32, the small
# R-MAT) and in global memory where it does not (rmat13's 110 k edges), and
# with the arena off; both drivers, both mappings, runs in a row on one
# workspace, from the greedy and from the empty matching.
@pytest.mark.parametrize("lds", ["on", "off"])
@pytest.mark.parametrize("combo", [dict(driver="apfb", mapping="wave"), dict(driver="apsb", mapping="wave"),
                                   dict(driver="apfb", mapping="thread", endpoints="one")],
                         ids=lambda c: "-".join(str(v) for v in c.values()))
@pytest.mark.parametrize("name", ["uniform2000", "grid32", "rmat10", "rmat13"])
def test_one_workgroup_lds(lds, combo, name):
    g = gg.workload(name)
    ref = _oracle_card(g)
    _set(wg_lds=lds, **combo)
    assert g.nc + g.nr <= 16384
    for _ in range(2):
        assert _gpu(g)[0] == ref, (lds, combo)
    assert _gpu(g, "empty", certify=False)[0] == _oracle_card(g, "empty"), (lds, combo)


# BFS level 0 in the root scan's pass (probe claims; phases that do not list
# their roots) and as a level of its own: both drivers, roots listed or
# scanned, both Alternate forms (the recorded-row one leaves the two-edge
# rounds), both FixMatching forms, low-degree graphs with probe claims too;
# runs in a row on one workspace.
@pytest.mark.parametrize("fuse", ["on", "off"])
@pytest.mark.parametrize("combo", [dict(driver="apfb", roots="auto", fix="auto"),
                                   dict(driver="apfb", roots="scan", fix="scan", alternate="fast"),
                                   dict(driver="apsb", roots="auto", fix="list"),
                                   dict(driver="apfb", roots="list", fix="auto", local_levels=0),
                                   dict(driver="apfb", roots="auto", fix="auto", wr_check="late", endpoints="one")],
                         ids=lambda c: "-".join(str(v) for v in c.values()))
@pytest.mark.parametrize("name", ["rmat13", "rmat15", "grid128", "uniform2000"])
def test_fused_level0(fuse, combo, name):
    g = gg.workload(name)
    ref = _oracle_card(g)
    _set(wg_threshold=0, claim="probe", fuse=fuse, **combo)
    for _ in range(2):
        assert _gpu(g)[0] == ref, (fuse, combo)
    assert _gpu(g, "empty", certify=False)[0] == _oracle_card(g, "empty"), (fuse, combo)


def test_deferred_levels_repeated():
    """Many runs in a row on one workspace with deferred grid levels (queue
    slots reused across levels, phases and runs; barriers between grid
    levels without fences), varying the participating blocks and the
    driver: every run equals the oracle's cardinality and is a valid
    matching."""
    for name in ("grid256p", "grid200", "rmat14"):
        g = gg.workload(name)
        ref = _oracle_card(g)
        ref0 = _oracle_card(g, "empty")
        for i in range(12):
            _set(wg_threshold=0, loop="device", flush="defer", claim=("max", "probe")[i % 2],
                 level_entries=(16, 128, 1024)[i % 3], driver=("apfb", "apsb")[(i // 3) % 2],
                 small_max=(0, 256)[(i // 6) % 2])
            assert _gpu(g, certify=False)[0] == ref, (name, i)
            assert _gpu(g, "empty", certify=False)[0] == ref0, (name, i)


# Grid levels with a varying number of participating blocks: every block
# (0), one block per frontier entry (1), few blocks (4096); no single-workgroup
# runs (small_max 0: every level crosses the grid barrier); APsB carries its
# stop flag through the barrier; both places of the WR root check.
ELASTIC = [dict(level_entries=0, idle_sleep=1, small_max=256, driver="apfb", wr_check="late"),
           dict(level_entries=1, idle_sleep=0, small_max=0, driver="apfb", wr_check="late"),
           dict(level_entries=64, idle_sleep=1, small_max=0, driver="apsb", wr_check="early"),
           dict(level_entries=4096, idle_sleep=64, small_max=256, driver="apsb", wr_check="late"),
           dict(level_entries=4096, idle_sleep=8, small_max=0, driver="apfb", wr_check="early"),
           dict(level_entries=1, idle_sleep=0, small_max=0, driver="apfb", wr_check="late", barrier="flags"),
           dict(level_entries=128, idle_sleep=8, small_max=256, driver="apsb", wr_check="late", barrier="counter"),
           dict(level_entries=0, idle_sleep=1, small_max=0, driver="apsb", wr_check="early", barrier="flags")]


@pytest.mark.parametrize("combo", ELASTIC, ids=lambda c: "-".join(str(v) for v in c.values()))
@pytest.mark.parametrize("name", ["grid256", "rmat15", "uniform2000"])
def test_elastic_grid_levels(combo, name):
    g = gg.workload(name)
    ref = _oracle_card(g)
    _set(wg_threshold=0, loop="device", **combo)
    card, _, _ = _gpu(g)
    assert card == ref, combo
    assert _gpu(g, "empty", certify=False)[0] == _oracle_card(g, "empty")


@pytest.mark.parametrize("name,init", [("grid256", "cheap"), ("grid200", "empty"), ("rmat15", "cheap"),
                                       ("rmat14", "empty")])
def test_medium_graphs(name, init):
    g = gg.workload(name)
    card, _, _ = _gpu(g, init)
    assert card == _oracle_card(g, init)


def test_uneven_and_rectangular():
    for nc, nr, d, s in [(5000, 800, 3, 1), (800, 5000, 6, 2), (20000, 20000, 2, 3), (40000, 9000, 1, 4)]:
        g = gg.uniform(nc, nr, d, s)
        assert _gpu(g)[0] == _oracle_card(g)
        assert _gpu(g, "empty")[0] == _oracle_card(g, "empty")


def test_validation_errors():
    _set(validate=1)
    g = gg.workload("grid64")
    dg = mcm.to_device(g)
    _, cm0, rm0 = mcm.cheap_init_host(g.colptr, g.rowind, g.nr)
    bad_c = cm0.copy()
    c = int(np.flatnonzero(bad_c >= 0)[0])
    bad_c[c] = (bad_c[c] + 7) % g.nr            # no longer symmetric
    with pytest.raises(mcm.McmError) as e:
        mcm.match(dg, torch.from_numpy(bad_c).cuda(), torch.from_numpy(rm0).cuda())
    assert e.value.code == mcm.MCM_EBADINIT
    bad_ri = g.rowind.copy()
    bad_ri[5] = g.nr + 3                         # row out of range
    dgb = mcm.DeviceGraph(g.nc, g.nr, dg.colptr, torch.from_numpy(bad_ri).cuda())
    with pytest.raises(mcm.McmError) as e:
        mcm.match(dgb)
    assert e.value.code == mcm.MCM_EINVAL
    # the valid input still passes with validation on
    assert mcm.match(dg, torch.from_numpy(cm0).cuda(), torch.from_numpy(rm0).cuda())[0] == _oracle_card(g)


def test_cover_rejects_non_maximum():
    g = gg.workload("grid64")
    _, cm0, rm0 = mcm.cheap_init_host(g.colptr, g.rowind, g.nr)
    if (cm0 >= 0).sum() == _oracle_card(g):
        pytest.skip("greedy already maximum")
    dg = mcm.to_device(g)
    with pytest.raises(mcm.McmError) as e:
        mcm.konig_cover(dg, torch.from_numpy(cm0).cuda(), torch.from_numpy(rm0).cuda())
    assert e.value.code == mcm.MCM_ENOTMAX


def test_stats_counters():
    _set(stats=1, wg_threshold=0)
    g = gg.workload("rmat13")
    card, _, _ = _gpu(g, certify=False)
    s = mcm.last_stats()
    assert s["card"] == card and s["phases"] >= 2 and s["levels"] >= s["phases"]
    assert s["edges_scanned"] > 0 and s["rows_found"] >= card - int((O.cheap_init(g)[0] >= 0).sum())


# ------------------------------------------------------------------ batched
def _batch_graphs(n, hi=4096):
    return [gg.batch_member(4, i, hi=hi) for i in range(n)]


@pytest.mark.parametrize("mapping", ["wave", "thread"])
def test_batched_equals_oracle_and_single(mapping):
    _set(mapping=mapping)
    graphs = _batch_graphs(300)
    inits = [mcm.cheap_init_host(g.colptr, g.rowind, g.nr) for g in graphs]
    b = mcm.pack_batch(graphs)
    icm = torch.from_numpy(np.concatenate([x[1] for x in inits])).cuda()
    irm = torch.from_numpy(np.concatenate([x[2] for x in inits])).cuda()
    total, cards, cm, rm = mcm.match_batched(b, icm, irm)
    cmh, rmh = cm.cpu().numpy(), rm.cpu().numpy()
    co = ro = 0
    for i, g in enumerate(graphs):
        ref = _oracle_card(g)
        assert cards[i] == ref, i
        assert O.check_matching(g, cmh[co:co + g.nc], rmh[ro:ro + g.nr]) == ref
        co += g.nc
        ro += g.nr
    assert total == cards.sum()
    # equal to per-graph mcm_match
    for i in range(0, 300, 37):
        g = graphs[i]
        assert _gpu(g, certify=False)[0] == cards[i]


def test_batched_empty_members_and_no_init():
    graphs = [gg.empty(0, 0), gg.complete(3, 4), gg.empty(5, 0), gg.path(9), gg.empty(0, 3), gg.star(6)]
    b = mcm.pack_batch(graphs)
    total, cards, cm, rm = mcm.match_batched(b)
    assert cards.tolist() == [0, 3, 0, 4, 0, 1]
    assert total == 8


# ------------------------------------------------------------------ full-size workloads (as timed by bench.py)
import functools  # noqa: E402

_full_workload = functools.lru_cache(maxsize=2)(gg.workload)  # generating rmat23 takes seconds


def _full_size_card(g, name):
    """The oracle's |M| of a full-size workload, stored by
    tests/golden/make_full_size_cards.py, after checking that the stored
    input is the one generated here (size and FNV-1a hash)."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_size_cards.txt")
    with open(path) as f:
        rows = {ln.split()[0]: ln.split() for ln in f if ln.strip() and not ln.startswith("#")}
    w = rows[name]
    assert (int(w[1]), int(w[2]), int(w[3]), int(w[4], 16)) == (g.nc, g.nr, g.nnz, g.fnv1a()), name
    return int(w[6])


@pytest.mark.parametrize("name", ["grid2048", "rmat23"])
def test_full_size_certified(name):
    """Full size: oracle-free exact certificate.  The output must be a valid
    matching and the GPU's Konig cover (checked by the oracle's verifier)
    proves it maximum by weak duality; for the grid the size must also lie in
    the closed-form window n - |Rdel u Cdel| <= nu <= n - ndel."""
    g = _full_workload(name)
    ref = _full_size_card(g, name)
    card, cm, rm = _gpu(g)
    assert card == ref
    if name == "grid2048":
        n = 2048 * 2048
        nd = int(np.floor(0.03 * n))
        _, dc, dr = gg.grid5(2048, nd, nd, 2, return_masks=True)
        assert n - int((dc | dr).sum()) <= card <= n - nd


@pytest.mark.parametrize("opts", [dict(claim="probe", flush="atomic", local_levels=0),
                                  dict(claim="max", flush="defer", local_levels=0),
                                  dict(claim="probe", flush="defer", local_levels=16),
                                  dict(schedule="async"),
                                  dict(schedule="async", claim="probe", alternate="classic", wr_check="early")],
                         ids=lambda d: "-".join(str(v) for v in d.values()))
@pytest.mark.parametrize("name", ["grid2048", "rmat23"])
def test_full_size_other_forms(name, opts):
    """The full-size workloads with the claim, flush and local-level forms
    that the defaults do not pick for them: a valid matching certified
    maximum by the GPU's Konig cover, the same size as with the defaults."""
    g = _full_workload(name)
    ref = _full_size_card(g, name)
    _set(**opts)
    card, _, _ = _gpu(g)
    assert card == ref, opts


@pytest.mark.parametrize("loop", ["device", "host"])
@pytest.mark.parametrize("name,driver", [("grid256", "apfb"), ("grid256p", "apfb"), ("rmat14", "apsb")])
def test_phase_record(name, driver, loop):
    """The per-phase record of a stats run agrees with the run's own
    counters: as many phases, levels summing to the level count, every phase
    but the last reaching an unmatched row and the last (complete BFS)
    reaching none, at least one end per augmentation; the permuted grid
    reaches the oracle's |M| too."""
    g = gg.workload(name)
    ref = _oracle_card(g)
    _set(wg_threshold=0, loop=loop, driver=driver, stats=1)
    card, _, _ = _gpu(g, certify=False)
    assert card == ref
    st = mcm.last_stats()
    lv, en = mcm.last_phases()
    assert len(lv) == st["phases"] and int(lv.sum()) == st["levels"]
    assert (en[:-1] > 0).all() and en[-1] == 0
    init = mcm.cheap_init_host(g.colptr, g.rowind, g.nr)[0]
    assert int(en.sum()) >= card - init
    # a run without stats keeps no record
    _set(stats=0)
    _gpu(g, certify=False)
    assert len(mcm.last_phases()[0]) == 0


def test_validation_rejects_malformed_colptr_before_the_init_check():
    """With validate=1 a malformed colptr is reported as MCM_EINVAL, and the
    check of the initial matching (which scans column ranges of rowind) is
    not run on it.  Every colptr value stays within [0, nnz], so the
    structural check itself reads only inside the arrays."""
    _set(validate=1)
    g = gg.workload("grid64")
    _, cm0, rm0 = mcm.cheap_init_host(g.colptr, g.rowind, g.nr)
    icm, irm = torch.from_numpy(cm0).cuda(), torch.from_numpy(rm0).cuda()
    ri = torch.from_numpy(g.rowind).cuda()
    c = g.nc // 2
    bad = g.colptr.copy()
    bad[c] = bad[c + 1] + 1                      # colptr[c] > colptr[c + 1]: decreasing
    assert 0 <= bad[c] <= g.nnz
    shifted = g.colptr.copy()
    shifted[0] = 1                               # colptr[0] != 0
    for cp in (bad, shifted):
        dgb = mcm.DeviceGraph(g.nc, g.nr, torch.from_numpy(cp).cuda(), ri)
        for thr in (1 << 30, 0):                 # one-workgroup and persistent paths
            _set(wg_threshold=thr)
            for init in ((icm, irm), (None, None)):
                with pytest.raises(mcm.McmError) as e:
                    mcm.match(dgb, *init)
                assert e.value.code == mcm.MCM_EINVAL
    _set(wg_threshold=16384)
    assert mcm.match(mcm.to_device(g), icm, irm)[0] == _oracle_card(g)


# ------------------------------------------------------------------ rows in any order, duplicates
def _shuffled_with_duplicates(g, seed, dup=0.1):
    """The same pattern with each column's rows shuffled and about `dup` of
    the entries stored twice (at random places of their column)."""
    rng = np.random.default_rng(seed)
    cols = []
    for c in range(g.nc):
        rows = g.rowind[g.colptr[c]:g.colptr[c + 1]].copy()
        if len(rows):
            extra = rows[rng.random(len(rows)) < dup]
            rows = np.concatenate([rows, extra])
            rng.shuffle(rows)
        cols.append(rows)
    colptr = np.zeros(g.nc + 1, np.int32)
    colptr[1:] = np.cumsum([len(r) for r in cols])
    rowind = np.concatenate(cols).astype(np.int32) if g.nnz else np.zeros(0, np.int32)
    return gg.Graph(g.nc, g.nr, colptr, rowind, g.name + "_shuf_dup")


@pytest.mark.parametrize("name", ["uniform2000", "grid128", "rmat13"])
def test_unsorted_rows_and_duplicates(name):
    """include/mcm.h allows rows of a column in any order and duplicated:
    every launch form (one workgroup, persistent device loop with either row
    claim, host loop, batched, the multi-graph launch) reaches the oracle's
    |M| on such input, with a valid matching certified by the Konig cover."""
    g0 = gg.workload(name)
    g = _shuffled_with_duplicates(g0, 11)
    assert g.nnz > g0.nnz and O.check_csc(g)
    ref = _oracle_card(g)
    assert ref == _oracle_card(g0)                # the same graph
    forms = [dict(wg_threshold=1 << 30), dict(wg_threshold=0, loop="device", claim="max"),
             dict(wg_threshold=0, loop="device", claim="probe", flush="atomic"),
             dict(wg_threshold=0, loop="host"), dict(wg_threshold=0, loop="device", alternate="classic")]
    for f in forms:
        _set(**f)
        for init in ("cheap", "empty"):
            assert _gpu(g, init)[0] == (ref if init == "cheap" else _oracle_card(g, "empty")), (f, init)
        for k, v in DEFAULTS.items():
            mcm.set_option(k, v)
    # batched: the graph twice, once through the workgroup kernel and once
    # through the multi-graph launch
    b = mcm.pack_batch([g, g0])
    for thr in (1 << 40, 1):
        _set(multi_threshold=thr)
        total, cards, cm, rm = mcm.match_batched(b)
        assert cards.tolist() == [_oracle_card(g, "empty")] * 2
        assert O.check_matching(g, cm[:g.nc].cpu().numpy(), rm[:g.nr].cpu().numpy()) == cards[0]
    _set(multi_threshold=1 << 15)


def test_two_streams_two_threads_small_graphs():
    """Calls on different streams use separate workspaces and may overlap:
    two host threads, each on its own stream, match small graphs (the
    one-workgroup kernel, not a cooperative launch) over and over; every
    result equals the oracle's."""
    import threading
    graphs = [gg.uniform(900, 1000, 3, 40 + i) for i in range(6)]
    refs = [_oracle_card(g) for g in graphs]
    dgs = [mcm.to_device(g) for g in graphs]
    inits = [mcm.cheap_init_host(g.colptr, g.rowind, g.nr) for g in graphs]
    inits = [(torch.from_numpy(c).cuda(), torch.from_numpy(r).cuda()) for _, c, r in inits]
    errors = []

    def worker(k):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for it in range(25):
                    i = (k + it) % len(graphs)
                    card, cm, rm = mcm.match(dgs[i], *inits[i], stream=s)
                    if card != refs[i]:
                        errors.append((k, it, i, card, refs[i]))
                    s.synchronize()
                    if O.check_matching(graphs[i], cm.cpu().numpy(), rm.cpu().numpy()) != card:
                        errors.append((k, it, i, "invalid"))
        except Exception as e:  # noqa: BLE001
            errors.append((k, repr(e)))

    th = [threading.Thread(target=worker, args=(k,)) for k in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors[:5]
