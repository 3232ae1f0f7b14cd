"""Batched matching through the C ABI: captured batch plans, the autotuner,
and the device-side cheap initial matching, all checked against the CPU
oracle (exact cardinalities, valid matchings)."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_1303_1379_amd import graphgen as gg, mcm  # noqa: E402


@pytest.fixture(autouse=True)
def _reset():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    defaults = dict(mapping="auto", autotune=0, tuning="", stats=0, wg_block=1024, batch_min=8,
                    multi_threshold=1 << 15, multi_group=0)
    for k, v in defaults.items():
        mcm.set_option(k, v)
    yield
    for k, v in defaults.items():
        mcm.set_option(k, v)


def _batch(n, hi=4096, seed=4):
    graphs = [gg.batch_member(seed, i, hi=hi) for i in range(n)]
    inits = [mcm.cheap_init_host(g.colptr, g.rowind, g.nr) for g in graphs]
    b = mcm.pack_batch(graphs)
    icm = torch.from_numpy(np.concatenate([x[1] for x in inits])).cuda()
    irm = torch.from_numpy(np.concatenate([x[2] for x in inits])).cuda()
    refs = [O.hopcroft_karp(g, *O.cheap_init(g))[0] for g in graphs]
    return graphs, b, icm, irm, refs


def _check_outputs(graphs, cm, rm, cards):
    cmh, rmh = cm.cpu().numpy(), rm.cpu().numpy()
    co = ro = 0
    for i, g in enumerate(graphs):
        assert O.check_matching(g, cmh[co:co + g.nc], rmh[ro:ro + g.nr]) == cards[i], i
        co += g.nc
        ro += g.nr


def test_plan_replays_match_eager_and_oracle():
    graphs, b, icm, irm, refs = _batch(160)
    total_e, cards_e, cm_e, rm_e = mcm.match_batched(b, icm, irm)
    assert cards_e.tolist() == refs
    plan = mcm.BatchPlan(b, icm, irm)
    single = gg.workload("grid128")
    dgs = mcm.to_device(single)
    for rep in range(4):
        total, cards = plan.run()
        torch.cuda.synchronize()
        assert total == total_e and cards.tolist() == refs, rep
        _check_outputs(graphs, plan.out_cmatch, plan.out_rmatch, cards)
        # the program's own eager work between replays
        mcm.match(dgs)
        mcm.match_batched(b, icm, irm)
        torch.cuda.synchronize()
    info = plan.info()
    assert info["ngraphs"] == 160 and info["mapping"] in ("wave", "thread")
    plan.close()


def test_plan_sees_new_contents_of_bound_arrays():
    graphs, b, icm, irm, refs = _batch(40)
    init_c = icm.clone()
    init_r = irm.clone()
    plan = mcm.BatchPlan(b, init_c, init_r)
    assert plan.run()[1].tolist() == refs
    # empty initial matching written into the bound arrays: same maximum
    init_c.fill_(-1)
    init_r.fill_(-1)
    torch.cuda.synchronize()
    total, cards = plan.run()
    assert cards.tolist() == refs
    _check_outputs(graphs, plan.out_cmatch, plan.out_rmatch, cards)
    plan.close()


def test_autotune_picks_a_candidate_and_caches_it(tmp_path):
    path = str(tmp_path / "tune.jsonl")
    mcm.set_option("tuning", path)
    mcm.set_option("autotune", 1)
    graphs, b, icm, irm, refs = _batch(96)
    plan = mcm.BatchPlan(b, icm, irm)
    info = plan.info()
    assert info["tuned"] and info["tuned_ms"] > 0
    assert info["block"] in (256, 512, 1024) and info["batch_min"] in (1, 8, 32)
    assert plan.run()[1].tolist() == refs
    plan.close()
    lines = [json.loads(x) for x in open(path).read().splitlines() if x.strip()]
    assert any(x["key"] == info["key"] for x in lines)
    # a later plan of the same size class reuses the cached choice without timing
    mcm.set_option("autotune", 0)
    plan2 = mcm.BatchPlan(b, icm, irm)
    i2 = plan2.info()
    assert i2["tuned"] and i2["block"] == info["block"] and i2["mapping"] == info["mapping"]
    assert plan2.run()[1].tolist() == refs
    plan2.close()
    # one-shot batched matching also picks up the cached configuration
    assert mcm.match_batched(b, icm, irm)[1].tolist() == refs


@pytest.mark.parametrize("name", ["uniform2000", "grid128", "rmat14"])
def test_device_cheap_init_is_maximal(name):
    g = gg.workload(name)
    dg = mcm.to_device(g)
    card0, cm, rm = mcm.cheap_init(dg)
    cmh, rmh = cm.cpu().numpy(), rm.cpu().numpy()
    assert O.check_matching(g, cmh, rmh) == card0
    cols, rows = g.edges()
    assert not np.any((cmh[cols] == -1) & (rmh[rows] == -1)), "not maximal"
    card, _, _ = mcm.match(dg, cm, rm)
    assert card == O.hopcroft_karp(g, *O.cheap_init(g))[0]


@pytest.mark.parametrize("group", [0, 8])
def test_large_members_in_multi_graph_launches(group):
    """Members above the size threshold go to groups of blocks, several per
    cooperative launch (group 8: all of them in one launch; default group:
    several launches); small members share the workgroup kernel.  Includes
    large degenerate members: no rows, no edges."""
    graphs = [gg.uniform(30000, 28000, 4, 31), gg.batch_member(5, 0, hi=3000), gg.grid5(200, 120, 100, 7),
              gg.empty(40000, 0), gg.uniform(20000, 20000, 3, 32), gg.batch_member(5, 1, hi=3000),
              gg.rmat(15, 8 << 15, 33, n_limit=30000), gg.empty(20000, 20000), gg.uniform(17000, 16000, 2, 34),
              gg.permutation_plus_noise(18000, 3, 35), gg.batch_member(5, 2, hi=3000)]
    big = [g.nc + g.nr > (1 << 15) for g in graphs]
    assert sum(big) >= 6 and not all(big)
    refs = [O.hopcroft_karp(g, *O.cheap_init(g))[0] for g in graphs]
    b = mcm.pack_batch(graphs)
    mcm.set_option("multi_group", group)
    total, cards, cm, rm = mcm.match_batched(b)
    torch.cuda.synchronize()
    assert cards.tolist() == refs and total == sum(refs)
    _check_outputs(graphs, cm, rm, cards)
    # the same batch with every member on the workgroup kernel, twice in a row
    mcm.set_option("multi_threshold", 0)
    for _ in range(2):
        total0, cards0, cm0, rm0 = mcm.match_batched(b)
        assert cards0.tolist() == refs
    _check_outputs(graphs, cm0, rm0, cards0)


@pytest.mark.parametrize("barrier", ["counter", "flags"])
def test_multi_graph_queue_runs_several_graphs_per_group(barrier):
    """More large members than block groups: every group takes graph after
    graph from the launch's queue (4 groups of 64 blocks, 22 large graphs of
    both kinds, plus degenerate ones), continuing its barrier epochs across
    graphs; every result equals the oracle's."""
    graphs = [gg.uniform(18000 + 500 * k, 17000 + 300 * k, 3 + k % 3, 60 + k) for k in range(16)]
    graphs += [gg.rmat(15, 6 << 15, 70 + k, n_limit=20000 + 1000 * k) for k in range(4)]
    graphs += [gg.empty(40000, 0), gg.empty(20000, 20000), gg.grid5(150, 600, 600, 9)]
    assert sum(g.nc + g.nr > (1 << 15) for g in graphs) >= 22
    refs = [O.hopcroft_karp(g, *O.cheap_init(g))[0] for g in graphs]
    b = mcm.pack_batch(graphs)
    mcm.set_option("multi_group", 64)
    mcm.set_option("barrier", barrier)
    try:
        for _ in range(2):
            total, cards, cm, rm = mcm.match_batched(b)
            torch.cuda.synchronize()
            assert cards.tolist() == refs
            _check_outputs(graphs, cm, rm, cards)
    finally:
        mcm.set_option("barrier", "counter")
