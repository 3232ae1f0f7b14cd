"""The continuous-batching server through the C ABI.  Every served result is
checked against the CPU oracle: exact cardinality, valid matching; the same
request gives the same cardinality alone and in a mix (the matching arrays
may differ: maximum matchings are not unique)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_1303_1379_amd import graphgen as gg, mcm, serving  # noqa: E402


@pytest.fixture(autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    yield


def _ref(g):
    return O.hopcroft_karp(g, *O.cheap_init(g))[0]


def _graphs():
    gs = [gg.uniform(3000, 2500, 4, 11), gg.grid5(96, 200, 150, 3), gg.rmat(13, 8 << 13, 12, n_limit=6000),
          gg.batch_member(4, 7, hi=20000), gg.uniform(1200, 1800, 2, 13), gg.permutation_plus_noise(2000, 2, 5),
          gg.uniform(70000, 70000, 4, 21)]   # above the batched-path size: multi-graph persistent launch
    return gs


def _served(server, g):
    t = server.submit(g)
    res = server.poll(t, wait_ms=60000)
    assert res is not None
    return res


def test_alone_equals_mix_equals_oracle():
    gs = _graphs()
    refs = [_ref(g) for g in gs]
    s = mcm.Server(2 << 30, max_batch=256)
    alone = []
    for g, ref in zip(gs, refs):
        card, info, cm, rm = _served(s, g)
        assert card == ref
        assert O.check_matching(g, cm, rm) == card
        alone.append(card)
        assert info["path"] == (1 if g.nc + g.nr > (1 << 15) else 0)
    # the same requests, three copies each, submitted together
    tickets = [(i, s.submit(gs[i])) for _ in range(3) for i in range(len(gs))]
    for i, t in tickets:
        res = s.poll(t, wait_ms=60000)
        assert res is not None
        card, info, cm, rm = res
        assert card == alone[i] == refs[i]
        assert O.check_matching(gs[i], cm, rm) == card
        assert info["path"] == (1 if gs[i].nc + gs[i].nr > (1 << 15) else 0)
        assert 1 <= info["batch_size"] <= (64 if info["path"] == 1 else 256)
    st = s.stats()
    assert st["completed"] == st["submitted"] == len(gs) * 4
    assert st["launches_grid"] >= 2 and st["max_batch_seen"] >= 2
    s.close()


def test_large_requests_share_multi_graph_launches():
    """Several large requests in flight together: every result exact, and
    the multi-graph launches together carry all of them."""
    gs = [gg.uniform(20000 + 1000 * k, 19000, 3, 40 + k) for k in range(6)]
    refs = [_ref(g) for g in gs]
    s = mcm.Server(2 << 30, max_batch=64)
    tickets = [s.submit(g) for g in gs for _ in range(2)]
    for k, t in enumerate(tickets):
        card, info, cm, rm = s.poll(t, wait_ms=60000)
        assert card == refs[k // 2]
        assert O.check_matching(gs[k // 2], cm, rm) == card
        assert info["path"] == 1
        assert 1 <= info["batch_size"] <= 64  # large requests per multi-graph launch, at most
    st = s.stats()
    assert st["launches_grid"] <= len(tickets) and st["completed"] == len(tickets)
    s.close()


def test_budget_admission_and_rejection():
    g = gg.uniform(20000, 20000, 6, 3)
    ref = _ref(g)
    per = 4 * (g.nc + 1) + 4 * g.nnz + 12 * g.nc + 28 * g.nr + 32 * g.nc + 4096
    budget = int(2.5 * per)   # about two requests at a time
    s = mcm.Server(budget, max_batch=64)
    ts = [s.submit(g) for _ in range(12)]
    for t in ts:
        card, info, cm, rm = s.poll(t, wait_ms=60000)
        assert card == ref
    st = s.stats()
    assert st["peak_bytes"] <= budget and st["bytes_in_use"] == 0
    big = gg.uniform(60000, 60000, 8, 4)
    with pytest.raises(mcm.McmError) as e:
        s.submit(big)
    assert e.value.code == mcm.MCM_ENOMEM
    assert s.stats()["rejected"] == 1
    s.close()


def test_empty_requests():
    s = mcm.Server(1 << 26)
    for nc, nr in [(0, 0), (5, 0), (0, 4), (6, 3)]:
        card, info, cm, rm = _served(s, gg.empty(nc, nr))
        assert card == 0 and (cm == -1).all() and (rm == -1).all()
    s.close()


def test_poisson_replay_checks_every_result():
    pool = serving.make_pool(16, seed=9, lo=1000, hi=30000)
    refs = [_ref(g) for g, _, _ in pool]
    seen = []

    def check(k, card, cm, rm):
        g = pool[k][0]
        assert card == refs[k]
        assert O.check_matching(g, cm, rm) == card
        seen.append(k)

    s = mcm.Server(1 << 30, max_batch=512)
    r = serving.replay(s, pool, 400, lam=2000.0, seed=3, warmup=50, check=check)
    assert len(seen) == 400
    assert r["p50_ms"] > 0 and r["p99_ms"] >= r["p50_ms"] and r["graphs_per_s"] > 0
    s.close()
