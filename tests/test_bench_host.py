"""Host-side pieces of bench.py (no GPU): the oracle legs and the roofline's
profile lookup."""
import importlib.util
import os

import pytest

import oracle as O
from paper_1303_1379_amd import graphgen as gg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_oracle_batch_leg(bench):
    graphs = [gg.batch_member(4, i) for i in range(40)]
    cards = [O.hopcroft_karp(g, *O.cheap_init(g))[0] for g in graphs]
    r = bench.oracle_batch(graphs, cards, 5.0)
    assert r["kind"] == "oracle" and r["unit"] == "graphs/s" and r["cores"] >= 1
    assert r["identical_cardinalities"] is True and r["value"] > 0
    # a wrong expected size is reported, not hidden
    bad = list(cards)
    bad[3] += 1
    assert bench.oracle_batch(graphs, bad, 5.0)["identical_cardinalities"] is False


def test_cpu_baseline_leg(bench):
    g = gg.workload("uniform2000")
    r = bench.cpu_baseline(g, 2.0)
    assert r["kind"] == "oracle" and r["cores"] == 1 and r["value"] > 0
    m = bench.cpu_model()
    assert m is None or isinstance(m, str)
    # to the maximum: the oracle's own result, its edges read, graph edges per second
    full = bench.cpu_baseline(g)
    card, _, _, phases, edges = O.hopcroft_karp_ex(g, *O.cheap_init(g))
    assert full["complete"] and full["card"] == card and full["phases"] == phases
    assert full["graph_teps"] > 0 and str(edges) in full["sample"]


def test_alg_bytes_model(bench):
    s = dict(edges_scanned=10, cols_expanded=3, cols_claimed=2, rows_found=1, alt_steps=4, roots=5, pass_bytes=100)
    assert bench.alg_bytes(s) == 8 * 10 + 16 * 3 + 16 * 2 + 12 + 20 * 4 + 4 * 5 + 100
    r = bench.roofline(8e9, 0.5, "k")
    assert r["achieved"] == 16.0 and r["frac"] == round(16.0 / 8000.0, 5) and r["bound"] == "hbm"


def test_traffic_profile_lookup(bench):
    # the committed summaries are read only when taken on the current kernel sources
    for wl in ("grid2048", "rmat23"):
        path = os.path.join(ROOT, "profiles", f"k_persistent_{wl}_traffic.txt")
        assert os.path.exists(path)
        with open(path) as f:
            text = f.read()
        current = f"kernel_source_hash: {bench.kernel_source_hash()}" in text
        t = bench.load_traffic(wl)
        assert (t is not None) == current
        if t is not None:
            assert t > 0
    assert bench.load_traffic("no-such-workload") is None


def test_batched_traffic_lookup(bench):
    # the batch summary is read only for the kernel instance and launch shape
    # it was taken on (mapping, block, blocks), whatever the plan's batch_min
    path = os.path.join(ROOT, "profiles", "k_match_wg_batched_traffic.txt")
    assert os.path.exists(path)
    with open(path) as f:
        text = f.read()
    current = f"kernel_source_hash: {bench.kernel_source_hash()}" in text
    shape = dict(mapping="wave", block=1024, blocks=256)
    assert f"plan_config: {bench.plan_config(dict(shape, batch_min=1))}" in text
    for bm in (1, 32):
        t = bench.load_traffic("batched", "k_match_wg", bench.plan_config(dict(shape, batch_min=bm)))
        assert (t is not None) == current
    for other in (dict(shape, mapping="thread"), dict(shape, block=512), dict(shape, blocks=128)):
        assert bench.load_traffic("batched", "k_match_wg", bench.plan_config(dict(other, batch_min=32))) is None
