"""mcm_match_noalloc through the C ABI: the entry point for callers that
cannot allocate, whose match state lives in the library's fixed device array.
Its results must meet the bar of mcm_match on the same inputs: the same
cardinality (which is the oracle's), a valid matching, and a Konig cover of
that size.  Calls follow each other on the one array, each smaller than the
one before (whatever a call leaves behind must not reach the next), across
the persistent multi-workgroup path (skewed and low-degree forms) and the
one-workgroup path; a graph whose state does not fit is refused before any
launch."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_1303_1379_amd import graphgen as gg, mcm  # noqa: E402

# largest first: each call runs on what the previous, larger one left in the array
SEQUENCE = ["rmat16", "grid256p", "grid128", "uniform2000"]


@pytest.fixture(autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    yield


def _check(g, dg, card, cm, rm, expect):
    assert card == expect, (g.name, card, expect)
    cmh, rmh = cm.cpu().numpy(), rm.cpu().numpy()
    assert O.check_matching(g, cmh, rmh) == card, g.name
    k, cc, rc = mcm.konig_cover(dg, cm, rm)
    assert k == card, g.name
    assert O.verify_cover(g, cmh, rmh, cc.cpu().numpy(), rc.cpu().numpy()) == 0, g.name


def test_noalloc_matches_like_mcm_match_on_calls_in_a_row():
    for round_ in range(2):  # the whole sequence twice: the second pass starts on the first's leftovers
        for name in SEQUENCE:
            g = gg.workload(name)
            cm0, rm0 = O.cheap_init(g)
            ref = O.hopcroft_karp(g, cm0, rm0)[0]
            dg = mcm.to_device(g)
            icm, irm = torch.from_numpy(cm0).cuda(), torch.from_numpy(rm0).cuda()
            card_m, cm_m, rm_m = mcm.match(dg, icm, irm)
            _check(g, dg, card_m, cm_m, rm_m, ref)
            ocm = torch.full((g.nc,), 7, dtype=torch.int32, device="cuda")
            orm = torch.full((g.nr,), 7, dtype=torch.int32, device="cuda")
            card = mcm.match_noalloc(dg, icm, irm, ocm, orm)
            _check(g, dg, card, ocm, orm, card_m)
            assert mcm.last_stats()["card"] == card
            # from the empty matching, outputs in place of the inputs
            ecm = torch.full((g.nc,), -1, dtype=torch.int32, device="cuda")
            erm = torch.full((g.nr,), -1, dtype=torch.int32, device="cuda")
            card_e = mcm.match_noalloc(dg, ecm, erm, ecm, erm)
            _check(g, dg, card_e, ecm, erm, ref)


def test_noalloc_refuses_a_graph_beyond_its_array_and_keeps_working():
    n = 1 << 22  # 4M columns and rows: about 300 MB of state, far beyond 64 MiB
    colptr = torch.zeros(n + 1, dtype=torch.int32, device="cuda")
    colptr[1:] = 1
    rowind = torch.zeros(1, dtype=torch.int32, device="cuda")
    dg = mcm.DeviceGraph(colptr=colptr, rowind=rowind, nc=n, nr=n)
    ocm = torch.empty(n, dtype=torch.int32, device="cuda")
    orm = torch.empty(n, dtype=torch.int32, device="cuda")
    with pytest.raises(mcm.McmError) as e:
        mcm.match_noalloc(dg, None, None, ocm, orm)
    assert e.value.code == mcm.MCM_ENOMEM
    assert "needs" in str(e.value) and "bytes" in str(e.value)
    # a call after the refusal is unaffected
    g = gg.workload("grid128")
    cm0, rm0 = O.cheap_init(g)
    dg = mcm.to_device(g)
    ocm = torch.empty(g.nc, dtype=torch.int32, device="cuda")
    orm = torch.empty(g.nr, dtype=torch.int32, device="cuda")
    card = mcm.match_noalloc(dg, torch.from_numpy(cm0).cuda(), torch.from_numpy(rm0).cuda(), ocm, orm)
    _check(g, dg, card, ocm, orm, O.hopcroft_karp(g, cm0, rm0)[0])


def test_noalloc_empty_graphs():
    for nc, nr in [(5, 0), (0, 4), (6, 3)]:
        g = gg.empty(nc, nr)
        dg = mcm.to_device(g)
        ocm = torch.full((max(nc, 1),), 9, dtype=torch.int32, device="cuda")[:nc]
        orm = torch.full((max(nr, 1),), 9, dtype=torch.int32, device="cuda")[:nr]
        card = mcm.match_noalloc(dg, None, None, ocm, orm)
        assert card == 0
        assert (ocm.cpu().numpy() == -1).all() and (orm.cpu().numpy() == -1).all()
