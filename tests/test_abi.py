"""The C ABI library without a GPU: it loads, exports every symbol that
include/mcm.h declares, validates options and arguments before touching the
device, and its host-side greedy initial matching follows the definition."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_1303_1379_amd import graphgen as gg, mcm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "mcm.h")).read()
    return sorted(set(re.findall(r"\b(mcm_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = mcm.lib()
    decl = _declared()
    assert set(decl) == set(mcm.EXPORTS)
    for name in decl:
        assert getattr(L, name) is not None


def test_version_and_strerror():
    assert mcm.version().startswith("mcm-gfx950")
    L = mcm.lib()
    for code in (-1, -2, -3, -4, -5, -6):
        assert L.mcm_strerror(code)


def test_options_roundtrip_and_rejects():
    for k, v in [("driver", "apsb"), ("bfs", "plain"), ("mapping", "thread"), ("loop", "host"),
                 ("validate", "1"), ("stats", "1"), ("block", "512"), ("wg_threshold", "100"),
                 ("level_entries", "0"), ("idle_sleep", "32"), ("wr_check", "early"), ("wr_check", "late"), ("multi_threshold", "0"),
                 ("multi_group", "8"), ("max_blocks", "32"), ("endpoints", "one"), ("barrier", "counter"),
                 ("claim", "max"), ("claim", "probe"), ("flush", "atomic"), ("flush", "defer"),
                 ("local_levels", "2"), ("local_levels", "auto"), ("local_edges", "0"), ("local_edges", "64"), ("wg_lds", "off"), ("wg_lds", "on"), ("fuse", "off"), ("fuse", "on"), ("alternate", "classic"), ("alternate", "fast"), ("roots", "list"), ("fix", "scan"), ("schedule", "async")]:
        old = mcm.get_option(k)
        mcm.set_option(k, v)
        assert mcm.get_option(k) == v
        mcm.set_option(k, old)
    for k, v in [("driver", "x"), ("bfs", "fast"), ("block", "65"), ("nope", "1"), ("validate", "2"),
                 ("level_entries", "-1"), ("idle_sleep", "5000"), ("wr_check", "soon"), ("multi_group", "4096"),
                 ("endpoints", "two"), ("barrier", "tree"), ("claim", "cas"), ("flush", "later"), ("local_levels", "17"), ("alternate", "slow"), ("local_edges", "-1"), ("wg_lds", "auto"), ("fuse", "1")]:
        with pytest.raises(mcm.McmError) as e:
            mcm.set_option(k, v)
        assert e.value.code == mcm.MCM_EINVAL


def test_argument_errors_before_device_work():
    L = mcm.lib()
    # negative sizes
    assert L.mcm_match(-1, 3, None, None, None, None, None, None, None) == mcm.MCM_EINVAL
    # exactly one init array given
    buf = (ctypes.c_int32 * 8)()
    p = ctypes.cast(buf, ctypes.c_void_p)
    assert L.mcm_match(2, 2, p, p, p, None, p, p, None) == mcm.MCM_EINVAL
    assert b"both" in L.mcm_strerror(-1)
    # NULL outputs
    assert L.mcm_match(2, 2, p, p, None, None, None, p, None) == mcm.MCM_EINVAL
    assert L.mcm_match_batched(-1, None, None, None, None, None, None, None, None, None) == mcm.MCM_EINVAL
    assert L.mcm_match_batched(0, None, None, None, None, None, None, None, None, None) == 0
    assert L.mcm_konig_cover(-2, 1, None, None, None, None, None, None, None) == mcm.MCM_EINVAL


@pytest.mark.parametrize("name", ["uniform2000", "grid64", "rmat12"])
def test_host_cheap_init_equals_definition(name):
    """The library's host greedy and the oracle's are separate code; both
    follow the same definition, so their outputs are identical."""
    g = gg.workload(name)
    card, cm, rm = mcm.cheap_init_host(g.colptr, g.rowind, g.nr)
    ocm, orm = O.cheap_init(g)
    assert (cm == ocm).all() and (rm == orm).all()
    assert card == int((ocm >= 0).sum())


def test_host_cheap_init_rejects_bad_csc():
    cp = np.array([0, 2, 1], np.int32)
    ri = np.array([0, 1], np.int32)
    with pytest.raises(mcm.McmError):
        mcm.cheap_init_host(cp, ri, 2)
    with pytest.raises(mcm.McmError):
        mcm.cheap_init_host(np.array([0, 1], np.int32), np.array([5], np.int32), 2)
