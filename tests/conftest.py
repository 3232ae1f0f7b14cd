import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built libmcm.so")
    config.addinivalue_line("markers", "slow: larger CPU cases")


@pytest.fixture(scope="session", autouse=True)
def _native_libs():
    """Build the CPU-side libraries if they are missing (the HIP library is
    built by __graft_entry__.build(); GPU tests fail loudly without it)."""
    from paper_1303_1379_amd import _build
    import oracle
    if not os.path.exists(_build.GEN_LIB):
        _build.build_gen()
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        oracle.build()
    yield


def load_golden(name):
    """Parse a tests/golden/*.txt fixture into a dict."""
    path = os.path.join(ROOT, "tests", "golden", name)
    d = {"edges": [], "match": []}
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, *vals = line.split()
            vals = [int(v) for v in vals]
            if key == "edge":
                d["edges"].append(tuple(vals))
            elif key == "match":
                d["match"].append(tuple(vals))
            elif len(vals) == 1 and key in ("nc", "nr", "expect_card", "expect_free_reached"):
                d[key] = vals[0]
            else:
                d[key] = vals
    return d
