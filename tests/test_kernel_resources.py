"""Register budget of the launches whose workgroups must all be resident at
once (cooperative launches that spin at grid barriers): compiled for gfx950,
they stay within the 128 registers per lane of a 1024-thread workgroup and
do not spill.  The single-graph kernel with the wave mapping sits at the
limit: a per-lane address into the list of augmenting-path ends, once kept
live through its whole phase loop, spilled until Alternate took that list
through a pointer the compiler cannot hoist.  The multi-graph
kernel sits close to the limit, and small additions have pushed it over
before.  No GPU needed: hipcc reports each kernel's resources at compile
time."""
import os
import re
import shutil
import subprocess

import pytest

from paper_1303_1379_amd import _build

COOPERATIVE = ("k_persistent_multi", "k_persistent")


def _resources():
    hipcc = _build.HIPCC
    if not (os.path.exists(hipcc) or shutil.which(hipcc)):
        pytest.skip("hipcc not available")
    out = os.path.join(_build.BUILD_DIR, "resources_check.o")
    os.makedirs(_build.BUILD_DIR, exist_ok=True)
    cmd = [hipcc] + _build.HIP_FLAGS + ["-c", os.path.join(_build.CSRC, "mcm_kernels.hip"), "-o", out,
                                        "-Rpass-analysis=kernel-resource-usage"]
    res = subprocess.run(cmd, capture_output=True, text=True, check=True)
    kernels, cur = {}, None
    for line in res.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            kernels[cur] = {}
            continue
        m = re.search(r"(VGPRs|ScratchSize \[bytes/lane\]): (\d+)", line)
        if m and cur:
            kernels[cur][m.group(1).split()[0]] = int(m.group(2))
    os.remove(out)
    return kernels


def test_cooperative_kernels_do_not_spill():
    kernels = _resources()
    coop = {k: v for k, v in kernels.items() if any(f"{n}I" in k for n in COOPERATIVE)}
    assert len(coop) >= 4, sorted(kernels)          # both mappings of both persistent kernels
    for name, r in coop.items():
        assert r.get("ScratchSize", 0) == 0, (name, r)
        assert r.get("VGPRs", 0) <= 128, (name, r)
