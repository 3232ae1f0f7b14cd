#!/usr/bin/env python3
"""Writes tests/golden/full_size_cards.txt: the oracle's maximum cardinality
of the full-size workloads (Hopcroft-Karp from the greedy initial matching),
with each input's size and FNV-1a hash so that a test can check that it
regenerated the same graph.  Calls only the oracle (and the seeded input
generators); nothing here runs on, or comes from, the GPU path.

    python tests/golden/make_full_size_cards.py [workload ...]
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1303_1379_amd import graphgen as gg  # noqa: E402

OUT = os.path.join(HERE, "full_size_cards.txt")


def main(names):
    lines = ["# workload nc nr nnz fnv1a init_card card hk_phases   (oracle: greedy init, then Hopcroft-Karp)"]
    for name in names:
        g = gg.workload(name)
        cm, rm = oracle.cheap_init(g)
        t0 = time.time()
        card, _, _, phases = oracle.hopcroft_karp(g, cm, rm)
        print(f"{name}: |M| = {card} in {time.time() - t0:.1f} s", flush=True)
        lines.append(f"{name} {g.nc} {g.nr} {g.nnz} {g.fnv1a():#018x} {int((cm >= 0).sum())} {card} {phases}")
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main(sys.argv[1:] or ["uniform2000", "grid2048", "grid2048p", "rmat23"])
