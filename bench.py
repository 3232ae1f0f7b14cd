#!/usr/bin/env python3
"""Benchmark: maximum-cardinality matching on one MI355X through libmcm.

One step = one mcm_match call on the headline workload (copy of the greedy
initial matching into the working state, all phases of APFB with
GPUBFS-WR, Alternate and FixMatching, unpack and count, stream
synchronised), with the graph and the initial matching already resident in
HBM.  The headline workload is the largest single graph of the suite that
fits one GPU: R-MAT at scale 23 (2^23 rows and columns, about 131 M
entries after duplicates are removed).

Prints ONE JSON line.  `value` is edges scanned per second (scanned edges
of the step counted by the library's device counters in an untimed run,
divided by the measured time per step).  `roofline` relates the
algorithmic bytes of the persistent matching kernel (fixed per-unit byte
model: 8 B per scanned edge, 16 B per expanded and per claimed column, 12 B
per unmatched row found, 20 B per Alternate step, 4 B per root, and the
per-phase passes: 4 B and 1/8 B per column the root scan reads, 8 B per row
FixMatching reads) to its average duration from HIP events over the timed
steps.  `cpu_baseline` is the CPU oracle (Hopcroft-Karp, one thread) run
to the maximum on the same input from the same greedy matching.

Further sections: `grid2048` (the mesh-like graph, its own roofline),
`uniform2000` (microseconds per match, median of 1000), `batched` (4096
uneven graphs in one captured launch vs a per-graph loop, with the
kernel's roofline).  With --serving also `serving` (Poisson arrivals
through the continuous-batching server: latency from the scheduled arrival,
capacity, and a per-request mcm_match loop over the same graphs); it is
not part of the default run.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Matching time & edges scanned/s (%HBM peak); batched graphs/s vs per-graph loop"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "grid2048": "5-point grid pattern on a 2048x2048 grid (4,194,304 rows and columns), 3% of columns and "
                "3% of rows emptied at random (seed 2), int32 CSC, greedy initial matching",
    "rmat23": "R-MAT (a=.57, b=.19, c=.19, d=.05), 2^23 rows x 2^23 columns, 16 samples per column, duplicates "
              "removed, random row/column permutation (seed 3), int32 CSC, greedy initial matching",
    "uniform2000": "2000 x 2000 uniform random bipartite graph, 4 row draws per column (seed 1), duplicates "
                   "removed, int32 CSC, greedy initial matching",
    "grid2048p": "grid2048 under a random row and column permutation (seed 7), int32 CSC, greedy initial matching",
}


def alg_bytes(s):
    """Algorithmic bytes of one match (or batch) from its device counters (see module doc)."""
    return (8 * s["edges_scanned"] + 16 * s["cols_expanded"] + 16 * s["cols_claimed"] + 12 * s["rows_found"]
            + 20 * s["alt_steps"] + 4 * s["roots"] + s["pass_bytes"])


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("mcm_kernels.hip", "mcm_internal.h"):
        with open(os.path.join(ROOT, "paper_1303_1379_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload, kernel="k_persistent", plan_config=None):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 counter summary (lines "key: value"), or None when missing,
    taken on other kernel sources, or (batched plans) on another launch
    configuration than `plan_config`."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    d = {}
    with open(path) as f:
        for line in f:
            k, sep, v = line.partition(":")
            if sep:
                d[k.strip()] = v.strip()
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    if plan_config is not None and d.get("plan_config") != plan_config:
        return None
    try:
        return float(d["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model():
    """Host CPU model name (from /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(g, budget_s=None):
    """The oracle (Hopcroft-Karp, one thread) on the same input from the same
    greedy matching: to the maximum (budget_s None), or phase by phase until
    budget_s seconds are spent.  Reported in its own edges scanned per
    second, and in graph edges per second (nnz / time) beside the GPU's."""
    import oracle
    cm0, rm0 = oracle.cheap_init(g)
    if budget_s is None:
        t0 = time.perf_counter()
        card, _, _, phases, edges = oracle.hopcroft_karp_ex(g, cm0, rm0)
        secs = time.perf_counter() - t0
        done = True
    else:
        smp = oracle.hopcroft_karp_sample(g, cm0, rm0, budget_s)
        card, phases, edges, secs, done = smp["card"], smp["phases"], smp["edges"], smp["seconds"], smp["done"]
    what = "complete run to the maximum" if done else f"first {phases} phases"
    return {"value": round(edges / secs, 1) if secs > 0 else None, "unit": "edges scanned/s", "cores": 1,
            "kind": "oracle",
            "sample": f"Hopcroft-Karp (single thread) on the same input from the same greedy matching, {what}: "
                      f"{edges} edges scanned in {secs:.2f} s",
            "phases": phases, "seconds": round(secs, 3), "card": int(card), "complete": bool(done),
            "graph_teps": round(g.nnz / secs, 1) if done and secs > 0 else None}


def oracle_batch(graphs, gpu_cards, budget_s):
    """The oracle over the batch on the host's cores: graphs in batch order,
    one thread per core (the C oracle runs without the interpreter lock), each
    from its own greedy matching (computed first, untimed, as for the GPU), in
    chunks until the time budget is spent; graphs per second over the graphs
    done, and whether their cardinalities equal the batched launch's."""
    import concurrent.futures as cf
    import oracle
    threads = max(1, min(os.cpu_count() or 1, 16))
    done, same, busy = 0, True, 0.0
    with cf.ThreadPoolExecutor(threads) as ex:
        while done < len(graphs) and busy < budget_s:
            chunk = graphs[done:done + 4 * threads]
            inits = list(ex.map(oracle.cheap_init, chunk))
            t0 = time.perf_counter()
            cards = list(ex.map(lambda a: oracle.hopcroft_karp(a[0], a[1][0], a[1][1])[0], zip(chunk, inits)))
            busy += time.perf_counter() - t0
            same &= cards == [int(c) for c in gpu_cards[done:done + len(chunk)]]
            done += len(chunk)
    return {"value": round(done / busy, 1) if busy > 0 else None, "unit": "graphs/s", "cores": threads,
            "kind": "oracle",
            "sample": f"Hopcroft-Karp per graph from its greedy matching, one thread per core, "
                      f"the first {done} of {len(graphs)} graphs in {busy:.2f} s of matching time",
            "identical_cardinalities": bool(same)}


def roofline(b, avg_s, kernel, traffic=None):
    """The roofline object for a kernel that moved `b` algorithmic bytes per
    launch in `avg_s` seconds on average."""
    achieved = b / avg_s / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic, "kernel": kernel,
            "alg_bytes_per_launch": int(b), "avg_launch_ms": round(avg_s * 1000.0, 4)}


def plan_config(info):
    """The kernel instance and launch shape of a batch plan, as its traffic
    summary names them (the plan's batch_min, how many frontier entries a
    wavefront takes at a time, splits the same reads differently and is
    not part of the key)."""
    return f"mapping={info['mapping']} block={info['block']} blocks={info['blocks']}"


def bench_batched(ngraphs, steps, cpu_budget_s=0.0):
    """Uneven batch (graph g: seed mix(4, g), sizes log-uniform in [64, 65536],
    degrees 2..12, half uniform / half banded, 2 % columns emptied): one
    batched launch (autotuned, hipGraph-captured plan) vs a per-graph loop of
    mcm_match on the same resident inputs; per-graph |M| must be identical.
    The roofline of the batched kernel takes its algorithmic bytes from the
    device counters of one batched call with the plan's configuration."""
    import numpy as np
    import torch
    from paper_1303_1379_amd import graphgen as gg, mcm
    t0 = time.time()
    graphs = [gg.batch_member(4, i) for i in range(ngraphs)]
    t_gen = time.time() - t0
    inits = [mcm.cheap_init_host(g.colptr, g.rowind, g.nr) for g in graphs]
    b = mcm.pack_batch(graphs)
    icm = torch.from_numpy(np.concatenate([x[1] for x in inits])).cuda()
    irm = torch.from_numpy(np.concatenate([x[2] for x in inits])).cuda()
    mcm.set_option("autotune", 1)
    plan = mcm.BatchPlan(b, icm, irm)
    mcm.set_option("autotune", 0)
    plan.run()
    ts, kms = [], []
    for _ in range(steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        total, cards = plan.run()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
        kms.append(mcm.last_stats()["kernel_ms"])
    info = plan.info()
    # counters of the same kernel and configuration (every member on the
    # one-workgroup kernel, as in the plan), untimed
    saved = {k: mcm.get_option(k) for k in ("stats", "mapping", "wg_block", "batch_min", "multi_threshold")}
    for k, v in (("stats", 1), ("mapping", info["mapping"]), ("wg_block", info["block"]),
                 ("batch_min", info["batch_min"]), ("multi_threshold", 0)):
        mcm.set_option(k, v)
    _, scards, _, _ = mcm.match_batched(b, icm, irm)
    st = mcm.last_stats()
    for k, v in saved.items():
        mcm.set_option(k, v)
    dgs = [mcm.to_device(g) for g in graphs]
    oc = np.cumsum([0] + [g.nc for g in graphs])
    orr = np.cumsum([0] + [g.nr for g in graphs])
    mcm.match(dgs[0], icm[0:oc[1]], irm[0:orr[1]])
    torch.cuda.synchronize()
    t = time.perf_counter()
    loop_cards = [mcm.match(dg, icm[oc[i]:oc[i + 1]], irm[orr[i]:orr[i + 1]])[0] for i, dg in enumerate(dgs)]
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t
    t_b = float(np.median(ts))
    return {"workload": f"{ngraphs} uneven graphs (sizes log-uniform 64..65536, degree 2..12, half uniform / half "
                        "banded, 2% columns emptied), greedy initial matchings",
            "sum_cols": int(sum(g.nc for g in graphs)), "sum_nnz": int(sum(g.nnz for g in graphs)),
            "batched_graphs_per_s": round(ngraphs / t_b, 1), "batched_ms": round(t_b * 1000, 3),
            "loop_graphs_per_s": round(ngraphs / t_loop, 1), "loop_ms": round(t_loop * 1000, 3),
            "ratio": round(t_loop / t_b, 2),
            "identical_cardinalities": loop_cards == cards.tolist() == scards.tolist(),
            "roofline": roofline(alg_bytes(st), float(np.mean(kms)) / 1000.0, "k_match_wg",
                                 load_traffic("batched", "k_match_wg", plan_config(info))),
            "edges_scanned": st["edges_scanned"], "plan": info, "generate_s": round(t_gen, 2),
            **({"cpu_baseline": oracle_batch(graphs, cards, cpu_budget_s)} if cpu_budget_s > 0 else {})}


def serve_loop(pool, nreq, seed=6):
    """The per-request alternative to the server: the same request sequence
    (drawn from the pool with the replay's seed), each matched by its own
    mcm_cheap_init + mcm_match call on inputs already resident on the device
    (no host copies, which favours the loop).  Returns graphs/s and the
    cardinalities by pool index."""
    import numpy as np
    import torch
    from paper_1303_1379_amd import mcm
    rng = np.random.default_rng(seed)
    rng.exponential(1.0, size=nreq)                      # same draws as the replay: gaps first,
    which = rng.integers(0, len(pool), size=nreq)        # then the pool index
    dgs = [mcm.to_device(g) for g, _, _ in pool]
    cards = {}
    mcm.match(dgs[0], *mcm.cheap_init(dgs[0])[1:])
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i in which.tolist():
        _, cm, rm = mcm.cheap_init(dgs[i])
        cards[i] = mcm.match(dgs[i], cm, rm, cm, rm)[0]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    return nreq / dt, cards


def bench_serving(pool_size, nreq, warmup, lam, cap_rate=20000.0, cap_req=6000, loop_req=600):
    """Poisson arrivals through the continuous-batching server (64 GB HBM
    budget); requests drawn from a pool of distinct graphs of the serving mix
    (n log-uniform 1e3..1e6 per side, degree 4..16, half uniform, half R-MAT).
    Latency runs from each request's scheduled arrival to its results on the
    host.  Capacity: the same server offered `cap_rate` requests/s.  Loop:
    the same requests one mcm_match call after another."""
    from paper_1303_1379_amd import mcm, serving
    t0 = time.time()
    pool = serving.make_pool(pool_size, seed=5)
    t_gen = time.time() - t0
    ref = {}

    def check(i, card, cm, rm):
        ref.setdefault(i, set()).add(int(card))

    srv = mcm.Server(64 << 30, max_batch=1024)
    r = serving.replay(srv, pool, nreq, lam=lam, seed=6, warmup=warmup, check=check)
    st = srv.stats()
    srv.close()
    srv = mcm.Server(64 << 30, max_batch=1024)
    cap = serving.replay(srv, pool, cap_req, lam=cap_rate, seed=8, warmup=0, check=check)
    srv.close()
    loop_gps, loop_cards = serve_loop(pool, loop_req)
    same = all(len(v) == 1 for v in ref.values()) and all(ref[i] == {c} for i, c in loop_cards.items() if i in ref)
    r.update({"pool_graphs": pool_size, "pool_mean_n": round(sum(g.nc for g, _, _ in pool) / pool_size, 1),
              "pool_mean_nnz": round(sum(g.nnz for g, _, _ in pool) / pool_size, 1), "budget_bytes": 64 << 30,
              "peak_bytes": st["peak_bytes"], "launches_batched": st["launches_batched"],
              "launches_multi_graph": st["launches_grid"], "max_batch": st["max_batch_seen"],
              "capacity": {"offered_rate": cap_rate, "requests": cap_req, "graphs_per_s": cap["graphs_per_s"],
                           "p50_ms": cap["p50_ms"], "p99_ms": cap["p99_ms"]},
              "loop_graphs_per_s": round(loop_gps, 1), "loop_requests": loop_req,
              "capacity_vs_loop": round(cap["graphs_per_s"] / loop_gps, 2),
              "identical_cardinalities": bool(same), "generate_s": round(t_gen, 2)})
    return r


def bench_single(name, steps, warmup, stats=True, copy_gbs=None):
    """One workload: counters of an untimed run, `warmup` untimed and `steps`
    timed mcm_match calls (inputs resident), the roofline of the persistent
    kernel (HIP events around its launch, on the stream it runs on)."""
    import numpy as np
    import torch
    from paper_1303_1379_amd import graphgen as gg, mcm
    t0 = time.time()
    g = gg.workload(name)
    t_gen = time.time() - t0
    init_card, cm0, rm0 = mcm.cheap_init_host(g.colptr, g.rowind, g.nr)
    dg = mcm.to_device(g)
    icm = torch.from_numpy(cm0).cuda()
    irm = torch.from_numpy(rm0).cuda()
    ocm = torch.empty_like(icm)
    orm = torch.empty_like(irm)
    st = None
    if stats:
        mcm.set_option("stats", 1)
        mcm.match(dg, icm, irm, ocm, orm)
        st = mcm.last_stats()
        mcm.set_option("stats", 0)
    for _ in range(warmup):
        mcm.match(dg, icm, irm, ocm, orm)
    torch.cuda.synchronize()
    kernel_ms, cards = [], []
    t_start = time.perf_counter()
    for _ in range(steps):
        card, _, _ = mcm.match(dg, icm, irm, ocm, orm)
        kernel_ms.append(mcm.last_stats()["kernel_ms"])
        cards.append(card)
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t_start) * 1000.0 / steps
    last = mcm.last_stats()
    assert len(set(cards)) == 1, f"{name}: cardinality varied across steps: {cards}"
    out = {"workload": f"{name}: {WORKLOADS[name]}", "ncols": g.nc, "nrows": g.nr, "nnz": g.nnz,
           "input_fnv1a": hex(g.fnv1a()), "card": cards[0], "init_card": int(init_card),
           "ms_per_step": round(ms_per_step, 4), "matching_ms_median": round(float(np.median(kernel_ms)), 4),
           "graph_teps": round(g.nnz / (ms_per_step / 1000.0), 1),
           "form": {"driver": mcm.get_option("driver"), "bfs": mcm.get_option("bfs"),
                    "mapping": mcm.get_option("mapping"), "loop": mcm.get_option("loop"),
                    "claim": ("probe", "max")[last["claim"]], "flush": ("atomic", "defer")[last["flush"]],
                    "wr_check": ("early", "late")[last["wr_check"]],
                    "local_levels": int(last["local_levels"]),
                    "alternate": ("classic", "fast")[last["alternate"]]},
           "generate_s": round(t_gen, 2), "_graph": g}
    if st is not None:
        edges = st["edges_scanned"]
        out["value"] = round(edges / (ms_per_step / 1000.0), 1)
        out.update(phases=st["phases"], levels=st["levels"], edges_scanned_per_step=edges)
        out["roofline"] = roofline(alg_bytes(st), float(np.mean(kernel_ms)) / 1000.0,
                                   "k_persistent<true>" if last["loop"] == 0 else "host loop", load_traffic(name))
        if copy_gbs is not None:
            out["roofline"]["measured_copy_gbs"] = copy_gbs
        out["block0_ms"] = {k: round(st[k], 2) for k in ("t_expand_ms", "t_flush_ms", "t_barrier_ms",
                                                         "t_small_ms", "t_augment_ms")}
    return out


def bench_uniform(reps=1000):
    """uniform2000: a 32 KB graph matched by one workgroup; microseconds per
    mcm_match call (wall clock, stream synchronised) and of the kernel (HIP
    events), medians of `reps`."""
    import numpy as np
    import torch
    from paper_1303_1379_amd import graphgen as gg, mcm
    g = gg.workload("uniform2000")
    _, cm0, rm0 = mcm.cheap_init_host(g.colptr, g.rowind, g.nr)
    dg = mcm.to_device(g)
    icm, irm = torch.from_numpy(cm0).cuda(), torch.from_numpy(rm0).cuda()
    ocm, orm = torch.empty_like(icm), torch.empty_like(irm)
    for _ in range(20):
        mcm.match(dg, icm, irm, ocm, orm)
    wall, kern, cards = [], [], set()
    for _ in range(reps):
        t = time.perf_counter()
        card, _, _ = mcm.match(dg, icm, irm, ocm, orm)
        wall.append((time.perf_counter() - t) * 1e6)
        kern.append(mcm.last_stats()["kernel_ms"] * 1000.0)
        cards.add(card)
    return {"workload": f"uniform2000: {WORKLOADS['uniform2000']}", "nnz": g.nnz, "card": cards.pop() if len(cards) == 1
            else sorted(cards), "calls": reps, "us_per_match_median": round(float(np.median(wall)), 2),
            "us_per_match_p90": round(float(np.percentile(wall, 90)), 2),
            "kernel_us_median": round(float(np.median(kern)), 2), "path": "one workgroup (k_match_wg)"}


VARIANTS = [(drv, bfs, mp, ep) for drv in ("apfb", "apsb") for bfs in ("wr", "plain") for mp in ("wave", "thread")
            for ep in (("all", "one") if bfs == "wr" else ("all",))]


def bench_variants(names, reps):
    """The paper's variant grid on each workload: driver APFB / APsB x BFS
    GPUBFS-WR / GPUBFS x edge mapping (edges of a wavefront batch dealt over
    its lanes / one column per lane), and for WR Alternate from every
    reached unmatched row or from one per root; each from the same greedy
    matching; median HIP-event matching time of `reps` runs, counters from
    one more."""
    import numpy as np
    import torch
    from paper_1303_1379_amd import graphgen as gg, mcm
    rows = []
    for name in names:
        g = gg.workload(name)
        _, cm0, rm0 = mcm.cheap_init_host(g.colptr, g.rowind, g.nr)
        dg = mcm.to_device(g)
        icm, irm = torch.from_numpy(cm0).cuda(), torch.from_numpy(rm0).cuda()
        cards = set()
        for drv, bfs, mp, ep in VARIANTS:
            for k, v in (("driver", drv), ("bfs", bfs), ("mapping", mp), ("endpoints", ep), ("stats", 1)):
                mcm.set_option(k, v)
            card, _, _ = mcm.match(dg, icm, irm)
            st = mcm.last_stats()
            mcm.set_option("stats", 0)
            ms = []
            for _ in range(reps):
                mcm.match(dg, icm, irm)
                ms.append(mcm.last_stats()["kernel_ms"])
            cards.add(card)
            rows.append({"workload": name, "driver": drv, "bfs": bfs, "mapping": mp, "endpoints": ep, "card": card,
                         "ms_median": round(float(np.median(ms)), 3), "phases": st["phases"],
                         "levels": st["levels"], "edges_scanned": st["edges_scanned"],
                         "alt_steps": st["alt_steps"], "fix_resets": st["fix_resets"],
                         "edges_per_s": round(st["edges_scanned"] / (float(np.median(ms)) / 1e3), 1)})
        assert len(cards) == 1, f"{name}: variants disagree on |M|: {cards}"
    for k, v in (("driver", "apfb"), ("bfs", "wr"), ("mapping", "auto"), ("endpoints", "auto")):
        mcm.set_option(k, v)
    return rows


def bench_phases(names, drivers=("apfb", "apsb")):
    """Per-phase BFS levels and augmenting-path ends (the paper's figure of
    levels per BFS iteration) for each workload and driver, GPUBFS-WR, from
    the same greedy matching; plus the matching time of a run without stats."""
    import numpy as np
    import torch
    from paper_1303_1379_amd import graphgen as gg, mcm
    rows = []
    for name in names:
        g = gg.workload(name)
        _, cm0, rm0 = mcm.cheap_init_host(g.colptr, g.rowind, g.nr)
        dg = mcm.to_device(g)
        icm, irm = torch.from_numpy(cm0).cuda(), torch.from_numpy(rm0).cuda()
        # BFS levels in the paper's sense: no local levels (every level is
        # one BFS layer and ends at a grid barrier)
        local0 = mcm.get_option("local_levels")
        mcm.set_option("local_levels", 0)
        for drv in drivers:
            mcm.set_option("driver", drv)
            mcm.set_option("stats", 1)
            card, _, _ = mcm.match(dg, icm, irm)
            lv, en = mcm.last_phases()
            mcm.set_option("stats", 0)
            mcm.match(dg, icm, irm)
            ms = mcm.last_stats()["kernel_ms"]
            rows.append({"workload": name, "driver": drv, "local_levels": 0, "card": card, "ms": round(ms, 3),
                         "phases": int(len(lv)),
                         "levels": int(lv.sum()), "levels_max": int(lv.max()) if len(lv) else 0,
                         "levels_mean": round(float(lv.mean()), 1) if len(lv) else 0.0,
                         "levels_per_phase": lv.tolist(), "ends_per_phase": en.tolist()})
        mcm.set_option("local_levels", local0)
    mcm.set_option("driver", "apfb")
    return rows


def measured_copy_gbs(nbytes=1 << 30, reps=5):
    """Device copy bandwidth: one elementwise kernel reading and writing
    nbytes each, timed with events on torch's stream (the stream it runs on)."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    torch.neg(a, out=b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = None
    for _ in range(reps):
        e0.record()
        torch.neg(a, out=b)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b
    return round(2 * nbytes / (best / 1e3) / 1e9, 1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat23", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-budget", type=float, default=0.0,
                    help="seconds of oracle time for cpu_baseline (0: run the oracle to the maximum)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle legs")
    ap.add_argument("--no-stats", action="store_true", help="skip the untimed counter run")
    ap.add_argument("--no-grid", action="store_true", help="skip the grid2048 section")
    ap.add_argument("--no-uniform", action="store_true", help="skip the uniform2000 section")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched section")
    ap.add_argument("--serving", action="store_true", help="add the serving section (not in the default run)")
    ap.add_argument("--grid-steps", type=int, default=3)
    ap.add_argument("--batch-graphs", type=int, default=4096)
    ap.add_argument("--serve-requests", type=int, default=20000, help="serving trace length (after 1000 warm-up)")
    ap.add_argument("--serve-rate", type=float, default=2000.0, help="serving: mean Poisson arrival rate, requests/s")
    ap.add_argument("--variants", default="",
                    help="instead of the bench line: the APFB/APsB x WR/plain x wave/thread grid on these "
                         "comma-separated workloads (one JSON line)")
    ap.add_argument("--phases", default="",
                    help="instead of the bench line: BFS levels and path ends per phase, APFB and APsB, on these "
                         "comma-separated workloads (one JSON line)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="instead of matching, stream this many bytes through one elementwise kernel (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: measures one GPU; --gpus {args.gpus} is not supported (independent graphs and "
              "requests would shard across GPUs with no exchange; one GPU's share is what is measured)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1303_1379_amd import mcm

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")

    if args.variants:
        names = [w for w in args.variants.split(",") if w]
        for w in names:
            if w not in WORKLOADS:
                ap.error(f"unknown workload {w}")
        print(json.dumps({"variants": bench_variants(names, max(args.steps, 1))}), flush=True)
        return

    if args.phases:
        names = [w for w in args.phases.split(",") if w]
        print(json.dumps({"phases": bench_phases(names)}), flush=True)
        return

    if args.copy_bytes:
        n = args.copy_bytes // 4
        a = torch.ones(n, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        for _ in range(args.warmup + args.steps):
            torch.neg(a, out=b)  # one elementwise kernel: reads and writes copy_bytes each
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 4, "launches": args.warmup + args.steps}))
        return

    mcm.set_option("stats", 0)
    copy_gbs = None if args.no_stats else measured_copy_gbs()
    h = bench_single(args.workload, args.steps, args.warmup, stats=not args.no_stats, copy_gbs=copy_gbs)
    g = h.pop("_graph")
    out = {
        "metric": METRIC,
        "value": h.pop("value", None),
        "unit": "edges scanned/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": h.pop("workload"), "ncols": h.pop("ncols"), "nrows": h.pop("nrows"),
                   "nnz": h.pop("nnz"), "input_fnv1a": h.pop("input_fnv1a"), **h.pop("form")},
    }
    rl = h.pop("roofline", None)
    out.update(h)
    if rl is not None:
        out["roofline"] = rl
    print(f"# {args.workload}: {out['ms_per_step']} ms per step", file=sys.stderr, flush=True)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(g, args.cpu_budget if args.cpu_budget > 0 else None)
        out["cpu_baseline"]["host_cpus"] = os.cpu_count()
        out["cpu_baseline"]["cpu_model"] = cpu_model()
        out["cpu_baseline"]["identical_cardinality"] = out["cpu_baseline"]["card"] == out["card"]
        print(f"# oracle: {out['cpu_baseline']['seconds']} s", file=sys.stderr, flush=True)
    del g
    if not args.no_grid and args.workload != "grid2048":
        gr = bench_single("grid2048", max(args.grid_steps, 1), 1, stats=not args.no_stats, copy_gbs=copy_gbs)
        gr.pop("_graph")
        out["grid2048"] = gr
        print(f"# grid2048: {gr['ms_per_step']} ms per step", file=sys.stderr, flush=True)
    if not args.no_uniform:
        out["uniform2000"] = bench_uniform(1000)
        print(f"# uniform2000: {out['uniform2000']['us_per_match_median']} us per match", file=sys.stderr, flush=True)
    if not args.no_batched:
        out["batched"] = bench_batched(args.batch_graphs, max(args.steps, 3), 0.0 if args.no_cpu else 10.0)
        print(f"# batched: {out['batched']['batched_ms']} ms", file=sys.stderr, flush=True)
    if args.serving:
        out["serving"] = bench_serving(48, args.serve_requests + 1000, 1000, args.serve_rate)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
