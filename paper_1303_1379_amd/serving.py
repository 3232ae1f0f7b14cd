"""Serving driver: a request pool and a Poisson-arrival replay through the
library's continuous-batching server (mcm_server_* in libmcm.so).

Request graphs follow the serving workload recipe: n = round(exp(U[ln lo,
ln hi])) vertices per side, average degree uniform in {dmin..dmax}, half
uniform random (distinct rows per column), half R-MAT (scale ceil(log2 n),
d*n samples, ids >= n rejected, duplicates removed).  Generating millions
of edges per request at the offered rate is beyond one host, so the replay
draws its requests from a pool of distinct pre-generated graphs (the pool
index of request i is drawn with the trace's own seed).
"""
from __future__ import annotations

import time

import numpy as np

from . import graphgen as gg
from . import mcm


def make_pool(count: int, seed: int = 5, lo: int = 1000, hi: int = 1000000, dmin: int = 4, dmax: int = 16):
    """`count` request graphs with the serving size/degree/kind mix, each
    with pinned host input and output buffers."""
    import torch
    _, n, deg, kind, rseed = gg.request_trace(seed, count, 2000.0, lo, hi, dmin, dmax)
    pool = []
    for i in range(count):
        g = gg.request_graph(int(n[i]), int(deg[i]), int(kind[i]), int(rseed[i]))
        cp = torch.from_numpy(g.colptr).pin_memory()
        ri = torch.from_numpy(g.rowind if g.nnz else np.zeros(1, np.int32)).pin_memory()
        pool.append((g, cp, ri))
    return pool


def replay(server: mcm.Server, pool, nreq: int, lam: float = 2000.0, seed: int = 6, warmup: int = 0,
           check=None):
    """Submit `nreq` requests with exponential gaps of rate `lam` (drawn
    from the pool), poll completions, and report latency percentiles over
    the requests after the first `warmup` and completed graphs/s over the
    makespan.  Latency runs from a request's scheduled arrival (not from the
    moment this loop got round to submitting it) to its results on the
    host; the time from submission is reported beside it.
    `check(pool_index, card, cmatch, rmatch)` (optional) is called for every
    completed request."""
    import torch
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / lam, size=nreq)
    which = rng.integers(0, len(pool), size=nreq)
    arrive = np.cumsum(gaps)
    outstanding = {}
    lat = np.zeros(nreq)
    lat_sub = np.zeros(nreq)
    paths = np.zeros(nreq, np.int32)
    batch = np.zeros(nreq, np.int32)
    t0 = time.perf_counter()
    i = 0
    done = 0
    t_first_done = None
    while done < nreq:
        now = time.perf_counter() - t0
        while i < nreq and arrive[i] <= now:
            g, cp, ri = pool[which[i]]
            cm = torch.empty(g.nc, dtype=torch.int32).pin_memory()
            rm = torch.empty(g.nr, dtype=torch.int32).pin_memory()
            tk = server.submit_pinned(g.nc, g.nr, cp, ri, cm, rm)
            outstanding[tk] = (i, time.perf_counter())
            i += 1
        for tk in list(outstanding):
            res = server.poll(tk)
            if res is None:
                continue
            card, info, cmh, rmh = res
            k, ts = outstanding.pop(tk)
            tdone = time.perf_counter()
            lat[k] = (tdone - (t0 + arrive[k])) * 1000.0
            lat_sub[k] = (tdone - ts) * 1000.0
            paths[k] = info["path"]
            batch[k] = info["batch_size"]
            if check is not None:
                check(int(which[k]), card, cmh, rmh)
            done += 1
        if i < nreq and not outstanding:
            time.sleep(max(0.0, min(arrive[i] - (time.perf_counter() - t0), 0.001)))
        else:
            time.sleep(0.0002)
    makespan = time.perf_counter() - t0
    lw = lat[warmup:]
    ls = lat_sub[warmup:]
    return {"requests": nreq, "warmup": warmup, "offered_rate": lam,
            "p50_ms": round(float(np.percentile(lw, 50)), 3), "p99_ms": round(float(np.percentile(lw, 99)), 3),
            "mean_ms": round(float(lw.mean()), 3), "latency_from": "scheduled arrival",
            "p50_from_submit_ms": round(float(np.percentile(ls, 50)), 3),
            "p99_from_submit_ms": round(float(np.percentile(ls, 99)), 3),
            "graphs_per_s": round(nreq / makespan, 1),
            "makespan_s": round(makespan, 3), "multi_graph_requests": int(paths.sum()),
            "mean_batch": round(float(batch[paths == 0].mean()) if (paths == 0).any() else 0.0, 1)}
