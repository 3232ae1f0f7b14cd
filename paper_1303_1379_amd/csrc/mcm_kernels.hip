// gfx950 kernels for maximum-cardinality bipartite matching: the BFS level
// expansion of GPUBFS / GPUBFS-WR (paper, Algorithms 2 and 4), Alternate
// (Algorithm 3), FixMatching, and the phase/level loop of Algorithm 1
// (APFB or APsB), in three launch forms:
//   * k_persistent  -- the whole match in one cooperative launch; levels,
//                      Alternate and Fix separated by a grid barrier;
//   * k_init_roots / k_level / k_alternate / k_fix -- one launch per step,
//                      driven by a host loop;
//   * k_match_wg    -- one workgroup matches one graph from start to end
//                      (small graphs, and the batched entry point).
//
// Data layout (all int32 unless noted):
//   rw[r]    (u64) low word = rmatch[r] (-1 unmatched, -2 reached unmatched
//            row this phase), high word = stamp of the phase that reached r.
//            A matched row r stands for its column rmatch[r]: the column is
//            visited exactly when its row is, so one 8-byte gather per
//            scanned edge decides both "matched?" and "visited?".  The paper
//            keeps the visit mark per column (bfs_array) and needs a second
//            dependent gather.
//   frontier entries int4 {col, root, beg, end}: the BFS-tree root travels
//   with the entry (the paper's root[] array, Algorithm 4) and the column's
//   adjacency range is fetched once when the column is claimed.
//   cdone[root] = phase stamp once the tree of `root` reached an unmatched
//   row (the paper's bfs_array[root] = L0 - 2, Algorithm 4).
//
// Concurrency.  A row (and with it the column it is matched to) is claimed
// by a 64-bit compare-and-swap on rw[r], so every column enters a frontier
// once per phase and pred/root always describe the claimer.  Alternate's
// flips race exactly as in the paper; the predecessor check (Algorithm 3)
// stops a walk on a column another walk already flipped, and FixMatching
// unmatches every row whose column does not point back.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mcm_internal.h"

namespace mcm {

#define DEV __device__ __forceinline__

constexpr int kEInternal = -5;  // MCM_EINTERNAL
constexpr int kEInval = -1;     // MCM_EINVAL
constexpr int kEBadInit = -4;   // MCM_EBADINIT

DEV uint32_t *line(uint32_t *ctrl, int l) { return ctrl + l * kLineWords; }

DEV uint32_t ld_agent(const uint32_t *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
DEV int32_t ld_agent_i(const int32_t *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
DEV void st_agent_i(int32_t *p, int32_t v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

DEV void set_status(uint32_t *ctrl, int code)
{
    int32_t *s = reinterpret_cast<int32_t *>(line(ctrl, L_STATUS));
    atomicCAS(s, 0, code);
}

DEV int32_t status_of(uint32_t *ctrl) { return ld_agent_i(reinterpret_cast<int32_t *>(line(ctrl, L_STATUS))); }

// inclusive prefix sum across the 64 lanes of a wavefront
DEV int wave_incl_scan(int x)
{
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

DEV int wave_max(int x)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x = max(x, __shfl_xor(x, o, 64));
    return x;
}

// Append `item` for every lane with p set; one atomic per wavefront reserves
// the slots, lanes write compacted (ballot + popcount prefix).
template <class T>
DEV void wave_push(bool p, const T &item, T *q, uint32_t *cnt)
{
    const uint64_t m = __ballot(p);
    if (m == 0) return;
    const int lane = __lane_id();
    const int leader = __ffsll((unsigned long long)m) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(cnt, (uint32_t)__popcll(m));
    base = __shfl(base, leader, 64);
    if (p) q[base + __popcll(m & ((1ull << lane) - 1ull))] = item;
}


// ---------------------------------------------------------------------
// One scanned edge (col -> r) of the BFS (Algorithm 2 body; Algorithm 4
// adds the root bookkeeping).  A matched, unvisited row is claimed and its
// column becomes a next-frontier entry; an unmatched, unvisited row is
// claimed as an augmenting-path end (rmatch = -2) and marks its root done.
DEV void visit_edge(const DevGraph &g, int col, int root, int r, uint32_t ph, int level, uint32_t flags,
                    bool &newcol, int4 &ne, bool &newend)
{
    uint64_t w = g.rw[r];
    if ((uint32_t)(w >> 32) == ph) return;           // reached earlier in this phase
    const int mate = (int)(uint32_t)w;
    if (mate >= 0) {
        const uint64_t nw = ((uint64_t)ph << 32) | (uint32_t)mate;
        if (atomicCAS((unsigned long long *)&g.rw[r], (unsigned long long)w, (unsigned long long)nw) == w) {
            g.pred[r] = col;
            ne = make_int4(mate, root, g.colptr[mate], g.colptr[mate + 1]);
            newcol = true;
            if (flags & F_LEVELS) g.clevel[mate] = level + 1;
        }
    } else if (mate == -1) {
        const uint64_t nw = ((uint64_t)ph << 32) | 0xFFFFFFFEull;
        if (atomicCAS((unsigned long long *)&g.rw[r], (unsigned long long)w, (unsigned long long)nw) == w) {
            g.pred[r] = col;
            newend = true;
            if (flags & F_WR) g.cdone[root] = ph;
        }
    }
}

struct LevelCounters {
    uint32_t *next;     // next frontier size
    uint32_t *nends;    // ends found in this phase
    uint32_t *found;    // set when this level reached an unmatched row
    uint64_t *stats;    // [8] or null
};

DEV void flush_stats(uint64_t *stats, uint64_t edges, uint64_t expanded, uint64_t claimed, uint64_t found)
{
    if (!stats) return;
    // one atomic per counter per wavefront
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        edges += __shfl_xor(edges, o, 64);
        expanded += __shfl_xor(expanded, o, 64);
        claimed += __shfl_xor(claimed, o, 64);
        found += __shfl_xor(found, o, 64);
    }
    if (__lane_id() == 0) {
        if (edges) atomicAdd((unsigned long long *)&stats[S_EDGES * 16], (unsigned long long)edges);
        if (expanded) atomicAdd((unsigned long long *)&stats[S_EXPANDED * 16], (unsigned long long)expanded);
        if (claimed) atomicAdd((unsigned long long *)&stats[S_CLAIMED * 16], (unsigned long long)claimed);
        if (found) atomicAdd((unsigned long long *)&stats[S_FOUND * 16], (unsigned long long)found);
    }
}

// Expand frontier entries [0, n) of `fq`, wavefront `wave` of `nwaves`
// taking batches of 64 entries.  WAVE: the edges of the 64 entries are
// dealt out 64 at a time across the lanes (load balanced, coalesced rowind
// reads); otherwise every lane walks its own column's edges.
template <bool WAVE>
DEV void expand_level(const DevGraph &g, const int4 *fq, uint32_t n, uint32_t wave, uint32_t nwaves, uint32_t ph,
                      int level, uint32_t flags, int4 *nfq, const LevelCounters &lc)
{
    const int lane = __lane_id();
    uint64_t s_edges = 0, s_exp = 0, s_claim = 0, s_found = 0;
    for (uint32_t base = wave * 64u; base < n; base += nwaves * 64u) {
        const uint32_t i = base + lane;
        int4 e = make_int4(0, 0, 0, 0);
        int deg = 0;
        if (i < n) {
            e = fq[i];
            deg = e.w - e.z;
            if ((flags & F_WR) && deg > 0 && g.cdone[e.y] == ph) deg = 0;  // root already has a path
        }
        if (flags & F_STATS) { s_edges += deg; s_exp += (deg > 0); }
        bool any_end = false;
        if (WAVE) {
            const int incl = wave_incl_scan(deg);
            const int excl = incl - deg;
            const int total = __shfl(incl, 63, 64);
            for (int eb = 0; eb < total; eb += 64) {
                const int k = eb + lane;
                // owner lane: the largest o with excl[o] <= k (excl is non-decreasing)
                int o = 0;
#pragma unroll
                for (int step = 32; step >= 1; step >>= 1) {
                    const int v = __shfl(excl, o + step, 64);
                    if (v <= k) o += step;
                }
                const int ocol = __shfl(e.x, o, 64);
                const int oroot = __shfl(e.y, o, 64);
                const int obeg = __shfl(e.z, o, 64);
                const int oexcl = __shfl(excl, o, 64);
                bool newcol = false, newend = false;
                int4 ne = make_int4(0, 0, 0, 0);
                int r = 0;
                if (k < total) {
                    r = g.rowind[obeg + (k - oexcl)];
                    visit_edge(g, ocol, oroot, r, ph, level, flags, newcol, ne, newend);
                }
                wave_push(newcol, ne, nfq, lc.next);
                wave_push(newend, r, g.ends, lc.nends);
                any_end |= newend;
                if (flags & F_STATS) { s_claim += newcol; s_found += newend; }
            }
        } else {
            const int maxdeg = wave_max(deg);
            for (int t = 0; t < maxdeg; ++t) {
                bool newcol = false, newend = false;
                int4 ne = make_int4(0, 0, 0, 0);
                int r = 0;
                if (t < deg) {
                    r = g.rowind[e.z + t];
                    visit_edge(g, e.x, e.y, r, ph, level, flags, newcol, ne, newend);
                }
                wave_push(newcol, ne, nfq, lc.next);
                wave_push(newend, r, g.ends, lc.nends);
                any_end |= newend;
                if (flags & F_STATS) { s_claim += newcol; s_found += newend; }
            }
        }
        if ((flags & F_APSB) && __ballot(any_end) != 0 && lane == 0) atomicOr(lc.found, 1u);
    }
    if (flags & F_STATS) flush_stats(lc.stats, s_edges, s_exp, s_claim, s_found);
}

// InitBfsArray (paper, section 3, before Algorithm 2; root filled as in
// Algorithm 4): every unmatched column with at least one edge becomes a
// root and an entry of the first frontier.  Columns without edges can never
// be matched and would expand nothing.
DEV void init_roots(const DevGraph &g, uint32_t wave, uint32_t nwaves, uint32_t flags, uint32_t *cnt)
{
    const int lane = __lane_id();
    for (uint32_t base = wave * 64u; base < (uint32_t)g.nc; base += nwaves * 64u) {
        const int c = (int)(base + lane);
        bool p = false;
        int4 e = make_int4(0, 0, 0, 0);
        if (c < g.nc) {
            const bool un = g.cmatch[c] == -1;
            if (un) {
                const int b = g.colptr[c], en = g.colptr[c + 1];
                if (en > b) { p = true; e = make_int4(c, c, b, en); }
            }
            if (flags & F_LEVELS) g.clevel[c] = un ? 0 : -1;
        }
        wave_push(p, e, g.fq0, cnt);
    }
}

// Alternate (Algorithm 3) from every reached unmatched row, one thread per
// row.  Guard of a walk that arrives at a root (its column has no mate).
DEV void alternate(const DevGraph &g, uint32_t nends, uint32_t tid, uint32_t nthreads, uint32_t flags,
                   uint32_t *ctrl, uint64_t *stats)
{
    uint64_t steps = 0;
    int32_t *rlo = reinterpret_cast<int32_t *>(g.rw);  // low word of rw[r] is at rlo[2r]
    for (uint32_t i = tid; i < nends; i += nthreads) {
        int r = g.ends[i];
        uint32_t guard = 0;
        while (r != -1) {
            const int c = ld_agent_i(&g.pred[r]);
            const int r2 = ld_agent_i(&g.cmatch[c]);
            if (r2 != -1 && ld_agent_i(&g.pred[r2]) == c) break;  // c already flipped by another walk
            st_agent_i(&g.cmatch[c], r);
            st_agent_i(&rlo[2 * (size_t)r], c);
            r = r2;
            ++steps;
            if (++guard > (uint32_t)g.nc + 1u) { set_status(ctrl, kEInternal); break; }
        }
    }
    if ((flags & F_STATS) && stats) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) steps += __shfl_xor(steps, o, 64);
        if (__lane_id() == 0 && steps) atomicAdd((unsigned long long *)&stats[S_ALT * 16], (unsigned long long)steps);
    }
}

// FixMatching: a row whose column points elsewhere lost a race and is
// unmatched; a row still marked -2 (its walk stopped before reaching it)
// returns to -1.  cmatch is not touched.
DEV void fix_matching(const DevGraph &g, uint32_t tid, uint32_t nthreads, uint32_t flags, uint64_t *stats)
{
    uint64_t resets = 0;
    int32_t *rlo = reinterpret_cast<int32_t *>(g.rw);
    for (uint32_t r = tid; r < (uint32_t)g.nr; r += nthreads) {
        const int m = rlo[2 * (size_t)r];
        if (m == -1) continue;
        if (m < 0 || g.cmatch[m] != (int)r) { rlo[2 * (size_t)r] = -1; resets += (m >= 0); }
    }
    if ((flags & F_STATS) && stats) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) resets += __shfl_xor(resets, o, 64);
        if (__lane_id() == 0 && resets) atomicAdd((unsigned long long *)&stats[S_FIX * 16], (unsigned long long)resets);
    }
}

// ---------------------------------------------------------------------
// Grid barrier for the cooperative launch: arrival counter + generation,
// agent-scope release before arriving and acquire after leaving, bounded
// wait.  Returns false (all blocks, eventually) once any block set a
// status, e.g. after a wait ran past the deadline.
DEV bool grid_barrier(uint32_t *ctrl, uint32_t nblocks, uint64_t timeout, int *s_ok)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        uint32_t *cnt = line(ctrl, L_BAR_COUNT);
        uint32_t *gen = line(ctrl, L_BAR_GEN);
        if (status_of(ctrl) != 0) {
            ok = 0;
        } else {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const uint32_t g0 = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t prev = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            if (prev == nblocks - 1) {
                __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(gen, g0 + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                const uint64_t t0 = wall_clock64();
                while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g0) {
                    if (status_of(ctrl) != 0) { ok = 0; break; }
                    if (wall_clock64() - t0 > timeout) { set_status(ctrl, kEInternal); ok = 0; break; }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        *s_ok = ok;
    }
    __syncthreads();
    return *s_ok != 0;
}

// ---------------------------------------------------------------------
// The phase loop of Algorithm 1, parameterised by how work is spread and
// synchronised: Grid (cooperative launch, all blocks) or Block (one
// workgroup owns the graph).
struct GridSync {
    uint32_t *ctrl;
    uint64_t timeout;
    int *s_ok;
    DEV uint32_t wave() const { return blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); }
    DEV uint32_t nwaves() const { return gridDim.x * (blockDim.x >> 6); }
    DEV uint32_t tid() const { return blockIdx.x * blockDim.x + threadIdx.x; }
    DEV uint32_t nthreads() const { return gridDim.x * blockDim.x; }
    DEV bool leader() const { return blockIdx.x == 0 && threadIdx.x == 0; }
    DEV bool sync() { return grid_barrier(ctrl, gridDim.x, timeout, s_ok); }
    DEV uint32_t load(uint32_t *p) const { return ld_agent(p); }
};

struct BlockSync {
    DEV uint32_t wave() const { return threadIdx.x >> 6; }
    DEV uint32_t nwaves() const { return blockDim.x >> 6; }
    DEV uint32_t tid() const { return threadIdx.x; }
    DEV uint32_t nthreads() const { return blockDim.x; }
    DEV bool leader() const { return threadIdx.x == 0; }
    DEV bool sync() { __syncthreads(); return true; }
    DEV uint32_t load(uint32_t *p) const { return *(volatile uint32_t *)p; }
};

// Counters of one run: either lines of the global control block (grid) or
// a small LDS array (block).  cnt[0..2] frontier sizes, cnt[3..5] found
// flags, cnt[6] ends, cnt[7] status (block only); `stride` words apart.
struct Counters {
    uint32_t *base;
    int stride;
    DEV uint32_t *fcount(int i) const { return base + (L_FCOUNT0 + i) * stride; }
    DEV uint32_t *found(int i) const { return base + (L_FOUND0 + i) * stride; }
    DEV uint32_t *nends() const { return base + L_NENDS * stride; }
};

// Runs phases until one finds no unmatched row (or only one phase with
// F_NOAUG).  Returns false if a barrier failed (status set).  *phases_out
// and *levels_out receive the phase and level counts (leader only).
template <bool WAVE, class Sync>
DEV bool run_phases(const DevGraph &g, Sync &s, const Counters &k, const RunOpt &o, uint32_t *ctrl, uint64_t *stats,
                    uint32_t *phases_out, uint32_t *levels_out)
{
    uint32_t total_levels = 0;
    uint32_t ph = 1;
    for (;; ++ph) {
        if (ph > o.max_phases) { if (s.leader()) set_status(ctrl, kEInternal); return false; }
        init_roots(g, s.wave(), s.nwaves(), o.flags, k.fcount(0));
        if (!s.sync()) return false;
        int L = 0;
        for (;;) {
            const uint32_t n = s.load(k.fcount(L % 3));
            if (n == 0) break;
            if ((uint32_t)L > o.max_levels) { if (s.leader()) set_status(ctrl, kEInternal); return false; }
            if (s.leader()) { *k.fcount((L + 2) % 3) = 0; *k.found((L + 2) % 3) = 0; }
            const int4 *cur = (L & 1) ? g.fq1 : g.fq0;
            int4 *nxt = (L & 1) ? g.fq0 : g.fq1;
            LevelCounters lc{k.fcount((L + 1) % 3), k.nends(), k.found(L % 3), (o.flags & F_STATS) ? stats : nullptr};
            expand_level<WAVE>(g, cur, n, s.wave(), s.nwaves(), ph, L, o.flags, nxt, lc);
            ++total_levels;
            if (!s.sync()) return false;
            if ((o.flags & F_APSB) && s.load(k.found(L % 3)) != 0) break;
            ++L;
        }
        const uint32_t ne = s.load(k.nends());
        if (ne == 0 || (o.flags & F_NOAUG)) break;
        alternate(g, ne, s.tid(), s.nthreads(), o.flags, ctrl, stats);
        if (!s.sync()) return false;
        fix_matching(g, s.tid(), s.nthreads(), o.flags, stats);
        if (s.leader()) {
            for (int i = 0; i < 3; ++i) { *k.fcount(i) = 0; *k.found(i) = 0; }
            *k.nends() = 0;
        }
        if (!s.sync()) return false;
    }
    if (s.leader()) { *phases_out = ph; *levels_out = total_levels; }
    return true;
}

// ---------------------------------------------------------------------
// Kernels

// Copy the initial matching into the working state, reset stamps.
__global__ void k_setup(DevGraph g, const int32_t *init_c, const int32_t *init_r, uint32_t *ctrl, uint32_t flags)
{
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nt = gridDim.x * blockDim.x;
    for (uint32_t c = tid; c < (uint32_t)g.nc; c += nt) {
        g.cmatch[c] = init_c ? init_c[c] : -1;
        g.cdone[c] = 0;
        if (flags & F_LEVELS) g.clevel[c] = -1;
    }
    for (uint32_t r = tid; r < (uint32_t)g.nr; r += nt) {
        g.rw[r] = (uint64_t)(uint32_t)(init_r ? init_r[r] : -1);
        if (flags & F_LEVELS) g.pred[r] = -1;
    }
    for (uint32_t i = tid; i < (uint32_t)(L_NLINES * kLineWords); i += nt) ctrl[i] = 0;
}

// Optional input validation (option validate=1).
__global__ void k_validate(int32_t nc, int32_t nr, const int32_t *colptr, const int32_t *rowind, const int32_t *init_c,
                           const int32_t *init_r, uint32_t *ctrl)
{
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nt = gridDim.x * blockDim.x;
    if (tid == 0 && colptr[0] != 0) set_status(ctrl, kEInval);
    for (uint32_t c = tid; c < (uint32_t)nc; c += nt)
        if (colptr[c + 1] < colptr[c]) set_status(ctrl, kEInval);
    const int64_t nnz = colptr[nc];
    for (int64_t j = tid; j < nnz; j += nt)
        if (rowind[j] < 0 || rowind[j] >= nr) set_status(ctrl, kEInval);
    if (!init_c) return;
    for (uint32_t c = tid; c < (uint32_t)nc; c += nt) {
        const int r = init_c[c];
        if (r == -1) continue;
        if (r < 0 || r >= nr || init_r[r] != (int)c) { set_status(ctrl, kEBadInit); continue; }
        bool on = false;
        for (int j = colptr[c]; j < colptr[c + 1] && !on; ++j) on = rowind[j] == r;
        if (!on) set_status(ctrl, kEBadInit);
    }
    for (uint32_t r = tid; r < (uint32_t)nr; r += nt) {
        const int c = init_r[r];
        if (c == -1) continue;
        if (c < 0 || c >= nc || init_c[c] != (int)r) set_status(ctrl, kEBadInit);
    }
}

template <bool WAVE>
__global__ void __launch_bounds__(1024) k_persistent(DevGraph g, uint32_t *ctrl, RunOpt o)
{
    __shared__ int s_ok;
    GridSync s{ctrl, o.timeout, &s_ok};
    Counters k{ctrl, kLineWords};
    uint64_t *stats = reinterpret_cast<uint64_t *>(line(ctrl, L_STAT0));
    uint32_t ph = 0, lv = 0;
    if (run_phases<WAVE>(g, s, k, o, ctrl, stats, &ph, &lv) && s.leader()) {
        *line(ctrl, L_PHASE) = ph;
        *line(ctrl, L_LEVELS) = lv;
    }
}

// Host-driven steps (one launch each).
__global__ void k_init_roots(DevGraph g, uint32_t *ctrl, uint32_t flags)
{
    GridSync s{ctrl, 0, nullptr};
    init_roots(g, s.wave(), s.nwaves(), flags, line(ctrl, L_FCOUNT0));
}

template <bool WAVE>
__global__ void __launch_bounds__(1024) k_level(DevGraph g, uint32_t *ctrl, uint32_t n, uint32_t ph, int L, uint32_t flags)
{
    GridSync s{ctrl, 0, nullptr};
    Counters k{ctrl, kLineWords};
    if (s.leader()) { *k.fcount((L + 2) % 3) = 0; *k.found((L + 2) % 3) = 0; }
    const int4 *cur = (L & 1) ? g.fq1 : g.fq0;
    int4 *nxt = (L & 1) ? g.fq0 : g.fq1;
    LevelCounters lc{k.fcount((L + 1) % 3), k.nends(), k.found(L % 3),
                     (flags & F_STATS) ? reinterpret_cast<uint64_t *>(line(ctrl, L_STAT0)) : nullptr};
    expand_level<WAVE>(g, cur, n, s.wave(), s.nwaves(), ph, L, flags, nxt, lc);
}

__global__ void k_alternate(DevGraph g, uint32_t *ctrl, uint32_t flags)
{
    GridSync s{ctrl, 0, nullptr};
    const uint32_t ne = *line(ctrl, L_NENDS);
    alternate(g, ne, s.tid(), s.nthreads(), flags, ctrl, reinterpret_cast<uint64_t *>(line(ctrl, L_STAT0)));
}

__global__ void k_fix(DevGraph g, uint32_t *ctrl, uint32_t flags)
{
    GridSync s{ctrl, 0, nullptr};
    fix_matching(g, s.tid(), s.nthreads(), flags, reinterpret_cast<uint64_t *>(line(ctrl, L_STAT0)));
    if (s.leader()) {
        Counters k{ctrl, kLineWords};
        for (int i = 0; i < 3; ++i) { *k.fcount(i) = 0; *k.found(i) = 0; }
        *k.nends() = 0;
    }
}

// Unpack rmatch, count |M| = #{c : cmatch[c] >= 0}.
__global__ void k_finish(DevGraph g, int32_t *out_r, uint32_t *ctrl)
{
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nt = gridDim.x * blockDim.x;
    for (uint32_t r = tid; r < (uint32_t)g.nr; r += nt) out_r[r] = (int32_t)(uint32_t)g.rw[r];
    uint64_t m = 0;
    for (uint32_t c = tid; c < (uint32_t)g.nc; c += nt) m += (g.cmatch[c] >= 0);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m += __shfl_xor(m, o, 64);
    if (__lane_id() == 0 && m) atomicAdd((unsigned long long *)line(ctrl, L_CARD), (unsigned long long)m);
}

// Konig cover from the state left by one complete BFS phase (stamp ph):
// reached columns are the unmatched ones and those whose row was claimed.
__global__ void k_cover(DevGraph g, uint32_t ph, uint8_t *col_cov, uint8_t *row_cov, uint32_t *ctrl)
{
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nt = gridDim.x * blockDim.x;
    uint64_t k = 0;
    for (uint32_t c = tid; c < (uint32_t)g.nc; c += nt) {
        const int r = g.cmatch[c];
        const uint8_t v = (r >= 0 && (uint32_t)(g.rw[r] >> 32) != ph) ? 1 : 0;
        col_cov[c] = v;
        k += v;
    }
    for (uint32_t r = tid; r < (uint32_t)g.nr; r += nt) {
        const uint8_t v = ((uint32_t)(g.rw[r] >> 32) == ph) ? 1 : 0;
        row_cov[r] = v;
        k += v;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) k += __shfl_xor(k, o, 64);
    if (__lane_id() == 0 && k) atomicAdd((unsigned long long *)line(ctrl, L_CARD), (unsigned long long)k);
}

// pred of reached rows for the level inspection entry point
__global__ void k_export_pred(DevGraph g, uint32_t ph, int32_t *row_pred)
{
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nt = gridDim.x * blockDim.x;
    for (uint32_t r = tid; r < (uint32_t)g.nr; r += nt)
        row_pred[r] = ((uint32_t)(g.rw[r] >> 32) == ph) ? g.pred[r] : -1;
}

// ---------------------------------------------------------------------
// One workgroup per graph.  Used for small single graphs and for batches;
// blocks take graphs from a queue (ordered largest first by the host) until
// it is empty.  Every graph gets its own state slices; counters live in LDS.
template <bool WAVE>
__global__ void __launch_bounds__(1024) k_match_wg(const BatchDesc *descs, const int32_t *order, int32_t ngraphs,
                                                   const int32_t *colptr_all, const int32_t *rowind_all,
                                                   const int32_t *init_c, const int32_t *init_r, int32_t *cmatch_all,
                                                   int32_t *out_r, uint64_t *rw_all, int32_t *pred_all,
                                                   uint32_t *cdone_all, int4 *fq_all, int32_t *ends_all,
                                                   int64_t *card, uint32_t *ctrl, RunOpt o)
{
    __shared__ uint32_t s_cnt[L_NLINES];
    __shared__ int32_t s_next;
    uint64_t *stats = reinterpret_cast<uint64_t *>(line(ctrl, L_STAT0));
    uint32_t *queue = line(ctrl, L_BAR_COUNT);  // graph queue head (no grid barrier in this kernel)
    BlockSync s;
    for (;;) {
        if (threadIdx.x == 0) s_next = (int32_t)atomicAdd(queue, 1u);
        __syncthreads();
        const int32_t qi = s_next;
        __syncthreads();
        if (qi >= ngraphs) break;
        const int32_t gi = order ? order[qi] : qi;
        const BatchDesc d = descs[gi];
        DevGraph g;
        g.colptr = colptr_all + d.colptr_off;
        g.rowind = rowind_all + d.rowind_off;
        g.nc = d.nc;
        g.nr = d.nr;
        g.cmatch = cmatch_all + d.col_off;
        g.rw = rw_all + d.row_off;
        g.pred = pred_all + d.row_off;
        g.cdone = cdone_all + d.col_off;
        g.fq0 = fq_all + 2 * d.col_off;
        g.fq1 = fq_all + 2 * d.col_off + d.nc;
        g.ends = ends_all + d.row_off;
        g.clevel = nullptr;
        // set up this graph's state
        for (int c = threadIdx.x; c < g.nc; c += blockDim.x) {
            g.cmatch[c] = init_c ? init_c[d.col_off + c] : -1;
            g.cdone[c] = 0;
        }
        for (int r = threadIdx.x; r < g.nr; r += blockDim.x)
            g.rw[r] = (uint64_t)(uint32_t)(init_r ? init_r[d.row_off + r] : -1);
        for (int i = threadIdx.x; i < L_NLINES; i += blockDim.x) s_cnt[i] = 0;
        __syncthreads();
        Counters k{s_cnt, 1};
        uint32_t ph = 0, lv = 0;
        const bool ok = (g.nc > 0 && g.nr > 0) ? run_phases<WAVE>(g, s, k, o, ctrl, stats, &ph, &lv) : true;
        __syncthreads();
        // unpack and count
        uint32_t m = 0;
        for (int r = threadIdx.x; r < g.nr; r += blockDim.x) out_r[d.row_off + r] = (int32_t)(uint32_t)g.rw[r];
        for (int c = threadIdx.x; c < g.nc; c += blockDim.x) m += (g.cmatch[c] >= 0);
        __syncthreads();
        if (threadIdx.x == 0) s_cnt[0] = 0;
        __syncthreads();
        if (m) atomicAdd(&s_cnt[0], m);
        __syncthreads();
        if (threadIdx.x == 0) {
            card[gi] = ok ? (int64_t)s_cnt[0] : (int64_t)kEInternal;
            atomicAdd((unsigned long long *)line(ctrl, L_CARD), (unsigned long long)s_cnt[0]);
            atomicMax(line(ctrl, L_PHASE), ph);
            atomicAdd(line(ctrl, L_LEVELS), lv);
        }
        __syncthreads();
    }
}

__global__ void k_zero_ctrl(uint32_t *ctrl)
{
    for (uint32_t i = threadIdx.x; i < (uint32_t)(L_NLINES * kLineWords); i += blockDim.x) ctrl[i] = 0;
}

// ---------------------------------------------------------------------
// Launch helpers called by the host driver (mcm_api.cpp).

hipError_t launch_zero_ctrl(uint32_t *ctrl, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_ctrl, dim3(1), dim3(256), 0, st, ctrl);
    return hipGetLastError();
}

hipError_t launch_setup(const DevGraph &g, const int32_t *ic, const int32_t *ir, uint32_t *ctrl, uint32_t flags,
                        hipStream_t st)
{
    const int64_t n = g.nc > g.nr ? g.nc : g.nr;
    int blocks = (int)((n + 255) / 256);
    if (blocks < 1) blocks = 1;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_setup, dim3(blocks), dim3(256), 0, st, g, ic, ir, ctrl, flags);
    return hipGetLastError();
}

hipError_t launch_validate(int32_t nc, int32_t nr, const int32_t *cp, const int32_t *ri, const int32_t *ic,
                           const int32_t *ir, uint32_t *ctrl, hipStream_t st)
{
    hipLaunchKernelGGL(k_validate, dim3(1024), dim3(256), 0, st, nc, nr, cp, ri, ic, ir, ctrl);
    return hipGetLastError();
}

hipError_t persistent_occupancy(bool wave, int block, int *blocks_per_cu)
{
    if (wave)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, reinterpret_cast<const void *>(&k_persistent<true>), block, 0);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, reinterpret_cast<const void *>(&k_persistent<false>), block, 0);
}

hipError_t launch_persistent(const DevGraph &g, uint32_t *ctrl, const RunOpt &o, bool wave, int blocks, int block,
                             hipStream_t st)
{
    DevGraph gg = g;
    uint32_t *cc = ctrl;
    RunOpt oo = o;
    void *args[] = {&gg, &cc, &oo};
    const void *fn = wave ? reinterpret_cast<const void *>(&k_persistent<true>)
                          : reinterpret_cast<const void *>(&k_persistent<false>);
    return hipLaunchCooperativeKernel(fn, dim3(blocks), dim3(block), args, 0, st);
}

hipError_t launch_init_roots(const DevGraph &g, uint32_t *ctrl, uint32_t flags, hipStream_t st)
{
    int blocks = (int)((g.nc + 255) / 256);
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_init_roots, dim3(blocks), dim3(256), 0, st, g, ctrl, flags);
    return hipGetLastError();
}

hipError_t launch_level(const DevGraph &g, uint32_t *ctrl, uint32_t n, uint32_t ph, int L, uint32_t flags, bool wave,
                        int max_blocks, hipStream_t st)
{
    int blocks = (int)((n + 255) / 256);
    if (blocks < 1) blocks = 1;
    if (blocks > max_blocks) blocks = max_blocks;
    if (wave)
        hipLaunchKernelGGL(k_level<true>, dim3(blocks), dim3(256), 0, st, g, ctrl, n, ph, L, flags);
    else
        hipLaunchKernelGGL(k_level<false>, dim3(blocks), dim3(256), 0, st, g, ctrl, n, ph, L, flags);
    return hipGetLastError();
}

hipError_t launch_alternate(const DevGraph &g, uint32_t *ctrl, uint32_t nends, uint32_t flags, hipStream_t st)
{
    int blocks = (int)((nends + 255) / 256);
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_alternate, dim3(blocks), dim3(256), 0, st, g, ctrl, flags);
    return hipGetLastError();
}

hipError_t launch_fix(const DevGraph &g, uint32_t *ctrl, uint32_t flags, hipStream_t st)
{
    int blocks = (int)((g.nr + 255) / 256);
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fix, dim3(blocks), dim3(256), 0, st, g, ctrl, flags);
    return hipGetLastError();
}

hipError_t launch_finish(const DevGraph &g, int32_t *out_r, uint32_t *ctrl, hipStream_t st)
{
    const int64_t n = g.nc > g.nr ? g.nc : g.nr;
    int blocks = (int)((n + 255) / 256);
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_finish, dim3(blocks), dim3(256), 0, st, g, out_r, ctrl);
    return hipGetLastError();
}

hipError_t launch_cover(const DevGraph &g, uint32_t ph, uint8_t *cc, uint8_t *rc, uint32_t *ctrl, hipStream_t st)
{
    const int64_t n = g.nc > g.nr ? g.nc : g.nr;
    int blocks = (int)((n + 255) / 256);
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_cover, dim3(blocks), dim3(256), 0, st, g, ph, cc, rc, ctrl);
    return hipGetLastError();
}

hipError_t launch_export_pred(const DevGraph &g, uint32_t ph, int32_t *row_pred, hipStream_t st)
{
    int blocks = (int)((g.nr + 255) / 256);
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_export_pred, dim3(blocks), dim3(256), 0, st, g, ph, row_pred);
    return hipGetLastError();
}

hipError_t launch_match_wg(const BatchDesc *descs, const int32_t *order, int32_t ngraphs, const int32_t *cp,
                           const int32_t *ri, const int32_t *ic, const int32_t *ir, int32_t *cm, int32_t *out_r,
                           uint64_t *rw, int32_t *pred, uint32_t *cdone, int4 *fq, int32_t *ends, int64_t *card,
                           uint32_t *ctrl, const RunOpt &o, bool wave, int blocks, int block, hipStream_t st)
{
    if (wave)
        hipLaunchKernelGGL(k_match_wg<true>, dim3(blocks), dim3(block), 0, st, descs, order, ngraphs, cp, ri, ic, ir,
                           cm, out_r, rw, pred, cdone, fq, ends, card, ctrl, o);
    else
        hipLaunchKernelGGL(k_match_wg<false>, dim3(blocks), dim3(block), 0, st, descs, order, ngraphs, cp, ri, ic, ir,
                           cm, out_r, rw, pred, cdone, fq, ends, card, ctrl, o);
    return hipGetLastError();
}

}  // namespace mcm
