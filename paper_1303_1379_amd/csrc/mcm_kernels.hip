// gfx950 kernels for maximum-cardinality bipartite matching: the BFS level
// expansion of GPUBFS / GPUBFS-WR (paper, Algorithms 2 and 4), Alternate
// (Algorithm 3), FixMatching, and the phase/level loop of Algorithm 1
// (APFB or APsB), in three launch forms:
//   * k_persistent  -- the whole match in one cooperative launch.  Levels
//                      with a large frontier are expanded by every block and
//                      separated by a grid barrier; a run of levels whose
//                      frontier stays small is expanded by block 0 alone,
//                      with workgroup barriers only;
//   * k_init_roots / k_level / k_alternate / k_fix -- one launch per step,
//                      driven by a host loop (the paper's arrangement);
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
//   adjacency range is fetched once, when the column is claimed.
//   cdone[root] = phase stamp once the tree of `root` reached an unmatched
//   row (the paper's bfs_array[root] = L0 - 2, Algorithm 4).
//
// Concurrency.  A row (and with it the column it is matched to) is claimed
// by a 64-bit compare-and-swap on rw[r], so every column enters a frontier
// once per phase and pred/root always describe the claimer.  Alternate's
// flips race exactly as in the paper; the predecessor check (Algorithm 3)
// stops a walk on a column another walk already flipped, and FixMatching
// unmatches every row whose column does not point back.  Work confined to
// one workgroup (a single-workgroup run of levels, a graph of the batched
// kernel) uses workgroup-scope atomics, which complete in the CU's L2
// instead of travelling to the memory-side coherence point.
//
// Queue pushes are staged per wavefront in LDS (ballot + popcount
// compaction) and reach the global queue in blocks: one atomic per staged
// batch of up to kStageQ entries and one per workgroup at the end of a
// level, instead of one per wavefront per 64 edges.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mcm_internal.h"

namespace mcm {

#define DEV __device__ __forceinline__

constexpr int kEInternal = -5;  // MCM_EINTERNAL
constexpr int kEInval = -1;     // MCM_EINVAL
constexpr int kEBadInit = -4;   // MCM_EBADINIT
constexpr int kAgent = __HIP_MEMORY_SCOPE_AGENT;
constexpr int kGroup = __HIP_MEMORY_SCOPE_WORKGROUP;

DEV uint32_t *line(uint32_t *ctrl, int l) { return ctrl + l * kLineWords; }

template <int S> DEV uint32_t ld_u(const uint32_t *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, S); }
template <int S> DEV int32_t ld_i(const int32_t *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, S); }
template <int S> DEV void st_i(int32_t *p, int32_t v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, S); }
template <int S> DEV void st_u(uint32_t *p, uint32_t v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, S); }
template <int S> DEV bool cas_u64(uint64_t *p, uint64_t expect, uint64_t desired)
{
    return __hip_atomic_compare_exchange_strong(p, &expect, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED, S);
}

DEV void set_status(uint32_t *ctrl, int code)
{
    int32_t *s = reinterpret_cast<int32_t *>(line(ctrl, L_STATUS));
    atomicCAS(s, 0, code);
}

DEV int32_t status_of(uint32_t *ctrl) { return ld_i<kAgent>(reinterpret_cast<int32_t *>(line(ctrl, L_STATUS))); }

// LDS written by some lanes of a wavefront and read by others
DEV void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

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

DEV uint64_t wave_sum(uint64_t x)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

DEV uint64_t lanemask_lt() { return (1ull << __lane_id()) - 1ull; }

// Add v, summed over the workgroup, to *dst with one atomic per workgroup
// (same-address atomics serialise, ~11 ns each; one per wavefront of a
// large grid costs a fifth of a millisecond).  Every thread calls it.
DEV void block_add(uint64_t v, uint64_t *dst)
{
    __shared__ uint64_t s_part[16];
    v = wave_sum(v);
    if (__lane_id() == 0) s_part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (uint32_t w = 0; w < (blockDim.x >> 6); ++w) t += s_part[w];
        if (t) atomicAdd((unsigned long long *)dst, (unsigned long long)t);
    }
    __syncthreads();
}

// ---------------------------------------------------------------------
// Per-wavefront staging of queue pushes.
struct Stage {
    int4 *q;      // LDS [kStageQ] frontier entries of this wavefront
    int32_t *e;   // LDS [kStageE] unmatched-row ends
    int nq, ne;   // fill (wavefront-uniform)
    int dq, de;   // entries already handed to the global queues since the last flush
};

DEV Stage make_stage(char *smem)
{
    const int waves = blockDim.x >> 6, w = threadIdx.x >> 6;
    Stage s;
    s.q = reinterpret_cast<int4 *>(smem) + w * kStageQ;
    s.e = reinterpret_cast<int32_t *>(smem + waves * kStageQ * 16) + w * kStageE;
    s.nq = s.ne = 0;
    s.dq = s.de = 0;
    return s;
}

// Word of the staging scratch that holds a level's batch counter (words
// 0..51 serve block_flush).
constexpr int kBatchCtr = 52;

// Elements per lane in flight in the per-phase passes over all columns or
// rows (the roots, FixMatching).
constexpr int kStream = 4;

DEV uint32_t *stage_tmp(char *smem)
{
    const int waves = blockDim.x >> 6;
    return reinterpret_cast<uint32_t *>(smem + waves * (kStageQ * 16 + kStageE * 4));
}

// An unmatched-row end; agent scope (`atomic`) where grid levels pass their
// barriers without fences (F_DEFER).
DEV void put_end(int32_t *ge, uint32_t i, int32_t r, bool atomic)
{
    if (atomic) __hip_atomic_store(ge + i, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else ge[i] = r;
}

// Hand a wavefront's staged ends to the global list now (its stage is full).
// `cap` (0: unchecked) bounds the list: entries past it are counted but not
// stored, and the reader sees the count exceed the capacity.
DEV void drain_ends(Stage &st, int32_t *ge, uint32_t *gcnt, bool atomic, uint32_t cap = 0)
{
    wave_lds_sync();
    uint32_t base = 0;
    if (__lane_id() == 0) base = atomicAdd(gcnt, (uint32_t)st.ne);
    base = __shfl(base, 0, 64);
    for (int i = __lane_id(); i < st.ne; i += 64)
        if (!cap || base + (uint32_t)i < cap) put_end(ge, base + i, st.e[i], atomic);
    wave_lds_sync();
    st.de += st.ne;
    st.ne = 0;
}

// Append end r for every lane with p set (wavefront-uniform call).
DEV void push_end(bool p, int32_t r, Stage &st, int32_t *ge, uint32_t *gcnt, bool atomic, uint32_t cap = 0)
{
    const uint64_t m = __ballot(p);
    if (m == 0) return;
    if (st.ne > kStageE - 64) drain_ends(st, ge, gcnt, atomic, cap);
    if (p) st.e[st.ne + __popcll(m & lanemask_lt())] = r;
    st.ne += __popcll(m);
}

// Where a wavefront's frontier entries go: queue q, its slots reserved from
// the 32-bit counter c32 or, for deferred grid levels, from the low word of
// the 64-bit counter c64 of the coming grid barrier.  With `atomic` every
// entry is stored as two agent-scope 64-bit words and read back by
// take_entry: no copy of it waits in one XCD's L2, and a reader can tell a
// slot that has not been written yet.
struct QSink {
    int4 *q;
    uint32_t *c32;
    uint64_t *c64;
    bool atomic;
    uint64_t cap = 0;  // slots of q (0: not checked); the level-free BFS checks every write
};

DEV void put_entry(const QSink &k, uint32_t i, const int4 &e)
{
    if (k.cap && i >= k.cap) return;  // never reached: a phase reserves at most qcap slots
    if (k.atomic) {
        uint64_t *p = reinterpret_cast<uint64_t *>(k.q + i);
        __hip_atomic_store(p, (uint64_t)(uint32_t)e.x | ((uint64_t)(uint32_t)e.y << 32), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(p + 1, (uint64_t)(uint32_t)e.z | ((uint64_t)(uint32_t)e.w << 32), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    } else {
        k.q[i] = e;
    }
}

// A consumed (or never written) slot of an atomic queue holds -1 in every
// word; no entry has a negative column or edge start.
constexpr uint64_t kNoEntry = ~0ull;

// Entry i of an atomic queue, which its writer may still be storing: poll
// (agent scope) until both words hold an entry, then leave -1 in the slot
// for the next level that reuses the queue.  Bounded: on the wait limit or
// a status it returns an entry with no edges (the next grid barrier then
// ends the run).
DEV int4 take_entry(int4 *q, uint32_t i, uint32_t *ctrl, uint64_t timeout)
{
    uint64_t *p = reinterpret_cast<uint64_t *>(q + i);
    uint64_t a = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint64_t b = __hip_atomic_load(p + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((int32_t)(uint32_t)a < 0 || (int32_t)(uint32_t)b < 0) {
        const uint64_t t0 = wall_clock64();
        for (;;) {
            __builtin_amdgcn_s_sleep(1);
            a = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            b = __hip_atomic_load(p + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((int32_t)(uint32_t)a >= 0 && (int32_t)(uint32_t)b >= 0) break;
            if (status_of(ctrl) != 0) return make_int4(0, 0, 0, 0);
            if (wall_clock64() - t0 > timeout) { set_status(ctrl, kEInternal); return make_int4(0, 0, 0, 0); }
        }
    }
    __hip_atomic_store(p, kNoEntry, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(p + 1, kNoEntry, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return make_int4((int)(uint32_t)a, (int)(uint32_t)(a >> 32), (int)(uint32_t)b, (int)(uint32_t)(b >> 32));
}

// Hand a wavefront's staged entries to the queue now (its LDS stage is full).
DEV void drain_entries(Stage &st, const QSink &k)
{
    wave_lds_sync();
    uint32_t base = 0;
    if (__lane_id() == 0)
        base = k.c64 ? (uint32_t)__hip_atomic_fetch_add(k.c64, (uint64_t)st.nq, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT)
                     : atomicAdd(k.c32, (uint32_t)st.nq);
    base = __shfl(base, 0, 64);
    for (int i = __lane_id(); i < st.nq; i += 64) put_entry(k, base + i, st.q[i]);
    wave_lds_sync();
    st.dq += st.nq;
    st.nq = 0;
}

// Append frontier entry e for every lane with p set (wavefront-uniform call).
DEV void push_q(bool p, const int4 &e, Stage &st, const QSink &k)
{
    const uint64_t m = __ballot(p);
    if (m == 0) return;
    if (st.nq > kStageQ - 64) drain_entries(st, k);
    if (p) st.q[st.nq + __popcll(m & lanemask_lt())] = e;
    st.nq += __popcll(m);
}

// The staged entries of wavefront w after a deferred flush: they go to
// slots [base + s_tmp[w], ...), base being what the counter barrier's
// addition returned to the workgroup.
DEV void write_deferred(Stage &st, const QSink &k, uint32_t base, const uint32_t *s_tmp)
{
    const uint32_t off = base + s_tmp[threadIdx.x >> 6];
    for (int i = __lane_id(); i < st.nq; i += 64) put_entry(k, off + i, st.q[i]);
    st.nq = 0;
}

// End of a level: every wavefront of the workgroup hands its staged entries
// to the global queues with one atomic per queue for the whole workgroup.
// All threads of the workgroup call it.  Returns what the workgroup added
// since the last flush: frontier entries in the low 31 bits, bit 31 set if
// it added any unmatched-row end.  Deferred (a grid level with F_DEFER):
// the frontier entries stay staged, s_tmp[w] holds wavefront w's offset
// among them, and the count returned is of the staged ones only (entries
// drained earlier were reserved from the barrier counter already); the
// unmatched-row ends are written as usual.
DEV uint32_t block_flush(Stage &st, const QSink &k, int32_t *ge, uint32_t *gecnt, uint32_t *s_tmp, bool defer)
{
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6, lane = __lane_id();
    wave_lds_sync();
    if (lane == 0) {
        s_tmp[w] = (uint32_t)st.nq;
        s_tmp[16 + w] = (uint32_t)st.ne;
        s_tmp[36 + w] = (uint32_t)(defer ? st.nq : st.dq + st.nq) | ((st.de + st.ne) > 0 ? 0x80000000u : 0u);
    }
    __syncthreads();
    if (w == 0) {
        // exclusive prefix of the per-wavefront counts by a wavefront scan
        const int a = lane < nw ? (int)s_tmp[lane] : 0, b = lane < nw ? (int)s_tmp[16 + lane] : 0;
        const uint32_t d = lane < nw ? s_tmp[36 + lane] : 0u;
        const int ia = wave_incl_scan(a), ib = wave_incl_scan(b);
        const uint32_t tq = (uint32_t)__shfl(ia, 63, 64), te = (uint32_t)__shfl(ib, 63, 64);
        const uint32_t added = (uint32_t)wave_sum((uint64_t)(d & 0x7fffffffu));
        const bool any_end = __ballot((d >> 31) != 0) != 0;
        uint32_t bq = 0, be = 0;
        if (lane == 0) {
            if (tq && !defer)
                bq = k.c64 ? (uint32_t)__hip_atomic_fetch_add(k.c64, (uint64_t)tq, __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_AGENT)
                           : atomicAdd(k.c32, tq);
            if (te) be = atomicAdd(gecnt, te);
        }
        if (lane < nw) { s_tmp[lane] = (uint32_t)(ia - a); s_tmp[16 + lane] = (uint32_t)(ib - b); }
        if (lane == 0) { s_tmp[32] = bq; s_tmp[33] = be; s_tmp[34] = added | (any_end ? 0x80000000u : 0u); }
    }
    __syncthreads();
    const uint32_t bq = s_tmp[32] + s_tmp[w], be = s_tmp[33] + s_tmp[16 + w];
    const uint32_t res = s_tmp[34];
    if (!defer) {
        for (int i = lane; i < st.nq; i += 64) put_entry(k, bq + i, st.q[i]);
        st.nq = 0;
    }
    for (int i = lane; i < st.ne; i += 64) put_end(ge, be + i, st.e[i], k.atomic);
    st.ne = 0;
    st.dq = st.de = 0;
    __syncthreads();
    return res;
}

// ---------------------------------------------------------------------
// One scanned edge (col -> r) of the BFS (Algorithm 2 body; Algorithm 4
// adds the root bookkeeping).  A matched, unvisited row is claimed and its
// column becomes a next-frontier entry; an unmatched, unvisited row is
// claimed as an augmenting-path end (rmatch = -2) and marks its root done.
//
// A claim after a probe is a compare-and-swap of the stamp half of the row
// word alone.  During a phase's BFS a row word changes only by claims, and
// every claim sets the stamp to the phase, so a stamp still equal to the
// probed one means an unchanged word.  The mate half stays as it is; an
// end's winner writes -2 there itself (no one reads it before the next grid
// barrier), as with the atomic-maximum claims.

// What a winning claim does (row r reached from column col of root's tree;
// mate = the row's mate, -1 for an end; `put_lo`: the claim left the mate
// half to be written).
template <int S>
DEV void claimed(const DevGraph &g, int col, int root, int r, int mate, int2 adj, bool put_lo, uint32_t ph,
                 int level, uint32_t flags, bool &newcol, int4 &ne, bool &newend, int colmate)
{
    int32_t *lo = reinterpret_cast<int32_t *>(g.rw) + 2 * (size_t)r;
    st_i<S>(&g.pred[r], col);
    if (flags & F_FASTALT) st_i<S>(&g.prow[r], colmate);
    if (mate >= 0) {
        if (put_lo) st_i<S>(lo, mate);
        ne = make_int4(mate, root, adj.x, adj.y);
        newcol = true;
        if (flags & F_LEVELS) {
            g.clevel[mate] = level + 1;
            if (g.croot) g.croot[mate] = root;
        }
    } else if ((flags & F_WR) && (flags & F_ENDPOINT)) {
        // one end per root: the first row reached; a later one returns to
        // unmatched (-1), its stamp keeping it out of this phase
        newend = __hip_atomic_exchange(&g.cdone[root], ph, __ATOMIC_RELAXED, S) != ph;
        st_i<S>(lo, newend ? -2 : -1);
    } else {
        st_i<S>(lo, -2);
        newend = true;
        if (flags & F_WR) st_u<S>(&g.cdone[root], ph);
    }
}

// The claim of a probed row: the stamp found (the probed one when the
// exchange happened).
template <int S>
DEV uint32_t claim_stamp(const DevGraph &g, int r, uint32_t seen, uint32_t ph)
{
    __hip_atomic_compare_exchange_strong(reinterpret_cast<uint32_t *>(g.rw) + 2 * (size_t)r + 1, &seen, ph,
                                         __ATOMIC_RELAXED, __ATOMIC_RELAXED, S);
    return seen;
}

template <int S>
DEV void visit_edge(const DevGraph &g, int col, int root, int r, uint32_t ph, int level, uint32_t flags,
                    bool &newcol, int4 &ne, bool &newend, bool &tried, int colmate)
{
    if (flags & F_MAXCLAIM) {
        // Low-degree rows: one atomic maximum of the phase stamp claims the
        // row and returns its old word (a row already stamped this phase is
        // left as it is); the mate's adjacency range comes from radj, loaded
        // alongside.  Stamps only grow during a run, so exactly one visitor
        // per phase sees an older stamp.  The maximum leaves 0 in the mate
        // half: the winner puts the mate back.
        const int2 adj = g.radj[r];
        const uint64_t old = __hip_atomic_fetch_max(&g.rw[r], (uint64_t)ph << 32, __ATOMIC_RELAXED, S);
        if ((uint32_t)(old >> 32) == ph) return;
        tried = true;
        claimed<S>(g, col, root, r, (int)(uint32_t)old, adj, true, ph, level, flags, newcol, ne, newend, colmate);
        return;
    }
    // agent scope reads the memory-side copy, which other XCDs' claims
    // update; a stale L2 copy would send every scanner of a popular row
    // into a failing compare-and-swap
    const uint64_t w = (S == kAgent) ? __hip_atomic_load(&g.rw[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : g.rw[r];
    const uint32_t seen = (uint32_t)(w >> 32);
    if (seen == ph) return;                           // reached earlier in this phase
    const int mate = (int)(uint32_t)w;
    if (mate < -1) return;
    tried = true;                                     // a compare-and-swap follows
    // adjacency range of the column behind r, fetched alongside the claim
    int2 adj = make_int2(0, 0);
    if (mate >= 0) adj = make_int2(g.colptr[mate], g.colptr[mate + 1]);
    if (claim_stamp<S>(g, r, seen, ph) == seen)
        claimed<S>(g, col, root, r, mate, adj, false, ph, level, flags, newcol, ne, newend, colmate);
}

// Two probed edges per lane (probe claims; wave mapping): the steps of
// visit_edge taken for both edges at once, each step's two memory accesses
// in flight together.  The probes go out for every lane, with or without an
// edge to visit (`on`), so that nothing branches between them, and both
// are decided before either claim goes out (the wavefront's vote on whether
// any claim follows needs both), so that no wait for the second probe falls
// between the claims.
template <int S>
DEV void visit_pair(const DevGraph &g, const int r[2], const bool on[2], uint32_t ph, bool claim[2], int mate[2],
                    int2 adj[2], bool won[2])
{
    uint64_t w[2];
    uint32_t seen[2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
        w[u] = (S == kAgent) ? __hip_atomic_load(&g.rw[r[u]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                             : g.rw[r[u]];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        seen[u] = (uint32_t)(w[u] >> 32);
        mate[u] = (int)(uint32_t)w[u];
        claim[u] = on[u] && seen[u] != ph && mate[u] >= -1;
        won[u] = false;
    }
    if (__ballot(claim[0] || claim[1]) == 0) return;  // a round of rows all reached before
    uint32_t found[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        found[u] = ~seen[u];
        if (claim[u]) {
            if (mate[u] >= 0) adj[u] = make_int2(g.colptr[mate[u]], g.colptr[mate[u] + 1]);
            found[u] = claim_stamp<S>(g, r[u], seen[u], ph);
        }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) won[u] = claim[u] && found[u] == seen[u];
}

struct LevelIO {
    QSink next;         // next frontier
    uint32_t *ecnt;     // ends found in this phase
    uint32_t *found;    // set when this level reached an unmatched row (APsB)
    uint32_t *ctrl;     // status (waits on entries of an atomic queue)
    bool defer;         // deferred flush (F_DEFER grid level)
};

DEV void add_stat(uint64_t *stats, int idx, uint64_t v)
{
    v = wave_sum(v);
    if (__lane_id() == 0 && v) atomicAdd((unsigned long long *)&stats[idx * 16], (unsigned long long)v);
}

// Statistics (stats=1) of one workgroup, kept in LDS so that no register
// holds them through the run: a count is reduced over the wavefront and
// added by its first lane (wavefront-uniform calls, all lanes active); the
// timers (StatIdx S_T_*) are kept by thread 0.  Indices are StatIdx.
constexpr int kAccN = 14;

struct Acc {
    uint64_t *c;  // LDS [kAccN]
    DEV void add(int i, uint64_t v) const
    {
        v = wave_sum(v);
        if (__lane_id() == 0 && v) __hip_atomic_fetch_add(&c[i], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    DEV void tick(int i, uint64_t dt) const
    {
        if (threadIdx.x == 0) c[i] += dt;
    }
    // Adds the counts to the control block's counters (timers too if
    // `timers`); every thread of the workgroup calls it.
    DEV void flush(uint64_t *stats, bool timers) const
    {
        __syncthreads();
        const int i = (int)threadIdx.x;
        if (i < S_T_EXPAND) {
            if (c[i]) atomicAdd((unsigned long long *)&stats[i * 16], (unsigned long long)c[i]);
        } else if (i < kAccN && timers) {
            stats[i * 16] += c[i];
        }
        __syncthreads();
        if (i < kAccN) c[i] = 0;
        __syncthreads();
    }
};

// Zeroed counters (and the level batch counter in the staging scratch,
// when given); every thread of the workgroup calls it.
DEV Acc make_acc(uint64_t *lds, uint32_t *s_tmp = nullptr)
{
    if (threadIdx.x < (unsigned)kAccN) lds[threadIdx.x] = 0;
    if (s_tmp && threadIdx.x == 0) s_tmp[kBatchCtr] = 0;
    __syncthreads();
    return Acc{lds};
}

// Expand frontier entries [0, n) of `fq`; wavefront `wave` of `nwaves`
// takes batches of 64 entries.  WAVE: the edges of the 64 entries are dealt
// out 64 at a time across the lanes (load balanced, coalesced rowind
// reads); otherwise every lane walks its own column's edges.  Every thread
// of the workgroup calls it (it ends with a workgroup flush).
// Entries per wavefront batch: spread a small frontier so that every busy
// wavefront gets about one chunk of edges (latency), a large one in full
// batches of 64 (throughput).
DEV uint32_t batch_size(uint32_t n, uint32_t nwaves, uint32_t bmin)
{
    uint32_t b = (n + nwaves - 1) / nwaves;
    if (b < bmin) b = bmin;
    return b < 1 ? 1u : (b > 64 ? 64u : b);
}

// Push frontier entry `e` (column e.x, root e.y, edges [e.z, e.w)); a column
// with more than `split` edges goes in as consecutive entries of at most
// `split` edges, so that the edges of one heavy column are expanded by
// several wavefronts.  Wavefront-uniform call.
DEV void push_entry(bool p, const int4 &e, uint32_t split, Stage &st, const QSink &q)
{
    const bool heavy = p && split != 0 && (uint32_t)(e.w - e.z) > split;
    if (__ballot(heavy) == 0) {
        push_q(p, e, st, q);
        return;
    }
    const int nch = p ? (heavy ? (int)((e.w - e.z + split - 1) / split) : 1) : 0;
    const int maxk = wave_max(nch);
    for (int k = 0; k < maxk; ++k) {
        const int b = e.z + k * (int)split;
        const int en = heavy ? min(e.w, b + (int)split) : e.w;
        push_q(k < nch, make_int4(e.x, e.y, b, en), st, q);
    }
}

// Expand one frontier entry per lane (lanes with `have`): visit its edges,
// claim rows, stage the columns claimed and the unmatched rows reached.
// Wavefront-uniform call.  `late`: the GPUBFS-WR root test beside each edge
// visit (wave mapping), else before the scan.
template <bool WAVE, int S, bool PAIR = false>
DEV void expand_entries(const DevGraph &g, const int4 e, const bool have, uint32_t ph, int level, uint32_t flags,
                        bool late, const RunOpt &o, const LevelIO &io, Stage &st, Acc &acc, bool &any_end)
{
    const int lane = __lane_id();
    int deg = 0;
    uint32_t rdone = 0;
    int cmate = -1;  // F_FASTALT: the entry column's mate (cmatch does not change during the BFS)
    if (have) {
        deg = e.w - e.z;
        if (flags & F_FASTALT) cmate = g.cmatch[e.x];
        if (late) rdone = ld_u<S>(&g.cdone[e.y]);
        else if ((flags & F_WR) && deg > 0 && ld_u<S>(&g.cdone[e.y]) == ph) deg = 0;
    }
    if (flags & F_STATS) {
        const bool live = !(late && rdone == ph);
        acc.add(S_EDGES, live ? (uint64_t)deg : 0u);
        acc.add(S_EXPANDED, (live && deg > 0) ? 1u : 0u);
    }
    if (WAVE) {
        const int incl = wave_incl_scan(deg);
        const int excl = incl - deg;
        const int total = __shfl(incl, 63, 64);
        // owner lane of edge k of the round: the largest o with excl[o] <= k
        // (excl is non-decreasing); a lane past the last edge takes the last
        // edge's owner (it visits nothing)
        auto owner = [&](int k) -> int {
            const int kk = k < total ? k : total - 1;
            int ow = 0;
#pragma unroll
            for (int step = 32; step >= 1; step >>= 1) {
                const int x = __shfl(excl, ow + step, 64);
                if (x <= kk) ow += step;
            }
            return ow;
        };
        // the row of edge k (the last edge's past the end)
        auto row = [&](int k, int own) -> int {
            const int kk = k < total ? k : total - 1;
            return g.rowind[__shfl(e.z, own, 64) + (kk - __shfl(excl, own, 64))];
        };
        // (every lane takes part in the shuffles: a shuffle from a lane
        // outside a branch reads zero)
        auto live = [&](int k, int own) -> bool {
            const uint32_t odone = late ? (uint32_t)__shfl((int)rdone, own, 64) : 0u;
            return k < total && (!late || odone != ph);
        };
        auto stage = [&](int r, bool newcol, const int4 &ne, bool newend, bool tried) {
            push_entry(newcol, ne, o.split, st, io.next);
            push_end(newend, r, st, g.ends, io.ecnt, io.next.atomic);
            any_end |= newend;
            if (flags & F_STATS) {
                acc.add(S_CLAIMED, newcol ? 1u : 0u);
                acc.add(S_FOUND, newend ? 1u : 0u);
                acc.add(S_TRIES, tried ? 1u : 0u);
            }
        };
        for (int eb = 0; eb < total;) {
            if (PAIR && !(flags & F_MAXCLAIM) && total - eb > 64) {
                // two edges per lane: 128 edges wait for about as many round
                // trips to memory as 64 (rows, probes, claims)
                const int k[2] = {eb + lane, eb + 64 + lane};
                const int own[2] = {owner(k[0]), owner(k[1])};
                const int r[2] = {row(k[0], own[0]), row(k[1], own[1])};
                const bool on[2] = {live(k[0], own[0]), live(k[1], own[1])};
                bool claim[2], won[2];
                int mate[2];
                int2 adj[2] = {make_int2(0, 0), make_int2(0, 0)};
                visit_pair<S>(g, r, on, ph, claim, mate, adj, won);
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int col = __shfl(e.x, own[u], 64), root = __shfl(e.y, own[u], 64);
                    const int omate = (flags & F_FASTALT) ? __shfl(cmate, own[u], 64) : -1;
                    bool newcol = false, newend = false;
                    int4 ne = make_int4(0, 0, 0, 0);
                    if (won[u])
                        claimed<S>(g, col, root, r[u], mate[u], adj[u], false, ph, level, flags, newcol, ne, newend,
                                   omate);
                    stage(r[u], newcol, ne, newend, claim[u]);
                }
                eb += 128;
            } else {
                // (the owner's column, root and mate are shuffled while the
                // row is loaded: low-degree graphs run long chains of such
                // rounds)
                const int k = eb + lane, own = owner(k);
                const int r = row(k, own);
                const int col = __shfl(e.x, own, 64), root = __shfl(e.y, own, 64);
                const int omate = (flags & F_FASTALT) ? __shfl(cmate, own, 64) : -1;
                bool newcol = false, newend = false, tried = false;
                int4 ne = make_int4(0, 0, 0, 0);
                if (live(k, own)) visit_edge<S>(g, col, root, r, ph, level, flags, newcol, ne, newend, tried, omate);
                stage(r, newcol, ne, newend, tried);
                eb += 64;
            }
        }
    } else {
        const int maxdeg = wave_max(deg);
        for (int t = 0; t < maxdeg; ++t) {
            bool newcol = false, newend = false, tried = false;
            int4 ne = make_int4(0, 0, 0, 0);
            int r = 0;
            if (t < deg) {
                r = g.rowind[e.z + t];
                visit_edge<S>(g, e.x, e.y, r, ph, level, flags, newcol, ne, newend, tried, cmate);
            }
            push_entry(newcol, ne, o.split, st, io.next);
            push_end(newend, r, st, g.ends, io.ecnt, io.next.atomic);
            any_end |= newend;
            if (flags & F_STATS) {
                acc.add(S_CLAIMED, newcol ? 1u : 0u);
                acc.add(S_FOUND, newend ? 1u : 0u);
                acc.add(S_TRIES, tried ? 1u : 0u);
            }
        }
    }
}

// SINGLE: a launch for one graph (mcm_match); the others (batches, the
// server's multi-graph launch) compile the recorded-row Alternate out.
// PAIR: the form with two-edge rounds for probe claims (expand_entries),
// which launches for one graph take unless rows are claimed by atomic
// maximum: low-degree graphs run long chains of small rounds, and with the
// two-edge code in their loop they ran 5% slower (grid2048).
// The forms the two-edge level code leaves out (its callers take it only
// without them): atomic-maximum claims, recorded rows, the root test beside
// the edge visit, level records, deferred and level-free levels.  Without
// their registers the level loop fits a 1024-thread workgroup's 128.
constexpr uint32_t kPairOff = F_MAXCLAIM | F_FASTALT | F_WR_LATE | F_LEVELS | F_DEFER | F_ASYNC;
DEV bool pair_form(uint32_t flags) { return (flags & kPairOff) == 0; }

template <bool WAVE, int S, bool SINGLE = true, bool PAIR = false>
DEV uint32_t expand_level(const DevGraph &g, int4 *fq, uint32_t n, uint32_t wave, uint32_t nwaves, uint32_t ph,
                          int level, const RunOpt &o, const LevelIO &io, Stage &st, uint32_t *s_tmp, Acc &acc,
                          uint32_t local = 0)
{
    const int lane = __lane_id();
    const uint32_t flags = PAIR ? (o.flags & ~kPairOff) : SINGLE ? o.flags : (o.flags & ~(uint32_t)F_FASTALT);
    const uint64_t t0 = (flags & F_STATS) ? wall_clock64() : 0;
    bool any_end = false;
    const uint32_t B = batch_size(n, nwaves, o.batch_min);
    // WR: a root that already has a path expands nothing more.  Early: the
    // entry's edges are dropped before the scan (fewer edges, but the scan
    // waits for the cdone load); late (wave mapping): the scan and the
    // rowind loads go ahead and the claims of such an entry are skipped.
    const bool late = WAVE && (flags & F_WR) && (flags & F_WR_LATE);
    // Batches: with at most one per wavefront (small frontiers), wavefront w
    // takes batch w.  With more, the batches of a workgroup are blk,
    // blk + nblk, blk + 2 nblk, ... (interleaved over the workgroups) and its
    // wavefronts take them in turn from an LDS counter, so that a wavefront
    // that drew light batches takes more (R-MAT batches range from 64 to
    // thousands of edges).
    const uint32_t wpb = blockDim.x >> 6, blk = wave / wpb, nblk = nwaves / wpb;
    const bool dyn = (uint64_t)nwaves * B < n;
    uint32_t *ctr = s_tmp + kBatchCtr;
    auto expand = [&](const int4 e, const bool have) {
        expand_entries<WAVE, S, PAIR>(g, e, have, ph, level, flags, late, o, io, st, acc, any_end);
    };
    // one batch of entries [base, base + B) of the frontier
    auto batch = [&](const uint32_t base) {
        const uint32_t i = base + lane;
        const bool have = (uint32_t)lane < B && i < n;
        int4 e = make_int4(0, 0, 0, 0);
        if (have) e = io.next.atomic ? take_entry(fq, i, io.ctrl, o.timeout) : fq[i];
        expand(e, have);
    };
    if (dyn) {
        for (;;) {
            uint32_t k = 0;
            if (lane == 0) k = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            k = __shfl(k, 0, 64);
            const uint64_t base64 = ((uint64_t)blk + (uint64_t)k * nblk) * B;
            if (base64 >= n) break;
            batch((uint32_t)base64);
        }
    } else if (wave * B < n) {
        batch(wave * B);
        // Local levels: the wavefront expands the newest entries it staged
        // (at most 64) itself, up to `local` times, before the level ends.
        // Every claim is still made once, from a column whose row was
        // claimed in the same tree, so the trees stay alternating BFS
        // trees; a column expanded this way is one level early for its tree
        // (levels are then no longer exact, so level-set runs pass 0).
        // A local level takes only the newest entries whose edges add up to
        // at most o.local_edges (at least one entry): the rest stay staged
        // for the next grid level, where every wavefront shares them, rather
        // than one wavefront scanning a thousand edges while the grid waits.
        for (uint32_t k = 0; k < local; ++k) {
            const int m = st.nq < 64 ? st.nq : 64;
            if (m == 0) break;
            wave_lds_sync();
            const int4 e = lane < m ? st.q[st.nq - m + lane] : make_int4(0, 0, 0, 0);
            int t = m;
            if (o.local_edges) {
                // edges of this entry and every newer one (lanes hold the
                // newest m in order, the newest last)
                const int d = lane < m ? e.w - e.z : 0;
                const int incl = wave_incl_scan(d);
                const int newer = __shfl(incl, 63, 64) - (incl - d);
                const uint64_t fit = __ballot(lane < m && (lane == m - 1 || (uint32_t)newer <= o.local_edges));
                t = __popcll(fit);
            }
            const bool have = lane >= m - t && lane < m;
            wave_lds_sync();
            st.nq -= t;
            expand(e, have);
        }
    }
    if ((flags & F_APSB) && __ballot(any_end) != 0 && lane == 0) atomicOr(io.found, 1u);
    const uint64_t t1 = (flags & F_STATS) ? wall_clock64() : 0;
    const uint32_t added = block_flush(st, io.next, g.ends, io.ecnt, s_tmp, io.defer);
    if (threadIdx.x == 0) *ctr = 0;  // every wavefront is past it (the flush ends with a barrier)
    if (flags & F_STATS) { acc.tick(S_T_EXPAND, t1 - t0); acc.tick(S_T_FLUSH, wall_clock64() - t1); }
    return added;
}

// ---------------------------------------------------------------------
// Level-free BFS of one APFB phase.  All frontier entries of the phase go
// through one queue (fq0, 2 * qcap slots, each used at most once per
// phase); wavefronts take entries as soon as they are written and expand
// the columns they claim themselves (their LDS stage is their local work
// list), so no grid barrier separates BFS levels.  A wavefront keeps at
// at most o.keep entries and hands older ones to the queue, where idle
// wavefronts take them.  One 64-bit control word counts the entries
// reserved in the queue (low half) and finished (high half): a wavefront
// finishes the entries it took only once its stage is empty again (every
// column they led to is expanded or handed on, and handing on reserves
// first), so equal halves mean that no entry is held anywhere and none can
// appear; the phase's BFS is then complete.  The trees stay alternating
// trees (each row is still claimed once per phase, from a column of the
// claimer's tree); they are no longer shortest-path trees, and the maximum
// is still certified, because a phase that finds no unmatched row has
// explored everything reachable from the unmatched columns.
// Hand the oldest entries of a wavefront's stage to the queue, keeping the
// newest `keep` (wavefront-uniform call).
DEV void drain_older(Stage &st, const QSink &k, int keep)
{
    const int n = st.nq - keep;
    if (n <= 0) return;
    wave_lds_sync();
    uint32_t base = 0;
    if (__lane_id() == 0)
        base = (uint32_t)__hip_atomic_fetch_add(k.c64, (uint64_t)n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    base = __shfl(base, 0, 64);
    for (int i = __lane_id(); i < n; i += 64) put_entry(k, base + i, st.q[i]);
    // move the kept entries to the front (they are the last `keep`, at most
    // 64 lanes x 2 rounds)
    int4 kept[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int i = __lane_id() + 64 * u;
        kept[u] = i < keep ? st.q[n + i] : make_int4(0, 0, 0, 0);
    }
    wave_lds_sync();
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int i = __lane_id() + 64 * u;
        if (i < keep) st.q[i] = kept[u];
    }
    wave_lds_sync();
    st.dq += n;
    st.nq = keep;
}

template <bool WAVE>
DEV void async_bfs(const DevGraph &g, uint32_t *ctrl, const RunOpt &o, uint32_t ph, uint32_t nwaves, Stage &st,
                   Acc &acc)
{
    const int lane = __lane_id();
    const uint32_t flags = o.flags;
    const bool late = WAVE && (flags & F_WR) && (flags & F_WR_LATE);
    uint64_t *aq = reinterpret_cast<uint64_t *>(line(ctrl, L_AQ));
    uint32_t *take = line(ctrl, L_AQ_TAKE);
    const QSink sink{g.fq0, nullptr, aq, true, 2 * g.qcap};
    const LevelIO io{sink, line(ctrl, L_NENDS), nullptr, ctrl, false};
    bool any_end = false;
    uint32_t held = 0;
    const uint64_t t0 = wall_clock64();
    uint32_t naps = 0;
    for (;;) {
        if (st.nq > 0) {
            // the newest (at most o.take) of the entries this wavefront keeps
            const int m = st.nq < (int)o.take ? st.nq : (int)o.take;
            wave_lds_sync();
            const bool have = lane < m;
            const int4 e = have ? st.q[st.nq - m + lane] : make_int4(0, 0, 0, 0);
            wave_lds_sync();
            st.nq -= m;
            expand_entries<WAVE, kAgent>(g, e, have, ph, 0, flags, late, o, io, st, acc, any_end);
            if (st.nq > (int)o.keep) drain_older(st, sink, (int)o.take);
            continue;
        }
        // stage empty: the entries taken are finished
        if (held) {
            if (lane == 0)
                __hip_atomic_fetch_add(aq, (uint64_t)held << 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            held = 0;
        }
        // take entries from the queue: slots [t, t + n), all reserved
        uint32_t t = 0, n = 0;
        int done = 0;
        if (lane == 0) {
            for (;;) {
                const uint32_t tk = ld_u<kAgent>(take);
                const uint64_t w = __hip_atomic_load(aq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t r = (uint32_t)w;
                if (r > 2 * g.qcap) { set_status(ctrl, kEInternal); done = 1; break; }  // never: see put_entry
                if (tk < r) {
                    n = batch_size(r - tk, nwaves, o.batch_min);
                    if (n > r - tk) n = r - tk;
                    uint32_t expect = tk;
                    if (__hip_atomic_compare_exchange_strong(take, &expect, tk + n, __ATOMIC_RELAXED,
                                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        t = tk;
                        naps = 0;
                        break;
                    }
                    continue;
                }
                if ((uint32_t)(w >> 32) == r) { done = 1; break; }  // all reserved entries finished
                if (status_of(ctrl) != 0) { done = 1; break; }
                if (wall_clock64() - t0 > o.timeout) { set_status(ctrl, kEInternal); done = 1; break; }
                // idle: back off (up to 64 s_sleep units)
                for (uint32_t k = 0; k < (1u << (naps < 6 ? naps : 6)); ++k) __builtin_amdgcn_s_sleep(1);
                ++naps;
            }
        }
        if (__shfl(done, 0, 64)) break;
        t = (uint32_t)__shfl((int)t, 0, 64);
        n = (uint32_t)__shfl((int)n, 0, 64);
        const bool have = (uint32_t)lane < n;
        const int4 e = have ? take_entry(g.fq0, t + lane, ctrl, o.timeout) : make_int4(0, 0, 0, 0);
        held = n;
        expand_entries<WAVE, kAgent>(g, e, have, ph, 0, flags, late, o, io, st, acc, any_end);
        if (st.nq > (int)o.keep) drain_older(st, sink, (int)o.take);
    }
    // the unmatched rows this wavefront reached and still stages
    if (st.ne) drain_ends(st, g.ends, io.ecnt, true);
    st.dq = st.de = 0;
    if ((flags & F_STATS) && threadIdx.x == 0) acc.tick(S_T_EXPAND, wall_clock64() - t0);
}

// InitBfsArray (paper, section 3, before Algorithm 2; root filled as in
// Algorithm 4): every unmatched column with at least one edge becomes a
// root and an entry of the first frontier.  Columns without edges can never
// be matched and would expand nothing.  Every thread of the workgroup calls
// it.
//
// Root lists (LIST, the launch for one graph, with g.rlist): a matched
// column never becomes unmatched again, so the roots of a phase are among
// those of the one before.  A phase whose predecessor had at most
// o.roots_max roots ("active"; phase 1: whose initial matching left at most
// that many columns unmatched) lists its roots in half ph & 1 of g.rlist;
// an active phase whose predecessor was active too scans only that
// predecessor's list instead of every column.  Reading a listed root
// gathers three words, so with many roots scanning every column is
// cheaper, and writing a list that the next phase would not read is
// skipped.  Every phase counts its roots in the low 31 bits of
// L_NRL0/L_NRL1 (by phase parity); bit 31 marks an active phase.  The
// count is also every workgroup's place in the list (atomicAdd), so the
// caller sets the mark only after the grid barrier that ends the scan
// (mark_active_phase).  Returns whether the phase is active.  The other
// launches scan every column and spare the registers.
template <bool LIST = false>
DEV bool init_roots(const DevGraph &g, uint32_t wave, uint32_t nwaves, const RunOpt &o, uint32_t *cnt, Stage &st,
                    uint32_t *s_tmp, Acc &acc, uint64_t *c64 = nullptr, uint32_t ph = 1, uint32_t *ctrl = nullptr)
{
    // the level-free BFS reserves root slots from its phase-long counter
    const QSink q = c64 ? QSink{g.fq0, nullptr, c64, true, 2 * g.qcap}
                        : QSink{g.fq0, cnt, nullptr, (o.flags & F_DEFER) != 0};
    const int lane = __lane_id();
    const uint32_t flags = o.flags;
    const uint32_t nc = (uint32_t)g.nc;
    if constexpr (!LIST) {
        // Every column, one pass: roots staged per wavefront and reserved
        // per stage drain (the launches for many graphs, whose register
        // budget has no room for the two-pass form below).
        for (uint32_t base = wave * 64u * kStream; base < nc; base += nwaves * 64u * kStream) {
            int cm[kStream], b[kStream], en[kStream];
#pragma unroll
            for (int u = 0; u < kStream; ++u) {
                const uint32_t c = min(base + 64u * u + (uint32_t)lane, nc - 1);
                cm[u] = g.cmatch[c];
                b[u] = g.colptr[c];
                en[u] = g.colptr[c + 1];
            }
#pragma unroll
            for (int u = 0; u < kStream; ++u) {
                const uint32_t c = base + 64u * u + (uint32_t)lane;
                const bool in = c < nc, un = in && cm[u] == -1;
                const bool p = un && en[u] > b[u];
                if ((flags & F_LEVELS) && in) {
                    g.clevel[c] = un ? 0 : -1;
                    if (g.croot) g.croot[c] = un ? (int)c : -1;
                }
                if (flags & F_STATS) acc.add(S_ROOTS, p ? 1u : 0u);
                push_entry(p, make_int4((int)c, (int)c, b[u], en[u]), o.split, st, q);
            }
        }
        if ((flags & F_STATS) && threadIdx.x == 0 && wave == 0) acc.tick(S_PASS, 4ull * nc + nc / 8);
        block_flush(st, q, g.ends, nullptr, s_tmp, false);
        return false;
    }
    const bool lists = LIST && g.rlist && ctrl;
    uint32_t *rl_cnt = lists ? line(ctrl, (ph & 1) ? L_NRL1 : L_NRL0) : nullptr;
    bool active = false, read = false;
    uint32_t nprev = 0;
    if (lists) {
        if (ph > 1) {
            const uint32_t w = ld_u<kAgent>(line(ctrl, ((ph - 1) & 1) ? L_NRL1 : L_NRL0));
            nprev = w & 0x7fffffffu;
            active = nprev <= o.roots_max;
            read = active && (w >> 31) != 0;
        } else {
            const uint64_t m0 = __hip_atomic_load(reinterpret_cast<uint64_t *>(line(ctrl, L_INIT_CARD)),
                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            active = (uint64_t)nc - m0 <= (uint64_t)o.roots_max;
        }
    }
    int32_t *rl_out = active ? g.rlist + (size_t)(ph & 1) * nc : nullptr;
    const int32_t *rl_in = read ? g.rlist + (size_t)((ph - 1) & 1) * nc : nullptr;
    // the columns to scan: the previous phase's roots, or all of them
    const uint32_t n = rl_in ? nprev : nc;
    const uint32_t split = o.split;
    // Two passes over the same columns: the first counts the frontier
    // entries (a root of more than `split` edges enters as several) and the
    // roots, one reservation per workgroup follows, and the second writes
    // entries (and listed roots) at their places.  One counter atomic per
    // workgroup instead of one per wavefront stage drain: with millions of
    // roots (rmat23) the drains' same-address atomics dominated the scan.
    // kStream chunks of 64 columns per wavefront and step, their loads
    // issued together (indices clamped, so every load is in bounds and
    // unconditional; a clamped lane is masked afterwards).
    auto scan = [&](auto &&visit) {
        for (uint32_t base = wave * 64u * kStream; base < n; base += nwaves * 64u * kStream) {
            int col[kStream], cm[kStream], b[kStream], en[kStream];
#pragma unroll
            for (int u = 0; u < kStream; ++u) {
                const uint32_t i = min(base + 64u * u + (uint32_t)lane, n - 1);
                col[u] = rl_in ? rl_in[i] : (int)i;
            }
#pragma unroll
            for (int u = 0; u < kStream; ++u) {
                cm[u] = g.cmatch[col[u]];
                b[u] = g.colptr[col[u]];
                en[u] = g.colptr[col[u] + 1];
            }
#pragma unroll
            for (int u = 0; u < kStream; ++u) {
                const bool in = base + 64u * u + (uint32_t)lane < n, un = in && cm[u] == -1;
                const bool p = un && en[u] > b[u];
                const uint32_t deg = p ? (uint32_t)(en[u] - b[u]) : 0u;
                const uint32_t nent = p ? ((split && deg > split) ? (deg + split - 1) / split : 1u) : 0u;
                visit(col[u], in, un, p, b[u], en[u], nent);
            }
        }
    };
    // pass 1: entries and roots of this wavefront (uniform sums)
    uint32_t went = 0, wroots = 0;
    scan([&](int, bool, bool, bool p, int, int, uint32_t nent) {
        went += (uint32_t)wave_sum((uint64_t)nent);
        wroots += (uint32_t)__popcll(__ballot(p));
    });
    // reservation: wavefront offsets by a scan in the workgroup, one atomic
    // per workgroup on the frontier counter and one on the root count
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane == 0) { s_tmp[w] = went; s_tmp[16 + w] = wroots; }
    __syncthreads();
    if (w == 0) {
        const int a = lane < nw ? (int)s_tmp[lane] : 0, r = lane < nw ? (int)s_tmp[16 + lane] : 0;
        const int ia = wave_incl_scan(a), ir = wave_incl_scan(r);
        const uint32_t ta = (uint32_t)__shfl(ia, 63, 64), tr = (uint32_t)__shfl(ir, 63, 64);
        uint32_t qb = 0, rb = 0;
        if (lane == 0) {
            if (ta) qb = q.c64 ? (uint32_t)__hip_atomic_fetch_add(q.c64, (uint64_t)ta, __ATOMIC_RELAXED,
                                                                  __HIP_MEMORY_SCOPE_AGENT)
                               : atomicAdd(q.c32, ta);
            if (tr && lists) rb = atomicAdd(rl_cnt, tr);
        }
        qb = (uint32_t)__shfl((int)qb, 0, 64);
        rb = (uint32_t)__shfl((int)rb, 0, 64);
        if (lane < nw) { s_tmp[32 + lane] = qb + (uint32_t)(ia - a); s_tmp[48 + lane] = rb + (uint32_t)(ir - r); }
    }
    __syncthreads();
    uint32_t qoff = s_tmp[32 + w], roff = s_tmp[48 + w];
    __syncthreads();
    // words 32..63 of s_tmp served the offsets; the level batch counter
    // among them starts every level at zero
    if (threadIdx.x == 0) s_tmp[kBatchCtr] = 0;
    // pass 2: the same columns, written at their places
    scan([&](int c, bool in, bool un, bool p, int b, int en, uint32_t nent) {
        const int incl = wave_incl_scan((int)nent);
        uint32_t at = qoff + (uint32_t)(incl - (int)nent);
        for (uint32_t k = 0; k < nent; ++k) {
            const int eb = b + (int)(k * split);
            const int ee = (nent > 1 && eb + (int)split < en) ? eb + (int)split : en;
            put_entry(q, at + k, make_int4(c, c, eb, ee));
        }
        qoff += (uint32_t)__shfl(incl, 63, 64);
        const uint64_t m = __ballot(p);
        if (active && p) put_end(rl_out, roff + (uint32_t)__popcll(m & lanemask_lt()), c, q.atomic);
        roff += (uint32_t)__popcll(m);
        if ((flags & F_LEVELS) && in) {
            g.clevel[c] = un ? 0 : -1;
            if (g.croot) g.croot[c] = un ? c : -1;
        }
        if (flags & F_STATS) acc.add(S_ROOTS, p ? 1u : 0u);
    });
    if ((flags & F_STATS) && threadIdx.x == 0 && wave == 0) acc.tick(S_PASS, 4ull * n + nc / 8);
    // nothing staged, and nothing counted as drained for the first level's
    // flush (its count of entries and its "reached an unmatched row" bit,
    // which stops an APsB level loop, start from zero here)
    st.nq = st.ne = 0;
    st.dq = st.de = 0;
    __syncthreads();
    return active;
}

// Whether phase ph lists its roots (the previous phase had at most
// o.roots_max of them; phase 1: the initial matching leaves at most that many
// columns unmatched).  Every block reads the same counts.
DEV bool roots_listed(const DevGraph &g, const RunOpt &o, uint32_t ph, uint32_t *ctrl)
{
    if (!g.rlist) return false;
    if (ph > 1) return (ld_u<kAgent>(line(ctrl, ((ph - 1) & 1) ? L_NRL1 : L_NRL0)) & 0x7fffffffu) <= o.roots_max;
    const uint64_t m0 = __hip_atomic_load(reinterpret_cast<uint64_t *>(line(ctrl, L_INIT_CARD)), __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
    return (uint64_t)g.nc - m0 <= (uint64_t)o.roots_max;
}

// LDS of the persistent kernel: the wavefront stages, and kRootQ root
// entries per wavefront for roots_level0 (up to 63 left from a step plus one
// step's 64 kStream columns).
constexpr int kRootQ = 64 * (kStream + 1);
inline constexpr int persistent_lds_bytes(int waves) { return stage_lds_bytes(waves) + waves * kRootQ * 16; }

// The root scan and BFS level 0 in one pass (F_FUSE0; a phase that does not
// list its roots): a wavefront gathers the roots of its columns (unmatched
// columns with edges) in LDS, 64 at a time, and expands them as a level-0
// frontier batch at once, instead of writing them to the frontier queue for
// a level that reads them back after one more grid barrier.  Level 1's
// entries go to fq1, as level 0's would.  Every wavefront still expands
// every root before the barrier that ends the pass, so the level sets are
// those of level 0.  Returns the workgroup's share for that barrier: the
// entries it added to level 1 (low 31 bits) and whether it reached an
// unmatched row (bit 31).  Counts the phase's roots into its root-list
// count (one addition per workgroup).
template <bool WAVE, bool PAIR>
DEV uint32_t roots_level0(const DevGraph &g, uint32_t wave, uint32_t nwaves, const RunOpt &o, uint32_t ph,
                          uint32_t *ctrl, Stage &st, uint32_t *s_tmp, Acc &acc)
{
    constexpr int kRootCnt = 53;  // s_tmp word: the workgroup's roots
    const int lane = __lane_id();
    const uint32_t flags = PAIR ? (o.flags & ~kPairOff) : o.flags;
    const uint32_t nc = (uint32_t)g.nc;
    const QSink next{g.fq1, line(ctrl, L_FCOUNT1), nullptr, false};
    const LevelIO io{next, line(ctrl, L_NENDS), line(ctrl, L_FOUND0), ctrl, false};
    const bool late = WAVE && (flags & F_WR) && (flags & F_WR_LATE);
    // this wavefront's root entries follow the stages' 64 words
    int4 *rq = reinterpret_cast<int4 *>(reinterpret_cast<char *>(s_tmp) + 64 * 4) + (threadIdx.x >> 6) * kRootQ;
    // nothing staged or counted as drained from before (Alternate's reports
    // use the stage of ends)
    st.nq = st.ne = 0;
    st.dq = st.de = 0;
    if (threadIdx.x == 0) s_tmp[kRootCnt] = 0;
    __syncthreads();
    bool any_end = false;
    int fill = 0;  // root entries gathered in rq (wavefront-uniform)
    // expands the newest n (<= 64) gathered entries
    auto expand = [&](int n) {
        wave_lds_sync();
        const bool have = lane < n;
        const int4 e = have ? rq[fill - n + lane] : make_int4(0, 0, 0, 0);
        wave_lds_sync();
        fill -= n;
        expand_entries<WAVE, kAgent, PAIR>(g, e, have, ph, 0, flags, late, o, io, st, acc, any_end);
    };
    for (uint32_t base = wave * 64u * kStream; base < nc; base += nwaves * 64u * kStream) {
        int cm[kStream], b[kStream], en[kStream];
#pragma unroll
        for (int u = 0; u < kStream; ++u) {
            const uint32_t c = min(base + 64u * u + (uint32_t)lane, nc - 1);
            cm[u] = g.cmatch[c];
            b[u] = g.colptr[c];
            en[u] = g.colptr[c + 1];
        }
        // the step's roots are gathered first (its loads' registers are free
        // again before any expansion), then expanded 64 at a time
#pragma unroll
        for (int u = 0; u < kStream; ++u) {
            const uint32_t c = base + 64u * u + (uint32_t)lane;
            const bool p = c < nc && cm[u] == -1 && en[u] > b[u];
            const uint64_t m = __ballot(p);
            if (p) rq[fill + (int)__popcll(m & lanemask_lt())] = make_int4((int)c, (int)c, b[u], en[u]);
            if (lane == 0 && m) atomicAdd(&s_tmp[kRootCnt], (uint32_t)__popcll(m));
            fill += __popcll(m);
            if (flags & F_STATS) acc.add(S_ROOTS, p ? 1u : 0u);
        }
        while (fill >= 64) expand(64);
    }
    if (fill) expand(fill);
    if ((flags & F_STATS) && threadIdx.x == 0 && wave == 0) acc.tick(S_PASS, 4ull * nc + nc / 8);
    if ((flags & F_APSB) && __ballot(any_end) != 0 && lane == 0) atomicOr(io.found, 1u);
    const uint32_t added = block_flush(st, next, g.ends, io.ecnt, s_tmp, false);
    if (threadIdx.x == 0) {
        if (g.rlist && s_tmp[kRootCnt]) atomicAdd(line(ctrl, (ph & 1) ? L_NRL1 : L_NRL0), s_tmp[kRootCnt]);
        s_tmp[kBatchCtr] = 0;
    }
    return added;
}

// After the grid barrier that ends phase ph's root scan (no workgroup adds
// to the count any more): mark the phase as active for the next one.
DEV void mark_active_phase(uint32_t *ctrl, uint32_t ph)
{
    atomicOr(line(ctrl, (ph & 1) ? L_NRL1 : L_NRL0), 0x80000000u);
}

// Alternate (Algorithm 3) from every reached unmatched row, one thread per
// row.  A walk that reaches a root (its column has no mate) ends there.
// A pointer that is the same in every lane of the wave (every caller's graph
// is one per workgroup or per grid), moved into scalar registers and hidden
// from the optimiser, which then cannot hoist addresses derived from it out
// of the loop around the call.
DEV const int32_t *fresh_uniform(const int32_t *p)
{
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    asm volatile("" : "+s"(lo), "+s"(hi));
    return reinterpret_cast<const int32_t *>(((uint64_t)hi << 32) | lo);
}

template <int S>
DEV void alternate(const DevGraph &g, uint32_t nends, uint32_t tid, uint32_t nthreads, uint32_t flags,
                   uint32_t *ctrl, Acc &acc)
{
    // the list of ends is read through a pointer the compiler takes as new
    // in every call, so that no per-lane address into it stays live (and
    // spilled) through a whole persistent loop
    const int32_t *ends = fresh_uniform(g.ends);
    uint64_t steps = 0;
    int32_t *rlo = reinterpret_cast<int32_t *>(g.rw);  // low word of rw[r] is rlo[2r]
    if (flags & F_FASTALT) {
        // The claim recorded, next to pred[r], the row prow[r] that held
        // pred[r] during the BFS, so a step loads the two together instead
        // of cmatch[pred[r]] after pred[r].  Without reading cmatch a walk
        // cannot see another walk's flips: where several ends of one tree
        // share the way to the root, each walk flips the shared part with
        // the same values; at the column where they join, the last flip
        // wins and FixMatching unmatches the other walk's row, as it does
        // for a walk that stops there.
        for (uint32_t i = tid; i < nends; i += nthreads) {
            int r = ends[i];
            int c = ld_i<S>(&g.pred[r]);
            int r2 = ld_i<S>(&g.prow[r]);
            uint32_t guard = 0;
            for (;;) {
                // the next row's pair is loaded with this column's range
                // (pred and prow do not change during Alternate)
                int nc2 = 0, nr2 = -1;
                if (r2 != -1) {
                    nc2 = ld_i<S>(&g.pred[r2]);
                    nr2 = ld_i<S>(&g.prow[r2]);
                }
                int2 adj = make_int2(0, 0);
                if (flags & F_MAXCLAIM) adj = make_int2(g.colptr[c], g.colptr[c + 1]);
                st_i<S>(&g.cmatch[c], r);
                st_i<S>(&rlo[2 * (size_t)r], c);
                if (flags & F_MAXCLAIM) g.radj[r] = adj;
                ++steps;
                if (r2 == -1) break;  // c was a root
                r = r2;
                c = nc2;
                r2 = nr2;
                if (++guard > (uint32_t)g.nc + 1u) { set_status(ctrl, kEInternal); break; }
            }
        }
        if (flags & F_STATS) acc.add(S_ALT, steps);
        return;
    }
    for (uint32_t i = tid; i < nends; i += nthreads) {
        int r = ends[i];
        int c = ld_i<S>(&g.pred[r]);
        uint32_t guard = 0;
        for (;;) {
            const int r2 = ld_i<S>(&g.cmatch[c]);
            // pred[r2] is both the conflict check and the next step's column
            // (pred does not change during Alternate): one load for the two
            const int c2 = r2 != -1 ? ld_i<S>(&g.pred[r2]) : -1;
            if (r2 != -1 && c2 == c) break;  // c already flipped by another walk
            st_i<S>(&g.cmatch[c], r);
            st_i<S>(&rlo[2 * (size_t)r], c);
            // every walk through r writes the same column (pred[r]), so the
            // range always belongs to the row's mate
            if (flags & F_MAXCLAIM) g.radj[r] = make_int2(g.colptr[c], g.colptr[c + 1]);
            ++steps;
            if (r2 == -1) break;             // reached the root
            r = r2;
            c = c2;
            if (++guard > (uint32_t)g.nc + 1u) { set_status(ctrl, kEInternal); break; }
        }
    }
    if (flags & F_STATS) acc.add(S_ALT, steps);
}

// Alternate as above, every walk also reporting each row it wrote, and the
// row a classic walk stops at (whose column it leaves pointing elsewhere),
// to the phase's list g.touched (counted in *tcnt), so that FixMatching
// visits only those rows.  Each lane walks one end at a time and takes its
// next end when its walk is done; the loop runs while any lane of the
// wavefront walks, and reports are compacted per wavefront in LDS (the
// stage of ends, empty after the BFS).  Wavefront-uniform call.
template <int S>
DEV void alternate_listed(const DevGraph &g, uint32_t nends, uint32_t tid, uint32_t nthreads, uint32_t flags,
                          uint32_t *ctrl, Acc &acc, Stage &st, uint32_t *tcnt)
{
    const int32_t *ends = fresh_uniform(g.ends);  // as in alternate
    uint64_t steps = 0;
    int32_t *rlo = reinterpret_cast<int32_t *>(g.rw);
    const bool fast = (flags & F_FASTALT) != 0;
    uint32_t i = tid, guard = 0;
    bool active = i < nends;
    // r: the walk's row; c: its column (pred[r]); fast walks also hold
    // r2 = prow[r], the next row (pred and prow do not change during
    // Alternate, so a step loads the next row's pair together with its own
    // column's range: one round trip per step)
    int r = 0, c = 0, r2 = -1;
    auto start = [&]() {
        r = ends[i];
        c = ld_i<S>(&g.pred[r]);
        if (fast) r2 = ld_i<S>(&g.prow[r]);
    };
    if (active) start();
    while (__ballot(active)) {
        int touched = -1;
        if (active) {
            bool done = false;
            if (fast) {
                int nc2 = 0, nr2 = -1;
                if (r2 != -1) {
                    nc2 = ld_i<S>(&g.pred[r2]);
                    nr2 = ld_i<S>(&g.prow[r2]);
                }
                int2 adj = make_int2(0, 0);
                if (flags & F_MAXCLAIM) adj = make_int2(g.colptr[c], g.colptr[c + 1]);
                st_i<S>(&g.cmatch[c], r);
                st_i<S>(&rlo[2 * (size_t)r], c);
                if (flags & F_MAXCLAIM) g.radj[r] = adj;
                ++steps;
                touched = r;
                if (r2 == -1) done = true;
                else { r = r2; c = nc2; r2 = nr2; }
            } else {
                const int r2 = ld_i<S>(&g.cmatch[c]);
                const int c2 = r2 != -1 ? ld_i<S>(&g.pred[r2]) : -1;
                touched = r;
                if (r2 != -1 && c2 == c) {
                    done = true;  // c already flipped by another walk; r keeps its old column
                } else {
                    st_i<S>(&g.cmatch[c], r);
                    st_i<S>(&rlo[2 * (size_t)r], c);
                    if (flags & F_MAXCLAIM) g.radj[r] = make_int2(g.colptr[c], g.colptr[c + 1]);
                    ++steps;
                    if (r2 == -1) done = true;
                    else { r = r2; c = c2; }
                }
            }
            if (!done && ++guard > (uint32_t)g.nc + 1u) { set_status(ctrl, kEInternal); done = true; }
            if (done) {
                i += nthreads;
                guard = 0;
                active = i < nends;
                if (active) start();
            }
        }
        push_end(touched >= 0, touched, st, g.touched, tcnt, true, (uint32_t)g.nr);
    }
    if (st.ne) drain_ends(st, g.touched, tcnt, true, (uint32_t)g.nr);
    st.de = 0;  // the reports are no level's unmatched rows
    if (flags & F_STATS) acc.add(S_ALT, steps);
}

// FixMatching over the rows the walks reported (duplicates are harmless:
// the rule only ever writes -1): the same rule as fix_matching.
DEV void fix_listed(const DevGraph &g, uint32_t n, uint32_t tid, uint32_t nthreads, uint32_t flags, Acc &acc)
{
    uint64_t resets = 0;
    int32_t *rlo = reinterpret_cast<int32_t *>(g.rw);
    for (uint32_t i = tid; i < n; i += nthreads) {
        const int r = g.touched[i];
        const int m = rlo[2 * (size_t)r];
        if (m == -1) continue;
        if (m < 0 || g.cmatch[m] != r) { rlo[2 * (size_t)r] = -1; resets += (m >= 0); }
    }
    if (flags & F_STATS) acc.add(S_FIX, resets);
}

// FixMatching: a row whose column points elsewhere lost a race and is
// unmatched; a row still marked -2 (its walk stopped before reaching it)
// returns to -1.  cmatch is not touched.  Only rows claimed in phase `ph`
// can be left so: every row a walk writes, stops at or leaves behind (the
// old mate of a flipped column is the walk's next row) was claimed in the
// phase, and so was every end marked -2.  The others keep a mate that
// points back, and their mate's column is not gathered (ph = 0: every
// matched row is checked).
DEV void fix_matching(const DevGraph &g, uint32_t ph, uint32_t tid, uint32_t nthreads, uint32_t flags, Acc &acc)
{
    uint64_t resets = 0;
    int32_t *rlo = reinterpret_cast<int32_t *>(g.rw);
    const uint32_t nr = (uint32_t)g.nr;
    // kStream rows per thread and step: their words, then their columns'
    // mates, loaded together (clamped indices, masked afterwards)
    for (uint32_t r0 = tid; r0 < nr; r0 += nthreads * kStream) {
        uint64_t w[kStream];
        int cm[kStream];
#pragma unroll
        for (int u = 0; u < kStream; ++u) w[u] = g.rw[min(r0 + u * nthreads, nr - 1)];
#pragma unroll
        for (int u = 0; u < kStream; ++u) {
            const int m = (int)(uint32_t)w[u];
            cm[u] = (m >= 0 && (ph == 0 || (uint32_t)(w[u] >> 32) == ph)) ? g.cmatch[m] : (int)(r0 + u * nthreads);
        }
#pragma unroll
        for (int u = 0; u < kStream; ++u) {
            const uint32_t r = r0 + u * nthreads;
            const int m = (int)(uint32_t)w[u];
            if (r >= nr || m == -1) continue;
            if (m < 0 || cm[u] != (int)r) { rlo[2 * (size_t)r] = -1; resets += (m >= 0); }
        }
    }
    if (flags & F_STATS) acc.add(S_FIX, resets);
}

// ---------------------------------------------------------------------
// Grid barrier of the cooperative launch.  Blocks 1 .. active-1 publish
// their arrival in their own flag line (no shared counter, no contention);
// wave 0 of block 0 polls those flags and then releases the next epoch
// together with the state of the level loop (level L, frontier size n, APsB
// stop flag), which it reads from counters once every arrival is in, or is
// given.  Blocks at or above `active` did nothing since their last barrier
// and do not arrive: block 0 may release further epochs before they look,
// so the state travels with the epoch and a late block adopts the latest
// one.  Two 64-bit words carry it: B = {epoch, L | stop << 31} is stored
// first, then A = {epoch, n} with release; a reader takes A, then B, and
// accepts the pair when both name the same epoch.  Agent-scope release
// before arriving; acquire after leaving, but only where `touches(state)`
// says the block will read data the others wrote before its next barrier
// (an acquire invalidates the XCD's L2 under the blocks still working
// there, so the blocks that sit the next level out skip it; their next
// acquire, when they take part again, orders everything released before).
// Every wait is bounded.  Returns false (in all blocks, eventually) once
// any block set a status.
// The blocks that synchronise: block `b` of a group of `n` (the whole grid,
// or one graph's share of a multi-graph launch).
struct Grp {
    uint32_t b, n;
};

struct LvState {
    uint32_t L, n, stop;
};

// What block 0 releases: L, and n and stop either given or read from a
// counter once every arrival is in; with `sum`, n and stop are block 0's
// own share, and every arriving block adds its share (carried in its
// arrival word: entries added in the low 31 bits, bit 31 = reached an
// unmatched row and the loop stops there).
struct Pub {
    uint32_t L, n, stop;
    const uint32_t *n_ptr, *stop_ptr;
    bool sum;
};

// Wait (thread 0) until block 0 or the last arrival has released `epoch`
// or a later one, and take the state it released; the acquire only where
// `touches` says so.  Returns false on a status or the wait limit.
template <class Touches>
DEV bool wait_release(uint32_t *ctrl, const uint64_t *wa, const uint64_t *wb, uint32_t epoch, uint64_t timeout,
                      bool arrived, uint32_t idle_sleep, Touches touches, uint32_t *s_st)
{
    const uint64_t t0 = wall_clock64();
    for (;;) {
        const uint64_t a = __hip_atomic_load(wa, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((int32_t)((uint32_t)a - epoch) >= 0) {
            // only a pair naming one epoch is taken: a stale B (or a newer
            // one) sends the reader round again
            const uint64_t w = __hip_atomic_load(wb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((uint32_t)w == (uint32_t)a) {
                const LvState x{(uint32_t)(w >> 32) & 0x7fffffffu, (uint32_t)(a >> 32), (uint32_t)(w >> 63)};
                if (touches(x)) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                s_st[0] = x.L;
                s_st[1] = x.n;
                s_st[2] = x.stop;
                s_st[3] = (uint32_t)a;
                return true;
            }
            continue;  // the releaser moved on between the two loads: read both again
        }
        if (status_of(ctrl) != 0) return false;
        if (wall_clock64() - t0 > timeout) { set_status(ctrl, kEInternal); return false; }
        // a block that did not arrive polls less often: many of them
        // polling one line slow every other access of the level
        if (arrived) __builtin_amdgcn_s_sleep(1);
        else for (uint32_t k = 0; k < idle_sleep; ++k) __builtin_amdgcn_s_sleep(1);
    }
}

// Release (thread 0): state B = {epoch, L | stop << 31} first, then
// A = {epoch, n} with release order.  `light` (a barrier between two grid
// levels whose shared data all travels in agent-scope atomics): no release
// fence, only the completion of this thread's earlier stores (the counter
// reset among them) before A; a reader that sees A before B goes round
// again.
DEV void release_state(uint64_t *wa, uint64_t *wb, uint32_t epoch, uint32_t L, uint32_t n, uint32_t stop,
                       uint32_t *s_st, bool light = false)
{
    __hip_atomic_store(wb, ((uint64_t)(L | stop << 31) << 32) | epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (light) {
        __builtin_amdgcn_s_waitcnt(0);
        __hip_atomic_store(wa, ((uint64_t)n << 32) | epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        __hip_atomic_store(wa, ((uint64_t)n << 32) | epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    s_st[0] = L;
    s_st[1] = n;
    s_st[2] = stop;
    s_st[3] = epoch;
}

// Two ways to close an epoch (option "barrier"):
//  flags   -- every arriving block but 0 stores {epoch, share} in its own
//             line; wave 0 of block 0 polls those lines, sums the shares
//             and releases (no contended address; two hops: the arrival,
//             then block 0's release);
//  counter -- every arriving block adds {1 arrival, stop bit, share} to a
//             64-bit counter of the epoch's parity (arrivals in bits 48..63,
//             stop bits in 32..47, shares in 0..31); the add that completes
//             the count returns the totals to the last block, which resets
//             the counter for two epochs later and releases (one hop, one
//             contended atomic per arriving block).
// The 64-bit counter of grid barrier epoch e (two, used alternately).
DEV uint64_t *bar_counter(uint32_t *ctrl, uint32_t e)
{
    return reinterpret_cast<uint64_t *>(line(ctrl, (e & 1) ? L_BAR_CNT1 : L_BAR_CNT0));
}

// No deferred frontier writes.
struct NoWrite {
    DEV void operator()(uint32_t) const {}
};

// `defer`: after arriving, every thread of the workgroup calls write(base)
// with the place that the counter addition returned for its staged
// frontier entries (F_DEFER grid levels).
template <class Touches, class Write = NoWrite>
DEV bool grid_barrier(uint32_t *ctrl, uint32_t *bar, uint32_t &epoch, uint64_t timeout, int *s_ok, Grp gr,
                      uint32_t active, uint32_t idle_sleep, bool counter, const Pub &pub, uint32_t share,
                      Touches touches, uint32_t *s_st, LvState *out, bool defer = false, Write write = NoWrite{})
{
    // deferred (counter barrier, F_DEFER grid level): everything the
    // workgroup wrote for others went in agent-scope atomics, so the arrival
    // needs no release fence (no L2 write-back), only the completion of
    // every wavefront's stores; whether a waiter acquires is up to touches
    if (defer) __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    ++epoch;
    uint64_t *wa = reinterpret_cast<uint64_t *>(line(ctrl, L_BAR_GEN));
    uint64_t *wb = reinterpret_cast<uint64_t *>(line(ctrl, L_BAR_GEN) + 16);
    if (counter) {
        // deferred: the low word of the counter also reserves the next
        // frontier's slots (deferred blocks add their staged entries, and
        // entries drained during the level were added before), so the value
        // the addition returns is where this workgroup's staged entries go;
        // they are written between the arrival and the wait
        int ok = 1;
        bool released = false;
        if (threadIdx.x == 0) {
            ok = status_of(ctrl) == 0;
            s_st[3] = epoch;
            s_st[4] = 0;
            if (ok && gr.b < active) {
                if (!defer) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                uint64_t *cnt = bar_counter(ctrl, epoch);
                const uint64_t mine = (1ull << 48) | ((uint64_t)(share >> 31) << 32) | (share & 0x7fffffffu);
                const uint64_t prev = __hip_atomic_fetch_add(cnt, mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint64_t tot = prev + mine;
                s_st[4] = (uint32_t)prev;
                if ((uint32_t)(tot >> 48) == active) {
                    __hip_atomic_store(cnt, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (!defer) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    uint32_t n = pub.n_ptr ? ld_u<kAgent>(pub.n_ptr) : pub.n;
                    uint32_t stop = pub.stop_ptr ? (uint32_t)(ld_u<kAgent>(pub.stop_ptr) != 0) : pub.stop;
                    if (pub.sum) {
                        n = (uint32_t)(tot & 0xffffffffu);
                        stop = ((tot >> 32) & 0xffffu) != 0 ? 1u : 0u;
                    }
                    release_state(wa, wb, epoch, pub.L, n, stop, s_st, defer);
                    if (defer && touches(LvState{pub.L, n, stop})) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    released = true;
                }
            }
            s_st[5] = (uint32_t)ok;
        }
        if (defer) {
            __syncthreads();
            if (gr.b < active && s_st[5]) write(s_st[4]);
        }
        if (threadIdx.x == 0) {
            if (ok && !released) ok = wait_release(ctrl, wa, wb, epoch, timeout, gr.b < active, idle_sleep, touches, s_st);
            *s_ok = ok;
        }
    } else if (gr.b == 0) {
        if (threadIdx.x < 64) {
            int ok = status_of(ctrl) == 0;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const uint64_t t0 = wall_clock64();
            uint64_t added = 0;
            bool ended = false;
            while (ok) {
                bool mine = true;
                added = 0;
                ended = false;
                for (uint32_t b = 1 + threadIdx.x; b < active; b += 64) {
                    const uint64_t v = __hip_atomic_load(reinterpret_cast<uint64_t *>(bar + (size_t)b * kLineWords),
                                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    mine &= (uint32_t)v == epoch;
                    added += (v >> 32) & 0x7fffffffu;
                    ended |= (v >> 63) != 0;
                }
                if (__ballot(!mine) == 0) break;
                if (status_of(ctrl) != 0) ok = 0;
                else if (wall_clock64() - t0 > timeout) { if (threadIdx.x == 0) set_status(ctrl, kEInternal); ok = 0; }
                __builtin_amdgcn_s_sleep(1);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const uint32_t all_added = (uint32_t)wave_sum(added);
            const bool any_ended = __ballot(ended) != 0;
            if (threadIdx.x == 0) {
                uint32_t n = pub.n_ptr ? ld_u<kAgent>(pub.n_ptr) : pub.n;
                uint32_t stop = pub.stop_ptr ? (uint32_t)(ld_u<kAgent>(pub.stop_ptr) != 0) : pub.stop;
                if (pub.sum) {
                    n += all_added;
                    stop |= any_ended ? 1u : 0u;
                }
                if (ok) release_state(wa, wb, epoch, pub.L, n, stop, s_st);
                *s_ok = ok;
            }
        }
    } else if (threadIdx.x == 0) {
        int ok = status_of(ctrl) == 0;
        s_st[3] = epoch;
        if (ok) {
            if (gr.b < active) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __hip_atomic_store(reinterpret_cast<uint64_t *>(bar + (size_t)gr.b * kLineWords),
                                   ((uint64_t)share << 32) | epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            ok = wait_release(ctrl, wa, wb, epoch, timeout, gr.b < active, idle_sleep, touches, s_st);
        }
        *s_ok = ok;
    }
    __syncthreads();
    *out = LvState{s_st[0], s_st[1], s_st[2]};
    epoch = s_st[3];
    return *s_ok != 0;
}

// Blocks that expand a grid level of n entries: one per `per` entries
// (per = 0: every block).
DEV uint32_t level_blocks(uint32_t n, uint32_t per, uint32_t nblocks)
{
    if (per == 0) return nblocks;
    const uint32_t a = (n + per - 1) / per;
    return a < 1 ? 1u : (a > nblocks ? nblocks : a);
}

// ---------------------------------------------------------------------
// A run of levels with small frontiers, expanded by the calling workgroup
// alone (block 0 of the persistent kernel).  Starts at level L with n0
// entries in the current queue, stops when the frontier is empty or larger
// than small_max (or, APsB, after a level that reached an unmatched row).
// Counters live in LDS (s_loc[0..2] frontier sizes, [3] found, [4] ends)
// and the frontier counters are written back to the control block at the
// end.  Returns the state reached (level, its frontier size, APsB stop);
// *levels grows by the number of levels expanded.
// Bound on one run, so that the blocks waiting at the grid barrier see
// progress well within their wait limit.
constexpr uint32_t kSmallRunLevels = 4096;

template <bool WAVE, bool SINGLE = true>
DEV LvState small_levels(const DevGraph &g, uint32_t *ctrl, const RunOpt &o, uint32_t ph, int L, uint32_t n0,
                         Stage &st, uint32_t *s_tmp, uint32_t *s_loc, Acc &acc, uint32_t *total_levels)
{
    const uint32_t flags = o.flags;
    if (threadIdx.x == 0) {
        s_loc[L % 3] = n0;
        s_loc[(L + 1) % 3] = 0;
        s_loc[(L + 2) % 3] = 0;
        s_loc[3] = 0;
        s_loc[4] = ld_u<kAgent>(line(ctrl, L_NENDS));
    }
    __syncthreads();
    uint32_t levels = 0, stop = 0;
    const uint32_t wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    for (;;) {
        const uint32_t n = *(volatile uint32_t *)&s_loc[L % 3];
        if (n == 0 || n > o.small_max || levels >= kSmallRunLevels) break;
        if ((uint32_t)L > o.max_levels) { if (threadIdx.x == 0) set_status(ctrl, kEInternal); break; }
        __syncthreads();
        if (threadIdx.x == 0) { s_loc[(L + 2) % 3] = 0; s_loc[3] = 0; }
        __syncthreads();
        int4 *cur = (L & 1) ? g.fq1 : g.fq0;
        const LevelIO io{QSink{(L & 1) ? g.fq0 : g.fq1, &s_loc[(L + 1) % 3], nullptr, (flags & F_DEFER) != 0},
                         &s_loc[4], &s_loc[3], ctrl, false};
        if (SINGLE && pair_form(o.flags))
            expand_level<WAVE, kGroup, SINGLE, true>(g, cur, n, wave, nwaves, ph, L, o, io, st, s_tmp, acc);
        else
            expand_level<WAVE, kGroup, SINGLE>(g, cur, n, wave, nwaves, ph, L, o, io, st, s_tmp, acc);
        ++levels;
        if ((flags & F_APSB) && *(volatile uint32_t *)&s_loc[3]) { stop = 1; break; }
        ++L;
    }
    __syncthreads();
    const uint32_t n = s_loc[L % 3];
    if (threadIdx.x == 0) {
        for (int i = 0; i < 3; ++i) {
            *line(ctrl, L_FCOUNT0 + i) = (i == L % 3) ? n : 0u;
            *line(ctrl, L_FOUND0 + i) = 0;
        }
        *line(ctrl, L_NENDS) = s_loc[4];
        *line(ctrl, L_SMALL_LEVELS) += levels;
    }
    *total_levels += levels;
    return LvState{(uint32_t)L, n, stop};
}

// The phase loop of Algorithm 1 over the whole grid (cooperative launch).
// SINGLE: the launch for one graph (mcm_match), with local levels (option
// local_levels) and the recorded-row Alternate.  The multi-graph launch
// compiles both out: local levels lengthened the serving latency there
// (p50 45 -> 50 ms at 2000 requests/s), and both cost registers.
template <bool WAVE, bool SINGLE = true>
DEV bool run_grid(const DevGraph &g, uint32_t *ctrl, uint32_t *bar, const RunOpt &o, uint64_t *stats, Acc &acc, Stage &st,
                  uint32_t *s_tmp, uint32_t *s_loc, int *s_ok, uint32_t *ph_out, uint32_t *lv_out, Grp gr,
                  uint32_t &epoch)
{
    const uint32_t flags = o.flags;
    const uint32_t wave = gr.b * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint32_t nwaves = gr.n * (blockDim.x >> 6);
    const uint32_t tid = gr.b * blockDim.x + threadIdx.x, nthreads = gr.n * blockDim.x;
    const bool leader = gr.b == 0 && threadIdx.x == 0;
    const bool timing = (flags & F_STATS) != 0;
    uint32_t total_levels = 0, ph = 1;
    auto fc = [&](int i) { return line(ctrl, L_FCOUNT0 + i); };
    auto fd = [&](int i) { return line(ctrl, L_FOUND0 + i); };
    // grid barrier (`active` blocks arrive; block 0 releases the loop state
    // `p` into s), with the time block 0 spends in it counted (stats=1)
    LvState s{0, 0, 0};
    const bool counter = (flags & F_BAR_COUNTER) != 0;
    // F_DEFER: grid levels reserve their next frontier through the counter
    // barrier, and all they share (queue entries, row words, pred, cdone,
    // ends) goes through agent-scope atomics
    const bool defer = counter && (flags & F_DEFER) != 0;
    // does this block read data that others wrote with ordinary stores
    // before its next barrier in state x? (it expands the level, or the
    // level loop ends and Alternate follows; a deferred grid level reads
    // nothing of the kind, so its L2 keeps the graph)
    auto in_level = [&](const LvState &x) -> bool {
        if (x.n == 0 || x.stop) return true;
        if (x.n <= o.small_max) return gr.b == 0;
        if (defer) return false;
        return gr.b < level_blocks(x.n, o.level_entries, gr.n);
    };
    auto always = [](const LvState &) -> bool { return true; };
    auto sync = [&](uint32_t active, const Pub &p, uint32_t share, bool dw, auto write) -> bool {
        const uint64_t t0 = timing ? wall_clock64() : 0;
        const bool ok = grid_barrier(ctrl, bar, epoch, o.timeout, s_ok, gr, active, o.idle_sleep, counter, p, share,
                                     in_level, s_loc + 8, &s, dw, write);
        if (timing) acc.tick(S_T_BARRIER, wall_clock64() - t0);
        return ok;
    };
    auto sync_all = [&](const Pub &p) -> bool {
        const uint64_t t0 = timing ? wall_clock64() : 0;
        const bool ok = grid_barrier(ctrl, bar, epoch, o.timeout, s_ok, gr, gr.n, o.idle_sleep, counter, p, 0u, always,
                                     s_loc + 8, &s);
        if (timing) acc.tick(S_T_BARRIER, wall_clock64() - t0);
        return ok;
    };
    const Pub none{0, 0, 0, nullptr, nullptr, false};
    for (;; ++ph) {
        if (ph > o.max_phases) { if (leader) set_status(ctrl, kEInternal); return false; }
        const uint32_t lv0 = total_levels;
        // every block read the previous phase's count of reported rows before
        // the barrier that ends this phase's root scan; the walks of this
        // phase report after it (an agent-scope store: the barriers between
        // deferred grid levels carry no release)
        auto reset_touch = [&]() { if (leader) st_u<kAgent>(line(ctrl, L_NTOUCH), 0u); };
        if (SINGLE && (flags & F_ASYNC)) {
            // level-free phase: roots reserved in the phase-long queue, one
            // grid barrier, then every wavefront works until the queue's
            // entries are all finished
            const bool act = init_roots<SINGLE>(g, wave, nwaves, o, nullptr, st, s_tmp, acc,
                                                reinterpret_cast<uint64_t *>(line(ctrl, L_AQ)), ph, ctrl);
            if (!sync_all(none)) return false;
            if (act && leader) mark_active_phase(ctrl, ph);
            reset_touch();
            async_bfs<WAVE>(g, ctrl, o, ph, nwaves, st, acc);
            ++total_levels;
            if (!sync_all(none)) return false;
            s = LvState{0, 0, 0};
        } else {
        bool act = false;
        if (SINGLE && (flags & F_FUSE0) && !roots_listed(g, o, ph, ctrl)) {
            // level 0 in the root scan's pass; the level loop goes on at 1
            uint32_t share = pair_form(flags) ? roots_level0<WAVE, true>(g, wave, nwaves, o, ph, ctrl, st, s_tmp, acc)
                                              : roots_level0<WAVE, false>(g, wave, nwaves, o, ph, ctrl, st, s_tmp, acc);
            if (!(flags & F_APSB)) share &= 0x7fffffffu;
            ++total_levels;
            if (!sync(gr.n, Pub{1u, share & 0x7fffffffu, share >> 31, nullptr, nullptr, true}, share, false,
                      NoWrite{}))
                return false;
        } else {
            act = init_roots<SINGLE>(g, wave, nwaves, o, fc(0), st, s_tmp, acc, nullptr, ph, ctrl);
            if (!sync_all(Pub{0, 0, 0, fc(0), nullptr, false})) return false;
        }
        if (act && leader) mark_active_phase(ctrl, ph);
        reset_touch();
        for (;;) {
            const int L = (int)s.L;
            if (s.n == 0 || s.stop) break;
            if ((uint32_t)L > o.max_levels) { if (leader) set_status(ctrl, kEInternal); return false; }
            if (s.n <= o.small_max) {
                Pub p = none;
                if (gr.b == 0) {
                    const uint64_t t0 = timing ? wall_clock64() : 0;
                    const LvState r =
                        small_levels<WAVE, SINGLE>(g, ctrl, o, ph, L, s.n, st, s_tmp, s_loc, acc, &total_levels);
                    if (timing) acc.tick(S_T_SMALL, wall_clock64() - t0);
                    p = Pub{r.L, r.n, r.stop, nullptr, nullptr, false};
                }
                if (!sync(1, p, 0u, false, NoWrite{})) return false;
                continue;
            }
            const uint32_t active = level_blocks(s.n, o.level_entries, gr.n);
            if (leader) { *fc((L + 2) % 3) = 0; *fd((L + 2) % 3) = 0; }
            // this block's share of the next frontier (and, APsB, whether it
            // reached an unmatched row) rides on its arrival
            uint32_t share = 0;
            // deferred: slots come from the counter of the barrier that ends
            // this level (epoch + 1)
            const QSink next{(L & 1) ? g.fq0 : g.fq1, fc((L + 1) % 3), defer ? bar_counter(ctrl, epoch + 1) : nullptr,
                             defer};
            if (gr.b < active) {
                int4 *cur = (L & 1) ? g.fq1 : g.fq0;
                const LevelIO io{next, line(ctrl, L_NENDS), fd(L % 3), ctrl, defer};
                const uint32_t lw = active * (blockDim.x >> 6);
                const uint32_t local = (!SINGLE || (flags & F_LEVELS)) ? 0u : o.local_levels;
                if (SINGLE && pair_form(flags))
                    share = expand_level<WAVE, kAgent, SINGLE, true>(g, cur, s.n, wave, lw, ph, L, o, io, st, s_tmp,
                                                                     acc, local);
                else
                    share = expand_level<WAVE, kAgent, SINGLE>(g, cur, s.n, wave, lw, ph, L, o, io, st, s_tmp, acc,
                                                               local);
                if (!(flags & F_APSB)) share &= 0x7fffffffu;
            }
            ++total_levels;
            if (!sync(active, Pub{(uint32_t)L + 1, share & 0x7fffffffu, share >> 31, nullptr, nullptr, true}, share,
                      defer, [&](uint32_t base) { write_deferred(st, next, base, s_tmp); }))
                return false;
        }
        }
        // APsB stop: the frontier of level left.L (left.n entries) is never
        // expanded; with deferred writes its slots are set back to -1 once
        // they are certainly written (after the next grid barrier)
        const LvState left = s;
        const uint32_t ne = ld_u<kAgent>(line(ctrl, L_NENDS));
        if (leader && timing && g.ptrace && ph <= (uint32_t)kPhaseTrace) {
            g.ptrace[2 * (ph - 1)] = total_levels - lv0;
            g.ptrace[2 * (ph - 1) + 1] = ne;
        }
        if (ne == 0 || (flags & F_NOAUG)) break;
        const uint64_t ta = timing ? wall_clock64() : 0;
        if (leader) {
            // the level loop is over (no block adds to these any more) and the
            // next root scan starts after Alternate's grid barrier
            for (int i = 0; i < 3; ++i) { *fc(i) = 0; *fd(i) = 0; }
            *reinterpret_cast<uint64_t *>(line(ctrl, L_AQ)) = 0;
            *line(ctrl, L_AQ_TAKE) = 0;
            // the next phase lists its roots in the half this phase read
            *line(ctrl, ((ph + 1) & 1) ? L_NRL1 : L_NRL0) = 0;
        }
        // the walks report the rows they touch when the phase found few ends
        // (o.fix_max); FixMatching then visits only those
        const bool listed = SINGLE && g.touched && ne <= o.fix_max;
        if (listed)
            alternate_listed<kAgent>(g, ne, tid, nthreads, flags, ctrl, acc, st, line(ctrl, L_NTOUCH));
        else
            alternate<kAgent>(g, ne, tid, nthreads, SINGLE ? flags : (flags & ~(uint32_t)F_FASTALT), ctrl, acc);
        if (!sync_all(none)) return false;
        // every block read the count of ends before this barrier; the next
        // phase's BFS adds to it after the next grid barrier
        if (leader) *line(ctrl, L_NENDS) = 0;
        // FixMatching over the rows the walks touched, unless more were
        // reported than the list holds (then over every row)
        const uint32_t ntouch = listed ? ld_u<kAgent>(line(ctrl, L_NTOUCH)) : 0xffffffffu;
        if (ntouch <= (uint32_t)g.nr) {
            fix_listed(g, ntouch, tid, nthreads, flags, acc);
            if (timing && gr.b == 0) acc.tick(S_PASS, 8ull * ntouch);
        } else {
            fix_matching(g, ph, tid, nthreads, flags, acc);
            if (timing && gr.b == 0) acc.tick(S_PASS, 8ull * (uint32_t)g.nr);
        }
        // No grid barrier between FixMatching and the next root scan: the
        // scan reads cmatch, colptr and the root list, which FixMatching does
        // not write, and the BFS that reads the row words FixMatching writes
        // starts after the scan's own barrier.  Two exceptions: the unread
        // frontier of an APsB stop, whose slots are set back to -1 here in
        // the queue the scan may write; and a next phase that expands level
        // 0 in the scan's pass (its BFS reads row words before any other
        // barrier).  Every block takes the same decision: the root count
        // that roots_listed reads is final since this phase's first barrier.
        const bool fuse_next = SINGLE && (flags & F_FUSE0) && !roots_listed(g, o, ph + 1, ctrl);
        if ((flags & F_DEFER) && left.stop) {
            const QSink lq{(left.L & 1) ? g.fq1 : g.fq0, nullptr, nullptr, true};
            for (uint32_t i = tid; i < left.n; i += nthreads) put_entry(lq, i, make_int4(-1, -1, -1, -1));
        }
        if (((flags & F_DEFER) && left.stop) || fuse_next)
            if (!sync_all(none)) return false;
        if (timing) acc.tick(S_T_AUGMENT, wall_clock64() - ta);
    }
    if (leader) { *ph_out = ph; *lv_out = total_levels; }
    if (timing) acc.flush(stats, gr.b == 0);
    return true;
}

// The phase loop of Algorithm 1 inside one workgroup (graph owned by it).
template <bool WAVE>
DEV bool run_block(const DevGraph &g, uint32_t *ctrl, const RunOpt &o, Acc &acc, Stage &st, uint32_t *s_tmp,
                   uint32_t *s_loc, uint32_t *ph_out, uint32_t *lv_out)
{
    const uint32_t flags = o.flags;
    const uint32_t wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    uint32_t total_levels = 0, ph = 1;
    for (;; ++ph) {
        if (ph > o.max_phases) { if (threadIdx.x == 0) set_status(ctrl, kEInternal); return false; }
        __syncthreads();
        if (threadIdx.x == 0) for (int i = 0; i < 5; ++i) s_loc[i] = 0;
        __syncthreads();
        init_roots(g, wave, nwaves, o, &s_loc[0], st, s_tmp, acc);
        int L = 0;
        for (;;) {
            const uint32_t n = *(volatile uint32_t *)&s_loc[L % 3];
            if (n == 0) break;
            if ((uint32_t)L > o.max_levels) { if (threadIdx.x == 0) set_status(ctrl, kEInternal); return false; }
            __syncthreads();
            if (threadIdx.x == 0) { s_loc[(L + 2) % 3] = 0; s_loc[3] = 0; }
            __syncthreads();
            int4 *cur = (L & 1) ? g.fq1 : g.fq0;
            const LevelIO io{QSink{(L & 1) ? g.fq0 : g.fq1, &s_loc[(L + 1) % 3], nullptr, false}, &s_loc[4],
                             &s_loc[3], ctrl, false};
            expand_level<WAVE, kGroup, false>(g, cur, n, wave, nwaves, ph, L, o, io, st, s_tmp, acc);
            ++total_levels;
            if ((flags & F_APSB) && *(volatile uint32_t *)&s_loc[3]) break;
            ++L;
        }
        const uint32_t ne = *(volatile uint32_t *)&s_loc[4];
        if (ne == 0 || (flags & F_NOAUG)) break;
        alternate<kGroup>(g, ne, threadIdx.x, blockDim.x, flags & ~(uint32_t)F_FASTALT, ctrl, acc);
        __syncthreads();
        fix_matching(g, ph, threadIdx.x, blockDim.x, flags, acc);
        if (flags & F_STATS) acc.tick(S_PASS, 8ull * (uint32_t)g.nr);
    }
    __syncthreads();
    *ph_out = ph;
    *lv_out = total_levels;
    return true;
}

// ---------------------------------------------------------------------
// Kernels

// Copy the initial matching into the working state, reset stamps and
// barrier flags, and count the initial matching's columns into the
// control block's L_INIT_CARD (which launch_zero_ctrl cleared before).
__global__ void k_setup(DevGraph g, const int32_t *init_c, const int32_t *init_r, uint32_t *ctrl, uint32_t *bar,
                        uint32_t flags)
{
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nt = gridDim.x * blockDim.x;
    const uint32_t nc = (uint32_t)g.nc, nr = (uint32_t)g.nr;
    uint64_t m0 = 0;
    // kStream elements per thread and step, their loads issued together
    // (indices clamped, stores masked)
    for (uint32_t c0 = tid; c0 < nc; c0 += nt * kStream) {
        int r[kStream];
#pragma unroll
        for (int u = 0; u < kStream; ++u) r[u] = init_c ? init_c[min(c0 + u * nt, nc - 1)] : -1;
#pragma unroll
        for (int u = 0; u < kStream; ++u) {
            const uint32_t c = c0 + u * nt;
            if (c >= nc) continue;
            g.cmatch[c] = r[u];
            m0 += r[u] >= 0;
            g.cdone[c] = 0;
            if (flags & F_LEVELS) {
                g.clevel[c] = -1;
                if (g.croot) g.croot[c] = -1;
            }
        }
    }
    if (flags & (F_DEFER | F_ASYNC))
        for (uint64_t i = tid; i < 2 * g.qcap; i += nt) g.fq0[i] = make_int4(-1, -1, -1, -1);
    for (uint32_t r0 = tid; r0 < nr; r0 += nt * kStream) {
        int m[kStream];
        int2 adj[kStream];
#pragma unroll
        for (int u = 0; u < kStream; ++u) m[u] = init_r ? init_r[min(r0 + u * nt, nr - 1)] : -1;
        if (flags & F_MAXCLAIM) {
#pragma unroll
            for (int u = 0; u < kStream; ++u)
                adj[u] = m[u] >= 0 ? make_int2(g.colptr[m[u]], g.colptr[m[u] + 1]) : make_int2(0, 0);
        }
#pragma unroll
        for (int u = 0; u < kStream; ++u) {
            const uint32_t r = r0 + u * nt;
            if (r >= nr) continue;
            g.rw[r] = (uint64_t)(uint32_t)m[u];
            if (flags & F_LEVELS) g.pred[r] = -1;
            if (flags & F_MAXCLAIM) g.radj[r] = adj[u];
        }
    }
    if (bar)
        for (uint32_t i = tid; i < (uint32_t)(kMaxGridBlocks * kLineWords); i += nt) bar[i] = 0;
    block_add(m0, reinterpret_cast<uint64_t *>(line(ctrl, L_INIT_CARD)));
}

// Optional input validation (option validate=1), in two launches: the CSC
// structure first; the initial matching only once the structure is known to
// be sound, because checking that a matched pair is an edge scans the
// column's range of rowind, which a malformed colptr would put out of
// bounds.
__global__ void k_validate_csc(int32_t nc, int32_t nr, const int32_t *colptr, const int32_t *rowind, uint32_t *ctrl)
{
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nt = gridDim.x * blockDim.x;
    if (tid == 0 && colptr[0] != 0) set_status(ctrl, kEInval);
    for (uint32_t c = tid; c < (uint32_t)nc; c += nt)
        if (colptr[c + 1] < colptr[c]) set_status(ctrl, kEInval);
    const int64_t nnz = colptr[nc];
    for (int64_t j = tid; j < nnz; j += nt)
        if (rowind[j] < 0 || rowind[j] >= nr) set_status(ctrl, kEInval);
}

// Runs after k_validate_csc left the status at 0: colptr starts at 0 and
// never decreases, so every [colptr[c], colptr[c+1]) lies in [0, nnz).
__global__ void k_validate_init(int32_t nc, int32_t nr, const int32_t *colptr, const int32_t *rowind,
                                const int32_t *init_c, const int32_t *init_r, uint32_t *ctrl)
{
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nt = gridDim.x * blockDim.x;
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
__global__ void __launch_bounds__(1024) k_persistent(DevGraph g, uint32_t *ctrl, uint32_t *bar, RunOpt o)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ int s_ok;
    __shared__ uint32_t s_loc[16];  // [0..7] level counters, [8..13] barrier state
    __shared__ uint64_t s_acc[kAccN];
    Stage st = make_stage(smem);
    uint32_t *s_tmp = stage_tmp(smem);
    uint64_t *stats = reinterpret_cast<uint64_t *>(line(ctrl, L_STAT0));
    Acc acc = make_acc(s_acc, stage_tmp(smem));
    uint32_t ph = 0, lv = 0, epoch = 0;
    if (run_grid<WAVE>(g, ctrl, bar, o, stats, acc, st, s_tmp, s_loc, &s_ok, &ph, &lv, Grp{blockIdx.x, gridDim.x},
                       epoch) &&
        blockIdx.x == 0 && threadIdx.x == 0) {
        *line(ctrl, L_PHASE) = ph;
        *line(ctrl, L_LEVELS) = lv;
    }
}

// ---------------------------------------------------------------------
// Several large graphs in one cooperative launch: graph i of the launch is
// matched by blocks [i*group, (i+1)*group) with the same phase loop as
// k_persistent, synchronised by a barrier of its own group (own control
// block and arrival lines).  One launch keeps all groups co-resident.
// State setup and the final unpack are separate launches before and after.
DEV DevGraph graph_of(const BatchDesc &d)
{
    DevGraph g;
    g.colptr = d.colptr;
    g.rowind = d.rowind;
    g.nc = d.nc;
    g.nr = d.nr;
    g.cmatch = d.out_c;
    g.rw = d.rw;
    g.pred = d.pred;
    g.cdone = d.cdone;
    g.fq0 = d.fq;
    g.fq1 = d.fq + (d.qcap ? d.qcap : d.nc);
    g.ends = d.ends;
    g.clevel = nullptr;
    return g;
}

// Completion mark of a graph of a multi-graph launch, in its card slot:
// the counts that k_finish_multi adds on top keep every reader seeing it.
constexpr int64_t kGraphDone = (int64_t)1 << 62;

// Before a multi-graph launch.  blockIdx.y = graph: working state from the
// initial matching, and card[graph] = kEInternal, which the group that
// completes the graph replaces by kGraphDone (k_finish_multi then adds |M|
// to it; a graph left unprocessed after a watchdog keeps the error).  The groups'
// control blocks and arrival lines, and the graph queue in the first
// control block, start at zero.
__global__ void k_setup_multi(const BatchDesc *descs, int32_t ngraphs, int32_t ngroups, uint32_t *ctrls,
                              uint32_t *bars, uint32_t bar_lines, int64_t *card)
{
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x, nt = gridDim.x * blockDim.x;
    for (int32_t gi = blockIdx.y; gi < ngraphs; gi += gridDim.y) {
        const BatchDesc d = descs[gi];
        for (uint32_t c = tid; c < (uint32_t)d.nc; c += nt) {
            d.out_c[c] = d.init_c ? d.init_c[c] : -1;
            d.cdone[c] = 0;
        }
        for (uint32_t r = tid; r < (uint32_t)d.nr; r += nt) d.rw[r] = (uint64_t)(uint32_t)(d.init_r ? d.init_r[r] : -1);
        if (tid == 0) card[gi] = kEInternal;
    }
    if (blockIdx.y == 0) {
        const uint32_t nctrl = (uint32_t)ngroups * L_NLINES * kLineWords, nbar = (uint32_t)ngroups * bar_lines * kLineWords;
        for (uint32_t i = tid; i < nctrl; i += nt) ctrls[i] = 0;
        for (uint32_t i = tid; i < nbar; i += nt) bars[i] = 0;
    }
}

// Many large graphs in one cooperative launch: the blocks form groups of
// `group` blocks (own control block and arrival lines each), and every
// group takes graph after graph from a queue (the L_QUEUE line of the
// first control block) and runs the phase loop of k_persistent on it with
// a barrier of its own, until the queue is empty.  Block 0 of a group takes
// the next index and the group learns it through a barrier that releases
// it as the frontier size.
template <bool WAVE>
__global__ void __launch_bounds__(1024) k_persistent_multi(const BatchDesc *descs, int32_t ngraphs, uint32_t group,
                                                           uint32_t *ctrls, uint32_t *bars, int64_t *card, RunOpt o)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ int s_ok;
    __shared__ uint32_t s_loc[16];  // [0..7] level counters, [8..13] barrier state
    __shared__ uint64_t s_acc[kAccN];
    // Forms this launch never runs, masked so that their code is dead: the
    // statistics (callers read them from other launches' control blocks),
    // level records, and the claim, flush, Alternate and BFS forms whose
    // buffers (radj, prow, checked queues) a batch descriptor does not carry.
    // The kernel sits at the 128-register limit of a 1024-thread block;
    // without this its registers spill.
    o.flags &= ~(uint32_t)(F_STATS | F_LEVELS | F_NOAUG | F_MAXCLAIM | F_DEFER | F_FASTALT | F_ASYNC | F_FUSE0);
    const uint32_t q = blockIdx.x / group;
    const Grp gr{blockIdx.x % group, group};
    uint32_t *ctrl = ctrls + (size_t)q * L_NLINES * kLineWords;
    uint32_t *bar = bars + (size_t)q * group * kLineWords;
    uint32_t *queue = line(ctrls, L_QUEUE);
    Stage st = make_stage(smem);
    uint32_t *s_tmp = stage_tmp(smem);
    uint64_t *stats = reinterpret_cast<uint64_t *>(line(ctrl, L_STAT0));
    Acc acc = make_acc(s_acc, stage_tmp(smem));
    const bool leader = gr.b == 0 && threadIdx.x == 0;
    auto always = [](const LvState &) -> bool { return true; };
    const bool counter = (o.flags & F_BAR_COUNTER) != 0;
    uint32_t epoch = 0;
    for (;;) {
        if (leader) {
            // the previous graph left its level counters behind
            for (int i = 0; i < 3; ++i) { *line(ctrl, L_FCOUNT0 + i) = 0; *line(ctrl, L_FOUND0 + i) = 0; }
            *line(ctrl, L_NENDS) = 0;
            // whichever block releases the barrier reads the index from here
            *line(ctrl, L_TAKE) = atomicAdd(queue, 1u);
        }
        LvState x;
        if (!grid_barrier(ctrl, bar, epoch, o.timeout, &s_ok, gr, group, o.idle_sleep, counter,
                          Pub{0, 0, 0, line(ctrl, L_TAKE), nullptr, false}, 0u, always, s_loc + 8, &x))
            return;
        const uint32_t gi = x.n;
        if (gi >= (uint32_t)ngraphs) return;  // the whole group: the queue is drained
        const BatchDesc d = descs[gi];
        bool ok = true;
        if (d.nc > 0 && d.nr > 0) {
            DevGraph g = graph_of(d);
            uint32_t ph = 0, lv = 0;
            ok = run_grid<WAVE, false>(g, ctrl, bar, o, stats, acc, st, s_tmp, s_loc, &s_ok, &ph, &lv, gr, epoch);
        }
        if (!ok) return;                      // watchdog: this graph and the group stop
        if (leader) card[gi] = kGraphDone;    // k_finish_multi counts |M| on top
    }
}

// blockIdx.y = graph: unpack rmatch and add |M| = #{c : cmatch[c] >= 0}
// to card[graph] for every graph a group completed; the others keep the
// error.  k_card_done then removes the completion mark.
__global__ void k_finish_multi(const BatchDesc *descs, int32_t ngraphs, int64_t *card)
{
    for (int32_t gi = blockIdx.y; gi < ngraphs; gi += gridDim.y) {
        const BatchDesc d = descs[gi];
        if (card[gi] < kGraphDone) continue;  // not completed: the error stays
        const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x, nt = gridDim.x * blockDim.x;
        for (uint32_t r = tid; r < (uint32_t)d.nr; r += nt) d.out_r[r] = (int32_t)(uint32_t)d.rw[r];
        uint64_t m = 0;
        for (uint32_t c = tid; c < (uint32_t)d.nc; c += nt) m += (d.out_c[c] >= 0);
        block_add(m, reinterpret_cast<uint64_t *>(&card[gi]));
    }
}

__global__ void k_card_done(int32_t ngraphs, int64_t *card)
{
    const int32_t gi = blockIdx.x * blockDim.x + threadIdx.x;
    if (gi < ngraphs && card[gi] >= kGraphDone) card[gi] -= kGraphDone;
}

// Host-driven steps (one launch each).
__global__ void k_init_roots(DevGraph g, uint32_t *ctrl, RunOpt o)
{
    extern __shared__ __align__(16) char smem[];
    Stage st = make_stage(smem);
    const uint32_t flags = o.flags;
    const uint32_t wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6), nwaves = gridDim.x * (blockDim.x >> 6);
    __shared__ uint64_t s_acc[kAccN];
    Acc acc = make_acc(s_acc);
    init_roots(g, wave, nwaves, o, line(ctrl, L_FCOUNT0), st, stage_tmp(smem), acc);
    if (flags & F_STATS) acc.flush(reinterpret_cast<uint64_t *>(line(ctrl, L_STAT0)), false);
}

template <bool WAVE>
__global__ void __launch_bounds__(1024) k_level(DevGraph g, uint32_t *ctrl, uint32_t n, uint32_t ph, int L, RunOpt o)
{
    const uint32_t flags = o.flags;
    extern __shared__ __align__(16) char smem[];
    Stage st = make_stage(smem);
    const uint32_t wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6), nwaves = gridDim.x * (blockDim.x >> 6);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *line(ctrl, L_FCOUNT0 + (L + 2) % 3) = 0;
        *line(ctrl, L_FOUND0 + (L + 2) % 3) = 0;
    }
    int4 *cur = (L & 1) ? g.fq1 : g.fq0;
    const LevelIO io{QSink{(L & 1) ? g.fq0 : g.fq1, line(ctrl, L_FCOUNT0 + (L + 1) % 3), nullptr, false},
                     line(ctrl, L_NENDS), line(ctrl, L_FOUND0 + L % 3), ctrl, false};
    __shared__ uint64_t s_acc[kAccN];
    Acc acc = make_acc(s_acc, stage_tmp(smem));
    if (!pair_form(o.flags))
        expand_level<WAVE, kAgent>(g, cur, n, wave, nwaves, ph, L, o, io, st, stage_tmp(smem), acc);
    else
        expand_level<WAVE, kAgent, true, true>(g, cur, n, wave, nwaves, ph, L, o, io, st, stage_tmp(smem), acc);
    if (flags & F_STATS) acc.flush(reinterpret_cast<uint64_t *>(line(ctrl, L_STAT0)), false);
}

__global__ void k_alternate(DevGraph g, uint32_t *ctrl, uint32_t flags)
{
    const uint32_t ne = *line(ctrl, L_NENDS);
    __shared__ uint64_t s_acc[kAccN];
    Acc acc = make_acc(s_acc);
    alternate<kAgent>(g, ne, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x, flags, ctrl, acc);
    if (flags & F_STATS) acc.flush(reinterpret_cast<uint64_t *>(line(ctrl, L_STAT0)), false);
}

__global__ void k_fix(DevGraph g, uint32_t *ctrl, uint32_t ph, uint32_t flags)
{
    __shared__ uint64_t s_acc[kAccN];
    Acc acc = make_acc(s_acc);
    fix_matching(g, ph, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x, flags, acc);
    if ((flags & F_STATS) && blockIdx.x == 0) acc.tick(S_PASS, 8ull * (uint32_t)g.nr);
    if (flags & F_STATS) acc.flush(reinterpret_cast<uint64_t *>(line(ctrl, L_STAT0)), false);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int i = 0; i < 3; ++i) { *line(ctrl, L_FCOUNT0 + i) = 0; *line(ctrl, L_FOUND0 + i) = 0; }
        *line(ctrl, L_NENDS) = 0;
    }
}

// Unpack rmatch, count |M| = #{c : cmatch[c] >= 0}.
__global__ void k_finish(DevGraph g, int32_t *out_r, uint32_t *ctrl)
{
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nt = gridDim.x * blockDim.x;
    const uint32_t nc = (uint32_t)g.nc, nr = (uint32_t)g.nr;
    // kStream elements per thread and step, their loads issued together
    for (uint32_t r0 = tid; r0 < nr; r0 += nt * kStream) {
        uint64_t w[kStream];
#pragma unroll
        for (int u = 0; u < kStream; ++u) w[u] = g.rw[min(r0 + u * nt, nr - 1)];
#pragma unroll
        for (int u = 0; u < kStream; ++u)
            if (r0 + u * nt < nr) out_r[r0 + u * nt] = (int32_t)(uint32_t)w[u];
    }
    uint64_t m = 0;
    for (uint32_t c0 = tid; c0 < nc; c0 += nt * kStream) {
        int cm[kStream];
#pragma unroll
        for (int u = 0; u < kStream; ++u) cm[u] = g.cmatch[min(c0 + u * nt, nc - 1)];
#pragma unroll
        for (int u = 0; u < kStream; ++u) m += (c0 + u * nt < nc && cm[u] >= 0);
    }
    block_add(m, reinterpret_cast<uint64_t *>(line(ctrl, L_CARD)));
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
    block_add(k, reinterpret_cast<uint64_t *>(line(ctrl, L_CARD)));
}

// pred of reached rows for the level inspection entry point
__global__ void k_export_pred(DevGraph g, uint32_t ph, int32_t *row_pred)
{
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nt = gridDim.x * blockDim.x;
    for (uint32_t r = tid; r < (uint32_t)g.nr; r += nt)
        row_pred[r] = ((uint32_t)(g.rw[r] >> 32) == ph) ? g.pred[r] : -1;
}

__global__ void k_zero_ctrl(uint32_t *ctrl)
{
    for (uint32_t i = threadIdx.x; i < (uint32_t)(L_NLINES * kLineWords); i += blockDim.x) ctrl[i] = 0;
}

// ---------------------------------------------------------------------
// One workgroup per graph.  Used for small single graphs and for batches;
// blocks take graphs from a queue (ordered largest first by the host) until
// it is empty.  Every graph gets its own state slices; counters live in LDS.
// The LDS arena of the one-workgroup kernel: a graph whose pattern and
// randomly accessed state fit in `arena` bytes is matched there (colptr,
// rowind, row words, pred, cdone and cmatch in LDS; frontier queues and
// ends stay in global memory, which they reach in staged, coalesced
// batches).  The kernel's code reaches LDS and global memory through the
// same pointers (flat addressing), so the matching steps are the same code.
DEV size_t lds_al(size_t b) { return (b + 15) & ~(size_t)15; }
DEV size_t lds_graph_bytes(int32_t nc, int32_t nr, int64_t nnz)
{
    return lds_al(4 * ((size_t)nc + 1)) + lds_al(4 * (size_t)nnz) + lds_al(8 * (size_t)nr) + lds_al(4 * (size_t)nr) +
           2 * lds_al(4 * (size_t)nc);
}

template <bool WAVE>
__global__ void __launch_bounds__(1024) k_match_wg(const BatchDesc *descs, const int32_t *order, int32_t ngraphs,
                                                   int64_t *card, uint32_t *ctrl, RunOpt o, uint32_t arena)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ uint32_t s_loc[16];  // [0..7] level counters, [8..13] barrier state
    __shared__ int32_t s_next;
    __shared__ uint32_t s_m;
    __shared__ uint64_t s_acc[kAccN];
    Acc acc = make_acc(s_acc, stage_tmp(smem));
    Stage st = make_stage(smem);
    uint32_t *s_tmp = stage_tmp(smem);
    uint64_t *stats = reinterpret_cast<uint64_t *>(line(ctrl, L_STAT0));
    uint32_t *queue = line(ctrl, L_QUEUE);
    for (;;) {
        if (threadIdx.x == 0) s_next = (int32_t)atomicAdd(queue, 1u);
        __syncthreads();
        const int32_t qi = s_next;
        __syncthreads();
        if (qi >= ngraphs) break;
        const int32_t gi = order ? order[qi] : qi;
        const BatchDesc d = descs[gi];
        DevGraph g;
        g.colptr = d.colptr;
        g.rowind = d.rowind;
        g.nc = d.nc;
        g.nr = d.nr;
        g.cmatch = d.out_c;
        g.rw = d.rw;
        g.pred = d.pred;
        g.cdone = d.cdone;
        g.fq0 = d.fq;
        g.fq1 = d.fq + d.nc;
        g.ends = d.ends;
        g.clevel = nullptr;
        const int64_t nnz = (arena && g.nc > 0 && g.nr > 0) ? (int64_t)d.colptr[g.nc] : -1;
        const bool in_lds = nnz >= 0 && lds_graph_bytes(g.nc, g.nr, nnz) <= arena;
        if (in_lds) {
            char *a = smem + stage_lds_bytes(blockDim.x >> 6);
            int32_t *lcp = reinterpret_cast<int32_t *>(a);
            a += lds_al(4 * ((size_t)g.nc + 1));
            int32_t *lri = reinterpret_cast<int32_t *>(a);
            a += lds_al(4 * (size_t)nnz);
            g.rw = reinterpret_cast<uint64_t *>(a);
            a += lds_al(8 * (size_t)g.nr);
            g.pred = reinterpret_cast<int32_t *>(a);
            a += lds_al(4 * (size_t)g.nr);
            g.cdone = reinterpret_cast<uint32_t *>(a);
            a += lds_al(4 * (size_t)g.nc);
            g.cmatch = reinterpret_cast<int32_t *>(a);
            for (int c = threadIdx.x; c <= g.nc; c += blockDim.x) lcp[c] = d.colptr[c];
            for (int64_t i = threadIdx.x; i < nnz; i += blockDim.x) lri[i] = d.rowind[i];
            g.colptr = lcp;
            g.rowind = lri;
        }
        if (threadIdx.x == 0) s_m = 0;
        __syncthreads();
        uint32_t m0 = 0;
        for (int c = threadIdx.x; c < g.nc; c += blockDim.x) {
            const int r = d.init_c ? d.init_c[c] : -1;
            g.cmatch[c] = r;
            m0 += r >= 0;
            g.cdone[c] = 0;
        }
        for (int r = threadIdx.x; r < g.nr; r += blockDim.x)
            g.rw[r] = (uint64_t)(uint32_t)(d.init_r ? d.init_r[r] : -1);
        if (m0) atomicAdd(&s_m, m0);
        __syncthreads();
        if (threadIdx.x == 0) {
            if (s_m) atomicAdd((unsigned long long *)line(ctrl, L_INIT_CARD), (unsigned long long)s_m);
            s_m = 0;
        }
        __syncthreads();
        uint32_t ph = 0, lv = 0;
        const bool ok = (g.nc > 0 && g.nr > 0) ? run_block<WAVE>(g, ctrl, o, acc, st, s_tmp, s_loc, &ph, &lv) : true;
        __syncthreads();
        uint32_t m = 0;
        for (int r = threadIdx.x; r < g.nr; r += blockDim.x) d.out_r[r] = (int32_t)(uint32_t)g.rw[r];
        for (int c = threadIdx.x; c < g.nc; c += blockDim.x) {
            if (in_lds) d.out_c[c] = g.cmatch[c];
            m += (g.cmatch[c] >= 0);
        }
        if (m) atomicAdd(&s_m, m);
        __syncthreads();
        if (threadIdx.x == 0) {
            card[gi] = ok ? (int64_t)s_m : (int64_t)kEInternal;
            atomicAdd((unsigned long long *)line(ctrl, L_CARD), (unsigned long long)s_m);
            atomicMax(line(ctrl, L_PHASE), ph);
            atomicAdd(line(ctrl, L_LEVELS), lv);
        }
        __syncthreads();
    }
    if (o.flags & F_STATS) acc.flush(stats, false);
}

// ---------------------------------------------------------------------
// Device-side cheap initial matching (the paper initialises every run with
// a cheap greedy matching, section 4).  Parallel form: every column scans
// its rows in stored order and takes the first one it can move from -1 to
// itself with a compare-and-swap.  An unmatched column ends with all its
// rows matched, so the result is a maximal matching; which one depends on
// the schedule, unlike the sequential greedy of mcm_cheap_init_host.
__global__ void k_unmatch_all(const BatchDesc *descs, int32_t ngraphs)
{
    for (int32_t gi = blockIdx.y; gi < ngraphs; gi += gridDim.y) {
        const BatchDesc d = descs[gi];
        const int32_t n = d.nc > d.nr ? d.nc : d.nr;
        for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
            if (i < d.nc) d.out_c[i] = -1;
            if (i < d.nr) d.out_r[i] = -1;
        }
    }
}

__global__ void k_cheap_init(const BatchDesc *descs, int32_t ngraphs)
{
    for (int32_t gi = blockIdx.y; gi < ngraphs; gi += gridDim.y) {
        const BatchDesc d = descs[gi];
        for (int32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < d.nc; c += gridDim.x * blockDim.x) {
            const int32_t e = d.colptr[c + 1];
            for (int32_t j = d.colptr[c]; j < e; ++j) {
                const int32_t r = d.rowind[j];
                if (d.out_r[r] != -1) continue;
                if (atomicCAS(&d.out_r[r], -1, c) == -1) {
                    d.out_c[c] = r;
                    break;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------
// Launch helpers called by the host driver (mcm_api.cpp).

static int clamp_blocks(int64_t work, int per, int lo, int hi)
{
    int64_t b = (work + per - 1) / per;
    if (b < lo) b = lo;
    if (b > hi) b = hi;
    return (int)b;
}

static hipError_t allow_lds(const void *fn, int bytes)
{
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

hipError_t launch_zero_ctrl(uint32_t *ctrl, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_ctrl, dim3(1), dim3(256), 0, st, ctrl);
    return hipGetLastError();
}

hipError_t launch_setup(const DevGraph &g, const int32_t *ic, const int32_t *ir, uint32_t *ctrl, uint32_t *bar,
                        uint32_t flags, hipStream_t st)
{
    // the control block is cleared first: k_setup counts into it
    hipLaunchKernelGGL(k_zero_ctrl, dim3(1), dim3(256), 0, st, ctrl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // at most 1024 blocks: each adds its count of the initial matching to
    // one word, and same-address atomics serialise (~11 ns each; 8192 blocks
    // cost ~90 us on an 8 M-vertex graph)
    const int64_t n = g.nc > g.nr ? g.nc : g.nr;
    hipLaunchKernelGGL(k_setup, dim3(clamp_blocks(n, 1024, 1, 1024)), dim3(256), 0, st, g, ic, ir, ctrl, bar, flags);
    return hipGetLastError();
}

hipError_t launch_validate_csc(int32_t nc, int32_t nr, const int32_t *cp, const int32_t *ri, uint32_t *ctrl,
                               hipStream_t st)
{
    hipLaunchKernelGGL(k_validate_csc, dim3(1024), dim3(256), 0, st, nc, nr, cp, ri, ctrl);
    return hipGetLastError();
}

hipError_t launch_validate_init(int32_t nc, int32_t nr, const int32_t *cp, const int32_t *ri, const int32_t *ic,
                                const int32_t *ir, uint32_t *ctrl, hipStream_t st)
{
    hipLaunchKernelGGL(k_validate_init, dim3(1024), dim3(256), 0, st, nc, nr, cp, ri, ic, ir, ctrl);
    return hipGetLastError();
}

static const void *persistent_fn(bool wave)
{
    return wave ? reinterpret_cast<const void *>(&k_persistent<true>) : reinterpret_cast<const void *>(&k_persistent<false>);
}

hipError_t persistent_occupancy(bool wave, int block, int *blocks_per_cu)
{
    const int lds = persistent_lds_bytes(block / 64);
    hipError_t e = allow_lds(persistent_fn(wave), lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, persistent_fn(wave), block, lds);
}

hipError_t launch_persistent(const DevGraph &g, uint32_t *ctrl, uint32_t *bar, const RunOpt &o, bool wave, int blocks,
                             int block, hipStream_t st)
{
    if (blocks > kMaxGridBlocks) return hipErrorInvalidValue;
    DevGraph gg = g;
    uint32_t *cc = ctrl, *bb = bar;
    RunOpt oo = o;
    void *args[] = {&gg, &cc, &bb, &oo};
    return hipLaunchCooperativeKernel(persistent_fn(wave), dim3(blocks), dim3(block), args,
                                      (unsigned)persistent_lds_bytes(block / 64), st);
}

hipError_t launch_init_roots(const DevGraph &g, uint32_t *ctrl, const RunOpt &o, hipStream_t st)
{
    hipLaunchKernelGGL(k_init_roots, dim3(clamp_blocks(g.nc, 256, 1, 4096)), dim3(256), stage_lds_bytes(4), st, g,
                       ctrl, o);
    return hipGetLastError();
}

hipError_t launch_level(const DevGraph &g, uint32_t *ctrl, uint32_t n, uint32_t ph, int L, const RunOpt &o, bool wave,
                        int max_blocks, hipStream_t st)
{
    // about batch_min entries per wavefront when n is small
    const int blocks = clamp_blocks(n, 4 * (int)(o.batch_min ? o.batch_min : 1), 1, max_blocks);
    if (wave)
        hipLaunchKernelGGL(k_level<true>, dim3(blocks), dim3(256), stage_lds_bytes(4), st, g, ctrl, n, ph, L, o);
    else
        hipLaunchKernelGGL(k_level<false>, dim3(blocks), dim3(256), stage_lds_bytes(4), st, g, ctrl, n, ph, L, o);
    return hipGetLastError();
}

hipError_t launch_alternate(const DevGraph &g, uint32_t *ctrl, uint32_t nends, uint32_t flags, hipStream_t st)
{
    hipLaunchKernelGGL(k_alternate, dim3(clamp_blocks(nends, 256, 1, 4096)), dim3(256), 0, st, g, ctrl, flags);
    return hipGetLastError();
}

hipError_t launch_fix(const DevGraph &g, uint32_t *ctrl, uint32_t ph, uint32_t flags, hipStream_t st)
{
    hipLaunchKernelGGL(k_fix, dim3(clamp_blocks(g.nr, 256, 1, 4096)), dim3(256), 0, st, g, ctrl, ph, flags);
    return hipGetLastError();
}

hipError_t launch_finish(const DevGraph &g, int32_t *out_r, uint32_t *ctrl, hipStream_t st)
{
    const int64_t n = g.nc > g.nr ? g.nc : g.nr;
    hipLaunchKernelGGL(k_finish, dim3(clamp_blocks(n, 2048, 1, 1024)), dim3(256), 0, st, g, out_r, ctrl);
    return hipGetLastError();
}

hipError_t launch_cover(const DevGraph &g, uint32_t ph, uint8_t *cc, uint8_t *rc, uint32_t *ctrl, hipStream_t st)
{
    const int64_t n = g.nc > g.nr ? g.nc : g.nr;
    hipLaunchKernelGGL(k_cover, dim3(clamp_blocks(n, 2048, 1, 1024)), dim3(256), 0, st, g, ph, cc, rc, ctrl);
    return hipGetLastError();
}

hipError_t launch_export_pred(const DevGraph &g, uint32_t ph, int32_t *row_pred, hipStream_t st)
{
    hipLaunchKernelGGL(k_export_pred, dim3(clamp_blocks(g.nr, 256, 1, 4096)), dim3(256), 0, st, g, ph, row_pred);
    return hipGetLastError();
}

hipError_t launch_match_wg(const BatchDesc *descs, const int32_t *order, int32_t ngraphs, int64_t *card,
                           uint32_t *ctrl, const RunOpt &o, bool wave, int blocks, int block, hipStream_t st, int arena)
{
    const int lds = stage_lds_bytes(block / 64) + arena;
    if (wave)
        hipLaunchKernelGGL(k_match_wg<true>, dim3(blocks), dim3(block), lds, st, descs, order, ngraphs, card, ctrl, o,
                           (uint32_t)arena);
    else
        hipLaunchKernelGGL(k_match_wg<false>, dim3(blocks), dim3(block), lds, st, descs, order, ngraphs, card, ctrl, o,
                           (uint32_t)arena);
    return hipGetLastError();
}

// Raise the dynamic-LDS limit of the one-workgroup kernel (outside any
// stream capture).
hipError_t prepare_match_wg(int block, int arena)
{
    const int lds = stage_lds_bytes(block / 64) + arena;
    hipError_t e = allow_lds(reinterpret_cast<const void *>(&k_match_wg<true>), lds);
    if (e != hipSuccess) return e;
    return allow_lds(reinterpret_cast<const void *>(&k_match_wg<false>), lds);
}

// Occupancy of the one-workgroup kernel (blocks per CU).
hipError_t match_wg_occupancy(bool wave, int block, int *per_cu)
{
    const void *fn = wave ? reinterpret_cast<const void *>(&k_match_wg<true>) : reinterpret_cast<const void *>(&k_match_wg<false>);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, fn, block, stage_lds_bytes(block / 64));
}

hipError_t launch_cheap_init(const BatchDesc *descs, int32_t ngraphs, hipStream_t st)
{
    const dim3 grid(256, (unsigned)(ngraphs < 65535 ? ngraphs : 65535));
    hipLaunchKernelGGL(k_unmatch_all, grid, dim3(256), 0, st, descs, ngraphs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cheap_init, grid, dim3(256), 0, st, descs, ngraphs);
    return hipGetLastError();
}

static const void *multi_fn(bool wave)
{
    return wave ? reinterpret_cast<const void *>(&k_persistent_multi<true>)
                : reinterpret_cast<const void *>(&k_persistent_multi<false>);
}

// Blocks per CU of the multi-graph persistent kernel at this block size.
hipError_t multi_occupancy(bool wave, int block, int *per_cu)
{
    const int lds = stage_lds_bytes(block / 64);
    hipError_t e = allow_lds(multi_fn(wave), lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, multi_fn(wave), block, lds);
}

// setup -> cooperative launch of ngroups groups of `group` blocks that take
// the ngraphs graphs from a queue -> finish; card[ngraphs] receives |M_g|
// (or kEInternal for a graph a watchdog left undone).  ctrls: ngroups
// control blocks; bars: ngroups * group arrival lines.
hipError_t launch_multi(const BatchDesc *descs, int32_t ngraphs, int group, int ngroups, uint32_t *ctrls,
                        uint32_t *bars, int64_t *card, const RunOpt &o, bool wave, int block, hipStream_t st)
{
    if (ngraphs <= 0) return hipSuccess;
    if (ngroups < 1 || group < 1) return hipErrorInvalidValue;
    const dim3 g2(256, (unsigned)(ngraphs < 65535 ? ngraphs : 65535));
    hipLaunchKernelGGL(k_setup_multi, g2, dim3(256), 0, st, descs, ngraphs, ngroups, ctrls, bars, (uint32_t)group,
                       card);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const BatchDesc *dd = descs;
    int32_t ng = ngraphs;
    uint32_t gp = (uint32_t)group;
    uint32_t *cc = ctrls, *bb = bars;
    int64_t *cd = card;
    RunOpt oo = o;
    void *args[] = {&dd, &ng, &gp, &cc, &bb, &cd, &oo};
    e = hipLaunchCooperativeKernel(multi_fn(wave), dim3((unsigned)(ngroups * group)), dim3(block), args,
                                   (unsigned)stage_lds_bytes(block / 64), st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_finish_multi, g2, dim3(256), 0, st, descs, ngraphs, card);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_card_done, dim3((unsigned)((ngraphs + 255) / 256)), dim3(256), 0, st, ngraphs, card);
    return hipGetLastError();
}

}  // namespace mcm
