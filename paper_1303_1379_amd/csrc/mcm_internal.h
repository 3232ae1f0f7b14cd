// Internal layout shared by the host driver and the gfx950 kernels.
#pragma once
#include <stdint.h>

namespace mcm {

// Control block: every field the kernels update concurrently sits on its
// own 128-byte line so that atomics on one do not contend with polls of
// another.
enum CtrlLine : int {
    L_QUEUE = 0,       // graph queue head of the one-workgroup-per-graph kernel
    L_BAR_GEN,         // grid barrier: epoch and loop state released by block 0 (two 64-bit words)
    L_FCOUNT0,         // frontier sizes, rotating over three levels
    L_FCOUNT1,
    L_FCOUNT2,
    L_FOUND0,          // "this level reached an unmatched row", rotating
    L_FOUND1,
    L_FOUND2,
    L_NENDS,           // unmatched rows reached in this phase
    L_STATUS,          // 0, or a negative mcm_status set by a device watchdog
    L_PHASE,           // phases run (== stamp of the last phase)
    L_LEVELS,          // BFS levels expanded, all phases
    L_CARD,            // |M| (64-bit)
    L_SMALL_LEVELS,    // levels expanded by single-workgroup runs (counter)
    L_BAR_CNT0,        // arrival counters of the counter barrier (64-bit), even and odd epochs
    L_BAR_CNT1,
    L_TAKE,            // multi-graph launch: the graph a group's block 0 took from the queue
    L_INIT_CARD,       // |M| of the initial matching (64-bit), counted by the setup
    L_AQ,              // level-free BFS: entries reserved (low 32 bits) and finished (high 32) in the
                       // phase-long queue, one 64-bit word
    L_AQ_TAKE,         // level-free BFS: entries taken from that queue
    L_NTOUCH,          // rows reported by the walks of this phase (length of DevGraph::touched)
    L_NRL0,            // roots listed in DevGraph::rlist, even and odd phases
    L_NRL1,
    L_STAT0,           // stats counters (64-bit each, own lines)
    L_NLINES = L_STAT0 + 14
};
constexpr int kLineWords = 32;        // 128 B / 4 B
constexpr int kPhaseTrace = 4096;     // phases whose (levels, ends) a stats run records
constexpr int kMaxGridBlocks = 2048;  // arrival flags of the grid barrier, one line each

enum StatIdx : int {
    S_EDGES = 0, S_EXPANDED, S_CLAIMED, S_FOUND, S_ALT, S_FIX, S_ROOTS, S_TRIES,
    S_PASS,      // bytes of the per-phase passes under the fixed byte model: 4 per column and 1/8 per
                 // column (visit reset) of the root scan, 8 per row of FixMatching
    S_T_EXPAND, S_T_FLUSH, S_T_BARRIER, S_T_SMALL, S_T_AUGMENT  // wall-clock ticks seen by block 0 (stats=1)
};

enum Flags : uint32_t {
    F_WR = 1u,        // GPUBFS-WR early exit (Algorithm 4)
    F_APSB = 2u,      // stop the level loop at the first level that finds a row
    F_STATS = 4u,     // count edges, claims, ...
    F_LEVELS = 8u,    // record column levels (inspection mode)
    F_NOAUG = 16u,    // one BFS phase only, no Alternate/Fix (levels, cover)
    F_WAVE = 32u,     // wave-balanced edge mapping (else one column per lane)
    F_WR_LATE = 64u,  // WR root check with the edge visit, off the load chain (wave mapping)
    F_ENDPOINT = 128u,  // WR: one augmenting-path end per root (the first reached), the others released
    F_BAR_COUNTER = 256u, // grid barrier: the last arrival of a counter releases (else block 0 polls flags)
    F_MAXCLAIM = 512u,    // claim a row with one atomic maximum of its stamp (no probe); needs radj
    F_DEFER = 1024u,      // grid levels: frontier slots reserved by the counter barrier's own addition,
                          // entries written after arriving (agent-scope words, -1 once consumed);
                          // needs F_BAR_COUNTER and qcap
    F_FASTALT = 2048u,    // claims record the row behind the claiming column; Alternate follows it
                          // (two independent loads per step); needs prow
    F_ASYNC = 4096u,      // APFB: a phase's BFS without levels (one phase-long queue that every
                          // wavefront takes entries from as they appear); needs qcap, excludes
                          // F_APSB and F_LEVELS
    F_FUSE0 = 8192u       // probe claims, launch for one graph: a phase that does not list its roots
                          // expands them as the root scan finds them (BFS level 0 in the scan's pass)
};

// Device view of one graph plus its working state.
struct DevGraph {
    const int32_t *colptr;   // [nc+1]
    const int32_t *rowind;   // [nnz]
    int32_t nc, nr;
    int32_t *cmatch;         // [nc]   column -> row (the output array)
    uint64_t *rw;            // [nr]   row word: low 32 = rmatch, high 32 = visit stamp
    int32_t *pred;           // [nr]   BFS predecessor column of a reached row
    uint32_t *cdone;         // [nc]   stamp of the phase in which root c found a row
    int4 *fq0, *fq1;         // [nc]   frontier queues {col, root, beg, end}
    int32_t *ends;           // [nr]   unmatched rows reached this phase
    int32_t *clevel;         // [nc]   column levels (F_LEVELS) or null
    uint64_t qcap = 0;       // entries in each of fq0 and fq1 (fq1 = fq0 + qcap; F_DEFER)
    int32_t *prow = nullptr; // [nr]   F_FASTALT: for a row claimed this phase, the mate of the column it
                             //        was claimed from (-1 for a root), or null
    int2 *radj = nullptr;    // [nr]   adjacency range {colptr[m], colptr[m+1]} of the row's mate m
                             //        (F_MAXCLAIM; meaningful while the row is matched), or null
    uint32_t *ptrace = nullptr;  // [2 * kPhaseTrace] per phase: BFS levels, unmatched rows reached
                                 // (recorded with F_STATS), or null
    int32_t *croot = nullptr;    // [nc]   F_LEVELS: root of the tree that reached each column, or null
    int32_t *touched = nullptr;  // [nr]   rows the walks of a phase wrote or stopped at, for FixMatching to
                                 //        visit instead of every row; null: FixMatching scans every row
    int32_t *rlist = nullptr;    // [2 nc] the roots of the previous phase and of this one (halves by phase
                                 //        parity), for the root scan to visit instead of every column; or null
};

// Options of one run, passed by value to the kernels.
struct RunOpt {
    uint32_t flags;        // Flags
    uint32_t max_phases;   // watchdog: phases
    uint32_t max_levels;   // watchdog: levels per phase
    uint32_t small_max;    // frontiers up to this size are expanded by one workgroup (0 = never)
    uint32_t batch_min;    // fewest frontier entries a wavefront takes per batch (1..64)
    uint32_t split;        // a column with more edges enters the frontier as several entries of at
                           // most `split` edges each (0 = never; queue capacity must allow it)
    uint32_t level_entries;  // grid levels: one block per this many frontier entries takes part
                             // (the rest wait for the level's end); 0 = every block, every level
    uint32_t idle_sleep;   // polls of a barrier waiter that did not arrive are this many s_sleep(1) apart
    uint32_t local_levels; // grid levels: times a wavefront expands its own newest entries before the
                           // level ends (0 = strictly level-synchronous)
    uint32_t local_edges;  // a local level takes the newest entries whose edges add up to at most this many
                           // (at least one entry; 0 = the newest 64 whatever their edges)
    uint32_t keep;         // level-free BFS: a wavefront keeps at most this many entries (hands older ones on)
    uint32_t take;         // level-free BFS: entries of its own a wavefront expands per step (1..64, <= keep)
    uint32_t roots_max;    // with a root list: a phase scans the previous phase's roots only when there are at
                           // most this many (else every column; reading a listed root gathers three words)
    uint32_t fix_max;      // with a touched-row list: Alternate reports its rows and FixMatching visits only
                           // those when the phase found at most this many ends (else every row is scanned)
    uint64_t timeout;      // wall-clock ticks a grid barrier may wait
};

// One graph of a batch: device addresses of its inputs, outputs and
// workspace slices (rw, pred, ends: nr entries; cdone: nc; fq: 2*nc).
struct BatchDesc {
    int32_t nc, nr;
    const int32_t *colptr, *rowind;
    const int32_t *init_c, *init_r;   // null = empty initial matching
    int32_t *out_c, *out_r;
    uint64_t *rw;
    int32_t *pred;
    uint32_t *cdone;
    int4 *fq;
    int32_t *ends;
    int64_t qcap;                     // entries per frontier queue (fq, fq + qcap); 0 = nc
};

// Per-wavefront LDS staging of queue pushes.
constexpr int kStageQ = 256;   // frontier entries per wavefront
constexpr int kStageE = 128;   // unmatched-row ends per wavefront
constexpr int kMaxWaves = 16;  // 1024-thread workgroups
// dynamic LDS bytes for a workgroup of `waves` wavefronts
inline constexpr int stage_lds_bytes(int waves) { return waves * (kStageQ * 16 + kStageE * 4) + 64 * 4; }

}  // namespace mcm
