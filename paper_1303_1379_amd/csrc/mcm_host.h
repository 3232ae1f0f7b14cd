// Host-side internals shared by the C ABI sources (mcm_api.cpp,
// mcm_batch.cpp, mcm_server.cpp): launch helpers of mcm_kernels.hip,
// options, the per-device workspace, error reporting.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "../../include/mcm.h"
#include "mcm_gate.h"
#include "mcm_internal.h"

namespace mcm {

// ---- launch helpers (mcm_kernels.hip)
hipError_t launch_zero_ctrl(uint32_t *ctrl, hipStream_t st);
hipError_t launch_setup(const DevGraph &, const int32_t *, const int32_t *, uint32_t *, uint32_t *, uint32_t,
                        hipStream_t);
hipError_t launch_validate_csc(int32_t, int32_t, const int32_t *, const int32_t *, uint32_t *, hipStream_t);
hipError_t launch_validate_init(int32_t, int32_t, const int32_t *, const int32_t *, const int32_t *, const int32_t *,
                                uint32_t *, hipStream_t);
hipError_t persistent_occupancy(bool, int, int *);
hipError_t launch_persistent(const DevGraph &, uint32_t *, uint32_t *, const RunOpt &, bool, int, int, hipStream_t);
hipError_t launch_init_roots(const DevGraph &, uint32_t *, const RunOpt &, hipStream_t);
hipError_t launch_level(const DevGraph &, uint32_t *, uint32_t, uint32_t, int, const RunOpt &, bool, int, hipStream_t);
hipError_t launch_alternate(const DevGraph &, uint32_t *, uint32_t, uint32_t, hipStream_t);
hipError_t launch_fix(const DevGraph &, uint32_t *, uint32_t ph, uint32_t flags, hipStream_t);
hipError_t launch_finish(const DevGraph &, int32_t *, uint32_t *, hipStream_t);
hipError_t launch_cover(const DevGraph &, uint32_t, uint8_t *, uint8_t *, uint32_t *, hipStream_t);
hipError_t launch_export_pred(const DevGraph &, uint32_t, int32_t *, hipStream_t);
// `arena`: bytes of LDS per workgroup for graphs matched in LDS (0 = none)
hipError_t launch_match_wg(const BatchDesc *descs, const int32_t *order, int32_t ngraphs, int64_t *card,
                           uint32_t *ctrl, const RunOpt &o, bool wave, int blocks, int block, hipStream_t st,
                           int arena = 0);
hipError_t prepare_match_wg(int block, int arena = 0);
hipError_t match_wg_occupancy(bool wave, int block, int *per_cu);
hipError_t launch_cheap_init(const BatchDesc *descs, int32_t ngraphs, hipStream_t st);
hipError_t multi_occupancy(bool wave, int block, int *per_cu);
constexpr int kMultiMax = 16;  // block groups (control blocks) of a multi-graph launch, upper bound
constexpr int64_t kMaxClaimDegree = 8;  // claim=auto: atomic-maximum claims up to this many edges per row on average
hipError_t launch_multi(const BatchDesc *descs, int32_t ngraphs, int group, int ngroups, uint32_t *ctrls,
                        uint32_t *bars, int64_t *card, const RunOpt &o, bool wave, int block, hipStream_t st);

namespace host {

// Holds the cooperative-launch gate for `owner` from construction until
// destruction; the destructor first waits for `stream`, so that the gate is
// released only once every launch made under it has completed, on every
// return path.
class CoopHold {
  public:
    CoopHold(const void *owner, hipStream_t stream) : owner_(owner), st_(stream) { coop_gate().enter(owner_); }
    ~CoopHold()
    {
        (void)hipStreamSynchronize(st_);
        coop_gate().leave(owner_);
    }
    CoopHold(const CoopHold &) = delete;
    CoopHold &operator=(const CoopHold &) = delete;

  private:
    const void *owner_;
    hipStream_t st_;
};

// Live batch plans and servers, so that mcm_shutdown can release what the
// caller did not, and a later destroy call of a released handle is ignored.
void register_handle(void *h, void (*destroy)(void *));
bool unregister_handle(void *h);

// ---- errors: negative status plus a thread-local message
int64_t fail(int64_t code, const char *fmt, ...);
const std::string &last_error();

#define HIPCHK(expr)                                                                                        \
    do {                                                                                                    \
        hipError_t e_ = (expr);                                                                             \
        if (e_ != hipSuccess)                                                                               \
            return ::mcm::host::fail(MCM_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                                     __LINE__);                                                             \
    } while (0)

// ---- options (mcm_set_option)
struct Options {
    bool apsb = false;        // driver
    bool wr = true;           // bfs
    int wr_check = 2;         // WR root check (wave mapping): 0 before the scan, 1 beside the edge visit,
                              // 2 auto (mcm_match: beside on low-degree graphs, before otherwise; 1 elsewhere)
    int endpoints = 2;        // WR path ends per root: 0 all reached, 1 the first only, 2 auto (1 for APsB)
    int claim = 2;            // row claim: 0 probe + compare-and-swap, 1 atomic maximum, 2 auto (by degree)
    int flush = 2;            // grid levels: 0 reserve by a queue atomic, 1 through the counter barrier, 2 auto (1)
    int local_levels = -1;    // grid levels: a wavefront expands its own new entries this many times more
                              // (-1 = auto: 16 with probe claims, 6 with atomic-maximum claims)
    int local_edges = 1024;   // a local level takes the newest staged entries of at most this many edges (0 = 64 entries)
    int alternate = 2;        // mcm_match's Alternate: 0 classic, 1 recorded rows, 2 auto (1 on low degree)
    int schedule = 0;         // mcm_match's BFS: 0 level-synchronous, 1 level-free, 2 auto (= 0)
    int fix = 2;              // mcm_match's FixMatching: 0 every row, 1 the rows the walks touched, 2 auto (1 in
                              // phases with at most nr/64 ends, else 0)
    int keep = 128;           // level-free BFS: entries a wavefront keeps before handing older ones on
    int take = 64;            // level-free BFS: entries of its own a wavefront expands per step
    int roots = 2;            // mcm_match's root scan: 0 every column, 1 the previous phase's roots, 2 auto (1 while
                              // they were at most nc/16, else 0; decided per phase on the device)
    int mapping = 2;          // 0 thread, 1 wave, 2 auto
    int loop = 2;             // 0 device, 1 host, 2 auto
    bool validate = false;
    bool stats = false;
    std::string tuning;       // autotuner cache file ("" = memory only)
    bool autotune = false;    // batch plans time the candidate configurations
    int block = 1024;         // persistent block size
    int blocks_per_cu = 1;    // 0 = occupancy limit
    int max_blocks = 0;       // cap on persistent blocks (0 = one set per CU)
    int wg_block = 1024;      // one-workgroup matcher block size
    int64_t wg_threshold = 16384;  // nc + nr at or below which one workgroup matches alone
    bool fuse = true;         // mcm_match, probe claims: BFS level 0 in the root scan's pass (phases that do not
                              // list their roots)
    bool wg_lds = true;       // mcm_match's one-workgroup path keeps a graph that fits in the workgroup's LDS
    int64_t small_max = 256;  // frontiers up to this size are expanded by one workgroup
    int batch_min = 8;        // fewest frontier entries per wavefront batch
    int split = 64;           // heavier columns enter the frontier in pieces of this many edges (0 = off)
    int level_entries = 128;  // grid levels: one block per this many frontier entries (0 = all blocks)
    bool bar_counter = true;  // grid barrier: last arrival of a counter releases (else flag lines)
    int idle_sleep = 8;       // barrier polls of blocks that sat a level out: s_sleep(1) count between
    int64_t multi_threshold = 1 << 15;  // batch members with nc + nr above this: multi-graph launches (0 = never)
    int multi_group = 0;      // blocks per group of a multi-graph launch (0 = CUs / 8)
    double timeout_s = 20.0;  // device barrier wait limit
};
Options opts();

// ---- per-device workspace (grow-only, one per device, guarded by workspace_mutex)
struct DevInfo {
    int ncu = 0;
    int lds_block = 65536;  // bytes of LDS a workgroup may use
    double clock_khz = 100000.0;
    std::string arch;
};

struct Workspace {
    int device = -1;
    size_t cap_nc = 0, cap_nr = 0, cap_q = 0;
    uint64_t *rw = nullptr;
    int32_t *pred = nullptr;
    uint32_t *cdone = nullptr;
    int4 *fq = nullptr;
    int32_t *ends = nullptr;
    int2 *radj = nullptr;        // mate adjacency ranges (atomic-maximum claims), grown on demand
    size_t cap_radj = 0;
    int32_t *prow = nullptr;     // rows recorded by the claims (alternate=fast), grown on demand
    size_t cap_prow = 0;
    int32_t *touched = nullptr;  // rows the walks of a phase touched (fix=list), grown on demand
    size_t cap_touched = 0;
    int32_t *rlist = nullptr;    // two halves of root lists (roots=list), grown on demand
    size_t cap_rlist = 0;
    int32_t *cwork = nullptr;
    uint32_t *ctrl = nullptr;
    uint32_t *bar = nullptr;     // grid barrier arrival flags
    BatchDesc *desc = nullptr;
    size_t cap_desc = 0;
    uint32_t *mctrl = nullptr;   // control blocks of a multi-graph launch
    uint32_t *mbar = nullptr;    // its arrival lines
    int32_t *order = nullptr;
    int64_t *card = nullptr;
    uint32_t *ptrace = nullptr;    // [2 * kPhaseTrace] per-phase record of a stats run
    uint32_t *h_ptrace = nullptr;  // pinned copy
    uint32_t *h_ctrl = nullptr;  // pinned
    BatchDesc *h_desc = nullptr; // pinned
    int32_t *h_order = nullptr;  // pinned
    int64_t *h_card = nullptr;   // pinned
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    DevInfo info;
};

// Where one match keeps its state and reads its results back: the
// per-device workspace (mcm_match), or slices of the static scratch array
// with plain host memory (mcm_match_noalloc).
struct RunBufs {
    uint64_t *rw = nullptr;
    int32_t *pred = nullptr;
    uint32_t *cdone = nullptr;
    int4 *fq = nullptr;          // two frontier queues: fq and fq + cap_q
    size_t cap_q = 0;
    int32_t *ends = nullptr;
    int2 *radj = nullptr;        // atomic-maximum claims only
    int32_t *prow = nullptr;     // recorded-row Alternate only
    int32_t *touched = nullptr;  // [nr] FixMatching list, or null (every row)
    int32_t *rlist = nullptr;    // [2 nc] root lists, or null (every column)
    uint32_t *ctrl = nullptr;    // control block [L_NLINES lines]
    uint32_t *bar = nullptr;     // [kMaxGridBlocks lines]
    uint32_t *ptrace = nullptr;  // [2 * kPhaseTrace] (stats runs), or null
    BatchDesc *desc = nullptr;   // one descriptor (one-workgroup path)
    int64_t *card = nullptr;     // one count (one-workgroup path)
    uint32_t *h_ctrl = nullptr;  // host copy of the control block
    uint32_t *h_ptrace = nullptr;  // host copy of the phase record, or null
    BatchDesc *h_desc = nullptr;   // host staging of the descriptor
    hipEvent_t ev0 = nullptr, ev1 = nullptr;  // timing, or none
    DevInfo info;
};

// The workspace of (device, stream), locked for the caller until `lk` is
// released: calls on different streams use different workspaces and may
// overlap (their cooperative launches still take turns at the gate).
Workspace &acquire_workspace(int dev, const void *stream, std::unique_lock<std::mutex> &lk);
int64_t ensure_base(Workspace &w, int dev);
int64_t ensure_graph(Workspace &w, size_t nc, size_t nr, size_t qcap);
int64_t ensure_desc(Workspace &w, size_t n);
int64_t get_device_info(int dev, DevInfo *info);

// The steps of one mcm_match call, shared with mcm_match_noalloc.
int64_t check_graph_args(int32_t nc, int32_t nr, const int32_t *colptr, const int32_t *rowind);
int64_t check_null_rowind(int32_t nc, int32_t nr, const int32_t *colptr, const int32_t *rowind, hipStream_t st);
// Frontier entries per level (nc + 1, plus one per `split` edges when split
// is on); reads nnz = colptr[nc] from the device when split is on or
// nnz_out is given, through `staging` (pinned host memory, a word the
// caller owns for the call) when it is not NULL.
int64_t queue_capacity(int32_t nc, const int32_t *colptr, uint32_t split, hipStream_t st, size_t *qcap,
                       int64_t *nnz_out, int32_t *staging = nullptr);
// The row-claim, flush, root-test, Alternate and BFS-schedule forms of one
// mcm_match run (nnz < 0 when unknown).
uint32_t match_flags(const Options &o, int32_t nc, int32_t nr, int64_t nnz, bool single_wg);
// One mcm_match run on the state buffers `b`, sized for the graph and
// `flags`: validation (option validate), the one-workgroup kernel or the
// persistent phase loop, finish; returns |M| or a negative status.
int64_t match_run(const RunBufs &b, const Options &o, uint32_t flags, bool single_wg, int32_t ncols, int32_t nrows,
                  const int32_t *colptr, const int32_t *rowind, const int32_t *init_cmatch,
                  const int32_t *init_rmatch, int32_t *out_cmatch, int32_t *out_rmatch, hipStream_t st,
                  const void *owner);

uint32_t *ctrl_line(uint32_t *ctrl, int l);
uint64_t ctrl_stat(uint32_t *ctrl, int s);
RunOpt run_opt(const Options &o, uint32_t flags, int64_t nc, const DevInfo &info);
uint32_t base_flags(const Options &o, int64_t nc, int64_t nnz_hint);
int current_device(int *dev);
void record_stats(uint32_t *hc, int64_t init_card, int64_t card, float ms, int loop, uint32_t flags,
                  double clock_khz, uint32_t local_levels = 0);
// The per-phase record of the last stats run of mcm_match (pairs of BFS
// levels and unmatched rows reached), or none.
void record_phases(const uint32_t *pairs, uint32_t phases);

}  // namespace host
}  // namespace mcm
