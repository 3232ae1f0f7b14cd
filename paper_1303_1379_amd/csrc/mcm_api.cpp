// Host driver and C ABI of libmcm.so (declared in include/mcm.h).
//
// Responsibilities: argument checks, the library-owned device workspace,
// choice of launch form (one workgroup for small graphs, a persistent
// cooperative launch, or a host-driven loop of per-level launches), error
// reporting, options and counters.  All matching arithmetic runs in the
// kernels of mcm_kernels.hip; the only host-side computation is the greedy
// initial matching, offered as its own entry point.
#include "mcm_host.h"

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <numeric>
#include <vector>

using namespace mcm;

namespace mcm {

CoopGate &coop_gate()
{
    static CoopGate g;
    return g;
}

namespace host {

// ------------------------------------------------------------------ live handles
std::mutex g_handles_mu;
std::map<void *, void (*)(void *)> g_handles;

void register_handle(void *h, void (*destroy)(void *))
{
    std::lock_guard<std::mutex> lk(g_handles_mu);
    g_handles[h] = destroy;
}

bool unregister_handle(void *h)
{
    std::lock_guard<std::mutex> lk(g_handles_mu);
    return g_handles.erase(h) == 1;
}

// ------------------------------------------------------------------ errors
thread_local std::string t_err;

const std::string &last_error() { return t_err; }

int64_t fail(int64_t code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    return code;
}


// ------------------------------------------------------------------ options
Options g_opt;
std::mutex g_opt_mu;

Options opts()
{
    std::lock_guard<std::mutex> lk(g_opt_mu);
    return g_opt;
}

// ------------------------------------------------------------------ workspace
// One workspace per (device, stream), each with its own lock.  Slots live
// until mcm_shutdown (map nodes do not move).
struct WsSlot {
    std::mutex mu;
    Workspace w;
};
std::mutex g_ws_map_mu;
std::map<std::pair<int, const void *>, std::unique_ptr<WsSlot>> g_ws_map;

Workspace &acquire_workspace(int dev, const void *stream, std::unique_lock<std::mutex> &lk)
{
    WsSlot *slot;
    {
        std::lock_guard<std::mutex> g(g_ws_map_mu);
        std::unique_ptr<WsSlot> &p = g_ws_map[{dev, stream}];
        if (!p) p.reset(new WsSlot());
        slot = p.get();
    }
    lk = std::unique_lock<std::mutex>(slot->mu);
    return slot->w;
}
mcm_stats g_stats;
std::mutex g_stats_mu;
std::vector<uint32_t> g_phases;  // per-phase (levels, ends) of the last stats run of mcm_match

void free_dev(void *p)
{
    if (p) (void)hipFree(p);
}

// Releases everything a device workspace holds (mcm_shutdown).
static void release_workspace(Workspace &w)
{
    if (w.device < 0) return;
    (void)hipSetDevice(w.device);
    (void)hipDeviceSynchronize();
    for (void *p : {(void *)w.rw, (void *)w.pred, (void *)w.cdone, (void *)w.fq, (void *)w.ends, (void *)w.radj,
                    (void *)w.prow, (void *)w.touched, (void *)w.rlist, (void *)w.cwork, (void *)w.ctrl, (void *)w.bar, (void *)w.desc, (void *)w.mctrl,
                    (void *)w.mbar, (void *)w.order, (void *)w.card, (void *)w.ptrace})
        free_dev(p);
    for (void *p : {(void *)w.h_ptrace, (void *)w.h_ctrl, (void *)w.h_desc, (void *)w.h_order, (void *)w.h_card})
        if (p) (void)hipHostFree(p);
    if (w.ev0) (void)hipEventDestroy(w.ev0);
    if (w.ev1) (void)hipEventDestroy(w.ev1);
    w = Workspace();
}

// Compute units, architecture name and the wall-clock rate of device `dev`
// (queries only, nothing is allocated).
int64_t get_device_info(int dev, DevInfo *info)
{
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    info->ncu = prop.multiProcessorCount;
    info->arch = prop.gcnArchName;
    info->lds_block = (int)prop.sharedMemPerBlock;
    int rate = 0;
    if (hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, dev) == hipSuccess && rate > 0)
        info->clock_khz = rate;
    return 0;
}

int64_t ensure_base(Workspace &w, int dev)
{
    if (w.device == dev && w.ctrl) return 0;
    w.device = dev;
    int64_t rc;
    if ((rc = get_device_info(dev, &w.info))) return rc;
    HIPCHK(hipMalloc(&w.ctrl, (size_t)L_NLINES * 128));
    HIPCHK(hipMalloc(&w.bar, (size_t)kMaxGridBlocks * 128));
    HIPCHK(hipMalloc(&w.mctrl, (size_t)kMultiMax * L_NLINES * 128));
    HIPCHK(hipMalloc(&w.mbar, (size_t)kMultiMax * kMaxGridBlocks * 128));
    HIPCHK(hipHostMalloc(reinterpret_cast<void **>(&w.h_ctrl), (size_t)L_NLINES * 128, hipHostMallocDefault));
    HIPCHK(hipMalloc(&w.ptrace, sizeof(uint32_t) * 2 * kPhaseTrace));
    HIPCHK(hipHostMalloc(reinterpret_cast<void **>(&w.h_ptrace), sizeof(uint32_t) * 2 * kPhaseTrace,
                         hipHostMallocDefault));
    HIPCHK(hipEventCreate(&w.ev0));
    HIPCHK(hipEventCreate(&w.ev1));
    return 0;
}

// Grow-only workspace: per-column and per-row state for nc x nr, and two
// frontier queues of at least qcap entries each (fq and fq + cap_q).
int64_t ensure_graph(Workspace &w, size_t nc, size_t nr, size_t qcap)
{
    if (nc > w.cap_nc) {
        free_dev(w.cdone); free_dev(w.cwork);
        w.cdone = nullptr; w.cwork = nullptr;
        size_t cap = std::max(nc, w.cap_nc + w.cap_nc / 2);
        if (hipMalloc(&w.cdone, sizeof(uint32_t) * cap) != hipSuccess ||
            hipMalloc(&w.cwork, sizeof(int32_t) * cap) != hipSuccess) {
            w.cap_nc = 0;
            return fail(MCM_ENOMEM, "workspace allocation for %zu columns failed", nc);
        }
        w.cap_nc = cap;
    }
    if (qcap > w.cap_q) {
        free_dev(w.fq);
        w.fq = nullptr;
        size_t cap = std::max(qcap, w.cap_q + w.cap_q / 2);
        if (hipMalloc(&w.fq, sizeof(int4) * 2 * cap) != hipSuccess) {
            w.cap_q = 0;
            return fail(MCM_ENOMEM, "frontier queues of %zu entries failed", qcap);
        }
        w.cap_q = cap;
    }
    if (nr > w.cap_nr) {
        free_dev(w.rw); free_dev(w.pred); free_dev(w.ends);
        w.rw = nullptr; w.pred = nullptr; w.ends = nullptr;
        size_t cap = std::max(nr, w.cap_nr + w.cap_nr / 2);
        if (hipMalloc(&w.rw, sizeof(uint64_t) * cap) != hipSuccess ||
            hipMalloc(&w.pred, sizeof(int32_t) * cap) != hipSuccess ||
            hipMalloc(&w.ends, sizeof(int32_t) * cap) != hipSuccess) {
            w.cap_nr = 0;
            return fail(MCM_ENOMEM, "workspace allocation for %zu rows failed", nr);
        }
        w.cap_nr = cap;
    }
    return 0;
}

// Mate adjacency ranges for nr rows (atomic-maximum claims only).
static int64_t ensure_radj(Workspace &w, size_t nr)
{
    if (nr <= w.cap_radj) return 0;
    free_dev(w.radj);
    w.radj = nullptr;
    const size_t cap = std::max(nr, w.cap_radj + w.cap_radj / 2);
    if (hipMalloc(&w.radj, sizeof(int2) * cap) != hipSuccess) {
        w.cap_radj = 0;
        return fail(MCM_ENOMEM, "workspace allocation for %zu row ranges failed", nr);
    }
    w.cap_radj = cap;
    return 0;
}

// Rows recorded by the claims for nr rows (alternate=fast only).
static int64_t ensure_prow(Workspace &w, size_t nr)
{
    if (nr <= w.cap_prow) return 0;
    free_dev(w.prow);
    w.prow = nullptr;
    const size_t cap = std::max(nr, w.cap_prow + w.cap_prow / 2);
    if (hipMalloc(&w.prow, sizeof(int32_t) * cap) != hipSuccess) {
        w.cap_prow = 0;
        return fail(MCM_ENOMEM, "workspace allocation for %zu recorded rows failed", nr);
    }
    w.cap_prow = cap;
    return 0;
}

// An int32 array of at least n elements, grown by half again when it must grow.
static int64_t ensure_i32(int32_t *&p, size_t &cap, size_t n, const char *what)
{
    if (n <= cap) return 0;
    free_dev(p);
    p = nullptr;
    const size_t c = std::max(n, cap + cap / 2);
    if (hipMalloc(&p, sizeof(int32_t) * c) != hipSuccess) {
        cap = 0;
        return fail(MCM_ENOMEM, "workspace allocation of %zu %s failed", n, what);
    }
    cap = c;
    return 0;
}

int64_t ensure_desc(Workspace &w, size_t n)
{
    if (n <= w.cap_desc) return 0;
    free_dev(w.desc); free_dev(w.order); free_dev(w.card);
    if (w.h_desc) (void)hipHostFree(w.h_desc);
    if (w.h_order) (void)hipHostFree(w.h_order);
    if (w.h_card) (void)hipHostFree(w.h_card);
    w.desc = nullptr; w.order = nullptr; w.card = nullptr; w.h_desc = nullptr; w.h_order = nullptr; w.h_card = nullptr;
    size_t cap = std::max(n, (size_t)64);
    if (hipMalloc(&w.desc, sizeof(BatchDesc) * cap) != hipSuccess ||
        hipMalloc(&w.order, sizeof(int32_t) * cap) != hipSuccess ||
        hipMalloc(&w.card, sizeof(int64_t) * cap) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&w.h_desc), sizeof(BatchDesc) * cap, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&w.h_order), sizeof(int32_t) * cap, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&w.h_card), sizeof(int64_t) * cap, hipHostMallocDefault) != hipSuccess) {
        w.cap_desc = 0;
        return fail(MCM_ENOMEM, "descriptor allocation for %zu graphs failed", n);
    }
    w.cap_desc = cap;
    return 0;
}

uint32_t *ctrl_line(uint32_t *ctrl, int l) { return ctrl + l * kLineWords; }

// Frontier entries per level: one per column, plus one per `split` edges
// of a split column.  Reads nnz = colptr[nc] from the device (into pinned
// memory when the caller gives some: a pageable target costs a staged copy).
int64_t queue_capacity(int32_t nc, const int32_t *colptr, uint32_t split, hipStream_t st, size_t *qcap,
                       int64_t *nnz_out, int32_t *staging)
{
    *qcap = (size_t)nc + 1;
    if (nnz_out) *nnz_out = -1;
    if (split == 0 && !nnz_out) return 0;
    int32_t word = 0;
    int32_t *dst = staging ? staging : &word;
    HIPCHK(hipMemcpyAsync(dst, colptr + nc, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const int32_t nnz = *dst;
    if (nnz < 0) return fail(MCM_EINVAL, "colptr[ncols] = %d < 0", nnz);
    if (nnz_out) *nnz_out = nnz;
    if (split != 0) *qcap += (size_t)nnz / split + 1;
    return 0;
}
uint64_t ctrl_stat(uint32_t *ctrl, int s) { return reinterpret_cast<uint64_t *>(ctrl_line(ctrl, L_STAT0))[s * 16]; }

RunOpt run_opt(const Options &o, uint32_t flags, int64_t nc, const DevInfo &info)
{
    RunOpt r;
    r.flags = flags;
    r.max_phases = (uint32_t)std::min<int64_t>(nc + 2, 0x7fffffff);
    r.max_levels = (uint32_t)std::min<int64_t>(nc + 2, 0x7fffffff);
    r.small_max = (uint32_t)o.small_max;
    r.batch_min = (uint32_t)o.batch_min;
    r.split = (uint32_t)o.split;
    r.level_entries = (uint32_t)o.level_entries;
    r.idle_sleep = (uint32_t)o.idle_sleep;
    // auto: 16 where rows are probed before their claim (skewed graphs: rmat23
    // 3.08-3.10 ms against 3.13 with 12, same box), 6 with atomic-maximum
    // claims (low-degree graphs: grid2048 no faster with 10 or 16)
    r.local_levels = o.local_levels >= 0 ? (uint32_t)o.local_levels : ((flags & F_MAXCLAIM) ? 6u : 16u);
    r.local_edges = (uint32_t)o.local_edges;
    r.take = (uint32_t)std::min(o.take, 64);
    r.keep = (uint32_t)std::max(o.keep, o.take);
    // roots=list: always the list; auto: while the previous phase had at most
    // nc/16 roots (a listed root costs three gathered words, a scanned column
    // 12 streamed bytes)
    r.roots_max = o.roots == 1 ? 0xffffffffu : (uint32_t)std::min<int64_t>(nc / 16, 0xffffffff);
    r.fix_max = 0xffffffffu;  // run_graph sets the rows-based bound of fix=auto
    r.timeout = (uint64_t)(o.timeout_s * info.clock_khz * 1000.0);
    return r;
}

// Runs the phase loop on one graph whose state was set up by launch_setup.
// flags decides APFB/APsB, WR, NOAUG.  Returns 0 or a negative status; the
// control block is copied to b.h_ctrl (stream synchronised), except after
// the persistent kernel when `sync_ctrl` is false: then the copies are left
// to the caller, which queues more work first (mcm_match's finish kernel),
// and one synchronisation serves both.
int64_t run_graph(const RunBufs &b, const Options &o, const DevGraph &g, uint32_t flags, hipStream_t st, int *loop_used,
                  bool sync_ctrl = true)
{
    const bool wave = (flags & F_WAVE) != 0;
    int loop = o.loop;
    if (loop == 2) loop = 0;
    *loop_used = loop;
    if (loop != 0) flags &= ~(uint32_t)F_DEFER;  // deferred writes belong to the persistent level loop
    RunOpt ro = run_opt(o, flags, g.nc, b.info);
    // fix=auto: reporting walk rows costs a same-address atomic per 64
    // reports, scanning every row 12 streamed bytes per row; list while a
    // phase has at most nr/64 ends (rmat23's first phase has ~800 000)
    if (o.fix == 2) ro.fix_max = (uint32_t)(g.nr / 64);
    if (loop == 0) {
        int occ = 0;
        HIPCHK(persistent_occupancy(wave, o.block, &occ));
        if (occ < 1) return fail(MCM_EHIP, "persistent kernel cannot be resident with block %d", o.block);
        int per_cu = o.blocks_per_cu > 0 ? std::min(o.blocks_per_cu, occ) : occ;
        int blocks = b.info.ncu * per_cu;
        if (o.max_blocks > 0 && blocks > o.max_blocks) blocks = o.max_blocks;
        if (blocks > kMaxGridBlocks) blocks = kMaxGridBlocks;
        if (b.ev0) HIPCHK(hipEventRecord(b.ev0, st));
        HIPCHK(launch_persistent(g, b.ctrl, b.bar, ro, wave, blocks, o.block, st));
        if (b.ev1) HIPCHK(hipEventRecord(b.ev1, st));
        if ((flags & F_STATS) && g.ptrace && b.h_ptrace)
            HIPCHK(hipMemcpyAsync(b.h_ptrace, g.ptrace, sizeof(uint32_t) * 2 * kPhaseTrace, hipMemcpyDeviceToHost, st));
        if (!sync_ctrl) return 0;
        HIPCHK(hipMemcpyAsync(b.h_ctrl, b.ctrl, (size_t)L_NLINES * 128, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        return 0;
    }
    // host-driven loop: one launch per step, control block read back after each level
    uint32_t *hc = b.h_ctrl;
    auto readback = [&]() -> int64_t {
        HIPCHK(hipMemcpyAsync(hc, b.ctrl, (size_t)L_NLINES * 128, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        return 0;
    };
    uint32_t phases = 0, levels = 0, levels_before = 0;
    int64_t rc;
    if (b.ev0) HIPCHK(hipEventRecord(b.ev0, st));
    for (uint32_t ph = 1;; ++ph) {
        if (ph > ro.max_phases) return fail(MCM_EINTERNAL, "phase bound exceeded");
        HIPCHK(launch_init_roots(g, b.ctrl, ro, st));
        if ((rc = readback())) return rc;
        uint32_t n = *ctrl_line(hc, L_FCOUNT0);
        int L = 0;
        while (n > 0) {
            if ((uint32_t)L > ro.max_levels) return fail(MCM_EINTERNAL, "level bound exceeded");
            HIPCHK(launch_level(g, b.ctrl, n, ph, L, ro, wave, b.info.ncu * 8, st));
            ++levels;
            if ((rc = readback())) return rc;
            if ((flags & F_APSB) && *ctrl_line(hc, L_FOUND0 + (L % 3))) break;
            n = *ctrl_line(hc, L_FCOUNT0 + ((L + 1) % 3));
            ++L;
        }
        const uint32_t ne = *ctrl_line(hc, L_NENDS);
        if ((flags & F_STATS) && b.h_ptrace && ph <= (uint32_t)kPhaseTrace) {
            b.h_ptrace[2 * (ph - 1)] = levels - levels_before;
            b.h_ptrace[2 * (ph - 1) + 1] = ne;
        }
        levels_before = levels;
        phases = ph;
        if (ne == 0 || (flags & F_NOAUG)) break;
        HIPCHK(launch_alternate(g, b.ctrl, ne, flags, st));
        HIPCHK(launch_fix(g, b.ctrl, ph, flags, st));
    }
    if (b.ev1) HIPCHK(hipEventRecord(b.ev1, st));
    // record counts in the device control block so both loops report alike
    hc[L_PHASE * kLineWords] = phases;
    hc[L_LEVELS * kLineWords] = levels;
    HIPCHK(hipMemcpyAsync(ctrl_line(b.ctrl, L_PHASE), ctrl_line(hc, L_PHASE), 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(ctrl_line(b.ctrl, L_LEVELS), ctrl_line(hc, L_LEVELS), 4, hipMemcpyHostToDevice, st));
    if ((rc = readback())) return rc;
    return 0;
}

uint32_t base_flags(const Options &o, int64_t nc, int64_t nnz_hint)
{
    uint32_t f = 0;
    if (o.wr) f |= F_WR;
    if (o.wr_check != 0) f |= F_WR_LATE;
    if (o.bar_counter) f |= F_BAR_COUNTER;
    if (o.endpoints == 1 || (o.endpoints == 2 && o.apsb)) f |= F_ENDPOINT;
    if (o.apsb) f |= F_APSB;
    if (o.stats) f |= F_STATS;
    bool wave = o.mapping == 1;
    if (o.mapping == 2) wave = true;
    (void)nc; (void)nnz_hint;
    if (wave) f |= F_WAVE;
    return f;
}

int current_device(int *dev)
{
    return hipGetDevice(dev) == hipSuccess ? 0 : -1;
}

void record_phases(const uint32_t *pairs, uint32_t phases)
{
    std::lock_guard<std::mutex> lk(g_stats_mu);
    g_phases.clear();
    if (pairs) g_phases.assign(pairs, pairs + 2 * (size_t)std::min<uint32_t>(phases, kPhaseTrace));
}

void record_stats(uint32_t *hc, int64_t init_card, int64_t card, float ms, int loop, uint32_t flags,
                  double clock_khz, uint32_t local_levels)
{
    std::lock_guard<std::mutex> lk(g_stats_mu);
    mcm_stats s{};
    s.phases = *ctrl_line(hc, L_PHASE);
    s.levels = *ctrl_line(hc, L_LEVELS);
    s.edges_scanned = (int64_t)ctrl_stat(hc, S_EDGES);
    s.cols_expanded = (int64_t)ctrl_stat(hc, S_EXPANDED);
    s.cols_claimed = (int64_t)ctrl_stat(hc, S_CLAIMED);
    s.rows_found = (int64_t)ctrl_stat(hc, S_FOUND);
    s.alt_steps = (int64_t)ctrl_stat(hc, S_ALT);
    s.fix_resets = (int64_t)ctrl_stat(hc, S_FIX);
    s.claims_tried = (int64_t)ctrl_stat(hc, S_TRIES);
    s.pass_bytes = (int64_t)ctrl_stat(hc, S_PASS);
    s.roots = (int64_t)ctrl_stat(hc, S_ROOTS);
    s.t_expand_ms = (double)ctrl_stat(hc, S_T_EXPAND) / clock_khz;
    s.t_flush_ms = (double)ctrl_stat(hc, S_T_FLUSH) / clock_khz;
    s.t_barrier_ms = (double)ctrl_stat(hc, S_T_BARRIER) / clock_khz;
    s.t_small_ms = (double)ctrl_stat(hc, S_T_SMALL) / clock_khz;
    s.t_augment_ms = (double)ctrl_stat(hc, S_T_AUGMENT) / clock_khz;
    s.init_card = init_card;
    s.card = card;
    s.kernel_ms = ms;
    s.loop = loop;
    s.mapping = (flags & F_WAVE) ? 1 : 0;
    s.claim = (flags & F_MAXCLAIM) ? 1 : 0;
    s.flush = (flags & F_DEFER) && loop == 0 ? 1 : 0;
    s.wr_check = (flags & F_WR_LATE) ? 1 : 0;
    s.alternate = (flags & F_FASTALT) ? 1 : 0;
    s.schedule = (flags & F_ASYNC) && loop == 0 ? 1 : 0;
    s.local_levels = local_levels;
    g_stats = s;
}

int64_t check_graph_args(int32_t nc, int32_t nr, const int32_t *colptr, const int32_t *rowind)
{
    if (nc < 0 || nr < 0) return fail(MCM_EINVAL, "ncols=%d nrows=%d must be >= 0", nc, nr);
    if (nc > 0 && !colptr) return fail(MCM_EINVAL, "colptr is NULL");
    (void)rowind;
    return 0;
}

// rowind may be NULL only for a graph without edges: checked by reading
// colptr[nc] before any kernel could touch rowind.
int64_t check_null_rowind(int32_t nc, int32_t nr, const int32_t *colptr, const int32_t *rowind, hipStream_t st)
{
    if (rowind || nc == 0 || nr == 0) return 0;
    int32_t nnz = -1;
    HIPCHK(hipMemcpyAsync(&nnz, colptr + nc, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (nnz != 0) return fail(MCM_EINVAL, "rowind is NULL but colptr[ncols] = %d", nnz);
    return 0;
}

// One workgroup matches one graph (small graphs).
int64_t run_single_wg(const RunBufs &b, const Options &o, int32_t nc, int32_t nr, const int32_t *colptr,
                      const int32_t *rowind, const int32_t *ic, const int32_t *ir, int32_t *oc, int32_t *orr,
                      uint32_t flags, hipStream_t st)
{
    BatchDesc d{};
    d.nc = nc;
    d.nr = nr;
    d.colptr = colptr;
    d.rowind = rowind;
    d.init_c = ic;
    d.init_r = ir;
    d.out_c = oc;
    d.out_r = orr;
    d.rw = b.rw;
    d.pred = b.pred;
    d.cdone = b.cdone;
    d.fq = b.fq;
    d.ends = b.ends;
    *b.h_desc = d;
    // the rest of the workgroup's LDS holds the graph when it fits (a
    // kilobyte is left for the kernel's static LDS)
    const int arena = o.wg_lds ? std::max(0, (b.info.lds_block - stage_lds_bytes(o.wg_block / 64) - 1024) & ~255) : 0;
    HIPCHK(prepare_match_wg(o.wg_block, arena));
    HIPCHK(hipMemcpyAsync(b.desc, b.h_desc, sizeof(BatchDesc), hipMemcpyHostToDevice, st));
    HIPCHK(launch_zero_ctrl(b.ctrl, st));
    RunOpt ro = run_opt(o, flags, nc, b.info);
    ro.split = 0;  // the graph's queue slices hold exactly nc entries
    if (b.ev0) HIPCHK(hipEventRecord(b.ev0, st));
    HIPCHK(launch_match_wg(b.desc, nullptr, 1, b.card, b.ctrl, ro, (flags & F_WAVE) != 0, 1, o.wg_block, st, arena));
    if (b.ev1) HIPCHK(hipEventRecord(b.ev1, st));
    HIPCHK(hipMemcpyAsync(b.h_ctrl, b.ctrl, (size_t)L_NLINES * 128, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return 0;
}

// The row-claim and Alternate forms of one mcm_match run (see the options
// claim, flush, wr_check and alternate); nnz < 0 when unknown.
uint32_t match_flags(const Options &o, int32_t nc, int32_t nr, int64_t nnz, bool single_wg)
{
    uint32_t flags = base_flags(o, nc, 0);
    // Atomic-maximum claims where rows have few edges: a row then has few
    // visitors per phase and the atomic replaces a probe plus a
    // compare-and-swap.  Hub rows (skewed degrees) keep the probe, which lets
    // all but the first visitor of a level skip the atomic.
    const bool low_degree = nnz >= 0 && nnz <= kMaxClaimDegree * (int64_t)nr;
    if (!single_wg && (o.claim == 1 || (o.claim == 2 && low_degree))) flags |= F_MAXCLAIM;
    // The WR root check: beside the edge visit on low-degree graphs (their
    // long chains of small levels would wait for the root's load before the
    // scan), before the scan on skewed ones (their large levels save the
    // rowind loads of trees that are done).
    if (!single_wg && o.wr_check == 2 && !low_degree) flags &= ~(uint32_t)F_WR_LATE;
    // Persistent level loop with the counter barrier: a grid level's next
    // frontier is reserved by the barrier's own addition, and grid levels
    // pass their barriers without fences (what they share is in agent-scope
    // atomics).  It pays where levels are many and small (low degree); on
    // skewed graphs (few, large levels) the per-entry checks cost more.
    if (!single_wg && o.bar_counter && o.loop != 1 && (o.flush == 1 || (o.flush == 2 && low_degree)))
        flags |= F_DEFER;
    // Alternate along recorded rows where walks are long (low-degree graphs:
    // grid2048 430 -> 413 ms); on skewed graphs the extra load per entry
    // and store per claim cost more than their short walks save, and without
    // WR (many ends per tree) walks would repeat their shared ways.
    if (!single_wg && (o.alternate == 1 || (o.alternate == 2 && low_degree && o.wr))) flags |= F_FASTALT;
    // Level 0 in the root scan's pass where rows are probed before their
    // claim (the two-edge rounds; deferred levels keep their checked queue
    // protocol, and the level-free schedule has no level 0)
    if (!single_wg && o.fuse && !(flags & (F_MAXCLAIM | F_DEFER))) flags |= F_FUSE0;
    // Level-free BFS (APFB on the device loop only, on request: measured
    // slower than the level loop on grid2048 by 14x): no grid barrier
    // between BFS levels; the deferred level forms do not apply then.
    if (!single_wg && !o.apsb && o.loop != 1 && o.schedule == 1) {
        flags |= F_ASYNC;
        flags &= ~(uint32_t)F_DEFER;
    }
    return flags;
}

// One mcm_match run on state buffers `b` (sized for the graph and `flags`):
// optional validation, then the one-workgroup kernel or setup, the phase
// loop and finish.  Returns |M| or a negative status; records the stats.
int64_t match_run(const RunBufs &b, const Options &o, uint32_t flags, bool single_wg, int32_t ncols, int32_t nrows,
                  const int32_t *colptr, const int32_t *rowind, const int32_t *init_cmatch,
                  const int32_t *init_rmatch, int32_t *out_cmatch, int32_t *out_rmatch, hipStream_t st,
                  const void *owner)
{
    int64_t rc;
    if (o.validate) {
        // the structure first; the initial matching (whose on-edge check
        // scans column ranges of rowind) only on a sound structure
        auto status = [&]() -> int64_t {
            HIPCHK(hipMemcpyAsync(b.h_ctrl, b.ctrl, (size_t)L_NLINES * 128, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            return (int32_t)*ctrl_line(b.h_ctrl, L_STATUS);
        };
        HIPCHK(launch_zero_ctrl(b.ctrl, st));
        HIPCHK(launch_validate_csc(ncols, nrows, colptr, rowind, b.ctrl, st));
        int64_t s = status();
        if (s == MCM_EINVAL) return fail(MCM_EINVAL, "malformed CSC input");
        if (s < 0) return s;
        if (init_cmatch) {
            HIPCHK(launch_validate_init(ncols, nrows, colptr, rowind, init_cmatch, init_rmatch, b.ctrl, st));
            s = status();
            if (s == MCM_EBADINIT) return fail(MCM_EBADINIT, "initial matching is inconsistent or not on edges");
            if (s < 0) return s;
        }
    }
    int loop = 0;
    float ms = 0.f;
    if (single_wg) {
        if ((rc = run_single_wg(b, o, ncols, nrows, colptr, rowind, init_cmatch, init_rmatch, out_cmatch, out_rmatch,
                                flags, st)))
            return rc;
        if (b.ev0) HIPCHK(hipEventElapsedTime(&ms, b.ev0, b.ev1));
        loop = 2;
        const int64_t card = (int64_t)*reinterpret_cast<uint64_t *>(ctrl_line(b.h_ctrl, L_CARD));
        const int32_t s = (int32_t)*ctrl_line(b.h_ctrl, L_STATUS);
        const int64_t init_card = (int64_t)*reinterpret_cast<uint64_t *>(ctrl_line(b.h_ctrl, L_INIT_CARD));
        record_stats(b.h_ctrl, init_card, card, ms, loop, flags, b.info.clock_khz);
        record_phases(nullptr, 0);  // the one-workgroup path keeps no per-phase record
        if (s != 0) return fail(MCM_EINTERNAL, "device watchdog fired (status %d)", s);
        return card;
    }

    DevGraph g;
    g.colptr = colptr;
    g.rowind = rowind;
    g.nc = ncols;
    g.nr = nrows;
    g.cmatch = out_cmatch;
    g.rw = b.rw;
    g.pred = b.pred;
    g.cdone = b.cdone;
    g.fq0 = b.fq;
    g.fq1 = b.fq + b.cap_q;
    g.ends = b.ends;
    g.clevel = nullptr;
    g.ptrace = (flags & F_STATS) ? b.ptrace : nullptr;
    g.radj = (flags & F_MAXCLAIM) ? b.radj : nullptr;
    g.prow = (flags & F_FASTALT) ? b.prow : nullptr;
    g.touched = o.fix != 0 ? b.touched : nullptr;
    g.rlist = o.roots != 0 ? b.rlist : nullptr;
    g.qcap = b.cap_q;
    CoopHold hold(owner, st);  // at most one cooperative launch in flight in the process
    HIPCHK(launch_setup(g, init_cmatch, init_rmatch, b.ctrl, b.bar, flags, st));
    // the control block is read once, after the finish kernel
    if ((rc = run_graph(b, o, g, flags, st, &loop, false))) return rc;
    HIPCHK(launch_finish(g, out_rmatch, b.ctrl, st));
    HIPCHK(hipMemcpyAsync(b.h_ctrl, b.ctrl, (size_t)L_NLINES * 128, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (b.ev0) HIPCHK(hipEventElapsedTime(&ms, b.ev0, b.ev1));
    const int32_t s = (int32_t)*ctrl_line(b.h_ctrl, L_STATUS);
    const int64_t card = (int64_t)*reinterpret_cast<uint64_t *>(ctrl_line(b.h_ctrl, L_CARD));
    const int64_t init_card = (int64_t)*reinterpret_cast<uint64_t *>(ctrl_line(b.h_ctrl, L_INIT_CARD));
    record_stats(b.h_ctrl, init_card, card, ms, loop, flags, b.info.clock_khz,
                 loop == 0 ? run_opt(o, flags, ncols, b.info).local_levels : 0u);
    record_phases((flags & F_STATS) && b.h_ptrace ? b.h_ptrace : nullptr, *ctrl_line(b.h_ctrl, L_PHASE));
    if (s != 0) return fail(MCM_EINTERNAL, "device watchdog fired (status %d)", s);
    return card;
}

RunBufs bufs_of(Workspace &w)
{
    RunBufs b;
    b.rw = w.rw;
    b.pred = w.pred;
    b.cdone = w.cdone;
    b.fq = w.fq;
    b.cap_q = w.cap_q;
    b.ends = w.ends;
    b.radj = w.radj;
    b.prow = w.prow;
    b.touched = w.touched;
    b.rlist = w.rlist;
    b.ctrl = w.ctrl;
    b.bar = w.bar;
    b.ptrace = w.ptrace;
    b.desc = w.desc;
    b.card = w.card;
    b.h_ctrl = w.h_ctrl;
    b.h_ptrace = w.h_ptrace;
    b.h_desc = w.h_desc;
    b.ev0 = w.ev0;
    b.ev1 = w.ev1;
    b.info = w.info;
    return b;
}

}  // namespace host
}  // namespace mcm

using namespace mcm::host;

// =================================================================== C ABI
extern "C" {

const char *mcm_version(void) { return "mcm-gfx950 0.1"; }

const char *mcm_strerror(int64_t status)
{
    if (status < 0 && !t_err.empty()) return t_err.c_str();
    switch (status) {
    case MCM_OK: return "ok";
    case MCM_EINVAL: return "invalid argument";
    case MCM_ENOMEM: return "out of memory";
    case MCM_EHIP: return "HIP runtime error";
    case MCM_EBADINIT: return "initial matching is not a matching of the graph";
    case MCM_EINTERNAL: return "internal bound exceeded (watchdog)";
    case MCM_ENOTMAX: return "matching is not maximum";
    default: return status >= 0 ? "ok" : "unknown error";
    }
}

int mcm_set_option(const char *key, const char *value)
{
    if (!key || !value) return (int)fail(MCM_EINVAL, "NULL option key or value");
    std::lock_guard<std::mutex> lk(g_opt_mu);
    std::string k(key), v(value);
    auto as_int = [&](int64_t lo, int64_t hi, int64_t *out) -> bool {
        char *end = nullptr;
        long long x = strtoll(value, &end, 10);
        if (!end || *end || end == value || x < lo || x > hi) return false;
        *out = x;
        return true;
    };
    int64_t x = 0;
    if (k == "driver") {
        if (v == "apfb") g_opt.apsb = false;
        else if (v == "apsb") g_opt.apsb = true;
        else return (int)fail(MCM_EINVAL, "driver must be apfb or apsb");
    } else if (k == "bfs") {
        if (v == "wr") g_opt.wr = true;
        else if (v == "plain") g_opt.wr = false;
        else return (int)fail(MCM_EINVAL, "bfs must be wr or plain");
    } else if (k == "mapping") {
        if (v == "thread") g_opt.mapping = 0;
        else if (v == "wave") g_opt.mapping = 1;
        else if (v == "auto") g_opt.mapping = 2;
        else return (int)fail(MCM_EINVAL, "mapping must be thread, wave or auto");
    } else if (k == "loop") {
        if (v == "device") g_opt.loop = 0;
        else if (v == "host") g_opt.loop = 1;
        else if (v == "auto") g_opt.loop = 2;
        else return (int)fail(MCM_EINVAL, "loop must be device, host or auto");
    } else if (k == "validate") {
        if (v == "0" || v == "1") g_opt.validate = v == "1";
        else return (int)fail(MCM_EINVAL, "validate must be 0 or 1");
    } else if (k == "stats") {
        if (v == "0" || v == "1") g_opt.stats = v == "1";
        else return (int)fail(MCM_EINVAL, "stats must be 0 or 1");
    } else if (k == "tuning") {
        g_opt.tuning = v;
    } else if (k == "autotune") {
        if (v == "0" || v == "1") g_opt.autotune = v == "1";
        else return (int)fail(MCM_EINVAL, "autotune must be 0 or 1");
    } else if (k == "block") {
        if (!as_int(64, 1024, &x) || x % 64) return (int)fail(MCM_EINVAL, "block must be a multiple of 64 in [64, 1024]");
        g_opt.block = (int)x;
    } else if (k == "blocks_per_cu") {
        if (!as_int(0, 32, &x)) return (int)fail(MCM_EINVAL, "blocks_per_cu must be in [0, 32]");
        g_opt.blocks_per_cu = (int)x;
    } else if (k == "max_blocks") {
        if (!as_int(0, kMaxGridBlocks, &x)) return (int)fail(MCM_EINVAL, "max_blocks must be in [0, 2048]");
        g_opt.max_blocks = (int)x;
    } else if (k == "wg_block") {
        if (!as_int(64, 1024, &x) || x % 64) return (int)fail(MCM_EINVAL, "wg_block must be a multiple of 64 in [64, 1024]");
        g_opt.wg_block = (int)x;
    } else if (k == "wg_threshold") {
        if (!as_int(0, (int64_t)1 << 40, &x)) return (int)fail(MCM_EINVAL, "wg_threshold must be >= 0");
        g_opt.wg_threshold = x;
    } else if (k == "batch_min") {
        if (!as_int(1, 64, &x)) return (int)fail(MCM_EINVAL, "batch_min must be in [1, 64]");
        g_opt.batch_min = (int)x;
    } else if (k == "split") {
        if (!as_int(0, (int64_t)1 << 30, &x) || (x != 0 && x < 64))
            return (int)fail(MCM_EINVAL, "split must be 0 or in [64, 2^30]");
        g_opt.split = (int)x;
    } else if (k == "level_entries") {
        if (!as_int(0, 1 << 30, &x)) return (int)fail(MCM_EINVAL, "level_entries must be in [0, 2^30]");
        g_opt.level_entries = (int)x;
    } else if (k == "endpoints") {
        if (v == "all") g_opt.endpoints = 0;
        else if (v == "one") g_opt.endpoints = 1;
        else if (v == "auto") g_opt.endpoints = 2;
        else return (int)fail(MCM_EINVAL, "endpoints must be all, one or auto");
    } else if (k == "alternate") {
        if (v == "fast") g_opt.alternate = 1;
        else if (v == "classic") g_opt.alternate = 0;
        else if (v == "auto") g_opt.alternate = 2;
        else return (int)fail(MCM_EINVAL, "alternate must be fast, classic or auto");
    } else if (k == "fuse") {
        if (v == "off") g_opt.fuse = false;
        else if (v == "on") g_opt.fuse = true;
        else return (int)fail(MCM_EINVAL, "fuse must be on or off");
    } else if (k == "wg_lds") {
        if (v == "off") g_opt.wg_lds = false;
        else if (v == "on") g_opt.wg_lds = true;
        else return (int)fail(MCM_EINVAL, "wg_lds must be on or off");
    } else if (k == "local_edges") {
        if (!as_int(0, 1 << 20, &x)) return (int)fail(MCM_EINVAL, "local_edges must be in [0, 1048576]");
        g_opt.local_edges = (int)x;
    } else if (k == "local_levels") {
        if (v == "auto") g_opt.local_levels = -1;
        else if (!as_int(0, 16, &x)) return (int)fail(MCM_EINVAL, "local_levels must be auto or in [0, 16]");
        else g_opt.local_levels = (int)x;
    } else if (k == "flush") {
        if (v == "atomic") g_opt.flush = 0;
        else if (v == "defer") g_opt.flush = 1;
        else if (v == "auto") g_opt.flush = 2;
        else return (int)fail(MCM_EINVAL, "flush must be atomic, defer or auto");
    } else if (k == "keep") {
        if (!as_int(1, 192, &x)) return (int)fail(MCM_EINVAL, "keep must be in [1, 192]");
        g_opt.keep = (int)x;
    } else if (k == "take") {
        if (!as_int(1, 64, &x)) return (int)fail(MCM_EINVAL, "take must be in [1, 64]");
        g_opt.take = (int)x;
    } else if (k == "fix") {
        if (v == "scan") g_opt.fix = 0;
        else if (v == "list") g_opt.fix = 1;
        else if (v == "auto") g_opt.fix = 2;
        else return (int)fail(MCM_EINVAL, "fix must be scan, list or auto");
    } else if (k == "roots") {
        if (v == "scan") g_opt.roots = 0;
        else if (v == "list") g_opt.roots = 1;
        else if (v == "auto") g_opt.roots = 2;
        else return (int)fail(MCM_EINVAL, "roots must be scan, list or auto");
    } else if (k == "schedule") {
        if (v == "levels") g_opt.schedule = 0;
        else if (v == "async") g_opt.schedule = 1;
        else if (v == "auto") g_opt.schedule = 2;
        else return (int)fail(MCM_EINVAL, "schedule must be levels, async or auto");
    } else if (k == "claim") {
        if (v == "probe") g_opt.claim = 0;
        else if (v == "max") g_opt.claim = 1;
        else if (v == "auto") g_opt.claim = 2;
        else return (int)fail(MCM_EINVAL, "claim must be probe, max or auto");
    } else if (k == "barrier") {
        if (v == "flags") g_opt.bar_counter = false;
        else if (v == "counter") g_opt.bar_counter = true;
        else return (int)fail(MCM_EINVAL, "barrier must be flags or counter");
    } else if (k == "wr_check") {
        if (v == "late") g_opt.wr_check = 1;
        else if (v == "early") g_opt.wr_check = 0;
        else if (v == "auto") g_opt.wr_check = 2;
        else return (int)fail(MCM_EINVAL, "wr_check must be early, late or auto");
    } else if (k == "idle_sleep") {
        if (!as_int(0, 4096, &x)) return (int)fail(MCM_EINVAL, "idle_sleep must be in [0, 4096]");
        g_opt.idle_sleep = (int)x;
    } else if (k == "multi_threshold") {
        if (!as_int(0, (int64_t)1 << 40, &x)) return (int)fail(MCM_EINVAL, "multi_threshold must be >= 0");
        g_opt.multi_threshold = x;
    } else if (k == "multi_group") {
        if (!as_int(0, kMaxGridBlocks, &x)) return (int)fail(MCM_EINVAL, "multi_group must be in [0, 2048]");
        g_opt.multi_group = (int)x;
    } else if (k == "small_max") {
        if (!as_int(0, (int64_t)1 << 30, &x)) return (int)fail(MCM_EINVAL, "small_max must be in [0, 2^30]");
        g_opt.small_max = x;
    } else if (k == "timeout_s") {
        char *end = nullptr;
        double d = strtod(value, &end);
        if (!end || *end || !(d > 0.0 && d <= 600.0)) return (int)fail(MCM_EINVAL, "timeout_s must be in (0, 600]");
        g_opt.timeout_s = d;
    } else {
        return (int)fail(MCM_EINVAL, "unknown option '%s'", key);
    }
    return MCM_OK;
}

int mcm_get_option(const char *key, char *buf, int32_t len)
{
    if (!key || !buf || len <= 0) return (int)fail(MCM_EINVAL, "bad arguments");
    Options o = opts();
    std::string k(key), v;
    static const char *maps[] = {"thread", "wave", "auto"};
    static const char *loops[] = {"device", "host", "auto"};
    if (k == "driver") v = o.apsb ? "apsb" : "apfb";
    else if (k == "bfs") v = o.wr ? "wr" : "plain";
    else if (k == "mapping") v = maps[o.mapping];
    else if (k == "loop") v = loops[o.loop];
    else if (k == "validate") v = o.validate ? "1" : "0";
    else if (k == "stats") v = o.stats ? "1" : "0";
    else if (k == "tuning") v = o.tuning;
    else if (k == "autotune") v = o.autotune ? "1" : "0";
    else if (k == "block") v = std::to_string(o.block);
    else if (k == "blocks_per_cu") v = std::to_string(o.blocks_per_cu);
    else if (k == "max_blocks") v = std::to_string(o.max_blocks);
    else if (k == "wg_block") v = std::to_string(o.wg_block);
    else if (k == "wg_threshold") v = std::to_string(o.wg_threshold);
    else if (k == "small_max") v = std::to_string(o.small_max);
    else if (k == "multi_threshold") v = std::to_string(o.multi_threshold);
    else if (k == "level_entries") v = std::to_string(o.level_entries);
    else if (k == "idle_sleep") v = std::to_string(o.idle_sleep);
    else if (k == "wr_check") v = o.wr_check == 0 ? "early" : (o.wr_check == 1 ? "late" : "auto");
    else if (k == "barrier") v = o.bar_counter ? "counter" : "flags";
    else if (k == "endpoints") v = o.endpoints == 0 ? "all" : (o.endpoints == 1 ? "one" : "auto");
    else if (k == "claim") v = o.claim == 0 ? "probe" : (o.claim == 1 ? "max" : "auto");
    else if (k == "schedule") v = o.schedule == 0 ? "levels" : (o.schedule == 1 ? "async" : "auto");
    else if (k == "fix") v = o.fix == 0 ? "scan" : (o.fix == 1 ? "list" : "auto");
    else if (k == "keep") v = std::to_string(o.keep);
    else if (k == "take") v = std::to_string(o.take);
    else if (k == "roots") v = o.roots == 0 ? "scan" : (o.roots == 1 ? "list" : "auto");
    else if (k == "flush") v = o.flush == 0 ? "atomic" : (o.flush == 1 ? "defer" : "auto");
    else if (k == "local_edges") v = std::to_string(o.local_edges);
    else if (k == "wg_lds") v = o.wg_lds ? "on" : "off";
    else if (k == "fuse") v = o.fuse ? "on" : "off";
    else if (k == "local_levels") v = o.local_levels < 0 ? "auto" : std::to_string(o.local_levels);
    else if (k == "alternate") v = o.alternate == 0 ? "classic" : (o.alternate == 1 ? "fast" : "auto");
    else if (k == "multi_group") v = std::to_string(o.multi_group);
    else if (k == "batch_min") v = std::to_string(o.batch_min);
    else if (k == "split") v = std::to_string(o.split);
    else if (k == "timeout_s") v = std::to_string(o.timeout_s);
    else return (int)fail(MCM_EINVAL, "unknown option '%s'", key);
    snprintf(buf, (size_t)len, "%s", v.c_str());
    return MCM_OK;
}

int mcm_last_stats(mcm_stats *out)
{
    if (!out) return (int)fail(MCM_EINVAL, "NULL stats pointer");
    std::lock_guard<std::mutex> lk(g_stats_mu);
    *out = g_stats;
    return MCM_OK;
}

int64_t mcm_last_phases(int32_t *levels, int32_t *ends, int64_t cap)
{
    if (cap < 0 || (cap > 0 && (!levels || !ends))) return fail(MCM_EINVAL, "NULL output or negative capacity");
    std::lock_guard<std::mutex> lk(g_stats_mu);
    const int64_t n = (int64_t)g_phases.size() / 2;
    for (int64_t i = 0; i < std::min(n, cap); ++i) {
        levels[i] = (int32_t)g_phases[2 * i];
        ends[i] = (int32_t)g_phases[2 * i + 1];
    }
    return n;
}

int64_t mcm_cheap_init_host(int32_t ncols, int32_t nrows, const int32_t *colptr, const int32_t *rowind, int32_t *cmatch,
                            int32_t *rmatch)
{
    if (ncols < 0 || nrows < 0 || (ncols > 0 && (!colptr || !cmatch)) || (nrows > 0 && !rmatch))
        return fail(MCM_EINVAL, "bad arguments to mcm_cheap_init_host");
    std::fill(cmatch, cmatch + ncols, -1);
    std::fill(rmatch, rmatch + nrows, -1);
    int64_t card = 0;
    for (int32_t c = 0; c < ncols; ++c) {
        const int32_t b = colptr[c], e = colptr[c + 1];
        if (e < b) return fail(MCM_EINVAL, "colptr decreases at column %d", c);
        for (int32_t j = b; j < e; ++j) {
            const int32_t r = rowind[j];
            if (r < 0 || r >= nrows) return fail(MCM_EINVAL, "row index %d out of range at %d", r, j);
            if (rmatch[r] < 0) {
                rmatch[r] = c;
                cmatch[c] = r;
                ++card;
                break;
            }
        }
    }
    return card;
}

int64_t mcm_match(int32_t ncols, int32_t nrows, const int32_t *colptr, const int32_t *rowind,
                  const int32_t *init_cmatch, const int32_t *init_rmatch, int32_t *out_cmatch, int32_t *out_rmatch,
                  void *stream)
{
    int64_t rc;
    if ((rc = check_graph_args(ncols, nrows, colptr, rowind))) return rc;
    if ((init_cmatch == nullptr) != (init_rmatch == nullptr))
        return fail(MCM_EINVAL, "init_cmatch and init_rmatch must both be NULL or both be given");
    if ((ncols > 0 && !out_cmatch) || (nrows > 0 && !out_rmatch)) return fail(MCM_EINVAL, "output array is NULL");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if ((rc = check_null_rowind(ncols, nrows, colptr, rowind, st))) return rc;
    if (ncols == 0 || nrows == 0) {
        if (ncols > 0) HIPCHK(hipMemsetAsync(out_cmatch, 0xff, sizeof(int32_t) * ncols, st));
        if (nrows > 0) HIPCHK(hipMemsetAsync(out_rmatch, 0xff, sizeof(int32_t) * nrows, st));
        HIPCHK(hipStreamSynchronize(st));
        return 0;
    }
    int dev = 0;
    if (current_device(&dev) || dev < 0 || dev >= 64) return fail(MCM_EHIP, "no current HIP device");
    const Options o = opts();
    std::unique_lock<std::mutex> lk;
    Workspace &w = acquire_workspace(dev, stream, lk);
    if ((rc = ensure_base(w, dev))) return rc;
    const bool single_wg = (int64_t)ncols + nrows <= o.wg_threshold;
    size_t qcap = 0;
    int64_t nnz = -1;
    // (the pinned control-block copy is free until the run reads it back)
    if ((rc = queue_capacity(ncols, colptr, single_wg ? 0u : (uint32_t)o.split, st, &qcap,
                             single_wg || (o.claim != 2 && o.flush != 2 && o.wr_check != 2 && o.alternate != 2)
                                 ? nullptr
                                 : &nnz,
                             reinterpret_cast<int32_t *>(w.h_ctrl))))
        return rc;
    if ((rc = ensure_graph(w, (size_t)ncols, (size_t)nrows, std::max(qcap, (size_t)ncols)))) return rc;
    if (single_wg && (rc = ensure_desc(w, 1))) return rc;
    const uint32_t flags = match_flags(o, ncols, nrows, nnz, single_wg);
    if ((flags & F_MAXCLAIM) && (rc = ensure_radj(w, (size_t)nrows))) return rc;
    if ((flags & F_FASTALT) && (rc = ensure_prow(w, (size_t)nrows))) return rc;
    if (!single_wg && o.fix != 0 && (rc = ensure_i32(w.touched, w.cap_touched, (size_t)nrows, "touched rows")))
        return rc;
    if (!single_wg && o.roots != 0 && (rc = ensure_i32(w.rlist, w.cap_rlist, 2 * (size_t)ncols, "listed roots")))
        return rc;
    return match_run(bufs_of(w), o, flags, single_wg, ncols, nrows, colptr, rowind, init_cmatch, init_rmatch,
                     out_cmatch, out_rmatch, st, stream);
}

// Shared by mcm_konig_cover, mcm_bfs_levels and mcm_bfs_forest: one
// complete BFS phase (no augmentation) from the caller's matching, on
// workspace copies, strictly level-synchronous.  Without `forest` it is
// GPUBFS with compare-and-swap claims (the schedule-independent level sets);
// with it, the BFS form the options select for mcm_match: GPUBFS-WR or
// GPUBFS ("bfs"), one end per root or all ("endpoints" one / other), claims
// by atomic maximum when "claim" is "max", deferred levels when "flush" is
// "defer", root test early or late ("wr_check").
static int64_t one_bfs_phase(Workspace &w, const Options &o, int32_t nc, int32_t nr, const int32_t *colptr,
                             const int32_t *rowind, const int32_t *cm, const int32_t *rm, int32_t *clevel,
                             int32_t *croot, bool forest, hipStream_t st, DevGraph *gout)
{
    int64_t rc;
    size_t qcap = 0;
    if ((rc = queue_capacity(nc, colptr, (uint32_t)o.split, st, &qcap, nullptr))) return rc;
    if ((rc = ensure_graph(w, (size_t)nc, (size_t)nr, qcap))) return rc;
    DevGraph g;
    g.colptr = colptr;
    g.rowind = rowind;
    g.nc = nc;
    g.nr = nr;
    g.cmatch = w.cwork;
    g.rw = w.rw;
    g.pred = w.pred;
    g.cdone = w.cdone;
    g.fq0 = w.fq;
    g.fq1 = w.fq + w.cap_q;
    g.ends = w.ends;
    g.clevel = clevel;
    g.croot = croot;
    g.qcap = w.cap_q;
    uint32_t flags = F_NOAUG | (clevel ? F_LEVELS : 0u);
    if (o.mapping != 0) flags |= F_WAVE;
    if (forest) {
        if (o.wr) flags |= F_WR;
        if (o.wr_check != 0) flags |= F_WR_LATE;
        if (o.endpoints == 1) flags |= F_ENDPOINT;
        if (o.bar_counter) flags |= F_BAR_COUNTER;
        if (o.bar_counter && o.loop != 1 && o.flush == 1) flags |= F_DEFER;
        if (o.claim == 1) {
            if ((rc = ensure_radj(w, (size_t)nr))) return rc;
            g.radj = w.radj;
            flags |= F_MAXCLAIM;
        }
    }
    HIPCHK(launch_setup(g, cm, rm, w.ctrl, w.bar, flags, st));
    int loop = 0;
    Options oo = o;
    if ((rc = run_graph(bufs_of(w), oo, g, flags, st, &loop))) return rc;
    const int32_t s = (int32_t)*ctrl_line(w.h_ctrl, L_STATUS);
    if (s != 0) return fail(MCM_EINTERNAL, "device watchdog fired (status %d)", s);
    *gout = g;
    return 0;
}

int64_t mcm_konig_cover(int32_t ncols, int32_t nrows, const int32_t *colptr, const int32_t *rowind,
                        const int32_t *cmatch, const int32_t *rmatch, uint8_t *col_in_cover, uint8_t *row_in_cover,
                        void *stream)
{
    int64_t rc;
    if ((rc = check_graph_args(ncols, nrows, colptr, rowind))) return rc;
    if ((ncols > 0 && (!cmatch || !col_in_cover)) || (nrows > 0 && (!rmatch || !row_in_cover)))
        return fail(MCM_EINVAL, "NULL matching or cover array");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if ((rc = check_null_rowind(ncols, nrows, colptr, rowind, st))) return rc;
    if (ncols == 0 || nrows == 0) {
        if (ncols > 0) HIPCHK(hipMemsetAsync(col_in_cover, 0, ncols, st));
        if (nrows > 0) HIPCHK(hipMemsetAsync(row_in_cover, 0, nrows, st));
        HIPCHK(hipStreamSynchronize(st));
        return 0;
    }
    int dev = 0;
    if (current_device(&dev) || dev < 0 || dev >= 64) return fail(MCM_EHIP, "no current HIP device");
    const Options o = opts();
    std::unique_lock<std::mutex> lk;
    Workspace &w = acquire_workspace(dev, stream, lk);
    if ((rc = ensure_base(w, dev))) return rc;
    CoopHold hold(stream, st);
    DevGraph g;
    if ((rc = one_bfs_phase(w, o, ncols, nrows, colptr, rowind, cmatch, rmatch, nullptr, nullptr, false, st, &g)))
        return rc;
    if (*ctrl_line(w.h_ctrl, L_NENDS) != 0) return fail(MCM_ENOTMAX, "the matching admits an augmenting path");
    HIPCHK(launch_cover(g, 1, col_in_cover, row_in_cover, w.ctrl, st));
    HIPCHK(hipMemcpyAsync(w.h_ctrl, w.ctrl, (size_t)L_NLINES * 128, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return (int64_t)*reinterpret_cast<uint64_t *>(ctrl_line(w.h_ctrl, L_CARD));
}

int64_t mcm_bfs_levels(int32_t ncols, int32_t nrows, const int32_t *colptr, const int32_t *rowind,
                       const int32_t *cmatch, const int32_t *rmatch, int32_t *col_level, int32_t *row_pred, void *stream)
{
    int64_t rc;
    if ((rc = check_graph_args(ncols, nrows, colptr, rowind))) return rc;
    if ((ncols > 0 && (!cmatch || !col_level)) || (nrows > 0 && (!rmatch || !row_pred)))
        return fail(MCM_EINVAL, "NULL matching or output array");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if ((rc = check_null_rowind(ncols, nrows, colptr, rowind, st))) return rc;
    if (ncols == 0 || nrows == 0) {
        // no edges: unmatched columns are level 0, nothing else is reached
        if (nrows > 0) HIPCHK(hipMemsetAsync(row_pred, 0xff, sizeof(int32_t) * nrows, st));
        if (ncols > 0) HIPCHK(hipMemsetAsync(col_level, 0, sizeof(int32_t) * ncols, st));
        HIPCHK(hipStreamSynchronize(st));
        return 0;
    }
    int dev = 0;
    if (current_device(&dev) || dev < 0 || dev >= 64) return fail(MCM_EHIP, "no current HIP device");
    const Options o = opts();
    std::unique_lock<std::mutex> lk;
    Workspace &w = acquire_workspace(dev, stream, lk);
    if ((rc = ensure_base(w, dev))) return rc;
    CoopHold hold(stream, st);
    DevGraph g;
    if ((rc = one_bfs_phase(w, o, ncols, nrows, colptr, rowind, cmatch, rmatch, col_level, nullptr, false, st, &g)))
        return rc;
    HIPCHK(launch_export_pred(g, 1, row_pred, st));
    HIPCHK(hipStreamSynchronize(st));
    return (int64_t)*ctrl_line(w.h_ctrl, L_NENDS);
}

int64_t mcm_bfs_forest(int32_t ncols, int32_t nrows, const int32_t *colptr, const int32_t *rowind,
                       const int32_t *cmatch, const int32_t *rmatch, int32_t *col_level, int32_t *col_root,
                       int32_t *row_pred, int32_t *ends, void *stream)
{
    int64_t rc;
    if ((rc = check_graph_args(ncols, nrows, colptr, rowind))) return rc;
    if ((ncols > 0 && (!cmatch || !col_level || !col_root)) || (nrows > 0 && (!rmatch || !row_pred || !ends)))
        return fail(MCM_EINVAL, "NULL matching or output array");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if ((rc = check_null_rowind(ncols, nrows, colptr, rowind, st))) return rc;
    if (ncols == 0 || nrows == 0) {
        // no edges: every column is unmatched, its own root at level 0
        std::vector<int32_t> id((size_t)ncols);
        std::iota(id.begin(), id.end(), 0);
        if (nrows > 0) HIPCHK(hipMemsetAsync(row_pred, 0xff, sizeof(int32_t) * nrows, st));
        if (ncols > 0) {
            HIPCHK(hipMemsetAsync(col_level, 0, sizeof(int32_t) * ncols, st));
            HIPCHK(hipMemcpyAsync(col_root, id.data(), sizeof(int32_t) * ncols, hipMemcpyHostToDevice, st));
        }
        HIPCHK(hipStreamSynchronize(st));
        return 0;
    }
    int dev = 0;
    if (current_device(&dev) || dev < 0 || dev >= 64) return fail(MCM_EHIP, "no current HIP device");
    const Options o = opts();
    std::unique_lock<std::mutex> lk;
    Workspace &w = acquire_workspace(dev, stream, lk);
    if ((rc = ensure_base(w, dev))) return rc;
    CoopHold hold(stream, st);
    DevGraph g;
    if ((rc = one_bfs_phase(w, o, ncols, nrows, colptr, rowind, cmatch, rmatch, col_level, col_root, true, st, &g)))
        return rc;
    const uint32_t nends = *ctrl_line(w.h_ctrl, L_NENDS);
    HIPCHK(launch_export_pred(g, 1, row_pred, st));
    if (nends) HIPCHK(hipMemcpyAsync(ends, g.ends, sizeof(int32_t) * nends, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return (int64_t)nends;
}

int mcm_shutdown(void)
{
    std::vector<std::pair<void *, void (*)(void *)>> live;
    {
        std::lock_guard<std::mutex> lk(g_handles_mu);
        live.assign(g_handles.begin(), g_handles.end());
        g_handles.clear();
    }
    for (auto &h : live) h.second(h.first);
    int dev = 0;
    const bool have_dev = current_device(&dev) == 0;
    {
        std::lock_guard<std::mutex> g(g_ws_map_mu);
        for (auto &kv : g_ws_map) {
            std::lock_guard<std::mutex> lk(kv.second->mu);
            release_workspace(kv.second->w);
        }
        g_ws_map.clear();
    }
    if (have_dev) (void)hipSetDevice(dev);
    return MCM_OK;
}

}  // extern "C"
