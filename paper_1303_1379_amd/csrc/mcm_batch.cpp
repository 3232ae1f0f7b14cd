// Many independent graphs per launch: mcm_match_batched (one shot),
// batch plans (descriptors uploaded once, launch sequence captured in a
// hipGraph and replayed), the autotuner that picks the mapping (one column
// per lane or edges spread over a wavefront), the workgroup size and the
// wavefront batch size, and the device-side cheap initial matching.
#include "mcm_host.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <numeric>
#include <optional>
#include <sstream>
#include <string>
#include <vector>

using namespace mcm;
using namespace mcm::host;

namespace {

// ------------------------------------------------------------------ configuration of the batched kernel
struct BatchCfg {
    bool wave = true;
    int block = 1024;
    int batch_min = 8;
    double ms = -1.0;  // measured by the autotuner, -1 if not tuned
};

int log2_bucket(int64_t x)
{
    int b = 0;
    while (x > 1) { x >>= 1; ++b; }
    return b;
}

std::string tune_key(const std::string &arch, int64_t ngraphs, int64_t nverts)
{
    std::ostringstream k;
    k << arch << "|batch|g" << log2_bucket(ngraphs) << "|v" << log2_bucket(nverts);
    return k.str();
}

// Autotuner cache: in memory, mirrored to a JSON-lines file when the option
// "tuning" names one.  One line per key:
//   {"key": "...", "wave": 1, "block": 1024, "batch_min": 8, "ms": 4.81}
std::mutex g_tune_mu;
std::map<std::string, BatchCfg> g_tune;
std::string g_tune_loaded;

void tune_load(const std::string &path)
{
    if (path.empty() || path == g_tune_loaded) return;
    g_tune_loaded = path;
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        char key[512];
        int wave = 1, block = 1024, bmin = 8;
        double ms = -1;
        if (sscanf(line.c_str(), " {\"key\": \"%511[^\"]\", \"wave\": %d, \"block\": %d, \"batch_min\": %d, \"ms\": %lf",
                   key, &wave, &block, &bmin, &ms) == 5) {
            if (block < 64 || block > 1024 || block % 64 || bmin < 1 || bmin > 64) continue;
            BatchCfg c;
            c.wave = wave != 0;
            c.block = block;
            c.batch_min = bmin;
            c.ms = ms;
            g_tune[key] = c;
        }
    }
}

void tune_save(const std::string &path)
{
    if (path.empty()) return;
    std::ofstream out(path + ".tmp");
    for (const auto &kv : g_tune)
        out << "{\"key\": \"" << kv.first << "\", \"wave\": " << (kv.second.wave ? 1 : 0) << ", \"block\": "
            << kv.second.block << ", \"batch_min\": " << kv.second.batch_min << ", \"ms\": " << kv.second.ms << "}\n";
    out.close();
    std::rename((path + ".tmp").c_str(), path.c_str());
}

bool tune_lookup(const std::string &path, const std::string &key, BatchCfg *out)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load(path);
    auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    *out = it->second;
    return true;
}

void tune_store(const std::string &path, const std::string &key, const BatchCfg &c)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load(path);
    g_tune[key] = c;
    tune_save(path);
}

// ------------------------------------------------------------------ descriptors
struct Extents {
    int64_t col_ext = 0, row_ext = 0, verts = 0;
};

int64_t check_batch(int32_t ngraphs, const mcm_graph *graphs, const int32_t *colptr_all, const int32_t *rowind_all,
                    const int32_t *ic, const int32_t *ir, int32_t *oc, int32_t *orr, Extents *ex)
{
    if (ngraphs < 0) return fail(MCM_EINVAL, "ngraphs < 0");
    if (ngraphs > 0 && !graphs) return fail(MCM_EINVAL, "graphs is NULL");
    if ((ic == nullptr) != (ir == nullptr)) return fail(MCM_EINVAL, "init arrays must both be NULL or both be given");
    for (int32_t i = 0; i < ngraphs; ++i) {
        const mcm_graph &d = graphs[i];
        if (d.ncols < 0 || d.nrows < 0 || d.colptr_off < 0 || d.rowind_off < 0 || d.col_off < 0 || d.row_off < 0)
            return fail(MCM_EINVAL, "graph %d: negative size or offset", i);
        if (d.ncols > 0 && !colptr_all) return fail(MCM_EINVAL, "colptr_all is NULL");
        if (d.ncols > 0 && d.nrows > 0 && !rowind_all) return fail(MCM_EINVAL, "rowind_all is NULL");
        if ((d.ncols > 0 && !oc) || (d.nrows > 0 && !orr)) return fail(MCM_EINVAL, "NULL packed output array");
        ex->col_ext = std::max(ex->col_ext, d.col_off + d.ncols);
        ex->row_ext = std::max(ex->row_ext, d.row_off + d.nrows);
        ex->verts += (int64_t)d.ncols + d.nrows;
    }
    return 0;
}

// Pointer descriptors for the packed layout; workspace slices use the
// caller's column/row offsets (queues: 2 entries per column).
void build_descs(int32_t ngraphs, const mcm_graph *graphs, const int32_t *cp, const int32_t *ri, const int32_t *ic,
                 const int32_t *ir, int32_t *oc, int32_t *orr, uint64_t *rw, int32_t *pred, uint32_t *cdone, int4 *fq,
                 int32_t *ends, BatchDesc *out, int32_t *order)
{
    for (int32_t i = 0; i < ngraphs; ++i) {
        const mcm_graph &g = graphs[i];
        BatchDesc d{};
        d.nc = g.ncols;
        d.nr = g.nrows;
        d.colptr = cp ? cp + g.colptr_off : nullptr;
        d.rowind = ri ? ri + g.rowind_off : nullptr;
        d.init_c = ic ? ic + g.col_off : nullptr;
        d.init_r = ir ? ir + g.row_off : nullptr;
        d.out_c = oc + g.col_off;
        d.out_r = orr + g.row_off;
        d.rw = rw + g.row_off;
        d.pred = pred + g.row_off;
        d.cdone = cdone + g.col_off;
        d.fq = fq + 2 * g.col_off;
        d.ends = ends + g.row_off;
        out[i] = d;
    }
    // largest first: the work queue hands the long-running graphs out early
    std::vector<int32_t> ord(ngraphs);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
        return (int64_t)graphs[a].ncols + graphs[a].nrows > (int64_t)graphs[b].ncols + graphs[b].nrows;
    });
    std::copy(ord.begin(), ord.end(), order);
}

int batch_blocks(const DevInfo &info, bool wave, int block, int32_t ngraphs)
{
    int per_cu = 1;
    if (match_wg_occupancy(wave, block, &per_cu) != hipSuccess || per_cu < 1) per_cu = 1;
    return (int)std::max<int64_t>(1, std::min<int64_t>(ngraphs, (int64_t)info.ncu * per_cu));
}

BatchCfg default_cfg(const Options &o)
{
    BatchCfg c;
    c.wave = o.mapping != 0;
    c.block = o.wg_block;
    c.batch_min = o.batch_min;
    return c;
}

}  // namespace

// =================================================================== C ABI
extern "C" {

int64_t mcm_match_batched(int32_t ngraphs, const mcm_graph *graphs, const int32_t *colptr_all,
                          const int32_t *rowind_all, const int32_t *init_cmatch_all, const int32_t *init_rmatch_all,
                          int32_t *out_cmatch_all, int32_t *out_rmatch_all, int64_t *out_card, void *stream)
{
    Extents ex;
    int64_t rc;
    if ((rc = check_batch(ngraphs, graphs, colptr_all, rowind_all, init_cmatch_all, init_rmatch_all, out_cmatch_all,
                          out_rmatch_all, &ex)))
        return rc;
    if (ngraphs == 0) return 0;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    int dev = 0;
    if (current_device(&dev) || dev < 0 || dev >= 64) return fail(MCM_EHIP, "no current HIP device");
    const Options o = opts();
    std::unique_lock<std::mutex> lk;
    Workspace &w = acquire_workspace(dev, stream, lk);
    if ((rc = ensure_base(w, dev))) return rc;
    const size_t ce = (size_t)std::max<int64_t>(ex.col_ext, 1), re = (size_t)std::max<int64_t>(ex.row_ext, 1);
    if ((rc = ensure_graph(w, ce, re, ce))) return rc;  // queues: 2 * col_ext entries in all
    if ((rc = ensure_desc(w, 2 * (size_t)ngraphs))) return rc;  // second half: large members, packed
    build_descs(ngraphs, graphs, colptr_all, rowind_all, init_cmatch_all, init_rmatch_all, out_cmatch_all,
                out_rmatch_all, w.rw, w.pred, w.cdone, w.fq, w.ends, w.h_desc, w.h_order);
    // Members above multi_threshold vertices are matched by groups of blocks,
    // several graphs per cooperative launch; the order is largest first, so
    // they are its prefix.
    // A member also has to exceed twice the average load of a resident
    // workgroup: with many graphs the workgroup kernel spreads even the
    // larger ones over all CUs, and the multi-graph launch, which runs
    // after it, would only add its own length.
    int32_t nlarge = 0;
    int64_t large_min = o.multi_threshold;
    if (o.multi_threshold > 0) {
        int per_cu = 1;
        if (match_wg_occupancy(o.mapping != 0, o.wg_block, &per_cu) != hipSuccess || per_cu < 1) per_cu = 1;
        large_min = std::max<int64_t>(large_min, 2 * ex.verts / std::max(1, w.info.ncu * per_cu));
    }
    if (o.multi_threshold > 0)
        while (nlarge < ngraphs) {
            const mcm_graph &g = graphs[w.h_order[nlarge]];
            if ((int64_t)g.ncols + g.nrows <= large_min) break;
            w.h_desc[ngraphs + nlarge] = w.h_desc[w.h_order[nlarge]];
            ++nlarge;
        }
    const int32_t nsmall = ngraphs - nlarge;
    BatchCfg cfg = default_cfg(o);
    if (o.mapping == 2) tune_lookup(o.tuning, tune_key(w.info.arch, ngraphs, ex.verts), &cfg);
    uint32_t flags = base_flags(o, 0, 0);
    if (cfg.wave) flags |= F_WAVE;
    else flags &= ~(uint32_t)F_WAVE;
    RunOpt ro = run_opt(o, flags, std::max<int64_t>(ex.col_ext, 1), w.info);
    ro.split = 0;  // per-graph queue slices hold exactly nc entries
    ro.batch_min = (uint32_t)cfg.batch_min;
    HIPCHK(prepare_match_wg(cfg.block));
    const int blocks = batch_blocks(w.info, cfg.wave, cfg.block, std::max(nsmall, 1));
    // multi-graph launch shape: `ngroups` groups of `group` blocks, all
    // co-resident (a cooperative launch must fit the device at once), take
    // the large members from a queue
    const bool mwave = (flags & F_WAVE) != 0;
    int group = 1, ngroups = 1;
    if (nlarge) {
        int occ = 0;
        HIPCHK(multi_occupancy(mwave, o.block, &occ));
        const int resident = w.info.ncu * std::max(occ, 0);
        if (resident < 1) return fail(MCM_EHIP, "multi-graph kernel does not fit a CU with block %d", o.block);
        group = o.multi_group > 0 ? o.multi_group : std::max(1, w.info.ncu / 8);
        group = std::min(group, std::min(resident, kMaxGridBlocks));
        ngroups = std::max(1, std::min(std::min(kMultiMax, resident / group), (int)nlarge));
    }
    RunOpt mro = run_opt(o, flags, std::max<int64_t>(ex.col_ext, 1), w.info);
    mro.split = 0;  // same queue slices as above
    // the multi-graph launch is cooperative: at most one such launch in flight in the process
    std::optional<CoopHold> hold;
    if (nlarge) hold.emplace(stream, st);
    HIPCHK(hipMemcpyAsync(w.desc, w.h_desc, sizeof(BatchDesc) * (ngraphs + nlarge), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(w.order, w.h_order, sizeof(int32_t) * ngraphs, hipMemcpyHostToDevice, st));
    HIPCHK(launch_zero_ctrl(w.ctrl, st));
    HIPCHK(hipEventRecord(w.ev0, st));
    if (nsmall)
        HIPCHK(launch_match_wg(w.desc, w.order + nlarge, nsmall, w.card, w.ctrl, ro, cfg.wave, blocks, cfg.block, st));
    if (nlarge)
        HIPCHK(launch_multi(w.desc + ngraphs, nlarge, group, ngroups, w.mctrl, w.mbar, w.card + ngraphs, mro, mwave,
                            o.block, st));
    HIPCHK(hipEventRecord(w.ev1, st));
    HIPCHK(hipMemcpyAsync(w.h_card, w.card, sizeof(int64_t) * (ngraphs + nlarge), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(w.h_ctrl, w.ctrl, (size_t)L_NLINES * 128, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, w.ev0, w.ev1));
    for (int32_t j = 0; j < nlarge; ++j) w.h_card[w.h_order[j]] = w.h_card[ngraphs + j];
    int64_t total = 0;
    bool bad = false;
    for (int32_t i = 0; i < ngraphs; ++i) {
        if (w.h_card[i] < 0) bad = true;
        else total += w.h_card[i];
        if (out_card) out_card[i] = w.h_card[i];
    }
    record_stats(w.h_ctrl, -1, total, ms, 2, flags, w.info.clock_khz);
    const int32_t s = (int32_t)*ctrl_line(w.h_ctrl, L_STATUS);
    if (bad || s != 0) return fail(MCM_EINTERNAL, "device watchdog fired in a batched graph (status %d)", s);
    return total;
}

}  // extern "C"

// ------------------------------------------------------------------ batch plans
struct mcm_batch_plan {
    int dev = -1;
    int32_t ngraphs = 0;
    BatchDesc *d_desc = nullptr;
    int32_t *d_order = nullptr;
    int64_t *d_card = nullptr;
    uint32_t *d_ctrl = nullptr;
    uint64_t *rw = nullptr;
    int32_t *pred = nullptr;
    uint32_t *cdone = nullptr;
    int4 *fq = nullptr;
    int32_t *ends = nullptr;
    int64_t *h_card = nullptr;    // pinned
    uint32_t *h_ctrl = nullptr;   // pinned
    BatchCfg cfg;
    uint32_t flags = 0;
    RunOpt ro{};
    int blocks = 1;
    bool tuned = false;
    std::string key;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double clock_khz = 100000.0;
};

namespace {

void plan_free(mcm_batch_plan *p)
{
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    if (p->ev0) (void)hipEventDestroy(p->ev0);
    if (p->ev1) (void)hipEventDestroy(p->ev1);
    for (void *q : {(void *)p->d_desc, (void *)p->d_order, (void *)p->d_card, (void *)p->d_ctrl, (void *)p->rw,
                    (void *)p->pred, (void *)p->cdone, (void *)p->fq, (void *)p->ends})
        if (q) (void)hipFree(q);
    if (p->h_card) (void)hipHostFree(p->h_card);
    if (p->h_ctrl) (void)hipHostFree(p->h_ctrl);
    delete p;
}

// One eager run of the plan's kernel with configuration c; returns ms.
int64_t plan_time(mcm_batch_plan *p, const BatchCfg &c, float *ms)
{
    RunOpt ro = p->ro;
    ro.batch_min = (uint32_t)c.batch_min;
    ro.flags = c.wave ? (ro.flags | F_WAVE) : (ro.flags & ~(uint32_t)F_WAVE);
    HIPCHK(prepare_match_wg(c.block));
    int blocks = 1;
    {
        int per_cu = 1;
        if (match_wg_occupancy(c.wave, c.block, &per_cu) != hipSuccess || per_cu < 1) per_cu = 1;
        int dev = 0;
        (void)hipGetDevice(&dev);
        hipDeviceProp_t prop;
        HIPCHK(hipGetDeviceProperties(&prop, dev));
        blocks = (int)std::max<int64_t>(1, std::min<int64_t>(p->ngraphs, (int64_t)prop.multiProcessorCount * per_cu));
    }
    HIPCHK(launch_zero_ctrl(p->d_ctrl, p->cap));
    HIPCHK(hipEventRecord(p->ev0, p->cap));
    HIPCHK(launch_match_wg(p->d_desc, p->d_order, p->ngraphs, p->d_card, p->d_ctrl, ro, c.wave, blocks, c.block,
                           p->cap));
    HIPCHK(hipEventRecord(p->ev1, p->cap));
    HIPCHK(hipStreamSynchronize(p->cap));
    HIPCHK(hipEventElapsedTime(ms, p->ev0, p->ev1));
    HIPCHK(hipMemcpy(p->h_ctrl, p->d_ctrl, (size_t)L_NLINES * 128, hipMemcpyDeviceToHost));
    if (*ctrl_line(p->h_ctrl, L_STATUS) != 0) return fail(MCM_EINTERNAL, "device watchdog fired while tuning");
    return 0;
}

// Times every candidate (mapping x workgroup size x wavefront batch) on the
// plan's own graphs and keeps the fastest.
int64_t plan_autotune(mcm_batch_plan *p, BatchCfg *best)
{
    int64_t rc;
    double best_ms = 1e30;
    for (int wave = 0; wave < 2; ++wave)
        for (int block : {256, 512, 1024})
            for (int bmin : {1, 8, 32}) {
                BatchCfg c;
                c.wave = wave != 0;
                c.block = block;
                c.batch_min = bmin;
                float ms = 0.f, m2 = 0.f;
                if ((rc = plan_time(p, c, &ms))) return rc;    // first run warms caches
                if ((rc = plan_time(p, c, &m2))) return rc;
                ms = std::min(ms, m2);
                if (ms < best_ms) {
                    best_ms = ms;
                    *best = c;
                    best->ms = ms;
                }
            }
    return 0;
}

int64_t plan_capture(mcm_batch_plan *p)
{
    HIPCHK(prepare_match_wg(p->cfg.block));
    HIPCHK(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
    // zeroing by a kernel: memset nodes are kept out of the graph
    hipError_t e = launch_zero_ctrl(p->d_ctrl, p->cap);
    if (e == hipSuccess)
        e = launch_match_wg(p->d_desc, p->d_order, p->ngraphs, p->d_card, p->d_ctrl, p->ro, p->cfg.wave, p->blocks,
                            p->cfg.block, p->cap);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->h_card, p->d_card, sizeof(int64_t) * p->ngraphs, hipMemcpyDeviceToHost, p->cap);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->h_ctrl, p->d_ctrl, (size_t)L_NLINES * 128, hipMemcpyDeviceToHost, p->cap);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(p->cap, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(MCM_EHIP, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    }
    p->graph = g;
    HIPCHK(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    return 0;
}

}  // namespace

extern "C" {

int64_t mcm_batch_plan_create(int32_t ngraphs, const mcm_graph *graphs, const int32_t *colptr_all,
                              const int32_t *rowind_all, const int32_t *init_cmatch_all,
                              const int32_t *init_rmatch_all, int32_t *out_cmatch_all, int32_t *out_rmatch_all,
                              mcm_batch_plan **plan)
{
    if (!plan) return fail(MCM_EINVAL, "plan is NULL");
    *plan = nullptr;
    Extents ex;
    int64_t rc;
    if ((rc = check_batch(ngraphs, graphs, colptr_all, rowind_all, init_cmatch_all, init_rmatch_all, out_cmatch_all,
                          out_rmatch_all, &ex)))
        return rc;
    if (ngraphs == 0) return fail(MCM_EINVAL, "a plan needs at least one graph");
    int dev = 0;
    if (current_device(&dev) || dev < 0 || dev >= 64) return fail(MCM_EHIP, "no current HIP device");
    const Options o = opts();
    mcm_batch_plan *p = new mcm_batch_plan();
    p->dev = dev;
    p->ngraphs = ngraphs;
    auto bail = [&](int64_t code) { plan_free(p); return code; };
    DevInfo info;
    {
        std::unique_lock<std::mutex> lk;
        Workspace &w = acquire_workspace(dev, nullptr, lk);
        if ((rc = ensure_base(w, dev))) return bail(rc);
        info = w.info;
    }
    p->clock_khz = info.clock_khz;
    const size_t ce = (size_t)std::max<int64_t>(ex.col_ext, 1), re = (size_t)std::max<int64_t>(ex.row_ext, 1);
    if (hipMalloc(&p->d_desc, sizeof(BatchDesc) * ngraphs) != hipSuccess ||
        hipMalloc(&p->d_order, sizeof(int32_t) * ngraphs) != hipSuccess ||
        hipMalloc(&p->d_card, sizeof(int64_t) * ngraphs) != hipSuccess ||
        hipMalloc(&p->d_ctrl, (size_t)L_NLINES * 128) != hipSuccess ||
        hipMalloc(&p->rw, sizeof(uint64_t) * re) != hipSuccess || hipMalloc(&p->pred, sizeof(int32_t) * re) != hipSuccess ||
        hipMalloc(&p->ends, sizeof(int32_t) * re) != hipSuccess ||
        hipMalloc(&p->cdone, sizeof(uint32_t) * ce) != hipSuccess || hipMalloc(&p->fq, sizeof(int4) * 2 * ce) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&p->h_card), sizeof(int64_t) * ngraphs, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&p->h_ctrl), (size_t)L_NLINES * 128, hipHostMallocDefault) != hipSuccess)
        return bail(fail(MCM_ENOMEM, "batch plan allocation failed"));
    if (hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&p->ev0) != hipSuccess ||
        hipEventCreate(&p->ev1) != hipSuccess)
        return bail(fail(MCM_EHIP, "batch plan stream/event creation failed"));
    std::vector<BatchDesc> hd(ngraphs);
    std::vector<int32_t> ho(ngraphs);
    build_descs(ngraphs, graphs, colptr_all, rowind_all, init_cmatch_all, init_rmatch_all, out_cmatch_all,
                out_rmatch_all, p->rw, p->pred, p->cdone, p->fq, p->ends, hd.data(), ho.data());
    if (hipMemcpy(p->d_desc, hd.data(), sizeof(BatchDesc) * ngraphs, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_order, ho.data(), sizeof(int32_t) * ngraphs, hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(MCM_EHIP, "descriptor upload failed"));

    p->flags = base_flags(o, 0, 0);
    p->ro = run_opt(o, p->flags, std::max<int64_t>(ex.col_ext, 1), info);
    p->ro.split = 0;
    p->key = tune_key(info.arch, ngraphs, ex.verts);
    p->cfg = default_cfg(o);
    BatchCfg cached;
    if (o.autotune) {
        BatchCfg best;
        if ((rc = plan_autotune(p, &best))) return bail(rc);
        p->cfg = best;
        p->tuned = true;
        tune_store(o.tuning, p->key, best);
    } else if (o.mapping == 2 && tune_lookup(o.tuning, p->key, &cached)) {
        p->cfg = cached;
        p->tuned = true;
    }
    if (p->cfg.wave) p->ro.flags |= F_WAVE;
    else p->ro.flags &= ~(uint32_t)F_WAVE;
    p->ro.batch_min = (uint32_t)p->cfg.batch_min;
    p->blocks = batch_blocks(info, p->cfg.wave, p->cfg.block, ngraphs);
    if ((rc = plan_capture(p))) return bail(rc);
    register_handle(p, [](void *h) { plan_free(static_cast<mcm_batch_plan *>(h)); });
    *plan = p;
    return 0;
}

int64_t mcm_batch_plan_run(mcm_batch_plan *p, int64_t *out_card, void *stream)
{
    if (!p) return fail(MCM_EINVAL, "plan is NULL");
    int dev = 0;
    if (current_device(&dev) || dev != p->dev) return fail(MCM_EINVAL, "plan belongs to device %d", p->dev);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    HIPCHK(hipEventRecord(p->ev0, st));
    HIPCHK(hipGraphLaunch(p->exec, st));
    HIPCHK(hipEventRecord(p->ev1, st));
    HIPCHK(hipStreamSynchronize(st));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, p->ev0, p->ev1));
    int64_t total = 0;
    bool bad = false;
    for (int32_t i = 0; i < p->ngraphs; ++i) {
        if (p->h_card[i] < 0) bad = true;
        else total += p->h_card[i];
        if (out_card) out_card[i] = p->h_card[i];
    }
    record_stats(p->h_ctrl, -1, total, ms, 2, p->ro.flags, p->clock_khz);
    if (bad || *ctrl_line(p->h_ctrl, L_STATUS) != 0)
        return fail(MCM_EINTERNAL, "device watchdog fired in a batched graph");
    return total;
}

int mcm_batch_plan_info(const mcm_batch_plan *p, char *buf, int32_t len)
{
    if (!p || !buf || len <= 0) return (int)fail(MCM_EINVAL, "bad arguments");
    snprintf(buf, (size_t)len,
             "{\"ngraphs\": %d, \"mapping\": \"%s\", \"block\": %d, \"batch_min\": %d, \"blocks\": %d, "
             "\"tuned\": %s, \"tuned_ms\": %.4f, \"key\": \"%s\"}",
             p->ngraphs, p->cfg.wave ? "wave" : "thread", p->cfg.block, p->cfg.batch_min, p->blocks,
             p->tuned ? "true" : "false", p->cfg.ms, p->key.c_str());
    return MCM_OK;
}

int mcm_batch_plan_destroy(mcm_batch_plan *p)
{
    // a plan that mcm_shutdown already released is not freed twice
    if (p && unregister_handle(p)) plan_free(p);
    return MCM_OK;
}

int64_t mcm_cheap_init(int32_t ncols, int32_t nrows, const int32_t *colptr, const int32_t *rowind, int32_t *cmatch,
                       int32_t *rmatch, void *stream)
{
    if (ncols < 0 || nrows < 0 || (ncols > 0 && (!colptr || !cmatch)) || (nrows > 0 && !rmatch))
        return fail(MCM_EINVAL, "bad arguments to mcm_cheap_init");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (ncols == 0 || nrows == 0) {
        if (ncols > 0) HIPCHK(hipMemsetAsync(cmatch, 0xff, sizeof(int32_t) * ncols, st));
        if (nrows > 0) HIPCHK(hipMemsetAsync(rmatch, 0xff, sizeof(int32_t) * nrows, st));
        HIPCHK(hipStreamSynchronize(st));
        return 0;
    }
    if (!rowind) {
        int32_t nnz = -1;
        HIPCHK(hipMemcpyAsync(&nnz, colptr + ncols, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (nnz != 0) return fail(MCM_EINVAL, "rowind is NULL but colptr[ncols] = %d", nnz);
    }
    int dev = 0;
    if (current_device(&dev) || dev < 0 || dev >= 64) return fail(MCM_EHIP, "no current HIP device");
    std::unique_lock<std::mutex> lk;
    Workspace &w = acquire_workspace(dev, stream, lk);
    int64_t rc;
    if ((rc = ensure_base(w, dev))) return rc;
    if ((rc = ensure_desc(w, 1))) return rc;
    BatchDesc d{};
    d.nc = ncols;
    d.nr = nrows;
    d.colptr = colptr;
    d.rowind = rowind;
    d.out_c = cmatch;
    d.out_r = rmatch;
    w.h_desc[0] = d;
    HIPCHK(hipMemcpyAsync(w.desc, w.h_desc, sizeof(BatchDesc), hipMemcpyHostToDevice, st));
    HIPCHK(launch_cheap_init(w.desc, 1, st));
    HIPCHK(launch_zero_ctrl(w.ctrl, st));
    // count |M0| with the finish kernel's column count
    DevGraph g{};
    g.nc = ncols;
    g.nr = 0;
    g.cmatch = cmatch;
    HIPCHK(launch_finish(g, nullptr, w.ctrl, st));
    HIPCHK(hipMemcpyAsync(w.h_ctrl, w.ctrl, (size_t)L_NLINES * 128, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return (int64_t)*reinterpret_cast<uint64_t *>(ctrl_line(w.h_ctrl, L_CARD));
}

}  // extern "C"
