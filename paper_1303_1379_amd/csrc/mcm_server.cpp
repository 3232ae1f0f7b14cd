// Continuous-batching matching server.
//
// Requests (one graph each, host CSC arrays) are admitted in arrival order
// while their device footprint fits an HBM budget; their inputs are copied
// on a copy stream into a device arena, and a worker thread keeps the
// compute stream busy: every launch takes all admitted requests whose
// inputs have arrived (one workgroup per graph, the batched kernel), while
// newly arriving requests are admitted, copied and queued for the next
// launch.  Requests larger than a threshold are matched several at a time
// by one cooperative launch of the persistent kernel in which each request
// has its own group of blocks (k_persistent_multi); launches of both kinds
// follow each other on one compute stream, so at most one cooperative
// launch is ever in flight.  Results are
// copied back on the copy stream; a request's memory returns to the budget
// when its results are on the host.  Every request starts from the device
// cheap matching (mcm_cheap_init) and is matched to maximum exactly as
// mcm_match would.
#include "mcm_host.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>
#include <vector>

using namespace mcm;
using namespace mcm::host;

namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator over one device allocation of `budget` bytes.
class Arena {
  public:
    int64_t init(size_t bytes)
    {
        cap_ = bytes;
        HIPCHK(hipMalloc(&base_, bytes));
        free_[0] = bytes;
        return 0;
    }
    void release()
    {
        if (base_) (void)hipFree(base_);
        base_ = nullptr;
    }
    // Returns offset or SIZE_MAX if no hole is large enough.
    size_t alloc(size_t bytes)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return off;
        }
        return SIZE_MAX;
    }
    void free(size_t off, size_t bytes)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    char *base() const { return base_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t cap() const { return cap_; }

  private:
    char *base_ = nullptr;
    size_t cap_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

enum ReqState { Q_PENDING, Q_COPYING, Q_READY, Q_RUNNING, Q_DONE };

constexpr int kMultiGraphs = 64;  // large requests per multi-graph launch, at most

struct Request {
    int64_t ticket = 0;
    int32_t nc = 0, nr = 0;
    int64_t nnz = 0;
    const int32_t *h_colptr = nullptr, *h_rowind = nullptr;
    int32_t *h_cmatch = nullptr, *h_rmatch = nullptr;
    ReqState state = Q_PENDING;
    size_t off = 0, bytes = 0;
    // device views inside the arena
    int32_t *colptr = nullptr, *rowind = nullptr, *cmatch = nullptr, *rmatch = nullptr;
    uint64_t *rw = nullptr;
    int32_t *pred = nullptr, *ends = nullptr;
    uint32_t *cdone = nullptr;
    int4 *fq = nullptr;
    size_t qcap = 0;
    bool big = false;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    bool card_known = false;
    mcm_request_info info{};
};

struct Slot {  // one in-flight launch: batched (one workgroup per graph) or multi-graph persistent
    BatchDesc *d_desc = nullptr, *h_desc = nullptr;
    int64_t *d_card = nullptr, *h_card = nullptr;
    uint32_t *d_ctrl = nullptr, *h_ctrl = nullptr;   // kMultiMax control blocks
    uint32_t *d_bar = nullptr;                        // arrival lines of the multi-graph launch
    hipEvent_t done = nullptr;
    bool busy = false;
    int ngroups = 0;                                  // > 0: a multi-graph launch
    std::vector<Request *> reqs;
};

}  // namespace

struct mcm_server {
    int dev = 0;
    DevInfo info;
    Options opt;
    int32_t max_batch = 1024;
    int64_t big_threshold = 1 << 15;  // nc + nr above which a request joins a multi-graph launch
    int group = 64;                   // blocks per large request in a multi-graph launch
    int multi_max = 4;                // large requests per multi-graph launch (kMultiGraphs)
    int ngroups = 1;                  // block groups of a multi-graph launch (they take requests from a queue)
    std::deque<Request *> big_ready;  // large requests waiting for a launch
    Arena arena;
    hipStream_t compute = nullptr, copy = nullptr;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request *> pending;            // waiting for memory, in arrival order
    std::vector<Request *> copying, running;  // inputs on their way; launched
    std::unordered_map<int64_t, Request *> live;  // every request not yet polled as done
    int64_t next_ticket = 1;
    std::atomic<bool> stop{false};
    std::thread worker;
    Clock::time_point t0;
    int64_t status = 0;                       // first fatal device error
    mcm_server_stats st{};

    double now_ms() const { return std::chrono::duration<double, std::milli>(Clock::now() - t0).count(); }
};

namespace {

size_t req_bytes(const mcm_server *s, int32_t nc, int32_t nr, int64_t nnz, bool big, size_t *qcap)
{
    // inputs, outputs, workspace (row word, predecessor, ends per row; root
    // stamp per column; two frontier queues)
    *qcap = (size_t)nc + 1;
    if (big && s->opt.split) *qcap += (size_t)nnz / s->opt.split + 1;
    const size_t q = big ? *qcap : (size_t)nc;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    return al(4 * ((size_t)nc + 1)) + al(4 * (size_t)nnz) + al(4 * (size_t)nc) + al(4 * (size_t)nr) +
           al(8 * (size_t)nr) + al(4 * (size_t)nr) + al(4 * (size_t)nr) + al(4 * (size_t)nc) + al(32 * q);
}

void carve(mcm_server *s, Request *r)
{
    char *p = s->arena.base() + r->off;
    auto take = [&](size_t b) { char *q = p; p += (b + 255) & ~(size_t)255; return q; };
    r->colptr = reinterpret_cast<int32_t *>(take(4 * ((size_t)r->nc + 1)));
    r->rowind = reinterpret_cast<int32_t *>(take(4 * (size_t)r->nnz));
    r->cmatch = reinterpret_cast<int32_t *>(take(4 * (size_t)r->nc));
    r->rmatch = reinterpret_cast<int32_t *>(take(4 * (size_t)r->nr));
    r->rw = reinterpret_cast<uint64_t *>(take(8 * (size_t)r->nr));
    r->pred = reinterpret_cast<int32_t *>(take(4 * (size_t)r->nr));
    r->ends = reinterpret_cast<int32_t *>(take(4 * (size_t)r->nr));
    r->cdone = reinterpret_cast<uint32_t *>(take(4 * (size_t)r->nc));
    r->fq = reinterpret_cast<int4 *>(take(32 * (r->big ? r->qcap : (size_t)r->nc)));
}

BatchDesc desc_of(const Request *r)
{
    BatchDesc d{};
    d.nc = r->nc;
    d.nr = r->nr;
    d.colptr = r->colptr;
    d.rowind = r->nnz ? r->rowind : nullptr;
    d.init_c = r->cmatch;  // the device cheap matching, computed in place
    d.init_r = r->rmatch;
    d.out_c = r->cmatch;
    d.out_r = r->rmatch;
    d.rw = r->rw;
    d.pred = r->pred;
    d.cdone = r->cdone;
    d.fq = r->fq;
    d.ends = r->ends;
    d.qcap = r->big ? (int64_t)r->qcap : 0;
    return d;
}

// Admission (caller holds mu): move requests from the head of `pending`
// into device memory while they fit; start their input copies.
void admit(mcm_server *s)
{
    while (!s->pending.empty()) {
        Request *r = s->pending.front();
        const size_t off = s->arena.alloc(r->bytes);
        if (off == SIZE_MAX) break;  // in order: wait for memory to come back
        s->pending.pop_front();
        r->off = off;
        carve(s, r);
        r->info.admit_ms = s->now_ms();
        if (hipMemcpyAsync(r->colptr, r->h_colptr, 4 * ((size_t)r->nc + 1), hipMemcpyHostToDevice, s->copy) != hipSuccess ||
            (r->nnz && hipMemcpyAsync(r->rowind, r->h_rowind, 4 * (size_t)r->nnz, hipMemcpyHostToDevice, s->copy) != hipSuccess) ||
            hipEventRecord(r->ev_in, s->copy) != hipSuccess) {
            s->status = MCM_EHIP;
            return;
        }
        r->state = Q_COPYING;
        s->copying.push_back(r);
        s->st.bytes_in_use = (int64_t)s->arena.used();
        s->st.peak_bytes = (int64_t)s->arena.peak();
    }
}

// Results of a finished launch: copy outputs back, then (in complete())
// release memory.  Caller holds mu.
int64_t start_copy_back(mcm_server *s, Request *r, hipEvent_t after)
{
    HIPCHK(hipStreamWaitEvent(s->copy, after, 0));
    if (r->nc) HIPCHK(hipMemcpyAsync(r->h_cmatch, r->cmatch, 4 * (size_t)r->nc, hipMemcpyDeviceToHost, s->copy));
    if (r->nr) HIPCHK(hipMemcpyAsync(r->h_rmatch, r->rmatch, 4 * (size_t)r->nr, hipMemcpyDeviceToHost, s->copy));
    HIPCHK(hipEventRecord(r->ev_out, s->copy));
    return 0;
}

int64_t launch_batch(mcm_server *s, Slot &slot, std::vector<Request *> &reqs)
{
    const int32_t n = (int32_t)reqs.size();
    for (int32_t i = 0; i < n; ++i) slot.h_desc[i] = desc_of(reqs[i]);
    HIPCHK(hipMemcpyAsync(slot.d_desc, slot.h_desc, sizeof(BatchDesc) * n, hipMemcpyHostToDevice, s->compute));
    HIPCHK(launch_cheap_init(slot.d_desc, n, s->compute));
    HIPCHK(launch_zero_ctrl(slot.d_ctrl, s->compute));
    uint32_t flags = base_flags(s->opt, 0, 0) & ~(uint32_t)F_STATS;
    RunOpt ro = run_opt(s->opt, flags, 1 << 30, s->info);
    ro.split = 0;
    int per_cu = 1;
    if (match_wg_occupancy((flags & F_WAVE) != 0, s->opt.wg_block, &per_cu) != hipSuccess || per_cu < 1) per_cu = 1;
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(n, (int64_t)s->info.ncu * per_cu));
    HIPCHK(launch_match_wg(slot.d_desc, nullptr, n, slot.d_card, slot.d_ctrl, ro, (flags & F_WAVE) != 0, blocks,
                           s->opt.wg_block, s->compute));
    HIPCHK(hipMemcpyAsync(slot.h_card, slot.d_card, sizeof(int64_t) * n, hipMemcpyDeviceToHost, s->compute));
    HIPCHK(hipMemcpyAsync(slot.h_ctrl, slot.d_ctrl, (size_t)L_NLINES * 128, hipMemcpyDeviceToHost, s->compute));
    HIPCHK(hipEventRecord(slot.done, s->compute));
    const double t = s->now_ms();
    for (int32_t i = 0; i < n; ++i) {
        Request *r = reqs[i];
        r->state = Q_RUNNING;
        r->info.start_ms = t;
        r->info.path = 0;
        r->info.batch_size = n;
        r->card_known = false;
        s->running.push_back(r);
        int64_t rc;
        if ((rc = start_copy_back(s, r, slot.done))) return rc;
    }
    slot.busy = true;
    slot.ngroups = 0;
    slot.reqs = reqs;
    s->st.launches_batched += 1;
    s->st.max_batch_seen = std::max<int64_t>(s->st.max_batch_seen, n);
    return 0;
}

// Up to multi_max large requests in one cooperative launch: ngroups groups
// of `group` blocks take them from a queue.
int64_t launch_multi_reqs(mcm_server *s, Slot &slot, std::vector<Request *> &reqs)
{
    const int32_t n = (int32_t)reqs.size();
    for (int32_t i = 0; i < n; ++i) slot.h_desc[i] = desc_of(reqs[i]);
    HIPCHK(hipMemcpyAsync(slot.d_desc, slot.h_desc, sizeof(BatchDesc) * n, hipMemcpyHostToDevice, s->compute));
    HIPCHK(launch_cheap_init(slot.d_desc, n, s->compute));
    const uint32_t flags = base_flags(s->opt, 0, 0) & ~(uint32_t)F_STATS;
    const RunOpt ro = run_opt(s->opt, flags, 1 << 30, s->info);
    const int ngroups = std::min(n, s->ngroups);
    HIPCHK(launch_multi(slot.d_desc, n, s->group, ngroups, slot.d_ctrl, slot.d_bar, slot.d_card, ro,
                        (flags & F_WAVE) != 0, s->opt.block, s->compute));
    HIPCHK(hipMemcpyAsync(slot.h_card, slot.d_card, sizeof(int64_t) * n, hipMemcpyDeviceToHost, s->compute));
    HIPCHK(hipMemcpyAsync(slot.h_ctrl, slot.d_ctrl, (size_t)ngroups * L_NLINES * 128, hipMemcpyDeviceToHost,
                          s->compute));
    HIPCHK(hipEventRecord(slot.done, s->compute));
    const double t = s->now_ms();
    for (int32_t i = 0; i < n; ++i) {
        Request *r = reqs[i];
        r->state = Q_RUNNING;
        r->info.start_ms = t;
        r->info.path = 1;
        r->info.batch_size = n;
        r->card_known = false;
        s->running.push_back(r);
        int64_t rc;
        if ((rc = start_copy_back(s, r, slot.done))) return rc;
    }
    slot.busy = true;
    slot.ngroups = ngroups;
    slot.reqs = reqs;
    s->st.launches_grid += 1;
    return 0;
}

void complete(mcm_server *s, Request *r)
{
    r->info.done_ms = s->now_ms();
    r->state = Q_DONE;
    s->arena.free(r->off, r->bytes);
    s->st.bytes_in_use = (int64_t)s->arena.used();
    s->st.completed += 1;
    s->st.in_flight -= 1;
}

void worker_loop(mcm_server *s)
{
    (void)hipSetDevice(s->dev);
    std::unique_lock<std::mutex> lk(s->mu);
    while (!s->stop.load()) {
        bool progressed = false;
        if (!s->status) admit(s);
        // requests whose inputs have arrived
        std::vector<Request *> small, big;
        for (size_t i = 0; i < s->copying.size();) {
            Request *r = s->copying[i];
            if (hipEventQuery(r->ev_in) == hipSuccess) {
                r->state = Q_READY;
                (r->big ? big : small).push_back(r);
                s->copying[i] = s->copying.back();
                s->copying.pop_back();
            } else {
                ++i;
            }
        }
        std::sort(small.begin(), small.end(), [](Request *a, Request *b) {
            return (int64_t)a->nc + a->nr > (int64_t)b->nc + b->nr;  // largest first
        });
        // one batched launch per free slot (two launches in flight at most);
        // ready requests that find no free slot wait for the next round
        while (!small.empty() && !s->status) {
            Slot *free_slot = nullptr;
            for (auto &sl : s->slots)
                if (!sl.busy) { free_slot = &sl; break; }
            if (!free_slot) break;
            const size_t k = std::min(small.size(), (size_t)s->max_batch);
            std::vector<Request *> take(small.begin(), small.begin() + k);
            small.erase(small.begin(), small.begin() + k);
            if (launch_batch(s, *free_slot, take)) s->status = MCM_EHIP;
            progressed = true;
        }
        for (Request *r : small) s->copying.push_back(r);  // retried next round (event already complete)
        // large requests: up to multi_max per cooperative launch, one launch per free slot
        for (Request *r : big) s->big_ready.push_back(r);
        while (!s->big_ready.empty() && !s->status) {
            Slot *free_slot = nullptr;
            for (auto &sl : s->slots)
                if (!sl.busy) { free_slot = &sl; break; }
            if (!free_slot) break;
            // the multi-graph launch is cooperative: it waits (the requests
            // stay ready) while another owner's cooperative launch is in
            // flight; the gate is left when this launch's slot completes
            if (!coop_gate().try_enter(s->compute)) break;
            std::vector<Request *> take;
            while (!s->big_ready.empty() && (int)take.size() < s->multi_max) {
                take.push_back(s->big_ready.front());
                s->big_ready.pop_front();
            }
            if (launch_multi_reqs(s, *free_slot, take)) {
                s->status = MCM_EHIP;
                if (!free_slot->busy) {  // nothing in flight under the gate for this slot
                    (void)hipStreamSynchronize(s->compute);
                    coop_gate().leave(s->compute);
                }
            }
            progressed = true;
        }
        // finished batched launches: their cards become known
        for (auto &sl : s->slots) {
            if (sl.busy && hipEventQuery(sl.done) == hipSuccess) {
                if (sl.ngroups > 0) coop_gate().leave(s->compute);
                for (int k = 0; k < std::max(sl.ngroups, 1); ++k)
                    if (*ctrl_line(sl.h_ctrl + (size_t)k * L_NLINES * kLineWords, L_STATUS) != 0)
                        s->status = MCM_EINTERNAL;
                for (size_t i = 0; i < sl.reqs.size(); ++i) {
                    sl.reqs[i]->info.card = sl.h_card[i];
                    sl.reqs[i]->card_known = true;
                }
                sl.busy = false;
                sl.reqs.clear();
                progressed = true;
            }
        }
        // results on the host
        for (size_t i = 0; i < s->running.size();) {
            Request *r = s->running[i];
            if (r->card_known && hipEventQuery(r->ev_out) == hipSuccess) {
                complete(s, r);
                s->running[i] = s->running.back();
                s->running.pop_back();
                progressed = true;
            } else {
                ++i;
            }
        }
        if (progressed) s->cv.notify_all();
        else s->cv.wait_for(lk, std::chrono::microseconds(50));
    }
}

}  // namespace

// Stops the worker and releases everything the server holds.
static void server_free(mcm_server *s)
{
    s->stop.store(true);
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    (void)hipStreamSynchronize(s->compute);
    (void)hipStreamSynchronize(s->copy);
    // multi-graph launches still counted in the gate have completed now
    for (auto &sl : s->slots)
        if (sl.busy && sl.ngroups > 0) coop_gate().leave(s->compute);
    for (auto &kv : s->live) {
        Request *r = kv.second;
        if (r->ev_in) (void)hipEventDestroy(r->ev_in);
        if (r->ev_out) (void)hipEventDestroy(r->ev_out);
        delete r;
    }
    for (auto &sl : s->slots) {
        for (void *q : {(void *)sl.d_desc, (void *)sl.d_card, (void *)sl.d_ctrl, (void *)sl.d_bar}) if (q) (void)hipFree(q);
        for (void *q : {(void *)sl.h_desc, (void *)sl.h_card, (void *)sl.h_ctrl}) if (q) (void)hipHostFree(q);
        if (sl.done) (void)hipEventDestroy(sl.done);
    }
    if (s->compute) (void)hipStreamDestroy(s->compute);
    if (s->copy) (void)hipStreamDestroy(s->copy);
    s->arena.release();
    delete s;
}

extern "C" {

int64_t mcm_server_create(int64_t hbm_budget_bytes, int32_t max_batch, mcm_server **out)
{
    if (!out || hbm_budget_bytes <= 0 || max_batch < 1) return fail(MCM_EINVAL, "bad server arguments");
    *out = nullptr;
    mcm_server *s = new mcm_server();
    auto bail = [&](int64_t code) {
        s->arena.release();
        delete s;
        return code;
    };
    if (current_device(&s->dev) || s->dev < 0 || s->dev >= 64) return bail(fail(MCM_EHIP, "no current HIP device"));
    {
        std::unique_lock<std::mutex> lk;
        Workspace &w = acquire_workspace(s->dev, nullptr, lk);
        int64_t rc;
        if ((rc = ensure_base(w, s->dev))) return bail(rc);
        s->info = w.info;
    }
    s->opt = opts();
    s->max_batch = max_batch;
    s->big_threshold = std::max<int64_t>(s->opt.wg_threshold, 1 << 15);
    if (s->arena.init((size_t)hbm_budget_bytes)) return bail(MCM_ENOMEM);
    if (hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(MCM_EHIP, "stream creation failed"));
    // large requests: groups of `group` blocks (one persistent block per CU), as many groups as the
    // device holds at once, up to kMultiGraphs requests per launch taken from the launch's queue
    s->group = s->opt.multi_group > 0 ? s->opt.multi_group : std::max(1, s->info.ncu / 8);
    {
        int occ = 0;
        if (multi_occupancy((base_flags(s->opt, 0, 0) & F_WAVE) != 0, s->opt.block, &occ) != hipSuccess || occ < 1)
            return bail(fail(MCM_EHIP, "multi-graph kernel cannot be resident with block %d", s->opt.block));
        s->group = std::min(s->group, s->info.ncu * occ);
        s->ngroups = std::max(1, std::min(kMultiMax, s->info.ncu * occ / s->group));
    }
    const int ndesc = std::max(max_batch, kMultiGraphs);
    s->multi_max = kMultiGraphs;
    s->slots.resize(2);
    for (auto &sl : s->slots) {
        if (hipMalloc(&sl.d_desc, sizeof(BatchDesc) * ndesc) != hipSuccess ||
            hipMalloc(&sl.d_card, sizeof(int64_t) * ndesc) != hipSuccess ||
            hipMalloc(&sl.d_ctrl, (size_t)kMultiMax * L_NLINES * 128) != hipSuccess ||
            hipMalloc(&sl.d_bar, (size_t)kMultiMax * s->group * 128) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&sl.h_desc), sizeof(BatchDesc) * ndesc, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&sl.h_card), sizeof(int64_t) * ndesc, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&sl.h_ctrl), (size_t)kMultiMax * L_NLINES * 128, hipHostMallocDefault) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess)
            return bail(fail(MCM_ENOMEM, "server slot allocation failed"));
    }
    if (prepare_match_wg(s->opt.wg_block) != hipSuccess) return bail(fail(MCM_EHIP, "kernel attribute failed"));
    s->st.budget_bytes = hbm_budget_bytes;
    s->t0 = Clock::now();
    s->worker = std::thread(worker_loop, s);
    register_handle(s, [](void *h) { server_free(static_cast<mcm_server *>(h)); });
    *out = s;
    return MCM_OK;
}

int64_t mcm_server_submit(mcm_server *s, int32_t ncols, int32_t nrows, const int32_t *colptr, const int32_t *rowind,
                          int32_t *cmatch, int32_t *rmatch)
{
    if (!s) return fail(MCM_EINVAL, "server is NULL");
    if (ncols < 0 || nrows < 0 || (ncols > 0 && (!colptr || !cmatch)) || (nrows > 0 && !rmatch))
        return fail(MCM_EINVAL, "bad request arguments");
    const int64_t nnz = ncols > 0 ? colptr[ncols] : 0;
    if (nnz < 0 || (nnz > 0 && !rowind) || (ncols > 0 && colptr[0] != 0)) return fail(MCM_EINVAL, "malformed CSC");
    Request *r = new Request();
    r->nc = ncols;
    r->nr = nrows;
    r->nnz = nnz;
    r->h_colptr = colptr;
    r->h_rowind = rowind;
    r->h_cmatch = cmatch;
    r->h_rmatch = rmatch;
    r->big = (int64_t)ncols + nrows > s->big_threshold;
    r->bytes = req_bytes(s, ncols, nrows, nnz, r->big, &r->qcap);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->status) { delete r; return fail(s->status, "server stopped after a device error"); }
    if (r->bytes > s->arena.cap()) {
        delete r;
        s->st.rejected += 1;
        return fail(MCM_ENOMEM, "request needs %zu bytes, budget is %zu", r->bytes, s->arena.cap());
    }
    r->ticket = s->next_ticket++;
    r->info.submit_ms = s->now_ms();
    s->st.submitted += 1;
    if (ncols == 0 || nrows == 0) {  // nothing to match: answer at once
        if (ncols) std::fill(cmatch, cmatch + ncols, -1);
        if (nrows) std::fill(rmatch, rmatch + nrows, -1);
        r->info.card = 0;
        r->info.admit_ms = r->info.start_ms = r->info.done_ms = r->info.submit_ms;
        r->state = Q_DONE;
        r->bytes = 0;
        s->live[r->ticket] = r;
        s->st.completed += 1;
        return r->ticket;
    }
    if (hipEventCreateWithFlags(&r->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&r->ev_out, hipEventDisableTiming) != hipSuccess) {
        if (r->ev_in) (void)hipEventDestroy(r->ev_in);
        delete r;
        return fail(MCM_EHIP, "event creation failed");
    }
    s->live[r->ticket] = r;
    s->pending.push_back(r);
    s->st.in_flight += 1;
    s->cv.notify_all();
    return r->ticket;
}

int64_t mcm_server_poll(mcm_server *s, int64_t ticket, mcm_request_info *info, double wait_ms)
{
    if (!s) return fail(MCM_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->live.find(ticket);
    if (it == s->live.end()) return fail(MCM_EINVAL, "unknown ticket %lld", (long long)ticket);
    Request *r = it->second;
    if (r->state != Q_DONE && wait_ms > 0) {
        const auto until = Clock::now() + std::chrono::microseconds((int64_t)(wait_ms * 1000));
        s->cv.wait_until(lk, until, [&] { return r->state == Q_DONE || s->status != 0; });
    }
    if (s->status && r->state != Q_DONE) return fail(s->status, "server stopped after a device error");
    if (r->state != Q_DONE) return 0;
    if (info) *info = r->info;
    s->live.erase(it);
    if (r->ev_in) (void)hipEventDestroy(r->ev_in);
    if (r->ev_out) (void)hipEventDestroy(r->ev_out);
    const int64_t card = r->info.card;
    delete r;
    return card < 0 ? fail(card, "request failed on the device") : 1;
}

int mcm_server_stats_get(mcm_server *s, mcm_server_stats *out)
{
    if (!s || !out) return (int)fail(MCM_EINVAL, "bad arguments");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    out->queued = (int64_t)s->pending.size();
    return MCM_OK;
}

int mcm_server_destroy(mcm_server *s)
{
    // a server that mcm_shutdown already released is not freed twice
    if (s && unregister_handle(s)) server_free(s);
    return MCM_OK;
}

}  // extern "C"
