// mcm_match_noalloc: mcm_match for callers that cannot allocate memory
// (code under stream capture, tight serving loops, harnesses that forbid
// device allocation).  The state of a match lives in one file-scope device
// array, `scratch`, of kScratchBytes; the host side keeps its control-block
// copy and descriptor staging in static host memory.  Nothing here calls
// hipMalloc, hipFree, hipHostMalloc or hipEventCreate.
//
// `scratch` is a host-side stand-in in host code: its device address is
// looked up once per device with hipGetSymbolAddress (with that device
// current) and only that address is handed to kernels and copies.  Every
// device holds its own copy of the array, at its own address, until the
// process ends.
//
// Calls on one device share the array, and calls that overlapped there
// would race on it; the library makes them take turns with a per-device
// lock held until the call's stream has finished with the array.  What the
// last call left in the array has no meaning for the next one: everything a
// match reads before writing is set by the match itself (the control block
// and barrier lines by their setup kernels, the working state from the
// initial matching).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "mcm_host.h"

using namespace mcm;
using namespace mcm::host;

namespace {

// 64 MiB: a graph needs 32 B per row, 12 B per column and 32 B per frontier
// queue entry (one per column, plus one per 64 edges of the columns split
// into 64-edge pieces), plus about 260 KB of control and barrier lines;
// for example up to about 800 000 vertices per side at 4 edges per column.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr size_t kAlign = 256;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct NoAllocDevice {
    std::mutex mu;                 // calls on this device take turns
    bool ready = false;            // set-up done (symbol address and device queries)
    unsigned char *ptr = nullptr;  // this device's copy of `scratch` (device address)
    DevInfo info;
    alignas(128) uint32_t h_ctrl[L_NLINES * kLineWords];  // host copy of the control block
    BatchDesc h_desc;              // host staging of the one-workgroup descriptor
};

NoAllocDevice g_dev[kMaxDevices];

size_t al(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }

// Once per device, with the device current: the device address of its copy
// of `scratch`, and the device facts the launches need.
int64_t setup_device(int dev, NoAllocDevice &d)
{
    if (d.ready) return 0;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(MCM_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
    int64_t rc;
    if ((rc = get_device_info(dev, &d.info))) return rc;
    d.ptr = static_cast<unsigned char *>(p);
    d.ready = true;
    return 0;
}

// The state slices of one match, carved from `base` (null: sizes only).
// Returns the bytes used.
size_t carve(unsigned char *base, size_t nc, size_t nr, size_t cap_q, uint32_t flags, bool single_wg,
             const Options &o, RunBufs *b)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        void *p = base ? base + off : nullptr;
        off += al(bytes);
        return p;
    };
    b->ctrl = static_cast<uint32_t *>(take((size_t)L_NLINES * 128));
    b->bar = static_cast<uint32_t *>(take((size_t)kMaxGridBlocks * 128));
    b->desc = static_cast<BatchDesc *>(take(sizeof(BatchDesc)));
    b->card = static_cast<int64_t *>(take(sizeof(int64_t)));
    b->rw = static_cast<uint64_t *>(take(8 * nr));
    b->pred = static_cast<int32_t *>(take(4 * nr));
    b->ends = static_cast<int32_t *>(take(4 * nr));
    b->cdone = static_cast<uint32_t *>(take(4 * nc));
    b->fq = static_cast<int4 *>(take(sizeof(int4) * 2 * cap_q));
    b->cap_q = cap_q;
    b->radj = (flags & F_MAXCLAIM) ? static_cast<int2 *>(take(sizeof(int2) * nr)) : nullptr;
    b->prow = (flags & F_FASTALT) ? static_cast<int32_t *>(take(4 * nr)) : nullptr;
    b->touched = (!single_wg && o.fix != 0) ? static_cast<int32_t *>(take(4 * nr)) : nullptr;
    b->rlist = (!single_wg && o.roots != 0) ? static_cast<int32_t *>(take(8 * nc)) : nullptr;
    b->ptrace = nullptr;  // no per-phase record (mcm_last_phases reports none after this call)
    b->h_ptrace = nullptr;
    b->ev0 = b->ev1 = nullptr;  // no event timing (kernel_ms reads 0)
    return off;
}

__global__ void k_fill_unmatched(int32_t *a, int32_t n)
{
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) a[i] = -1;
}

hipError_t fill_unmatched(int32_t *a, int32_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int blocks = (int)std::min<int64_t>(1024, ((int64_t)n + 255) / 256);
    hipLaunchKernelGGL(k_fill_unmatched, dim3(blocks), dim3(256), 0, st, a, n);
    return hipGetLastError();
}

}  // namespace

extern "C" int64_t mcm_match_noalloc(int32_t ncols, int32_t nrows, const int32_t *colptr, const int32_t *rowind,
                                     const int32_t *init_cmatch, const int32_t *init_rmatch, int32_t *out_cmatch,
                                     int32_t *out_rmatch, void *stream)
{
    int64_t rc;
    if ((rc = check_graph_args(ncols, nrows, colptr, rowind))) return rc;
    if ((init_cmatch == nullptr) != (init_rmatch == nullptr))
        return fail(MCM_EINVAL, "init_cmatch and init_rmatch must both be NULL or both be given");
    if ((ncols > 0 && !out_cmatch) || (nrows > 0 && !out_rmatch)) return fail(MCM_EINVAL, "output array is NULL");
    int dev = 0;
    if (current_device(&dev) || dev < 0 || dev >= kMaxDevices) return fail(MCM_EHIP, "no current HIP device");
    NoAllocDevice &d = g_dev[dev];
    std::lock_guard<std::mutex> lk(d.mu);
    if ((rc = setup_device(dev, d))) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    // on every return path the stream is done with the array before the
    // lock passes to the next call (destroyed before `lk`)
    struct StreamDone {
        hipStream_t s;
        ~StreamDone() { (void)hipStreamSynchronize(s); }
    } done{st};
    if ((rc = check_null_rowind(ncols, nrows, colptr, rowind, st))) return rc;
    if (ncols == 0 || nrows == 0) {
        HIPCHK(fill_unmatched(out_cmatch, ncols, st));
        HIPCHK(fill_unmatched(out_rmatch, nrows, st));
        HIPCHK(hipStreamSynchronize(st));
        return 0;
    }
    const Options o = opts();
    const bool single_wg = (int64_t)ncols + nrows <= o.wg_threshold;
    size_t qcap = 0;
    int64_t nnz = -1;
    if ((rc = queue_capacity(ncols, colptr, single_wg ? 0u : (uint32_t)o.split, st, &qcap,
                             single_wg ? nullptr : &nnz)))
        return rc;
    const uint32_t flags = match_flags(o, ncols, nrows, nnz, single_wg);
    const size_t cap_q = std::max(qcap, (size_t)ncols);
    RunBufs b;
    const size_t need = carve(nullptr, (size_t)ncols, (size_t)nrows, cap_q, flags, single_wg, o, &b);
    if (need > kScratchBytes)
        return fail(MCM_ENOMEM,
                    "mcm_match_noalloc: a graph of %d columns and %d rows needs %zu bytes of state, the fixed "
                    "array holds %zu",
                    ncols, nrows, need, kScratchBytes);
    carve(d.ptr, (size_t)ncols, (size_t)nrows, cap_q, flags, single_wg, o, &b);
    b.h_ctrl = d.h_ctrl;
    b.h_desc = &d.h_desc;
    b.info = d.info;
    return match_run(b, o, flags, single_wg, ncols, nrows, colptr, rowind, init_cmatch, init_rmatch, out_cmatch,
                     out_rmatch, st, stream);
}
