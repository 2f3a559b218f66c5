// Estimator entry point that allocates nothing, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation).
//
// ile_marginalize keeps its per-tile partials in a per-job device buffer that
// it grows on demand.  This variant keeps them in `scratch`, a file-scope
// device array of fixed size: every GPU the library runs on holds one copy of
// it until the process ends.  Host code must not pass the array's name to a
// kernel (on the host it is a stand-in symbol, not a device address): each
// device's address is looked up once, with that device current, when a
// context is created on it, and only that address is used afterwards.
#include <mutex>

#include "ile_ctx.h"

namespace {

constexpr size_t kScratchBytes = size_t(1) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

namespace ile {

// Look up this device's copy of the scratch array (the device must be
// current).  Called by ile_ctx_create; later calls for the device return at once.
ile_status noalloc_init_device(int device) {
    if (device < 0 || device >= kMaxDevices) return set_err(ILE_E_INVALID, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return ILE_OK;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) return dev_fail(nullptr, e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch symbol address");
    g_scratch_ptr[device] = p;
    return ILE_OK;
}

}  // namespace ile

using namespace ile;

extern "C" size_t ile_marginalize_noalloc_max(void) {
    // tiles hold marg_tile(n) samples; the largest n whose partials fit
    const int64_t cap = (int64_t)(kScratchBytes / sizeof(MargPartial));
    return (size_t)cap * (size_t)marg_tile(INT64_C(1) << 40);
}

extern "C" ile_status ile_marginalize_noalloc(ile_job *job, int64_t n, const void *lw, uint32_t flags,
                                              ile_marg *out, ile_stream stream) {
    if (!job) return set_err(ILE_E_INVALID, "null job");
    ile_status s = ctx_check(job->ctx);
    if (s != ILE_OK) return s;
    if (n < 0 || (n > 0 && !lw)) return set_err(ILE_E_INVALID, "bad lw");
    const int64_t tile = marg_tile(n);
    const int64_t np = std::max<int64_t>(1, (n + tile - 1) / tile);
    if ((size_t)np * sizeof(MargPartial) > kScratchBytes)
        return set_err(ILE_E_TOO_BIG, "ile_marginalize_noalloc: n = " + std::to_string(n) +
                                          " needs more partials than the fixed scratch holds (at most " +
                                          std::to_string(ile_marginalize_noalloc_max()) + " samples)");
    void *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        const int dev = job->ctx->device;
        ptr = (dev >= 0 && dev < kMaxDevices) ? g_scratch_ptr[dev] : nullptr;
    }
    if (!ptr) return set_err(ILE_E_STATE, "scratch of this device not initialised");
    hipStream_t st = (hipStream_t)stream;
    MargPartial *part = (MargPartial *)ptr;
    hipError_t e = hipSuccess;
    if (n > 0) e = launch_marg_partials(job->policy, lw, n, tile, part, st);
    if (e != hipSuccess) return dev_fail(job->ctx, e, "marginal partials (no-alloc)");
    e = launch_marg_combine(part, n > 0 ? (int)np : 0, n, job->d_ms, (flags & ILE_MARG_RESET) ? 1 : 0, st);
    if (e != hipSuccess) return dev_fail(job->ctx, e, "marginal combine (no-alloc)");
    if (out) {
        // job->h_ms is pinned host memory made when the job was prepared
        e = hipMemcpyAsync(job->h_ms, job->d_ms, sizeof(MargState), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return dev_fail(job->ctx, e, "read estimator (no-alloc)");
        marg_from_state(*job->h_ms, out);
    }
    return ILE_OK;
}
