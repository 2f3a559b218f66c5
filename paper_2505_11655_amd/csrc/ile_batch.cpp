// Batched estimator entry point: many jobs' log-weights reduced in one
// partials launch and one combine launch, each job with the same tile
// decomposition as its single-job reduction (bitwise-identical results).
// Descriptors, tile partials and the per-job result copies live in one
// scratch slot of the context.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "ile.h"
#include "ile_ctx.h"
#include "ile_internal.h"

using namespace ile;

namespace ile {

ile_status marg_batch(ile_ctx *ctx, ile_job *const *jobs, int n_jobs, const int64_t *n, const void *const *lw,
                      const uint32_t *flags, ile_marg *out, hipStream_t st) {
    std::vector<MargJob> mj(n_jobs);
    std::vector<Tile> tiles;
    const int policy = jobs[0]->policy == kFP32 ? kFP32 : kFP64;
    for (int j = 0; j < n_jobs; j++) {
        const int lwp = jobs[j]->policy == kFP32 ? kFP32 : kFP64;
        if (lwp != policy) return set_err(ILE_E_INVALID, "batched estimator needs one lw type");
        mj[j].lw = lw[j];
        mj[j].n = n[j];
        mj[j].tile_begin = (int32_t)tiles.size();
        const int64_t mt = marg_tile(n[j]);   // the single-job tile
        for (int64_t t = 0; t < n[j]; t += mt) tiles.push_back(Tile{j, 0, t, std::min(t + mt, n[j])});
        mj[j].tile_end = (int32_t)tiles.size();
        mj[j].state = jobs[j]->d_ms;
        mj[j].out_idx = out ? j : -1;
        mj[j].reset = (flags[j] & ILE_MARG_RESET) ? 1 : 0;
    }
    const size_t part_bytes = std::max<size_t>(tiles.size(), 1) * sizeof(MargPartial);
    const size_t off_out = (part_bytes + 255) / 256 * 256;
    const size_t extra = off_out + (size_t)n_jobs * sizeof(MargState);
    std::lock_guard<std::mutex> lk(ctx->batch_mu);
    void *dj = nullptr, *dt = nullptr, *dx = nullptr, *hx = nullptr;
    int slot = -1;
    ile_status s = batch_upload(ctx, mj.data(), mj.size() * sizeof(MargJob), tiles.data(), tiles.size() * sizeof(Tile),
                                &dj, &dt, &slot, st, extra, &dx, &hx);
    if (s != ILE_OK) return s;
    MargPartial *d_part = (MargPartial *)dx;
    MargState *d_out = (MargState *)((char *)dx + off_out);
    MargState *h_out = (MargState *)((char *)hx + off_out);
    hipError_t e = launch_marg_batch(policy, (const MargJob *)dj, n_jobs, (const Tile *)dt, (int)tiles.size(), d_part,
                                     out ? d_out : nullptr, st);
    if (e != hipSuccess) return dev_fail(ctx, e, "batched estimator");
    if (out) {
        e = hipMemcpyAsync(h_out, d_out, (size_t)n_jobs * sizeof(MargState), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return dev_fail(ctx, e, "read batched estimator");
        for (int j = 0; j < n_jobs; j++) marg_from_state(h_out[j], &out[j]);
    }
    return batch_done(ctx, slot, st);
}
}  // namespace ile

extern "C" ile_status ile_marginalize_batch(ile_job *const *jobs, int32_t n_jobs, const int64_t *n,
                                            const void *const *lw, uint32_t flags, ile_marg *out, ile_stream stream) {
    if (n_jobs <= 0) return ILE_OK;
    if (!jobs || !n || !lw || !jobs[0]) return set_err(ILE_E_INVALID, "null argument");
    ile_ctx *ctx = jobs[0]->ctx;
    ile_status s = ctx_check(ctx);
    if (s != ILE_OK) return s;
    for (int j = 0; j < n_jobs; j++) {
        if (!jobs[j] || jobs[j]->ctx != ctx) return set_err(ILE_E_INVALID, "jobs must share one context");
        if (n[j] < 0 || (n[j] > 0 && !lw[j])) return set_err(ILE_E_INVALID, "bad lw");
    }
    std::vector<uint32_t> fl(n_jobs, flags);
    return marg_batch(ctx, jobs, n_jobs, n, lw, fl.data(), out, (hipStream_t)stream);
}
