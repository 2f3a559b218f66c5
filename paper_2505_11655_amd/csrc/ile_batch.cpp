// Batched estimator entry point: many jobs' log-weights reduced in one
// partials launch and one combine launch, each job with the same tile
// decomposition as its single-job reduction (bitwise-identical results).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "ile.h"
#include "ile_ctx.h"
#include "ile_internal.h"

using namespace ile;

namespace ile {
constexpr int64_t kMargTileB = 16384;  // must equal the single-job tile

ile_status marg_batch(ile_ctx *ctx, ile_job *const *jobs, int n_jobs, const int64_t *n, const void *const *lw,
                      uint32_t flags, ile_marg *out, hipStream_t st) {
    std::vector<MargJob> mj(n_jobs);
    std::vector<Tile> tiles;
    const int policy = jobs[0]->policy == kFP32 ? kFP32 : kFP64;
    for (int j = 0; j < n_jobs; j++) {
        const int lwp = jobs[j]->policy == kFP32 ? kFP32 : kFP64;
        if (lwp != policy) return set_err(ILE_E_INVALID, "batched estimator needs one lw type");
        mj[j].lw = lw[j];
        mj[j].n = n[j];
        mj[j].tile_begin = (int32_t)tiles.size();
        for (int64_t t = 0; t < n[j]; t += kMargTileB) tiles.push_back(Tile{j, 0, t, std::min(t + kMargTileB, n[j])});
        mj[j].tile_end = (int32_t)tiles.size();
        mj[j].state = jobs[j]->d_ms;
        mj[j].out = nullptr;
        mj[j].reset = (flags & ILE_MARG_RESET) ? 1 : 0;
    }
    std::lock_guard<std::mutex> lk(ctx->batch_mu);
    hipError_t e;
    if (tiles.size() > ctx->part_cap || (size_t)n_jobs > ctx->mout_cap) {
        if ((e = hipDeviceSynchronize()) != hipSuccess) return dev_fail(ctx, e, "sync before growth");
        if (tiles.size() > ctx->part_cap) {
            if (ctx->d_part) (void)hipFree(ctx->d_part);
            ctx->d_part = nullptr;
            const size_t cap = std::max<size_t>(tiles.size() * 2, 4096);
            if ((e = hipMalloc((void **)&ctx->d_part, cap * sizeof(MargPartial))) != hipSuccess)
                return dev_fail(ctx, e, "partials");
            ctx->part_cap = cap;
        }
        if ((size_t)n_jobs > ctx->mout_cap) {
            if (ctx->d_mout) (void)hipFree(ctx->d_mout);
            if (ctx->h_mout) (void)hipHostFree(ctx->h_mout);
            ctx->d_mout = nullptr;
            ctx->h_mout = nullptr;
            const size_t cap = std::max<size_t>((size_t)n_jobs * 2, 256);
            if ((e = hipMalloc((void **)&ctx->d_mout, cap * sizeof(MargState))) != hipSuccess)
                return dev_fail(ctx, e, "result copies");
            if ((e = hipHostMalloc((void **)&ctx->h_mout, cap * sizeof(MargState), hipHostMallocDefault)) !=
                hipSuccess)
                return dev_fail(ctx, e, "pinned results");
            ctx->mout_cap = cap;
        }
    }
    if (out)
        for (int j = 0; j < n_jobs; j++) mj[j].out = ctx->d_mout + j;
    void *dj = nullptr, *dt = nullptr;
    ile_status s = batch_upload(ctx, mj.data(), mj.size() * sizeof(MargJob), tiles.data(), tiles.size() * sizeof(Tile),
                                &dj, &dt, st);
    if (s != ILE_OK) return s;
    e = launch_marg_batch(policy, (const MargJob *)dj, n_jobs, (const Tile *)dt, (int)tiles.size(), ctx->d_part, st);
    if (e != hipSuccess) return dev_fail(ctx, e, "batched estimator");
    if ((e = hipEventRecord(ctx->batch_ev, st)) != hipSuccess) return dev_fail(ctx, e, "batch event");
    if (out) {
        e = hipMemcpyAsync(ctx->h_mout, ctx->d_mout, (size_t)n_jobs * sizeof(MargState), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return dev_fail(ctx, e, "read batched estimator");
        for (int j = 0; j < n_jobs; j++) marg_from_state(ctx->h_mout[j], &out[j]);
    }
    return ILE_OK;
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
    return marg_batch(ctx, jobs, n_jobs, n, lw, flags, out, (hipStream_t)stream);
}
