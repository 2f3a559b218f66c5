// Host side of the adaptive-volume integrator (Section "Adaptive volume
// integration"): the job's grid buffers, and the reset / draw / update /
// readback entry points.  The grid itself (bin count, cell list, active
// volume) lives in device memory and is read there by the kernels, so draws
// and updates queue without host synchronisation.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "ile_ctx.h"

using namespace ile;

namespace ile {
namespace {

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// One allocation: [state | histogram | cells 0 | cells 1 | set keys | set
// indices | per-sample slots | per-block counts].
struct AvLayout {
    size_t st, hist, cells0, cells1, hkey, hidx, slot, bcnt, total;
    uint64_t hcap;
};

AvLayout av_layout(int64_t cap) {
    AvLayout L{};
    uint64_t h = 1024;
    while (h < (uint64_t)2 * (uint64_t)cap) h <<= 1;   // load factor <= 1/2
    L.hcap = h;
    size_t o = 0;
    L.st = o;
    o += align256(sizeof(AvDev));
    L.hist = o;
    o += align256(2 * 256 * 2 * sizeof(unsigned long long));
    L.cells0 = o;
    o += align256((size_t)cap * 8 * sizeof(uint16_t));
    L.cells1 = o;
    o += align256((size_t)cap * 8 * sizeof(uint16_t));
    L.hkey = o;
    o += align256(h * sizeof(unsigned long long));
    L.hidx = o;
    o += align256(h * sizeof(uint32_t));
    L.slot = o;
    o += align256((size_t)cap * sizeof(uint32_t));
    L.bcnt = o;
    o += align256(((size_t)cap / 256 + 2) * sizeof(uint32_t));
    L.total = o;
    return L;
}

AvBufs av_bufs(void *mem, const AvLayout &L) {
    char *m = (char *)mem;
    AvBufs b{};
    b.st = (AvDev *)(m + L.st);
    b.hist = (unsigned long long *)(m + L.hist);
    b.cells[0] = (uint16_t *)(m + L.cells0);
    b.cells[1] = (uint16_t *)(m + L.cells1);
    b.hkey = (unsigned long long *)(m + L.hkey);
    b.hidx = (uint32_t *)(m + L.hidx);
    b.hmask = L.hcap - 1;
    b.slot = (uint32_t *)(m + L.slot);
    b.bcnt = (uint32_t *)(m + L.bcnt);
    return b;
}

void default_av_dims(const ile_job *job, int *nd, int dims[7]) {
    int k = 0;
    for (int c = 0; c < 7; c++)
        if (!(job->dist_marg && c == 3)) dims[k++] = c;
    *nd = k;
}

ile_status av_reset_dims(ile_job *job, int nd, const int *dims, hipStream_t st) {
    hipError_t e = launch_av_reset(job->av, nd, dims, st);
    if (e != hipSuccess) return dev_fail(job->ctx, e, "adaptive-volume reset");
    return ILE_OK;
}

void state_out(const AvDev &S, ile_av_state *out) {
    std::memset(out, 0, sizeof *out);
    out->n_dim = S.d;
    for (int k = 0; k < 7; k++) out->dims[k] = k < S.d ? S.dims[k] : -1;
    out->n_bins = S.nb;
    out->n_cells = S.n_cells;
    out->ln_vol = S.ln_vol;
    out->lnL_thr = S.thr;
    out->n_min = S.n_min;
    out->n_live = S.n_live;
    out->vol_mc = S.vol_mc;
}

ile_status av_readback(ile_job *job, hipStream_t st) {
    hipError_t e = hipMemcpyAsync(job->h_av, job->av.st, sizeof(AvDev), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return dev_fail(job->ctx, e, "adaptive-volume state readback");
    return ILE_OK;
}

}  // namespace

// One launch per stage for all jobs (theta type for draws, log-weight type
// for updates: `policy` names it); descriptors go through a scratch slot.
ile_status av_batch(ile_ctx *ctx, bool update, int policy, const std::vector<AvJob> &jobs, hipStream_t st) {
    if (jobs.empty()) return ILE_OK;
    if (jobs.size() > 65535) return set_err(ILE_E_INVALID, "too many jobs in one adaptive-volume launch");
    std::lock_guard<std::mutex> lk(ctx->batch_mu);
    void *dj = nullptr, *dn = nullptr;
    int slot = -1;
    ile_status s = batch_upload(ctx, jobs.data(), jobs.size() * sizeof(AvJob), nullptr, 0, &dj, &dn, &slot, st);
    if (s != ILE_OK) return s;
    const hipError_t e = update ? launch_av_update(policy, (const AvJob *)dj, jobs.data(), (int)jobs.size(), st)
                                : launch_av_draw(policy, (const AvJob *)dj, jobs.data(), (int)jobs.size(), st);
    if (e != hipSuccess) return dev_fail(ctx, e, update ? "adaptive-volume update" : "adaptive-volume draw");
    return batch_done(ctx, slot, st);
}

size_t av_bytes_for(int64_t cap) { return av_layout(std::max<int64_t>(cap, 4096)).total; }

ile_status av_ensure(ile_job *job, int64_t cap, hipStream_t st) {
    if (job->av_mem && cap <= job->av_cap) return ILE_OK;
    ile_ctx *ctx = job->ctx;
    const int64_t ncap = std::max<int64_t>(cap, std::max<int64_t>(job->av_cap * 2, 4096));
    const AvLayout L = av_layout(ncap);
    void *mem = nullptr;
    ile_status s = ctx_alloc(ctx, &mem, L.total, "adaptive-volume grid");
    if (s != ILE_OK) return s;
    if (!job->h_av) {
        job->h_av = (AvDev *)pin_alloc(ctx, sizeof(AvDev));
        if (!job->h_av) {
            ctx_free(ctx, mem, L.total);
            return set_err(ILE_E_NOMEM, "pinned adaptive-volume state");
        }
    }
    const AvBufs nb = av_bufs(mem, L);
    const bool fresh = job->av_mem == nullptr;
    if (!fresh) {
        // keep the grid: the state and both cell buffers move to the new block
        const size_t cells = (size_t)job->av_cap * 8 * sizeof(uint16_t);
        hipError_t e = hipMemcpyAsync(nb.st, job->av.st, sizeof(AvDev), hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(nb.cells[0], job->av.cells[0], cells, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(nb.cells[1], job->av.cells[1], cells, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);   // before the old block returns to the pool
        if (e != hipSuccess) {
            ctx_free(ctx, mem, L.total);
            return dev_fail(ctx, e, "adaptive-volume grid growth");
        }
        ctx_free(ctx, job->av_mem, job->av_bytes);
    }
    job->av_mem = mem;
    job->av_bytes = L.total;
    job->av_cap = ncap;
    job->av = nb;
    if (fresh) {
        int nd, dims[7];
        default_av_dims(job, &nd, dims);
        return av_reset_dims(job, nd, dims, st);
    }
    return ILE_OK;
}

}  // namespace ile

extern "C" ile_status ile_av_reset(ile_job *job, int32_t n_dim, const int32_t *dims, ile_stream stream) {
    if (!job) return set_err(ILE_E_INVALID, "null job");
    ile_status s = ctx_check(job->ctx);
    if (s != ILE_OK) return s;
    int nd = 0, dd[7];
    if (n_dim == 0) {
        default_av_dims(job, &nd, dd);
    } else {
        if (n_dim < 0 || n_dim > 7 || !dims) return set_err(ILE_E_INVALID, "n_dim must be 0..7 with dims");
        for (int k = 0; k < n_dim; k++) {
            if (dims[k] < 0 || dims[k] > 6 || (k > 0 && dims[k] <= dims[k - 1]))
                return set_err(ILE_E_INVALID, "dims must be strictly increasing theta columns 0..6");
            if (job->dist_marg && dims[k] == 3)
                return set_err(ILE_E_INVALID, "the distance column is not sampled with dist_marg");
            dd[k] = dims[k];
        }
        nd = n_dim;
    }
    hipStream_t st = (hipStream_t)stream;
    if ((s = av_ensure(job, 1, st)) != ILE_OK) return s;
    return av_reset_dims(job, nd, dd, st);
}

extern "C" ile_status ile_av_draw(ile_job *job, uint64_t seed, uint32_t round, int64_t first_index, int64_t n,
                                  void *theta_out, int64_t ld, void *lnpmps_out, ile_stream stream) {
    if (!job) return set_err(ILE_E_INVALID, "null job");
    ile_status s = ctx_check(job->ctx);
    if (s != ILE_OK) return s;
    if (n < 0 || ld < n || first_index < 0) return set_err(ILE_E_INVALID, "need n >= 0, ld >= n, first_index >= 0");
    if (n == 0) return ILE_OK;
    if (!theta_out) return set_err(ILE_E_INVALID, "null theta_out");
    hipStream_t st = (hipStream_t)stream;
    if ((s = av_ensure(job, 1, st)) != ILE_OK) return s;
    AvJob j{};
    j.b = job->av;
    j.pr = job->pr;
    j.seed = seed;
    j.round = round;
    j.first = first_index;
    j.n = n;
    j.theta = theta_out;
    j.ld = ld;
    j.lnpmps = lnpmps_out;
    return av_batch(job->ctx, false, job->policy, {j}, st);
}

extern "C" ile_status ile_av_update(ile_job *job, uint64_t seed, uint32_t round, int64_t first_index, int64_t n,
                                    const void *lw, const ile_av_opts *opts, ile_av_state *out,
                                    ile_stream stream) {
    if (!job) return set_err(ILE_E_INVALID, "null job");
    ile_status s = ctx_check(job->ctx);
    if (s != ILE_OK) return s;
    if (n < 0 || n >= ((int64_t)1 << 31) || first_index < 0)
        return set_err(ILE_E_INVALID, "need 0 <= n < 2^31 and first_index >= 0");
    const double p_thr = opts && opts->p_thr != 0 ? opts->p_thr : 0.999;
    const int64_t n_min_live = opts && opts->n_min_live != 0 ? opts->n_min_live : 1000;
    const int max_bins = opts && opts->max_bins != 0 ? opts->max_bins : kAvMaxBins;
    if (!(p_thr > 0 && p_thr <= 1)) return set_err(ILE_E_INVALID, "p_thr must be in (0, 1]");
    if (n_min_live < 1) return set_err(ILE_E_INVALID, "n_min_live must be >= 1");
    if (max_bins < 1 || max_bins > kAvMaxBins) return set_err(ILE_E_INVALID, "max_bins must be 1..511");
    hipStream_t st = (hipStream_t)stream;
    if ((s = av_ensure(job, std::max<int64_t>(n, 1), st)) != ILE_OK) return s;
    if (n > 0) {
        if (!lw) return set_err(ILE_E_INVALID, "null lw");
        AvJob j{};
        j.b = job->av;
        j.seed = seed;
        j.round = round;
        j.first = first_index;
        j.n = n;
        j.lw = lw;
        j.p_thr = p_thr;
        j.n_min_live = n_min_live;
        j.max_bins = max_bins;
        if ((s = av_batch(job->ctx, true, job->policy, {j}, st)) != ILE_OK) return s;
    }
    if (out) {
        if ((s = av_readback(job, st)) != ILE_OK) return s;
        state_out(*job->h_av, out);
    }
    return ILE_OK;
}

extern "C" ile_status ile_av_get(ile_job *job, ile_av_state *out, int32_t *cells, int64_t cap, ile_stream stream) {
    if (!job) return set_err(ILE_E_INVALID, "null job");
    ile_status s = ctx_check(job->ctx);
    if (s != ILE_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    if ((s = av_ensure(job, 1, st)) != ILE_OK) return s;
    if ((s = av_readback(job, st)) != ILE_OK) return s;
    const AvDev S = *job->h_av;
    if (out) state_out(S, out);
    if (cells && cap > 0) {
        const int64_t m = std::min<int64_t>(cap, S.n_cells);
        std::vector<uint16_t> h((size_t)m * 8);
        hipError_t e = hipMemcpy(h.data(), S.cur ? job->av.cells[1] : job->av.cells[0], h.size() * sizeof(uint16_t),
                                 hipMemcpyDeviceToHost);
        if (e != hipSuccess) return dev_fail(job->ctx, e, "adaptive-volume cell readback");
        for (int64_t j = 0; j < m; j++)
            for (int k = 0; k < S.d; k++) cells[j * S.d + k] = h[j * 8 + k];
    }
    return ILE_OK;
}

extern "C" ile_status ile_fair_draw(ile_job *job, int64_t n, const void *lw, uint64_t seed, uint32_t round,
                                    int64_t k, int64_t *idx_out, const void *theta, int64_t ld, void *theta_out,
                                    int64_t ld_out, ile_stream stream) {
    if (!job) return set_err(ILE_E_INVALID, "null job");
    ile_status s = ctx_check(job->ctx);
    if (s != ILE_OK) return s;
    if (n < 1 || k < 0) return set_err(ILE_E_INVALID, "need n >= 1 and k >= 0");
    if (!lw) return set_err(ILE_E_INVALID, "null lw");
    if (theta_out && (!theta || ld < n || ld_out < k)) return set_err(ILE_E_INVALID, "theta_out needs theta, ld >= n, ld_out >= k");
    if (!idx_out && !theta_out) return set_err(ILE_E_INVALID, "no output");
    if (k == 0) return ILE_OK;
    hipStream_t st = (hipStream_t)stream;
    const size_t need = fair_scratch_bytes(n);
    if (need > job->fair_cap) {
        hipError_t e = hipStreamSynchronize(st);   // queued draws may still read the old scratch
        if (e != hipSuccess) return dev_fail(job->ctx, e, "sync before fair-draw scratch growth");
        ctx_free(job->ctx, job->fair_mem, job->fair_cap);
        job->fair_mem = nullptr;
        job->fair_cap = 0;
        if ((s = ctx_alloc(job->ctx, &job->fair_mem, need, "fair-draw scratch")) != ILE_OK) return s;
        job->fair_cap = need;
    }
    hipError_t e = launch_fair_draw(job->policy, lw, n, seed, round, k, idx_out, theta, ld, theta_out, ld_out,
                                    job->fair_mem, st);
    if (e != hipSuccess) return dev_fail(job->ctx, e, "fair draw");
    return ILE_OK;
}
