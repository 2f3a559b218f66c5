// Host side of the product-form adaptive Cartesian sampler: the job's
// marginals (device state), and the reset / draw / update / readback entry
// points.  Draws and updates queue on the stream and read the marginals in
// device memory.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ile_ctx.h"
#include "k_qv.h"

using namespace ile;

namespace ile {

namespace {

void default_ac_dims(const ile_job *job, int *nd, int dims[7]) {
    int k = 0;
    for (int c = 0; c < 7; c++)
        if (!(job->dist_marg && c == 3)) dims[k++] = c;
    *nd = k;
}

}  // namespace

ile_status ac_ensure(ile_job *job, hipStream_t st) {
    if (job->d_ac) return ILE_OK;
    ile_status s = ctx_alloc(job->ctx, (void **)&job->d_ac, sizeof(AcDev), "adaptive Cartesian marginals");
    if (s != ILE_OK) return s;
    int nd, dims[7];
    default_ac_dims(job, &nd, dims);
    const hipError_t e = launch_ac_reset(job->d_ac, nd, dims, st);
    if (e != hipSuccess) return dev_fail(job->ctx, e, "adaptive Cartesian reset");
    return ILE_OK;
}

ile_status ac_batch(ile_ctx *ctx, bool update, int policy, const std::vector<AcJob> &jobs, hipStream_t st) {
    if (jobs.empty()) return ILE_OK;
    if (jobs.size() > 65535) return set_err(ILE_E_INVALID, "too many jobs in one adaptive Cartesian launch");
    std::lock_guard<std::mutex> lk(ctx->batch_mu);
    void *dj = nullptr, *dn = nullptr;
    int slot = -1;
    ile_status s = batch_upload(ctx, jobs.data(), jobs.size() * sizeof(AcJob), nullptr, 0, &dj, &dn, &slot, st);
    if (s != ILE_OK) return s;
    const hipError_t e = update ? launch_ac_update(policy, (const AcJob *)dj, jobs.data(), (int)jobs.size(), st)
                                : launch_ac_draw(policy, (const AcJob *)dj, jobs.data(), (int)jobs.size(), st);
    if (e != hipSuccess) return dev_fail(ctx, e, update ? "adaptive Cartesian update" : "adaptive Cartesian draw");
    return batch_done(ctx, slot, st);
}

}  // namespace ile

extern "C" ile_status ile_ac_reset(ile_job *job, int32_t n_dim, const int32_t *dims, ile_stream stream) {
    if (!job) return set_err(ILE_E_INVALID, "null job");
    ile_status s = ctx_check(job->ctx);
    if (s != ILE_OK) return s;
    int nd = 0, dd[7];
    if (n_dim == 0) {
        default_ac_dims(job, &nd, dd);
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
    if ((s = ac_ensure(job, st)) != ILE_OK) return s;
    const hipError_t e = launch_ac_reset(job->d_ac, nd, dd, st);
    if (e != hipSuccess) return dev_fail(job->ctx, e, "adaptive Cartesian reset");
    return ILE_OK;
}

extern "C" ile_status ile_ac_draw(ile_job *job, uint64_t seed, uint32_t round, int64_t first_index, int64_t n,
                                  void *theta_out, int64_t ld, void *lnpmps_out, ile_stream stream) {
    if (!job) return set_err(ILE_E_INVALID, "null job");
    ile_status s = ctx_check(job->ctx);
    if (s != ILE_OK) return s;
    if (n < 0 || ld < n || first_index < 0) return set_err(ILE_E_INVALID, "need n >= 0, ld >= n, first_index >= 0");
    if (n == 0) return ILE_OK;
    if (!theta_out) return set_err(ILE_E_INVALID, "null theta_out");
    hipStream_t st = (hipStream_t)stream;
    if ((s = ac_ensure(job, st)) != ILE_OK) return s;
    AcJob j{};
    j.st = job->d_ac;
    j.pr = job->pr;
    j.seed = seed;
    j.round = round;
    j.first = first_index;
    j.n = n;
    j.theta = theta_out;
    j.ld = ld;
    j.lnpmps = lnpmps_out;
    return ac_batch(job->ctx, false, job->policy, {j}, st);
}

extern "C" ile_status ile_ac_update(ile_job *job, uint64_t seed, uint32_t round, int64_t first_index, int64_t n,
                                    const void *lw, double floor_frac, ile_stream stream) {
    if (!job) return set_err(ILE_E_INVALID, "null job");
    ile_status s = ctx_check(job->ctx);
    if (s != ILE_OK) return s;
    if (n < 0 || first_index < 0) return set_err(ILE_E_INVALID, "need n >= 0 and first_index >= 0");
    const double fl = floor_frac == 0 ? 0.1 : floor_frac;
    if (!(fl > 0 && fl <= 1)) return set_err(ILE_E_INVALID, "floor must be in (0, 1]");
    hipStream_t st = (hipStream_t)stream;
    if ((s = ac_ensure(job, st)) != ILE_OK) return s;
    if (n == 0) return ILE_OK;
    if (!lw) return set_err(ILE_E_INVALID, "null lw");
    AcJob j{};
    j.st = job->d_ac;
    j.seed = seed;
    j.round = round;
    j.first = first_index;
    j.n = n;
    j.lw = lw;
    j.floor = fl;
    return ac_batch(job->ctx, true, job->policy, {j}, st);
}

extern "C" ile_status ile_ac_get(ile_job *job, int32_t *n_dim, int32_t *dims, double *pi, ile_stream stream) {
    if (!job) return set_err(ILE_E_INVALID, "null job");
    ile_status s = ctx_check(job->ctx);
    if (s != ILE_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    if ((s = ac_ensure(job, st)) != ILE_OK) return s;
    std::vector<char> h(sizeof(AcDev));
    hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipMemcpy(h.data(), job->d_ac, sizeof(AcDev), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return dev_fail(job->ctx, e, "adaptive Cartesian readback");
    AcDev S;
    std::memcpy(&S, h.data(), sizeof S);
    if (n_dim) *n_dim = S.d;
    if (dims)
        for (int k = 0; k < 7; k++) dims[k] = k < S.d ? S.dims[k] : -1;
    if (pi)
        for (int k = 0; k < S.d; k++)
            for (int b = 0; b < kAcBins; b++) pi[k * kAcBins + b] = S.pi[k][b];
    return ILE_OK;
}

extern "C" ile_status ile_overlaps(ile_ctx *ctx, const ile_qv_shape *sh, const void *hlm, const void *data,
                                   const double *inv_psd, void *Q, void *U, void *V, ile_stream stream) {
    if (!ctx || !sh) return set_err(ILE_E_INVALID, "null argument");
    ile_status s = ctx_check(ctx);
    if (s != ILE_OK) return s;
    if (sh->n_points < 1 || sh->n_modes < 1 || sh->n_det < 1 || sh->n_freq < 4 || sh->n_time < 1 ||
        sh->n_time > sh->n_freq || sh->n_modes > 1000 || !(sh->df > 0) || !(sh->f_hi >= sh->f_lo) || sh->f_lo < 0)
        return set_err(ILE_E_INVALID, "bad overlap shape");
    if (!hlm || !data || !Q || !U || !V) return set_err(ILE_E_INVALID, "null array");
    if (sh->route < ILE_QV_AUTO || sh->route > ILE_QV_DECIMATED) return set_err(ILE_E_INVALID, "bad overlap route");
    const int64_t n = sh->n_freq;
    std::vector<int64_t> band, msig;
    for (int64_t m = 0; m < n; m++) {
        const int64_t ms = m < (n + 1) / 2 ? m : m - n;   // FFT-order signed index
        const double af = std::fabs((double)ms * sh->df);
        if (af >= sh->f_lo && af <= sh->f_hi) {
            band.push_back(m);
            msig.push_back(ms);
        }
    }
    if (band.empty()) return set_err(ILE_E_INVALID, "no grid frequency inside the band");
    const int64_t n_band = (int64_t)band.size();
    const int64_t cols = (int64_t)sh->n_points * sh->n_det * sh->n_modes;
    int radix = 0;
    if (sh->route != ILE_QV_DIRECT) {
        radix = qv_radix(n, n_band, sh->n_time, sh->win_half, sh->route == ILE_QV_DECIMATED);
        if (radix == 0 && sh->route == ILE_QV_DECIMATED)
            return set_err(ILE_E_INVALID, "decimated route needs a radix in {2, 4, 8, 16} dividing n_freq that "
                                          "puts the window on at most 64 decimated times");
    }
    auto plan = [&](int r, int &ns_, size_t &need_) {
        ns_ = r ? qv_dec_slices(n, cols, sh->n_time, sh->win_half, r) : qv_slices(n_band, cols, sh->n_time);
        need_ = r ? qv_dec_scratch_bytes(n, n_band, cols, sh->n_time, sh->win_half, r, ns_)
                  : qv_scratch_bytes(n, n_band, cols, sh->n_time, ns_);
    };
    int ns = 0;
    size_t need = 0;
    plan(radix, ns, need);
    void *scratch = nullptr;
    const std::string prev_err = ile_last_error();   // kept if the fallback succeeds
    s = ctx_alloc(ctx, &scratch, need, "overlap scratch");
    if (s != ILE_OK && radix && sh->route == ILE_QV_AUTO) {
        // the decimated route's partial sums (n per column) do not fit where
        // the direct route's X (n_band per column) may: take the direct route
        radix = 0;
        plan(radix, ns, need);
        s = ctx_alloc(ctx, &scratch, need, "overlap scratch");
        if (s == ILE_OK) set_err(ILE_OK, prev_err);
    }
    if (s != ILE_OK) return s;
    // the band lists go through pinned staging, so that nothing in the call
    // waits for the stream before the final synchronisation
    const size_t stage_bytes = (size_t)n_band * (radix ? 8 : 16);
    char *stage = (char *)pin_alloc(ctx, stage_bytes);
    if (!stage) {
        ctx_free(ctx, scratch, need);
        return set_err(ILE_E_NOMEM, "pinned staging");
    }
    std::memcpy(stage, band.data(), (size_t)n_band * 8);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    if (radix) {
        e = launch_qv_dec(hlm, data, inv_psd, n, sh->n_modes, sh->n_det, sh->n_points, sh->df, sh->f_lo, sh->f_hi,
                          (const int64_t *)stage, n_band, sh->n_time, sh->win_half, radix, Q, U, V, scratch, ns, st);
    } else {
        std::memcpy(stage + (size_t)n_band * 8, msig.data(), (size_t)n_band * 8);
        e = launch_qv(hlm, data, inv_psd, n, sh->n_modes, sh->n_det, sh->n_points, sh->df, (const int64_t *)stage,
                      (const int64_t *)(stage + (size_t)n_band * 8), n_band, sh->n_time, sh->win_half, Q, U, V,
                      scratch, ns, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);   // the staging and the scratch are released below
    else (void)hipStreamSynchronize(st);
    ctx_free(ctx, scratch, need);
    pin_free(ctx, stage, stage_bytes);
    if (e != hipSuccess) return dev_fail(ctx, e, "overlaps");
    return ILE_OK;
}
