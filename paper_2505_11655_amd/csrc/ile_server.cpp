// Continuous-batching server for marginal-likelihood jobs.
//
// A job is one intrinsic point: its Q/U/V inputs (copied at submit), a sample
// budget (plain) or a round size with a refit rule (adaptive).  One scheduler
// thread owns a HIP stream and loops:
//   1. admit queued jobs in arrival order while a slot is free and the job's
//      device footprint fits the budget (prepare: upload and keep resident);
//   2. build one pass over every admitted job: its next chunk (plain) or round
//      (adaptive) of samples;
//   3. launch, for all of them together, one counter-based draw, one lnL
//      launch per compiled kernel class, and one estimator launch; read back
//      the per-job pooled estimator states (the only host sync per pass);
//   4. finish jobs whose budget is spent or whose n_eff reached the target (or
//      whose round cap is hit), refit the proposal of the others from this
//      round's samples, free finished jobs' memory, post their results.
// Jobs that arrive while a pass runs are admitted in the next pass, so their
// work overlaps with the jobs already on the device.  With a backlog, queued
// jobs are also admitted while a pass's kernels run (before its one
// synchronisation): their host preparation overlaps the device work, their
// uploads follow the pass on the stream, and they join the active set at the
// next pass in arrival order.  Every quantity a job
// computes depends only on its own inputs, key and chunk sizes (draw counters,
// per-sample likelihood, fixed estimator tiles), so its result is bitwise the
// same alone or in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ile.h"
#include "ile_ctx.h"
#include "ile_internal.h"

using namespace ile;

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

enum ReqState { kQueued, kActive, kDone };

struct Req {
    uint64_t id = 0;
    // host copy of the problem
    std::vector<int32_t> ml, mm;
    std::vector<double> pos, resp, Q, U, V;
    ile_problem prob{};
    ile_job_opts jo{};
    size_t footprint = 0;
    // device state while admitted
    ile_job *job = nullptr;
    void *d_theta = nullptr, *d_lr = nullptr, *d_lw = nullptr;
    size_t buf_bytes = 0;
    // mixture pool (adaptive mixture jobs with ILE_POOL_MIXTURE): every round's
    // theta [7][pool_cap], lnL, ln sum p_s,q/p and pooled weights, and the
    // proposal of every round
    void *d_pth = nullptr, *d_pL = nullptr, *d_plw = nullptr;
    double *d_plmix = nullptr;
    GmmDev *d_hist = nullptr;
    int64_t pool_cap = 0;
    int64_t chunk = 0;        // samples per pass
    int64_t done = 0;         // samples evaluated
    int32_t rounds = 0;
    ReqState state = kQueued;
    bool cancel = false;
    ile_result res{};
};

}  // namespace

struct ile_server {
    ile_ctx *ctx = nullptr;
    ile_server_opts opts{};
    size_t budget = 0, used = 0;
    std::thread th;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    uint64_t next_id = 1;
    std::deque<Req *> queue;
    std::vector<Req *> ready;    // admitted during a pass; active from the next one
    std::vector<Req *> active;
    std::unordered_map<uint64_t, std::unique_ptr<Req>> all;
    int64_t n_done = 0;
    hipStream_t stream = nullptr;
    // Input uploads of the jobs admitted while a pass runs: a stream of their
    // own, so that the copies run beside the pass's kernels instead of after
    // them; the next pass waits for them through up_ev.  Jobs admitted
    // between passes upload on `stream` itself, where a wait across streams
    // would only add latency.  Created at the first admission during a pass,
    // so a server that never admits during a pass runs on one stream.
    hipStream_t up = nullptr;
    hipEvent_t up_ev = nullptr;
    bool up_pending = false;   // uploads queued on `up` since the last wait (scheduler thread only)
    bool failed = false;
};

namespace {

size_t theta_bytes(int policy) { return policy == kFP64 ? 8 : 4; }
size_t lw_bytes(int policy) { return policy == kFP32 ? 4 : 8; }
size_t lnl_bytes(int policy) { return policy == kFP32 ? 4 : 8; }

bool pools_mixture(const Req *r) {
    return r->jo.adaptive && r->jo.integrator == ILE_INT_GMM && r->jo.pool == ILE_POOL_MIXTURE;
}
int max_rounds_of(const Req *r) { return r->jo.max_rounds > 0 ? r->jo.max_rounds : 32; }

int64_t chunk_of(const ile_server *s, const Req *r) {
    if (r->jo.adaptive) return r->jo.round_samples > 0 ? r->jo.round_samples : 65536;
    int64_t c = s->opts.chunk_samples > 0 ? s->opts.chunk_samples : (1 << 20);
    // a time-marginalised sample costs ~30-50x a pointwise one
    if (r->jo.tmarg_oversample) c = std::max<int64_t>(1, c / 16);
    return std::max<int64_t>(1, std::min(c, r->jo.n_samples));
}

// Device bytes a job holds while admitted (inputs in the policy's precision,
// sample buffers for one pass, estimator partials, mixture and EM workspace).
size_t footprint_of(const ile_server *s, const Req *r) {
    const ile_problem &P = r->prob;
    const int policy = P.precision;
    const size_t cr = policy == kFP32 ? 4 : 8;
    const int kp = P.n_det == 1 ? 2 : P.n_det;
    const int nm = 21;   // upper bound on compiled slots
    const size_t inputs = (size_t)kp * P.n_time * nm * 2 * cr + 2 * (size_t)(nm * (nm + 1) / 2) * kp * 2 * cr;
    const int64_t c = chunk_of(s, r);
    const size_t bufs = (size_t)c * (8 * theta_bytes(policy) + lw_bytes(policy));
    // the estimator's partials: one per marg_tile(c) samples of a chunk
    const int64_t mt = marg_tile(c);
    size_t extra = sizeof(MargState) + (size_t)((c + mt - 1) / mt + 1) * sizeof(MargPartial);
    if (r->jo.adaptive && r->jo.integrator == ILE_INT_AV)
        extra += av_bytes_for(c);
    else if (r->jo.adaptive && r->jo.integrator == ILE_INT_AC)
        extra += sizeof(AcDev);
    else if (r->jo.adaptive)
        extra += sizeof(GmmDev) + em_work_bytes(c) + 64 * sizeof(uint32_t);
    if (pools_mixture(r)) {
        const int64_t cap = (int64_t)max_rounds_of(r) * c;
        // pooled estimator partials over the whole pool, theta, lnL, ln sum, lw, proposals
        extra += (size_t)((cap + marg_tile(cap) - 1) / marg_tile(cap) + 1) * sizeof(MargPartial);
        extra += (size_t)cap * (7 * theta_bytes(policy) + lnl_bytes(policy) + 8 + lw_bytes(policy)) +
                 (size_t)(max_rounds_of(r) + 1) * sizeof(GmmDev);
    }
    return inputs + bufs + extra;
}

void finish(ile_server *s, Req *r, int status, const ile_marg *m) {
    r->res.status = status;
    if (m) r->res.marg = *m;
    r->res.rounds = r->rounds;
    r->res.samples = r->done;
    r->res.t_finish_ns = now_ns();
    if (r->job) {
        // a job that never joined a pass may still have its uploads in flight
        if (r->res.t_start_ns == 0) {
            if (s->up) (void)hipStreamSynchronize(s->up);
            (void)hipStreamSynchronize(s->stream);
        }
        const int policy = r->prob.precision;
        ctx_free(s->ctx, r->d_theta, (size_t)7 * r->chunk * theta_bytes(policy));
        ctx_free(s->ctx, r->d_lr, (size_t)r->chunk * theta_bytes(policy));
        ctx_free(s->ctx, r->d_lw, (size_t)r->chunk * lw_bytes(policy));
        r->d_theta = r->d_lr = r->d_lw = nullptr;
        if (r->pool_cap) {
            ctx_free(s->ctx, r->d_pth, (size_t)7 * r->pool_cap * theta_bytes(policy));
            ctx_free(s->ctx, r->d_pL, (size_t)r->pool_cap * lnl_bytes(policy));
            ctx_free(s->ctx, r->d_plmix, (size_t)r->pool_cap * sizeof(double));
            ctx_free(s->ctx, r->d_plw, (size_t)r->pool_cap * lw_bytes(policy));
            ctx_free(s->ctx, r->d_hist, (size_t)(max_rounds_of(r) + 1) * sizeof(GmmDev));
            r->d_pth = r->d_pL = r->d_plw = nullptr;
            r->d_plmix = nullptr;
            r->d_hist = nullptr;
            r->pool_cap = 0;
        }
        job_release_nosync(r->job);   // the server stream has no queued work for it
        r->job = nullptr;
    }
    s->used -= std::min(s->used, r->footprint);
    r->state = kDone;
    s->n_done++;
    // the host copy of the inputs is no longer needed
    r->Q.clear(); r->Q.shrink_to_fit();
    r->U.clear(); r->U.shrink_to_fit();
    r->V.clear(); r->V.shrink_to_fit();
}

// Admit one request: prepare its job and allocate its pass buffers; its
// uploads go on `up` (s->up during a pass, s->stream between passes).
ile_status admit(ile_server *s, Req *r, hipStream_t up) {
    ile_job *job = nullptr;
    if (up != s->stream) s->up_pending = true;
    ile_status st = job_create(s->ctx, &r->prob, &job, up, true);
    if (st != ILE_OK) return st;
    r->job = job;
    r->chunk = chunk_of(s, r);
    const int policy = r->prob.precision;
    const size_t tb = theta_bytes(policy);
    if (r->jo.adaptive && r->jo.integrator == ILE_INT_AV && (st = av_ensure(job, r->chunk, up)) != ILE_OK)
        return st;
    if (r->jo.adaptive && r->jo.integrator == ILE_INT_AC && (st = ac_ensure(job, up)) != ILE_OK) return st;
    if ((st = ctx_alloc(s->ctx, &r->d_theta, (size_t)7 * r->chunk * tb, "theta")) != ILE_OK) return st;
    if ((st = ctx_alloc(s->ctx, &r->d_lr, (size_t)r->chunk * tb, "ln p - ln ps")) != ILE_OK) return st;
    if ((st = ctx_alloc(s->ctx, &r->d_lw, (size_t)r->chunk * lw_bytes(policy), "lw")) != ILE_OK) return st;
    if (pools_mixture(r)) {
        const int64_t cap = (int64_t)max_rounds_of(r) * r->chunk;
        r->pool_cap = cap;   // set first: finish() frees whatever was allocated
        if ((st = ctx_alloc(s->ctx, &r->d_pth, (size_t)7 * cap * tb, "pool theta")) != ILE_OK ||
            (st = ctx_alloc(s->ctx, &r->d_pL, (size_t)cap * lnl_bytes(policy), "pool lnL")) != ILE_OK ||
            (st = ctx_alloc(s->ctx, (void **)&r->d_plmix, (size_t)cap * sizeof(double), "pool ln sum")) != ILE_OK ||
            (st = ctx_alloc(s->ctx, &r->d_plw, (size_t)cap * lw_bytes(policy), "pool lw")) != ILE_OK ||
            (st = ctx_alloc(s->ctx, (void **)&r->d_hist, (size_t)(max_rounds_of(r) + 1) * sizeof(GmmDev),
                            "pool proposals")) != ILE_OK)
            return st;
    }
    r->res.t_admit_ns = now_ns();
    return ILE_OK;
}

int max_active_of(const ile_server *s) { return s->opts.max_active > 0 ? s->opts.max_active : 256; }

// The upload stream, created on first use; the pass stream if that fails.
hipStream_t upload_stream(ile_server *s) {
    if (s->up) return s->up;
    if (hipStreamCreateWithFlags(&s->up, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        s->up = nullptr;
        return s->stream;
    }
    if (hipEventCreateWithFlags(&s->up_ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipStreamDestroy(s->up);
        s->up = nullptr;
        s->up_ev = nullptr;
        return s->stream;
    }
    return s->up;
}

// Admit queued jobs while a pass's kernels run, up to max_active of them, in
// arrival order and within the budget (a cancelled job at the front waits for
// the scheduler, which finishes it).  Every queued job would be admitted
// before the next pass anyway; here its host preparation overlaps the pass's
// kernels and its uploads run on the upload stream beside them, so nothing is
// queued on the pass stream ahead of the pass's own estimator.
void pre_admit(ile_server *s) {
    const int maxa = max_active_of(s);
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->queue.empty()) return;
    while (!s->queue.empty() && (int)s->ready.size() < maxa && !s->failed && !s->stop) {
        Req *r = s->queue.front();
        if (r->cancel || s->used + r->footprint > s->budget) break;
        s->queue.pop_front();
        s->used += r->footprint;
        lk.unlock();
        const ile_status st = admit(s, r, upload_stream(s));
        lk.lock();
        if (st != ILE_OK) {
            finish(s, r, st, nullptr);
            continue;
        }
        s->ready.push_back(r);
    }
}

// One scheduling pass over the active set.  Returns false on a device error.
bool run_pass(ile_server *s, std::vector<Req *> &act) {
    hipStream_t st = s->stream;
    if (s->up_pending) {   // the inputs of the jobs admitted since the last pass
        if (hipEventRecord(s->up_ev, s->up) != hipSuccess || hipStreamWaitEvent(st, s->up_ev, 0) != hipSuccess)
            return false;
        s->up_pending = false;
    }
    const int64_t t_start = now_ns();
    // draws, grouped by theta type
    std::vector<DrawJob> d32, d64;
    std::vector<AvJob> av32, av64;   // adaptive-volume draws by theta type
    std::vector<AcJob> ac32, ac64;   // adaptive Cartesian draws by theta type
    std::vector<BatchItem> items, tm1, tm4;   // pointwise; time-marginalised with R = 1, 4
    std::vector<int64_t> nthis(act.size());
    for (size_t i = 0; i < act.size(); i++) {
        Req *r = act[i];
        if (r->res.t_start_ns == 0) r->res.t_start_ns = t_start;
        const int64_t n = r->jo.adaptive ? r->chunk : std::min(r->chunk, r->jo.n_samples - r->done);
        nthis[i] = n;
        // a pooled job draws straight into its pool, at this round's slice
        void *th_out = r->d_theta;
        int64_t ld = n;
        void *lnl_out = nullptr;
        if (r->pool_cap) {
            const int policy = r->prob.precision;
            th_out = (char *)r->d_pth + (size_t)r->rounds * r->chunk * theta_bytes(policy);
            ld = r->pool_cap;
            lnl_out = (char *)r->d_pL + (size_t)r->rounds * r->chunk * lnl_bytes(policy);
            if (r->rounds >= 1 && hipMemcpyAsync(r->d_hist + r->rounds, r->job->d_gmm, sizeof(GmmDev),
                                                 hipMemcpyDeviceToDevice, st) != hipSuccess)
                return false;
        }
        const BatchItem bi{r->job, n, th_out, ld, r->d_lr, lnl_out, r->d_lw};
        (r->jo.tmarg_oversample == 4 ? tm4 : r->jo.tmarg_oversample == 1 ? tm1 : items).push_back(bi);
        if (r->jo.adaptive && r->jo.integrator == ILE_INT_AV) {
            AvJob aj{};
            aj.b = r->job->av;
            aj.pr = r->job->pr;
            aj.seed = r->jo.seed;
            aj.round = (uint32_t)r->rounds;
            aj.n = n;
            aj.theta = r->d_theta;
            aj.ld = n;
            aj.lnpmps = r->d_lr;
            (r->prob.precision == kFP64 ? av64 : av32).push_back(aj);
            continue;
        }
        if (r->jo.adaptive && r->jo.integrator == ILE_INT_AC) {
            AcJob cj{};
            cj.st = r->job->d_ac;
            cj.pr = r->job->pr;
            cj.seed = r->jo.seed;
            cj.round = (uint32_t)r->rounds;
            cj.n = n;
            cj.theta = r->d_theta;
            cj.ld = n;
            cj.lnpmps = r->d_lr;
            (r->prob.precision == kFP64 ? ac64 : ac32).push_back(cj);
            continue;
        }
        DrawJob dj{};
        dj.gmm = r->job->has_prop ? r->job->d_gmm : nullptr;
        dj.pr = r->job->pr;
        dj.seed = r->jo.seed;
        dj.round = r->jo.adaptive ? (uint32_t)r->rounds : 0u;
        dj.first = r->jo.adaptive ? 0 : r->done;
        dj.theta = th_out;
        dj.ld = ld;
        dj.lnpmps = r->d_lr;
        dj.n = n;
        (r->prob.precision == kFP64 ? d64 : d32).push_back(dj);
    }
    if (!d32.empty() && draw_batch(s->ctx, kFP32, d32, st) != ILE_OK) return false;
    if (!d64.empty() && draw_batch(s->ctx, kFP64, d64, st) != ILE_OK) return false;
    if (av_batch(s->ctx, false, kFP32, av32, st) != ILE_OK) return false;
    if (av_batch(s->ctx, false, kFP64, av64, st) != ILE_OK) return false;
    if (ac_batch(s->ctx, false, kFP32, ac32, st) != ILE_OK) return false;
    if (ac_batch(s->ctx, false, kFP64, ac64, st) != ILE_OK) return false;
    if (!items.empty() && eval_batch(s->ctx, items, st) != ILE_OK) return false;
    if (!tm1.empty() && tmarg_batch(s->ctx, tm1, 1, st) != ILE_OK) return false;
    if (!tm4.empty() && tmarg_batch(s->ctx, tm4, 4, st) != ILE_OK) return false;
    // mixture pools: every sample reweighted by the mixture of the rounds' proposals
    {
        std::vector<PoolJob> pj[3];
        for (size_t i = 0; i < act.size(); i++) {
            Req *r = act[i];
            if (!r->pool_cap) continue;
            PoolJob q{};
            q.theta = r->d_pth;
            q.ld = r->pool_cap;
            q.lnL = r->d_pL;
            q.lmix = r->d_plmix;
            q.lw = r->d_plw;
            q.hist = r->d_hist;
            q.pr = r->job->pr;
            q.n_round = r->chunk;
            q.round = r->rounds;
            pj[r->prob.precision].push_back(q);
        }
        for (int pol = 0; pol < 3; pol++)
            if (!pj[pol].empty() && pool_batch(s->ctx, pol, pj[pol], st) != ILE_OK) return false;
    }
    // the next jobs' host preparation overlaps the kernels queued so far
    pre_admit(s);
    // estimator, grouped by lw type (float for FP32, double otherwise)
    std::vector<ile_marg> res(act.size());
    for (int g = 0; g < 2; g++) {
        std::vector<ile_job *> jobs;
        std::vector<int64_t> ns;
        std::vector<const void *> lws;
        std::vector<uint32_t> fl;
        std::vector<size_t> idx;
        for (size_t i = 0; i < act.size(); i++) {
            const bool f32 = act[i]->prob.precision == kFP32;
            if ((g == 0) != f32) continue;
            jobs.push_back(act[i]->job);
            if (act[i]->pool_cap) {   // the whole pool, re-estimated from scratch
                ns.push_back((int64_t)(act[i]->rounds + 1) * act[i]->chunk);
                lws.push_back(act[i]->d_plw);
                fl.push_back(ILE_MARG_RESET);
            } else {
                ns.push_back(nthis[i]);
                lws.push_back(act[i]->d_lw);
                fl.push_back(act[i]->done == 0 && act[i]->rounds == 0 ? ILE_MARG_RESET : ILE_MARG_POOL);
            }
            idx.push_back(i);
        }
        if (jobs.empty()) continue;
        std::vector<ile_marg> out(jobs.size());
        if (marg_batch(s->ctx, jobs.data(), (int)jobs.size(), ns.data(), lws.data(), fl.data(), out.data(), st) !=
            ILE_OK)
            return false;
        for (size_t q = 0; q < idx.size(); q++) res[idx[q]] = out[q];
    }
    // completion and refits
    std::vector<Req *> refit;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (size_t i = 0; i < act.size(); i++) {
            Req *r = act[i];
            r->done += nthis[i];
            r->rounds += 1;
            bool fin;
            if (r->jo.adaptive) {
                const int maxr = r->jo.max_rounds > 0 ? r->jo.max_rounds : 32;
                const double tgt = r->jo.n_eff_target > 0 ? r->jo.n_eff_target : 1000.0;
                fin = res[i].n_eff >= tgt || r->rounds >= maxr;
            } else {
                fin = r->done >= r->jo.n_samples;
            }
            if (r->cancel) {
                finish(s, r, ILE_E_CANCELLED, &res[i]);
            } else if (fin) {
                finish(s, r, ILE_OK, &res[i]);
            } else if (r->jo.adaptive) {
                refit.push_back(r);
            }
        }
        s->active.erase(std::remove_if(s->active.begin(), s->active.end(), [](Req *r) { return r->state == kDone; }),
                        s->active.end());
    }
    s->cv_done.notify_all();
    // adaptive-volume jobs: refine the grid from the round just evaluated
    // (drawn with round index rounds - 1)
    {
        std::vector<AvJob> u32, u64;   // by log-weight type
        for (Req *r : refit) {
            if (r->jo.integrator != ILE_INT_AV) continue;
            AvJob aj{};
            aj.b = r->job->av;
            aj.seed = r->jo.seed;
            aj.round = (uint32_t)(r->rounds - 1);
            aj.n = r->chunk;
            aj.lw = r->d_lw;
            aj.p_thr = 0.999;
            aj.n_min_live = 1000;
            aj.max_bins = kAvMaxBins;
            (r->prob.precision == kFP32 ? u32 : u64).push_back(aj);
        }
        if (av_batch(s->ctx, true, kFP32, u32, st) != ILE_OK) return false;
        if (av_batch(s->ctx, true, kFP64, u64, st) != ILE_OK) return false;
        std::vector<AcJob> c32, c64;
        for (Req *r : refit) {
            if (r->jo.integrator != ILE_INT_AC) continue;
            AcJob cj{};
            cj.st = r->job->d_ac;
            cj.seed = r->jo.seed;
            cj.round = (uint32_t)(r->rounds - 1);
            cj.n = r->chunk;
            cj.lw = r->d_lw;
            cj.floor = 0.1;
            (r->prob.precision == kFP32 ? c32 : c64).push_back(cj);
        }
        if (ac_batch(s->ctx, true, kFP32, c32, st) != ILE_OK) return false;
        if (ac_batch(s->ctx, true, kFP64, c64, st) != ILE_OK) return false;
    }
    // one batched refit per precision policy; each job's mass draws use its
    // own key and round
    ile_gmm_opts o{};
    o.n_comp = 8;
    o.n_iter = 8;
    o.eps_def = 0.05;
    o.z_draws = 65536;
    o.temper_ess = 1.0 / 16.0;
    for (int pol = 0; pol < 3; pol++)
        for (int sh = 0; sh < 2; sh++) {
            std::vector<AdaptItem> items;
            for (Req *r : refit) {
                if (r->job->policy != pol || r->jo.integrator != ILE_INT_GMM || (r->jo.phase_shear != 0) != (sh != 0))
                    continue;
                // this round's samples (in the pool at slice rounds - 1) and their own weights
                const void *th = r->d_theta;
                int64_t ld = r->chunk;
                if (r->pool_cap) {
                    th = (const char *)r->d_pth + (size_t)(r->rounds - 1) * r->chunk * theta_bytes(pol);
                    ld = r->pool_cap;
                }
                items.push_back(AdaptItem{r->job, r->chunk, th, ld, r->d_lw, r->jo.seed ^ 0x9E3779B97F4A7C15ull,
                                          (uint32_t)r->rounds});
            }
            o.phase_shear = sh;
            if (!items.empty() && adapt_batch(s->ctx, pol, items, &o, st) != ILE_OK) return false;
        }
    return true;
}

void scheduler(ile_server *s) {
    (void)hipSetDevice(s->ctx->device);
    for (;;) {
        std::vector<Req *> act;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty() || !s->ready.empty() || !s->active.empty(); });
            if (s->stop) break;
            // cancelled jobs still in the queue
            for (auto it = s->queue.begin(); it != s->queue.end();) {
                if ((*it)->cancel) {
                    finish(s, *it, ILE_E_CANCELLED, nullptr);
                    it = s->queue.erase(it);
                } else {
                    ++it;
                }
            }
            const int maxa = max_active_of(s);
            // jobs admitted during the last pass join first (they arrived earlier)
            size_t nr = 0;
            for (; nr < s->ready.size(); nr++) {
                Req *r = s->ready[nr];
                if (r->cancel) {
                    finish(s, r, ILE_E_CANCELLED, nullptr);
                    continue;
                }
                if ((int)s->active.size() >= maxa) break;
                r->state = kActive;
                s->active.push_back(r);
            }
            s->ready.erase(s->ready.begin(), s->ready.begin() + (std::ptrdiff_t)nr);
            while (s->ready.empty() && !s->queue.empty() && (int)s->active.size() < maxa && !s->failed) {
                Req *r = s->queue.front();
                if (s->used + r->footprint > s->budget) break;   // arrival order: wait for memory
                s->queue.pop_front();
                s->used += r->footprint;
                lk.unlock();
                ile_status st = admit(s, r, s->stream);
                lk.lock();
                if (st != ILE_OK) {
                    finish(s, r, st, nullptr);
                    continue;
                }
                r->state = kActive;
                s->active.push_back(r);
            }
            act = s->active;
        }
        s->cv_done.notify_all();
        if (act.empty()) continue;
        if (!run_pass(s, act)) {
            // nothing queued may still use freed buffers
            if (s->up) (void)hipStreamSynchronize(s->up);
            (void)hipStreamSynchronize(s->stream);
            std::lock_guard<std::mutex> lk(s->mu);
            s->failed = true;
            for (Req *r : s->active) finish(s, r, ILE_E_DEVICE, nullptr);
            s->active.clear();
            for (Req *r : s->ready) finish(s, r, ILE_E_DEVICE, nullptr);
            s->ready.clear();
            for (Req *r : s->queue) finish(s, r, ILE_E_DEVICE, nullptr);
            s->queue.clear();
            s->cv_done.notify_all();
        }
    }
}

}  // namespace

extern "C" ile_status ile_server_create(ile_ctx *ctx, const ile_server_opts *opts, ile_server **out) {
    ile_status st = ctx_check(ctx);
    if (st != ILE_OK) return st;
    if (!out) return set_err(ILE_E_INVALID, "null output");
    ile_server *s = new ile_server();
    s->ctx = ctx;
    if (opts) s->opts = *opts;
    s->budget = s->opts.hbm_budget_bytes ? s->opts.hbm_budget_bytes : ctx->budget;
    hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete s;
        return dev_fail(ctx, e, "server stream");
    }
    s->th = std::thread(scheduler, s);
    *out = s;
    return ILE_OK;
}

extern "C" ile_status ile_server_submit(ile_server *s, const ile_problem *Pin, const ile_job_opts *jo,
                                        uint64_t *job_id) {
    if (!s || !Pin || !jo || !job_id) return set_err(ILE_E_INVALID, "null argument");
    // device arrays are copied to the host here (the copy below keeps host data)
    HostProblem hp;
    const ile_problem *P = nullptr;
    if (Pin->mem_is_device) {
        ile_status cs = ctx_check(s->ctx);
        if (cs != ILE_OK) return cs;
    }
    ile_status ps = problem_on_host(Pin, &hp, &P);
    if (ps != ILE_OK) return ps;
    if (P->n_det < 1 || P->n_det > 3 || P->n_modes < 1 || P->n_modes > kMaxModes || P->n_time < 4 || !P->Q ||
        !P->U || !P->mode_l || !P->mode_m || !P->det_pos || !P->det_resp)
        return set_err(ILE_E_INVALID, "bad problem shape");
    if (!jo->adaptive && jo->n_samples < 1) return set_err(ILE_E_INVALID, "n_samples must be >= 1");
    if (jo->integrator != ILE_INT_GMM && jo->integrator != ILE_INT_AV && jo->integrator != ILE_INT_AC)
        return set_err(ILE_E_INVALID, "integrator must be ILE_INT_GMM, ILE_INT_AV or ILE_INT_AC");
    if (jo->adaptive && jo->round_samples >= ((int64_t)1 << 31))
        return set_err(ILE_E_INVALID, "round_samples must be below 2^31");
    if (jo->pool != ILE_POOL_ROUNDS && jo->pool != ILE_POOL_MIXTURE)
        return set_err(ILE_E_INVALID, "pool must be ILE_POOL_ROUNDS or ILE_POOL_MIXTURE");
    if ((jo->pool == ILE_POOL_MIXTURE || jo->phase_shear) && !(jo->adaptive && jo->integrator == ILE_INT_GMM))
        return set_err(ILE_E_INVALID, "pool and phase_shear apply to adaptive mixture jobs");
    if (jo->phase_shear != 0 && jo->phase_shear != 1) return set_err(ILE_E_INVALID, "phase_shear must be 0 or 1");
    if (jo->pool == ILE_POOL_MIXTURE) {
        const int64_t rs = jo->round_samples > 0 ? jo->round_samples : 65536;
        const int64_t mr = jo->max_rounds > 0 ? jo->max_rounds : 32;
        if (mr * rs > ((int64_t)1 << 28))
            return set_err(ILE_E_INVALID, "a mixture pool holds at most 2^28 samples (max_rounds x round_samples)");
    }
    if (jo->tmarg_oversample != 0) {
        if (jo->tmarg_oversample != 1 && jo->tmarg_oversample != 4)
            return set_err(ILE_E_INVALID, "tmarg_oversample must be 0, 1 or 4");
        if (jo->adaptive || (P->precision != ILE_FP32 && P->precision != ILE_FP64))
            return set_err(ILE_E_INVALID, "time-marginalised jobs are plain FP32/FP64 jobs");
    }
    auto r = std::make_unique<Req>();
    const int K = P->n_det, n = P->n_modes, T = P->n_time;
    r->ml.assign(P->mode_l, P->mode_l + n);
    r->mm.assign(P->mode_m, P->mode_m + n);
    r->pos.assign(P->det_pos, P->det_pos + 3 * K);
    r->resp.assign(P->det_resp, P->det_resp + 9 * K);
    r->Q.assign(P->Q, P->Q + (size_t)K * n * T * 2);
    r->U.assign(P->U, P->U + (size_t)K * n * n * 2);
    if (P->V) r->V.assign(P->V, P->V + (size_t)K * n * n * 2);
    r->prob = *P;
    r->prob.mode_l = r->ml.data();
    r->prob.mode_m = r->mm.data();
    r->prob.det_pos = r->pos.data();
    r->prob.det_resp = r->resp.data();
    r->prob.Q = r->Q.data();
    r->prob.U = r->U.data();
    r->prob.V = P->V ? r->V.data() : nullptr;
    r->jo = *jo;
    r->footprint = footprint_of(s, r.get());
    if (r->footprint > s->budget) return set_err(ILE_E_TOO_BIG, "job footprint exceeds the server budget");
    r->res.t_arrival_ns = now_ns();
    r->res.status = ILE_PENDING;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->failed) return set_err(ILE_E_DEVICE, "server failed after a device error");
    r->id = s->next_id++;
    *job_id = r->id;
    s->queue.push_back(r.get());
    s->all[r->id] = std::move(r);
    s->cv_work.notify_one();
    return ILE_OK;
}

extern "C" ile_status ile_server_poll(ile_server *s, uint64_t id, ile_result *out) {
    if (!s || !out) return set_err(ILE_E_INVALID, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(id);
    if (it == s->all.end()) return set_err(ILE_E_INVALID, "unknown job id");
    *out = it->second->res;
    return it->second->state == kDone ? ILE_OK : ILE_PENDING;
}

extern "C" ile_status ile_server_wait(ile_server *s, uint64_t id, int64_t timeout_ms, ile_result *out) {
    if (!s || !out) return set_err(ILE_E_INVALID, "null argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(id);
    if (it == s->all.end()) return set_err(ILE_E_INVALID, "unknown job id");
    Req *r = it->second.get();
    auto pred = [&] { return r->state == kDone; };
    if (timeout_ms < 0) {
        s->cv_done.wait(lk, pred);
    } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred)) {
        *out = r->res;
        return set_err(ILE_E_TIMEOUT, "wait timed out");
    }
    *out = r->res;
    return ILE_OK;
}

extern "C" ile_status ile_server_cancel(ile_server *s, uint64_t id) {
    if (!s) return set_err(ILE_E_INVALID, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(id);
    if (it == s->all.end()) return set_err(ILE_E_INVALID, "unknown job id");
    it->second->cancel = true;
    s->cv_work.notify_one();
    return ILE_OK;
}

extern "C" ile_status ile_server_stats(ile_server *s, int64_t *active, int64_t *queued, int64_t *done) {
    if (!s) return set_err(ILE_E_INVALID, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    if (active) *active = (int64_t)(s->active.size() + s->ready.size());
    if (queued) *queued = (int64_t)s->queue.size();
    if (done) *done = s->n_done;
    return ILE_OK;
}

extern "C" void ile_server_destroy(ile_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (Req *r : s->queue) r->cancel = true;
        for (Req *r : s->ready) r->cancel = true;
        for (Req *r : s->active) r->cancel = true;
    }
    s->cv_work.notify_all();
    if (s->th.joinable()) s->th.join();
    (void)hipSetDevice(s->ctx->device);
    if (s->up) (void)hipStreamSynchronize(s->up);
    (void)hipStreamSynchronize(s->stream);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (Req *r : s->active) finish(s, r, ILE_E_CANCELLED, nullptr);
        for (Req *r : s->ready) finish(s, r, ILE_E_CANCELLED, nullptr);
        for (Req *r : s->queue) finish(s, r, ILE_E_CANCELLED, nullptr);
        s->active.clear();
        s->ready.clear();
        s->queue.clear();
    }
    s->cv_done.notify_all();
    if (s->up_ev) (void)hipEventDestroy(s->up_ev);
    if (s->up) (void)hipStreamDestroy(s->up);
    (void)hipStreamDestroy(s->stream);
    delete s;
}
