// Host side of the C ABI declared in include/ile.h: validation, mode
// filtering and placement, precision conversion and layout, residency,
// launches and result read-back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "ile.h"
#include "ile_ctx.h"
#include "ile_internal.h"

using namespace ile;

namespace {
thread_local std::string g_err;
}

namespace ile {

ile_status set_err(ile_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

ile_status dev_fail(ile_ctx *ctx, hipError_t e, const char *what) {
    if (ctx) ctx->sticky = true;
    char buf[512];
    snprintf(buf, sizeof buf, "HIP error in %s: %s", what, hipGetErrorString(e));
    g_err = buf;
    return ILE_E_DEVICE;
}

size_t eval_lds_limit() {
    static size_t lim = 0;
    if (lim == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
            lim = (size_t)v;
        else
            lim = 65536;
    }
    return lim;
}

hipError_t launch_eval(int set, int kdet, int policy, bool dm, size_t lds_bytes, const EvalJob *d_jobs,
                       const Tile *d_tiles, int n_tiles, int block, hipStream_t st) {
#define ILE_SP(S)                                                                                            \
    if (set == S) {                                                                                          \
        if (policy == 0) return launch_eval_sp<S, 0>(kdet, dm, lds_bytes, d_jobs, d_tiles, n_tiles, block, st); \
        if (policy == 1) return launch_eval_sp<S, 1>(kdet, dm, lds_bytes, d_jobs, d_tiles, n_tiles, block, st); \
        if (policy == 2) return dm ? hipErrorInvalidValue                                                 \
                                   : launch_ref_sp<S>(kdet, lds_bytes, d_jobs, d_tiles, n_tiles, block, st); \
    }
    ILE_SP(0)
    ILE_SP(1)
    ILE_SP(2)
    ILE_SP(3)
#undef ILE_SP
    return hipErrorInvalidValue;
}

hipError_t launch_tmarg(int set, int kdet, int policy, int R, bool dm, size_t lds_bytes, const EvalJob *d_jobs,
                        const Tile *d_tiles, int n_tiles, int block, hipStream_t st) {
#define ILE_TM(S)                                                                                             \
    if (set == S) {                                                                                           \
        if (policy == 0) return launch_tmarg_sp<S, 0>(kdet, R, dm, lds_bytes, d_jobs, d_tiles, n_tiles, block, st); \
        if (policy == 1) return launch_tmarg_sp<S, 1>(kdet, R, dm, lds_bytes, d_jobs, d_tiles, n_tiles, block, st); \
    }
    ILE_TM(0)
    ILE_TM(1)
    ILE_TM(2)
    ILE_TM(3)
#undef ILE_TM
    return hipErrorInvalidValue;
}

// Contraction element size of a policy (Q, U, V storage).
// (FP32 windows in the FP32 + FP64-cancellation policy as well)
static size_t creal_size(int policy) { return policy == kFP64 ? sizeof(double) : sizeof(float); }
size_t theta_size(int policy) { return policy == kFP64 ? sizeof(double) : sizeof(float); }
size_t out_size(int policy) { return policy == kFP32 ? sizeof(float) : sizeof(double); }

// Detectors of a job read through L1/L2 by the LDS-staged kernel (the same
// rule as the kernels' instantiation), the bytes of the other detectors'
// windows that it stages, and whether such a kernel exists for the job and
// its staged part fits the device.
static int job_global_dets(const ile_job *job, bool tmarg) {
    return tmarg ? tmarg_global_dets(job->set, job->kp, job->policy)
                 : lds_global_dets(job->set, job->kp, job->policy);
}
size_t job_window_bytes(const ile_job *job, bool tmarg) {
    const int staged = job->kp - job_global_dets(job, tmarg);
    const size_t series = job->policy == kMixed ? (size_t)job->kp * job->n_time * sizeof(double) : 0;
    return (size_t)std::max(staged, 0) * job->n_time * kSets[job->set].n * 2 * creal_size(job->policy) + series;
}
bool job_lds_ok(const ile_job *job, bool tmarg) {
    const bool compiled = tmarg ? tmarg_lds_compiled(job->set, job->kp, job->policy)
                                : lnl_lds_compiled(job->set, job->kp, job->policy);
    return compiled && job_window_bytes(job, tmarg) <= eval_lds_limit();
}

// Launch geometry of one eval over n samples of a job (single-job path).
void eval_geometry(const ile_job *job, int64_t n, size_t *lds, int64_t *tile, int *block) {
    const size_t win = job_window_bytes(job, false);
    const int64_t cus = 256;
    // stage the window in LDS only when each block gets enough samples to pay for it
    if (job_lds_ok(job, false) && n >= (int64_t)2 * cus * 16384) {
        *lds = win;
        *block = lds_block_threads(job->set, job->policy);
        *tile = std::max<int64_t>(16384, (n + 2 * cus - 1) / (2 * cus));
    } else {
        *lds = 0;
        *block = 256;
        int64_t t = (n + 4 * cus - 1) / (4 * cus);
        t = ((t + 255) / 256) * 256;
        *tile = std::min<int64_t>(std::max<int64_t>(t, 256), 8192);
    }
}

ile_status ctx_check(ile_ctx *ctx) {
    if (!ctx) return set_err(ILE_E_INVALID, "null context");
    if (ctx->sticky) return set_err(ILE_E_DEVICE, "context is in a failed state after an earlier device error");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return dev_fail(ctx, e, "hipSetDevice");
    return ILE_OK;
}

// Power-of-two size class (at least 4 KiB) of a request.
static size_t size_class(size_t bytes) {
    size_t c = 4096;
    while (c < bytes) c <<= 1;
    return c;
}

// Return every cached buffer to the runtime (caller holds ctx->mu).
static void pool_trim_locked(ile_ctx *ctx) {
    for (auto &kv : ctx->dev_pool)
        for (void *q : kv.second) {
            (void)hipFree(q);
            ctx->used -= kv.first;
        }
    ctx->dev_pool.clear();
    ctx->pool_cached = 0;
}

// Device allocation through the context's pool.  The budget counts a buffer
// from its first allocation until the pool is trimmed (cached buffers stay
// counted, and are trimmed when a new class would not fit).
ile_status ctx_alloc(ile_ctx *ctx, void **p, size_t bytes, const char *what) {
    *p = nullptr;
    if (bytes == 0) return ILE_OK;
    const size_t cls = size_class(bytes);
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto it = ctx->dev_pool.find(cls);
        if (it != ctx->dev_pool.end() && !it->second.empty()) {
            *p = it->second.back();
            it->second.pop_back();
            ctx->pool_cached -= cls;
            return ILE_OK;
        }
        if (ctx->budget && ctx->used + cls > ctx->budget) pool_trim_locked(ctx);
        if (ctx->budget && ctx->used + cls > ctx->budget)
            return set_err(ILE_E_TOO_BIG, std::string("device budget exceeded allocating ") + what);
        ctx->used += cls;
    }
    hipError_t e = hipMalloc(p, cls);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        std::lock_guard<std::mutex> lk(ctx->mu);
        pool_trim_locked(ctx);
        e = hipMalloc(p, cls);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            ctx->used -= cls;
            *p = nullptr;
            return set_err(ILE_E_NOMEM, std::string("hipMalloc failed for ") + what);
        }
    }
    return ILE_OK;
}

// Back to the pool; the caller guarantees no queued work still uses it.
void ctx_free(ile_ctx *ctx, void *p, size_t bytes) {
    if (!p) return;
    const size_t cls = size_class(bytes);
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->dev_pool[cls].push_back(p);
    ctx->pool_cached += cls;
}

void *pin_alloc(ile_ctx *ctx, size_t bytes) {
    const size_t cls = size_class(bytes);
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto it = ctx->pin_pool.find(cls);
        if (it != ctx->pin_pool.end() && !it->second.empty()) {
            void *p = it->second.back();
            it->second.pop_back();
            return p;
        }
    }
    void *p = nullptr;
    if (hipHostMalloc(&p, cls, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void pin_free(ile_ctx *ctx, void *p, size_t bytes) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->pin_pool[size_class(bytes)].push_back(p);
}

void ctx_pool_release(ile_ctx *ctx) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    pool_trim_locked(ctx);
    for (auto &kv : ctx->pin_pool)
        for (void *q : kv.second) (void)hipHostFree(q);
    ctx->pin_pool.clear();
}

// Distance table shared by every job of a context with the same prior.
ile_status ctx_dist_table(ile_ctx *ctx, const PriorDev &pr, DistTable *out, hipStream_t st) {
    std::lock_guard<std::mutex> lk(ctx->dist_mu);
    auto key = std::make_tuple(pr.d_min, pr.d_max, pr.d_ref);
    auto it = ctx->dist.find(key);
    if (it != ctx->dist.end()) {
        *out = it->second.tab;
        return ILE_OK;
    }
    void *buf = nullptr;
    ile_status s = ctx_alloc(ctx, &buf, dist_table_bytes(), "distance table");
    if (s != ILE_OK) return s;
    DistTable tb{};
    hipError_t e = build_dist_table(&tb, (double *)buf, pr, st);
    if (e != hipSuccess) return dev_fail(ctx, e, "build_dist_table");
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return dev_fail(ctx, e, "distance table build");
    ctx->dist[key] = ile_ctx::DistEntry{tb, buf};
    *out = tb;
    return ILE_OK;
}

}  // namespace ile

// ===================================================================== context
extern "C" ile_status ile_ctx_create(int hip_device, size_t hbm_budget_bytes, ile_ctx **out) {
    if (!out) return set_err(ILE_E_INVALID, "null output pointer");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) return set_err(ILE_E_DEVICE, "no HIP device available");
    if (hip_device < 0 || hip_device >= n) return set_err(ILE_E_INVALID, "device index out of range");
    e = hipSetDevice(hip_device);
    if (e != hipSuccess) return dev_fail(nullptr, e, "hipSetDevice");
    // this device's copy of the no-alloc estimator's scratch array
    ile_status sc = noalloc_init_device(hip_device);
    if (sc != ILE_OK) return sc;
    ile_ctx *c = new ile_ctx();
    c->device = hip_device;
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) == hipSuccess && hbm_budget_bytes == 0) hbm_budget_bytes = tot;
    c->budget = hbm_budget_bytes;
    *out = c;
    return ILE_OK;
}

extern "C" void ile_ctx_destroy(ile_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto &kv : ctx->dist) (void)hipFree(kv.second.buf);
    for (auto &sl : ctx->slots) {
        if (sl.d) (void)hipFree(sl.d);
        if (sl.h) (void)hipHostFree(sl.h);
        if (sl.ev) (void)hipEventDestroy(sl.ev);
    }
    ctx_pool_release(ctx);
    delete ctx;
}

extern "C" const char *ile_last_error(void) { return g_err.c_str(); }

// ===================================================================== prepare
namespace {

int set_slot(int set, int l, int m) {
    for (int a = 0; a < kSets[set].n; a++)
        if (kSets[set].l[a] == l && kSets[set].m[a] == m) return a;
    return -1;
}

template <class R>
void fill_tables(const ile_problem *P, const std::vector<int> &keep, const std::vector<int> &slot, int set, int kp,
                 std::vector<R> &Qh, std::vector<R> &Uh, std::vector<R> &Vh) {
    using cd = std::complex<double>;
    const int NM = kSets[set].n, T = P->n_time, K = P->n_det, n = P->n_modes;
    const PairTable pt = make_pairs(set);
    Qh.assign((size_t)kp * T * NM * 2, R(0));
    for (int k = 0; k < K; k++)
        for (size_t q = 0; q < keep.size(); q++) {
            const int a = keep[q], s = slot[q];
            for (int i = 0; i < T; i++) {
                const double *src = P->Q + 2 * (((size_t)k * n + a) * T + i);
                R *dst = &Qh[2 * (((size_t)k * T + i) * NM + s)];
                dst[0] = (R)src[0];
                dst[1] = (R)src[1];
            }
        }
    // user mode of each slot (-1: empty)
    std::vector<int> user(NM, -1);
    for (size_t q = 0; q < keep.size(); q++) user[slot[q]] = keep[q];
    auto U = [&](int k, int a, int b) {
        const double *p = P->U + 2 * (((size_t)k * n + a) * n + b);
        return cd(p[0], p[1]);
    };
    auto V = [&](int k, int a, int b) {
        if (!P->V) return cd(0, 0);
        const double *p = P->V + 2 * (((size_t)k * n + a) * n + b);
        return cd(p[0], p[1]);
    };
    Uh.assign((size_t)pt.P * kp * 2, R(0));
    Vh.assign((size_t)pt.P * kp * 2, R(0));
    for (int j = 0; j < pt.P; j++) {
        // U-order entry j
        {
            const int p = pt.u_pair[j], sa = pt.a[p], sb = pt.b[p];
            const int ua = user[sa], ub = user[sb];
            if (ua >= 0 && ub >= 0)
                for (int k = 0; k < K; k++) {
                    cd h = 0.5 * (U(k, ua, ub) + std::conj(U(k, ub, ua)));  // Hermitian part
                    if (sa != sb) {
                        h *= 2.0;
                        if (kSets[set].m[sa] < kSets[set].m[sb]) h = std::conj(h);
                    } else {
                        h = cd(h.real(), 0.0);
                    }
                    Uh[2 * ((size_t)j * kp + k)] = (R)h.real();
                    Uh[2 * ((size_t)j * kp + k) + 1] = (R)h.imag();
                }
        }
        {
            const int p = pt.v_pair[j], sa = pt.a[p], sb = pt.b[p];
            const int ua = user[sa], ub = user[sb];
            if (ua >= 0 && ub >= 0)
                for (int k = 0; k < K; k++) {
                    cd v = 0.5 * (V(k, ua, ub) + V(k, ub, ua));  // symmetric part
                    if (sa != sb) v *= 2.0;
                    Vh[2 * ((size_t)j * kp + k)] = (R)v.real();
                    Vh[2 * ((size_t)j * kp + k) + 1] = (R)v.imag();
                }
        }
    }
}

// FP32 + FP64-cancellation policy: U and V as full [kp][NM][NM] complex FP64
// matrices in slot order (Hermitian / symmetric parts), and the pair weights
// of the offset form, [kp][P] x (Ur + Vr, Ur - Vr, -Ui - Vi, Ui - Vi), doubled
// off the diagonal, pairs a <= b in their plain order.
void fill_mixed(const ile_problem *P, const std::vector<int> &keep, const std::vector<int> &slot, int set, int kp,
                std::vector<double> &U64, std::vector<double> &V64, std::vector<float> &W) {
    using cd = std::complex<double>;
    const int NM = kSets[set].n, K = P->n_det, n = P->n_modes;
    const PairTable pt = make_pairs(set);
    std::vector<int> user(NM, -1);
    for (size_t q = 0; q < keep.size(); q++) user[slot[q]] = keep[q];
    auto U = [&](int k, int a, int b) {
        const double *p = P->U + 2 * (((size_t)k * n + a) * n + b);
        return cd(p[0], p[1]);
    };
    auto V = [&](int k, int a, int b) {
        if (!P->V) return cd(0, 0);
        const double *p = P->V + 2 * (((size_t)k * n + a) * n + b);
        return cd(p[0], p[1]);
    };
    U64.assign((size_t)kp * NM * NM * 2, 0.0);
    V64.assign((size_t)kp * NM * NM * 2, 0.0);
    for (int k = 0; k < K; k++)
        for (int sa = 0; sa < NM; sa++)
            for (int sb = 0; sb < NM; sb++) {
                const int ua = user[sa], ub = user[sb];
                if (ua < 0 || ub < 0) continue;
                cd h = 0.5 * (U(k, ua, ub) + std::conj(U(k, ub, ua)));
                if (sa == sb) h = cd(h.real(), 0.0);
                const cd v = 0.5 * (V(k, ua, ub) + V(k, ub, ua));
                const size_t o = 2 * (((size_t)k * NM + sa) * NM + sb);
                U64[o] = h.real();
                U64[o + 1] = h.imag();
                V64[o] = v.real();
                V64[o + 1] = v.imag();
            }
    // The quadratic form over the real vector v = (dr_0, di_0, dr_1, di_1, ...)
    // of the amplitude offsets, per detector: the upper triangle (row by row)
    // of M with M_ii the diagonal and M_ij = 2 S_ij (i < j), S the symmetric
    // matrix of delta^+ U delta + Re(delta^T V delta).  Per pair a <= b
    // (weight f = 2 off the diagonal, 1 on it) the coefficients of
    // (dr_a dr_b, di_a di_b, dr_a di_b, di_a dr_b) are
    // f (Ur + Vr, Ur - Vr, -Ui - Vi, Ui - Vi).
    const int NV = 2 * NM, NT = NV * (NV + 1) / 2;
    auto tri = [&](int i, int j) { return (size_t)(i * (2 * NV - i + 1)) / 2 + (size_t)(j - i); };
    W.assign((size_t)kp * NT, 0.0f);
    std::vector<double> Mk((size_t)NT);
    for (int k = 0; k < K; k++) {
        std::fill(Mk.begin(), Mk.end(), 0.0);
        for (int p = 0; p < pt.P; p++) {
            const int sa = pt.a[p], sb = pt.b[p];
            const size_t o = 2 * (((size_t)k * NM + sa) * NM + sb);
            const double ur = U64[o], ui = U64[o + 1], vr = V64[o], vi = V64[o + 1];
            const double f = sa == sb ? 1.0 : 2.0;
            Mk[tri(2 * sa, 2 * sb)] += f * (ur + vr);
            Mk[tri(2 * sa + 1, 2 * sb + 1)] += f * (ur - vr);
            Mk[tri(2 * sa, 2 * sb + 1)] += f * (-ui - vi);
            if (sa < sb)
                Mk[tri(2 * sa + 1, 2 * sb)] += f * (ui - vi);
            else
                Mk[tri(2 * sa, 2 * sa + 1)] += f * (ui - vi);   // di_a dr_a = dr_a di_a
        }
        for (int t = 0; t < NT; t++) W[(size_t)k * NT + t] = (float)Mk[t];
    }
}

}  // namespace

ile_status ile::problem_on_host(const ile_problem *P, HostProblem *out, const ile_problem **use) {
    *use = P;
    if (!P || !P->mem_is_device) return ILE_OK;
    const int K = P->n_det, n = P->n_modes, T = P->n_time;
    if (K < 1 || K > 3 || n < 1 || n > kMaxModes || T < 4) return set_err(ILE_E_INVALID, "bad shapes");
    if (!P->mode_l || !P->mode_m || !P->det_pos || !P->det_resp || !P->Q || !P->U)
        return set_err(ILE_E_INVALID, "null input array");
    out->ml.resize(n);
    out->mm.resize(n);
    out->pos.resize(3 * (size_t)K);
    out->resp.resize(9 * (size_t)K);
    out->Q.resize((size_t)K * n * T * 2);
    out->U.resize((size_t)K * n * n * 2);
    if (P->V) out->V.resize((size_t)K * n * n * 2);
    auto cp = [](void *dst, const void *src, size_t bytes) {
        return hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost);
    };
    hipError_t e = cp(out->ml.data(), P->mode_l, n * sizeof(int32_t));
    if (e == hipSuccess) e = cp(out->mm.data(), P->mode_m, n * sizeof(int32_t));
    if (e == hipSuccess) e = cp(out->pos.data(), P->det_pos, out->pos.size() * sizeof(double));
    if (e == hipSuccess) e = cp(out->resp.data(), P->det_resp, out->resp.size() * sizeof(double));
    if (e == hipSuccess) e = cp(out->Q.data(), P->Q, out->Q.size() * sizeof(double));
    if (e == hipSuccess) e = cp(out->U.data(), P->U, out->U.size() * sizeof(double));
    if (e == hipSuccess && P->V) e = cp(out->V.data(), P->V, out->V.size() * sizeof(double));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_err(ILE_E_INVALID, std::string("copying device inputs: ") + hipGetErrorString(e));
    }
    out->p = *P;
    out->p.mem_is_device = 0;
    out->p.mode_l = out->ml.data();
    out->p.mode_m = out->mm.data();
    out->p.det_pos = out->pos.data();
    out->p.det_resp = out->resp.data();
    out->p.Q = out->Q.data();
    out->p.U = out->U.data();
    out->p.V = P->V ? out->V.data() : nullptr;
    *use = &out->p;
    return ILE_OK;
}

extern "C" ile_status ile_prepare(ile_ctx *ctx, const ile_problem *P, ile_job **out) {
    ile_status s = ctx_check(ctx);
    if (s != ILE_OK) return s;
    HostProblem hp;
    const ile_problem *use = nullptr;
    if ((s = problem_on_host(P, &hp, &use)) != ILE_OK) return s;
    return job_create(ctx, use, out, nullptr, false);
}

ile_status ile::job_create(ile_ctx *ctx, const ile_problem *P, ile_job **out, hipStream_t st, bool async) {
    ile_status s = ctx_check(ctx);
    if (s != ILE_OK) return s;
    if (!out || !P) return set_err(ILE_E_INVALID, "null argument");
    *out = nullptr;
    const int K = P->n_det, n = P->n_modes, T = P->n_time;
    if (K < 1 || K > 3) return set_err(ILE_E_INVALID, "n_det must be 1..3");
    if (n < 1 || n > kMaxModes) return set_err(ILE_E_INVALID, "n_modes must be 1..21");
    if (T < 4) return set_err(ILE_E_INVALID, "n_time must be >= 4");
    if (!P->mode_l || !P->mode_m || !P->det_pos || !P->det_resp || !P->Q || !P->U)
        return set_err(ILE_E_INVALID, "null input array");
    if (P->precision < 0 || P->precision > 2) return set_err(ILE_E_INVALID, "unknown precision policy");
    if (P->precision == kMixed && P->prior.dist_marg)
        return set_err(ILE_E_INVALID, "the distance table is not available with ILE_FP32_CANCEL64");
    if (!(P->dt_s > 0) || !std::isfinite(P->tau0_s) || !std::isfinite(P->gmst_rad))
        return set_err(ILE_E_INVALID, "bad window or gmst");
    if (!(P->d_ref_mpc > 0)) return set_err(ILE_E_INVALID, "d_ref must be > 0");
    if (!(P->prior.t_window > 0) || !(P->prior.d_min > 0) || !(P->prior.d_max > P->prior.d_min))
        return set_err(ILE_E_INVALID, "bad prior ranges");
    if (!(P->mode_filter_eps >= 0)) return set_err(ILE_E_INVALID, "mode_filter_eps must be >= 0");
    for (int a = 0; a < n; a++) {
        const int l = P->mode_l[a], m = P->mode_m[a];
        if (l < 2 || l > 4 || m < -l || m > l) return set_err(ILE_E_INVALID, "mode (l,m) outside l=2..4, |m|<=l");
        for (int b = 0; b < a; b++)
            if (P->mode_l[b] == l && P->mode_m[b] == m) return set_err(ILE_E_INVALID, "duplicate mode");
    }
    // finiteness and symmetry of the inputs
    const size_t nq = (size_t)K * n * T * 2, nu = (size_t)K * n * n * 2;
    for (size_t i = 0; i < nq; i++)
        if (!std::isfinite(P->Q[i])) return set_err(ILE_E_INVALID, "non-finite Q");
    double umax = 0.0, vmax = 0.0;
    for (size_t i = 0; i < nu; i++) {
        if (!std::isfinite(P->U[i]) || (P->V && !std::isfinite(P->V[i]))) return set_err(ILE_E_INVALID, "non-finite U or V");
        umax = std::max(umax, std::fabs(P->U[i]));
        if (P->V) vmax = std::max(vmax, std::fabs(P->V[i]));
    }
    for (int k = 0; k < K; k++)
        for (int a = 0; a < n; a++)
            for (int b = 0; b < n; b++) {
                const double *u1 = P->U + 2 * (((size_t)k * n + a) * n + b);
                const double *u2 = P->U + 2 * (((size_t)k * n + b) * n + a);
                if (std::fabs(u1[0] - u2[0]) > 1e-9 * umax || std::fabs(u1[1] + u2[1]) > 1e-9 * umax)
                    return set_err(ILE_E_INVALID, "U is not Hermitian");
                if (P->V) {
                    const double *v1 = P->V + 2 * (((size_t)k * n + a) * n + b);
                    const double *v2 = P->V + 2 * (((size_t)k * n + b) * n + a);
                    if (std::fabs(v1[0] - v2[0]) > 1e-9 * vmax || std::fabs(v1[1] - v2[1]) > 1e-9 * vmax)
                        return set_err(ILE_E_INVALID, "V is not symmetric");
                }
            }
    if (!P->V) {
        bool pos = false, neg = false;
        for (int a = 0; a < n; a++) {
            pos = pos || P->mode_m[a] > 0;
            neg = neg || P->mode_m[a] < 0;
        }
        if (pos && neg) return set_err(ILE_E_INVALID, "V may be NULL only if all m share a sign");
    }
    for (int k = 0; k < K; k++)
        for (int c = 0; c < 3; c++)
            if (!std::isfinite(P->det_pos[3 * k + c])) return set_err(ILE_E_INVALID, "non-finite detector position");
    for (int i = 0; i < 9 * K; i++)
        if (!std::isfinite(P->det_resp[i])) return set_err(ILE_E_INVALID, "non-finite detector response");

    // mode filter: keep (l,m) iff some |U_0[lm][l'm'] / U_0[22][22]| > eps (detector 0)
    std::vector<int> keep;
    if (P->mode_filter_eps > 0) {
        int a22 = -1;
        for (int a = 0; a < n; a++)
            if (P->mode_l[a] == 2 && P->mode_m[a] == 2) a22 = a;
        if (a22 < 0) return set_err(ILE_E_INVALID, "mode filter needs the (2,2) mode");
        const double *u22 = P->U + 2 * ((size_t)a22 * n + a22);
        const double ref = std::hypot(u22[0], u22[1]);
        if (!(ref > 0)) return set_err(ILE_E_INVALID, "mode filter needs U_22,22 > 0");
        for (int a = 0; a < n; a++) {
            double mx = 0.0;
            for (int b = 0; b < n; b++) {
                const double *u = P->U + 2 * ((size_t)a * n + b);
                mx = std::max(mx, std::hypot(u[0], u[1]) / ref);
            }
            if (mx > P->mode_filter_eps) keep.push_back(a);
        }
    } else {
        for (int a = 0; a < n; a++) keep.push_back(a);
    }
    // smallest compiled set containing every kept mode
    int set = -1;
    std::vector<int> slot(keep.size());
    for (int sidx = 0; sidx < kNumSets && set < 0; sidx++) {
        bool all = true;
        for (size_t q = 0; q < keep.size() && all; q++) {
            slot[q] = set_slot(sidx, P->mode_l[keep[q]], P->mode_m[keep[q]]);
            all = slot[q] >= 0;
        }
        if (all) set = sidx;
    }
    if (set < 0) return set_err(ILE_E_INVALID, "mode list not representable");
    const int kp = K == 1 ? 2 : K;

    ile_job *job = new ile_job();
    job->ctx = ctx;
    job->policy = P->precision;
    job->set = set;
    job->kp = kp;
    job->n_det = K;
    job->n_time = T;
    job->n_kept = (int)keep.size();
    job->dist_marg = P->prior.dist_marg != 0;
    job->pr = PriorDev{P->prior.t_window, P->prior.d_min, P->prior.d_max, P->d_ref_mpc, job->dist_marg ? 1 : 0};

    std::vector<char> Qb, Ub, Vb;
    std::vector<double> q64, u64, v64;   // mixed policy: the reference builder's inputs
    if (job->policy == kFP32) {
        std::vector<float> q, u, v;
        fill_tables<float>(P, keep, slot, set, kp, q, u, v);
        Qb.assign((char *)q.data(), (char *)(q.data() + q.size()));
        Ub.assign((char *)u.data(), (char *)(u.data() + u.size()));
        Vb.assign((char *)v.data(), (char *)(v.data() + v.size()));
    } else if (job->policy == kMixed) {
        // FP32 window and offset-form pair weights for the kernel; FP64
        // window and overlaps for the reference builder
        std::vector<float> q, u, v, w;
        fill_tables<float>(P, keep, slot, set, kp, q, u, v);
        std::vector<double> ud, vd;
        fill_tables<double>(P, keep, slot, set, kp, q64, ud, vd);
        fill_mixed(P, keep, slot, set, kp, u64, v64, w);
        Qb.assign((char *)q.data(), (char *)(q.data() + q.size()));
        Ub.assign((char *)w.data(), (char *)(w.data() + w.size()));
    } else {
        std::vector<double> q, u, v;
        fill_tables<double>(P, keep, slot, set, kp, q, u, v);
        Qb.assign((char *)q.data(), (char *)(q.data() + q.size()));
        Ub.assign((char *)u.data(), (char *)(u.data() + u.size()));
        Vb.assign((char *)v.data(), (char *)(v.data() + v.size()));
    }
    job->q_bytes = Qb.size();
    job->uv_bytes = Ub.size();
    auto cleanup = [&](ile_status stt) {
        job_release_nosync(job);
        return stt;
    };
    // one blob [Q | U table | V table | estimator state], 256-byte aligned parts
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t oQ = 0, oU = al(Qb.size()), oV = oU + al(Ub.size()), oM = oV + al(Vb.size());
    // mixed policy: [FP64 window | U | V | r, G (FP32) | R series | C0 | reference point]
    const int NMs = kSets[set].n;
    const size_t rg_bytes = job->policy == kMixed ? (size_t)2 * kp * NMs * 2 * sizeof(float) : 0;
    const size_t R_bytes = job->policy == kMixed ? (size_t)kp * T * sizeof(double) : 0;
    const size_t oQ64 = oM + al(sizeof(MargState)), oU64 = oQ64 + al(q64.size() * 8), oV64 = oU64 + al(u64.size() * 8);
    const size_t org = oV64 + al(v64.size() * 8), oR = org + al(rg_bytes), oC0 = oR + al(R_bytes);
    const size_t oTh = oC0 + (job->policy == kMixed ? 256 : 0);
    job->blob_bytes = job->policy == kMixed ? oTh + al(7 * sizeof(double)) : oM + al(sizeof(MargState));
    if ((s = ctx_alloc(ctx, &job->d_blob, job->blob_bytes, "job inputs")) != ILE_OK) return cleanup(s);
    job->h_blob = pin_alloc(ctx, job->blob_bytes);
    job->h_ms = (MargState *)pin_alloc(ctx, sizeof(MargState));
    if (!job->h_blob || !job->h_ms) return cleanup(set_err(ILE_E_NOMEM, "pinned staging"));
    char *hb = (char *)job->h_blob;
    std::memset(hb, 0, job->blob_bytes);      // mixed: no reference until one is set (r = 0)
    std::memcpy(hb + oQ, Qb.data(), Qb.size());
    std::memcpy(hb + oU, Ub.data(), Ub.size());
    std::memcpy(hb + oV, Vb.data(), Vb.size());
    const MargState ms0{-INFINITY, 0.0, 0.0, 0, 0, -1};
    std::memcpy(hb + oM, &ms0, sizeof ms0);
    if (job->policy == kMixed) {
        std::memcpy(hb + oQ64, q64.data(), q64.size() * 8);
        std::memcpy(hb + oU64, u64.data(), u64.size() * 8);
        std::memcpy(hb + oV64, v64.data(), v64.size() * 8);
        char *db = (char *)job->d_blob;
        job->rb.theta_ref = (const double *)(db + oTh);
        job->rb.Q64 = (const double *)(db + oQ64);
        job->rb.U64 = (const double *)(db + oU64);
        job->rb.V64 = (const double *)(db + oV64);
        job->rb.rg = (float *)(db + org);
        job->rb.R = (double *)(db + oR);
        job->rb.C0 = (double *)(db + oC0);
        job->h_ref = (double *)pin_alloc(ctx, 7 * sizeof(double));
        if (!job->h_ref) return cleanup(set_err(ILE_E_NOMEM, "pinned staging"));
    }
    job->d_Q = (char *)job->d_blob + oQ;
    job->d_Ut = (char *)job->d_blob + oU;
    job->d_Vt = (char *)job->d_blob + oV;
    job->d_ms = (MargState *)((char *)job->d_blob + oM);
    hipError_t e = hipMemcpyAsync(job->d_blob, job->h_blob, job->blob_bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !async) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return cleanup(dev_fail(ctx, e, "upload job inputs"));

    EvalJob &ej = job->ej;
    std::memset(&ej, 0, sizeof ej);
    ej.Q = job->d_Q;
    ej.Ut = job->d_Ut;
    ej.Vt = job->d_Vt;
    ej.ref_rg = job->rb.rg;
    ej.ref_R = job->rb.R;
    ej.ref_C0 = job->rb.C0;
    ej.tau0 = P->tau0_s;
    ej.inv_dt = 1.0 / P->dt_s;
    ej.gmst = P->gmst_rad;
    ej.d_ref = P->d_ref_mpc;
    ej.n_time = T;
    const double c_si = 299792458.0;
    for (int k = 0; k < kp; k++) {
        const int ks = k < K ? k : 0;      // padded detector: same position, zero response
        for (int c = 0; c < 3; c++) ej.xc[k][c] = P->det_pos[3 * ks + c] / c_si;
        const double *d = P->det_resp + 9 * ks;
        const double f = k < K ? 1.0 : 0.0;
        ej.D[k][0] = f * d[0];
        ej.D[k][1] = f * d[4];
        ej.D[k][2] = f * d[8];
        ej.D[k][3] = f * 0.5 * (d[1] + d[3]);
        ej.D[k][4] = f * 0.5 * (d[2] + d[6]);
        ej.D[k][5] = f * 0.5 * (d[5] + d[7]);
        for (int c = 0; c < 3; c++) ej.xcf[k][c] = (float)ej.xc[k][c];
        for (int c = 0; c < 6; c++) ej.Df[k][c] = (float)ej.D[k][c];
    }
    ej.gmstf = (float)ej.gmst;
    ej.tau0f = (float)ej.tau0;
    ej.inv_dtf = (float)ej.inv_dt;
    ej.d_reff = (float)ej.d_ref;
    if (job->dist_marg) {
        if ((s = ctx_dist_table(ctx, job->pr, &ej.dt, nullptr)) != ILE_OK) return cleanup(s);
    }
    job->device_bytes = job->blob_bytes;
    *out = job;
    return ILE_OK;
}

extern "C" ile_status ile_job_info_get(const ile_job *job, ile_job_info *info) {
    if (!job || !info) return set_err(ILE_E_INVALID, "null argument");
    info->n_modes_kept = job->n_kept;
    info->mode_slots = kSets[job->set].n;
    info->n_det_slots = job->kp;
    info->device_bytes = job->device_bytes + job->part_cap * sizeof(MargPartial) + job->em_cap +
                         (job->d_gmm ? sizeof(GmmDev) : 0) + job->av_bytes + job->fair_cap +
                         (job->d_ac ? sizeof(AcDev) : 0);
    return ILE_OK;
}

void ile::job_release_nosync(ile_job *job) {
    if (!job) return;
    ile_ctx *ctx = job->ctx;
    ctx_free(ctx, job->d_blob, job->blob_bytes);
    ctx_free(ctx, job->d_part, job->part_cap * sizeof(MargPartial));
    ctx_free(ctx, job->d_em, job->em_cap);
    ctx_free(ctx, job->d_gmm, sizeof(GmmDev));
    ctx_free(ctx, job->d_zcount, kMaxComp * sizeof(uint32_t));
    ctx_free(ctx, job->av_mem, job->av_bytes);
    ctx_free(ctx, job->fair_mem, job->fair_cap);
    ctx_free(ctx, job->d_ac, sizeof(AcDev));
    pin_free(ctx, job->h_av, sizeof(AvDev));
    pin_free(ctx, job->h_blob, job->blob_bytes);
    pin_free(ctx, job->h_ms, sizeof(MargState));
    pin_free(ctx, job->h_gmm, sizeof(GmmDev));
    pin_free(ctx, job->h_ref, 7 * sizeof(double));
    delete job;
}

extern "C" void ile_job_release(ile_job *job) {
    if (!job) return;
    (void)hipSetDevice(job->ctx->device);
    (void)hipDeviceSynchronize();   // the caller's queued work may still use the buffers
    job_release_nosync(job);
}

// ================================================================ reference
namespace ile {
// Rebuild a mixed-policy job's reference terms from the point at
// job->rb.theta_ref (on the stream).
ile_status ref_rebuild(ile_job *job, hipStream_t st) {
    hipError_t e = launch_ref_build(job->set, job->kp, job->ej, job->rb, st);
    if (e != hipSuccess) return dev_fail(job->ctx, e, "reference build");
    return ILE_OK;
}
// Mixed-policy jobs: the reference point becomes the mean of the heaviest
// component of the job's (device) mixture.
ile_status ref_from_proposal(ile_job *job, hipStream_t st) {
    if (job->policy != kMixed || !job->d_gmm) return ILE_OK;
    hipError_t e = launch_ref_from_gmm(job->d_gmm, job->pr, (double *)job->rb.theta_ref, st);
    if (e != hipSuccess) return dev_fail(job->ctx, e, "reference from mixture");
    return ref_rebuild(job, st);
}
}  // namespace ile

extern "C" ile_status ile_set_reference(ile_job *job, const double *theta_ref, ile_stream stream) {
    if (!job || !theta_ref) return set_err(ILE_E_INVALID, "null argument");
    ile_status s = ctx_check(job->ctx);
    if (s != ILE_OK) return s;
    if (job->policy != kMixed) return ILE_OK;
    hipStream_t st = (hipStream_t)stream;
    // the pinned staging is reused by the next call: copy and wait
    std::memcpy(job->h_ref, theta_ref, 7 * sizeof(double));
    hipError_t e = hipMemcpyAsync((void *)job->rb.theta_ref, job->h_ref, 7 * sizeof(double), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return dev_fail(job->ctx, e, "reference upload");
    return ref_rebuild(job, st);
}

// ===================================================================== eval
extern "C" ile_status ile_eval_lnL(ile_job *job, int64_t n, const void *theta, int64_t ld, const void *lnpmps,
                                   void *lnL_out, void *lw_out, ile_stream stream) {
    // one job is a batch of one: the same kernels and descriptors, so a
    // sample's lnL does not depend on which entry point evaluated it
    if (!job) return set_err(ILE_E_INVALID, "null job");
    return ile_eval_lnL_batch(&job, 1, &n, &theta, &ld, &lnpmps, &lnL_out, &lw_out, stream);
}

extern "C" ile_status ile_eval_lnL_batch(ile_job *const *jobs, int32_t n_jobs, const int64_t *n,
                                         const void *const *theta, const int64_t *ld, const void *const *lnpmps,
                                         void *const *lnL_out, void *const *lw_out, ile_stream stream) {
    if (n_jobs <= 0) return ILE_OK;
    if (!jobs || !n || !theta || !ld || !lnL_out) return set_err(ILE_E_INVALID, "null argument");
    ile_ctx *ctx = jobs[0] ? jobs[0]->ctx : nullptr;
    ile_status s = ctx_check(ctx);
    if (s != ILE_OK) return s;
    std::vector<BatchItem> items;
    for (int j = 0; j < n_jobs; j++) {
        if (!jobs[j] || jobs[j]->ctx != ctx) return set_err(ILE_E_INVALID, "jobs must share one context");
        if (n[j] < 0 || ld[j] < n[j]) return set_err(ILE_E_INVALID, "need n >= 0 and ld >= n");
        if (n[j] > 0 && (!theta[j] || !lnL_out[j])) return set_err(ILE_E_INVALID, "null theta or lnL_out");
        items.push_back(BatchItem{jobs[j], n[j], theta[j], ld[j], lnpmps ? lnpmps[j] : nullptr, lnL_out[j],
                                  lw_out ? lw_out[j] : nullptr});
    }
    return eval_batch(ctx, items, (hipStream_t)stream);
}

extern "C" ile_status ile_eval_lnL_tmarg(ile_job *job, int64_t n, const void *theta, int64_t ld,
                                         const void *lnpmps, void *lnL_out, void *lw_out, int32_t oversample,
                                         ile_stream stream) {
    if (!job) return set_err(ILE_E_INVALID, "null job");
    return ile_eval_lnL_tmarg_batch(&job, 1, &n, &theta, &ld, &lnpmps, &lnL_out, &lw_out, oversample, stream);
}

extern "C" ile_status ile_eval_lnL_tmarg_batch(ile_job *const *jobs, int32_t n_jobs, const int64_t *n,
                                               const void *const *theta, const int64_t *ld,
                                               const void *const *lnpmps, void *const *lnL_out,
                                               void *const *lw_out, int32_t oversample, ile_stream stream) {
    if (n_jobs <= 0) return ILE_OK;
    if (!jobs || !n || !theta || !ld || !lnL_out) return set_err(ILE_E_INVALID, "null argument");
    ile_ctx *ctx = jobs[0] ? jobs[0]->ctx : nullptr;
    ile_status s = ctx_check(ctx);
    if (s != ILE_OK) return s;
    std::vector<BatchItem> items;
    for (int j = 0; j < n_jobs; j++) {
        if (!jobs[j] || jobs[j]->ctx != ctx) return set_err(ILE_E_INVALID, "jobs must share one context");
        if (n[j] < 0 || ld[j] < n[j]) return set_err(ILE_E_INVALID, "need n >= 0 and ld >= n");
        if (n[j] > 0 && (!theta[j] || !lnL_out[j])) return set_err(ILE_E_INVALID, "null theta or lnL_out");
        items.push_back(BatchItem{jobs[j], n[j], theta[j], ld[j], lnpmps ? lnpmps[j] : nullptr, lnL_out[j],
                                  lw_out ? lw_out[j] : nullptr});
    }
    return tmarg_batch(ctx, items, oversample, (hipStream_t)stream);
}

namespace ile {

// Time-marginalised evaluation: jobs grouped by compiled kernel, the window
// staged in LDS whenever it fits (each sample does hundreds of nodes of work).
ile_status tmarg_batch(ile_ctx *ctx, const std::vector<BatchItem> &items, int R, hipStream_t st) {
    if (R != 1 && R != 4) return set_err(ILE_E_INVALID, "oversample must be 1 or 4");
    std::map<std::tuple<int, int, int, int>, std::vector<int>> groups;
    for (size_t i = 0; i < items.size(); i++) {
        const ile_job *j = items[i].job;
        if (j->policy == kMixed) return set_err(ILE_E_INVALID, "time marginalisation supports FP32 and FP64 jobs");
        if (items[i].n == 0) continue;
        groups[std::make_tuple(j->set, j->kp, j->policy, j->dist_marg ? 1 : 0)].push_back((int)i);
    }
    std::lock_guard<std::mutex> lk(ctx->batch_mu);
    for (auto &g : groups) {
        const auto &idx = g.second;
        size_t win = 0;
        bool lds = true;
        for (int i : idx) {
            win = std::max(win, job_window_bytes(items[i].job, true));
            lds = lds && job_lds_ok(items[i].job, true);
        }
        const int policy = std::get<2>(g.first);
        const int block = tmarg_block_threads(policy);
        const int64_t tile = lds ? 4 * block : block;
        std::vector<EvalJob> ej;
        std::vector<Tile> tiles;
        for (int i : idx) {
            const BatchItem &b = items[i];
            EvalJob e = b.job->ej;
            e.theta = b.theta;
            e.ld = b.ld;
            e.lnpmps = b.lnpmps;
            e.lnL = b.lnL;
            e.lw = b.lw;
            e.n = b.n;
            const double dt = 1.0 / e.inv_dt, tw = b.job->pr.t_window;
            const double half = std::floor(R * tw / dt + 1e-9);
            if (!(half >= 0 && half < 1e6)) return set_err(ILE_E_INVALID, "time window too long for marginalisation");
            e.tm_half = (int)half;
            e.tm_lnw = std::log(dt / (R * 2.0 * tw));
            const int jid = (int)ej.size();
            ej.push_back(e);
            for (int64_t t0 = 0; t0 < b.n; t0 += tile) tiles.push_back(Tile{jid, 0, t0, std::min(t0 + tile, b.n)});
        }
        if (tiles.size() > (size_t)INT32_MAX) return set_err(ILE_E_INVALID, "too many samples for one launch");
        void *dj = nullptr, *dt = nullptr;
        int slot = -1;
        ile_status s = batch_upload(ctx, ej.data(), ej.size() * sizeof(EvalJob), tiles.data(),
                                    tiles.size() * sizeof(Tile), &dj, &dt, &slot, st);
        if (s != ILE_OK) return s;
        hipError_t e = launch_tmarg(std::get<0>(g.first), std::get<1>(g.first), policy, R, std::get<3>(g.first) != 0,
                                    lds ? win : 0,
                                    (const EvalJob *)dj, (const Tile *)dt, (int)tiles.size(), block, st);
        if (e != hipSuccess) return dev_fail(ctx, e, "time-marginalised eval launch");
        if ((s = batch_done(ctx, slot, st)) != ILE_OK) return s;
    }
    return ILE_OK;
}

// Group jobs by compiled kernel, upload the descriptors and tile lists through
// the context's pinned staging buffer, and launch one kernel per group.
ile_status eval_batch(ile_ctx *ctx, const std::vector<BatchItem> &items, hipStream_t st) {
    std::map<std::tuple<int, int, int, int>, std::vector<int>> groups;
    for (size_t i = 0; i < items.size(); i++) {
        const ile_job *j = items[i].job;
        if (items[i].n == 0) continue;
        groups[std::make_tuple(j->set, j->kp, j->policy, (int)j->dist_marg)].push_back((int)i);
    }
    std::lock_guard<std::mutex> lk(ctx->batch_mu);
    for (auto &g : groups) {
        const auto &idx = g.second;
        int64_t total = 0;
        size_t win = 0;
        bool lds_ok = true;
        for (int i : idx) {
            total += items[i].n;
            const ile_job *j = items[i].job;
            win = std::max(win, job_window_bytes(j, false));
            lds_ok = lds_ok && job_lds_ok(j, false);
        }
        const int64_t cus = 256;
        const bool lds = lds_ok && total >= (int64_t)2 * cus * 16384 && total / (int64_t)idx.size() >= 65536;
        // without LDS staging: about four 256-thread blocks per CU over the
        // whole batch (small batches would otherwise leave most CUs idle),
        // 256 to 8192 samples per tile
        int64_t tile = 65536;
        if (!lds) {
            tile = (total + 4 * cus - 1) / (4 * cus);
            tile = std::min<int64_t>(std::max<int64_t>((tile + 255) / 256 * 256, 256), 8192);
        }
        std::vector<EvalJob> ej;
        std::vector<Tile> tiles;
        for (int i : idx) {
            const BatchItem &b = items[i];
            EvalJob e = b.job->ej;
            e.theta = b.theta;
            e.ld = b.ld;
            e.lnpmps = b.lnpmps;
            e.lnL = b.lnL;
            e.lw = b.lw;
            e.n = b.n;
            const int jid = (int)ej.size();
            ej.push_back(e);
            for (int64_t t0 = 0; t0 < b.n; t0 += tile) tiles.push_back(Tile{jid, 0, t0, std::min(t0 + tile, b.n)});
        }
        void *dj = nullptr, *dt = nullptr;
        int slot = -1;
        ile_status s = batch_upload(ctx, ej.data(), ej.size() * sizeof(EvalJob), tiles.data(),
                                    tiles.size() * sizeof(Tile), &dj, &dt, &slot, st);
        if (s != ILE_OK) return s;
        const auto &key = g.first;
        hipError_t e = launch_eval(std::get<0>(key), std::get<1>(key), std::get<2>(key), std::get<3>(key) != 0,
                                   lds ? win : 0, (const EvalJob *)dj, (const Tile *)dt, (int)tiles.size(),
                                   lds ? lds_block_threads(std::get<0>(key), std::get<2>(key)) : 256, st);
        if (e != hipSuccess) return dev_fail(ctx, e, "batched eval launch");
        if ((s = batch_done(ctx, slot, st)) != ILE_OK) return s;
    }
    return ILE_OK;
}

ile_status batch_upload(ile_ctx *ctx, const void *a, size_t na, const void *b, size_t nb, void **da, void **db,
                        int *slot_out, hipStream_t st, size_t extra, void **dextra, void **hextra) {
    const size_t oa = 0, ob = (na + 255) / 256 * 256, copy = ob + nb;
    const size_t oe = (copy + 255) / 256 * 256, need = oe + extra;
    const int si = ctx->next_slot;
    ctx->next_slot = (si + 1) % ile_ctx::kSlots;
    ile_ctx::Slot &sl = ctx->slots[si];
    hipError_t e;
    if (!sl.ev && (e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming)) != hipSuccess)
        return dev_fail(ctx, e, "event create");
    if (sl.armed && (e = hipEventSynchronize(sl.ev)) != hipSuccess) return dev_fail(ctx, e, "scratch slot wait");
    sl.armed = false;
    if (need > sl.cap) {
        if (sl.d) (void)hipFree(sl.d);
        if (sl.h) (void)hipHostFree(sl.h);
        sl.d = nullptr;
        sl.h = nullptr;
        sl.cap = 0;
        const size_t cap = std::max<size_t>(need * 2, 1 << 16);
        if ((e = hipMalloc(&sl.d, cap)) != hipSuccess) return dev_fail(ctx, e, "batch scratch");
        if ((e = hipHostMalloc(&sl.h, cap, hipHostMallocDefault)) != hipSuccess)
            return dev_fail(ctx, e, "batch staging");
        sl.cap = cap;
    }
    std::memcpy((char *)sl.h + oa, a, na);
    if (nb) std::memcpy((char *)sl.h + ob, b, nb);
    if ((e = hipMemcpyAsync(sl.d, sl.h, copy, hipMemcpyHostToDevice, st)) != hipSuccess)
        return dev_fail(ctx, e, "batch upload");
    *da = (char *)sl.d + oa;
    *db = (char *)sl.d + ob;
    if (dextra) *dextra = (char *)sl.d + oe;
    if (hextra) *hextra = (char *)sl.h + oe;
    *slot_out = si;
    return ILE_OK;
}

ile_status batch_done(ile_ctx *ctx, int slot, hipStream_t st) {
    ile_ctx::Slot &sl = ctx->slots[slot];
    hipError_t e = hipEventRecord(sl.ev, st);
    if (e != hipSuccess) return dev_fail(ctx, e, "slot event");
    sl.armed = true;
    return ILE_OK;
}

// Counter-based draws for several jobs of one theta type in one launch.
ile_status draw_batch(ile_ctx *ctx, int policy, const std::vector<DrawJob> &jobs, hipStream_t st) {
    const int64_t tile = 2048;
    std::vector<Tile> tiles;
    for (size_t j = 0; j < jobs.size(); j++)
        for (int64_t t = 0; t < jobs[j].n; t += tile) tiles.push_back(Tile{(int32_t)j, 0, t, std::min(t + tile, jobs[j].n)});
    if (tiles.empty()) return ILE_OK;
    std::lock_guard<std::mutex> lk(ctx->batch_mu);
    void *dj = nullptr, *dt = nullptr;
    int slot = -1;
    ile_status s = batch_upload(ctx, jobs.data(), jobs.size() * sizeof(DrawJob), tiles.data(),
                                tiles.size() * sizeof(Tile), &dj, &dt, &slot, st);
    if (s != ILE_OK) return s;
    bool mix = false;
    for (const DrawJob &j : jobs) mix = mix || j.gmm != nullptr;
    hipError_t e =
        launch_draw(policy, (const DrawJob *)dj, (const Tile *)dt, (int)tiles.size(), jobs[0], tile, mix, st);
    if (e != hipSuccess) return dev_fail(ctx, e, "batched draw");
    return batch_done(ctx, slot, st);
}

ile_status pool_batch(ile_ctx *ctx, int policy, const std::vector<PoolJob> &jobs, hipStream_t st) {
    if (jobs.empty()) return ILE_OK;
    std::vector<PoolJob> pj(jobs);
    int64_t nt = 0;
    for (PoolJob &q : pj) {
        q.tile_begin = nt;
        nt += ((int64_t)(q.round + 1) * q.n_round + kPoolTileSamples - 1) / kPoolTileSamples;
    }
    std::lock_guard<std::mutex> lk(ctx->batch_mu);
    void *dj = nullptr, *dt = nullptr;
    int slot = -1;
    ile_status s = batch_upload(ctx, pj.data(), pj.size() * sizeof(PoolJob), nullptr, 0, &dj, &dt, &slot, st);
    if (s != ILE_OK) return s;
    hipError_t e = launch_pool_mix(policy, (const PoolJob *)dj, (int)pj.size(), nt, st);
    if (e != hipSuccess) return dev_fail(ctx, e, "mixture pool update");
    return batch_done(ctx, slot, st);
}

}  // namespace ile

// ================================================================ marginalise
namespace ile {

void marg_from_state(const MargState &m, ile_marg *out) {
    out->n = m.n;
    out->n_nonfinite = m.n_bad;
    out->max_lw = m.m;
    out->argmax = m.argmax;
    if (!(m.m > -INFINITY) || m.n == 0) {
        out->ln_L = -INFINITY;
        out->ln_sigma = -INFINITY;
        out->n_eff = 0.0;
        out->n_ess = 0.0;
        out->argmax = -1;
        return;
    }
    out->ln_L = m.m + std::log(m.s1) - std::log((double)m.n);
    out->n_eff = m.s1;
    out->n_ess = m.s1 * m.s1 / m.s2;
    if (m.n > 1) {
        const double v = ((double)m.n * m.s2 / (m.s1 * m.s1) - 1.0) / (double)(m.n - 1);
        out->ln_sigma = out->ln_L + 0.5 * std::log(v > 0 ? v : 0.0);
    } else {
        out->ln_sigma = -INFINITY;
    }
}

ile_status job_marg_launch(ile_job *job, int64_t n, const void *lw, bool reset, hipStream_t st) {
    ile_ctx *ctx = job->ctx;
    const int64_t tile = marg_tile(n);
    const int64_t np = std::max<int64_t>(1, (n + tile - 1) / tile);
    if ((size_t)np > job->part_cap) {
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) return dev_fail(ctx, e, "sync before partials growth");
        ctx_free(ctx, job->d_part, job->part_cap * sizeof(MargPartial));
        job->d_part = nullptr;
        job->part_cap = 0;
        ile_status s = ctx_alloc(ctx, (void **)&job->d_part, (size_t)np * sizeof(MargPartial), "partials");
        if (s != ILE_OK) return s;
        job->part_cap = (size_t)np;
    }
    hipError_t e = hipSuccess;
    if (n > 0) e = launch_marg_partials(job->policy, lw, n, tile, job->d_part, st);
    if (e != hipSuccess) return dev_fail(ctx, e, "marginal partials");
    e = launch_marg_combine(job->d_part, n > 0 ? (int)np : 0, n, job->d_ms, reset ? 1 : 0, st);
    if (e != hipSuccess) return dev_fail(ctx, e, "marginal combine");
    return ILE_OK;
}
}  // namespace ile

extern "C" ile_status ile_marginalize(ile_job *job, int64_t n, const void *lw, uint32_t flags, ile_marg *out,
                                      ile_stream stream) {
    if (!job) return set_err(ILE_E_INVALID, "null job");
    ile_status s = ctx_check(job->ctx);
    if (s != ILE_OK) return s;
    if (n < 0 || (n > 0 && !lw)) return set_err(ILE_E_INVALID, "bad lw");
    hipStream_t st = (hipStream_t)stream;
    if ((s = job_marg_launch(job, n, lw, (flags & ILE_MARG_RESET) != 0, st)) != ILE_OK) return s;
    if (out) {
        hipError_t e = hipMemcpyAsync(job->h_ms, job->d_ms, sizeof(MargState), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return dev_fail(job->ctx, e, "read estimator");
        marg_from_state(*job->h_ms, out);
    }
    return ILE_OK;
}

// ====================================================================== draws
extern "C" ile_status ile_draw(ile_job *job, uint64_t seed, uint32_t round, int64_t first_index, int64_t n,
                               void *theta_out, int64_t ld, void *lnpmps_out, ile_stream stream) {
    if (!job) return set_err(ILE_E_INVALID, "null job");
    ile_status s = ctx_check(job->ctx);
    if (s != ILE_OK) return s;
    if (n < 0 || ld < n || first_index < 0) return set_err(ILE_E_INVALID, "need n >= 0, ld >= n, first >= 0");
    if (n == 0) return ILE_OK;
    if (!theta_out) return set_err(ILE_E_INVALID, "null theta_out");
    DrawJob dj{};
    dj.gmm = job->has_prop ? job->d_gmm : nullptr;
    dj.pr = job->pr;
    dj.seed = seed;
    dj.round = round;
    dj.first = first_index;
    dj.theta = theta_out;
    dj.ld = ld;
    dj.lnpmps = lnpmps_out;
    dj.n = n;
    const int64_t tile = 2048;
    const int64_t nt = (n + tile - 1) / tile;
    if (nt > INT32_MAX) return set_err(ILE_E_INVALID, "too many samples for one launch");
    hipError_t e =
        launch_draw(job->policy, nullptr, nullptr, (int)nt, dj, tile, dj.gmm != nullptr, (hipStream_t)stream);
    if (e != hipSuccess) return dev_fail(job->ctx, e, "draw launch");
    return ILE_OK;
}

// =================================================================== proposal
namespace ile {

static void default_dims(const ile_job *job, int *nd, int dims[7]) {
    int k = 0;
    for (int c = 0; c < 7; c++)
        if (!(job->dist_marg && c == 3)) dims[k++] = c;
    *nd = k;
}

static ile_status ensure_gmm(ile_job *job) {
    if (job->d_gmm) return ILE_OK;
    ile_status s = ctx_alloc(job->ctx, (void **)&job->d_gmm, sizeof(GmmDev), "mixture state");
    if (s != ILE_OK) return s;
    s = ctx_alloc(job->ctx, (void **)&job->d_zcount, kMaxComp * sizeof(uint32_t), "mass counters");
    if (s != ILE_OK) return s;
    job->h_gmm = (GmmDev *)pin_alloc(job->ctx, sizeof(GmmDev));
    if (!job->h_gmm) return set_err(ILE_E_NOMEM, "pinned mixture buffer");
    return ILE_OK;
}

// Factor the job's uploaded mixture and estimate its in-support masses.
static ile_status factor_and_mass(ile_job *job, const ile_gmm_opts *o, hipStream_t st) {
    ile_ctx *ctx = job->ctx;
    EmJob e{};
    e.gmm = job->d_gmm;
    e.zcount = job->d_zcount;
    e.pr = job->pr;
    e.z_seed = o ? o->seed : 0x243F6A8885A308D3ull;
    e.z_round = o ? o->round : 0;
    e.z_draws = (o && o->z_draws > 0) ? o->z_draws : 65536;
    std::lock_guard<std::mutex> lk(ctx->batch_mu);
    void *dj = nullptr, *dn = nullptr;
    int slot = -1;
    ile_status s = batch_upload(ctx, &e, sizeof e, nullptr, 0, &dj, &dn, &slot, st);
    if (s != ILE_OK) return s;
    hipError_t err = launch_gmm_factor((const EmJob *)dj, 1, st);
    if (err == hipSuccess) err = launch_gmm_mass((const EmJob *)dj, 1, st);
    if (err != hipSuccess) return dev_fail(ctx, err, "factor and in-support mass");
    return batch_done(ctx, slot, st);
}

}  // namespace ile

extern "C" ile_status ile_set_proposal(ile_job *job, const ile_gmm_params *p, const ile_gmm_opts *opts,
                                       ile_stream stream) {
    if (!job || !p) return set_err(ILE_E_INVALID, "null argument");
    ile_status s = ctx_check(job->ctx);
    if (s != ILE_OK) return s;
    if (p->n_comp < 1 || p->n_comp > kMaxComp) return set_err(ILE_E_INVALID, "n_comp must be 1..16");
    if (!(p->eps_def >= 0 && p->eps_def < 1)) return set_err(ILE_E_INVALID, "eps_def must be in [0,1)");
    if (p->shear < -1 || p->shear > 1) return set_err(ILE_E_INVALID, "shear must be -1, 0 or 1");
    if ((s = ensure_gmm(job)) != ILE_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return dev_fail(job->ctx, e, "sync before proposal upload");
    GmmDev &g = *job->h_gmm;
    std::memset(&g, 0, sizeof g);
    default_dims(job, &g.n_dim, g.dims);
    g.n_comp = p->n_comp;
    g.eps_def = p->eps_def;
    g.shear = p->shear;   // the default columns always hold both phases
    double wsum = 0.0;
    for (int j = 0; j < p->n_comp; j++) {
        if (!(p->weight[j] >= 0) || !std::isfinite(p->weight[j])) return set_err(ILE_E_INVALID, "bad weight");
        wsum += p->weight[j];
    }
    if (!(wsum > 0)) return set_err(ILE_E_INVALID, "weights sum to zero");
    for (int j = 0; j < p->n_comp; j++) {
        g.w[j] = p->weight[j];
        for (int a = 0; a < g.n_dim; a++) {
            g.mean[j][a] = p->mean[j][a];
            for (int b = 0; b < g.n_dim; b++) g.cov[j][a][b] = p->cov[j][a][b];
        }
    }
    if ((e = hipMemcpyAsync(job->d_gmm, job->h_gmm, sizeof(GmmDev), hipMemcpyHostToDevice, st)) != hipSuccess)
        return dev_fail(job->ctx, e, "proposal upload");
    if ((s = factor_and_mass(job, opts, st)) != ILE_OK) return s;
    if ((e = hipMemcpyAsync(job->h_gmm, job->d_gmm, sizeof(GmmDev), hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return dev_fail(job->ctx, e, "proposal readback");
    if (!job->h_gmm->valid) return set_err(ILE_E_INVALID, "a covariance is not positive definite");
    job->has_prop = true;
    return ref_from_proposal(job, st);
}

extern "C" ile_status ile_get_proposal(ile_job *job, ile_gmm_params *p, ile_stream stream) {
    if (!job || !p) return set_err(ILE_E_INVALID, "null argument");
    ile_status s = ctx_check(job->ctx);
    if (s != ILE_OK) return s;
    if (!job->has_prop) return set_err(ILE_E_STATE, "job has no proposal");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(job->h_gmm, job->d_gmm, sizeof(GmmDev), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return dev_fail(job->ctx, e, "proposal readback");
    const GmmDev &g = *job->h_gmm;
    std::memset(p, 0, sizeof *p);
    p->n_comp = g.n_comp;
    p->n_dim = g.n_dim;
    for (int a = 0; a < 7; a++) p->dims[a] = a < g.n_dim ? g.dims[a] : -1;
    p->eps_def = g.eps_def;
    p->shear = g.shear;
    for (int j = 0; j < g.n_comp; j++) {
        p->weight[j] = g.w[j];
        p->ln_Z[j] = g.lnZ[j];
        for (int a = 0; a < 7; a++) {
            p->mean[j][a] = g.mean[j][a];
            for (int b = 0; b < 7; b++) p->cov[j][a][b] = g.cov[j][a][b];
        }
    }
    return ILE_OK;
}

namespace ile {
ile_status adapt_batch(ile_ctx *ctx, int policy, const std::vector<AdaptItem> &items, const ile_gmm_opts *o,
                       hipStream_t st) {
    if (items.empty()) return ILE_OK;
    const int n_comp = (o && o->n_comp > 0) ? o->n_comp : 8;
    const int n_iter = (o && o->n_iter > 0) ? o->n_iter : 8;
    const double eps = (o && o->eps_def >= 0 && o->eps_def < 1) ? o->eps_def : 0.05;
    if (n_comp > kMaxComp) return set_err(ILE_E_INVALID, "n_comp must be 1..16");
    if (n_iter > 1000) return set_err(ILE_E_INVALID, "n_iter must be at most 1000");
    const double temper = (o && o->temper_ess > 0) ? std::min(o->temper_ess, 1.0) : 0.0;
    const int64_t z_draws = (o && o->z_draws > 0) ? o->z_draws : 65536;
    if (items.size() > 65535) return set_err(ILE_E_INVALID, "too many jobs in one refit");
    std::vector<EmJob> ej(items.size());
    for (size_t k = 0; k < items.size(); k++) {
        const AdaptItem &it = items[k];
        ile_job *job = it.job;
        if (job->policy != policy) return set_err(ILE_E_INVALID, "refit batch mixes precision policies");
        ile_status s;
        if ((s = ensure_gmm(job)) != ILE_OK) return s;
        const size_t need = em_work_bytes(it.n);
        if (need > job->em_cap) {
            hipError_t e = hipStreamSynchronize(st);
            if (e != hipSuccess) return dev_fail(ctx, e, "sync before EM workspace growth");
            ctx_free(ctx, job->d_em, job->em_cap);
            job->d_em = nullptr;
            job->em_cap = 0;
            if ((s = ctx_alloc(ctx, (void **)&job->d_em, need, "EM workspace")) != ILE_OK) return s;
            job->em_cap = need;
        }
        EmJob &e = ej[k];
        e.theta = it.theta;
        e.ld = it.ld;
        e.lw = it.lw;
        e.n = it.n;
        e.gmm = job->d_gmm;
        e.work = job->d_em;
        e.zcount = job->d_zcount;
        e.pr = job->pr;
        e.n_comp = n_comp;
        e.first = job->has_prop ? 0 : 1;
        default_dims(job, &e.n_dim, e.dims);
        e.eps_def = eps;
        e.temper = temper;
        e.shear_auto = (o && o->phase_shear) ? 1 : 0;
        e.z_seed = it.z_seed;
        e.z_round = it.z_round;
        e.z_draws = z_draws;
    }
    {
        std::lock_guard<std::mutex> lk(ctx->batch_mu);
        void *dj = nullptr, *dn = nullptr;
        int slot = -1;
        ile_status s = batch_upload(ctx, ej.data(), ej.size() * sizeof(EmJob), nullptr, 0, &dj, &dn, &slot, st);
        if (s != ILE_OK) return s;
        hipError_t e = launch_em_batch(policy, (const EmJob *)dj, ej.data(), (int)ej.size(), n_iter, st);
        if (e == hipSuccess) e = launch_gmm_mass((const EmJob *)dj, (int)ej.size(), st);
        if (e != hipSuccess) return dev_fail(ctx, e, "batched mixture refit");
        if ((s = batch_done(ctx, slot, st)) != ILE_OK) return s;
    }
    for (const AdaptItem &it : items) {
        it.job->has_prop = true;
        ile_status s = ref_from_proposal(it.job, st);
        if (s != ILE_OK) return s;
    }
    return ILE_OK;
}

ile_status job_adapt(ile_job *job, int64_t n, const void *theta, int64_t ld, const void *lw, const ile_gmm_opts *o,
                     hipStream_t st) {
    AdaptItem it{job, n, theta, ld, lw, o ? o->seed : 0x243F6A8885A308D3ull, o ? o->round : 0u};
    return adapt_batch(job->ctx, job->policy, std::vector<AdaptItem>{it}, o, st);
}
}  // namespace ile

extern "C" ile_status ile_adapt_proposal(ile_job *job, int64_t n, const void *theta, int64_t ld, const void *lw,
                                         const ile_gmm_opts *opts, ile_gmm_params *out, ile_stream stream) {
    if (!job) return set_err(ILE_E_INVALID, "null job");
    ile_status s = ctx_check(job->ctx);
    if (s != ILE_OK) return s;
    if (n < 1 || ld < n || !theta || !lw) return set_err(ILE_E_INVALID, "need n >= 1, ld >= n and data");
    if ((s = job_adapt(job, n, theta, ld, lw, opts, (hipStream_t)stream)) != ILE_OK) return s;
    if (out) return ile_get_proposal(job, out, stream);
    return ILE_OK;
}
