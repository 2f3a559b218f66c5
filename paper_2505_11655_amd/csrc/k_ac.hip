// Product-form adaptive Cartesian (AC) sampling prior: one adaptive
// piecewise-constant marginal per sampled coordinate of the prior's CDF cube
// (kAcBins equal bins), the sampler with product form whose one-dimensional
// marginals are updated after each block of evaluations (Section "Evaluating
// the marginalized likelihood").
//   draw: column c's uniform U (the prior draw's words) selects the first bin
//         b with cum > U; x = (b + (U - cum[b-1]) / pi[b]) / nb (the inverse CDF
//         of the marginal); ln p - ln p_s = -sum_k ln(nb pi[k][b_k]).
//   update: each marginal becomes the histogram of the round's fixed-point
//         masses q_i = floor(exp(lw_i - max lw) 2^40) over its bins, mixed with
//         the uniform: pi = (1 - floor) h / total + floor / nb; cumulative sums
//         sequential in bin order, the last set to 1.  Integer histograms make
//         the update independent of accumulation order.  A sample's bins are
//         regenerated from its Philox counter and the marginals it was drawn
//         from.  With no finite weight the marginals are kept.
#include "ile_internal.h"

namespace ile {

namespace {

constexpr int kAcThreads = 256;

__device__ __forceinline__ void ac_words(uint64_t seed, uint64_t i, uint32_t r, uint32_t *w) {
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (int b = 0; b < 4; b++) {
        const U4 o = philox4x32_10(U4{(uint32_t)i, (uint32_t)(i >> 32), r, (uint32_t)b}, k0, k1);
        w[4 * b + 0] = o.x;
        w[4 * b + 1] = o.y;
        w[4 * b + 2] = o.z;
        w[4 * b + 3] = o.w;
    }
}

// First bin with cum > U (the last bin if none).
__device__ __forceinline__ int ac_bin(const double *cum, double U) {
    int lo = 0, hi = kAcBins - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cum[mid] > U)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// Unit-cube coordinates and ln p - ln p_s of one sample; bins[k] of each marginal.
__device__ __forceinline__ double ac_unit(const AcDev &S, const uint32_t *w, double u[7], int bins[7]) {
    double lr = 0.0;
#pragma unroll
    for (int c = 0; c < 7; c++) {
        const double U = u53(w[2 * c], w[2 * c + 1]);
        const int k = S.kcol[c];
        u[c] = U;
        bins[c] = -1;
        if (k >= 0) {
            const int b = ac_bin(S.cum[k], U);
            const double lo = b > 0 ? S.cum[k][b - 1] : 0.0;
            u[c] = ((double)b + (U - lo) / S.pi[k][b]) / (double)kAcBins;
            lr -= S.lnbp[k][b];
            bins[c] = b;
        }
    }
    return lr;
}

// Cumulative sums and ln(nb pi) of marginal k from its pi (one thread).
__device__ __forceinline__ void ac_derive(AcDev &S, int k) {
    double run = 0.0;
    for (int b = 0; b < kAcBins; b++) {
        run += S.pi[k][b];
        S.cum[k][b] = run;
        S.lnbp[k][b] = log((double)kAcBins * S.pi[k][b]);
    }
    S.cum[k][kAcBins - 1] = 1.0;
}

__global__ void k_ac_reset(AcDev *S_, int d, int d0, int d1, int d2, int d3, int d4, int d5, int d6) {
    AcDev &S = *S_;
    const int dims[7] = {d0, d1, d2, d3, d4, d5, d6};
    if (threadIdx.x == 0) {
        S.d = d;
        for (int c = 0; c < 7; c++) S.kcol[c] = -1;
        for (int k = 0; k < 7; k++) {
            S.dims[k] = k < d ? dims[k] : -1;
            if (k < d) S.kcol[dims[k]] = k;
        }
    }
    if ((int)threadIdx.x < 7) {
        const int k = threadIdx.x;
        for (int b = 0; b < kAcBins; b++) S.pi[k][b] = 1.0 / kAcBins;
        ac_derive(S, k);
    }
}

#define AC_JOB const AcJob &J = jobs[blockIdx.z]
#define AC_SAMPLES(s) \
    for (int64_t s = (int64_t)blockIdx.x * kAcThreads + threadIdx.x; s < J.n; s += (int64_t)gridDim.x * kAcThreads)

template <class TT>
__global__ void __launch_bounds__(kAcThreads) k_ac_draw(const AcJob *__restrict__ jobs) {
    AC_JOB;
    const AcDev &S = *J.st;
    TT *th_out = (TT *)J.theta;
    TT *lr_out = (TT *)J.lnpmps;
    AC_SAMPLES(s) {
        uint32_t w[16];
        ac_words(J.seed, (uint64_t)(J.first + s), J.round, w);
        double u[7], th[7];
        int bins[7];
        const double lr = ac_unit(S, w, u, bins);
        prior_map(J.pr, u, th);
#pragma unroll
        for (int c = 0; c < 7; c++) th_out[c * J.ld + s] = (TT)th[c];
        if (lr_out) lr_out[s] = (TT)lr;
    }
}

__global__ void k_ac_begin(const AcJob *__restrict__ jobs) {
    AC_JOB;
    AcDev &S = *J.st;
    if (threadIdx.x == 0) {
        S.key_max = 0;
        S.n_fin = 0;
    }
    for (int i = threadIdx.x; i < 7 * kAcBins; i += blockDim.x) (&S.hist[0][0])[i] = 0;
}

template <class TO>
__global__ void __launch_bounds__(kAcThreads) k_ac_max(const AcJob *__restrict__ jobs) {
    AC_JOB;
    const TO *lw = (const TO *)J.lw;
    unsigned long long km = 0, cnt = 0;
    AC_SAMPLES(s) {
        const TO v = lw[s];
        if (isfinite(v)) {
            const unsigned long long k = ord_key(v);
            km = k > km ? k : km;
            cnt += 1;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long k2 = __shfl_xor(km, o);
        km = k2 > km ? k2 : km;
        cnt += __shfl_xor(cnt, o);
    }
    if ((threadIdx.x & 63) == 0 && cnt) {
        atomicMax(&J.st->key_max, km);
        atomicAdd(&J.st->n_fin, cnt);
    }
}

template <class TO>
__global__ void __launch_bounds__(kAcThreads) k_ac_hist(const AcJob *__restrict__ jobs) {
    AC_JOB;
    const AcDev &S = *J.st;
    if (S.n_fin == 0 || (int64_t)blockIdx.x * kAcThreads >= J.n) return;
    __shared__ unsigned long long h[7 * kAcBins];
    for (int i = threadIdx.x; i < 7 * kAcBins; i += kAcThreads) h[i] = 0;
    __syncthreads();
    constexpr int nbits = sizeof(TO) * 8;
    const double vmax = ord_value(S.key_max, nbits);
    const TO *lw = (const TO *)J.lw;
    AC_SAMPLES(s) {
        const TO v = lw[s];
        if (!isfinite(v)) continue;
        const unsigned long long q = mass_fx((double)v, vmax);
        if (q == 0) continue;
        uint32_t w[16];
        ac_words(J.seed, (uint64_t)(J.first + s), J.round, w);
        double u[7];
        int bins[7];
        (void)ac_unit(S, w, u, bins);
#pragma unroll
        for (int c = 0; c < 7; c++)
            if (bins[c] >= 0) atomicAdd(&h[S.kcol[c] * kAcBins + bins[c]], q);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 7 * kAcBins; i += kAcThreads)
        if (h[i]) atomicAdd(&(&J.st->hist[0][0])[i], h[i]);
}

// New marginals; one thread per marginal (the histograms of every marginal
// sum to the same total).
__global__ void k_ac_finish(const AcJob *__restrict__ jobs) {
    AC_JOB;
    AcDev &S = *J.st;
    const int k = threadIdx.x;
    if (S.n_fin == 0 || k >= S.d) return;
    unsigned long long tot = 0;
    for (int b = 0; b < kAcBins; b++) tot += S.hist[k][b];
    if (tot == 0) return;
    const double keep = 1.0 - J.floor, add = J.floor / kAcBins;
    for (int b = 0; b < kAcBins; b++) {
        // rounded product, then rounded sum (no fused multiply-add): the
        // marginal is defined by these two roundings
        const double h = __dmul_rn(keep, (double)S.hist[k][b] / (double)tot);
        S.pi[k][b] = __dadd_rn(h, add);
    }
    ac_derive(S, k);
}

int ac_grid(int64_t n, int per) {
    const int64_t g = (n + (int64_t)kAcThreads * per - 1) / ((int64_t)kAcThreads * per);
    return (int)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

int64_t ac_max_n(const AcJob *h, int n_jobs) {
    int64_t m = 0;
    for (int k = 0; k < n_jobs; k++) m = h[k].n > m ? h[k].n : m;
    return m;
}

template <class TO>
hipError_t ac_update_t(const AcJob *d, int n_jobs, int64_t nmax, hipStream_t st) {
    const unsigned nz = (unsigned)n_jobs;
    hipLaunchKernelGGL(k_ac_begin, dim3(1, 1, nz), dim3(256), 0, st, d);
    hipLaunchKernelGGL(k_ac_max<TO>, dim3(ac_grid(nmax, 16), 1, nz), dim3(kAcThreads), 0, st, d);
    hipLaunchKernelGGL(k_ac_hist<TO>, dim3(ac_grid(nmax, 4), 1, nz), dim3(kAcThreads), 0, st, d);
    hipLaunchKernelGGL(k_ac_finish, dim3(1, 1, nz), dim3(64), 0, st, d);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_ac_reset(AcDev *S, int d, const int *dims, hipStream_t st) {
    int dd[7] = {-1, -1, -1, -1, -1, -1, -1};
    for (int k = 0; k < d && k < 7; k++) dd[k] = dims[k];
    hipLaunchKernelGGL(k_ac_reset, dim3(1), dim3(64), 0, st, S, d, dd[0], dd[1], dd[2], dd[3], dd[4], dd[5], dd[6]);
    return hipGetLastError();
}

hipError_t launch_ac_draw(int policy, const AcJob *d_jobs, const AcJob *h_jobs, int n_jobs, hipStream_t st) {
    const int64_t nmax = ac_max_n(h_jobs, n_jobs);
    if (n_jobs <= 0 || nmax <= 0) return hipSuccess;
    const dim3 grid(ac_grid(nmax, 4), 1, (unsigned)n_jobs);
    if (policy == kFP64)
        hipLaunchKernelGGL(k_ac_draw<double>, grid, dim3(kAcThreads), 0, st, d_jobs);
    else
        hipLaunchKernelGGL(k_ac_draw<float>, grid, dim3(kAcThreads), 0, st, d_jobs);
    return hipGetLastError();
}

hipError_t launch_ac_update(int policy, const AcJob *d_jobs, const AcJob *h_jobs, int n_jobs, hipStream_t st) {
    const int64_t nmax = ac_max_n(h_jobs, n_jobs);
    if (n_jobs <= 0 || nmax <= 0) return hipSuccess;
    if (policy == kFP32) return ac_update_t<float>(d_jobs, n_jobs, nmax, st);
    return ac_update_t<double>(d_jobs, n_jobs, nmax, st);
}

}  // namespace ile
