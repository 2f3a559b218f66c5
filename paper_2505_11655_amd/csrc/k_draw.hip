// Counter-based extrinsic draws for eq. (lnL:MonteCarlo): theta ~ p_s, with
// p_s the prior or the mixture proposal (1-eps) sum_j pi_j N_j/Z_j + eps p.
//
// Counter layout (key = seed words; each block gives four words):
//   sample i, round r, attempt a, block b:  (i lo, i hi, r, 16 a + b).
// Prior draw: 7 uniforms from blocks 0..3 of attempt 0 (words 2c, 2c+1),
// mapped by inverse CDFs.  Mixture draw: the selector is the first uniform of
// block 0 (attempt 0); the prior fallback and the non-mixture columns use
// blocks 1..4 of attempt 0; attempt a = 1..64 of a component draws z from
// four Box-Muller pairs of blocks 1..4 of attempt a (never the words of the
// prior draw, so the fallback is independent of the rejections) and accepts
// x = mu + L z if every bounded column is inside its interval and every
// periodic offset lies in (-P/2, P/2]; after 64 rejected attempts the prior
// draw is kept.  The density of the draw is therefore
//   p_s(x) = [eps + (1-eps) sum_j pi_j r_j] p(x)
//          + (1-eps) sum_j pi_j (1 - r_j) N_j(x) p_rest(x) / Z_j,
// r_j = (1 - Z_j)^64 the chance that all attempts fail, p_rest the prior of
// the columns outside the mixture (pi_j normalised).
//
// Two instantiations per sample type: prior-only launches (no mixture code,
// so the kernel stays small and occupancy high) and launches where some job
// carries a mixture.  Mixture columns are addressed through select chains on
// the (uniform) column index, so every per-sample array stays in registers.
#include "ile_sincos.h"
#include <type_traits>

#include "ile_internal.h"

namespace ile {

namespace {

constexpr int kDrawThreads = 256;
constexpr int kMaxAttempts = 64;
constexpr double kPi = 3.14159265358979323846;

__device__ __forceinline__ void words(uint64_t seed, uint64_t i, uint32_t r, uint32_t a, int b0, int nb,
                                      uint32_t *w) {
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (int b = 0; b < nb; b++) {
        U4 o = philox4x32_10(U4{(uint32_t)i, (uint32_t)(i >> 32), r, a * 16u + (uint32_t)(b0 + b)}, k0, k1);
        w[4 * b + 0] = o.x;
        w[4 * b + 1] = o.y;
        w[4 * b + 2] = o.z;
        w[4 * b + 3] = o.w;
    }
}

__device__ __forceinline__ void support(const PriorDev &pr, int col, double &lo, double &hi, double &P) {
    P = 0.0;
    switch (col) {
    case 0: lo = 0.0; hi = 2 * kPi; P = 2 * kPi; break;
    case 1: lo = -0.5 * kPi; hi = 0.5 * kPi; break;
    case 2: lo = -pr.t_window; hi = pr.t_window; break;
    case 3: lo = pr.d_min; hi = pr.d_max; break;
    case 4: lo = -1.0; hi = 1.0; break;
    case 5: lo = 0.0; hi = 2 * kPi; P = 2 * kPi; break;
    default: lo = 0.0; hi = kPi; P = kPi; break;
    }
}

// v[c] for a uniform column index c, without dynamic register indexing
__device__ __forceinline__ double pick7(const double v[7], int c) {
    double r = v[0];
#pragma unroll
    for (int k = 1; k < 7; k++) r = (c == k) ? v[k] : r;
    return r;
}

__device__ __forceinline__ double ln_prior(const PriorDev &pr, const double th[7]) {
    double lp = -log(2 * kPi) + log(0.5 * cos(th[1])) - log(2.0 * pr.t_window) - log(2.0) - log(2 * kPi) -
                log(kPi);
    if (!pr.dist_marg) {
        const double a3 = pr.d_min * pr.d_min * pr.d_min, b3 = pr.d_max * pr.d_max * pr.d_max;
        lp += log(3.0 * th[3] * th[3] / (b3 - a3));
    }
    return lp;
}

__device__ __forceinline__ void prior_from_words(const PriorDev &pr, const uint32_t *w, double th[7]) {
    double u[7];
#pragma unroll
    for (int c = 0; c < 7; c++) u[c] = u53(w[2 * c], w[2 * c + 1]);
    prior_map(pr, u, th);
}

// wrapped difference in (-P/2, P/2]: d - P floor(d/P), folded; for |d| < P
// the same value without the division
__device__ __forceinline__ double wrapd(double d, double P) {
    if (P <= 0.0) return d;
    double r;
    if (d >= 0.0 && d < P)
        r = d;
    else if (d < 0.0 && d >= -P)
        r = d + P;
    else
        r = d - P * floor(d / P);
    return r > 0.5 * P ? r - P : r;
}

// ln of the prior density of one column (the prior factorises by column).
__device__ __forceinline__ double ln_prior_col(const PriorDev &pr, int c, const double th[7]) {
    switch (c) {
    case 0: return -log(2 * kPi);
    case 1: return log(0.5 * cos(th[1]));
    case 2: return -log(2.0 * pr.t_window);
    case 3: {
        if (pr.dist_marg) return 0.0;
        const double a3 = pr.d_min * pr.d_min * pr.d_min, b3 = pr.d_max * pr.d_max * pr.d_max;
        return log(3.0 * th[3] * th[3] / (b3 - a3));
    }
    case 4: return -log(2.0);
    case 5: return -log(2 * kPi);
    default: return -log(kPi);
    }
}

typedef __attribute__((address_space(4))) const GmmDev cgmm;

// Running log-sum-exp: m the running maximum, s the sum of e^{t - m}.
// FAST: the exponential of the (FP64) difference taken in FP32, for sums
// whose terms need only FP32 relative accuracy.
template <bool FAST = false>
__device__ __forceinline__ void lse_add(double &m, double &s, double t) {
    if (!(t > -INFINITY)) return;
    auto ex = [](double x) { return FAST ? (double)__expf((float)x) : exp(x); };
    if (t > m) {
        s = s * ex(m - t) + 1.0;
        m = t;
    } else {
        s += ex(t - m);
    }
}

// The mixture's columns (uniform): count, shear, theta column and period of
// each mixture dimension.
struct MixCols {
    int d, shear;
    int col[7];
    double P[7], iP[7];
};
__device__ __forceinline__ MixCols mix_cols(cgmm &g) {
    MixCols mc;
    mc.d = g.n_dim;
    mc.shear = g.shear;
#pragma unroll
    for (int a = 0; a < 7; a++) {
        mc.col[a] = a < mc.d ? g.dims[a] : 0;
        const int c = mc.col[a];
        mc.P[a] = (a < mc.d && (c == 0 || c == 5)) ? 2 * kPi : ((a < mc.d && c == 6) ? kPi : 0.0);
        mc.iP[a] = mc.P[a] > 0.0 ? 1.0 / mc.P[a] : 0.0;
    }
    return mc;
}
// A sample's mixture coordinates (phase shear applied) and ln of the prior of
// the mixture columns (the other columns' prior cancels in ln p_s - ln p).
__device__ __forceinline__ void mix_coords(const MixCols &mc, const PriorDev &pr, const double th[7], double xm[7],
                                           double &lpm) {
    lpm = 0.0;
#pragma unroll
    for (int a = 0; a < 7; a++) {
        if (a < mc.d) lpm += ln_prior_col(pr, mc.col[a], th);
        const double v = pick7(th, mc.col[a]);
        xm[a] = (mc.col[a] == 6 && mc.shear) ? shear_phase(th[6], th[5], mc.shear) : v;
    }
}
// t_k = ln p_s(x_k) - ln p(x_k) for NS samples of one mixture (the density of
// a mixture draw above):
//   t = ln[ sum_j e^{lnc_j} N_j(x) / p_mix(x) + e^{ln_fb} ],
// by a running log-sum-exp.  The mixture is read through the scalar cache
// (the component loop is uniform) and applied row by row to every sample; a
// periodic offset is wrapped as u - P rint(u / P) (the floor form's value
// except at exactly half a period, where both images are equally far).
// D > 0: the mixture's dimension count fixed at compile time (it must equal
// mc.d), which removes the per-dimension tests from the unrolled loops.
template <int NS, bool FAST = false, int D = 0>
__device__ __forceinline__ void mix_log_ratio(cgmm &g, const MixCols &mc, const double (&xm)[NS][7],
                                              const double (&lpm)[NS], double (&t)[NS]) {
    const int d = D > 0 ? D : mc.d;
    const double c0 = -0.5 * d * log(2 * kPi);
    double mm[NS], ss[NS];
#pragma unroll
    for (int k = 0; k < NS; k++) {
        mm[k] = -INFINITY;
        ss[k] = 0.0;
        lse_add(mm[k], ss[k], g.ln_fb);
    }
    const int nc = g.n_comp;
    for (int j = 0; j < nc; j++) {
        if (g.lnc[j] == -INFINITY) continue;
        const double cj = g.lnc[j] - g.logdet_half[j] + c0;
        double df[NS][7], qf[NS];
#pragma unroll
        for (int a = 0; a < 7; a++) {
            const double mu = g.mean[j][a];
#pragma unroll
            for (int k = 0; k < NS; k++) {
                const double u = xm[k][a] - mu;
                df[k][a] = a < d ? u - mc.P[a] * rint(u * mc.iP[a]) : 0.0;
            }
        }
#pragma unroll
        for (int k = 0; k < NS; k++) qf[k] = 0.0;
#pragma unroll
        for (int a = 0; a < 7; a++) {
            if (a >= d) break;
            double y[NS];
#pragma unroll
            for (int k = 0; k < NS; k++) y[k] = 0.0;
#pragma unroll
            for (int b = 0; b <= a; b++) {
                const double lab = g.Linv[j][a][b];
#pragma unroll
                for (int k = 0; k < NS; k++) y[k] = fma(lab, df[k][b], y[k]);
            }
#pragma unroll
            for (int k = 0; k < NS; k++) qf[k] = fma(y[k], y[k], qf[k]);
        }
#pragma unroll
        for (int k = 0; k < NS; k++) lse_add<FAST>(mm[k], ss[k], cj - 0.5 * qf[k] - lpm[k]);
    }
#pragma unroll
    for (int k = 0; k < NS; k++) t[k] = mm[k] > -INFINITY ? mm[k] + log(ss[k]) : -INFINITY;
}

// One candidate from component j: words w[0..15] give four Box-Muller pairs.
// On acceptance the mixture columns of th are overwritten; on rejection th is
// left as it was.
// D > 0: the mixture's dimension count as a compile-time constant (it must
// equal g.n_dim).
template <int D = 0>
__device__ __forceinline__ bool gmm_candidate(const GmmDev &g, const PriorDev &pr, int j, const uint32_t *w,
                                              double th[7]) {
    double z[8];
#pragma unroll
    for (int p = 0; p < 4; p++) {
        const double u1 = u53(w[4 * p], w[4 * p + 1]), u2 = u53(w[4 * p + 2], w[4 * p + 3]);
        const double r = sqrt(-2.0 * log(u1));
        double s, c;
        sincos_rad(2 * kPi * u2, &s, &c);   // FP64 reduction + series (no large-argument path)
        z[2 * p] = r * c;
        z[2 * p + 1] = r * s;
    }
    const int d = D > 0 ? D : g.n_dim;
    double x[7];
#pragma unroll
    for (int a = 0; a < 7; a++) {
        x[a] = 0.0;
        if (a < d) {
            double off = 0.0;
#pragma unroll
            for (int b = 0; b <= a; b++) off += g.L[j][a][b] * z[b];
            double lo, hi, P;
            support(pr, g.dims[a], lo, hi, P);
            double v = g.mean[j][a] + off;
            if (P > 0.0) {
                if (!(off > -0.5 * P && off <= 0.5 * P)) return false;
                v = v - P * floor((v - lo) / P);
            } else if (!(v >= lo && v <= hi)) {
                return false;
            }
            x[a] = v;
        }
    }
#pragma unroll
    for (int a = 0; a < 7; a++) {
        if (a < d) {
            const int c = g.dims[a];
#pragma unroll
            for (int k = 0; k < 7; k++) th[k] = (c == k) ? x[a] : th[k];
        }
    }
    return true;
}

// Mixture draw of sample idx (theta only; the density follows for a pair).
template <int D = 0>
__device__ __forceinline__ void draw_mix(const DrawJob &J, const GmmDev &g, uint64_t idx, double th[7]) {
    uint32_t w[20];
    words(J.seed, idx, J.round, 0, 0, 5, w);
    prior_from_words(J.pr, w + 4, th);
    const double usel = u53(w[0], w[1]);
    if (usel >= g.eps_def) {
        const double v = (usel - g.eps_def) / (1.0 - g.eps_def);
        double tot = 0.0;
        for (int j = 0; j < g.n_comp; j++) tot += g.w[j];
        int jsel = -1;
        double acc = 0.0;
        for (int j = 0; j < g.n_comp; j++) {
            if (!(g.w[j] > 0.0)) continue;
            acc += g.w[j] / tot;
            jsel = j;
            if (v < acc) break;
        }
        for (int a = 1; a <= kMaxAttempts && jsel >= 0; a++) {
            uint32_t wa[16];
            words(J.seed, idx, J.round, (uint32_t)a, 1, 4, wa);
            if (gmm_candidate<D>(g, J.pr, jsel, wa, th)) {
                // accepted in the mixture's coordinates: back to psi
                if (g.shear) th[6] = shear_phase(th[6], th[5], -g.shear);
                break;
            }
        }
    }
}

template <class TT, bool MIX>
__device__ __forceinline__ void draw_range(const DrawJob &J, int64_t begin, int64_t end) {
    TT *__restrict__ th_out = (TT *)J.theta;
    TT *__restrict__ lr_out = (TT *)J.lnpmps;
    if (!MIX || J.gmm == nullptr) {
        for (int64_t s = begin + threadIdx.x; s < end; s += kDrawThreads) {
            const uint64_t idx = (uint64_t)(J.first + s);
            double th[7];
            uint32_t w[16];
            words(J.seed, idx, J.round, 0, 0, 4, w);
            prior_from_words(J.pr, w, th);
#pragma unroll
            for (int c = 0; c < 7; c++) th_out[c * J.ld + s] = (TT)th[c];
            if (lr_out) lr_out[s] = (TT)0;
        }
        return;
    }
    // mixture draws: theta, then ln p - ln p_s from the mixture read through
    // the scalar cache
    cgmm &g = *(cgmm *)J.gmm;
    const MixCols mc = mix_cols(g);
    // the common dimension counts (six with the distance integrated, seven
    // otherwise) compiled as constants
    auto samples = [&](auto D_) {
        constexpr int D = decltype(D_)::value;
        for (int64_t s = begin + threadIdx.x; s < end; s += kDrawThreads) {
            double th[1][7], xm[1][7], lpm[1], t[1];
            draw_mix<D>(J, *J.gmm, (uint64_t)(J.first + s), th[0]);
            mix_coords(mc, J.pr, th[0], xm[0], lpm[0]);
            mix_log_ratio<1, false, D>(g, mc, xm, lpm, t);
#pragma unroll
            for (int c = 0; c < 7; c++) th_out[c * J.ld + s] = (TT)th[0][c];
            if (lr_out) lr_out[s] = (TT)(-t[0]);
        }
    };
    if (mc.d == 6)
        samples(std::integral_constant<int, 6>{});
    else if (mc.d == 7)
        samples(std::integral_constant<int, 7>{});
    else
        samples(std::integral_constant<int, 0>{});
}

template <class TT, bool MIX>
__global__ void __launch_bounds__(kDrawThreads)
    k_draw(const DrawJob *__restrict__ jobs, const Tile *__restrict__ tiles, const DrawJob single, int64_t tile) {
    if (jobs != nullptr) {
        const Tile tl = tiles[blockIdx.x];
        draw_range<TT, MIX>(jobs[tl.job], tl.begin, tl.end);
    } else {
        const int64_t b = (int64_t)blockIdx.x * tile;
        draw_range<TT, MIX>(single, b, b + tile < single.n ? b + tile : single.n);
    }
}

template <class TT>
void launch_draw_t(bool mix, const DrawJob *d_jobs, const Tile *d_tiles, int n_tiles, const DrawJob &single,
                   int64_t tile, hipStream_t st) {
    if (mix)
        hipLaunchKernelGGL((k_draw<TT, true>), dim3(n_tiles), dim3(kDrawThreads), 0, st, d_jobs, d_tiles, single,
                           tile);
    else
        hipLaunchKernelGGL((k_draw<TT, false>), dim3(n_tiles), dim3(kDrawThreads), 0, st, d_jobs, d_tiles, single,
                           tile);
}

// Mixture pool update (see PoolJob).  A block takes kPoolTileSamples samples
// of one job, kPoolSpt per thread held in registers in the mixture's
// coordinates; each proposal q adds t_q = ln p_s,q(x) - ln p(x) (mix_log_ratio)
// to every sample's running log-sum over proposals.
constexpr int kPoolSpt = 2;
static_assert(kPoolTileSamples == (int64_t)kPoolSpt * kDrawThreads, "pool tile = samples per thread x block");


template <class TT, class TO, class TL>
__global__ void __launch_bounds__(kDrawThreads)
    k_pool_mix(const PoolJob *__restrict__ jobs, const int n_jobs) {
    // this block's job: the last whose first block is at or before it
    int jb = 0;
    for (int q = 1; q < n_jobs; q++)
        if (jobs[q].tile_begin <= (int64_t)blockIdx.x) jb = q;
    const PoolJob &J = jobs[jb];
    const int64_t begin = ((int64_t)blockIdx.x - J.tile_begin) * kPoolTileSamples;
    const int64_t end = min(begin + kPoolTileSamples, (int64_t)(J.round + 1) * J.n_round);
    const TT *__restrict__ th = (const TT *)J.theta;
    const TO *__restrict__ L = (const TO *)J.lnL;
    TL *__restrict__ lw = (TL *)J.lw;
    const int r = J.round;
    const int64_t first_new = (int64_t)r * J.n_round;
    const double ln_rounds = log((double)(r + 1));
    cgmm *hist = (cgmm *)J.hist;
    // the mixture columns are the same for every proposal of the job
    MixCols mc{};
    if (r > 0) mc = mix_cols(hist[r]);
    double xm[kPoolSpt][7], lpm[kPoolSpt], m[kPoolSpt], sum[kPoolSpt];
    int q0[kPoolSpt];
#pragma unroll
    for (int k = 0; k < kPoolSpt; k++) {
        const int64_t i = begin + threadIdx.x + (int64_t)k * kDrawThreads;
        double x[7];
#pragma unroll
        for (int c = 0; c < 7; c++) x[c] = i < end ? (double)th[c * J.ld + i] : 0.0;
        mix_coords(mc, J.pr, x, xm[k], lpm[k]);
        const bool fresh = i >= first_new;
        m[k] = (fresh || i >= end) ? 0.0 : J.lmix[i];   // the prior's term, e^0, is in every sum
        sum[k] = 1.0;
        q0[k] = i >= end ? r + 1 : (fresh ? 1 : r);
    }
    const int qlo = end > first_new ? 1 : r;
    // the FP32 policy's pooled weights need FP32 relative accuracy only
    constexpr bool kFast = sizeof(TO) == 4;
    auto proposals = [&](auto D_) {
        constexpr int D = decltype(D_)::value;
        for (int q = qlo; q <= r; q++) {
            double t[kPoolSpt];
            mix_log_ratio<kPoolSpt, kFast, D>(hist[q], mc, xm, lpm, t);
#pragma unroll
            for (int k = 0; k < kPoolSpt; k++)
                if (q >= q0[k]) lse_add<kFast>(m[k], sum[k], t[k]);
        }
    };
    if (mc.d == 6)
        proposals(std::integral_constant<int, 6>{});
    else if (mc.d == 7)
        proposals(std::integral_constant<int, 7>{});
    else
        proposals(std::integral_constant<int, 0>{});
#pragma unroll
    for (int k = 0; k < kPoolSpt; k++) {
        const int64_t i = begin + threadIdx.x + (int64_t)k * kDrawThreads;
        if (i >= end) continue;
        const double lm = m[k] + log(sum[k]);
        J.lmix[i] = lm;
        lw[i] = (TL)((double)L[i] - lm + ln_rounds);
    }
}

}  // namespace

hipError_t launch_pool_mix(int policy, const PoolJob *d_jobs, int n_jobs, int64_t n_tiles, hipStream_t st) {
    if (n_tiles <= 0 || n_jobs <= 0) return hipSuccess;
    if (n_tiles > INT32_MAX) return hipErrorInvalidValue;
    const dim3 grid((unsigned)n_tiles), block(kDrawThreads);
    if (policy == kFP64)
        hipLaunchKernelGGL((k_pool_mix<double, double, double>), grid, block, 0, st, d_jobs, n_jobs);
    else if (policy == kFP32)
        hipLaunchKernelGGL((k_pool_mix<float, float, float>), grid, block, 0, st, d_jobs, n_jobs);
    else
        hipLaunchKernelGGL((k_pool_mix<float, double, double>), grid, block, 0, st, d_jobs, n_jobs);
    return hipGetLastError();
}

hipError_t launch_draw(int policy, const DrawJob *d_jobs, const Tile *d_tiles, int n_tiles, const DrawJob &single,
                       int64_t tile, bool mix, hipStream_t st) {
    if (n_tiles <= 0) return hipSuccess;
    if (policy == kFP64)
        launch_draw_t<double>(mix, d_jobs, d_tiles, n_tiles, single, tile, st);
    else
        launch_draw_t<float>(mix, d_jobs, d_tiles, n_tiles, single, tile, st);
    return hipGetLastError();
}

// ------------------------------------------------------------------ in-support mass
// Z_j of each job's mixture: the fraction of z_draws candidates of component j
// (Philox counter (i, 0x5A000000 + j, round, block)) that fall in the support.
namespace {

constexpr int kZThreads = 256;
constexpr int kZBlocks = 64;

__global__ void k_gmm_zero(const EmJob *__restrict__ jobs) {
    if (threadIdx.x < kMaxComp) jobs[blockIdx.z].zcount[threadIdx.x] = 0u;
}

__global__ void __launch_bounds__(kZThreads) k_gmm_inbox(const EmJob *__restrict__ jobs) {
    const EmJob &J = jobs[blockIdx.z];
    const GmmDev &g = *J.gmm;
    const int j = blockIdx.y;
    __shared__ uint32_t sacc[kZThreads];
    uint32_t acc = 0;
    if (j < g.n_comp) {
        const uint32_t k0 = (uint32_t)J.z_seed, k1 = (uint32_t)(J.z_seed >> 32);
        for (int64_t i = (int64_t)blockIdx.x * kZThreads + threadIdx.x; i < J.z_draws;
             i += (int64_t)gridDim.x * kZThreads) {
            uint32_t w[16];
#pragma unroll
            for (int b = 0; b < 4; b++) {
                U4 o = philox4x32_10(U4{(uint32_t)i, 0x5A000000u + (uint32_t)j, J.z_round, (uint32_t)b}, k0, k1);
                w[4 * b] = o.x; w[4 * b + 1] = o.y; w[4 * b + 2] = o.z; w[4 * b + 3] = o.w;
            }
            double th[7] = {0, 0, 0, J.pr.d_ref, 0, 0, 0};
            acc += gmm_candidate(g, J.pr, j, w, th) ? 1u : 0u;
        }
    }
    sacc[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kZThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sacc[threadIdx.x] += sacc[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && j < g.n_comp) atomicAdd(&J.zcount[j], sacc[0]);
}

__global__ void k_gmm_setz(const EmJob *__restrict__ jobs) {
    const EmJob &J = jobs[blockIdx.z];
    GmmDev *g = J.gmm;
    const int j = threadIdx.x;
    if (j < g->n_comp) {
        const double c = (double)J.zcount[j];
        g->lnZ[j] = log((c > 0 ? c : 0.5) / (double)J.z_draws);
    }
    __syncthreads();
    if (j != 0) return;
    // constants of the draw density: r_j = (1 - Z_j)^64, pi_j normalised
    double tot = 0.0;
    for (int q = 0; q < g->n_comp; q++) tot += g->w[q] > 0.0 ? g->w[q] : 0.0;
    const double eps = g->eps_def;
    double fb = eps;
    for (int q = 0; q < kMaxComp; q++) {
        if (q >= g->n_comp || !(g->w[q] > 0.0) || !(tot > 0.0)) {
            g->lnc[q] = -INFINITY;
            continue;
        }
        const double pi = g->w[q] / tot, z = exp(g->lnZ[q]);
        const double lr = (double)kMaxAttempts * log1p(-(z < 1.0 ? z : 1.0));   // ln r_j
        fb += (1.0 - eps) * pi * exp(lr);
        // ln(1 - r_j), accurate on both sides of r_j = 1/2
        const double l1mr = lr > -0.69314718055994531 ? log(-expm1(lr)) : log1p(-exp(lr));
        g->lnc[q] = log1p(-eps) + log(pi) + l1mr - g->lnZ[q];
    }
    g->ln_fb = fb > 0.0 ? log(fb) : -INFINITY;
}

}  // namespace

hipError_t launch_gmm_mass(const EmJob *d_jobs, int n_jobs, hipStream_t st) {
    if (n_jobs <= 0) return hipSuccess;
    if (n_jobs > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gmm_zero, dim3(1, 1, n_jobs), dim3(64), 0, st, d_jobs);
    hipLaunchKernelGGL(k_gmm_inbox, dim3(kZBlocks, kMaxComp, n_jobs), dim3(kZThreads), 0, st, d_jobs);
    hipLaunchKernelGGL(k_gmm_setz, dim3(1, 1, n_jobs), dim3(64), 0, st, d_jobs);
    return hipGetLastError();
}

}  // namespace ile
