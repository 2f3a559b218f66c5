// Gaussian-mixture sampling prior (paper: GMM sampling priors for a chosen
// subset of dimensions, refit from weighted samples).  All steps run on the
// device in FP64 with deterministic fixed-order reductions:
//
//   factor : Cholesky L_j of Sigma_j, L_j^{-1}, sum ln diag(L_j), ln pi_j;
//   weights: w_i = e^{beta (lw_i - max lw)}, beta the tempering exponent;
//   init   : means at the n_comp highest-weight distinct samples (among the
//            2 n_comp highest), common covariance = weighted second moment of
//            the differences (wrapped for periodic columns) about the best
//            sample minus the outer product of their mean, plus the floor;
//   EM     : responsibilities from the untruncated components
//            pi_j N(wrap(x - mu_j); Sigma_j); means from the wrapped offsets
//            about the current mu_j; covariances centred on the new offsets;
//            Sigma_j += 1e-8 diag(range^2).  A component with no weight keeps
//            its mean and covariance.
//
// Every kernel serves a batch of jobs (blockIdx.z = job): the refits of all
// jobs of a serving pass are one launch per stage.  Per-sample stages tile
// each job's samples (kEmTile per block); per-job stages are one block each.
#include <type_traits>

#include "ile_internal.h"

#include <algorithm>

namespace ile {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kEmThreads = 256;
constexpr int kTopThreads = 128;
constexpr int kTopK = 2 * kMaxComp;
constexpr int64_t kEmTile = 8192;
constexpr int kBetaGrid = 48;   // beta_k = 2^(-k/4)
constexpr int kBetaChunk = 8;   // grid values per block reduction

// Work buffer of one job (doubles): scalars, old means, offsets, then the
// per-tile partials of each stage and the responsibilities.
constexpr int kWMax = 0, kWCount = 1, kWBeta = 2, kWPart = 64;
struct EmLayout {
    int64_t nblk;
    size_t stat, init, beta, max, top, R, total;
};
__host__ __device__ inline EmLayout em_layout(int64_t n) {
    EmLayout L;
    L.nblk = (n + kEmTile - 1) / kEmTile;
    L.stat = kWPart;
    L.init = L.stat + (size_t)kMaxComp * L.nblk * 36;
    L.beta = L.init + (size_t)L.nblk * 36;
    L.max = L.beta + (size_t)L.nblk * 2 * kBetaGrid;
    L.top = L.max + (size_t)L.nblk * 2;
    L.R = L.top + (size_t)L.nblk * 2 * kTopK;
    L.total = L.R + (size_t)kMaxComp * n;
    return L;
}

__device__ __forceinline__ double col_period(int col) {
    return (col == 0 || col == 5) ? 2 * kPi : (col == 6 ? kPi : 0.0);
}
__device__ __forceinline__ double col_range(const PriorDev &pr, int col) {
    switch (col) {
    case 0: return 2 * kPi;
    case 1: return kPi;
    case 2: return 2 * pr.t_window;
    case 3: return pr.d_max - pr.d_min;
    case 4: return 2.0;
    case 5: return 2 * kPi;
    default: return kPi;
    }
}
// wrapped difference in (-P/2, P/2]: d - P floor(d/P), folded; for |d| < P
// (both ends inside one period) the same value without the division
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

__device__ void factor_one(GmmDev &g, int j) {
    const int d = g.n_dim;
    double L[7][7], Li[7][7];
    for (int a = 0; a < 7; a++)
        for (int b = 0; b < 7; b++) { L[a][b] = 0.0; Li[a][b] = 0.0; }
    bool ok = true;
    for (int c = 0; c < d; c++) {
        double s = g.cov[j][c][c];
        for (int k = 0; k < c; k++) s -= L[c][k] * L[c][k];
        if (!(s > 0.0)) { ok = false; s = 1e-300; }
        L[c][c] = sqrt(s);
        for (int r = c + 1; r < d; r++) {
            double t = g.cov[j][r][c];
            for (int k = 0; k < c; k++) t -= L[r][k] * L[c][k];
            L[r][c] = t / L[c][c];
        }
    }
    // inverse of the lower factor, column by column (forward substitution)
    for (int c = 0; c < d; c++) {
        for (int r = 0; r < d; r++) {
            double t = (r == c) ? 1.0 : 0.0;
            for (int k = 0; k < r; k++) t -= L[r][k] * Li[k][c];
            Li[r][c] = (r < c) ? 0.0 : t / L[r][r];
        }
    }
    double ld = 0.0;
    for (int c = 0; c < d; c++) ld += log(L[c][c]);
    for (int a = 0; a < 7; a++)
        for (int b = 0; b < 7; b++) { g.L[j][a][b] = L[a][b]; g.Linv[j][a][b] = Li[a][b]; }
    g.logdet_half[j] = ld;
    g.logw[j] = (g.w[j] > 0.0) ? log(g.w[j]) : -INFINITY;
    if (!ok) g.valid = 0;
}

template <class TT>
__device__ __forceinline__ double load_col(const TT *th, int64_t ld, int col, int64_t i) {
    return (double)th[col * ld + i];
}

// Column col of sample i in the mixture's coordinates (phase shear of column 6).
template <class TT>
__device__ __forceinline__ double load_mix(const TT *th, int64_t ld, int col, int64_t i, int shear) {
    const double v = (double)th[col * ld + i];
    if (col != 6 || shear == 0) return v;
    return shear_phase(v, (double)th[5 * ld + i], shear);
}

__device__ __forceinline__ bool finite_d(double v) { return v > -INFINITY && v < INFINITY; }

__device__ __forceinline__ double sample_weight(double lwv, double mlw, double beta) {
    return finite_d(lwv) ? exp(beta * (lwv - mlw)) : 0.0;
}

// Block sum of NV doubles per thread into out[0..NV): a butterfly within
// each wave (lane 0's association order is fixed), then the waves in order.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *out) {
    __shared__ double red[kEmThreads / 64][NV];
#pragma unroll
    for (int c = 0; c < NV; c++) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[c] += __shfl_xor(v[c], off, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int c = 0; c < NV; c++) red[w][c] = v[c];
    }
    __syncthreads();
    for (int c = threadIdx.x; c < NV; c += blockDim.x) {
        double s = red[0][c];
        for (int q = 1; q < kEmThreads / 64; q++) s += red[q][c];
        out[c] = s;
    }
    __syncthreads();
}

// ------------------------------------------------------------- weights
// per tile: max of the finite lw and their count
template <class TL>
__global__ void __launch_bounds__(kEmThreads) k_em_scan(const EmJob *__restrict__ jobs) {
    const EmJob &J = jobs[blockIdx.z];
    const EmLayout Lo = em_layout(J.n);
    if (blockIdx.x >= Lo.nblk) return;
    const TL *__restrict__ lw = (const TL *)J.lw;
    const int64_t b0 = (int64_t)blockIdx.x * kEmTile, b1 = min(b0 + kEmTile, J.n);
    double m = -INFINITY, c = 0.0;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += kEmThreads) {
        const double v = (double)lw[i];
        if (finite_d(v)) {
            m = fmax(m, v);
            c += 1.0;
        }
    }
    __shared__ double sm[kEmThreads], sc[kEmThreads];
    sm[threadIdx.x] = m;
    sc[threadIdx.x] = c;
    __syncthreads();
    for (int w = kEmThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
            sc[threadIdx.x] += sc[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        J.work[Lo.max + 2 * blockIdx.x] = sm[0];
        J.work[Lo.max + 2 * blockIdx.x + 1] = sc[0];
    }
}

__global__ void k_em_scan_final(const EmJob *__restrict__ jobs) {
    const EmJob &J = jobs[blockIdx.z];
    if (threadIdx.x != 0) return;
    const EmLayout Lo = em_layout(J.n);
    double m = -INFINITY, c = 0.0;
    for (int64_t b = 0; b < Lo.nblk; b++) {
        m = fmax(m, J.work[Lo.max + 2 * b]);
        c += J.work[Lo.max + 2 * b + 1];
    }
    J.work[kWMax] = m;
    J.work[kWCount] = c;
    J.work[kWBeta] = 1.0;
}

// Tempering exponent: the largest beta_k = 2^(-k/4) whose tempered weights
// have (sum w^beta)^2 / sum w^(2 beta) >= frac * (finite samples).  Per tile:
// the 48 pairs (sum w^beta_k, sum w^(2 beta_k)).
template <class TL>
__global__ void __launch_bounds__(kEmThreads) k_em_beta(const EmJob *__restrict__ jobs) {
    const EmJob &J = jobs[blockIdx.z];
    const EmLayout Lo = em_layout(J.n);
    if (blockIdx.x >= Lo.nblk || !(J.temper > 0.0)) return;
    const TL *__restrict__ lw = (const TL *)J.lw;
    const double mlw = J.work[kWMax];
    constexpr int kPer = (int)(kEmTile / kEmThreads);
    const int64_t b0 = (int64_t)blockIdx.x * kEmTile;
    double x[kPer];
#pragma unroll
    for (int s = 0; s < kPer; s++) {
        const int64_t i = b0 + threadIdx.x + (int64_t)s * kEmThreads;
        const double v = i < J.n ? (double)lw[i] : -INFINITY;
        x[s] = finite_d(v) ? v - mlw : -INFINITY;
    }
    double *out = J.work + Lo.beta + (size_t)blockIdx.x * 2 * kBetaGrid;
    for (int c0 = 0; c0 < kBetaGrid; c0 += kBetaChunk) {
        double acc[2 * kBetaChunk];
#pragma unroll
        for (int q = 0; q < kBetaChunk; q++) {
            const double b = exp2(-(double)(c0 + q) / 4.0);
            double s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int s = 0; s < kPer; s++) {
                const double e = exp(b * x[s]);
                s1 += e;
                s2 += e * e;
            }
            acc[2 * q] = s1;
            acc[2 * q + 1] = s2;
        }
        block_sum<2 * kBetaChunk>(acc, out + 2 * c0);
    }
}

__global__ void k_em_beta_final(const EmJob *__restrict__ jobs) {
    const EmJob &J = jobs[blockIdx.z];
    if (threadIdx.x != 0 || !(J.temper > 0.0)) return;
    const EmLayout Lo = em_layout(J.n);
    const double target = J.temper * J.work[kWCount];
    double beta = exp2(-(double)(kBetaGrid - 1) / 4.0);
    for (int k = 0; k < kBetaGrid; k++) {
        double s1 = 0.0, s2 = 0.0;
        for (int64_t b = 0; b < Lo.nblk; b++) {
            s1 += J.work[Lo.beta + (size_t)b * 2 * kBetaGrid + 2 * k];
            s2 += J.work[Lo.beta + (size_t)b * 2 * kBetaGrid + 2 * k + 1];
        }
        if (s1 * s1 / s2 >= target) {
            beta = exp2(-(double)k / 4.0);
            break;
        }
    }
    J.work[kWBeta] = beta;
}

// ---------------------------------------------------------------- first fit
struct Cand {
    double v;
    int64_t i;
};
__device__ __forceinline__ bool better(const Cand &a, const Cand &b) {
    return a.v > b.v || (a.v == b.v && a.i < b.i);
}
__device__ __forceinline__ void merge_top(const Cand *A, const Cand *B, Cand *out) {
    int ia = 0, ib = 0;
    for (int k = 0; k < kTopK; k++) out[k] = better(B[ib], A[ia]) ? B[ib++] : A[ia++];
}

// per tile: the kTopK highest finite lw (ties: lower index first)
template <class TL>
__global__ void __launch_bounds__(kTopThreads) k_em_top(const EmJob *__restrict__ jobs) {
    const EmJob &J = jobs[blockIdx.z];
    const EmLayout Lo = em_layout(J.n);
    if (!J.first || blockIdx.x >= Lo.nblk) return;
    const TL *__restrict__ lw = (const TL *)J.lw;
    __shared__ Cand lists[kTopThreads][kTopK];
    Cand loc[kTopK];
    for (int k = 0; k < kTopK; k++) loc[k] = Cand{-INFINITY, INT64_MAX};
    const int64_t b0 = (int64_t)blockIdx.x * kEmTile, b1 = min(b0 + kEmTile, J.n);
    for (int64_t i = b0 + threadIdx.x; i < b1; i += kTopThreads) {
        const double v = (double)lw[i];
        if (!finite_d(v)) continue;
        Cand c{v, i};
        if (!better(c, loc[kTopK - 1])) continue;
        int k = kTopK - 1;
        while (k > 0 && better(c, loc[k - 1])) { loc[k] = loc[k - 1]; k--; }
        loc[k] = c;
    }
    for (int k = 0; k < kTopK; k++) lists[threadIdx.x][k] = loc[k];
    __syncthreads();
    for (int w = kTopThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            Cand out[kTopK];
            merge_top(lists[threadIdx.x], lists[threadIdx.x + w], out);
            for (int k = 0; k < kTopK; k++) lists[threadIdx.x][k] = out[k];
        }
        __syncthreads();
    }
    if (threadIdx.x < kTopK) {
        double *o = J.work + Lo.top + (size_t)blockIdx.x * 2 * kTopK;
        o[2 * threadIdx.x] = lists[0][threadIdx.x].v;
        o[2 * threadIdx.x + 1] = (double)lists[0][threadIdx.x].i;
    }
}

// merge the tiles' lists; reset the mixture and place the means at the
// highest-weight distinct samples
template <class TT>
__global__ void k_em_top_final(const EmJob *__restrict__ jobs) {
    const EmJob &J = jobs[blockIdx.z];
    if (!J.first) return;
    GmmDev *g = J.gmm;
    {   // zero the whole state
        double *p = (double *)g;
        const size_t nd = sizeof(GmmDev) / sizeof(double);
        for (size_t k = threadIdx.x; k < nd; k += blockDim.x) p[k] = 0.0;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const EmLayout Lo = em_layout(J.n);
    Cand cur[kTopK], nxt[kTopK], add[kTopK];
    for (int k = 0; k < kTopK; k++) cur[k] = Cand{-INFINITY, INT64_MAX};
    for (int64_t b = 0; b < Lo.nblk; b++) {
        const double *o = J.work + Lo.top + (size_t)b * 2 * kTopK;
        for (int k = 0; k < kTopK; k++) add[k] = Cand{o[2 * k], (int64_t)o[2 * k + 1]};
        merge_top(cur, add, nxt);
        for (int k = 0; k < kTopK; k++) cur[k] = nxt[k];
    }
    g->n_dim = J.n_dim;
    for (int a = 0; a < 7; a++) g->dims[a] = a < J.n_dim ? J.dims[a] : 0;
    g->eps_def = J.eps_def;
    g->valid = 1;
    const TT *th = (const TT *)J.theta;
    const int d = J.n_dim, nc = J.n_comp;
    // phase shear from the inclination of the best sample: face-on
    // (cos iota >= 1/2, where the m = +2 end of each multiplet dominates) the
    // ridge runs along psi + phi_c, face-off along psi - phi_c; in between
    // there is no single ridge and the phases stay as they are
    g->shear = 0;
    if (J.shear_auto && cur[0].v > -INFINITY) {
        const double ci = load_col(th, J.ld, 4, cur[0].i);
        g->shear = ci >= 0.5 ? 1 : (ci <= -0.5 ? -1 : 0);
    }
    // candidates: the 2 n_comp highest-weight samples (kTopK = 2 kMaxComp
    // holds them for every n_comp), scanned in that order
    const int ncand = 2 * nc < kTopK ? 2 * nc : kTopK;
    int got = 0;
    for (int k = 0; k < ncand && got < nc; k++) {
        if (!(cur[k].v > -INFINITY)) break;
        double x[7];
        for (int a = 0; a < d; a++) x[a] = load_mix(th, J.ld, J.dims[a], cur[k].i, g->shear);
        bool dup = false;
        for (int q = 0; q < got && !dup; q++) {
            bool same = true;
            for (int a = 0; a < d; a++) same = same && (x[a] == g->mean[q][a]);
            dup = same;
        }
        if (dup) continue;
        for (int a = 0; a < d; a++) g->mean[got][a] = x[a];
        got++;
    }
    if (got == 0) got = 1;  // no finite weight: keep the first mean as is
    for (int q = got; q < nc; q++)
        for (int a = 0; a < d; a++) g->mean[q][a] = g->mean[got - 1][a];
    g->n_comp = nc;
}

// first fit: weighted moments of the differences about the best sample
template <class TT, class TL>
__global__ void __launch_bounds__(kEmThreads) k_em_init(const EmJob *__restrict__ jobs) {
    const EmJob &J = jobs[blockIdx.z];
    const EmLayout Lo = em_layout(J.n);
    if (!J.first || blockIdx.x >= Lo.nblk) return;
    const TT *__restrict__ th = (const TT *)J.theta;
    const TL *__restrict__ lw = (const TL *)J.lw;
    const GmmDev *g = J.gmm;
    const int d = g->n_dim;
    const double mlw = J.work[kWMax], beta = J.work[kWBeta];
    double acc[36];
    for (int c = 0; c < 36; c++) acc[c] = 0.0;
    const int64_t b0 = (int64_t)blockIdx.x * kEmTile, b1 = min(b0 + kEmTile, J.n);
    for (int64_t i = b0 + threadIdx.x; i < b1; i += kEmThreads) {
        const double w = sample_weight((double)lw[i], mlw, beta);
        double x[7];
#pragma unroll
        for (int a = 0; a < 7; a++) {
            x[a] = 0.0;
            if (a < d) {
                const int col = g->dims[a];
                x[a] = wrapd(load_mix(th, J.ld, col, i, g->shear) - g->mean[0][a], col_period(col));
            }
        }
        acc[0] += w;
        int k = 1;
#pragma unroll
        for (int a = 0; a < 7; a++) acc[k++] += w * x[a];
#pragma unroll
        for (int a = 0; a < 7; a++)
#pragma unroll
            for (int b = 0; b <= a; b++) acc[k++] += w * x[a] * x[b];
    }
    block_sum<36>(acc, J.work + Lo.init + (size_t)blockIdx.x * 36);
}

__global__ void k_em_init_final(const EmJob *__restrict__ jobs) {
    const EmJob &J = jobs[blockIdx.z];
    if (!J.first || threadIdx.x != 0) return;
    const EmLayout Lo = em_layout(J.n);
    GmmDev *g = J.gmm;
    double s[36];
    for (int c = 0; c < 36; c++) s[c] = 0.0;
    for (int64_t b = 0; b < Lo.nblk; b++)
        for (int c = 0; c < 36; c++) s[c] += J.work[Lo.init + (size_t)b * 36 + c];
    const int d = g->n_dim;
    double mu[7];
    for (int a = 0; a < 7; a++) mu[a] = (a < d) ? s[1 + a] / s[0] : 0.0;
    double cov[7][7];
    int k = 8;
    for (int a = 0; a < 7; a++)
        for (int b = 0; b <= a; b++) {
            const double v = s[k++] / s[0] - mu[a] * mu[b];
            cov[a][b] = v;
            cov[b][a] = v;
        }
    for (int a = 0; a < d; a++) {
        const double r = col_range(J.pr, g->dims[a]);
        cov[a][a] += 1e-8 * r * r;
    }
    for (int j = 0; j < g->n_comp; j++) {
        g->w[j] = 1.0 / g->n_comp;
        for (int a = 0; a < 7; a++)
            for (int b = 0; b < 7; b++) g->cov[j][a][b] = (a < d && b < d) ? cov[a][b] : 0.0;
    }
}

// only_first: factor just the jobs that had a first fit
__global__ void k_gmm_factor(const EmJob *__restrict__ jobs, int only_first) {
    const EmJob &J = jobs[blockIdx.z];
    if (only_first && !J.first) return;
    GmmDev *g = J.gmm;
    const int j = threadIdx.x;
    if (j == 0) g->valid = 1;
    __syncthreads();
    if (j < g->n_comp) factor_one(*g, j);
}

// ------------------------------------------------------------------ EM
// Responsibilities times weights, R_ij = w_i pi_j N_j(x_i) / sum_k pi_k N_k(x_i).
// The block stages its job's mixture (means, packed inverse factors and the
// constant ln pi_j - ln det^(1/2) - d/2 ln 2pi) in LDS.
// The EM kernels take the mixture's dimension count D as a compile-time
// constant for the common counts (six with the distance integrated, seven
// otherwise; D = 0: the count read at run time), which removes the
// per-dimension tests from their unrolled loops.  A kernel compiled for D
// checks the mixture's count and runs the general body for any other.
template <class TT, class TL, int D>
__device__ __forceinline__ void em_resp_body(const EmJob &J, double (&s_mean)[kMaxComp][7],
                                             double (&s_li)[kMaxComp][28], double (&s_c)[kMaxComp],
                                             double (&s_lr)[kMaxComp][kEmThreads]) {
    const EmLayout Lo = em_layout(J.n);
    const TT *__restrict__ th = (const TT *)J.theta;
    const TL *__restrict__ lw = (const TL *)J.lw;
    const GmmDev *g = J.gmm;
    double *R = J.work + Lo.R;
    const int64_t n = J.n;
    const int d = D > 0 ? D : g->n_dim, nc = g->n_comp;
    for (int t = threadIdx.x; t < kMaxComp * 28; t += kEmThreads) {
        const int j = t / 28, k = t % 28;
        int a = 0;
        while ((a + 1) * (a + 2) / 2 <= k) a++;
        const int b = k - a * (a + 1) / 2;
        s_li[j][k] = j < nc ? g->Linv[j][a][b] : 0.0;
        if (k < 7) s_mean[j][k] = j < nc ? g->mean[j][k] : 0.0;
        if (k == 0)
            s_c[j] = (j < nc && g->logw[j] != -INFINITY)
                         ? g->logw[j] - g->logdet_half[j] - 0.5 * d * log(2 * kPi)
                         : -INFINITY;
    }
    __syncthreads();
    int col[7];
    double P[7];
#pragma unroll
    for (int a = 0; a < 7; a++) {
        col[a] = a < d ? g->dims[a] : 0;
        P[a] = col_period(col[a]);
    }
    const int shear = g->shear;
    const double mlw = J.work[kWMax], beta = J.work[kWBeta];
    for (int64_t i = (int64_t)blockIdx.x * kEmThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kEmThreads) {
        const double w = sample_weight((double)lw[i], mlw, beta);
        double x[7];
#pragma unroll
        for (int a = 0; a < 7; a++) x[a] = load_col(th, J.ld, col[a], i);   // col[a] valid: loads in flight together
        if (shear) {
            const double phi = (double)th[5 * J.ld + i];
#pragma unroll
            for (int a = 0; a < 7; a++)
                if (a < d && col[a] == 6) x[a] = shear_phase(x[a], phi, shear);
        }
#pragma unroll
        for (int a = 0; a < 7; a++) x[a] = a < d ? x[a] : 0.0;
        double m = -INFINITY;
#pragma unroll 1
        for (int j = 0; j < nc; j++) {
            double lrj = -INFINITY;
            if (s_c[j] != -INFINITY) {
                double df[7];
#pragma unroll
                for (int a = 0; a < 7; a++) df[a] = a < d ? wrapd(x[a] - s_mean[j][a], P[a]) : 0.0;
                double q = 0.0;
                int k = 0;
#pragma unroll
                for (int a = 0; a < 7; a++) {
                    double y = 0.0;
#pragma unroll
                    for (int b = 0; b <= a; b++) y += s_li[j][k++] * df[b];
                    q += a < d ? y * y : 0.0;
                }
                lrj = s_c[j] - 0.5 * q;
                m = fmax(m, lrj);
            }
            s_lr[j][threadIdx.x] = lrj;
        }
        double sum = 0.0;
#pragma unroll 1
        for (int j = 0; j < nc; j++) {
            const double l = s_lr[j][threadIdx.x];
            const double e = (l == -INFINITY) ? 0.0 : exp(l - m);
            s_lr[j][threadIdx.x] = e;
            sum += e;
        }
        const double scale = (m > -INFINITY) ? w / sum : 0.0;
#pragma unroll 1
        for (int j = 0; j < nc; j++) R[(size_t)j * n + i] = s_lr[j][threadIdx.x] * scale;
    }
}

template <class TT, class TL, int D>
__global__ void __launch_bounds__(kEmThreads) k_em_resp(const EmJob *__restrict__ jobs) {
    const EmJob &J = jobs[blockIdx.z];
    __shared__ double s_mean[kMaxComp][7], s_li[kMaxComp][28], s_c[kMaxComp];
    __shared__ double s_lr[kMaxComp][kEmThreads];   // per-thread ln pi_j N_j, then e^{. - max}
    if (D > 0 && J.gmm->n_dim == D)
        em_resp_body<TT, TL, D>(J, s_mean, s_li, s_c, s_lr);
    else
        em_resp_body<TT, TL, 0>(J, s_mean, s_li, s_c, s_lr);
}

// W_j, first and second moments of the offsets D = wrap(x - mu_j) about the
// current mean, per tile (one pass: the covariance centred on the mean offset
// m_j is S2/W - m_j m_j^T, the same quantity as the centred two-pass sum)
template <class TT, int D>
__device__ __forceinline__ void em_stat_body(const EmJob &J) {
    const EmLayout Lo = em_layout(J.n);
    const GmmDev *g = J.gmm;
    const int j = blockIdx.y;
    const TT *__restrict__ th = (const TT *)J.theta;
    const double *R = J.work + Lo.R;
    const int d = D > 0 ? D : g->n_dim;
    double mu[7], P[7];
    int col[7];
#pragma unroll
    for (int a = 0; a < 7; a++) {
        col[a] = a < d ? g->dims[a] : 0;
        mu[a] = a < d ? g->mean[j][a] : 0.0;
        P[a] = col_period(col[a]);
    }
    const int shear = g->shear;
    double acc[36];
#pragma unroll
    for (int c = 0; c < 36; c++) acc[c] = 0.0;
    const int64_t b0 = (int64_t)blockIdx.x * kEmTile, b1 = min(b0 + kEmTile, J.n);
    for (int64_t i = b0 + threadIdx.x; i < b1; i += kEmThreads) {
        const double r = R[(size_t)j * J.n + i];
        // all seven column loads first (col[a] is a valid column, 0 beyond
        // d), so that they are in flight together
        double v[7];
#pragma unroll
        for (int a = 0; a < 7; a++) v[a] = load_col(th, J.ld, col[a], i);
        if (shear) {
            const double phi = (double)th[5 * J.ld + i];
#pragma unroll
            for (int a = 0; a < 7; a++)
                if (a < d && col[a] == 6) v[a] = shear_phase(v[a], phi, shear);
        }
        double x[7];
#pragma unroll
        for (int a = 0; a < 7; a++) x[a] = (a < d) ? wrapd(v[a] - mu[a], P[a]) : 0.0;
        acc[0] += r;
        int k = 1;
        // with D fixed the moments of absent dimensions are skipped: they
        // stay 0, as the sums of r x 0 they replace
#pragma unroll
        for (int a = 0; a < 7; a++, k++)
            if (D == 0 || a < D) acc[k] += r * x[a];
#pragma unroll
        for (int a = 0; a < 7; a++)
#pragma unroll
            for (int b = 0; b <= a; b++, k++)
                if (D == 0 || a < D) acc[k] += r * x[a] * x[b];
    }
    block_sum<36>(acc, J.work + Lo.stat + ((size_t)j * Lo.nblk + blockIdx.x) * 36);
}

template <class TT, int D>
__global__ void __launch_bounds__(kEmThreads) k_em_stat(const EmJob *__restrict__ jobs) {
    const EmJob &J = jobs[blockIdx.z];
    const EmLayout Lo = em_layout(J.n);
    if (blockIdx.x >= Lo.nblk || (int)blockIdx.y >= J.gmm->n_comp) return;
    if (D > 0 && J.gmm->n_dim == D)
        em_stat_body<TT, D>(J);
    else
        em_stat_body<TT, 0>(J);
}

// M-step: weights, means (old mean + offset, wrapped into the period),
// covariances + floor, then the factorisation
__global__ void k_em_update(const EmJob *__restrict__ jobs) {
    const EmJob &J = jobs[blockIdx.z];
    const EmLayout Lo = em_layout(J.n);
    GmmDev *g = J.gmm;
    const int j = threadIdx.x;
    __shared__ double W[kMaxComp];
    const int nc = g->n_comp, d = g->n_dim;
    double s[36];
    for (int c = 0; c < 36; c++) s[c] = 0.0;
    if (j < nc)
        for (int64_t b = 0; b < Lo.nblk; b++)
            for (int c = 0; c < 36; c++) s[c] += J.work[Lo.stat + ((size_t)j * Lo.nblk + b) * 36 + c];
    if (j < kMaxComp) W[j] = (j < nc) ? s[0] : 0.0;
    if (j == 0) g->valid = 1;
    __syncthreads();
    if (j >= nc) return;
    double tot = 0.0;
    for (int q = 0; q < nc; q++) tot += W[q];
    g->w[j] = s[0] / tot;
    if (s[0] > 0.0) {
        const double Wj = s[0];
        double m[7];
        for (int a = 0; a < 7; a++) m[a] = a < d ? s[1 + a] / Wj : 0.0;
        int k = 8;
        for (int a = 0; a < 7; a++)
            for (int b = 0; b <= a; b++) {
                const double v = (a < d && b < d) ? s[k] / Wj - m[a] * m[b] : 0.0;
                k++;
                g->cov[j][a][b] = v;
                g->cov[j][b][a] = v;
            }
        for (int a = 0; a < d; a++) {
            const double rg = col_range(J.pr, g->dims[a]);
            g->cov[j][a][a] += 1e-8 * rg * rg;
            double mu = g->mean[j][a] + m[a];
            const double P = col_period(g->dims[a]);
            if (P > 0.0) mu = mu - P * floor(mu / P);
            g->mean[j][a] = mu;
        }
    }
    factor_one(*g, j);
}

template <class TT, class TL, int D>
void launch_em_t(const EmJob *d_jobs, int n_jobs, int64_t nblk_max, int64_t rblk, bool any_first, int n_iter,
                 hipStream_t st) {
    const dim3 jz(1, 1, n_jobs), tiles(nblk_max, 1, n_jobs);
    hipLaunchKernelGGL((k_em_scan<TL>), tiles, dim3(kEmThreads), 0, st, d_jobs);
    hipLaunchKernelGGL(k_em_scan_final, jz, dim3(64), 0, st, d_jobs);
    hipLaunchKernelGGL((k_em_beta<TL>), tiles, dim3(kEmThreads), 0, st, d_jobs);
    hipLaunchKernelGGL(k_em_beta_final, jz, dim3(64), 0, st, d_jobs);
    if (any_first) {
        hipLaunchKernelGGL((k_em_top<TL>), tiles, dim3(kTopThreads), 0, st, d_jobs);
        hipLaunchKernelGGL((k_em_top_final<TT>), jz, dim3(256), 0, st, d_jobs);
        hipLaunchKernelGGL((k_em_init<TT, TL>), tiles, dim3(kEmThreads), 0, st, d_jobs);
        hipLaunchKernelGGL(k_em_init_final, jz, dim3(64), 0, st, d_jobs);
        hipLaunchKernelGGL(k_gmm_factor, jz, dim3(64), 0, st, d_jobs, 1);
    }
    const dim3 comp(nblk_max, kMaxComp, n_jobs);
    for (int it = 0; it < n_iter; it++) {
        hipLaunchKernelGGL((k_em_resp<TT, TL, D>), dim3(rblk, 1, n_jobs), dim3(kEmThreads), 0, st, d_jobs);
        hipLaunchKernelGGL((k_em_stat<TT, D>), comp, dim3(kEmThreads), 0, st, d_jobs);
        hipLaunchKernelGGL(k_em_update, jz, dim3(64), 0, st, d_jobs);
    }
}

}  // namespace

size_t em_work_bytes(int64_t n) { return em_layout(n).total * sizeof(double); }

hipError_t launch_gmm_factor(const EmJob *d_jobs, int n_jobs, hipStream_t st) {
    if (n_jobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gmm_factor, dim3(1, 1, n_jobs), dim3(64), 0, st, d_jobs, 0);
    return hipGetLastError();
}

hipError_t launch_em_batch(int policy, const EmJob *d_jobs, const EmJob *h_jobs, int n_jobs, int n_iter,
                           hipStream_t st) {
    if (n_jobs <= 0) return hipSuccess;
    if (n_jobs > 65535) return hipErrorInvalidValue;
    int64_t nblk_max = 1, nmax = 1;
    bool any_first = false;
    for (int k = 0; k < n_jobs; k++) {
        if (h_jobs[k].n < 1) return hipErrorInvalidValue;
        nblk_max = std::max<int64_t>(nblk_max, em_layout(h_jobs[k].n).nblk);
        nmax = std::max<int64_t>(nmax, h_jobs[k].n);
        any_first = any_first || h_jobs[k].first;
    }
    const int64_t rblk = std::min<int64_t>((nmax + kEmThreads - 1) / kEmThreads, 4096);
    if (nblk_max > INT32_MAX) return hipErrorInvalidValue;
    // the mixtures' dimension count, when every job of the batch shares it
    // (each mixture takes its job's default columns; the kernels check)
    int dim = h_jobs[0].n_dim;
    for (int k = 1; k < n_jobs; k++)
        if (h_jobs[k].n_dim != dim) dim = 0;
    auto go = [&](auto D_) {
        constexpr int D = decltype(D_)::value;
        if (policy == kFP64)
            launch_em_t<double, double, D>(d_jobs, n_jobs, nblk_max, rblk, any_first, n_iter, st);
        else if (policy == kFP32)
            launch_em_t<float, float, D>(d_jobs, n_jobs, nblk_max, rblk, any_first, n_iter, st);
        else
            launch_em_t<float, double, D>(d_jobs, n_jobs, nblk_max, rblk, any_first, n_iter, st);
    };
    if (dim == 6)
        go(std::integral_constant<int, 6>{});
    else if (dim == 7)
        go(std::integral_constant<int, 7>{});
    else
        go(std::integral_constant<int, 0>{});
    return hipGetLastError();
}

}  // namespace ile
