// Gaussian-mixture sampling prior (paper: GMM sampling priors for a chosen
// subset of dimensions, refit from weighted samples).  All steps run on the
// device in FP64 with deterministic fixed-order reductions:
//
//   factor : Cholesky L_j of Sigma_j, L_j^{-1}, sum ln diag(L_j), ln pi_j;
//   init   : means at the n_comp highest-weight distinct samples (among the
//            2 n_comp highest), common covariance = weighted second moment of
//            the differences (wrapped for periodic columns) about the best
//            sample minus the outer product of their mean, plus the floor;
//   EM     : weights w_i = e^{lw_i - max lw}; responsibilities from the
//            untruncated components pi_j N(wrap(x - mu_j); Sigma_j); means
//            from the wrapped offsets about the current mu_j; covariances
//            centred on the new offsets; Sigma_j += 1e-8 diag(range^2).  A
//            component with no weight keeps its mean and covariance.
#include "ile_internal.h"

namespace ile {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kEmThreads = 256;
constexpr int kTopThreads = 128;
constexpr int kTopK = 2 * kMaxComp;
constexpr int64_t kEmTile = 4096;

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
__device__ __forceinline__ double wrapd(double d, double P) {
    if (P <= 0.0) return d;
    double r = d - P * floor(d / P);
    return r > 0.5 * P ? r - P : r;
}

// Work buffer (doubles):
//   [0] max lw   [1] index of the max   [2] tempering exponent beta
//   [8 .. 8+16*8) old means   [256 ..) per-component offsets m_j (16*8)
//   [512 ..) partials
constexpr int kWMax = 0, kWBeta = 2, kWOldMean = 8, kWOff = 256, kWPart = 512;
constexpr int kBetaGrid = 48;   // beta_k = 2^(-k/4)

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

__global__ void k_gmm_factor(GmmDev *g) {
    const int j = threadIdx.x;
    if (j == 0) g->valid = 1;
    __syncthreads();
    if (j < g->n_comp) factor_one(*g, j);
}

template <class TT>
__device__ __forceinline__ double load_col(const TT *th, int64_t ld, int col, int64_t i) {
    return (double)th[col * ld + i];
}

// ---------------------------------------------------------------- top-k
struct Cand {
    double v;
    int64_t i;
};
__device__ __forceinline__ bool better(const Cand &a, const Cand &b) {
    return a.v > b.v || (a.v == b.v && a.i < b.i);
}

template <class TT, class TL>
__global__ void __launch_bounds__(kTopThreads)
    k_em_top(const TT *__restrict__ th, int64_t ld, const TL *__restrict__ lw, int64_t n, GmmDev *g, int n_comp,
             double *work) {
    __shared__ Cand lists[kTopThreads][kTopK];
    Cand loc[kTopK];
    for (int k = 0; k < kTopK; k++) loc[k] = Cand{-INFINITY, INT64_MAX};
    for (int64_t i = threadIdx.x; i < n; i += kTopThreads) {
        const double v = (double)lw[i];
        if (!(v > -INFINITY && v < INFINITY)) continue;
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
            int ia = 0, ib = 0;
            const Cand *A = lists[threadIdx.x], *B = lists[threadIdx.x + w];
            for (int k = 0; k < kTopK; k++) out[k] = better(B[ib], A[ia]) ? B[ib++] : A[ia++];
            for (int k = 0; k < kTopK; k++) lists[threadIdx.x][k] = out[k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const Cand *top = lists[0];
        work[kWMax] = top[0].v;
        work[kWMax + 1] = (double)top[0].i;
        const int d = g->n_dim;
        int got = 0;
        for (int k = 0; k < kTopK && got < n_comp; k++) {
            if (!(top[k].v > -INFINITY)) break;
            double x[7];
            for (int a = 0; a < d; a++) x[a] = load_col(th, ld, g->dims[a], top[k].i);
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
        for (int q = got; q < n_comp; q++)
            for (int a = 0; a < d; a++) g->mean[q][a] = g->mean[got - 1][a];
        g->n_comp = n_comp;
    }
}

// max of lw (finite values) - used by warm-started EM calls
template <class TL>
__global__ void __launch_bounds__(kEmThreads) k_em_max(const TL *__restrict__ lw, int64_t n, double *work) {
    __shared__ double sm[kEmThreads];
    double m = -INFINITY;
    for (int64_t i = threadIdx.x; i < n; i += kEmThreads) {
        const double v = (double)lw[i];
        if (v > -INFINITY && v < INFINITY) m = fmax(m, v);
    }
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int w = kEmThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) work[kWMax] = sm[0];
}

// block-sum of NV doubles held per thread, written to out[0..NV)
template <int NV>
__device__ void block_sum(double (&v)[NV], double *out) {
    __shared__ double red[kEmThreads];
    for (int c = 0; c < NV; c++) {
        red[threadIdx.x] = v[c];
        __syncthreads();
        for (int w = kEmThreads / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[c] = red[0];
        __syncthreads();
    }
}

__device__ __forceinline__ double sample_weight(double lwv, double mlw, double beta) {
    return (lwv > -INFINITY && lwv < INFINITY) ? exp(beta * (lwv - mlw)) : 0.0;
}

// Tempering exponent: the largest beta_k = 2^(-k/4) whose tempered weights
// have (sum w^beta)^2 / sum w^(2 beta) >= frac * (finite samples); frac <= 0
// gives beta = 1.  One block; each grid value is a fixed-order block sum.
template <class TL>
__global__ void __launch_bounds__(kEmThreads)
    k_em_beta(const TL *__restrict__ lw, int64_t n, double frac, double *work) {
    __shared__ double r1[kEmThreads], r2[kEmThreads];
    __shared__ double cnt_s;
    const double mlw = work[kWMax];
    if (!(frac > 0.0)) {
        if (threadIdx.x == 0) work[kWBeta] = 1.0;
        return;
    }
    double c = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kEmThreads) {
        const double v = (double)lw[i];
        c += (v > -INFINITY && v < INFINITY) ? 1.0 : 0.0;
    }
    r1[threadIdx.x] = c;
    __syncthreads();
    for (int w = kEmThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) r1[threadIdx.x] += r1[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) cnt_s = r1[0];
    __syncthreads();
    const double target = frac * cnt_s;
    double beta = exp2(-(double)(kBetaGrid - 1) / 4.0);
    for (int k = 0; k < kBetaGrid; k++) {
        const double b = exp2(-(double)k / 4.0);
        double s1 = 0.0, s2 = 0.0;
        for (int64_t i = threadIdx.x; i < n; i += kEmThreads) {
            const double e = sample_weight((double)lw[i], mlw, b);
            s1 += e;
            s2 += e * e;
        }
        r1[threadIdx.x] = s1;
        r2[threadIdx.x] = s2;
        __syncthreads();
        for (int w = kEmThreads / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) {
                r1[threadIdx.x] += r1[threadIdx.x + w];
                r2[threadIdx.x] += r2[threadIdx.x + w];
            }
            __syncthreads();
        }
        const bool ok = r1[0] * r1[0] / r2[0] >= target;
        __syncthreads();
        if (ok) {
            beta = b;
            break;
        }
    }
    if (threadIdx.x == 0) work[kWBeta] = beta;
}

// first fit: weighted moments of the differences about the best sample
template <class TT, class TL>
__global__ void __launch_bounds__(kEmThreads)
    k_em_init_part(const TT *__restrict__ th, int64_t ld, const TL *__restrict__ lw, int64_t n, const GmmDev *g,
                   PriorDev pr, double *work) {
    const int d = g->n_dim;
    const double mlw = work[kWMax], beta = work[kWBeta];
    double acc[36];
    for (int c = 0; c < 36; c++) acc[c] = 0.0;
    const int64_t b0 = (int64_t)blockIdx.x * kEmTile, b1 = min(b0 + kEmTile, n);
    for (int64_t i = b0 + threadIdx.x; i < b1; i += kEmThreads) {
        const double w = sample_weight((double)lw[i], mlw, beta);
        double x[7];
        for (int a = 0; a < d; a++) {
            const int col = g->dims[a];
            x[a] = wrapd(load_col(th, ld, col, i) - g->mean[0][a], col_period(col));
        }
        acc[0] += w;
        int k = 1;
        for (int a = 0; a < 7; a++) acc[k++] += (a < d) ? w * x[a] : 0.0;
        for (int a = 0; a < 7; a++)
            for (int b = 0; b <= a; b++) acc[k++] += (a < d) ? w * x[a] * x[b] : 0.0;
    }
    block_sum<36>(acc, work + kWPart + (size_t)blockIdx.x * 36);
}

__global__ void k_em_init_final(GmmDev *g, int nblk, PriorDev pr, double *work) {
    if (threadIdx.x != 0) return;
    double s[36];
    for (int c = 0; c < 36; c++) s[c] = 0.0;
    for (int b = 0; b < nblk; b++)
        for (int c = 0; c < 36; c++) s[c] += work[kWPart + (size_t)b * 36 + c];
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
        const double r = col_range(pr, g->dims[a]);
        cov[a][a] += 1e-8 * r * r;
    }
    for (int j = 0; j < g->n_comp; j++) {
        g->w[j] = 1.0 / g->n_comp;
        for (int a = 0; a < 7; a++)
            for (int b = 0; b < 7; b++) g->cov[j][a][b] = (a < d && b < d) ? cov[a][b] : 0.0;
    }
}

// ------------------------------------------------------------------ EM
template <class TT, class TL>
__global__ void __launch_bounds__(kEmThreads)
    k_em_resp(const TT *__restrict__ th, int64_t ld, const TL *__restrict__ lw, int64_t n, const GmmDev *g,
              double *work, double *R) {
    const int d = g->n_dim, nc = g->n_comp;
    const double mlw = work[kWMax], beta = work[kWBeta];
    for (int64_t i = (int64_t)blockIdx.x * kEmThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kEmThreads) {
        const double w = sample_weight((double)lw[i], mlw, beta);
        double x[7];
        for (int a = 0; a < d; a++) x[a] = load_col(th, ld, g->dims[a], i);
        double lr[kMaxComp];
        double m = -INFINITY;
        for (int j = 0; j < nc; j++) {
            if (g->logw[j] == -INFINITY) { lr[j] = -INFINITY; continue; }
            double q = 0.0, df[7];
            for (int a = 0; a < d; a++) df[a] = wrapd(x[a] - g->mean[j][a], col_period(g->dims[a]));
            for (int a = 0; a < d; a++) {
                double y = 0.0;
                for (int b = 0; b <= a; b++) y += g->Linv[j][a][b] * df[b];
                q += y * y;
            }
            lr[j] = g->logw[j] - 0.5 * q - g->logdet_half[j] - 0.5 * d * log(2 * kPi);
            m = fmax(m, lr[j]);
        }
        double s = 0.0;
        for (int j = 0; j < nc; j++) s += (lr[j] == -INFINITY) ? 0.0 : exp(lr[j] - m);
        for (int j = 0; j < nc; j++)
            R[(size_t)j * n + i] = (lr[j] == -INFINITY || !(m > -INFINITY)) ? 0.0 : w * exp(lr[j] - m) / s;
    }
}

// pass 1: W_j and first moments of the wrapped offsets about the current mean
template <class TT>
__global__ void __launch_bounds__(kEmThreads)
    k_em_stat1(const TT *__restrict__ th, int64_t ld, int64_t n, const GmmDev *g, const double *R, double *work) {
    const int j = blockIdx.y;
    const int d = g->n_dim;
    double acc[8];
    for (int c = 0; c < 8; c++) acc[c] = 0.0;
    if (j < g->n_comp) {
        const int64_t b0 = (int64_t)blockIdx.x * kEmTile, b1 = min(b0 + kEmTile, n);
        for (int64_t i = b0 + threadIdx.x; i < b1; i += kEmThreads) {
            const double r = R[(size_t)j * n + i];
            acc[0] += r;
            for (int a = 0; a < 7; a++)
                acc[1 + a] += (a < d) ? r * wrapd(load_col(th, ld, g->dims[a], i) - g->mean[j][a],
                                                  col_period(g->dims[a]))
                                      : 0.0;
        }
    }
    block_sum<8>(acc, work + kWPart + ((size_t)j * gridDim.x + blockIdx.x) * 8);
}

__global__ void k_em_mean(GmmDev *g, int nblk, double *work) {
    const int j = threadIdx.x;
    __shared__ double W[kMaxComp];
    const int nc = g->n_comp, d = g->n_dim;
    double s[8];
    for (int c = 0; c < 8; c++) s[c] = 0.0;
    if (j < nc)
        for (int b = 0; b < nblk; b++)
            for (int c = 0; c < 8; c++) s[c] += work[kWPart + ((size_t)j * nblk + b) * 8 + c];
    if (j < kMaxComp) W[j] = (j < nc) ? s[0] : 0.0;
    __syncthreads();
    if (j < nc) {
        double tot = 0.0;
        for (int q = 0; q < nc; q++) tot += W[q];
        for (int a = 0; a < 7; a++) work[kWOldMean + j * 8 + a] = g->mean[j][a];
        work[kWOff + j * 8 + 7] = s[0];
        for (int a = 0; a < 7; a++) work[kWOff + j * 8 + a] = (s[0] > 0.0 && a < d) ? s[1 + a] / s[0] : 0.0;
        g->w[j] = s[0] / tot;
        if (s[0] > 0.0) {
            for (int a = 0; a < d; a++) {
                double mu = g->mean[j][a] + work[kWOff + j * 8 + a];
                const double P = col_period(g->dims[a]);
                if (P > 0.0) mu = mu - P * floor(mu / P);
                g->mean[j][a] = mu;
            }
        }
    }
}

// pass 2: centred second moments about the new offsets
template <class TT>
__global__ void __launch_bounds__(kEmThreads)
    k_em_stat2(const TT *__restrict__ th, int64_t ld, int64_t n, const GmmDev *g, const double *R, double *work,
               int nblk1) {
    const int j = blockIdx.y;
    const int d = g->n_dim;
    double acc[28];
    for (int c = 0; c < 28; c++) acc[c] = 0.0;
    if (j < g->n_comp) {
        const double *mo = work + kWOldMean + j * 8;
        const double *off = work + kWOff + j * 8;
        const int64_t b0 = (int64_t)blockIdx.x * kEmTile, b1 = min(b0 + kEmTile, n);
        for (int64_t i = b0 + threadIdx.x; i < b1; i += kEmThreads) {
            const double r = R[(size_t)j * n + i];
            double x[7];
            for (int a = 0; a < 7; a++)
                x[a] = (a < d) ? wrapd(load_col(th, ld, g->dims[a], i) - mo[a], col_period(g->dims[a])) - off[a]
                               : 0.0;
            int k = 0;
            for (int a = 0; a < 7; a++)
                for (int b = 0; b <= a; b++) acc[k++] += r * x[a] * x[b];
        }
    }
    block_sum<28>(acc, work + kWPart + (size_t)kMaxComp * nblk1 * 8 + ((size_t)j * gridDim.x + blockIdx.x) * 28);
}

__global__ void k_em_cov(GmmDev *g, int nblk, PriorDev pr, double *work, int nblk1) {
    const int j = threadIdx.x;
    if (j == 0) g->valid = 1;
    __syncthreads();
    if (j >= g->n_comp) return;
    const double W = work[kWOff + j * 8 + 7];
    if (W > 0.0) {
        double s[28];
        for (int c = 0; c < 28; c++) s[c] = 0.0;
        const double *base = work + kWPart + (size_t)kMaxComp * nblk1 * 8;
        for (int b = 0; b < nblk; b++)
            for (int c = 0; c < 28; c++) s[c] += base[((size_t)j * nblk + b) * 28 + c];
        const int d = g->n_dim;
        int k = 0;
        for (int a = 0; a < 7; a++)
            for (int b = 0; b <= a; b++) {
                double v = (a < d && b < d) ? s[k] / W : 0.0;
                k++;
                g->cov[j][a][b] = v;
                g->cov[j][b][a] = v;
            }
        for (int a = 0; a < d; a++) {
            const double r = col_range(pr, g->dims[a]);
            g->cov[j][a][a] += 1e-8 * r * r;
        }
    }
    factor_one(*g, j);
}

}  // namespace

size_t em_work_bytes(int64_t n) {
    const int64_t nblk = (n + kEmTile - 1) / kEmTile;
    const size_t part = (size_t)kMaxComp * nblk * (8 + 28) + (size_t)nblk * 36;
    return (kWPart + part) * sizeof(double) + (size_t)kMaxComp * n * sizeof(double);
}

hipError_t launch_gmm_factor(GmmDev *d_gmm, hipStream_t st) {
    hipLaunchKernelGGL(k_gmm_factor, dim3(1), dim3(64), 0, st, d_gmm);
    return hipGetLastError();
}

#define ILE_DISPATCH_TL(policy, BODY)            \
    do {                                         \
        if ((policy) == kFP64) {                 \
            using TT = double;                   \
            using TL = double;                   \
            BODY;                                \
        } else if ((policy) == kFP32) {          \
            using TT = float;                    \
            using TL = float;                    \
            BODY;                                \
        } else {                                 \
            using TT = float;                    \
            using TL = double;                   \
            BODY;                                \
        }                                        \
    } while (0)

hipError_t launch_em_prepare(int policy, const void *lw, int64_t n, double *d_work, size_t work_bytes,
                             double temper_frac, hipStream_t st) {
    if (work_bytes < em_work_bytes(n)) return hipErrorInvalidValue;
    // only the weight type matters here (FP64 for the FP64 and mixed policies)
    if (policy == kFP32) {
        hipLaunchKernelGGL((k_em_max<float>), dim3(1), dim3(kEmThreads), 0, st, (const float *)lw, n, d_work);
        hipLaunchKernelGGL((k_em_beta<float>), dim3(1), dim3(kEmThreads), 0, st, (const float *)lw, n, temper_frac,
                           d_work);
    } else {
        hipLaunchKernelGGL((k_em_max<double>), dim3(1), dim3(kEmThreads), 0, st, (const double *)lw, n, d_work);
        hipLaunchKernelGGL((k_em_beta<double>), dim3(1), dim3(kEmThreads), 0, st, (const double *)lw, n,
                           temper_frac, d_work);
    }
    return hipGetLastError();
}

hipError_t launch_em_top(int policy, const void *theta, int64_t ld, const void *lw, int64_t n, GmmDev *d_gmm,
                         int n_comp, double *d_work, size_t work_bytes, PriorDev pr, hipStream_t st) {
    if (work_bytes < em_work_bytes(n)) return hipErrorInvalidValue;
    const int64_t nblk = (n + kEmTile - 1) / kEmTile;
    ILE_DISPATCH_TL(policy, {
        hipLaunchKernelGGL((k_em_top<TT, TL>), dim3(1), dim3(kTopThreads), 0, st, (const TT *)theta, ld,
                           (const TL *)lw, n, d_gmm, n_comp, d_work);
        hipLaunchKernelGGL((k_em_init_part<TT, TL>), dim3(nblk), dim3(kEmThreads), 0, st, (const TT *)theta, ld,
                           (const TL *)lw, n, d_gmm, pr, d_work);
    });
    hipLaunchKernelGGL(k_em_init_final, dim3(1), dim3(1), 0, st, d_gmm, (int)nblk, pr, d_work);
    hipLaunchKernelGGL(k_gmm_factor, dim3(1), dim3(64), 0, st, d_gmm);
    return hipGetLastError();
}

hipError_t launch_em_iter(int policy, const void *theta, int64_t ld, const void *lw, int64_t n, GmmDev *d_gmm,
                          double *d_work, size_t work_bytes, PriorDev pr, hipStream_t st) {
    if (work_bytes < em_work_bytes(n)) return hipErrorInvalidValue;
    const int64_t nblk = (n + kEmTile - 1) / kEmTile;
    double *R = d_work + kWPart + (size_t)kMaxComp * nblk * (8 + 28) + (size_t)nblk * 36;
    const int64_t rb = (n + kEmThreads - 1) / kEmThreads;
    const int rblk = (int)(rb < 4096 ? rb : 4096);
    ILE_DISPATCH_TL(policy, {
        hipLaunchKernelGGL((k_em_resp<TT, TL>), dim3(rblk), dim3(kEmThreads), 0, st, (const TT *)theta, ld,
                           (const TL *)lw, n, d_gmm, d_work, R);
        hipLaunchKernelGGL((k_em_stat1<TT>), dim3(nblk, kMaxComp), dim3(kEmThreads), 0, st, (const TT *)theta, ld,
                           n, d_gmm, R, d_work);
        hipLaunchKernelGGL(k_em_mean, dim3(1), dim3(64), 0, st, d_gmm, (int)nblk, d_work);
        hipLaunchKernelGGL((k_em_stat2<TT>), dim3(nblk, kMaxComp), dim3(kEmThreads), 0, st, (const TT *)theta, ld,
                           n, d_gmm, R, d_work, (int)nblk);
    });
    hipLaunchKernelGGL(k_em_cov, dim3(1), dim3(64), 0, st, d_gmm, (int)nblk, pr, d_work, (int)nblk);
    return hipGetLastError();
}

}  // namespace ile
