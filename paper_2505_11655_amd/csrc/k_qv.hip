// Inner products of eq. (QUV) from the modes and the data on the GPU (the
// precompute behind every likelihood: Q time series over the narrow window,
// and the mode-mode matrices U and V), in FP64, for several intrinsic points
// sharing one data set:
//   Q[p][k][a][i] = 2 df sum_f e^{2 pi i f tau_i} conj(h_pa(f)) d_k(f) w_k(f),
//   U[p][k][a][b] = 2 df sum_f conj(h_pa(f)) h_pb(f) w_k(f),
//   V[p][k][a][b] = 2 df sum_f h_pa(-f) h_pb(f) w_k(f),
// over the band f_lo <= |f| <= f_hi of the two-sided grid f_m = m' df (m' the
// signed FFT-order index), tau_i = (i - win_half) / (n df).
// Q is a dense complex product [window times] x [band] . [band] x [(p, k, a)]:
// X = 2 df conj(h) d w is formed once per band bin and column, the phases come
// from a table e^{2 pi i r / n} at r = (m' j) mod n (exact integer phase), and
// a register-tiled kernel (4 x 4 outputs per thread, LDS-staged tiles of
// phases and X) accumulates over a slice of the band; slices are summed in
// order by a second kernel (deterministic).  On this chip FP64 matrix cores
// have the same peak as the FP64 vector ALUs, so the product stays on the
// VALU.  U and V use the symmetries U_ba = conj(U_ab), V_ba = V_ab: only
// a <= b is summed (one block per pair, fixed-order tree reduction).
#include "ile_internal.h"

namespace ile {

namespace {

constexpr int kQvThreads = 256;
constexpr int kQvTT = 64;     // window times per tile
constexpr int kQvTC = 64;     // columns per tile
constexpr int kQvMB = 16;     // band bins per LDS stage

struct z2 {
    double re, im;
};

__global__ void k_qv_twiddle(double2 *__restrict__ tw, int64_t n) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        double s, c;
        sincospi(2.0 * (double)r / (double)n, &s, &c);
        tw[r] = make_double2(c, s);
    }
}

// X[b][col] = 2 df conj(h_pa(f_b)) d_k(f_b) w_k(f_b), col = (p * nd + k) * na + a.
__global__ void k_qv_x(const double2 *__restrict__ hlm, const double2 *__restrict__ data,
                       const double *__restrict__ inv_psd, const int64_t *__restrict__ band, int64_t n_band,
                       int64_t n, int na, int nd, int np, double df, double2 *__restrict__ X) {
    const int64_t cols = (int64_t)np * nd * na;
    const int64_t total = n_band * cols;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = e / cols, col = e % cols;
        const int a = (int)(col % na);
        const int k = (int)((col / na) % nd);
        const int64_t p = col / ((int64_t)na * nd);
        const int64_t m = band[b];
        const double2 h = hlm[(p * na + a) * n + m];
        const double2 d = data[(int64_t)k * n + m];
        const double w = 2.0 * df * (inv_psd ? inv_psd[(int64_t)k * n + m] : 1.0);
        // conj(h) d
        const double re = h.x * d.x + h.y * d.y, im = h.x * d.y - h.y * d.x;
        X[e] = make_double2(re * w, im * w);
    }
}

// Partial Q of one (time tile, column tile, band slice).
__global__ void __launch_bounds__(kQvThreads)
    k_qv_q(const double2 *__restrict__ X, const double2 *__restrict__ tw, const int64_t *__restrict__ msig,
           int64_t n_band, int64_t n, int64_t cols, int n_time, int win_half, int64_t slice,
           double2 *__restrict__ part) {
    __shared__ z2 sE[kQvMB][kQvTT];
    __shared__ z2 sX[kQvMB][kQvTC];
    const int t0 = blockIdx.x * kQvTT;
    const int64_t c0 = (int64_t)blockIdx.y * kQvTC;
    const int64_t b_lo = (int64_t)blockIdx.z * slice;
    const int64_t b_hi = b_lo + slice < n_band ? b_lo + slice : n_band;
    const int tid = threadIdx.x;
    const int ti = tid & 15, tc = tid >> 4;
    double ar[4][4], ai[4][4];
#pragma unroll
    for (int r = 0; r < 4; r++)
#pragma unroll
        for (int s = 0; s < 4; s++) {
            ar[r][s] = 0.0;
            ai[r][s] = 0.0;
        }
    for (int64_t bb = b_lo; bb < b_hi; bb += kQvMB) {
        // stage: 16 band bins x 64 times of phases, 16 x 64 of X
        for (int e = tid; e < kQvMB * kQvTT; e += kQvThreads) {
            const int lb = e / kQvTT, lt = e % kQvTT;
            const int64_t b = bb + lb;
            const int t = t0 + lt;
            z2 v{0.0, 0.0};
            if (b < b_hi && t < n_time) {
                const int64_t j = (int64_t)(t - win_half);
                int64_t r = (msig[b] * j) % n;
                r = r < 0 ? r + n : r;
                const double2 w = tw[r];
                v = z2{w.x, w.y};
            }
            sE[lb][lt] = v;
        }
        for (int e = tid; e < kQvMB * kQvTC; e += kQvThreads) {
            const int lb = e / kQvTC, lc = e % kQvTC;
            const int64_t b = bb + lb;
            const int64_t c = c0 + lc;
            z2 v{0.0, 0.0};
            if (b < b_hi && c < cols) {
                const double2 x = X[b * cols + c];
                v = z2{x.x, x.y};
            }
            sX[lb][lc] = v;
        }
        __syncthreads();
#pragma unroll 4
        for (int lb = 0; lb < kQvMB; lb++) {
            z2 e[4], x[4];
#pragma unroll
            for (int r = 0; r < 4; r++) e[r] = sE[lb][ti + 16 * r];
#pragma unroll
            for (int s = 0; s < 4; s++) x[s] = sX[lb][tc + 16 * s];
#pragma unroll
            for (int r = 0; r < 4; r++)
#pragma unroll
                for (int s = 0; s < 4; s++) {
                    ar[r][s] = fma(e[r].re, x[s].re, fma(-e[r].im, x[s].im, ar[r][s]));
                    ai[r][s] = fma(e[r].re, x[s].im, fma(e[r].im, x[s].re, ai[r][s]));
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; r++)
#pragma unroll
        for (int s = 0; s < 4; s++) {
            const int t = t0 + ti + 16 * r;
            const int64_t c = c0 + tc + 16 * s;
            if (t < n_time && c < cols)
                part[((int64_t)blockIdx.z * cols + c) * n_time + t] = make_double2(ar[r][s], ai[r][s]);
        }
}

// Q[col][t] = sum over slices in order.
__global__ void k_qv_reduce(const double2 *__restrict__ part, int n_slices, int64_t cols, int n_time,
                            double2 *__restrict__ Q) {
    const int64_t total = cols * n_time;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        double re = 0.0, im = 0.0;
        for (int s = 0; s < n_slices; s++) {
            const double2 v = part[(int64_t)s * total + e];
            re += v.x;
            im += v.y;
        }
        Q[e] = make_double2(re, im);
    }
}

// U and V of one (point, detector, pair a <= b): a fixed-order tree reduction.
__global__ void __launch_bounds__(kQvThreads)
    k_qv_uv(const double2 *__restrict__ hlm, const double *__restrict__ inv_psd, const int64_t *__restrict__ band,
            int64_t n_band, int64_t n, int na, int nd, double df, double2 *__restrict__ U, double2 *__restrict__ V) {
    const int npair = na * (na + 1) / 2;
    const int pk = blockIdx.x / npair;     // p * nd + k
    int q = blockIdx.x % npair;
    int a = 0;
    while (q >= na - a) {
        q -= na - a;
        a++;
    }
    const int b = a + q;
    const int k = pk % nd;
    const int64_t p = pk / nd;
    const double2 *ha = hlm + (p * na + a) * n;
    const double2 *hb = hlm + (p * na + b) * n;
    double ur = 0.0, ui = 0.0, vr = 0.0, vi = 0.0;
    for (int64_t e = threadIdx.x; e < n_band; e += kQvThreads) {
        const int64_t m = band[e];
        const int64_t mn = m == 0 ? 0 : n - m;
        const double w = inv_psd ? inv_psd[(int64_t)k * n + m] : 1.0;
        const double2 x = ha[m], y = hb[m], z = ha[mn];
        ur += w * (x.x * y.x + x.y * y.y);
        ui += w * (x.x * y.y - x.y * y.x);
        vr += w * (z.x * y.x - z.y * y.y);
        vi += w * (z.x * y.y + z.y * y.x);
    }
    __shared__ double s[4][kQvThreads];
    s[0][threadIdx.x] = ur;
    s[1][threadIdx.x] = ui;
    s[2][threadIdx.x] = vr;
    s[3][threadIdx.x] = vi;
    __syncthreads();
    for (int o = kQvThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int c = 0; c < 4; c++) s[c][threadIdx.x] += s[c][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double f = 2.0 * df;
        const int64_t base = (int64_t)pk * na * na;
        const double ui_ab = a == b ? 0.0 : f * s[1][0];   // the diagonal <h_a|h_a> is real
        U[base + a * na + b] = make_double2(f * s[0][0], ui_ab);
        U[base + b * na + a] = make_double2(f * s[0][0], -ui_ab);
        V[base + a * na + b] = make_double2(f * s[2][0], f * s[3][0]);
        V[base + b * na + a] = make_double2(f * s[2][0], f * s[3][0]);
    }
}

}  // namespace

size_t qv_scratch_bytes(int64_t n, int64_t n_band, int64_t cols, int n_time, int n_slices) {
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    return al((size_t)n * 16) + al((size_t)n_band * 8) * 2 + al((size_t)n_band * cols * 16) +
           al((size_t)n_slices * cols * n_time * 16);
}

int qv_slices(int64_t n_band, int64_t cols, int n_time) {
    const int64_t tiles = (int64_t)((n_time + kQvTT - 1) / kQvTT) * ((cols + kQvTC - 1) / kQvTC);
    int64_t s = (1024 + tiles - 1) / tiles;
    const int64_t smax = (n_band + 63) / 64;
    s = s > smax ? smax : s;
    return (int)(s < 1 ? 1 : s);
}

hipError_t launch_qv(const void *hlm, const void *data, const double *inv_psd, int64_t n, int na, int nd, int np,
                     double df, const int64_t *h_band, const int64_t *h_msig, int64_t n_band, int n_time,
                     int win_half, void *Q, void *U, void *V, void *scratch, int n_slices, hipStream_t st) {
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    char *w = (char *)scratch;
    double2 *tw = (double2 *)w;
    w += al((size_t)n * 16);
    int64_t *band = (int64_t *)w;
    w += al((size_t)n_band * 8);
    int64_t *msig = (int64_t *)w;
    w += al((size_t)n_band * 8);
    const int64_t cols = (int64_t)np * nd * na;
    double2 *X = (double2 *)w;
    w += al((size_t)n_band * cols * 16);
    double2 *part = (double2 *)w;
    hipError_t e = hipMemcpyAsync(band, h_band, (size_t)n_band * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(msig, h_msig, (size_t)n_band * 8, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_qv_twiddle, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, tw, n);
    const int64_t xe = n_band * cols;
    hipLaunchKernelGGL(k_qv_x, dim3((unsigned)std::min<int64_t>((xe + 255) / 256, 65536)), dim3(256), 0, st,
                       (const double2 *)hlm, (const double2 *)data, inv_psd, band, n_band, n, na, nd, np, df, X);
    const int64_t slice = ((n_band + n_slices - 1) / n_slices + kQvMB - 1) / kQvMB * kQvMB;
    const int ns = (int)((n_band + slice - 1) / slice);
    dim3 grid((unsigned)((n_time + kQvTT - 1) / kQvTT), (unsigned)((cols + kQvTC - 1) / kQvTC), (unsigned)ns);
    hipLaunchKernelGGL(k_qv_q, grid, dim3(kQvThreads), 0, st, X, tw, msig, n_band, n, cols, n_time, win_half, slice,
                       part);
    const int64_t qe = cols * n_time;
    hipLaunchKernelGGL(k_qv_reduce, dim3((unsigned)std::min<int64_t>((qe + 255) / 256, 65536)), dim3(256), 0, st,
                       part, ns, cols, n_time, (double2 *)Q);
    const int npair = na * (na + 1) / 2;
    hipLaunchKernelGGL(k_qv_uv, dim3((unsigned)((int64_t)np * nd * npair)), dim3(kQvThreads), 0, st,
                       (const double2 *)hlm, inv_psd, band, n_band, n, na, nd, df, (double2 *)U, (double2 *)V);
    return hipGetLastError();
}

}  // namespace ile
