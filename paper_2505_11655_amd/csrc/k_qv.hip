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
// the product runs on the FP64 matrix cores (16 x 16 x 4 steps, the operands
// held in registers so that each LDS or memory read feeds several matrix
// steps) over a slice of the band; slices are summed in order by a second
// kernel (deterministic).  U and V use the symmetries U_ba = conj(U_ab),
// V_ba = V_ab: only a <= b is summed (one block per pair, fixed-order tree
// reduction).
// The decimated route splits the DFT behind Q once (the first step of a
// decimation-in-frequency FFT, Section "Reduce duplication of inner products"
// weighs FFTs against the direct sum): with n = R N2, m = m2 + N2 a (m the
// unsigned grid index, 0 <= m2 < N2, 0 <= a < R) and j = i - win_half =
// R p + q (0 <= q < R),
//   e^{2 pi i m j / n} = e^{2 pi i m2 p / N2} e^{2 pi i m2 q / n} e^{2 pi i a q / R},
// so Q(j) = sum_m2 e^{2 pi i m2 p / N2} Y_q(m2) with the radix-R partial sums
// Y_q(m2) = e^{2 pi i m2 q / n} sum_a X(m2 + N2 a) (X zero off the band).
// Y is formed by a streaming kernel, and the remaining sum is the direct
// route's matrix-core product over N2 bins, R columns per column and only
// the decimated times p of the window (at most 64: one time tile).  Every
// factor is a table value at an exact integer index.
#include "ile_internal.h"
#include "k_qv.h"

namespace ile {

namespace {

constexpr int kQvThreads = 256;
constexpr int kQvTT = 64;     // window times per block tile (direct route)
constexpr int kQvNS = 4;      // 16-column tiles per wave
// columns per block tile: two waves across a 64-time tile, four across a
// 32-time tile
constexpr int qv_tc(int tt) { return tt == 64 ? 32 * kQvNS : 64 * kQvNS; }
constexpr int kQvTC = qv_tc(kQvTT);
constexpr int kQvKB = 32;     // band bins per LDS stage of phases

__global__ void k_qv_twiddle(double2 *__restrict__ tw, int64_t n) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        double s, c;
        sincospi(2.0 * (double)r / (double)n, &s, &c);
        tw[r] = make_double2(c, s);
    }
}

// X[b][col] = 2 df conj(h_pa(f_b)) d_k(f_b) w_k(f_b), col = (p * nd + k) * na + a.
// One column per thread (its (p, k, a) decoded once), kQvXRun consecutive
// bins per block row: the writes are coalesced along the columns, and each
// cache line of a mode row serves several bins.
constexpr int kQvXRun = 16;
__global__ void __launch_bounds__(kQvThreads)
    k_qv_x(const double2 *__restrict__ hlm, const double2 *__restrict__ data, const double *__restrict__ inv_psd,
           const int64_t *__restrict__ band, int64_t n_band, int64_t n, int na, int nd, int np, double df,
           double2 *__restrict__ X) {
    const int64_t cols = (int64_t)np * nd * na;
    const int64_t col = (int64_t)blockIdx.x * kQvThreads + threadIdx.x;
    if (col >= cols) return;
    const int a = (int)(col % na);
    const int k = (int)((col / na) % nd);
    const int64_t p = col / ((int64_t)na * nd);
    const double2 *h = hlm + (p * na + a) * n;
    const double2 *dk = data + (int64_t)k * n;
    const double *wk = inv_psd ? inv_psd + (int64_t)k * n : nullptr;
    for (int64_t b0 = (int64_t)blockIdx.y * kQvXRun; b0 < n_band; b0 += (int64_t)gridDim.y * kQvXRun) {
        const int64_t b1 = b0 + kQvXRun < n_band ? b0 + kQvXRun : n_band;
        for (int64_t b = b0; b < b1; b++) {
            const int64_t m = band[b];
            const double2 hv = h[m];
            const double2 d = dk[m];
            const double w = 2.0 * df * (wk ? wk[m] : 1.0);
            // conj(h) d
            const double re = hv.x * d.x + hv.y * d.y, im = hv.x * d.y - hv.y * d.x;
            X[b * cols + col] = make_double2(re * w, im * w);
        }
    }
}

// Partial Q of one (time tile, column tile, band slice) on the FP64 matrix
// cores.  A block of four waves covers TT = 64 window times x 128 columns (two
// waves along the times, two along the columns) or TT = 32 times x 256
// columns (four waves along the columns); each wave a 32 x 64 sub-tile as
// 2 x 4 tiles of 16 x 16 (kQvNS = 4 column tiles),
// with the real and the imaginary part of every tile in its own accumulator.
// One step of v_mfma_f64_16x16x4f64 takes four band bins: lane l holds the A
// element (time l % 16, bin l / 16) and the B element (bin l / 16, column
// l % 16), and its four results are times l / 16 + 4 r (r = 0..3) of column
// l % 16.  Each complex product is four real ones, Re += Er Xr - Ei Xi,
// Im += Er Xi + Ei Xr.
// The phases of a stage of 32 bins x TT times sit in LDS (the column waves of
// a time range share them), double-buffered: every thread reads its TT / 8
// phases of the next stage (one bin, TT / 8 consecutive times: one 64-bit
// remainder, then r += m' mod n per time) from the table during the
// stage's first matrix step, after that step's X reads (the memory counter
// retires in order, so waiting for X then never waits for the table), and
// writes them to LDS after the stage's last step.  X is read by each wave
// straight from memory (no other wave of the block uses it), one step ahead.
// Blocks are numbered so that the time tiles of one column tile run on one
// XCD and share its L2.
typedef double qv_d4 __attribute__((ext_vector_type(4)));

template <int TT>
__global__ void __launch_bounds__(kQvThreads)
    k_qv_q(const double2 *__restrict__ X, const double2 *__restrict__ tw, const int64_t *__restrict__ msig,
           int64_t n_band, int64_t n, int64_t cols, int n_time, int win_half, int64_t slice, int n_tt, int n_tc,
           double2 *__restrict__ part) {
    static_assert(TT == 64 || TT == 32, "time tile of 64 or 32");
    constexpr int TC = qv_tc(TT);
    constexpr int PT = TT / 8;   // phases per thread and stage
    __shared__ double2 sE[2][kQvKB][TT];
    const int64_t nb = gridDim.x;
    const int64_t h = blockIdx.x;
    const int64_t lid = nb % 8 == 0 ? (h % 8) * (nb / 8) + h / 8 : h;
    const int tt = (int)(lid % n_tt);
    const int tc = (int)((lid / n_tt) % n_tc);
    const int64_t z = lid / ((int64_t)n_tt * n_tc);
    const int64_t b_lo = z * slice;
    const int64_t b_hi = b_lo + slice < n_band ? b_lo + slice : n_band;
    const int t0 = tt * TT;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    // the wave's first time within the tile and first column
    const int wt = TT == 64 ? 32 * (wv & 1) : 0;
    const int64_t cw = (int64_t)tc * TC + 16 * kQvNS * (TT == 64 ? (wv >> 1) : wv);
    // this thread's share of a phase stage: bin gb, times gt .. gt + PT - 1
    const int gb = threadIdx.x >> 3, gt = (threadIdx.x & 7) * PT;
    static_assert(kQvThreads * PT == kQvKB * TT, "PT phases per thread and stage");
    // m' of the thread's bin in the stage at bb (the bin itself when msig is
    // null); a bin past the slice gets m' = 0 and a zero phase (its X, read
    // at a clamped index, is then multiplied by 0)
    auto bin_m = [&](int64_t bb, double &f) -> int64_t {
        const int64_t b = bb + gb;
        f = b < b_hi ? 1.0 : 0.0;
        return b < b_hi ? (msig ? msig[b] : b) : 0;
    };
    // The thread's PT phases for bin m', r = m' (t - win_half) mod n,
    // then r += m' mod n per time (r stays in [0, n)).  Rows past the window
    // need no mask: they are never stored.
    auto phase_get = [&](int64_t m, double f, double2 (&pv)[PT]) {
        int64_t r = (m * (int64_t)(t0 + gt - win_half)) % n;
        r = r < 0 ? r + n : r;
        int64_t step = m % n;
        step = step < 0 ? step + n : step;
#pragma unroll
        for (int q = 0; q < PT; q++) {
            const double2 w = tw[r];
            pv[q] = make_double2(w.x * f, w.y * f);
            r += step;
            r = r >= n ? r - n : r;
        }
    };
    qv_d4 accR[2][kQvNS], accI[2][kQvNS];
#pragma unroll
    for (int r = 0; r < 2; r++)
#pragma unroll
        for (int s = 0; s < kQvNS; s++) {
            accR[r][s] = qv_d4{0.0, 0.0, 0.0, 0.0};
            accI[r][s] = qv_d4{0.0, 0.0, 0.0, 0.0};
        }
    // X of one step of four bins: the lane's bin b4 + lk, its columns.
    // Indices past the slice or the columns are clamped to a valid element
    // (unconditional loads): such a bin has a zero phase, such a column is
    // never stored.
    auto load_x = [&](int64_t b4, double2 (&x)[kQvNS]) {
        const int64_t b = b4 + lk;
        const int64_t bc = b < b_hi ? b : b_hi - 1;
#pragma unroll
        for (int s = 0; s < kQvNS; s++) {
            const int64_t c = cw + 16 * s + li;
            const double2 w = X[bc * cols + (c < cols ? c : cols - 1)];
            x[s] = make_double2(w.x, w.y);
        }
    };
    {
        double2 pv[PT];
        double f;
        const int64_t m = bin_m(b_lo, f);
        phase_get(m, f, pv);
#pragma unroll
        for (int q = 0; q < PT; q++) sE[0][gb][gt + q] = pv[q];
    }
    double f_next;
    int64_t m_next = bin_m(b_lo + kQvKB, f_next);   // read one stage before it is used
    double2 xc[kQvNS];
    load_x(b_lo, xc);
    __syncthreads();
    int buf = 0;
    for (int64_t bb = b_lo; bb < b_hi; bb += kQvKB) {
        const int nk = b_hi - bb < kQvKB ? (int)(b_hi - bb) : kQvKB;
        const bool more = bb + kQvKB < b_hi;
        double2 pv[PT];
        for (int ks = 0; ks < nk; ks += 4) {
            // the next step's X is in flight while this step's products run
            double2 xn[kQvNS];
            load_x(bb + ks + 4, xn);
            // the next stage's phases: read during the first step, written
            // after the last
            if (more && ks == 0) {
                phase_get(m_next, f_next, pv);
                m_next = bin_m(bb + 2 * kQvKB, f_next);
            }
            double2 e[2];
#pragma unroll
            for (int r = 0; r < 2; r++) e[r] = sE[buf][ks + lk][wt + 16 * r + li];
#pragma unroll
            for (int r = 0; r < 2; r++) {
                const double ni = -e[r].y;
#pragma unroll
                for (int s = 0; s < kQvNS; s++) {
                    accR[r][s] = __builtin_amdgcn_mfma_f64_16x16x4f64(e[r].x, xc[s].x, accR[r][s], 0, 0, 0);
                    accR[r][s] = __builtin_amdgcn_mfma_f64_16x16x4f64(ni, xc[s].y, accR[r][s], 0, 0, 0);
                    accI[r][s] = __builtin_amdgcn_mfma_f64_16x16x4f64(e[r].x, xc[s].y, accI[r][s], 0, 0, 0);
                    accI[r][s] = __builtin_amdgcn_mfma_f64_16x16x4f64(e[r].y, xc[s].x, accI[r][s], 0, 0, 0);
                }
            }
#pragma unroll
            for (int s = 0; s < kQvNS; s++) xc[s] = xn[s];
        }
        if (more) {
#pragma unroll
            for (int q = 0; q < PT; q++) sE[buf ^ 1][gb][gt + q] = pv[q];
        }
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int r = 0; r < 2; r++)
#pragma unroll
        for (int s = 0; s < kQvNS; s++)
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int t = t0 + wt + 16 * r + lk + 4 * q;
                const int64_t c = cw + 16 * s + li;
                if (t < n_time && c < cols)
                    part[(z * cols + c) * n_time + t] = make_double2(accR[r][s][q], accI[r][s][q]);
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

// Stage one of the decimated route: Y[m2][col R + q] for every column and
// m2 in [0, N2), from the R aliases m2 + N2 a (X = 2 df conj(h) d w on the
// band's bins, 0 elsewhere).  A block covers kDecM consecutive m2 (the lanes
// of a wave, so that every read of a mode row, the data and the weight is
// one contiguous run) by kDecC columns (one per wave).  The outputs of each
// (m2, column) go through LDS, at most eight q at a time (two passes for
// R = 16, which keeps the block's LDS near 33 KB), and the tile's rows are
// written out from there in runs of whole cache lines.
constexpr int kDecM = 64;
constexpr int kDecC = kQvThreads / 64;

// In place, v[q] <- sum_a v[a] e^{2 pi i a q / R} (R a power of two): radix-2
// decimation in time over the bit-reversed inputs, log2 R passes of R / 2
// butterflies, wr[r] = e^{2 pi i r / R}; a butterfly with twiddle 1 skips its
// product.
template <int R>
__device__ __forceinline__ void dft_radix2(double2 (&v)[R], const double2 (&wr)[R]) {
    constexpr int LG = R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : 4;
    static_assert((1 << LG) == R, "R in {2, 4, 8, 16}");
#pragma unroll
    for (int a = 0; a < R; a++) {
        int b = 0;
#pragma unroll
        for (int k = 0; k < LG; k++) b |= ((a >> k) & 1) << (LG - 1 - k);
        if (a < b) {
            const double2 t = v[a];
            v[a] = v[b];
            v[b] = t;
        }
    }
#pragma unroll
    for (int len = 2; len <= R; len <<= 1) {
        const int half = len / 2, step = R / len;
#pragma unroll
        for (int st = 0; st < R; st += len)
#pragma unroll
            for (int j = 0; j < half; j++) {
                const double2 u = v[st + j], x = v[st + j + half];
                double2 t = x;
                if (j != 0) {
                    const double2 w = wr[j * step];
                    t = make_double2(x.x * w.x - x.y * w.y, x.x * w.y + x.y * w.x);
                }
                v[st + j] = make_double2(u.x + t.x, u.y + t.y);
                v[st + j + half] = make_double2(u.x - t.x, u.y - t.y);
            }
    }
}
template <int R>
__global__ void __launch_bounds__(kQvThreads)
    k_qv_dec1(const double2 *__restrict__ hlm, const double2 *__restrict__ data, const double *__restrict__ inv_psd,
              const double2 *__restrict__ tw, int64_t n, int na, int nd, int np, double df, double f_lo, double f_hi,
              int64_t n_mt, double2 *__restrict__ Y) {
    constexpr int QC = R < 8 ? R : 8;       // q per LDS pass
    constexpr int RW = kDecC * QC + 1;      // LDS row (one element of padding)
    __shared__ double2 sY[kDecM * RW];
    const int64_t cols = (int64_t)np * nd * na;
    const int64_t n2 = n / R;
    // blocks numbered so that consecutive tiles run on one XCD: the columns
    // of one mode row for the other detectors (na columns apart) then find
    // its lines in that XCD's L2
    const int64_t nbk = gridDim.x, hb = blockIdx.x;
    const int64_t lid = nbk % 8 == 0 ? (hb % 8) * (nbk / 8) + hb / 8 : hb;
    const int64_t mt = lid % n_mt, ct = lid / n_mt;
    const int64_t m2_0 = mt * kDecM, col0 = ct * kDecC;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t m2 = m2_0 + lane, col = col0 + wv;
    const bool live = m2 < n2 && col < cols;
    double2 yq[R];
    if (live) {
        const int a = (int)(col % na);
        const int k = (int)((col / na) % nd);
        const int64_t p = col / ((int64_t)na * nd);
        const double2 *h = hlm + (p * na + a) * n;
        const double2 *dk = data + (int64_t)k * n;
        const double *wk = inv_psd ? inv_psd + (int64_t)k * n : nullptr;
        // every alias's reads are issued before any is used; the band test is
        // the host's (|m' df| in [f_lo, f_hi], m' the signed index), and a
        // mode value off the band is not read
        double2 hv[R], dv[R];
        double wpsd[R];
        bool inb[R];
#pragma unroll
        for (int al = 0; al < R; al++) {
            const int64_t m = m2 + n2 * al;
            const int64_t ms = m < (n + 1) / 2 ? m : m - n;
            const double af = fabs((double)ms * df);
            inb[al] = af >= f_lo && af <= f_hi;
            hv[al] = make_double2(0.0, 0.0);
            if (inb[al]) hv[al] = h[m];
            dv[al] = dk[m];
            wpsd[al] = wk ? wk[m] : 1.0;
        }
        double2 x[R];
#pragma unroll
        for (int al = 0; al < R; al++) {
            const double w = inb[al] ? 2.0 * df * wpsd[al] : 0.0;
            const double2 hh = hv[al], d = dv[al];
            x[al] = make_double2((hh.x * d.x + hh.y * d.y) * w, (hh.x * d.y - hh.y * d.x) * w);
        }
        double2 wr[R];   // e^{2 pi i r / R}
#pragma unroll
        for (int r = 0; r < R; r++) wr[r] = tw[(int64_t)r * n2];
        dft_radix2<R>(x, wr);
#pragma unroll
        for (int q = 0; q < R; q++) {
            const double2 t = tw[m2 * q];   // e^{2 pi i m2 q / n}, m2 q < n
            yq[q] = make_double2(x[q].x * t.x - x[q].y * t.y, x[q].x * t.y + x[q].y * t.x);
        }
    }
    const int64_t ncol = cols - col0 < kDecC ? cols - col0 : kDecC;
#pragma unroll
    for (int h = 0; h < R / QC; h++) {
        if (h > 0) __syncthreads();   // the previous pass's reads are done
        if (live) {
#pragma unroll
            for (int q = 0; q < QC; q++) sY[lane * RW + wv * QC + q] = yq[h * QC + q];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < kDecM * kDecC * QC; e += kQvThreads) {
            const int row = e / (kDecC * QC), c = e % (kDecC * QC);
            const int cl = c / QC, q = h * QC + c % QC;
            if (m2_0 + row < n2 && cl < ncol)
                Y[(m2_0 + row) * cols * R + (col0 + cl) * R + q] = sY[row * RW + c];
        }
    }
}

// Q[col][i] of the decimated route: the slice partials of decimated column
// col R + q at decimated time p - p_lo, j = i - win_half = R p + q, summed
// in slice order.
__global__ void k_qv_dec_reduce(const double2 *__restrict__ part, int n_slices, int64_t cols, int radix, int n_t2,
                                int n_time, int win_half, int p_lo, double2 *__restrict__ Q) {
    const int64_t total = cols * n_time;
    const int64_t stride = cols * radix * n_t2;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t col = e / n_time;
        const int j = (int)(e % n_time) - win_half;
        const int pd = j >= 0 ? j / radix : -((-j + radix - 1) / radix);
        const int q = j - pd * radix;
        const int64_t src = (col * radix + q) * n_t2 + (pd - p_lo);
        double re = 0.0, im = 0.0;
        for (int s = 0; s < n_slices; s++) {
            const double2 v = part[(int64_t)s * stride + src];
            re += v.x;
            im += v.y;
        }
        Q[e] = make_double2(re, im);
    }
}

// U and V: a block per (point, band slice, detector group of up to kUvDet,
// pair group of up to kQvThreads pairs a <= b).  The block stages chunks of
// its band slice in LDS: h_a(f) and h_a(-f) of every mode and w_k(f) of its
// detectors.  Each thread accumulates one pair for all the group's detectors
// over every G-th bin of a chunk (G bin lanes per pair); the lanes are summed
// in lane order, and the slices in slice order by k_qv_uv_sum (with one slice
// the block writes U and V itself).  Deterministic for a given launch shape.
constexpr int kUvDet = 4;
constexpr int kUvChunk = 128;  // bins per LDS chunk (fewer for many modes)

__device__ __forceinline__ void uv_pair(int q, int na, int &a, int &b) {
    a = 0;
    while (q >= na - a) {
        q -= na - a;
        a++;
    }
    b = a + q;
}

__device__ __forceinline__ void uv_store(double2 *U, double2 *V, int64_t base, int na, int a, int b, double f,
                                         const double (&s)[4]) {
    const double ui = a == b ? 0.0 : f * s[1];   // the diagonal <h_a|h_a> is real
    U[base + a * na + b] = make_double2(f * s[0], ui);
    U[base + b * na + a] = make_double2(f * s[0], -ui);
    V[base + a * na + b] = make_double2(f * s[2], f * s[3]);
    V[base + b * na + a] = make_double2(f * s[2], f * s[3]);
}

__global__ void __launch_bounds__(kQvThreads)
    k_qv_uv(const double2 *__restrict__ hlm, const double *__restrict__ inv_psd, const int64_t *__restrict__ band,
            int64_t n_band, int64_t n, int na, int nd, double df, int64_t slice, int n_sl, int cb, int n_dg,
            double *__restrict__ partial, double2 *__restrict__ U, double2 *__restrict__ V) {
    extern __shared__ double uv_lds[];
    const int npair = na * (na + 1) / 2;
    const int64_t p = blockIdx.x;
    const int sl = blockIdx.y;
    const int dg = (int)(blockIdx.z % n_dg), pg = (int)(blockIdx.z / n_dg);
    const int k0 = dg * kUvDet;
    const int nk = nd - k0 < kUvDet ? nd - k0 : kUvDet;
    const int pair0 = pg * kQvThreads;
    const int np_here = npair - pair0 < kQvThreads ? npair - pair0 : kQvThreads;
    const int G = kQvThreads / np_here;
    const int tid = threadIdx.x;
    const bool active = tid < np_here * G;
    const int lp = tid % np_here, g = tid / np_here;
    int a = 0, b = 0;
    uv_pair(pair0 + lp, na, a, b);
    double2 *sH = (double2 *)uv_lds;            // [na][cb]  h_a(f)
    double2 *sM = sH + (size_t)na * cb;         // [na][cb]  h_a(-f)
    double *sW = (double *)(sM + (size_t)na * cb);   // [kUvDet][cb]
    double acc[kUvDet][4];
#pragma unroll
    for (int kk = 0; kk < kUvDet; kk++)
#pragma unroll
        for (int c = 0; c < 4; c++) acc[kk][c] = 0.0;
    const int64_t e_lo = (int64_t)sl * slice;
    const int64_t e_hi = e_lo + slice < n_band ? e_lo + slice : n_band;
    for (int64_t eb = e_lo; eb < e_hi; eb += cb) {
        const int ncb = e_hi - eb < cb ? (int)(e_hi - eb) : cb;
        __syncthreads();
        for (int s = tid; s < na * ncb; s += kQvThreads) {
            const int am = s / ncb, c = s % ncb;
            const int64_t m = band[eb + c];
            const int64_t mn = m == 0 ? 0 : n - m;
            const double2 *h = hlm + (p * na + am) * n;
            sH[am * cb + c] = h[m];
            sM[am * cb + c] = h[mn];
        }
        for (int s = tid; s < nk * ncb; s += kQvThreads) {
            const int kk = s / ncb, c = s % ncb;
            sW[kk * cb + c] = inv_psd ? inv_psd[(int64_t)(k0 + kk) * n + band[eb + c]] : 1.0;
        }
        __syncthreads();
        if (active) {
            for (int c = g; c < ncb; c += G) {
                const double2 x = sH[a * cb + c], y = sH[b * cb + c], z = sM[a * cb + c];
                const double p0 = x.x * y.x + x.y * y.y, p1 = x.x * y.y - x.y * y.x;   // conj(h_a) h_b
                const double p2 = z.x * y.x - z.y * y.y, p3 = z.x * y.y + z.y * y.x;   // h_a(-f) h_b
#pragma unroll
                for (int kk = 0; kk < kUvDet; kk++) {
                    if (kk < nk) {
                        const double w = sW[kk * cb + c];
                        acc[kk][0] += w * p0;
                        acc[kk][1] += w * p1;
                        acc[kk][2] += w * p2;
                        acc[kk][3] += w * p3;
                    }
                }
            }
        }
    }
    // bin lanes summed in lane order
    __syncthreads();
    double *red = uv_lds;   // [kQvThreads][kUvDet * 4]
#pragma unroll
    for (int kk = 0; kk < kUvDet; kk++)
#pragma unroll
        for (int c = 0; c < 4; c++) red[tid * kUvDet * 4 + kk * 4 + c] = acc[kk][c];
    __syncthreads();
    if (!active || g != 0) return;
    for (int kk = 0; kk < nk; kk++) {
        double s[4] = {0.0, 0.0, 0.0, 0.0};
        for (int gg = 0; gg < G; gg++)
#pragma unroll
            for (int c = 0; c < 4; c++) s[c] += red[(gg * np_here + lp) * kUvDet * 4 + kk * 4 + c];
        const int64_t pk = p * nd + k0 + kk;
        if (n_sl == 1) {
            uv_store(U, V, pk * na * na, na, a, b, 2.0 * df, s);
        } else {
            double *o = partial + ((pk * npair + pair0 + lp) * n_sl + sl) * 4;
#pragma unroll
            for (int c = 0; c < 4; c++) o[c] = s[c];
        }
    }
}

// U and V from the slice partials, summed in slice order.
__global__ void k_qv_uv_sum(const double *__restrict__ partial, int64_t n_pk, int na, int n_sl, double df,
                            double2 *__restrict__ U, double2 *__restrict__ V) {
    const int npair = na * (na + 1) / 2;
    const int64_t total = n_pk * npair;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t pk = e / npair;
        int a, b;
        uv_pair((int)(e % npair), na, a, b);
        double s[4] = {0.0, 0.0, 0.0, 0.0};
        for (int sl = 0; sl < n_sl; sl++)
#pragma unroll
            for (int c = 0; c < 4; c++) s[c] += partial[(e * n_sl + sl) * 4 + c];
        uv_store(U, V, pk * na * na, na, a, b, 2.0 * df, s);
    }
}

// U and V (k_qv_uv, then k_qv_uv_sum over its band slices): band slices so
// that the grid has about 1024 blocks, the slice partials held in `part`
// (part_bytes long; free once Q has been reduced from it).
void launch_uv(const void *hlm, const double *inv_psd, const int64_t *band, int64_t n_band, int64_t n, int na,
               int nd, int np, double df, double *part, int64_t part_bytes, void *U, void *V, hipStream_t st) {
    const int npair = na * (na + 1) / 2;
    const int n_dg = (nd + kUvDet - 1) / kUvDet;
    const int n_pg = (npair + kQvThreads - 1) / kQvThreads;
    const int cb = (int)std::max<int64_t>(1, std::min<int64_t>(kUvChunk, 49152 / ((int64_t)na * 32 + kUvDet * 8)));
    const int64_t blocks1 = (int64_t)np * n_dg * n_pg;
    int64_t n_sl = std::max<int64_t>(1, std::min<int64_t>((1024 + blocks1 - 1) / blocks1, (n_band + 4 * cb - 1) / (4 * cb)));
    const int64_t per_sl = (int64_t)np * nd * npair * 32;
    n_sl = std::min<int64_t>(n_sl, std::max<int64_t>(1, part_bytes / per_sl));
    const int64_t uslice = (n_band + n_sl - 1) / n_sl;
    n_sl = (n_band + uslice - 1) / uslice;
    const size_t lds = std::max<size_t>((size_t)cb * ((size_t)na * 32 + kUvDet * 8), (size_t)kQvThreads * kUvDet * 4 * 8);
    hipLaunchKernelGGL(k_qv_uv, dim3((unsigned)np, (unsigned)n_sl, (unsigned)(n_dg * n_pg)), dim3(kQvThreads), lds, st,
                       (const double2 *)hlm, inv_psd, band, n_band, n, na, nd, df, uslice, (int)n_sl, cb, n_dg,
                       part, (double2 *)U, (double2 *)V);
    if (n_sl > 1) {
        const int64_t ue = (int64_t)np * nd * npair;
        hipLaunchKernelGGL(k_qv_uv_sum, dim3((unsigned)std::min<int64_t>((ue + 255) / 256, 65536)), dim3(256), 0, st,
                           part, (int64_t)np * nd, na, (int)n_sl, df, (double2 *)U, (double2 *)V);
    }
}

}  // namespace

size_t qv_scratch_bytes(int64_t n, int64_t n_band, int64_t cols, int n_time, int n_slices) {
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    return al((size_t)n * 16) + al((size_t)n_band * 8) * 2 + al((size_t)n_band * cols * 16) +
           al((size_t)n_slices * cols * n_time * 16);
}

namespace {

// Band slices per call: at least two rounds of resident blocks (256 CUs x 2
// blocks of k_qv_q), at least 128 bins per slice, and the fewest slices whose
// last round is at least 90 % full.

int slices_for(int64_t n_band, int64_t tiles) {
    constexpr int64_t kResident = 256 * 2;
    int64_t smax = (n_band + 127) / 128;
    smax = smax < 1 ? 1 : smax;
    int64_t best = 1;
    double best_eff = -1.0;
    for (int64_t s = 1; s <= smax && s <= 64; s++) {
        const int64_t blocks = tiles * s;
        const int64_t rounds = (blocks + kResident - 1) / kResident;
        const double eff = (double)blocks / (double)(rounds * kResident);
        if (blocks >= 2 * kResident && eff >= 0.9) return (int)s;
        if (eff > best_eff + 1e-9) {
            best_eff = eff;
            best = s;
        }
    }
    return (int)best;
}

}  // namespace

int qv_slices(int64_t n_band, int64_t cols, int n_time) {
    return slices_for(n_band, (int64_t)((n_time + kQvTT - 1) / kQvTT) * ((cols + kQvTC - 1) / kQvTC));
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
    const int64_t xruns = std::min<int64_t>((n_band + kQvXRun - 1) / kQvXRun, 65535);
    hipLaunchKernelGGL(k_qv_x, dim3((unsigned)((cols + kQvThreads - 1) / kQvThreads), (unsigned)xruns),
                       dim3(kQvThreads), 0, st, (const double2 *)hlm, (const double2 *)data, inv_psd, band, n_band, n,
                       na, nd, np, df, X);
    const int64_t slice = ((n_band + n_slices - 1) / n_slices + kQvKB - 1) / kQvKB * kQvKB;
    const int ns = (int)((n_band + slice - 1) / slice);
    const int n_tt = (n_time + kQvTT - 1) / kQvTT;
    const int n_tc = (int)((cols + kQvTC - 1) / kQvTC);
    hipLaunchKernelGGL(k_qv_q<kQvTT>, dim3((unsigned)((int64_t)n_tt * n_tc * ns)), dim3(kQvThreads), 0, st, X, tw, msig,
                       n_band, n, cols, n_time, win_half, slice, n_tt, n_tc, part);
    const int64_t qe = cols * n_time;
    hipLaunchKernelGGL(k_qv_reduce, dim3((unsigned)std::min<int64_t>((qe + 255) / 256, 65536)), dim3(256), 0, st,
                       part, ns, cols, n_time, (double2 *)Q);
    launch_uv(hlm, inv_psd, band, n_band, n, na, nd, np, df, (double *)part, (int64_t)ns * cols * n_time * 16, U, V,
              st);
    return hipGetLastError();
}

namespace {

int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// The decimated times p_lo .. p_lo + n_t2 - 1 that the window covers.
void dec_window(int n_time, int win_half, int radix, int &p_lo, int &n_t2) {
    p_lo = floor_div(-win_half, radix);
    n_t2 = floor_div(n_time - 1 - win_half, radix) - p_lo + 1;
}

// The decimated times' tile height (32 or 64; 0 when they do not fit one).
int dec_tile(int n_t2) { return n_t2 <= 32 ? 32 : (n_t2 <= 64 ? 64 : 0); }

// Cost per column in complex matrix-core products: the direct sum takes
// (padded window) x n_band; the decimated one (tile height) x n for the
// product, about 49 per bin for the radix partial sums' 16-byte element
// written and read back (Y against X), at the measured rates (6.1e12
// products/s, 4 TB/s), and 2R per bin for their R-point sums on the vector
// units.
double dec_cost(int64_t n, int tile, int radix) { return (double)(tile + 49 + 2 * radix) * (double)n; }

}  // namespace

int qv_radix(int64_t n, int64_t n_band, int n_time, int win_half, bool force) {
    int best = 0;
    double best_cost = 0.0;
    for (int r = 2; r <= 16; r *= 2) {
        if (n % r != 0) continue;
        int p_lo, n_t2;
        dec_window(n_time, win_half, r, p_lo, n_t2);
        const int tile = dec_tile(n_t2);
        if (tile == 0) continue;
        const double c = dec_cost(n, tile, r);
        if (best == 0 || c < best_cost) {
            best = r;
            best_cost = c;
        }
    }
    if (best == 0 || force) return best;
    const double direct = (double)((n_time + kQvTT - 1) / kQvTT * kQvTT + 49) * (double)n_band;
    return best_cost < direct ? best : 0;
}

int qv_dec_slices(int64_t n, int64_t cols, int n_time, int win_half, int radix) {
    int p_lo, n_t2;
    dec_window(n_time, win_half, radix, p_lo, n_t2);
    const int64_t tc = qv_tc(dec_tile(n_t2));
    return slices_for(n / radix, (cols * radix + tc - 1) / tc);
}

size_t qv_dec_scratch_bytes(int64_t n, int64_t n_band, int64_t cols, int n_time, int win_half, int radix,
                            int n_slices) {
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    int p_lo, n_t2;
    dec_window(n_time, win_half, radix, p_lo, n_t2);
    return al((size_t)n * 16) + al((size_t)(n / radix) * 16) + al((size_t)n_band * 8) + al((size_t)n * cols * 16) + al((size_t)n_slices * cols * radix * n_t2 * 16);
}

hipError_t launch_qv_dec(const void *hlm, const void *data, const double *inv_psd, int64_t n, int na, int nd,
                         int np, double df, double f_lo, double f_hi, const int64_t *h_band, int64_t n_band,
                         int n_time, int win_half, int radix, void *Q, void *U, void *V, void *scratch,
                         int n_slices, hipStream_t st) {
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    const int64_t n2 = n / radix;
    const int64_t cols = (int64_t)np * nd * na;
    const int64_t cols2 = cols * radix;
    int p_lo, n_t2;
    dec_window(n_time, win_half, radix, p_lo, n_t2);
    char *w = (char *)scratch;
    double2 *tw = (double2 *)w;
    w += al((size_t)n * 16);
    double2 *tw2 = (double2 *)w;
    w += al((size_t)n2 * 16);
    int64_t *band = (int64_t *)w;
    w += al((size_t)n_band * 8);
    double2 *Y = (double2 *)w;
    w += al((size_t)n * cols * 16);
    double2 *part = (double2 *)w;
    hipError_t e = hipMemcpyAsync(band, h_band, (size_t)n_band * 8, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_qv_twiddle, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, tw, n);
    hipLaunchKernelGGL(k_qv_twiddle, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, tw2, n2);
    const int64_t n_mt = (n2 + kDecM - 1) / kDecM;
    const dim3 g1((unsigned)(n_mt * ((cols + kDecC - 1) / kDecC)));
    switch (radix) {
    case 2:
        hipLaunchKernelGGL(k_qv_dec1<2>, g1, dim3(kQvThreads), 0, st, (const double2 *)hlm, (const double2 *)data,
                           inv_psd, tw, n, na, nd, np, df, f_lo, f_hi, n_mt, Y);
        break;
    case 4:
        hipLaunchKernelGGL(k_qv_dec1<4>, g1, dim3(kQvThreads), 0, st, (const double2 *)hlm, (const double2 *)data,
                           inv_psd, tw, n, na, nd, np, df, f_lo, f_hi, n_mt, Y);
        break;
    case 8:
        hipLaunchKernelGGL(k_qv_dec1<8>, g1, dim3(kQvThreads), 0, st, (const double2 *)hlm, (const double2 *)data,
                           inv_psd, tw, n, na, nd, np, df, f_lo, f_hi, n_mt, Y);
        break;
    case 16:
        hipLaunchKernelGGL(k_qv_dec1<16>, g1, dim3(kQvThreads), 0, st, (const double2 *)hlm, (const double2 *)data,
                           inv_psd, tw, n, na, nd, np, df, f_lo, f_hi, n_mt, Y);
        break;
    default:
        return hipErrorInvalidValue;
    }
    // the product over the N2 decimated bins (m2 itself as the signed index:
    // its phase only enters modulo N2) at decimated times p = t + p_lo
    const int64_t slice = ((n2 + n_slices - 1) / n_slices + kQvKB - 1) / kQvKB * kQvKB;
    const int ns = (int)((n2 + slice - 1) / slice);
    const int tile = dec_tile(n_t2);
    const int n_tc = (int)((cols2 + qv_tc(tile) - 1) / qv_tc(tile));
    if (tile == 32)
        hipLaunchKernelGGL(k_qv_q<32>, dim3((unsigned)((int64_t)n_tc * ns)), dim3(kQvThreads), 0, st, Y, tw2,
                           (const int64_t *)nullptr, n2, n2, cols2, n_t2, -p_lo, slice, 1, n_tc, part);
    else if (tile == 64)
        hipLaunchKernelGGL(k_qv_q<64>, dim3((unsigned)((int64_t)n_tc * ns)), dim3(kQvThreads), 0, st, Y, tw2,
                           (const int64_t *)nullptr, n2, n2, cols2, n_t2, -p_lo, slice, 1, n_tc, part);
    else
        return hipErrorInvalidValue;
    const int64_t qe = cols * n_time;
    hipLaunchKernelGGL(k_qv_dec_reduce, dim3((unsigned)std::min<int64_t>((qe + 255) / 256, 65536)), dim3(256), 0, st,
                       part, ns, cols, radix, n_t2, n_time, win_half, p_lo, (double2 *)Q);
    launch_uv(hlm, inv_psd, band, n_band, n, na, nd, np, df, (double *)part, (int64_t)ns * cols2 * n_t2 * 16, U, V,
              st);
    return hipGetLastError();
}

}  // namespace ile
