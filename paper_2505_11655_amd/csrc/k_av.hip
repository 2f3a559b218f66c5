// Adaptive volume integration (Section "Adaptive volume integration") on the
// GPU: the sampler is uniform over a set of active hypercubes of a grid of nb
// bins per sampled column, in the unit cube of the prior's CDF coordinates u
// (theta = inverse-CDF map of u), so ln p - ln p_s = ln V with V the active
// volume.  After a round of n samples with log-weights lw:
//   1. threshold: the largest lw value v such that the samples at or above v
//      hold at least min(ceil(p_thr * total), total) of the fixed-point masses
//      q_i = floor(exp(lw_i - max lw) 2^40) and number at least
//      min(n_min_live, n_finite).  Found by two radix selects (one on the
//      enclosed mass, one on the count) over order-preserving integer keys of
//      lw, eight bits per pass; integer sums make it independent of the order
//      of accumulation.
//   2. refinement, eq. (nbins_V): nb' = ceil((1/dV)^(1/d)) with
//      dV = V n_min / (n sqrt(n_min)), clamped to [1, max_bins].
//   3. the new active cells: the cells of the nb' grid holding a sample at or
//      above the threshold, each listed once, in order of its first such
//      sample (an open-addressing set keeps each cell's lowest sample index;
//      a block-count scan compacts the first samples in index order).
// A sample's u is regenerated from its Philox counter and the grid it was
// drawn from, so the update needs no stored coordinates.
//
// Counter layout (the prior draw's): sample i of round r uses blocks 0..3 of
// attempt 0, ctr = (i lo, i hi, r, b); column c takes u53(w[2c], w[2c+1]) and
// the cell is floor(u53(w14, w15) n_cells) (at most n_cells - 1), so the
// one-cell grid draws exactly the prior.
#include "ile_internal.h"

namespace ile {

namespace {

constexpr int kAvThreads = 256;
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;
constexpr unsigned long long kEmpty = ~0ull;

__device__ __forceinline__ void av_words(uint64_t seed, uint64_t i, uint32_t r, uint32_t *w) {
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

// Unit-cube coordinates of one sample drawn from the grid (nb, n_cells, cells).
__device__ __forceinline__ void av_unit(const AvDev &S, const uint16_t *cells, const uint32_t *w, double u[7]) {
    const double sel = floor(u53(w[14], w[15]) * (double)S.n_cells);
    int64_t j = (int64_t)sel;
    if (j > S.n_cells - 1) j = S.n_cells - 1;
    const uint16_t *cj = cells + j * 8;
    const double nbd = (double)S.nb;
#pragma unroll
    for (int c = 0; c < 7; c++) {
        const double U = u53(w[2 * c], w[2 * c + 1]);
        const int k = S.kcol[c];
        u[c] = k >= 0 ? ((double)cj[k] + U) / nbd : U;
    }
}

__device__ __forceinline__ const uint16_t *cur_cells(const AvBufs &b, const AvDev &S) {
    return S.cur ? b.cells[1] : b.cells[0];
}

__device__ __forceinline__ unsigned long long mix64(unsigned long long x) {
    x ^= x >> 30;
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 27;
    x *= 0x94D049BB133111EBull;
    x ^= x >> 31;
    return x;
}

__global__ void k_av_reset(AvBufs b, int d, int d0, int d1, int d2, int d3, int d4, int d5, int d6) {
    if (threadIdx.x != 0) return;
    AvDev &S = *b.st;
    const int dims[7] = {d0, d1, d2, d3, d4, d5, d6};
    S.d = d;
    for (int c = 0; c < 7; c++) S.kcol[c] = -1;
    for (int k = 0; k < 7; k++) {
        S.dims[k] = k < d ? dims[k] : -1;
        if (k < d) S.kcol[dims[k]] = k;
    }
    S.nb = 1;
    S.nb_next = 1;
    S.cur = 0;
    S.valid = 0;
    S.n_cells = 1;
    S.n_cells_next = 1;
    S.ln_vol = 0.0;
    S.thr = -INFINITY;
    S.n_min = 0;
    S.n_live = 0;
    S.vol_mc = 0.0;
    for (int k = 0; k < 8; k++) b.cells[0][k] = 0;
}

// Samples of job blockIdx.z: each block strides over its job's samples.
#define AV_JOB const AvJob &J = jobs[blockIdx.z]
#define AV_SAMPLES(s) \
    for (int64_t s = (int64_t)blockIdx.x * kAvThreads + threadIdx.x; s < J.n; s += (int64_t)gridDim.x * kAvThreads)

template <class TT>
__global__ void __launch_bounds__(kAvThreads) k_av_draw(const AvJob *__restrict__ jobs) {
    AV_JOB;
    const AvDev &S = *J.b.st;
    const uint16_t *cells = cur_cells(J.b, S);
    const double lnv = S.ln_vol;
    TT *th_out = (TT *)J.theta;
    TT *lr_out = (TT *)J.lnpmps;
    AV_SAMPLES(s) {
        uint32_t w[16];
        av_words(J.seed, (uint64_t)(J.first + s), J.round, w);
        double u[7], th[7];
        av_unit(S, cells, w, u);
        prior_map(J.pr, u, th);
#pragma unroll
        for (int c = 0; c < 7; c++) th_out[c * J.ld + s] = (TT)th[c];
        if (lr_out) lr_out[s] = (TT)lnv;
    }
}

__global__ void k_av_begin(const AvJob *__restrict__ jobs) {
    AV_JOB;
    AvDev &S = *J.b.st;
    if (threadIdx.x == 0) {
        S.key_max = 0;
        S.n_fin = 0;
        S.total = 0;
        for (int c = 0; c < 2; c++) {
            S.prefix[c] = 0;
            S.above_cnt[c] = 0;
            S.above_mass[c] = 0;
            S.target[c] = 0;
            S.last_cnt[c] = 0;
        }
        S.valid = 0;
        S.thr = -INFINITY;
        S.n_min = 0;
        S.n_live = J.n;
        S.vol_mc = 0.0;
    }
    for (int i = threadIdx.x; i < 2 * 256 * 2; i += blockDim.x) J.b.hist[i] = 0;
}

template <class TO>
__global__ void __launch_bounds__(kAvThreads) k_av_max(const AvJob *__restrict__ jobs) {
    AV_JOB;
    const TO *lw = (const TO *)J.lw;
    unsigned long long km = 0, cnt = 0;
    AV_SAMPLES(s) {
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
    __shared__ unsigned long long smk[kAvThreads / 64], smc[kAvThreads / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        smk[wv] = km;
        smc[wv] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kAvThreads / 64; i++) {
            km = smk[i] > km ? smk[i] : km;
            cnt += smc[i];
        }
        if (cnt) {
            atomicMax(&J.b.st->key_max, km);
            atomicAdd(&J.b.st->n_fin, cnt);
        }
    }
}

// One radix-select pass: digit (key >> shift) & 255 of every finite sample
// whose higher digits match the chain's prefix; chain 0 counts and sums the
// fixed-point masses, chain 1 counts.
template <class TO>
__global__ void __launch_bounds__(kAvThreads) k_av_hist(const AvJob *__restrict__ jobs, int shift) {
    AV_JOB;
    const AvDev &S = *J.b.st;
    if (S.n_fin == 0 || (int64_t)blockIdx.x * kAvThreads >= J.n) return;
    __shared__ unsigned long long h[2 * 256 * 2];
    for (int i = threadIdx.x; i < 2 * 256 * 2; i += kAvThreads) h[i] = 0;
    __syncthreads();
    constexpr int nbits = sizeof(TO) * 8;
    const bool top = shift + 8 == nbits;
    const unsigned long long p0 = top ? 0 : (S.prefix[0] >> (shift + 8));
    const unsigned long long p1 = top ? 0 : (S.prefix[1] >> (shift + 8));
    const double vmax = ord_value(S.key_max, nbits);
    const TO *lw = (const TO *)J.lw;
    AV_SAMPLES(s) {
        const TO v = lw[s];
        if (!isfinite(v)) continue;
        const unsigned long long k = ord_key(v);
        const unsigned long long hi = top ? 0 : (k >> (shift + 8));
        const int dg = (int)((k >> shift) & 255u);
        if (hi == p0) {
            atomicAdd(&h[(0 * 256 + dg) * 2 + 0], 1ull);
            atomicAdd(&h[(0 * 256 + dg) * 2 + 1], mass_fx((double)v, vmax));
        }
        if (hi == p1) atomicAdd(&h[(1 * 256 + dg) * 2 + 0], 1ull);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 2 * 256 * 2; i += kAvThreads)
        if (h[i]) atomicAdd(&J.b.hist[i], h[i]);
}

// Each chain's digit: thread d holds bucket d; suffix sums from the top
// bucket down give the enclosed count and mass at and above each bucket, and
// the chosen digit is the highest bucket where the chain's target is reached.
// After the last pass: the threshold, n_min and eq. (nbins_V).  The selection
// state is read once, carried in LDS between threads, and written back.
__global__ void __launch_bounds__(256) k_av_pick(const AvJob *__restrict__ jobs, int shift, int nbits) {
    AV_JOB;
    AvDev &S = *J.b.st;
    if (S.n_fin == 0) return;
    unsigned long long *H = J.b.hist;
    const int d = threadIdx.x;
    __shared__ unsigned long long sc[256], sm[256];
    __shared__ unsigned long long t_target[2], t_acnt[2], t_amass[2], t_prefix[2], t_last[2];
    __shared__ int pick;
    if (d < 2) {
        t_target[d] = S.target[d];
        t_acnt[d] = S.above_cnt[d];
        t_amass[d] = S.above_mass[d];
        t_prefix[d] = S.prefix[d];
        t_last[d] = S.last_cnt[d];
    }
    if (shift + 8 == nbits) {
        sm[d] = H[(0 * 256 + d) * 2 + 1];
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (d < o) sm[d] += sm[d + o];
            __syncthreads();
        }
        if (d == 0) {
            const unsigned long long tot = sm[0], nfin = S.n_fin;
            const unsigned long long tm = (unsigned long long)ceil(J.p_thr * (double)tot);
            t_target[0] = tm < tot ? tm : tot;
            t_target[1] = (unsigned long long)J.n_min_live < nfin ? (unsigned long long)J.n_min_live : nfin;
            S.total = tot;
            S.target[0] = t_target[0];
            S.target[1] = t_target[1];
            S.valid = 1;
        }
    }
    __syncthreads();
    for (int c = 0; c < 2; c++) {
        // suffix sums: position r = 255 - d holds bucket d, inclusive prefix over r
        const unsigned long long cc = H[(c * 256 + d) * 2 + 0], mm = H[(c * 256 + d) * 2 + 1];
        sc[255 - d] = cc;
        sm[255 - d] = mm;
        if (d == 0) pick = -1;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {
            const unsigned long long ac = d >= o ? sc[d - o] : 0ull, am = d >= o ? sm[d - o] : 0ull;
            __syncthreads();
            sc[d] += ac;
            sm[d] += am;
            __syncthreads();
        }
        const unsigned long long suf_c = sc[255 - d], suf_m = sm[255 - d];
        const bool hit = c == 0 ? (t_amass[0] + suf_m >= t_target[0]) : (t_acnt[1] + suf_c >= t_target[1]);
        if (hit) atomicMax(&pick, d);
        __syncthreads();
        if (d == pick) {
            t_last[c] = cc;
            t_acnt[c] += suf_c - cc;
            t_amass[c] += suf_m - mm;
            t_prefix[c] |= (unsigned long long)d << shift;
        }
        __syncthreads();
    }
    if (d < 2) {
        S.above_cnt[d] = t_acnt[d];
        S.above_mass[d] = t_amass[d];
        S.prefix[d] = t_prefix[d];
        S.last_cnt[d] = t_last[d];
    }
    if (d == 0 && shift == 0) {
        const int c = t_prefix[0] <= t_prefix[1] ? 0 : 1;
        const int64_t n_min = (int64_t)(t_acnt[c] + t_last[c]);
        const double ln_vol = S.ln_vol;
        S.thr_key = t_prefix[c];
        S.n_min = n_min;
        S.thr = ord_value(t_prefix[c], nbits);
        S.vol_mc = exp(ln_vol) * (double)n_min / (double)J.n;
        const double ln_dv = ln_vol + 0.5 * log((double)n_min) - log((double)J.n);
        const double x = exp(-ln_dv / (double)S.d);
        double nbd = ceil(x - 1e-9);
        nbd = nbd < 1.0 ? 1.0 : (nbd > (double)J.max_bins ? (double)J.max_bins : nbd);
        S.nb_next = (int)nbd;
    }
    for (int i = d; i < 2 * 256 * 2; i += 256) H[i] = 0;
}

__global__ void __launch_bounds__(kAvThreads) k_av_hclear(const AvJob *__restrict__ jobs) {
    AV_JOB;
    const AvDev &S = *J.b.st;
    if (!S.valid) return;
    // only the part of the set an update of J.n samples can use (>= 2 J.n slots)
    uint64_t used = 1024;
    while (used < (uint64_t)2 * (uint64_t)J.n) used <<= 1;
    used = used - 1 < J.b.hmask ? used : J.b.hmask + 1;
    for (uint64_t i = (uint64_t)blockIdx.x * kAvThreads + threadIdx.x; i < used; i += (uint64_t)gridDim.x * kAvThreads) {
        J.b.hkey[i] = kEmpty;
        J.b.hidx[i] = kNoSlot;
    }
}

// The set of one update uses its first `used` slots (a power of two >= 2n).
__device__ __forceinline__ uint64_t av_set_mask(const AvJob &J) {
    uint64_t used = 1024;
    while (used < (uint64_t)2 * (uint64_t)J.n) used <<= 1;
    return (used - 1 < J.b.hmask ? used : J.b.hmask + 1) - 1;
}

// Cells (of the refined grid) of the samples at or above the threshold, into
// the set; each slot keeps the lowest sample index that reached it.
template <class TO>
__global__ void __launch_bounds__(kAvThreads) k_av_insert(const AvJob *__restrict__ jobs) {
    AV_JOB;
    const AvDev &S = *J.b.st;
    if (!S.valid) return;
    const unsigned long long thr = S.thr_key;
    const unsigned long long nb2 = (unsigned long long)S.nb_next;
    const double nb2d = (double)S.nb_next;
    const uint16_t *cells = cur_cells(J.b, S);
    const uint64_t mask = av_set_mask(J);
    const TO *lw = (const TO *)J.lw;
    AV_SAMPLES(s) {
        const TO v = lw[s];
        uint32_t sl = kNoSlot;
        if (isfinite(v) && ord_key(v) >= thr) {
            uint32_t w[16];
            av_words(J.seed, (uint64_t)(J.first + s), J.round, w);
            double u[7];
            av_unit(S, cells, w, u);
            unsigned long long id = 0;
#pragma unroll
            for (int c = 6; c >= 0; c--) {
                if (S.kcol[c] >= 0) {
                    double f = floor(u[c] * nb2d);
                    f = f > nb2d - 1.0 ? nb2d - 1.0 : f;
                    id = id * nb2 + (unsigned long long)f;
                }
            }
            uint64_t h = mix64(id) & mask;
            for (uint64_t probe = 0; probe <= mask; probe++) {
                const unsigned long long prev = atomicCAS(&J.b.hkey[h], kEmpty, id);
                if (prev == kEmpty || prev == id) {
                    atomicMin(&J.b.hidx[h], (uint32_t)s);
                    sl = (uint32_t)h;
                    break;
                }
                h = (h + 1) & mask;
            }
        }
        J.b.slot[s] = sl;
    }
}

// The sample is the first (lowest index) of its cell.
__device__ __forceinline__ bool av_first(const AvJob &J, int64_t s) {
    if (s >= J.n) return false;
    const uint32_t sl = J.b.slot[s];
    return sl != kNoSlot && J.b.hidx[sl] == (uint32_t)s;
}

__global__ void __launch_bounds__(kAvThreads) k_av_count(const AvJob *__restrict__ jobs) {
    AV_JOB;
    const AvDev &S = *J.b.st;
    if (!S.valid || (int64_t)blockIdx.x * kAvThreads >= J.n) return;
    const int64_t s = (int64_t)blockIdx.x * kAvThreads + threadIdx.x;
    const int c = __syncthreads_count(av_first(J, s));
    if (threadIdx.x == 0) J.b.bcnt[blockIdx.x] = (uint32_t)c;
}

// Exclusive scan of the per-block counts in place; the total is the new
// number of cells.
constexpr int kScanThreads = 1024;
__global__ void __launch_bounds__(kScanThreads) k_av_scan(const AvJob *__restrict__ jobs) {
    AV_JOB;
    AvDev &S = *J.b.st;
    if (!S.valid) return;
    const int nblk = (int)((J.n + kAvThreads - 1) / kAvThreads);
    __shared__ unsigned long long sm[kScanThreads];
    const int per = (nblk + kScanThreads - 1) / kScanThreads;
    const int lo = threadIdx.x * per, hi = lo + per < nblk ? lo + per : nblk;
    unsigned long long loc = 0;
    for (int i = lo; i < hi; i++) loc += J.b.bcnt[i];
    sm[threadIdx.x] = loc;
    __syncthreads();
    for (int o = 1; o < kScanThreads; o <<= 1) {
        const unsigned long long add = threadIdx.x >= (unsigned)o ? sm[threadIdx.x - o] : 0ull;
        __syncthreads();
        sm[threadIdx.x] += add;
        __syncthreads();
    }
    unsigned long long run = sm[threadIdx.x] - loc;
    for (int i = lo; i < hi; i++) {
        const uint32_t c = J.b.bcnt[i];
        J.b.bcnt[i] = (uint32_t)run;
        run += c;
    }
    if (threadIdx.x == kScanThreads - 1) S.n_cells_next = (int64_t)sm[kScanThreads - 1];
}

__global__ void __launch_bounds__(kAvThreads) k_av_compact(const AvJob *__restrict__ jobs) {
    AV_JOB;
    const AvDev &S = *J.b.st;
    if (!S.valid || (int64_t)blockIdx.x * kAvThreads >= J.n) return;
    const int64_t s = (int64_t)blockIdx.x * kAvThreads + threadIdx.x;
    const bool f = av_first(J, s);
    const unsigned long long m = __ballot(f);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __shared__ int wc[kAvThreads / 64];
    if (lane == 0) wc[wv] = __popcll(m);
    __syncthreads();
    if (!f) return;
    int off = 0;
    for (int i = 0; i < wv; i++) off += wc[i];
    const int rank = __popcll(m & ((1ull << lane) - 1ull));
    const int64_t pos = (int64_t)J.b.bcnt[blockIdx.x] + off + rank;
    uint16_t *out = (S.cur ? J.b.cells[0] : J.b.cells[1]) + pos * 8;
    unsigned long long id = J.b.hkey[J.b.slot[s]];
    const unsigned long long nb2 = (unsigned long long)S.nb_next;
    for (int k = 0; k < 8; k++) {
        if (k < S.d) {
            out[k] = (uint16_t)(id % nb2);
            id /= nb2;
        } else {
            out[k] = 0;
        }
    }
}

__global__ void k_av_finish(const AvJob *__restrict__ jobs) {
    AV_JOB;
    if (threadIdx.x != 0) return;
    AvDev &S = *J.b.st;
    if (!S.valid) return;
    S.cur ^= 1;
    S.nb = S.nb_next;
    S.n_cells = S.n_cells_next;
    S.ln_vol = log((double)S.n_cells) - S.d * log((double)S.nb);
}

int grid_for(int64_t n, int per_thread) {
    const int64_t g = (n + (int64_t)kAvThreads * per_thread - 1) / ((int64_t)kAvThreads * per_thread);
    return (int)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

template <class TO>
hipError_t av_update_t(const AvJob *d, int n_jobs, int64_t nmax, hipStream_t st) {
    constexpr int nbits = sizeof(TO) * 8;
    const unsigned nz = (unsigned)n_jobs;
    hipLaunchKernelGGL(k_av_begin, dim3(1, 1, nz), dim3(256), 0, st, d);
    hipLaunchKernelGGL(k_av_max<TO>, dim3(grid_for(nmax, 16), 1, nz), dim3(kAvThreads), 0, st, d);
    for (int shift = nbits - 8; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(k_av_hist<TO>, dim3(grid_for(nmax, 16), 1, nz), dim3(kAvThreads), 0, st, d, shift);
        hipLaunchKernelGGL(k_av_pick, dim3(1, 1, nz), dim3(256), 0, st, d, shift, nbits);
    }
    uint64_t used = 1024;
    while (used < (uint64_t)2 * (uint64_t)nmax) used <<= 1;
    hipLaunchKernelGGL(k_av_hclear, dim3(grid_for((int64_t)used, 4), 1, nz), dim3(kAvThreads), 0, st, d);
    hipLaunchKernelGGL(k_av_insert<TO>, dim3(grid_for(nmax, 4), 1, nz), dim3(kAvThreads), 0, st, d);
    const int nblk = (int)((nmax + kAvThreads - 1) / kAvThreads);
    hipLaunchKernelGGL(k_av_count, dim3(nblk, 1, nz), dim3(kAvThreads), 0, st, d);
    hipLaunchKernelGGL(k_av_scan, dim3(1, 1, nz), dim3(kScanThreads), 0, st, d);
    hipLaunchKernelGGL(k_av_compact, dim3(nblk, 1, nz), dim3(kAvThreads), 0, st, d);
    hipLaunchKernelGGL(k_av_finish, dim3(1, 1, nz), dim3(64), 0, st, d);
    return hipGetLastError();
}

int64_t max_n(const AvJob *h, int n_jobs) {
    int64_t m = 0;
    for (int k = 0; k < n_jobs; k++) m = h[k].n > m ? h[k].n : m;
    return m;
}

}  // namespace

hipError_t launch_av_reset(const AvBufs &b, int d, const int *dims, hipStream_t st) {
    int dd[7] = {-1, -1, -1, -1, -1, -1, -1};
    for (int k = 0; k < d && k < 7; k++) dd[k] = dims[k];
    hipLaunchKernelGGL(k_av_reset, dim3(1), dim3(64), 0, st, b, d, dd[0], dd[1], dd[2], dd[3], dd[4], dd[5], dd[6]);
    return hipGetLastError();
}

hipError_t launch_av_draw(int policy, const AvJob *d_jobs, const AvJob *h_jobs, int n_jobs, hipStream_t st) {
    const int64_t nmax = max_n(h_jobs, n_jobs);
    if (n_jobs <= 0 || nmax <= 0) return hipSuccess;
    const dim3 grid(grid_for(nmax, 4), 1, (unsigned)n_jobs);
    if (policy == kFP64)
        hipLaunchKernelGGL(k_av_draw<double>, grid, dim3(kAvThreads), 0, st, d_jobs);
    else
        hipLaunchKernelGGL(k_av_draw<float>, grid, dim3(kAvThreads), 0, st, d_jobs);
    return hipGetLastError();
}

hipError_t launch_av_update(int policy, const AvJob *d_jobs, const AvJob *h_jobs, int n_jobs, hipStream_t st) {
    const int64_t nmax = max_n(h_jobs, n_jobs);
    if (n_jobs <= 0 || nmax <= 0) return hipSuccess;
    if (policy == kFP32) return av_update_t<float>(d_jobs, n_jobs, nmax, st);
    return av_update_t<double>(d_jobs, n_jobs, nmax, st);
}

}  // namespace ile
