// Fair draws from weighted samples: the last step of an ILE run (extrinsic
// samples drawn fairly from the weighted Monte Carlo samples) and of the
// posterior construction.  k independent draws with replacement; index i has
// probability q_i / sum q with q_i = floor(exp(lw_i - max lw) 2^40) (0 for
// non-finite lw).  Integer masses give exact prefix sums, so every draw's
// index is independent of the order of accumulation:
//   1. max lw (order-preserving integer keys);
//   2. per-tile sums of q, an exclusive scan of the tile sums, and per-tile
//      inclusive prefix sums cum[i];
//   3. draw j: Philox counter (j lo, j hi, round, 16 * 5), r = w0 2^32 + w1,
//      target = floor(r * total / 2^64); the index is the first i with
//      cum[i] > target (binary search).  With total = 0 the index is -1.
#include "ile_internal.h"

namespace ile {

namespace {

constexpr int kFairThreads = 256;
constexpr int kFairPer = 16;                       // samples per thread of a tile
constexpr int kFairTile = kFairThreads * kFairPer;
constexpr uint32_t kFairAttempt = 5;

template <class TO>
__device__ __forceinline__ unsigned long long fmass(const TO *lw, int64_t i, int64_t n, double vmax) {
    if (i >= n) return 0ull;
    const TO v = lw[i];
    if (!isfinite(v)) return 0ull;
    return mass_fx((double)v, vmax);
}

// scratch: [0] max key, [1] total, [2 ..] per-tile sums / offsets
__global__ void k_fair_init(unsigned long long *scratch) {
    if (threadIdx.x == 0) {
        scratch[0] = 0;
        scratch[1] = 0;
    }
}

template <class TO>
__global__ void __launch_bounds__(kFairThreads) k_fair_max(const TO *__restrict__ lw, int64_t n,
                                                           unsigned long long *scratch) {
    unsigned long long km = 0;
    for (int64_t i = (int64_t)blockIdx.x * kFairThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kFairThreads) {
        const TO v = lw[i];
        if (isfinite(v)) {
            const unsigned long long k = ord_key(v);
            km = k > km ? k : km;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long k2 = __shfl_xor(km, o);
        km = k2 > km ? k2 : km;
    }
    if ((threadIdx.x & 63) == 0 && km) atomicMax(&scratch[0], km);
}

// Block-wide inclusive scan of one value per thread (LDS, Hillis-Steele).
__device__ __forceinline__ unsigned long long block_incl_scan(unsigned long long v, unsigned long long *sm) {
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < kFairThreads; o <<= 1) {
        const unsigned long long a = threadIdx.x >= (unsigned)o ? sm[threadIdx.x - o] : 0ull;
        __syncthreads();
        sm[threadIdx.x] += a;
        __syncthreads();
    }
    return sm[threadIdx.x];
}

template <class TO>
__global__ void __launch_bounds__(kFairThreads) k_fair_tiles(const TO *__restrict__ lw, int64_t n,
                                                             unsigned long long *scratch) {
    if (scratch[0] == 0) return;   // no finite sample
    constexpr int nbits = sizeof(TO) * 8;
    const double vmax = ord_value(scratch[0], nbits);
    const int64_t base = (int64_t)blockIdx.x * kFairTile + (int64_t)threadIdx.x * kFairPer;
    unsigned long long s = 0;
    for (int k = 0; k < kFairPer; k++) s += fmass(lw, base + k, n, vmax);
    __shared__ unsigned long long sm[kFairThreads];
    const unsigned long long tot = block_incl_scan(s, sm);
    if (threadIdx.x == kFairThreads - 1) scratch[2 + blockIdx.x] = tot;
}

// Exclusive scan of the tile sums in place; the total into scratch[1].
constexpr int kFairScanThreads = 1024;
__global__ void __launch_bounds__(kFairScanThreads) k_fair_scan(unsigned long long *scratch, int ntiles) {
    if (scratch[0] == 0) return;
    unsigned long long *ts = scratch + 2;
    __shared__ unsigned long long sm[kFairScanThreads];
    const int per = (ntiles + kFairScanThreads - 1) / kFairScanThreads;
    const int lo = threadIdx.x * per, hi = lo + per < ntiles ? lo + per : ntiles;
    unsigned long long loc = 0;
    for (int i = lo; i < hi; i++) loc += ts[i];
    sm[threadIdx.x] = loc;
    __syncthreads();
    for (int o = 1; o < kFairScanThreads; o <<= 1) {
        const unsigned long long a = threadIdx.x >= (unsigned)o ? sm[threadIdx.x - o] : 0ull;
        __syncthreads();
        sm[threadIdx.x] += a;
        __syncthreads();
    }
    unsigned long long run = sm[threadIdx.x] - loc;
    for (int i = lo; i < hi; i++) {
        const unsigned long long c = ts[i];
        ts[i] = run;
        run += c;
    }
    if (threadIdx.x == kFairScanThreads - 1) scratch[1] = sm[kFairScanThreads - 1];
}

template <class TO>
__global__ void __launch_bounds__(kFairThreads) k_fair_cum(const TO *__restrict__ lw, int64_t n,
                                                           const unsigned long long *scratch,
                                                           unsigned long long *__restrict__ cum) {
    if (scratch[0] == 0) return;
    constexpr int nbits = sizeof(TO) * 8;
    const double vmax = ord_value(scratch[0], nbits);
    const int64_t base = (int64_t)blockIdx.x * kFairTile + (int64_t)threadIdx.x * kFairPer;
    unsigned long long q[kFairPer], s = 0;
#pragma unroll
    for (int k = 0; k < kFairPer; k++) {
        q[k] = fmass(lw, base + k, n, vmax);
        s += q[k];
    }
    __shared__ unsigned long long sm[kFairThreads];
    unsigned long long run = block_incl_scan(s, sm) - s + scratch[2 + blockIdx.x];
#pragma unroll
    for (int k = 0; k < kFairPer; k++) {
        run += q[k];
        if (base + k < n) cum[base + k] = run;
    }
}

template <class TT>
__global__ void __launch_bounds__(kFairThreads)
    k_fair_pick(const unsigned long long *__restrict__ cum, int64_t n, const unsigned long long *scratch,
                uint64_t seed, uint32_t round, int64_t k, int64_t *__restrict__ idx, const TT *__restrict__ theta,
                int64_t ld, TT *__restrict__ theta_out, int64_t ld_out) {
    const unsigned long long total = scratch[0] ? scratch[1] : 0ull;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int64_t j = (int64_t)blockIdx.x * kFairThreads + threadIdx.x; j < k; j += (int64_t)gridDim.x * kFairThreads) {
        int64_t pick = -1;
        if (total > 0) {
            const U4 w = philox4x32_10(U4{(uint32_t)j, (uint32_t)((uint64_t)j >> 32), round, 16u * kFairAttempt}, k0,
                                       k1);
            const unsigned long long r = ((unsigned long long)w.x << 32) | w.y;
            const unsigned long long target = __umul64hi(r, total);
            int64_t lo = 0, hi = n - 1;   // first i with cum[i] > target (cum[n-1] = total > target)
            while (lo < hi) {
                const int64_t mid = lo + (hi - lo) / 2;
                if (cum[mid] > target)
                    hi = mid;
                else
                    lo = mid + 1;
            }
            pick = lo;
        }
        if (idx) idx[j] = pick;
        if (theta_out) {
#pragma unroll
            for (int c = 0; c < 7; c++) theta_out[c * ld_out + j] = pick >= 0 ? theta[c * ld + pick] : (TT)NAN;
        }
    }
}

template <class TO, class TT>
hipError_t fair_t(const TO *lw, int64_t n, uint64_t seed, uint32_t round, int64_t k, int64_t *idx, const TT *theta,
                  int64_t ld, TT *theta_out, int64_t ld_out, unsigned long long *cum, unsigned long long *scratch,
                  hipStream_t st) {
    const int ntiles = (int)((n + kFairTile - 1) / kFairTile);
    int gmax = (int)((n + kFairThreads * 16 - 1) / (kFairThreads * 16));
    gmax = gmax < 1 ? 1 : (gmax > 2048 ? 2048 : gmax);
    hipLaunchKernelGGL(k_fair_init, dim3(1), dim3(64), 0, st, scratch);
    hipLaunchKernelGGL(k_fair_max<TO>, dim3(gmax), dim3(kFairThreads), 0, st, lw, n, scratch);
    hipLaunchKernelGGL(k_fair_tiles<TO>, dim3(ntiles), dim3(kFairThreads), 0, st, lw, n, scratch);
    hipLaunchKernelGGL(k_fair_scan, dim3(1), dim3(kFairScanThreads), 0, st, scratch, ntiles);
    hipLaunchKernelGGL(k_fair_cum<TO>, dim3(ntiles), dim3(kFairThreads), 0, st, lw, n, scratch, cum);
    int gk = (int)((k + kFairThreads - 1) / kFairThreads);
    gk = gk < 1 ? 1 : (gk > 4096 ? 4096 : gk);
    hipLaunchKernelGGL(k_fair_pick<TT>, dim3(gk), dim3(kFairThreads), 0, st, cum, n, scratch, seed, round, k, idx,
                       theta, ld, theta_out, ld_out);
    return hipGetLastError();
}

}  // namespace

size_t fair_scratch_bytes(int64_t n) {
    const int64_t ntiles = (n + kFairTile - 1) / kFairTile;
    return (size_t)n * 8 + (size_t)(ntiles + 2) * 8 + 256;
}

hipError_t launch_fair_draw(int policy, const void *lw, int64_t n, uint64_t seed, uint32_t round, int64_t k,
                            int64_t *idx, const void *theta, int64_t ld, void *theta_out, int64_t ld_out,
                            void *scratch, hipStream_t st) {
    if (n <= 0 || k <= 0) return hipSuccess;
    unsigned long long *cum = (unsigned long long *)scratch;
    unsigned long long *sc = cum + n;
    if (policy == kFP32)
        return fair_t<float, float>((const float *)lw, n, seed, round, k, idx, (const float *)theta, ld,
                                    (float *)theta_out, ld_out, cum, sc, st);
    if (policy == kFP64)
        return fair_t<double, double>((const double *)lw, n, seed, round, k, idx, (const double *)theta, ld,
                                      (double *)theta_out, ld_out, cum, sc, st);
    return fair_t<double, float>((const double *)lw, n, seed, round, k, idx, (const float *)theta, ld,
                                 (float *)theta_out, ld_out, cum, sc, st);
}

}  // namespace ile
