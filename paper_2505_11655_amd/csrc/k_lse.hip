// Monte Carlo marginal of eq. (lnL:MonteCarlo) with eq. (neff), as a
// deterministic two-stage reduction in FP64 of the 4-tuple
//   (m = max lw, S1 = sum e^{lw-m}, S2 = sum e^{2(lw-m)}, argmax)
// plus the count of non-finite lw (zero weight).  Stage 1: one block per tile
// of consecutive samples; each lane reads 16-byte chunks (8 samples per lane
// per step, each wave-wide load one contiguous kilobyte), rescales its running
// (m, S1, S2) once per step to the step's maximum and then adds one
// exponential per sample; a fixed-shape tree in LDS combines the lanes.
// Stage 2: one block combines the tiles in index order and pools the result
// into the job's state.  The result depends only on n and the tile size,
// never on scheduling.
#include "ile_internal.h"

namespace ile {

namespace {

constexpr int kLseThreads = 256;

struct Acc {
    double m, s1, s2;
    int64_t bad, am;
};

// Terms with lw - m below -kSkip are under 2^-54 of the largest term and do
// not change an FP64 sum that holds it; their exponential is not evaluated.
constexpr double kSkip = 37.5;

// Push B samples x[0..B) with indices idx[k] (increasing): one rescale to the
// batch maximum, then one exponential per sample.
template <int B>
__device__ __forceinline__ void acc_batch(Acc &a, const double *x, const int64_t *idx) {
    double bm = -INFINITY;
    int64_t bi = INT64_MAX;
#pragma unroll
    for (int k = 0; k < B; k++) {
        if (!(x[k] > -INFINITY && x[k] < INFINITY)) {
            a.bad++;
        } else if (x[k] > bm) {
            bm = x[k];
            bi = idx[k];
        }
    }
    if (bm > a.m) {
        const double r = exp(a.m - bm);   // 0 when a.m = -inf
        a.s1 *= r;
        a.s2 *= r * r;
        a.m = bm;
        a.am = bi;
    } else if (bm == a.m && bi < a.am) {
        a.am = bi;
    }
#pragma unroll
    for (int k = 0; k < B; k++) {
        const double d = x[k] - a.m;
        if (d > -kSkip && x[k] < INFINITY) {
            const double e = exp(d);
            a.s1 += e;
            a.s2 += e * e;
        }
    }
}

// Stage-1 reduction of lw[begin, end) for the calling thread.
template <class TL>
__device__ __forceinline__ Acc tile_scan(const TL *lw, int64_t begin, int64_t end) {
    typedef __attribute__((address_space(1))) const TL gTL;
    constexpr int kEpc = 16 / (int)sizeof(TL);   // elements per 16-byte chunk
    constexpr int kNch = 8 / kEpc;               // chunks per lane per step (8 samples)
    constexpr int64_t kStep = (int64_t)kLseThreads * kNch * kEpc;
    Acc a{-INFINITY, 0.0, 0.0, 0, INT64_MAX};
    const int t = threadIdx.x;
    int64_t i = begin;
    if ((((uintptr_t)(lw + begin)) & 15) == 0) {
        gTL *g = (gTL *)lw;
        for (; i + kStep <= end; i += kStep) {
            double x[8];
            int64_t ix[8];
#pragma unroll
            for (int c = 0; c < kNch; c++) {
                const int64_t e0 = i + ((int64_t)c * kLseThreads + t) * kEpc;
                typedef TL vec_t __attribute__((ext_vector_type(kEpc)));
                typedef __attribute__((address_space(1))) const vec_t gvec_t;
                const vec_t v = *(gvec_t *)(g + e0);
#pragma unroll
                for (int e = 0; e < kEpc; e++) x[kEpc * c + e] = (double)v[e];
#pragma unroll
                for (int e = 0; e < kEpc; e++) ix[kEpc * c + e] = e0 + e;
            }
            acc_batch<8>(a, x, ix);
        }
    }
    for (int64_t j = i + t; j < end; j += kLseThreads) {
        const double x = (double)lw[j];
        acc_batch<1>(a, &x, &j);
    }
    return a;
}

// Combine b into a (a holds the lower sample indices on ties).
__device__ __forceinline__ void acc_merge(Acc &a, const Acc &b) {
    a.bad += b.bad;
    if (b.m == -INFINITY) return;
    if (a.m == -INFINITY) {
        a.m = b.m; a.s1 = b.s1; a.s2 = b.s2; a.am = b.am;
        return;
    }
    if (b.m > a.m) {
        const double r = exp(a.m - b.m);
        a.s1 = a.s1 * r + b.s1;
        a.s2 = a.s2 * r * r + b.s2;
        a.m = b.m;
        a.am = b.am;
    } else {
        const double r = exp(b.m - a.m);
        a.s1 += b.s1 * r;
        a.s2 += b.s2 * r * r;
        if (b.m == a.m && b.am < a.am) a.am = b.am;
    }
}

__device__ void block_reduce(Acc &a) {
    __shared__ double sm[kLseThreads], s1[kLseThreads], s2[kLseThreads];
    __shared__ int64_t sb[kLseThreads], sa[kLseThreads];
    const int t = threadIdx.x;
    sm[t] = a.m; s1[t] = a.s1; s2[t] = a.s2; sb[t] = a.bad; sa[t] = a.am;
    __syncthreads();
    for (int w = kLseThreads / 2; w > 0; w >>= 1) {
        if (t < w) {
            Acc x{sm[t], s1[t], s2[t], sb[t], sa[t]};
            Acc y{sm[t + w], s1[t + w], s2[t + w], sb[t + w], sa[t + w]};
            acc_merge(x, y);
            sm[t] = x.m; s1[t] = x.s1; s2[t] = x.s2; sb[t] = x.bad; sa[t] = x.am;
        }
        __syncthreads();
    }
    a = Acc{sm[0], s1[0], s2[0], sb[0], sa[0]};
}

template <class TL>
__global__ void __launch_bounds__(kLseThreads)
    k_marg_partials(const TL *__restrict__ lw, int64_t n, int64_t tile, MargPartial *__restrict__ part) {
    const int64_t b0 = (int64_t)blockIdx.x * tile;
    const int64_t b1 = min(b0 + tile, n);
    Acc a = tile_scan<TL>(lw, b0, b1);
    block_reduce(a);
    if (threadIdx.x == 0) part[blockIdx.x] = MargPartial{a.m, a.s1, a.s2, a.bad, a.am};
}

__global__ void __launch_bounds__(kLseThreads)
    k_marg_combine(const MargPartial *__restrict__ part, int n_part, int64_t n, MargState *st, int reset) {
    // each thread folds a contiguous run of tiles, then the fixed tree
    Acc a{-INFINITY, 0.0, 0.0, 0, INT64_MAX};
    const int per = (n_part + kLseThreads - 1) / kLseThreads;
    const int p0 = threadIdx.x * per, p1 = min(p0 + per, n_part);
    for (int p = p0; p < p1; p++) {
        const MargPartial q = part[p];
        acc_merge(a, Acc{q.m, q.s1, q.s2, q.n_bad, q.argmax});
    }
    block_reduce(a);
    if (threadIdx.x == 0) {
        if (reset) {
            st->m = -INFINITY; st->s1 = 0.0; st->s2 = 0.0; st->n = 0; st->n_bad = 0; st->argmax = -1;
        }
        // pool: argmax indices of a new batch are offset by the samples already pooled
        Acc old{st->m, st->s1, st->s2, st->n_bad, st->argmax};
        Acc nw = a;
        if (nw.m != -INFINITY) nw.am += st->n;
        acc_merge(old, nw);
        st->m = old.m; st->s1 = old.s1; st->s2 = old.s2; st->n_bad = old.bad;
        st->argmax = (old.m == -INFINITY) ? -1 : old.am;
        st->n += n;
    }
}

}  // namespace

hipError_t launch_marg_partials(int policy, const void *lw, int64_t n, int64_t tile, MargPartial *d_part,
                                hipStream_t st) {
    const int64_t nb = (n + tile - 1) / tile;
    if (nb <= 0) return hipSuccess;
    if (policy == kFP32)
        hipLaunchKernelGGL(k_marg_partials<float>, dim3(nb), dim3(kLseThreads), 0, st, (const float *)lw, n,
                           tile, d_part);
    else
        hipLaunchKernelGGL(k_marg_partials<double>, dim3(nb), dim3(kLseThreads), 0, st, (const double *)lw,
                           n, tile, d_part);
    return hipGetLastError();
}

hipError_t launch_marg_combine(const MargPartial *d_part, int n_part, int64_t n, MargState *d_state, int reset,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_marg_combine, dim3(1), dim3(kLseThreads), 0, st, d_part, n_part, n, d_state, reset);
    return hipGetLastError();
}

}  // namespace ile

// ------------------------------------------------------------- many jobs
// Stage 1 over a tile list spanning several jobs (each tile inside one job);
// stage 2 with one block per job combining that job's tiles in order.  A job's
// result depends only on its own samples and the fixed tile size.
namespace ile {

namespace {

template <class TL>
__global__ void __launch_bounds__(kLseThreads)
    k_marg_partials_batch(const MargJob *__restrict__ jobs, const Tile *__restrict__ tiles,
                          MargPartial *__restrict__ part) {
    const Tile tl = tiles[blockIdx.x];
    const TL *__restrict__ lw = (const TL *)jobs[tl.job].lw;
    Acc a = tile_scan<TL>(lw, tl.begin, tl.end);
    block_reduce(a);
    if (threadIdx.x == 0) part[blockIdx.x] = MargPartial{a.m, a.s1, a.s2, a.bad, a.am};
}

__global__ void __launch_bounds__(kLseThreads) k_marg_combine_batch(const MargJob *__restrict__ jobs,
                                                                    const MargPartial *__restrict__ part,
                                                                    MargState *__restrict__ out) {
    const MargJob &J = jobs[blockIdx.x];
    Acc a{-INFINITY, 0.0, 0.0, 0, INT64_MAX};
    const int np = J.tile_end - J.tile_begin;
    const int per = (np + kLseThreads - 1) / kLseThreads;
    const int p0 = J.tile_begin + threadIdx.x * per, p1 = min(p0 + per, J.tile_end);
    for (int p = p0; p < p1; p++) {
        const MargPartial q = part[p];
        acc_merge(a, Acc{q.m, q.s1, q.s2, q.n_bad, q.argmax});
    }
    block_reduce(a);
    if (threadIdx.x == 0) {
        MargState *st = J.state;
        if (J.reset) {
            st->m = -INFINITY; st->s1 = 0.0; st->s2 = 0.0; st->n = 0; st->n_bad = 0; st->argmax = -1;
        }
        Acc old{st->m, st->s1, st->s2, st->n_bad, st->argmax};
        Acc nw = a;
        if (nw.m != -INFINITY) nw.am += st->n;
        acc_merge(old, nw);
        st->m = old.m; st->s1 = old.s1; st->s2 = old.s2; st->n_bad = old.bad;
        st->argmax = (old.m == -INFINITY) ? -1 : old.am;
        st->n += J.n;
        if (out && J.out_idx >= 0) out[J.out_idx] = *st;
    }
}

}  // namespace

hipError_t launch_marg_batch(int policy, const MargJob *d_jobs, int n_jobs, const Tile *d_tiles, int n_tiles,
                             MargPartial *d_part, MargState *d_out, hipStream_t st) {
    if (n_tiles > 0) {
        if (policy == kFP32)
            hipLaunchKernelGGL(k_marg_partials_batch<float>, dim3(n_tiles), dim3(kLseThreads), 0, st, d_jobs,
                               d_tiles, d_part);
        else
            hipLaunchKernelGGL(k_marg_partials_batch<double>, dim3(n_tiles), dim3(kLseThreads), 0, st, d_jobs,
                               d_tiles, d_part);
    }
    if (n_jobs > 0)
        hipLaunchKernelGGL(k_marg_combine_batch, dim3(n_jobs), dim3(kLseThreads), 0, st, d_jobs, d_part, d_out);
    return hipGetLastError();
}

}  // namespace ile
