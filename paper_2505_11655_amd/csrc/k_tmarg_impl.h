// Time-marginalised likelihood per extrinsic sample: the (time) x (extrinsic)
// array of eq. (lnL:MatrixForm) integrated over the geocentric time prior,
//   ln L_t = ln sum_j (dt / (R 2 t_w)) exp( s T1(t_j) - s^2 T2 / 4 ),
// on the nodes t_j = j dt / R, |j| <= tm_half (dt: the window's sample step).
// T2 does not depend on t.  With tau_k(t) = t - x_k.n/c, the window position
// of node j = R q + r in detector k is u0_k + q + r/R, so the integer part is
// i0_k + q + c_kr (c_kr in {0, 1}) and the four Lagrange weights depend only
// on (k, r): they are computed once per sample as five-tap weights over the
// samples i0_k + q - 1 .. i0_k + q + 3.  Per lattice step q each detector
// needs one new
//   G_k(i) = sum_a Re[ conj(F_k) y_a e^{i m_a phi} Q_k,a(i) ],
// and each node costs five FMAs per detector plus one exponential; the sum
// over nodes is a chunked log-sum-exp (one rescale per lattice step at most)
// accumulated in FP64.  A node whose stencil leaves the window contributes
// nothing (its pointwise lnL is -inf).
// With the distance integrated (DM) every node's value is the table's
// ln L_D(T1(t_j), T2) instead of s T1(t_j) - s^2 T2 / 4 (T1, T2 at s = 1):
//   ln L_{t,D} = ln sum_j (dt / (R 2 t_w)) L_D(T1(t_j), T2),
// the time and distance integrals taken together; the table row of T2 is
// set up once per sample and each node interpolates along a only (FP64).
#pragma once

#include "k_lnl_impl.h"

namespace ile {

template <int S, int K, int POL, bool LDS, int R, bool DM>
struct TmargKernel {
    using LK = LnlKernel<S, K, POL, LDS, false>;
    using Tp = PolTypes<POL>;
    using TT = typename Tp::TT;
    using TS = typename Tp::TS;
    using TG = typename Tp::TG;
    using TE = typename Tp::TE;
    using TA = typename Tp::TA;
    using TO = typename Tp::TO;
    using ccpx = typename LK::ccpx;
    static constexpr int NM = LK::NM;
    static constexpr int NE = LK::NE;
    static constexpr bool kT2First = sizeof(TA) == 8 || DM;   // DM: the table row needs T2 first
    using TV = std::conditional_t<DM, double, TA>;             // node values
    // With the window in LDS the G rows (a different row per lane) load the
    // LDS beyond its bandwidth; reading the first detector through L1/L2
    // instead balances the two paths (measured, 256 x 2^16 samples: HLV 9
    // modes 33.8 -> 25.5 ms, two of three detectors through L1/L2 39.5 ms;
    // HL 5 modes 16.0 -> 14.5 ms).  Only the other detectors are staged.
    static constexpr int kGlobalDets = LDS ? tmarg_global_dets(S, K, POL) : K;

    __device__ __forceinline__ static TA expT(TA x) {
        if constexpr (sizeof(TA) == 4)
            return __expf(x);
        else
            return exp(x);
    }

    __device__ __forceinline__ static void run(const EvalJob &J, const int64_t begin, const int64_t end,
                                               cpx<TA> *smem) {
        const int T = J.n_time;
        const cpx<TA> *__restrict__ Qg = (const cpx<TA> *)J.Q;
        if constexpr (LDS) {
            const size_t nwords = (size_t)(K - kGlobalDets) * T * NM * sizeof(cpx<TA>) / 8;
            const uint2 *src = (const uint2 *)(Qg + (size_t)kGlobalDets * T * NM);
            uint2 *dst = (uint2 *)smem;
            for (size_t w = threadIdx.x; w < nwords; w += blockDim.x) dst[w] = src[w];
            __syncthreads();
        }
        ccpx *Ut = (ccpx *)J.Ut;
        ccpx *Vt = (ccpx *)J.Vt;
        const TT *__restrict__ th = (const TT *)J.theta;
        const TT *__restrict__ lr = (const TT *)J.lnpmps;
        TO *__restrict__ outL = (TO *)J.lnL;
        TO *__restrict__ outW = (TO *)J.lw;
        const int64_t ld = J.ld;
        const int jh = J.tm_half;
        // lattice steps covering nodes -jh..jh (floor division)
        const int q_lo = (-jh >= 0) ? (-jh) / R : -((jh + R - 1) / R);
        const int q_hi = jh / R;

        for (int64_t i = begin + threadIdx.x; i < end; i += blockDim.x) {
            asm volatile("" : "+s"(Ut), "+s"(Vt));
            const TT al = th[i], de = th[ld + i], DD = th[3 * ld + i];
            const TT ci = th[4 * ld + i], ph = th[5 * ld + i], ps = th[6 * ld + i];
            const bool ok = DD > (TT)0 && ci >= (TT)-1 && ci <= (TT)1;

            TG Fr[K], Fi[K];
            TS uu[K];
            TG y[NM];
            TE Er[NE], Ei[NE];
            LK::geometry(J, al, de, (TT)0, ci, ph, ps, Fr, Fi, uu, y, Er, Ei);
            const TA s = pick<TA>(J.d_ref, J.d_reff) / (TA)DD;
            // T2 does not depend on t.  FP32: formed after the time loop, so its
            // temporaries never coexist with the loop state; FP64 (one wave per
            // SIMD, registers to spare): before it, like the pointwise kernel.
            TA T2 = (TA)0;
            if constexpr (kT2First) T2 = LK::template quad_T2<false>(Fr, Fi, y, Er, Ei, Ut, Vt);
            DistRow drow{};
            if constexpr (DM) drow = dist_row(J.dt, (double)T2);

            // c_k,a = conj(F_k) y_a e^{i m_a phi}: Re(c Q) = cr Q.re - cm Q.im
            TA cr[K][NM], cm[K][NM];
#pragma unroll
            for (int k = 0; k < K; k++) {
                static_for<0, NM>([&](auto A_) {
                    constexpr int a = decltype(A_)::value;
                    constexpr int m = kSets[S].m[a];
                    const TA er = (TA)Er[m < 0 ? -m : m];
                    const TA ei = (m < 0) ? -(TA)Ei[-m] : (TA)Ei[m];
                    const TA zr = (TA)y[a] * er, zi = (TA)y[a] * ei;
                    cr[k][a] = (TA)Fr[k] * zr + (TA)Fi[k] * zi;
                    cm[k][a] = (TA)Fr[k] * zi - (TA)Fi[k] * zr;
                });
            }
            // per detector: base index, five-tap weights per sub-step r, and
            // the lattice steps q for which every detector's stencil is inside
            int i0[K];
            TA w5[K][R][5];
            int qmin[R], qmax[R];
#pragma unroll
            for (int r = 0; r < R; r++) {
                qmin[r] = INT32_MIN / 2;
                qmax[r] = INT32_MAX / 2;
            }
#pragma unroll
            for (int k = 0; k < K; k++) {
                const TS fl = dfloor(uu[k]);
                // keep the base index representable; a sample this far out has no valid node
                const TS flc = fmin(fmax(fl, (TS)(-4 * T)), (TS)(4 * T));
                i0[k] = (int)flc;
                const TA f0 = (TA)(uu[k] - fl);
#pragma unroll
                for (int r = 0; r < R; r++) {
                    TA f = f0 + (TA)r / (TA)R;
                    const int c = f >= (TA)1 ? 1 : 0;
                    f -= (TA)c;
                    const TA fm1 = f - (TA)1, fm2 = f - (TA)2, fp1 = f + (TA)1;
                    const TA w0 = -f * fm1 * fm2 * (TA)(1.0 / 6.0);
                    const TA w1 = fp1 * fm1 * fm2 * (TA)0.5;
                    const TA w2 = -fp1 * f * fm2 * (TA)0.5;
                    const TA w3 = fp1 * f * fm1 * (TA)(1.0 / 6.0);
                    w5[k][r][0] = c ? (TA)0 : w0;
                    w5[k][r][1] = c ? w0 : w1;
                    w5[k][r][2] = c ? w1 : w2;
                    w5[k][r][3] = c ? w2 : w3;
                    w5[k][r][4] = c ? w3 : (TA)0;
                    // node (q, r) of detector k uses samples i0 + q + c - 1 .. i0 + q + c + 2
                    const int lo = 1 - i0[k] - c, hi = T - 3 - i0[k] - c;
                    qmin[r] = max(qmin[r], lo);
                    qmax[r] = min(qmax[r], hi);
                }
            }
            // window G_k(i0 + q - 1 + t), t = 0..4: each step appends the
            // newest sample; the four steps before q_lo only fill the window
            // (their nodes lie below -tm_half and are masked)
            TA G[K][5];
#pragma unroll
            for (int k = 0; k < K; k++)
#pragma unroll
                for (int t = 0; t < 5; t++) G[k][t] = (TA)0;
            TV mx = (TV)-INFINITY;
            double sum = 0.0;
#pragma unroll 1
            for (int q = q_lo - 4; q <= q_hi; q++) {
                // The newest window row of the detectors.  In FP32, up to 27
                // complex values (3 detectors x 9 modes), every detector's row
                // is loaded before any is used: left to itself the allocator
                // recycled one destination register and waited for every
                // load in turn (37 against 24 ms, 256 x 2^16 samples, HLV 9
                // modes).  Larger sets, and FP64, go one detector at a time:
                // holding all their rows costs more registers than it saves.
                constexpr int kGroup = (sizeof(TA) == 4 && K * NM <= 27) ? K : 1;
#pragma unroll
                for (int k0 = 0; k0 < K; k0 += kGroup) {
                    if constexpr (kGroup == 1) fence();
                    cpx<TA> qv[kGroup][NM];
#pragma unroll
                    for (int kk = 0; kk < kGroup; kk++) {
                        const int k = k0 + kk;
                        const int ic = min(max(i0[k] + q + 3, 0), T - 1);
                        const cpx<TA> *qr = (k < kGlobalDets ? Qg + (size_t)k * T * NM
                                                             : smem + (size_t)(k - kGlobalDets) * T * NM) +
                                            (size_t)ic * NM;
                        static_for<0, NM>([&](auto A_) {
                            constexpr int a = decltype(A_)::value;
                            qv[kk][a] = qr[a];
                        });
                    }
#pragma unroll
                    for (int kk = 0; kk < kGroup; kk++) {
                        const int k = k0 + kk;
#pragma unroll
                        for (int t = 0; t < 4; t++) G[k][t] = G[k][t + 1];
                        TA g = (TA)0;
                        static_for<0, NM>([&](auto A_) {
                            constexpr int a = decltype(A_)::value;
                            g = fma(cr[k][a], qv[kk][a].re, g);
                            g = fma(-cm[k][a], qv[kk][a].im, g);
                        });
                        G[k][4] = g;
                    }
                }
                TV x[R];
                TV cmax = (TV)-INFINITY;
#pragma unroll
                for (int r = 0; r < R; r++) {
                    const int j = R * q + r;
                    const bool valid = j >= -jh && j <= jh && q >= qmin[r] && q <= qmax[r];
                    TA t1 = (TA)0;
#pragma unroll
                    for (int k = 0; k < K; k++)
#pragma unroll
                        for (int t = 0; t < 5; t++) t1 = fma(w5[k][r][t], G[k][t], t1);
                    if constexpr (DM)
                        x[r] = valid ? dist_at(J.dt, drow, (double)t1) : -INFINITY;
                    else
                        x[r] = valid ? s * t1 : (TA)-INFINITY;
                    cmax = fmax(cmax, x[r]);
                }
                if (cmax > mx) {
                    if constexpr (DM)
                        sum = (mx > -INFINITY) ? sum * exp(mx - cmax) : 0.0;
                    else
                        sum = (mx > (TA)-INFINITY) ? sum * (double)expT(mx - cmax) : 0.0;
                    mx = cmax;
                }
                TV part = (TV)0;
#pragma unroll
                for (int r = 0; r < R; r++) {
                    if constexpr (DM)
                        part += (x[r] > -INFINITY) ? exp(x[r] - mx) : 0.0;
                    else
                        part += (x[r] > (TA)-INFINITY) ? expT(x[r] - mx) : (TA)0;
                }
                sum += (double)part;
            }
            if constexpr (!kT2First) {
                // the table pointers look redefined here, so the scalar loads
                // of the pair tables are not hoisted over the time loop
                fence();
                asm volatile("" : "+s"(Ut), "+s"(Vt));
                T2 = LK::template quad_T2<false>(Fr, Fi, y, Er, Ei, Ut, Vt);
            }
            double lnLt = -INFINITY;
            if constexpr (DM) {
                if (ok && mx > -INFINITY) lnLt = (double)mx + log(sum) + J.tm_lnw;
            } else {
                if (ok && mx > (TA)-INFINITY)
                    lnLt = (double)mx + log(sum) - (double)(s * s * T2 * (TA)0.25) + J.tm_lnw;
            }
            const TO outv = (TO)lnLt;
            if (outL) outL[i] = outv;
            if (outW) outW[i] = outv + (lr ? (TO)lr[i] : (TO)0);
        }
    }
};

template <int S, int K, int POL, bool LDS, int R, bool DM>
__global__ void __launch_bounds__(tmarg_block_threads(POL), 1)
    k_lnl_tmarg(const EvalJob *__restrict__ jobs, const Tile *__restrict__ tiles) {
    extern __shared__ __align__(16) char ile_smem[];
    using TA = typename PolTypes<POL>::TA;
    const Tile tl = tiles[blockIdx.x];
    TmargKernel<S, K, POL, LDS, R, DM>::run(jobs[tl.job], tl.begin, tl.end, (cpx<TA> *)ile_smem);
}

// Launch the time-marginalised kernel of mode set S and policy POL (FP32 or
// FP64) for oversampling R in {1, 4}, with the distance integrated (dm) or not.
template <int S, int POL>
hipError_t launch_tmarg_sp(int kdet, int R, bool dm, size_t lds_bytes, const EvalJob *jobs, const Tile *tiles,
                           int n_tiles, int nthreads, hipStream_t st) {
    if (n_tiles <= 0) return hipSuccess;
    const bool lds = lds_bytes > 0;
    if (nthreads <= 0 || nthreads > tmarg_block_threads(POL) || nthreads % 64) return hipErrorInvalidValue;
    dim3 grid(n_tiles), block(nthreads);
    auto go2 = [&](auto KK, auto LL, auto RR, auto DD) -> hipError_t {
        constexpr int K = decltype(KK)::value;
        constexpr bool L = decltype(LL)::value;
        constexpr int RV = decltype(RR)::value;
        constexpr bool DMV = decltype(DD)::value;
        if constexpr (L && !tmarg_lds_compiled(S, K, POL)) {
            return hipErrorInvalidValue;
        } else {
            auto fn = k_lnl_tmarg<S, K, POL, L, RV, DMV>;
            if (L) {
                hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                   (int)lds_bytes);
                if (e != hipSuccess) return e;
            }
            hipLaunchKernelGGL(fn, grid, block, L ? lds_bytes : 0, st, jobs, tiles);
            return hipGetLastError();
        }
    };
    auto go = [&](auto KK, auto LL, auto RR) -> hipError_t {
        return dm ? go2(KK, LL, RR, std::true_type{}) : go2(KK, LL, RR, std::false_type{});
    };
    using T2 = std::integral_constant<int, 2>;
    using T3 = std::integral_constant<int, 3>;
    using BT = std::true_type;
    using BF = std::false_type;
    using R1 = std::integral_constant<int, 1>;
    using R4 = std::integral_constant<int, 4>;
    if (R != 1 && R != 4) return hipErrorInvalidValue;
    if (kdet == 2) {
        if (lds) return R == 1 ? go(T2{}, BT{}, R1{}) : go(T2{}, BT{}, R4{});
        return R == 1 ? go(T2{}, BF{}, R1{}) : go(T2{}, BF{}, R4{});
    }
    if (kdet == 3) {
        if (lds) return R == 1 ? go(T3{}, BT{}, R1{}) : go(T3{}, BT{}, R4{});
        return R == 1 ? go(T3{}, BF{}, R1{}) : go(T3{}, BF{}, R4{});
    }
    return hipErrorInvalidValue;
}

}  // namespace ile
