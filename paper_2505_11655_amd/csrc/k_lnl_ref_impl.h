// Likelihood of the FP32 + FP64-cancellation policy, eq. (def:lnL:Decomposed)
// written about a reference point.
//
// Per detector the likelihood is a real quadratic function of the complex
// mode amplitudes c_k,a = s F_k Y_a (s = D_ref/D):
//     lnL = sum_k [ Re(c_k^+ Qhat_k) - 1/4 c_k^+ U_k c_k - 1/4 Re(c_k^T V_k c_k) ].
// With a reference r_k (the amplitudes of a reference point theta_ref,
// rounded to FP32 so that they are exact in both precisions) and
// delta_k = c_k - r_k this is exactly
//     lnL = [ sum_k Re(r_k^+ Qhat_k) - C0 ]                          (FP64)
//         + sum_k Re(delta_k^+ (Qhat_k - G_k))                        (FP32)
//         - 1/4 sum_k [ delta_k^+ U_k delta_k + Re(delta_k^T V_k delta_k) ]   (FP32)
// with G_k = (U_k r_k + conj(V_k r_k)) / 2 and C0 = 1/2 sum_k Re(r_k^+ G_k).
// The two terms of size rho^2 that cancel in lnL are in the first bracket:
// its Q part is Re(r_k^+ Qhat_k) = sum_j w_j R_k[i+j], the interpolant of the
// real series R_k[i] = Re(r_k^+ Q_k[i]) formed once per reference in FP64,
// evaluated here with FP64 weights; C0 is an FP64 constant.  Everything that
// remains scales with |delta|: the rounding of Q, U, V, G and of the sums to
// FP32 then costs eps |delta| rho^2 instead of eps rho^2.  Any reference
// gives the same lnL up to rounding (no reference: r = 0, plain FP32
// arithmetic); a reference near the samples gives the accuracy.
//
// The quadratic form over delta is, per detector, a real quadratic form in
// the 2n components v = (dr_0, di_0, dr_1, ...): with M the upper triangle of
// its matrix (off-diagonal entries doubled) it is sum_i v_i sum_{j>=i} M_ij v_j,
// one fused multiply-add per entry plus one per row: (2n)(2n+1)/2 + 2n
// instructions per detector (189 for 9 modes, against 8 per mode pair, 360,
// when every product of a pair is formed on its own).
#pragma once

#include "k_lnl_impl.h"

namespace ile {

template <int S, int K, bool LDS>
struct RefKernel {
    using LKG = LnlKernel<S, K, kFP64, false, false>;   // FP64 geometry
    using MS = MSet<S>;
    static constexpr int NM = MS::n;
    static constexpr int NE = LKG::NE;
    static constexpr int kG = LDS ? lds_global_dets(S, K, kMixed) : 0;
    static constexpr int NV = 2 * NM, NT = NV * (NV + 1) / 2;
    typedef __attribute__((address_space(4))) const EvalJob cjob;
    typedef __attribute__((address_space(4))) const float cf1;
    typedef __attribute__((address_space(4))) const cpx<float> ccf;

    __device__ __forceinline__ static void run(const EvalJob *Jp, const int64_t begin, const int64_t end,
                                               char *smem) {
        const EvalJob &J = *Jp;
        const int T = J.n_time;
        const cpx<float> *__restrict__ Qg = (const cpx<float> *)J.Q;
        const double *__restrict__ Rg = J.ref_R;
        cpx<float> *sQ = (cpx<float> *)smem;
        double *sR = (double *)(smem + (size_t)(K - kG) * T * NM * sizeof(cpx<float>));
        if constexpr (LDS) {
            // stage the windows of detectors kG..K-1 and every detector's
            // reference series (offsets in 8-byte words)
            const size_t nq = (size_t)(K - kG) * T * NM;
            const uint2 *src = (const uint2 *)(Qg + (size_t)kG * T * NM);
            uint2 *dst = (uint2 *)sQ;
            for (size_t w = threadIdx.x; w < nq; w += blockDim.x) dst[w] = src[w];
            const size_t nr = (size_t)K * T;
            for (size_t w = threadIdx.x; w < nr; w += blockDim.x) sR[w] = Rg[w];
            __syncthreads();
        }
        const float *__restrict__ th = (const float *)J.theta;
        const float *__restrict__ lr = (const float *)J.lnpmps;
        double *__restrict__ outL = (double *)J.lnL;
        double *__restrict__ outW = (double *)J.lw;
        const int64_t ld = J.ld;
        cf1 *Wt = (cf1 *)J.Ut;                       // [K][NT] quadratic-form rows
        ccf *rg = (ccf *)J.ref_rg;                   // r [K][NM], then G [K][NM]
        const double *C0p = J.ref_C0;

        for (int64_t i = begin + threadIdx.x; i < end; i += blockDim.x) {
            // table and descriptor pointers look loop-variant: their scalar
            // loads stream per sample instead of holding registers throughout
            asm volatile("" : "+s"(Wt), "+s"(rg));
            cjob *Jc = (cjob *)Jp;
            asm volatile("" : "+s"(Jc));
            const float al = th[i], de = th[ld + i], tt = th[2 * ld + i], DD = th[3 * ld + i];
            const float ci = th[4 * ld + i], ph = th[5 * ld + i], ps = th[6 * ld + i];
            bool ok = DD > 0.0f && ci >= -1.0f && ci <= 1.0f;

            // The amplitudes c = s F_k Y_a are formed in FP64 and only their
            // offsets from the reference are rounded to FP32: FP32 rounding of
            // c itself would move lnL at first order in its gradient,
            // ~eps rho sqrt(2 dlnL) per mode, which reaches 1e-3 fifty units
            // below the peak at SNR 400.
            double Fr[K], Fi[K];
            double uu[K];
            double y[NM];
            double Er[NE], Ei[NE];
            LKG::geometry(*Jc, (double)al, (double)de, (double)tt, (double)ci, (double)ph, (double)ps, Fr, Fi, uu, y,
                          Er, Ei);
            const double s = Jc->d_ref / (double)DD;
            // Y_a = y_a e^{-i m_a phi}
            double Yr[NM], Yi[NM];
            static_for<0, NM>([&](auto A_) {
                constexpr int a = decltype(A_)::value;
                constexpr int m = kSets[S].m[a];
                constexpr int am = m < 0 ? -m : m;
                Yr[a] = y[a] * Er[am];
                Yi[a] = (m > 0) ? -y[a] * Ei[am] : y[a] * Ei[am];   // Ei[0] = 0
            });

            double A = 0.0;   // sum_k Re(r_k^+ Qhat_k), FP64
            float B = 0.0f;   // linear term in delta
            float Cq = 0.0f;  // quadratic term in delta
#pragma unroll
            for (int k = 0; k < K; k++) {
                fence();
                const double fl = floor(uu[k]);
                ok = ok && (fl >= 1.0) && (fl <= (double)(T - 3));
                const double flc = fmin(fmax(fl, 1.0), (double)(T - 3));
                const int i0 = (int)flc;
                const double fd = uu[k] - fl;
                // reference part: FP64 Lagrange weights on the FP64 series
                {
                    const double fm1 = fd - 1.0, fm2 = fd - 2.0, fp1 = fd + 1.0;
                    const double w0 = -fd * fm1 * fm2 * (1.0 / 6.0);
                    const double w1 = fp1 * fm1 * fm2 * 0.5;
                    const double w2 = -fp1 * fd * fm2 * 0.5;
                    const double w3 = fp1 * fd * fm1 * (1.0 / 6.0);
                    const double *R = (LDS ? sR : Rg) + (size_t)k * T + (i0 - 1);
                    A = fma(w0, R[0], A);
                    A = fma(w1, R[1], A);
                    A = fma(w2, R[2], A);
                    A = fma(w3, R[3], A);
                }
                // amplitude offsets delta_k,a = s F_k Y_a - r_k,a and the linear term
                const float f = (float)fd;
                const float fm1 = f - 1.0f, fm2 = f - 2.0f, fp1 = f + 1.0f;
                const float w0 = -f * fm1 * fm2 * (1.0f / 6.0f);
                const float w1 = fp1 * fm1 * fm2 * 0.5f;
                const float w2 = -fp1 * f * fm2 * 0.5f;
                const float w3 = fp1 * f * fm1 * (1.0f / 6.0f);
                const cpx<float> *q = (LDS && k >= kG) ? sQ + ((size_t)(k - kG) * T + (i0 - 1)) * NM
                                                       : Qg + ((size_t)k * T + (i0 - 1)) * NM;
                const double sFr = s * Fr[k], sFi = s * Fi[k];
                float dr[NM], di[NM];
                static_for<0, NM>([&](auto A_) {
                    constexpr int a = decltype(A_)::value;
                    // (fields read one by one: an aggregate does not copy out
                    // of the constant address space)
                    const float rre = rg[k * NM + a].re, rim = rg[k * NM + a].im;
                    const float gre = rg[K * NM + k * NM + a].re, gim = rg[K * NM + k * NM + a].im;
                    dr[a] = (float)fma(sFr, Yr[a], fma(-sFi, Yi[a], -(double)rre));
                    di[a] = (float)fma(sFr, Yi[a], fma(sFi, Yr[a], -(double)rim));
                    const cpx<float> q0 = q[a], q1 = q[NM + a], q2 = q[2 * NM + a], q3 = q[3 * NM + a];
                    const float qr = w0 * q0.re + w1 * q1.re + w2 * q2.re + w3 * q3.re;
                    const float qi = w0 * q0.im + w1 * q1.im + w2 * q2.im + w3 * q3.im;
                    B = fma(dr[a], qr - gre, B);
                    B = fma(di[a], qi - gim, B);
                });
                // quadratic form, row by row of the upper triangle
                static_for<0, NV>([&](auto I_) {
                    constexpr int i = decltype(I_)::value;
                    constexpr int row = (i * (2 * NV - i + 1)) / 2;
                    const float vi = (i & 1) ? di[i >> 1] : dr[i >> 1];
                    float t = 0.0f;
                    static_for<i, NV>([&](auto J_) {
                        constexpr int j = decltype(J_)::value;
                        const float vj = (j & 1) ? di[j >> 1] : dr[j >> 1];
                        t = fma(Wt[k * NT + row + (j - i)], vj, t);
                    });
                    Cq = fma(vi, t, Cq);
                });
            }
            const double lnL = (A - *C0p) + (double)fma(-0.25f, Cq, B);
            const double outv = ok ? lnL : -INFINITY;
            if (outL) outL[i] = outv;
            if (outW) outW[i] = outv + (lr ? (double)lr[i] : 0.0);
        }
    }
};

template <int S>
constexpr int ref_block_threads() {
    return lds_block_threads(S, kMixed);
}

template <int S, int K, bool LDS>
__global__ void __launch_bounds__(ref_block_threads<S>(), 1)
    k_lnl_ref(const EvalJob *__restrict__ jobs, const Tile *__restrict__ tiles) {
    extern __shared__ __align__(16) char ile_smem[];
    const Tile tl = tiles[blockIdx.x];
    RefKernel<S, K, LDS>::run(jobs + tl.job, tl.begin, tl.end, ile_smem);
}

// The reference of a job: r_k = s F_k Y(theta_ref) (FP64 geometry, rounded
// to FP32 and back so that both precisions hold it exactly), the series
// R_k[i] = Re(r_k^+ Q_k[i]) from the FP64 window, G_k = (U_k r_k +
// conj(V_k r_k))/2 and C0 = 1/2 sum_k Re(r_k^+ G_k) from the FP64 overlaps.
// A reference outside the support (D <= 0, |cos iota| > 1, non-finite) gives
// r = 0.  One block.
template <int S, int K>
__global__ void __launch_bounds__(256) k_ref_build(const EvalJob J, RefBuild rb) {
    constexpr int NM = kSets[S].n;
    using LK64 = LnlKernel<S, K, kFP64, false, false>;
    constexpr int NE = LK64::NE;
    __shared__ double sr[K][NM][2];
    __shared__ double red[256];
    if (threadIdx.x == 0) {
        const double *t = rb.theta_ref;
        const bool ok = t[3] > 0.0 && t[4] >= -1.0 && t[4] <= 1.0 && isfinite(t[0]) && isfinite(t[1]) &&
                        isfinite(t[2]) && isfinite(t[5]) && isfinite(t[6]);
        double Fr[K], Fi[K], uu[K], y[NM], Er[NE], Ei[NE];
        LK64::geometry(J, t[0], t[1], t[2], ok ? t[4] : 0.0, t[5], t[6], Fr, Fi, uu, y, Er, Ei);
        const double s = ok ? J.d_ref / t[3] : 0.0;
        for (int k = 0; k < K; k++)
            for (int a = 0; a < NM; a++) {
                const int m = kSets[S].m[a];
                const int am = m < 0 ? -m : m;
                const double yr = y[a] * Er[am];
                const double yi = (m > 0) ? -y[a] * Ei[am] : y[a] * Ei[am];
                const double cr = s * (Fr[k] * yr - Fi[k] * yi);
                const double cim = s * (Fr[k] * yi + Fi[k] * yr);
                sr[k][a][0] = ok ? (double)(float)cr : 0.0;
                sr[k][a][1] = ok ? (double)(float)cim : 0.0;
                rb.rg[2 * (k * NM + a)] = (float)sr[k][a][0];
                rb.rg[2 * (k * NM + a) + 1] = (float)sr[k][a][1];
            }
    }
    __syncthreads();
    const int T = J.n_time;
    // R_k[i] = Re(sum_a conj(r_a) Q_a[i]) = sum_a (r_re Q_re + r_im Q_im)
    for (int w = threadIdx.x; w < K * T; w += blockDim.x) {
        const int k = w / T, i = w - k * T;
        const double *q = rb.Q64 + 2 * ((size_t)(k * T + i) * NM);
        double acc = 0.0;
        for (int a = 0; a < NM; a++) acc += sr[k][a][0] * q[2 * a] + sr[k][a][1] * q[2 * a + 1];
        rb.R[w] = acc;
    }
    // G_k,a = (sum_b U_ab r_b + conj(V_ab r_b)) / 2 and the C0 partials
    double part = 0.0;
    for (int w = threadIdx.x; w < K * NM; w += blockDim.x) {
        const int k = w / NM, a = w - k * NM;
        double gr = 0.0, gi = 0.0;
        for (int b = 0; b < NM; b++) {
            const double *u = rb.U64 + 2 * (((size_t)k * NM + a) * NM + b);
            const double *v = rb.V64 + 2 * (((size_t)k * NM + a) * NM + b);
            const double rr = sr[k][b][0], ri = sr[k][b][1];
            gr += (u[0] * rr - u[1] * ri) + (v[0] * rr - v[1] * ri);
            gi += (u[0] * ri + u[1] * rr) - (v[0] * ri + v[1] * rr);
        }
        gr *= 0.5;
        gi *= 0.5;
        rb.rg[2 * (K * NM + w)] = (float)gr;
        rb.rg[2 * (K * NM + w) + 1] = (float)gi;
        part += sr[k][a][0] * gr + sr[k][a][1] * gi;
    }
    red[threadIdx.x] = part;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *rb.C0 = 0.5 * red[0];
}

template <int S>
hipError_t launch_ref_sp(int kdet, size_t lds_bytes, const EvalJob *jobs, const Tile *tiles, int n_tiles,
                         int nthreads, hipStream_t st) {
    if (n_tiles <= 0) return hipSuccess;
    const bool lds = lds_bytes > 0;
    if (nthreads <= 0 || nthreads > ref_block_threads<S>() || nthreads % 64) return hipErrorInvalidValue;
    dim3 grid(n_tiles), block(nthreads);
    auto go = [&](auto KK, auto LL) -> hipError_t {
        constexpr int K = decltype(KK)::value;
        constexpr bool L = decltype(LL)::value;
        if constexpr (L && !lnl_lds_compiled(S, K, kMixed)) {
            return hipErrorInvalidValue;
        } else {
            auto fn = k_lnl_ref<S, K, L>;
            if (L) {
                hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                   (int)lds_bytes);
                if (e != hipSuccess) return e;
            }
            hipLaunchKernelGGL(fn, grid, block, L ? lds_bytes : 0, st, jobs, tiles);
            return hipGetLastError();
        }
    };
    using T2 = std::integral_constant<int, 2>;
    using T3 = std::integral_constant<int, 3>;
    if (kdet == 2) return lds ? go(T2{}, std::true_type{}) : go(T2{}, std::false_type{});
    if (kdet == 3) return lds ? go(T3{}, std::true_type{}) : go(T3{}, std::false_type{});
    return hipErrorInvalidValue;
}

template <int S>
hipError_t launch_ref_build_sp(int kdet, const EvalJob &job, const RefBuild &rb, hipStream_t st) {
    if (kdet == 2)
        hipLaunchKernelGGL((k_ref_build<S, 2>), dim3(1), dim3(256), 0, st, job, rb);
    else if (kdet == 3)
        hipLaunchKernelGGL((k_ref_build<S, 3>), dim3(1), dim3(256), 0, st, job, rb);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace ile
