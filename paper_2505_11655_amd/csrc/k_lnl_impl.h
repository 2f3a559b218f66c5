// Fused per-sample log-likelihood kernel, eq. (def:lnL:Decomposed):
//   lnL = s Re sum_k sum_lm (F_k Y_lm)^* Q_k,lm(tau_k)
//         - s^2/4 sum_k [ |F_k|^2 Y^+ U_k Y + Re(F_k^2 Y^T V_k Y) ],  s = D_ref/D.
// One thread evaluates one sample at a time; a block owns one tile of one job.
//
// Work per sample (all of it in registers):
//   sky: n = (cos d cos h, cos d sin h, sin d), h = alpha - gmst, and the basis
//        e_a = (-sin h, cos h, 0), e_d = (-sin d cos h, -sin d sin h, cos d);
//   F_k = e^{-2i psi} [(e_a.D.e_a - e_d.D.e_d) - 2i e_a.D.e_d]  (equal to F+ + iFx
//        for X = -cos psi e_a + sin psi e_d, Y = sin psi e_a + cos psi e_d);
//   tau_k = t - x_k.n / c;
//   Y_lm = y_lm(iota) e^{-i m phi} with real y_lm from Wigner's formula in
//        cos(iota/2), sin(iota/2), and e^{i j phi} by repeated products;
//   T1 from the 4-tap Lagrange cubic of Q at tau_k (window in LDS or L2);
//   T2 from the pair sums grouped by m_a - m_b (U, Hermitian) and m_a + m_b
//        (V, symmetric): each pair costs one product y_a y_b and two FMAs per
//        detector; the phase e^{i(m_a - m_b) phi} is applied once per group.
#pragma once

#include <type_traits>

#include "ile_internal.h"
#include "ile_sincos.h"

namespace ile {

template <class T>
struct cpx {
    T re, im;
};

template <int POL>
struct PolTypes;
// Which arithmetic each part uses.  In the mixed policy only quantities that
// act as a point perturbation of the complex amplitudes z_k = s F_k Y (F_k,
// y_lm) stay FP32: lnL is stationary in z near its maximum, so their rounding
// enters at second order.  Everything that defines the quadratic form itself
// (delays and interpolation weights, the phase table e^{i j phi}, Q/U/V and
// the sums) is FP64, because its rounding enters at first order, ~eps rho^2.
template <>
struct PolTypes<kFP64> {
    using TT = double;  // theta, ln p - ln p_s
    using TS = double;  // sky direction and delays
    using TG = double;  // polarisation response and harmonic amplitudes
    using TE = double;  // phase table e^{i j phi}
    using TA = double;  // Q/U/V contractions and the combine
    using TO = double;  // lnL, lw
};
// FP32: the sky direction and the delays are FP64 as well.  The stencil
// position u = (tau - tau0)/dt is a few hundred samples, where an FP32 value
// is quantised to 3e-5 samples, and FP32 sines of the sky angles move the
// delays by about 1e-5 samples; either one shifts the phase of Q by enough to
// move lnL by ~1e-4 at SNR 20.  In FP64 the position is exact to rounding;
// its integer part picks the stencil and only the fraction becomes FP32.
template <>
struct PolTypes<kFP32> {
    using TT = float;
    using TS = double;
    using TG = float;
    using TE = float;
    using TA = float;
    using TO = float;
};
template <>
struct PolTypes<kMixed> {
    using TT = float;
    using TS = double;
    using TG = float;
    using TE = double;
    using TA = double;
    using TO = double;
};

// Angles go through an FP64 Cody-Waite reduction and a truncated series
// (ile_sincos.h): exact reduction for any angle a sample carries, and no
// large-argument branch (the library routines compute theirs as well: 124
// instructions for an FP32 sine and cosine).  FP32 results use an FP32 series.
__device__ __forceinline__ void dsincos(float x, float *s, float *c) { sincos_rad(x, s, c); }
__device__ __forceinline__ void dsincos(double x, double *s, double *c) { sincos_rad(x, s, c); }
// Sky angles: with FP32 geometry downstream (FP32 and mixed policies) only the
// delays need FP64, to ~1e-9 of a window sample: the shorter series.
template <class TS, class TG>
__device__ __forceinline__ void sky_sincos(TS x, TS *s, TS *c) {
    if constexpr (sizeof(TS) == 8 && sizeof(TG) == 4)
        sincos_rad_sky(x, s, c);
    else
        dsincos(x, s, c);
}
__device__ __forceinline__ float dfloor(float x) { return floorf(x); }
__device__ __forceinline__ double dfloor(double x) { return floor(x); }
__device__ __forceinline__ float dsqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double dsqrt(double x) { return sqrt(x); }

// A job constant in the requested precision (FP32 copies are made on the host).
template <class T>
__device__ __forceinline__ T pick(double d, float f) {
    if constexpr (std::is_same<T, float>::value)
        return f;
    else
        return d;
}

// Compiler-only ordering point (emits no instruction): memory operations are
// not moved across it, which bounds how many loads the scheduler keeps in
// flight (and in registers) at once.
__device__ __forceinline__ void fence() { asm volatile("" ::: "memory"); }

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Distance-marginalised lnL from the residual table (bicubic Lagrange),
// ln L_D = r(a, b) + a^2, a = T1/sqrt(T2), b = ln T2.  Out of table: -inf.
// The table coordinates are computed in TC (the policy's contraction type:
// FP32 for the FP32 policy, where T1 and T2 are FP32 values themselves);
// the FP64 table values are interpolated in FP64.
template <class TC, class TB>
__device__ __forceinline__ double dist_lookup(const TB &tb, TC T1, TC T2) {
    // branch-free: an input outside the table (or T2 <= 0, or NaN) reads the
    // clamped first cell and returns -inf
    const bool pos = T2 > (TC)0;
    const TC T2s = pos ? T2 : (TC)1;
    TC b, a, u;
    if constexpr (sizeof(TC) == 4) {
        b = logf(T2s);
        a = T1 / sqrtf(T2s);
        u = asinhf(a * (float)tb.inv_a_scale);
    } else {
        b = log(T2s);
        a = T1 / sqrt(T2s);
        u = asinh(a * tb.inv_a_scale);
    }
    const TC xu = (u - (TC)tb.u0) * (TC)tb.inv_du;
    const TC xb = (b - (TC)tb.b0) * (TC)tb.inv_db;
    TC fu = floor(xu), fb = floor(xb);
    const bool in = pos && fu >= (TC)1 && fu <= (TC)(tb.nu - 3) && fb >= (TC)1 && fb <= (TC)(tb.nb - 3);
    fu = in ? fu : (TC)1;
    fb = in ? fb : (TC)1;
    const int iu = (int)fu, ib = (int)fb;
    const double gu = (double)(xu - fu), gb = (double)(xb - fb);
    const double wu[4] = {-gu * (gu - 1.0) * (gu - 2.0) / 6.0, (gu + 1.0) * (gu - 1.0) * (gu - 2.0) * 0.5,
                          -(gu + 1.0) * gu * (gu - 2.0) * 0.5, (gu + 1.0) * gu * (gu - 1.0) / 6.0};
    const double wb[4] = {-gb * (gb - 1.0) * (gb - 2.0) / 6.0, (gb + 1.0) * (gb - 1.0) * (gb - 2.0) * 0.5,
                          -(gb + 1.0) * gb * (gb - 2.0) * 0.5, (gb + 1.0) * gb * (gb - 1.0) / 6.0};
    double r = 0.0;
#pragma unroll
    for (int jb = 0; jb < 4; jb++) {
        const double *row = tb.r + (size_t)(ib - 1 + jb) * tb.nu + (iu - 1);
        const double acc = wu[0] * row[0] + wu[1] * row[1] + wu[2] * row[2] + wu[3] * row[3];
        r += wb[jb] * acc;
    }
    return in ? r + (double)a * (double)a : -INFINITY;
}

// The same table along one row of constant T2, for the time-marginalised
// likelihood (a sample's T2 is the same at every time node): the b position
// and weights are formed once, and each node costs the a-direction only.  All
// in FP64.
struct DistRow {
    double inv_sqrt_T2;
    double wb[4];
    int ib;
    bool ok;
};
template <class TB>
__device__ __forceinline__ DistRow dist_row(const TB &tb, double T2) {
    DistRow d;
    d.ok = T2 > 0.0;
    const double T2s = d.ok ? T2 : 1.0;
    d.inv_sqrt_T2 = 1.0 / sqrt(T2s);
    const double xb = (log(T2s) - tb.b0) * tb.inv_db;
    double fb = floor(xb);
    d.ok = d.ok && fb >= 1.0 && fb <= (double)(tb.nb - 3);
    fb = d.ok ? fb : 1.0;
    d.ib = (int)fb;
    const double gb = xb - fb;
    d.wb[0] = -gb * (gb - 1.0) * (gb - 2.0) / 6.0;
    d.wb[1] = (gb + 1.0) * (gb - 1.0) * (gb - 2.0) * 0.5;
    d.wb[2] = -(gb + 1.0) * gb * (gb - 2.0) * 0.5;
    d.wb[3] = (gb + 1.0) * gb * (gb - 1.0) / 6.0;
    return d;
}
template <class TB>
__device__ __forceinline__ double dist_at(const TB &tb, const DistRow &d, double T1) {
    const double a = T1 * d.inv_sqrt_T2;
    const double xu = (asinh(a * tb.inv_a_scale) - tb.u0) * tb.inv_du;
    double fu = floor(xu);
    const bool in = d.ok && fu >= 1.0 && fu <= (double)(tb.nu - 3);
    fu = in ? fu : 1.0;
    const int iu = (int)fu;
    const double gu = xu - fu;
    const double wu[4] = {-gu * (gu - 1.0) * (gu - 2.0) / 6.0, (gu + 1.0) * (gu - 1.0) * (gu - 2.0) * 0.5,
                          -(gu + 1.0) * gu * (gu - 2.0) * 0.5, (gu + 1.0) * gu * (gu - 1.0) / 6.0};
    double r = 0.0;
#pragma unroll
    for (int jb = 0; jb < 4; jb++) {
        const double *row = tb.r + (size_t)(d.ib - 1 + jb) * tb.nu + (iu - 1);
        r += d.wb[jb] * (wu[0] * row[0] + wu[1] * row[1] + wu[2] * row[2] + wu[3] * row[3]);
    }
    return in ? r + a * a : -INFINITY;
}

template <int S, int K, int POL, bool LDS, bool DM>
struct LnlKernel {
    using MS = MSet<S>;
    using Tp = PolTypes<POL>;
    using TT = typename Tp::TT;
    using TS = typename Tp::TS;
    using TG = typename Tp::TG;
    using TE = typename Tp::TE;
    using TA = typename Tp::TA;
    using TO = typename Tp::TO;
    static constexpr int NM = MS::n;
    static constexpr int LM = MS::lmax;
    static constexpr int NE = 2 * LM + 1;  // e^{i j phi}, j = 0..2 lmax
    // detectors read through L1/L2 by the LDS-staged variant (their windows
    // do not fit next to the others)
    static constexpr int kG = LDS ? lds_global_dets(S, K, POL) : 0;

    // Sky direction, polarisation response F_k, stencil positions
    // u_k = (tau_k - tau0)/dt in window samples with tau_k = t - x_k.n/c (at
    // time tt), harmonic amplitudes y_lm(iota) and the phase table e^{i j phi}.
    template <class JT>
    __device__ __forceinline__ static void geometry(const JT &J, const TT al, const TT de, const TT tt,
                                                    const TT ci, const TT ph, const TT ps, TG (&Fr)[K], TG (&Fi)[K],
                                                    TS (&uu)[K], TG (&y)[NM], TE (&Er)[NE], TE (&Ei)[NE]) {
        // ---- sky direction, polarisation basis, delays
        TS sd, cd, sh, ch;
        sky_sincos<TS, TG>((TS)de, &sd, &cd);
        sky_sincos<TS, TG>((TS)al - pick<TS>(J.gmst, J.gmstf), &sh, &ch);
        const TS n0 = cd * ch, n1 = cd * sh, n2 = sd;
        const TG ea0 = (TG)(-sh), ea1 = (TG)ch;
        const TG ed0 = (TG)(-sd * ch), ed1 = (TG)(-sd * sh), ed2 = (TG)cd;
        TG s2p, c2p;
        dsincos((TG)2 * (TG)ps, &s2p, &c2p);
#pragma unroll
        for (int k = 0; k < K; k++) {
            const TG dxx = pick<TG>(J.D[k][0], J.Df[k][0]), dyy = pick<TG>(J.D[k][1], J.Df[k][1]);
            const TG dzz = pick<TG>(J.D[k][2], J.Df[k][2]), dxy = pick<TG>(J.D[k][3], J.Df[k][3]);
            const TG dxz = pick<TG>(J.D[k][4], J.Df[k][4]), dyz = pick<TG>(J.D[k][5], J.Df[k][5]);
            const TG A = dxx * ea0 * ea0 + dyy * ea1 * ea1 + (TG)2 * dxy * ea0 * ea1;
            const TG B = dxx * ed0 * ed0 + dyy * ed1 * ed1 + dzz * ed2 * ed2 +
                         (TG)2 * (dxy * ed0 * ed1 + dxz * ed0 * ed2 + dyz * ed1 * ed2);
            const TG C = dxx * ea0 * ed0 + dyy * ea1 * ed1 + dxy * (ea0 * ed1 + ea1 * ed0) +
                         dxz * ea0 * ed2 + dyz * ea1 * ed2;
            const TG Gr = A - B, Gi = (TG)-2 * C;
            Fr[k] = c2p * Gr + s2p * Gi;
            Fi[k] = c2p * Gi - s2p * Gr;
            const TS dly = pick<TS>(J.xc[k][0], J.xcf[k][0]) * n0 + pick<TS>(J.xc[k][1], J.xcf[k][1]) * n1 +
                           pick<TS>(J.xc[k][2], J.xcf[k][2]) * n2;
            uu[k] = (((TS)tt - dly) - pick<TS>(J.tau0, J.tau0f)) * pick<TS>(J.inv_dt, J.inv_dtf);
        }

        // ---- harmonics y_lm(iota) and phases e^{i j phi}
        const TG c = (TG)ci;
        const TG chalf = dsqrt(fmax((TG)0.5 * ((TG)1 + c), (TG)0));
        const TG shalf = dsqrt(fmax((TG)0.5 * ((TG)1 - c), (TG)0));
        TG cp[2 * LM + 1], sp[2 * LM + 1];
        cp[0] = (TG)1;
        sp[0] = (TG)1;
#pragma unroll
        for (int j = 1; j <= 2 * LM; j++) {
            cp[j] = cp[j - 1] * chalf;
            sp[j] = sp[j - 1] * shalf;
        }
        static_for<0, NM>([&](auto A_) {
            constexpr int a = decltype(A_)::value;
            constexpr WTerm w = wigner_terms(kSets[S].l[a], kSets[S].m[a]);
            TG acc = (TG)0;
            static_for<0, w.nt>([&](auto T_) {
                constexpr int t = decltype(T_)::value;
                acc += (TG)w.coef[t] * cp[w.p[t]] * sp[w.q[t]];
            });
            y[a] = acc;
        });
        TE sph, cph;
        dsincos((TE)ph, &sph, &cph);
        Er[0] = (TE)1;
        Ei[0] = (TE)0;
#pragma unroll
        for (int j = 1; j < NE; j++) {
            Er[j] = Er[j - 1] * cph - Ei[j - 1] * sph;
            Ei[j] = Er[j - 1] * sph + Ei[j - 1] * cph;
        }
    }

    // The quadratic form T2 from the pair tables (read through the scalar cache).
    // CHAIN: the phase rotations of the pair groups as explicit FMA chains
    // (two instructions where acc + (x y - z w) costs three); off for the
    // time-marginalised kernel, whose register budget the chained form
    // exceeds (it then spills).
    typedef __attribute__((address_space(4))) const cpx<TA> ccpx;
    template <bool CHAIN = true>
    __device__ __forceinline__ static TA quad_T2(const TG (&Fr)[K], const TG (&Fi)[K], const TG (&y)[NM],
                                                 const TE (&Er)[NE], const TE (&Ei)[NE], ccpx *Ut, ccpx *Vt) {
        // ---- T2 = sum_k |F_k|^2 Y^+ U_k Y + Re(F_k^2 Y^T V_k Y)
        TA uk[K], vr[K], vi[K];
#pragma unroll
        for (int k = 0; k < K; k++) {
            uk[k] = (TA)0;
            vr[k] = (TA)0;
            vi[k] = (TA)0;
        }
        constexpr PairTable pt = MS::pt;
        static_for<0, NE>([&](auto G_) {
            constexpr int g = decltype(G_)::value;
            fence();
            TA Ar[K], Ai[K];
#pragma unroll
            for (int k = 0; k < K; k++) {
                Ar[k] = (TA)0;
                Ai[k] = (TA)0;
            }
            static_for<pt.u_start[g], pt.u_start[g + 1]>([&](auto J_) {
                constexpr int j = decltype(J_)::value;
                constexpr int p = pt.u_pair[j];
                const TA py = (TA)y[pt.a[p]] * (TA)y[pt.b[p]];
#pragma unroll
                for (int k = 0; k < K; k++) {
                    Ar[k] += py * Ut[j * K + k].re;
                    if constexpr (g > 0) Ai[k] += py * Ut[j * K + k].im;
                }
            });
#pragma unroll
            for (int k = 0; k < K; k++) {
                if constexpr (g == 0) {
                    uk[k] += Ar[k];
                } else if constexpr (CHAIN) {
                    uk[k] = fma((TA)Er[g], Ar[k], uk[k]);
                    uk[k] = fma(-(TA)Ei[g], Ai[k], uk[k]);
                } else {
                    uk[k] += (TA)Er[g] * Ar[k] - (TA)Ei[g] * Ai[k];
                }
            }
        });
        static_for<0, 4 * LM + 1>([&](auto G_) {
            constexpr int g = decltype(G_)::value;
            fence();
            constexpr int sm = g - 2 * LM;
            if constexpr (pt.v_start[g + 1] > pt.v_start[g]) {
                TA Br[K], Bi[K];
#pragma unroll
                for (int k = 0; k < K; k++) {
                    Br[k] = (TA)0;
                    Bi[k] = (TA)0;
                }
                static_for<pt.v_start[g], pt.v_start[g + 1]>([&](auto J_) {
                    constexpr int j = decltype(J_)::value;
                    constexpr int p = pt.v_pair[j];
                    const TA py = (TA)y[pt.a[p]] * (TA)y[pt.b[p]];
#pragma unroll
                    for (int k = 0; k < K; k++) {
                        Br[k] += py * Vt[j * K + k].re;
                        Bi[k] += py * Vt[j * K + k].im;
                    }
                });
                // e^{-i sm phi}
                const TA er = (TA)Er[sm < 0 ? -sm : sm];
                const TA ei = (sm < 0) ? (TA)Ei[-sm] : -(TA)Ei[sm];
#pragma unroll
                for (int k = 0; k < K; k++) {
                    if constexpr (CHAIN) {
                        vr[k] = fma(er, Br[k], vr[k]);
                        vr[k] = fma(-ei, Bi[k], vr[k]);
                        vi[k] = fma(er, Bi[k], vi[k]);
                        vi[k] = fma(ei, Br[k], vi[k]);
                    } else {
                        vr[k] += er * Br[k] - ei * Bi[k];
                        vi[k] += er * Bi[k] + ei * Br[k];
                    }
                }
            }
        });
        TA T2 = (TA)0;
#pragma unroll
        for (int k = 0; k < K; k++) {
            const TA fr = (TA)Fr[k], fi = (TA)Fi[k];
            T2 += (fr * fr + fi * fi) * uk[k] + (fr * fr - fi * fi) * vr[k] - (TA)2 * fr * fi * vi[k];
        }
        return T2;
    }

    // The job descriptor as seen through the constant address space: its
    // fields load through the scalar cache.
    typedef __attribute__((address_space(4))) const EvalJob cjob;

    __device__ __forceinline__ static void run(const EvalJob *Jp, const int64_t begin, const int64_t end,
                                               cpx<TA> *smem) {
        const EvalJob &J = *Jp;
        const int T = J.n_time;
        const cpx<TA> *__restrict__ Qg = (const cpx<TA> *)J.Q;
        if constexpr (LDS) {
            // stage the windows of detectors kG..K-1 of this job
            const size_t nwords = (size_t)(K - kG) * T * NM * sizeof(cpx<TA>) / 8;
            const uint2 *src = (const uint2 *)(Qg + (size_t)kG * T * NM);
            uint2 *dst = (uint2 *)smem;
            for (size_t w = threadIdx.x; w < nwords; w += blockDim.x) dst[w] = src[w];
            __syncthreads();
        }
        // The pair tables are read-only for the whole launch and every lane of
        // a block reads the same entry: reading them through the constant
        // address space lets them come through the scalar cache into SGPRs
        // (operands of the FMAs) instead of per-sample vector loads.
        ccpx *Ut = (ccpx *)J.Ut;
        ccpx *Vt = (ccpx *)J.Vt;
        const TT *__restrict__ th = (const TT *)J.theta;
        const TT *__restrict__ lr = (const TT *)J.lnpmps;
        TO *__restrict__ outL = (TO *)J.lnL;
        TO *__restrict__ outW = (TO *)J.lw;
        const int64_t ld = J.ld;

        for (int64_t i = begin + threadIdx.x; i < end; i += blockDim.x) {
            // Empty statement (emits no instruction): the table pointers look
            // loop-variant, so the scalar loads stream per sample instead of
            // being hoisted into more SGPRs than exist (which spills them).
            asm volatile("" : "+s"(Ut), "+s"(Vt));
            // Likewise the descriptor: its geometry constants (FP64 detector
            // positions, response tensors, window origin) are re-read per
            // sample through the scalar cache instead of holding scalar
            // registers across the pair sums, which need them all.
            cjob *Jc = (cjob *)Jp;
            asm volatile("" : "+s"(Jc));
            const TT al = th[i], de = th[ld + i], tt = th[2 * ld + i], DD = th[3 * ld + i];
            const TT ci = th[4 * ld + i], ph = th[5 * ld + i], ps = th[6 * ld + i];
            bool ok = (DM || DD > (TT)0) && (ci >= (TT)-1 && ci <= (TT)1);

            TG Fr[K], Fi[K];
            TS uu[K];
            TG y[NM];
            TE Er[NE], Ei[NE];
            geometry(*Jc, al, de, tt, ci, ph, ps, Fr, Fi, uu, y, Er, Ei);

            // ---- T1 = sum_k Re[conj(F_k) sum_a y_a e^{i m_a phi} Qhat_k,a]
            TA T1 = (TA)0;
#pragma unroll
            for (int k = 0; k < K; k++) {
                fence();
                // integer part of the stencil position in its own precision;
                // the fraction (exact: u - floor(u)) in the contraction type
                const TS fl = dfloor(uu[k]);
                ok = ok && (fl >= (TS)1) && (fl <= (TS)(T - 3));
                const TS flc = fmin(fmax(fl, (TS)1), (TS)(T - 3));
                const int i0 = (int)flc;
                const TA f = (TA)(uu[k] - fl);
                const TA fm1 = f - (TA)1, fm2 = f - (TA)2, fp1 = f + (TA)1;
                const TA w0 = -f * fm1 * fm2 * (TA)(1.0 / 6.0);
                const TA w1 = fp1 * fm1 * fm2 * (TA)0.5;
                const TA w2 = -fp1 * f * fm2 * (TA)0.5;
                const TA w3 = fp1 * f * fm1 * (TA)(1.0 / 6.0);
                const cpx<TA> *q = (LDS && k >= kG) ? smem + ((size_t)(k - kG) * T + (i0 - 1)) * NM
                                                    : Qg + ((size_t)k * T + (i0 - 1)) * NM;
                TA ar = (TA)0, ai = (TA)0;
                static_for<0, NM>([&](auto A_) {
                    constexpr int a = decltype(A_)::value;
                    constexpr int m = kSets[S].m[a];
                    const cpx<TA> q0 = q[a], q1 = q[NM + a], q2 = q[2 * NM + a], q3 = q[3 * NM + a];
                    const TA qr = w0 * q0.re + w1 * q1.re + w2 * q2.re + w3 * q3.re;
                    const TA qi = w0 * q0.im + w1 * q1.im + w2 * q2.im + w3 * q3.im;
                    const TA er = (TA)Er[m < 0 ? -m : m];
                    const TA ei = (m < 0) ? -(TA)Ei[-m] : (TA)Ei[m];
                    const TA zr = (TA)y[a] * er, zi = (TA)y[a] * ei;
                    // explicit FMA chains: ar + (zr qr - zi qi) written as
                    // such costs a multiply, an FMA and an add
                    ar = fma(zr, qr, ar);
                    ar = fma(-zi, qi, ar);
                    ai = fma(zr, qi, ai);
                    ai = fma(zi, qr, ai);
                });
                T1 = fma((TA)Fr[k], ar, T1);
                T1 = fma((TA)Fi[k], ai, T1);
            }

            const TA T2 = quad_T2(Fr, Fi, y, Er, Ei, Ut, Vt);

            // ---- combine
            TA lnL;
            if constexpr (DM) {
                lnL = (TA)dist_lookup<TA>(Jc->dt, T1, T2);
            } else {
                const TA s = pick<TA>(Jc->d_ref, Jc->d_reff) / (TA)DD;
                lnL = s * T1 - s * s * T2 * (TA)0.25;
            }
            TO outv = ok ? (TO)lnL : (TO)-INFINITY;
            if (outL) outL[i] = outv;
            if (outW) outW[i] = outv + (lr ? (TO)lr[i] : (TO)0);
        }
    }
};

// Minimum waves per SIMD asked of the register allocator: two, except for the
// 17/21-mode sets with FP64 contractions and the 21-mode set in FP32, whose
// live state does not fit in 256 VGPRs without spilling.
template <int S, int POL>
constexpr int lnl_min_waves() {
    return ((S >= 2 && POL != kFP32) || S == 3) ? 1 : 2;
}

template <int S, int K, int POL, bool LDS, bool DM>
__global__ void __launch_bounds__(LDS ? lds_block_threads(S, POL) : 256, (lnl_min_waves<S, POL>()))
    k_lnl(const EvalJob *__restrict__ jobs, const Tile *__restrict__ tiles) {
    extern __shared__ __align__(16) char ile_smem[];
    using TA = typename PolTypes<POL>::TA;
    const Tile tl = tiles[blockIdx.x];
    LnlKernel<S, K, POL, LDS, DM>::run(jobs + tl.job, tl.begin, tl.end, (cpx<TA> *)ile_smem);
}


template <int S, int POL>
hipError_t launch_eval_sp(int kdet, bool dm, size_t lds_bytes, const EvalJob *jobs, const Tile *tiles, int n_tiles,
                          int nthreads, hipStream_t st) {
    if (n_tiles <= 0) return hipSuccess;
    const bool lds = lds_bytes > 0;
    if (nthreads <= 0 || nthreads > (lds ? lds_block_threads(S, POL) : 256) || nthreads % 64) return hipErrorInvalidValue;
    if (dm && POL == kMixed) return hipErrorInvalidValue;
    dim3 grid(n_tiles), block(nthreads);
    auto go = [&](auto KK, auto LL, auto DD) -> hipError_t {
        constexpr int K = decltype(KK)::value;
        constexpr bool L = decltype(LL)::value;
        constexpr bool D = decltype(DD)::value;
        if constexpr ((L && !lnl_lds_compiled(S, K, POL)) || (D && POL == kMixed)) {
            return hipErrorInvalidValue;
        } else {
            auto fn = k_lnl<S, K, POL, L, D>;
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
    using BT = std::true_type;
    using BF = std::false_type;
    if (kdet == 2) {
        if (lds) return dm ? go(T2{}, BT{}, BT{}) : go(T2{}, BT{}, BF{});
        return dm ? go(T2{}, BF{}, BT{}) : go(T2{}, BF{}, BF{});
    }
    if (kdet == 3) {
        if (lds) return dm ? go(T3{}, BT{}, BT{}) : go(T3{}, BT{}, BF{});
        return dm ? go(T3{}, BF{}, BT{}) : go(T3{}, BF{}, BF{});
    }
    return hipErrorInvalidValue;
}

}  // namespace ile
