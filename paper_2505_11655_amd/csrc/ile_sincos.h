// Sine and cosine of an FP64 angle for the likelihood kernels.
//
// Method: Cody-Waite argument reduction (W. J. Cody and W. Waite, "Software
// Manual for the Elementary Functions", 1980) by pi/2 held as two doubles,
// r = (x - k P1) - k P2 with k = rint(2x/pi), each step one fused
// multiply-add; then the Taylor series of sin and cos on |r| <= pi/4 (+ the
// rounding of k), truncated after r^17 and r^16, where the first omitted
// terms are below 1e-19 and 3e-18.  The quadrant k mod 4 maps (sin r, cos r)
// to (sin x, cos x).
//
// Accuracy (full series): a few units in the last place for |x| < 2^50.  With the FMA the
// first reduction step is exact, and pi/2 - P1 - P2 is ~1e-33, so the
// reduction keeps full precision far beyond the angles a sample carries.
// Unlike the general library routine it has no large-argument branch, which
// keeps it short and its register use small.
#pragma once

#include <hip/hip_runtime.h>

namespace ile {

// An FP64 constant the compiler must materialise where it is used (two
// scalar moves) instead of hoisting it out of the sample loop, where each one
// would hold a scalar register pair for the whole loop body; the likelihood's
// pair tables need those registers.
__host__ __device__ __forceinline__ double kconst(double v) {
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" : "+s"(v));
#endif
    return v;
}

// Reduction: x = k pi/2 + r, |r| <= pi/4 (+ the rounding of k); q = k mod 4.
__host__ __device__ __forceinline__ double reduce_pio2(const double x, double *kq) {
    constexpr double kTwoOverPi = 0.63661977236758134308;   // 2/pi
    constexpr double kP1 = 1.5707963267948966192;            // pi/2 rounded to double
    constexpr double kP2 = 6.1232339957367660360e-17;        // pi/2 - kP1 rounded to double
    const double k = rint(x * kconst(kTwoOverPi));
    double r = fma(-k, kconst(kP1), x);
    r = fma(-k, kconst(kP2), r);
    *kq = k - 4.0 * floor(k * 0.25);                         // exact for |k| < 2^53
    return r;
}

// (sin r, cos r) -> (sin x, cos x) for quadrant q of x = q pi/2 + r.
template <class T>
__host__ __device__ __forceinline__ void quadrant(const double kq, const T sr, const T cr, T *s, T *c) {
    const bool swap = kq == 1.0 || kq == 3.0;
    const T sv = swap ? cr : sr;
    const T cv = swap ? sr : cr;
    *s = (kq >= 2.0) ? -sv : sv;
    *c = (kq == 1.0 || kq == 2.0) ? -cv : cv;
}

// Full FP64 accuracy: series to r^17 (sin) and r^16 (cos).  Used where the
// result stays FP64 (the FP64 policy).
__host__ __device__ __forceinline__ void sincos_rad(const double x, double *s, double *c) {
    double kq;
    const double r = reduce_pio2(x, &kq);
    const double r2 = r * r;
    // sin r = r - r^3/3! + ... + r^17/17!
    double ps = kconst(1.0 / 355687428096000.0);                    //  1/17!
    ps = fma(ps, r2, kconst(-1.0 / 1307674368000.0));               // -1/15!
    ps = fma(ps, r2, kconst(1.0 / 6227020800.0));                   //  1/13!
    ps = fma(ps, r2, kconst(-1.0 / 39916800.0));                    // -1/11!
    ps = fma(ps, r2, kconst(1.0 / 362880.0));                       //  1/9!
    ps = fma(ps, r2, kconst(-1.0 / 5040.0));                        // -1/7!
    ps = fma(ps, r2, kconst(1.0 / 120.0));                          //  1/5!
    ps = fma(ps, r2, kconst(-1.0 / 6.0));                           // -1/3!
    const double sr = fma(ps * r2, r, r);
    // cos r = 1 - r^2/2! + ... + r^16/16!
    double pc = kconst(1.0 / 20922789888000.0);                     //  1/16!
    pc = fma(pc, r2, kconst(-1.0 / 87178291200.0));                 // -1/14!
    pc = fma(pc, r2, kconst(1.0 / 479001600.0));                    //  1/12!
    pc = fma(pc, r2, kconst(-1.0 / 3628800.0));                     // -1/10!
    pc = fma(pc, r2, kconst(1.0 / 40320.0));                        //  1/8!
    pc = fma(pc, r2, kconst(-1.0 / 720.0));                         // -1/6!
    pc = fma(pc, r2, kconst(1.0 / 24.0));                           //  1/4!
    pc = fma(pc, r2, -0.5);                                 // -1/2!
    const double cr = fma(pc, r2, 1.0);
    quadrant(kq, sr, cr, s, c);
}

// Sky-direction grade: series to r^11 and r^12 (first omitted terms below
// 8e-12 and 4e-13), enough for delays of at most ~90 window samples to stay
// within 1e-9 of a sample.  Fewer 64-bit coefficients than the full series
// (each one occupies a scalar register pair).
__host__ __device__ __forceinline__ void sincos_rad_sky(const double x, double *s, double *c) {
    double kq;
    const double r = reduce_pio2(x, &kq);
    const double r2 = r * r;
    double ps = kconst(-1.0 / 39916800.0);                          // -1/11!
    ps = fma(ps, r2, kconst(1.0 / 362880.0));                       //  1/9!
    ps = fma(ps, r2, kconst(-1.0 / 5040.0));                        // -1/7!
    ps = fma(ps, r2, kconst(1.0 / 120.0));                          //  1/5!
    ps = fma(ps, r2, kconst(-1.0 / 6.0));                           // -1/3!
    const double sr = fma(ps * r2, r, r);
    double pc = kconst(1.0 / 479001600.0);                          //  1/12!
    pc = fma(pc, r2, kconst(-1.0 / 3628800.0));                     // -1/10!
    pc = fma(pc, r2, kconst(1.0 / 40320.0));                        //  1/8!
    pc = fma(pc, r2, kconst(-1.0 / 720.0));                         // -1/6!
    pc = fma(pc, r2, kconst(1.0 / 24.0));                           //  1/4!
    pc = fma(pc, r2, -0.5);                                 // -1/2!
    const double cr = fma(pc, r2, 1.0);
    quadrant(kq, sr, cr, s, c);
}

// FP32 results: the FP64 reduction (exact for any float angle), then FP32
// series to r^9 and r^10 (first omitted terms below 2e-9 and 1.2e-10, under
// FP32 rounding).  FP32 coefficients are instruction literals.
__host__ __device__ __forceinline__ void sincos_rad(const float x, float *s, float *c) {
    double kq;
    const float r = (float)reduce_pio2((double)x, &kq);
    const float r2 = r * r;
    float ps = 1.0f / 362880.0f;                            //  1/9!
    ps = fmaf(ps, r2, -1.0f / 5040.0f);                     // -1/7!
    ps = fmaf(ps, r2, 1.0f / 120.0f);                       //  1/5!
    ps = fmaf(ps, r2, -1.0f / 6.0f);                        // -1/3!
    const float sr = fmaf(ps * r2, r, r);
    float pc = -1.0f / 3628800.0f;                          // -1/10!
    pc = fmaf(pc, r2, 1.0f / 40320.0f);                     //  1/8!
    pc = fmaf(pc, r2, -1.0f / 720.0f);                      // -1/6!
    pc = fmaf(pc, r2, 1.0f / 24.0f);                        //  1/4!
    pc = fmaf(pc, r2, -0.5f);                               // -1/2!
    const float cr = fmaf(pc, r2, 1.0f);
    quadrant(kq, sr, cr, s, c);
}

}  // namespace ile
