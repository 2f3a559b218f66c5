// Distance-marginalised likelihood table.  With T1, T2 evaluated at s = 1
// (D = D_ref), the likelihood at distance D is exp(s T1 - s^2 T2 / 4), s = D_ref/D,
// and the distance-marginalised value is
//   L_D(T1, T2) = int p(D) exp(s T1 - s^2 T2 / 4) dD,   p(D) = 3 D^2 / (Dmax^3 - Dmin^3).
// In v = ln s this is C int exp(-3 v + E(e^v)) dv, C = 3 D_ref^3 / (Dmax^3 - Dmin^3),
// E(s) = s T1 - s^2 T2 / 4.  The table stores the residual
//   r = ln L_D - a^2,   a = T1 / sqrt(T2)   (a^2 = T1^2/T2 = max over all s of E),
// which is analytic in (T1, T2); a reference clamped to [s_min, s_max] would
// have a curvature jump where the best scale crosses a bound.  Nodes (u, b):
// a = a_scale sinh(u), b = ln T2.  Each node is one FP64 composite
// Gauss-Legendre quadrature (integrand scaled by its maximum over the range)
// with breakpoints at geometric multiples of the local width around the
// maximum of the integrand.
#include "ile_internal.h"

namespace ile {

namespace {

constexpr int kNu = 4096, kNb = 4096;
constexpr double kAMax = 200.0, kAScale = 1.0;
constexpr double kB0 = -13.815510557964274;   // ln 1e-6
constexpr double kB1 = 23.025850929940457;    // ln 1e10

// 10-point Gauss-Legendre nodes and weights on [-1, 1]
__constant__ double kGLx[10] = {-0.9739065285171717, -0.8650633666889845, -0.6794095682990244,
                                -0.4333953941292472, -0.1488743389816312, 0.1488743389816312,
                                0.4333953941292472,  0.6794095682990244,  0.8650633666889845,
                                0.9739065285171717};
__constant__ double kGLw[10] = {0.0666713443086881, 0.1494513491505806, 0.2190863625159820,
                                0.2692667193099963, 0.2955242247147529, 0.2955242247147529,
                                0.2692667193099963, 0.2190863625159820, 0.1494513491505806,
                                0.0666713443086881};

__global__ void __launch_bounds__(256) k_dist_table(double *tab, double s_min, double s_max, double lnC) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= kNu * kNb) return;
    const int iu = idx % kNu, ib = idx / kNu;
    const double du = 2.0 * asinh(kAMax / kAScale) / (kNu - 1);
    const double db = (kB1 - kB0) / (kNb - 1);
    const double u = -asinh(kAMax / kAScale) + iu * du;
    const double b = kB0 + ib * db;
    const double T2 = exp(b);
    const double T1 = kAScale * sinh(u) * sqrt(T2);
    const double sc = fmin(fmax(2.0 * T1 / T2, s_min), s_max);
    const double Emax = sc * T1 - sc * sc * T2 * 0.25;
    const double vlo = log(s_min), vhi = log(s_max);
    // maximum of g(v) = -3 v + E(e^v): (T2/2) s^2 - T1 s + 3 = 0, larger root
    double vp;
    const double disc = T1 * T1 - 6.0 * T2;
    if (disc >= 0.0 && T1 > 0.0) {
        const double sp = (T1 + sqrt(disc)) / T2;
        vp = fmin(fmax(log(sp), vlo), vhi);
    } else {
        vp = vlo;
    }
    const double sp = exp(vp);
    const double g1 = -3.0 + (T1 - sp * T2 * 0.5) * sp;
    const double g2 = -(T2 * 0.5) * sp * sp + (T1 - sp * T2 * 0.5) * sp;
    const double h = 1.0 / sqrt(fabs(g2) + g1 * g1 + 1e-30);
    // breakpoints: vp +- h * {0.5,1,2,4,8,16,32,64,128}, clipped
    double br[24];
    int nbk = 0;
    br[nbk++] = vlo;
    for (int k = 8; k >= 0; k--) {
        const double x = vp - h * (0.5 * (double)(1 << k));
        if (x > vlo && x < vhi) br[nbk++] = x;
    }
    if (vp > vlo && vp < vhi) br[nbk++] = vp;
    for (int k = 0; k <= 8; k++) {
        const double x = vp + h * (0.5 * (double)(1 << k));
        if (x > vlo && x < vhi) br[nbk++] = x;
    }
    br[nbk++] = vhi;
    double acc = 0.0;
    for (int q = 0; q + 1 < nbk; q++) {
        const double a0 = br[q], a1 = br[q + 1];
        // two panels per interval
        for (int p = 0; p < 2; p++) {
            const double lo = a0 + (a1 - a0) * 0.5 * p, hi = lo + (a1 - a0) * 0.5;
            const double c = 0.5 * (lo + hi), r = 0.5 * (hi - lo);
            for (int t = 0; t < 10; t++) {
                const double v = c + r * kGLx[t];
                const double s = exp(v);
                acc += r * kGLw[t] * exp(-3.0 * v + (s * T1 - s * s * T2 * 0.25) - Emax);
            }
        }
    }
    tab[idx] = lnC + log(acc) + Emax - T1 * T1 / T2;
}

}  // namespace

size_t dist_table_bytes() { return (size_t)kNu * kNb * sizeof(double); }

hipError_t build_dist_table(DistTable *tb, double *d_buf, PriorDev pr, hipStream_t st) {
    const double s_min = pr.d_ref / pr.d_max, s_max = pr.d_ref / pr.d_min;
    const double lnC = log(3.0 * pr.d_ref * pr.d_ref * pr.d_ref /
                           (pr.d_max * pr.d_max * pr.d_max - pr.d_min * pr.d_min * pr.d_min));
    hipLaunchKernelGGL(k_dist_table, dim3((kNu * kNb + 255) / 256), dim3(256), 0, st, d_buf, s_min, s_max, lnC);
    tb->r = d_buf;
    tb->nu = kNu;
    tb->nb = kNb;
    tb->u0 = -asinh(kAMax / kAScale);
    tb->du = 2.0 * asinh(kAMax / kAScale) / (kNu - 1);
    tb->b0 = kB0;
    tb->db = (kB1 - kB0) / (kNb - 1);
    tb->s_min = s_min;
    tb->s_max = s_max;
    tb->a_scale = kAScale;
    tb->inv_du = 1.0 / tb->du;
    tb->inv_db = 1.0 / tb->db;
    tb->inv_a_scale = 1.0 / kAScale;
    return hipGetLastError();
}

}  // namespace ile
