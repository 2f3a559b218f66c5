/*
 * Plain FP64 CPU oracle for the ILE extrinsic-likelihood path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or table with the HIP
 * path.  Every routine is the plain definition from the paper, written for
 * readability: no blocking, no fusion, no symmetry tricks, no fast-math.
 *
 * Paper: arXiv 2505.11655, Section "Review of the RIFT likelihood",
 *   eq. (def:lnL:Decomposed) and eq. (QUV), eq. (lnL:MonteCarlo), eq. (neff);
 *   Appendix "Spherical harmonic frame conventions", eq. (hlm).
 *
 * Conventions (readings where the paper is silent or inconsistent):
 *   - F_k := F+ + i Fx makes the printed decomposition exact for
 *     h = h+ - i hx and h_k = F+ h+ + Fx hx.
 *   - n_hat points to the source; tau_k = t - x_k . n_hat / c.
 *   - Y_lm = -2Y_lm(iota, -phi_c) (phi_* = 0 in eq. hlm); psi enters only
 *     through the polarisation basis.
 *   - Q between window samples: 4-point Lagrange cubic, stencil i-1..i+2,
 *     valid for 1 <= i <= T-3, else lnL = -inf.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_C_SI 299792458.0
#define ORC_PI 3.14159265358979323846

typedef struct {
    int n_det, n_modes, n_time;
    const int *mode_l, *mode_m;     /* [n_modes] */
    const double *det_pos;          /* [n_det][3] metres, Earth-fixed */
    const double *det_resp;         /* [n_det][3][3] */
    double gmst, tau0, dt;          /* tau_i = tau0 + i dt */
    const double *Q;                /* [n_det][n_modes][n_time] complex (re,im) */
    const double *U;                /* [n_det][n_modes][n_modes] complex */
    const double *V;                /* same, or NULL for zero */
    double d_ref;
} orc_problem;

/* ------------------------------------------------------------------ geometry */

/* Polarisation basis and antenna response by the tensor definition:
 * X = -cos(psi) e_a + sin(psi) e_d,  Y = sin(psi) e_a + cos(psi) e_d,
 * F+ = X^T D X - Y^T D Y,  Fx = X^T D Y + Y^T D X. */
void orc_antenna(const double *D, double ra, double dec, double psi, double gmst,
                 double *Fp, double *Fx)
{
    double h = ra - gmst;
    double ea[3] = {-sin(h), cos(h), 0.0};
    double ed[3] = {-sin(dec) * cos(h), -sin(dec) * sin(h), cos(dec)};
    double X[3], Y[3];
    for (int i = 0; i < 3; i++) {
        X[i] = -cos(psi) * ea[i] + sin(psi) * ed[i];
        Y[i] = sin(psi) * ea[i] + cos(psi) * ed[i];
    }
    double xdx = 0, ydy = 0, xdy = 0, ydx = 0;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            xdx += X[i] * D[3 * i + j] * X[j];
            ydy += Y[i] * D[3 * i + j] * Y[j];
            xdy += X[i] * D[3 * i + j] * Y[j];
            ydx += Y[i] * D[3 * i + j] * X[j];
        }
    *Fp = xdx - ydy;
    *Fx = xdy + ydx;
}

/* x . n_hat / c with n_hat = (cos dec cos h, cos dec sin h, sin dec), h = ra - gmst. */
double orc_delay(const double *x, double ra, double dec, double gmst)
{
    double h = ra - gmst;
    double n[3] = {cos(dec) * cos(h), cos(dec) * sin(h), sin(dec)};
    return (x[0] * n[0] + x[1] * n[1] + x[2] * n[2]) / ORC_C_SI;
}

/* ---------------------------------------------------------------- harmonics */

static double orc_fact(int n)
{
    double r = 1.0;
    for (int i = 2; i <= n; i++) r *= i;
    return r;
}

/* Wigner small-d d^l_{mp,m}(beta), explicit factorial sum. */
double orc_wigner_d(int l, int mp, int m, double beta)
{
    double cb = cos(0.5 * beta), sb = sin(0.5 * beta);
    double pref = sqrt(orc_fact(l + mp) * orc_fact(l - mp) * orc_fact(l + m) * orc_fact(l - m));
    int kmin = (m - mp > 0) ? m - mp : 0;
    int kmax = (l + m < l - mp) ? l + m : l - mp;
    double sum = 0.0;
    for (int k = kmin; k <= kmax; k++) {
        int sgn_exp = k - m + mp;
        double sgn = (sgn_exp % 2 == 0) ? 1.0 : -1.0;
        double den = orc_fact(l + m - k) * orc_fact(k) * orc_fact(l - k - mp) * orc_fact(k - m + mp);
        sum += sgn * pow(cb, 2 * l - 2 * k + m - mp) * pow(sb, 2 * k - m + mp) / den;
    }
    return pref * sum;
}

/* Spin-weight -2 harmonic -2Y_lm(theta, phi) = sqrt((2l+1)/4pi) d^l_{m,2}(theta) e^{i m phi}. */
double complex orc_sylm(int l, int m, double theta, double phi)
{
    double norm = sqrt((2.0 * l + 1.0) / (4.0 * ORC_PI));
    return norm * orc_wigner_d(l, m, 2, theta) * cexp(I * (double)m * phi);
}

/* ------------------------------------------------------------ interpolation */

/* Lagrange cubic weights on nodes {-1,0,1,2} at fractional position f. */
void orc_lagrange4(double f, double w[4])
{
    const double x[4] = {-1.0, 0.0, 1.0, 2.0};
    for (int i = 0; i < 4; i++) {
        double p = 1.0;
        for (int j = 0; j < 4; j++)
            if (j != i) p *= (f - x[j]) / (x[i] - x[j]);
        w[i] = p;
    }
}

/* ---------------------------------------------------------------- likelihood */

static double complex orc_Q(const orc_problem *P, int k, int a, int i)
{
    const double *q = P->Q + 2 * (((size_t)k * P->n_modes + a) * P->n_time + i);
    return q[0] + I * q[1];
}
static double complex orc_U(const orc_problem *P, int k, int a, int b)
{
    const double *u = P->U + 2 * (((size_t)k * P->n_modes + a) * P->n_modes + b);
    return u[0] + I * u[1];
}
static double complex orc_V(const orc_problem *P, int k, int a, int b)
{
    if (!P->V) return 0.0;
    const double *v = P->V + 2 * (((size_t)k * P->n_modes + a) * P->n_modes + b);
    return v[0] + I * v[1];
}

/* eq. (def:lnL:Decomposed) given the per-detector Q values already evaluated at tau_k.
 * Full double loops over mode pairs; no use of the U/V symmetries. */
static void orc_lnL_core(const orc_problem *P, const double th[7], const double complex *Qhat,
                         double *lnL, double *T1o, double *T2o)
{
    double ra = th[0], dec = th[1], D = th[3], ci = th[4], phi = th[5], psi = th[6];
    int K = P->n_det, n = P->n_modes;
    double iota = acos(ci);
    double complex Y[32];
    for (int a = 0; a < n; a++) Y[a] = orc_sylm(P->mode_l[a], P->mode_m[a], iota, -phi);
    double T1 = 0.0, T2 = 0.0;
    for (int k = 0; k < K; k++) {
        double Fp, Fx;
        orc_antenna(P->det_resp + 9 * k, ra, dec, psi, P->gmst, &Fp, &Fx);
        double complex F = Fp + I * Fx;
        double complex t1 = 0.0;
        for (int a = 0; a < n; a++) t1 += conj(F * Y[a]) * Qhat[k * n + a];
        T1 += creal(t1);
        double complex uk = 0.0, vk = 0.0;
        for (int a = 0; a < n; a++)
            for (int b = 0; b < n; b++) {
                uk += conj(Y[a]) * Y[b] * orc_U(P, k, a, b);
                vk += Y[a] * Y[b] * orc_V(P, k, a, b);
            }
        T2 += creal(conj(F) * F) * creal(uk) + creal(F * F * vk);
    }
    double s = P->d_ref / D;
    *lnL = s * T1 - s * s * T2 / 4.0;
    if (T1o) *T1o = T1;
    if (T2o) *T2o = T2;
}

/* Detector times tau_k for one sample. */
void orc_sample_tau(const orc_problem *P, const double th[7], double *tau)
{
    for (int k = 0; k < P->n_det; k++)
        tau[k] = th[2] - orc_delay(P->det_pos + 3 * k, th[0], th[1], P->gmst);
}

/* One sample with caller-supplied Q values at tau_k (Qhat[k][a], complex). */
void orc_lnL_qhat(const orc_problem *P, const double th[7], const double *Qhat_ri,
                  double *lnL, double *T1, double *T2)
{
    double complex Qh[8 * 32];
    int N = P->n_det * P->n_modes;
    for (int j = 0; j < N; j++) Qh[j] = Qhat_ri[2 * j] + I * Qhat_ri[2 * j + 1];
    orc_lnL_core(P, th, Qh, lnL, T1, T2);
}

/* One sample: Q interpolated from the window (Lagrange cubic). */
static void orc_lnL_one(const orc_problem *P, const double th[7], double *lnL, double *T1, double *T2)
{
    int K = P->n_det, n = P->n_modes;
    if (!(th[3] > 0.0) || !(fabs(th[4]) <= 1.0)) {
        *lnL = -INFINITY; *T1 = NAN; *T2 = NAN;
        return;
    }
    double complex Qh[8 * 32];
    for (int k = 0; k < K; k++) {
        double tau = th[2] - orc_delay(P->det_pos + 3 * k, th[0], th[1], P->gmst);
        double u = (tau - P->tau0) / P->dt;
        double fl = floor(u);
        if (!(fl >= 1.0 && fl <= (double)(P->n_time - 3))) {
            *lnL = -INFINITY; *T1 = NAN; *T2 = NAN;
            return;
        }
        int i = (int)fl;
        double w[4];
        orc_lagrange4(u - fl, w);
        for (int a = 0; a < n; a++) {
            double complex q = 0.0;
            for (int j = 0; j < 4; j++) q += w[j] * orc_Q(P, k, a, i - 1 + j);
            Qh[k * n + a] = q;
        }
    }
    orc_lnL_core(P, th, Qh, lnL, T1, T2);
}

/* Many samples: theta is SoA [7][ld]; outputs may be NULL except lnL. */
void orc_lnL(const orc_problem *P, int64_t n, const double *theta, int64_t ld,
             double *lnL, double *T1, double *T2, int nthreads)
{
    (void)nthreads;
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t i = 0; i < n; i++) {
        double th[7];
        for (int c = 0; c < 7; c++) th[c] = theta[c * ld + i];
        double l, t1, t2;
        orc_lnL_one(P, th, &l, &t1, &t2);
        lnL[i] = l;
        if (T1) T1[i] = t1;
        if (T2) T2[i] = t2;
    }
}

/* ------------------------------------------------------------- marginalise */

typedef struct {
    double ln_L, ln_sigma, n_eff, n_ess, max_lw;
    int64_t argmax, n, n_nonfinite;
} orc_marg;

/* eq. (lnL:MonteCarlo) on the given log-weights, with eq. (neff):
 * m = max lw, S1 = sum e^{lw-m}, S2 = sum e^{2(lw-m)};
 * ln L = m + ln S1 - ln N;  n_eff = S1;  n_ESS = S1^2/S2;
 * sigma/L = sqrt((N S2/S1^2 - 1)/(N-1)).
 * Non-finite lw (-inf or NaN) carry zero weight and are counted. */
void orc_marginalize(int64_t n, const double *lw, orc_marg *out)
{
    double m = -INFINITY;
    int64_t am = -1, bad = 0;
    for (int64_t i = 0; i < n; i++) {
        if (!isfinite(lw[i])) { bad++; continue; }
        if (lw[i] > m) { m = lw[i]; am = i; }
    }
    out->n = n;
    out->n_nonfinite = bad;
    out->argmax = am;
    out->max_lw = m;
    if (am < 0) {
        out->ln_L = -INFINITY; out->ln_sigma = -INFINITY; out->n_eff = 0.0; out->n_ess = 0.0;
        return;
    }
    long double s1 = 0.0L, s2 = 0.0L;
    for (int64_t i = 0; i < n; i++) {
        if (!isfinite(lw[i])) continue;
        long double e = expl((long double)lw[i] - (long double)m);
        s1 += e;
        s2 += e * e;
    }
    out->ln_L = m + (double)logl(s1) - log((double)n);
    out->n_eff = (double)s1;
    out->n_ess = (double)(s1 * s1 / s2);
    if (n > 1) {
        long double v = ((long double)n * s2 / (s1 * s1) - 1.0L) / (long double)(n - 1);
        out->ln_sigma = out->ln_L + 0.5 * (double)logl(v > 0 ? v : 0.0L);
    } else {
        out->ln_sigma = -INFINITY;
    }
}

/* ------------------------------------------------------------------ Philox */

/* Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of
 * (hi,lo) = M * x products with Weyl key schedule. */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; r++) {
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------ sample draws */
/*
 * Counter layout shared by definition with the device generator (each side
 * has its own implementation of the same published Philox-4x32-10):
 *   key = (seed lo, seed hi);
 *   sample i of round r, attempt a, block b:  ctr = (i lo, i hi, r, a*16 + b);
 *   in-box mass draw i of component j, round r, block b:
 *       ctr = (i, 0x5A000000 + j, r, b).
 * A uniform in (0,1) takes two words (w0, w1):
 *   u = ((w0 >> 5) * 2^26 + (w1 >> 6) + 0.5) * 2^-53.
 */

typedef struct {
    double t_window, d_min, d_max;   /* prior support; alpha,phi in [0,2pi), psi in [0,pi) */
    int dist_marg;                   /* 1: distance not sampled (theta[3] = d_ref) */
    double d_ref;
} orc_prior;

static double orc_u53(uint32_t w0, uint32_t w1)
{
    return ((double)(w0 >> 5) * 67108864.0 + (double)(w1 >> 6) + 0.5) * (1.0 / 9007199254740992.0);
}

static void orc_words(uint64_t seed, uint64_t i, uint32_t r, uint32_t a, int nblocks, uint32_t *w)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int b = 0; b < nblocks; b++) {
        uint32_t ctr[4] = {(uint32_t)i, (uint32_t)(i >> 32), r, a * 16u + (uint32_t)b};
        orc_philox4x32_10(ctr, key, w + 4 * b);
    }
}

/* Prior in the sampled coordinates:
 *   alpha ~ U[0,2pi), p(dec) = cos(dec)/2, t ~ U[-tw,tw], p(D) = 3D^2/(Dmax^3-Dmin^3),
 *   cos(iota) ~ U[-1,1], phi_c ~ U[0,2pi), psi ~ U[0,pi). */
double orc_ln_prior(const orc_prior *pr, const double th[7])
{
    double lp = -log(2.0 * ORC_PI) + log(0.5 * cos(th[1])) - log(2.0 * pr->t_window)
              - log(2.0) - log(2.0 * ORC_PI) - log(ORC_PI);
    if (!pr->dist_marg)
        lp += log(3.0 * th[3] * th[3] / (pow(pr->d_max, 3) - pow(pr->d_min, 3)));
    return lp;
}

/* Inverse-CDF map of seven uniforms onto the prior. */
static void orc_prior_from_u(const orc_prior *pr, const double u[7], double th[7])
{
    th[0] = 2.0 * ORC_PI * u[0];
    th[1] = asin(2.0 * u[1] - 1.0);
    th[2] = -pr->t_window + 2.0 * pr->t_window * u[2];
    if (pr->dist_marg) {
        th[3] = pr->d_ref;
    } else {
        double a3 = pow(pr->d_min, 3), b3 = pow(pr->d_max, 3);
        th[3] = cbrt(a3 + u[3] * (b3 - a3));
    }
    th[4] = 2.0 * u[4] - 1.0;
    th[5] = 2.0 * ORC_PI * u[5];
    th[6] = ORC_PI * u[6];
}

void orc_draw_prior(const orc_prior *pr, uint64_t seed, uint32_t round, int64_t i0, int64_t n,
                    double *theta, int64_t ld, double *ln_p)
{
    for (int64_t s = 0; s < n; s++) {
        uint32_t w[16];
        orc_words(seed, (uint64_t)(i0 + s), round, 0, 4, w);
        double u[7], th[7];
        for (int c = 0; c < 7; c++) u[c] = orc_u53(w[2 * c], w[2 * c + 1]);
        orc_prior_from_u(pr, u, th);
        for (int c = 0; c < 7; c++) theta[c * ld + s] = th[c];
        if (ln_p) ln_p[s] = orc_ln_prior(pr, th);
    }
}

/* ------------------------------------------------- adaptive-volume draws */
/*
 * Adaptive volume integration (Section "Adaptive volume integration"): the
 * sampler is uniform over a set of active hypercubes of the unit cube of the
 * prior's CDF coordinates u (theta = inverse-CDF map of u, as for the prior
 * draw), so p(theta)/p_s(theta) = V, the active volume.
 * Grid: nb bins per dimension over the n_dim sampled columns dims[]; cells
 * [n_cells][n_dim] integer coordinates.  Sample i of round r uses the words of
 * the prior draw (attempt 0, blocks 0..3): the cell is the floor of
 * u53(w14, w15) * n_cells (at most n_cells - 1), and column c of the cell's
 * k-th dimension takes u_c = (cell_k + u53(w[2c], w[2c+1])) / nb.  With one
 * cell and nb = 1 this is the prior draw itself.  u_out: [n_dim][n] or NULL.
 */
void orc_draw_av(const orc_prior *pr, int n_dim, const int *dims, int nb, int64_t n_cells, const int32_t *cells,
                 uint64_t seed, uint32_t round, int64_t i0, int64_t n, double *theta, int64_t ld, double *u_out)
{
    for (int64_t s = 0; s < n; s++) {
        uint32_t w[16];
        orc_words(seed, (uint64_t)(i0 + s), round, 0, 4, w);
        double sel = floor(orc_u53(w[14], w[15]) * (double)n_cells);
        int64_t j = (int64_t)sel;
        if (j > n_cells - 1) j = n_cells - 1;
        double u[7], th[7];
        for (int c = 0; c < 7; c++) u[c] = orc_u53(w[2 * c], w[2 * c + 1]);
        for (int k = 0; k < n_dim; k++) {
            int c = dims[k];
            u[c] = ((double)cells[j * n_dim + k] + orc_u53(w[2 * c], w[2 * c + 1])) / (double)nb;
            if (u_out) u_out[(int64_t)k * n + s] = u[c];
        }
        orc_prior_from_u(pr, u, th);
        for (int c = 0; c < 7; c++) theta[c * ld + s] = th[c];
    }
}

/* ------------------------------------------- adaptive Cartesian draws */
/*
 * Product-form adaptive Cartesian (AC) sampling prior (the sampler with one
 * adaptive one-dimensional marginal per coordinate, Section "Evaluating the
 * marginalized likelihood"), in the prior's CDF coordinates: each sampled
 * column k has nb equal bins with probabilities pi[k][b] and cumulative sums
 * cum[k][b] (cum[k][nb-1] = 1).  Sample i of round r uses the prior draw's
 * words; column c's uniform U = u53(w[2c], w[2c+1]) selects the first bin b
 * with cum > U and x = (b + (U - cum[b-1]) / pi[b]) / nb (the inverse CDF of
 * the piecewise-constant density).  ln p - ln p_s = -sum_k ln(nb pi[k][b_k]),
 * with lnbp[k][b] = ln(nb pi[k][b]) given.  bins_out: [n_dim][n] or NULL.
 */
void orc_draw_ac(const orc_prior *pr, int n_dim, const int *dims, int nb, const double *pi, const double *cum,
                 const double *lnbp, uint64_t seed, uint32_t round, int64_t i0, int64_t n, double *theta,
                 int64_t ld, double *lnpmps, int32_t *bins_out)
{
    for (int64_t s = 0; s < n; s++) {
        uint32_t w[16];
        orc_words(seed, (uint64_t)(i0 + s), round, 0, 4, w);
        double u[7], th[7], lr = 0.0;
        for (int c = 0; c < 7; c++) u[c] = orc_u53(w[2 * c], w[2 * c + 1]);
        for (int k = 0; k < n_dim; k++) {
            const int c = dims[k];
            const double U = u[c];
            int b = 0;
            while (b < nb - 1 && !(cum[k * nb + b] > U)) b++;
            const double lo = b > 0 ? cum[k * nb + b - 1] : 0.0;
            u[c] = ((double)b + (U - lo) / pi[k * nb + b]) / (double)nb;
            lr -= lnbp[k * nb + b];
            if (bins_out) bins_out[(int64_t)k * n + s] = b;
        }
        orc_prior_from_u(pr, u, th);
        for (int c = 0; c < 7; c++) theta[c * ld + s] = th[c];
        if (lnpmps) lnpmps[s] = lr;
    }
}

/* ---------------------------------------------------------- Gaussian mixture */

#define ORC_GMM_MAXC 16
#define ORC_GMM_MAXD 7
typedef struct {
    int n_comp, n_dim;
    int dims[ORC_GMM_MAXD];              /* theta column of each GMM dimension */
    double weight[ORC_GMM_MAXC];         /* pi_j */
    double mean[ORC_GMM_MAXC][ORC_GMM_MAXD];
    double cov[ORC_GMM_MAXC][ORC_GMM_MAXD][ORC_GMM_MAXD];
    double ln_Z[ORC_GMM_MAXC];           /* in-support mass of each component */
    double eps_def;                      /* defensive prior weight */
    int shear;                           /* 0, or +-1: the mixture's psi column is
                                            (psi + shear phi_c) mod pi */
} orc_gmm;

/* Mixture coordinates of a sample.  With shear s = +-1 (columns 5 and 6 both
 * in the mixture) column 6 becomes y = (psi + s phi_c) mod pi.  The map is a
 * shear of the (phi_c, psi) torus onto itself with unit Jacobian, so a
 * density in (phi_c, y) is the same density in (phi_c, psi).  For a source
 * seen face-on the likelihood depends on phi_c and psi nearly only through
 * psi + phi_c (face-off: psi - phi_c), so its ridge runs along phi_c at fixed y. */
static void orc_gmm_coords(const orc_gmm *g, const double th[7], double x[7])
{
    for (int c = 0; c < 7; c++) x[c] = th[c];
    if (g->shear) {
        double y = th[6] + g->shear * th[5];
        x[6] = y - ORC_PI * floor(y / ORC_PI);
    }
}

/* Support of a theta column: periodic (period > 0) or bounded [lo, hi]. */
static void orc_col_support(const orc_prior *pr, int col, double *lo, double *hi, double *period)
{
    *period = 0.0;
    switch (col) {
    case 0: *lo = 0; *hi = 2 * ORC_PI; *period = 2 * ORC_PI; break;
    case 1: *lo = -ORC_PI / 2; *hi = ORC_PI / 2; break;
    case 2: *lo = -pr->t_window; *hi = pr->t_window; break;
    case 3: *lo = pr->d_min; *hi = pr->d_max; break;
    case 4: *lo = -1; *hi = 1; break;
    case 5: *lo = 0; *hi = 2 * ORC_PI; *period = 2 * ORC_PI; break;
    default: *lo = 0; *hi = ORC_PI; *period = ORC_PI; break;
    }
}

/* Difference wrapped into (-P/2, P/2]. */
static double orc_wrap_diff(double d, double period)
{
    if (period <= 0) return d;
    double r = d - period * floor(d / period);      /* [0, P) */
    if (r > 0.5 * period) r -= period;
    return r;
}

/* Textbook Cholesky, lower triangular; returns 0 on failure. */
static int orc_cholesky(int n, double A[ORC_GMM_MAXD][ORC_GMM_MAXD], double L[ORC_GMM_MAXD][ORC_GMM_MAXD])
{
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) L[i][j] = 0.0;
    for (int j = 0; j < n; j++) {
        double s = A[j][j];
        for (int k = 0; k < j; k++) s -= L[j][k] * L[j][k];
        if (!(s > 0)) return 0;
        L[j][j] = sqrt(s);
        for (int i = j + 1; i < n; i++) {
            double t = A[i][j];
            for (int k = 0; k < j; k++) t -= L[i][k] * L[j][k];
            L[i][j] = t / L[j][j];
        }
    }
    return 1;
}

/* ln N(wrap(x - mu_j); 0, Sigma_j) for one component. */
double orc_gmm_comp_logpdf(const orc_prior *pr, const orc_gmm *g, int j, const double th[7])
{
    int d = g->n_dim;
    double L[ORC_GMM_MAXD][ORC_GMM_MAXD], S[ORC_GMM_MAXD][ORC_GMM_MAXD];
    for (int a = 0; a < d; a++)
        for (int b = 0; b < d; b++) S[a][b] = g->cov[j][a][b];
    if (!orc_cholesky(d, S, L)) return NAN;
    double diff[ORC_GMM_MAXD], y[ORC_GMM_MAXD], x[7];
    orc_gmm_coords(g, th, x);
    for (int a = 0; a < d; a++) {
        double lo, hi, P;
        orc_col_support(pr, g->dims[a], &lo, &hi, &P);
        diff[a] = orc_wrap_diff(x[g->dims[a]] - g->mean[j][a], P);
    }
    double q = 0.0, ld = 0.0;
    for (int a = 0; a < d; a++) {
        double t = diff[a];
        for (int b = 0; b < a; b++) t -= L[a][b] * y[b];
        y[a] = t / L[a][a];
        q += y[a] * y[a];
        ld += log(L[a][a]);
    }
    return -0.5 * q - ld - 0.5 * d * log(2.0 * ORC_PI);
}

/* Prior density of one column (the prior is a product over columns). */
static double orc_ln_prior_col(const orc_prior *pr, int c, const double th[7])
{
    switch (c) {
    case 0: return -log(2.0 * ORC_PI);
    case 1: return log(0.5 * cos(th[1]));
    case 2: return -log(2.0 * pr->t_window);
    case 3: return pr->dist_marg ? 0.0 : log(3.0 * th[3] * th[3] / (pow(pr->d_max, 3) - pow(pr->d_min, 3)));
    case 4: return -log(2.0);
    case 5: return -log(2.0 * ORC_PI);
    default: return -log(ORC_PI);
    }
}

/* Density of one draw of orc_draw_gmm below.  The selector picks the prior
 * with probability eps, else component j with probability
 * pi_j = weight_j / sum weight.  A component then makes up to `attempts`
 * independent candidates; the first accepted one has density N_j(x)/Z_j on
 * the mixture columns (Z_j its acceptance probability), and if all fail
 * (probability r_j = (1 - Z_j)^attempts) the independent prior draw is kept.
 * Columns outside the mixture always come from the prior draw.  So
 *   p_s(x) = eps p(x) + (1-eps) sum_j pi_j [ (1 - r_j) N_j(x) p_rest(x) / Z_j
 *                                            + r_j p(x) ],
 * p_rest the prior of the columns outside the mixture.  attempts <= 0 stands
 * for unlimited attempts (r_j = 0). */
double orc_gmm_ln_ps_n(const orc_prior *pr, const orc_gmm *g, const double th[7], int attempts)
{
    double lp = orc_ln_prior(pr, th);
    double lrest = 0.0;
    for (int c = 0; c < 7; c++) {
        int in = 0;
        for (int a = 0; a < g->n_dim; a++) in |= (g->dims[a] == c);
        if (!in) lrest += orc_ln_prior_col(pr, c, th);
    }
    double tot = 0.0;
    for (int j = 0; j < g->n_comp; j++)
        if (g->weight[j] > 0) tot += g->weight[j];
    double terms[ORC_GMM_MAXC + 1];
    int nt = 0;
    double fallback = g->eps_def;
    for (int j = 0; j < g->n_comp; j++) {
        if (!(g->weight[j] > 0)) continue;
        double pi = g->weight[j] / tot;
        double Z = exp(g->ln_Z[j]);
        double r = attempts > 0 ? pow(1.0 - (Z < 1.0 ? Z : 1.0), attempts) : 0.0;
        fallback += (1.0 - g->eps_def) * pi * r;
        terms[nt++] = log((1.0 - g->eps_def) * pi * (1.0 - r)) + orc_gmm_comp_logpdf(pr, g, j, th)
                      + lrest - g->ln_Z[j];
    }
    if (fallback > 0) terms[nt++] = log(fallback) + lp;
    double m = -INFINITY;
    for (int t = 0; t < nt; t++) if (terms[t] > m) m = terms[t];
    if (!isfinite(m)) return m;
    double s = 0.0;
    for (int t = 0; t < nt; t++) s += exp(terms[t] - m);
    return m + log(s);
}

/* Proposal draw of one candidate from component j at attempt a: x = mu + L z,
 * z from Box-Muller pairs.  Returns 1 if accepted (every bounded coordinate in
 * its interval, every periodic offset within half a period). */
static int orc_gmm_candidate(const orc_prior *pr, const orc_gmm *g, int j,
                             double L[ORC_GMM_MAXD][ORC_GMM_MAXD], const uint32_t *w, double th[7])
{
    int d = g->n_dim;
    double z[8];
    for (int p = 0; p < 4; p++) {
        double u1 = orc_u53(w[4 * p + 0], w[4 * p + 1]);
        double u2 = orc_u53(w[4 * p + 2], w[4 * p + 3]);
        double r = sqrt(-2.0 * log(u1));
        z[2 * p] = r * cos(2.0 * ORC_PI * u2);
        z[2 * p + 1] = r * sin(2.0 * ORC_PI * u2);
    }
    for (int a = 0; a < d; a++) {
        double off = 0.0;
        for (int b = 0; b <= a; b++) off += L[a][b] * z[b];
        double lo, hi, P;
        orc_col_support(pr, g->dims[a], &lo, &hi, &P);
        double x = g->mean[j][a] + off;
        if (P > 0) {
            if (!(off > -0.5 * P && off <= 0.5 * P)) return 0;
            x = x - P * floor((x - lo) / P);
        } else if (!(x >= lo && x <= hi)) {
            return 0;
        }
        th[g->dims[a]] = x;
    }
    return 1;
}

#define ORC_GMM_MAX_ATTEMPTS 64

/* ln p_s of the draws below (64 attempts per component). */
double orc_gmm_ln_ps(const orc_prior *pr, const orc_gmm *g, const double th[7])
{
    return orc_gmm_ln_ps_n(pr, g, th, ORC_GMM_MAX_ATTEMPTS);
}

/* Draw from p_s: block 0 of attempt 0 selects prior (u < eps) or a component
 * by cumulative weight; a component is then sampled by rejection, attempt
 * a = 1..64 using blocks 1..4 of attempt a.  Columns outside the GMM come from
 * the prior draw of attempt 0 (blocks 1..4), whose words no candidate uses.
 * If no attempt is accepted the prior draw is used.  Returns ln p - ln p_s
 * per sample. */
void orc_draw_gmm(const orc_prior *pr, const orc_gmm *g, uint64_t seed, uint32_t round,
                  int64_t i0, int64_t n, double *theta, int64_t ld, double *lnpmps)
{
    double L[ORC_GMM_MAXC][ORC_GMM_MAXD][ORC_GMM_MAXD];
    for (int j = 0; j < g->n_comp; j++) {
        double S[ORC_GMM_MAXD][ORC_GMM_MAXD];
        for (int a = 0; a < g->n_dim; a++)
            for (int b = 0; b < g->n_dim; b++) S[a][b] = g->cov[j][a][b];
        orc_cholesky(g->n_dim, S, L[j]);
    }
    for (int64_t s = 0; s < n; s++) {
        uint64_t idx = (uint64_t)(i0 + s);
        uint32_t w[20];
        orc_words(seed, idx, round, 0, 5, w);
        double u[7], th[7];
        for (int c = 0; c < 7; c++) u[c] = orc_u53(w[4 + 2 * c], w[4 + 2 * c + 1]);
        orc_prior_from_u(pr, u, th);
        double usel = orc_u53(w[0], w[1]);
        if (usel >= g->eps_def) {
            double v = (usel - g->eps_def) / (1.0 - g->eps_def);
            double tot = 0.0;
            for (int j = 0; j < g->n_comp; j++) tot += g->weight[j];
            int jsel = -1;
            double acc = 0.0;
            for (int j = 0; j < g->n_comp; j++) {
                if (!(g->weight[j] > 0)) continue;
                acc += g->weight[j] / tot;
                jsel = j;
                if (v < acc) break;
            }
            for (int a = 1; a <= ORC_GMM_MAX_ATTEMPTS && jsel >= 0; a++) {
                uint32_t wa[20];
                orc_words(seed, idx, round, (uint32_t)a, 5, wa);
                double cand[7];
                memcpy(cand, th, sizeof cand);
                if (orc_gmm_candidate(pr, g, jsel, L[jsel], wa + 4, cand)) {
                    memcpy(th, cand, sizeof cand);
                    if (g->shear) {    /* back from (phi_c, y) to (phi_c, psi) */
                        double p = cand[6] - g->shear * cand[5];
                        th[6] = p - ORC_PI * floor(p / ORC_PI);
                    }
                    break;
                }
            }
        }
        for (int c = 0; c < 7; c++) theta[c * ld + s] = th[c];
        if (lnpmps) lnpmps[s] = orc_ln_prior(pr, th) - orc_gmm_ln_ps(pr, g, th);
    }
}

/* ln p_s (64 attempts) of n samples [7][ld]. */
void orc_gmm_ln_ps_batch(const orc_prior *pr, const orc_gmm *g, int64_t n, const double *theta, int64_t ld,
                         double *out)
{
    for (int64_t i = 0; i < n; i++) {
        double th[7];
        for (int c = 0; c < 7; c++) th[c] = theta[c * ld + i];
        out[i] = orc_gmm_ln_ps(pr, g, th);
    }
}

/* In-support mass of component j from m Philox candidates (block b = 0..3 of
 * counter (i, 0x5A000000 + j, round, b)). */
double orc_gmm_inbox_mass(const orc_prior *pr, const orc_gmm *g, int j, uint64_t seed,
                          uint32_t round, int64_t m)
{
    double S[ORC_GMM_MAXD][ORC_GMM_MAXD], L[ORC_GMM_MAXD][ORC_GMM_MAXD];
    for (int a = 0; a < g->n_dim; a++)
        for (int b = 0; b < g->n_dim; b++) S[a][b] = g->cov[j][a][b];
    orc_cholesky(g->n_dim, S, L);
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    int64_t acc = 0;
    for (int64_t i = 0; i < m; i++) {
        uint32_t w[16];
        for (int b = 0; b < 4; b++) {
            uint32_t ctr[4] = {(uint32_t)i, 0x5A000000u + (uint32_t)j, round, (uint32_t)b};
            orc_philox4x32_10(ctr, key, w + 4 * b);
        }
        double th[7] = {0, 0, 0, pr->d_ref, 0, 0, 0};
        acc += orc_gmm_candidate(pr, g, j, L, w, th);
    }
    return (double)acc / (double)m;
}
