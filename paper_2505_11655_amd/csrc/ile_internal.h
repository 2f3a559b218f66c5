// Internal declarations of the gfx950 ILE library: compile-time mode sets and
// pair tables, device-side job descriptors, the counter-based generator, and
// the launch entry points shared between the C ABI and the serving loop.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace ile {

// ------------------------------------------------------------------ policies
enum Policy : int { kFP64 = 0, kFP32 = 1, kMixed = 2 };

// Threads per block of the LDS-staged likelihood kernel: one window per CU,
// as many waves as the register use of the mode set (index 0..3, 5/9/17/21
// modes) and policy allows without spilling: 1024 (128 VGPRs) for FP32 and
// FP32 + FP64 cancellation with up to 9 modes, 256 for the 21-mode set (its
// window leaves room for one block per CU anyway) and for FP64 with 17 modes,
// 512 otherwise.
constexpr int lds_block_threads(int set, int policy) {
    return ((policy == kFP32 || policy == kMixed) && set <= 1) ? 1024
           : (set >= 3 || (set == 2 && policy == kFP64))       ? 256
                                                               : 512;
}
// Threads per block of the time-marginalised kernel (its per-sample state is
// larger than the pointwise kernel's: two waves per SIMD in FP32, one in FP64).
constexpr int tmarg_block_threads(int policy) { return policy == kFP32 ? 512 : 256; }

// ----------------------------------------------------------------- mode sets
// Compiled harmonic sets.  A job's mode list is placed into the smallest set
// that contains it (absent slots get zero Q, U and V).
constexpr int kMaxModes = 21;
constexpr int kNumSets = 4;
struct ModeList {
    int n;
    int l[kMaxModes];
    int m[kMaxModes];
};
constexpr ModeList kSets[kNumSets] = {
    {5, {2, 2, 2, 2, 2}, {-2, -1, 0, 1, 2}},
    {9, {2, 2, 2, 2, 2, 3, 3, 3, 3}, {-2, -1, 0, 1, 2, -3, -2, 2, 3}},
    {17, {2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 4, 4, 4, 4, 4, 4},
     {-2, -1, 0, 1, 2, -3, -2, -1, 1, 2, 3, -4, -3, -2, 2, 3, 4}},
    {21, {2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 3, 4, 4, 4, 4, 4, 4, 4, 4, 4},
     {-2, -1, 0, 1, 2, -3, -2, -1, 0, 1, 2, 3, -4, -3, -2, -1, 0, 1, 2, 3, 4}},
};

// Detectors whose Q window an LDS-staged likelihood kernel reads through
// L1/L2 instead of LDS: the fewest that bring the staged part of the compiled
// 410-sample windows within 160 KiB (kp: compiled detector count; kp when not
// even one detector fits).
// The FP32 + FP64-cancellation policy stages FP32 windows and, for every
// detector, its FP64 reference series (410 doubles).
constexpr int lds_global_dets(int set, int kp, int policy) {
    const long per = 410L * kSets[set].n * 2 * (policy == kFP64 ? 8 : 4);
    const long fixed = policy == kMixed ? 410L * 8 * kp : 0;
    for (int g = 0; g < kp; g++)
        if ((kp - g) * per + fixed <= 163840L) return g;
    return kp;
}
// The time-marginalised kernel always reads at least the first detector
// through L1/L2 (its per-lane row reads exceed the LDS bandwidth otherwise).
constexpr int tmarg_global_dets(int set, int kp, int policy) {
    const int g = lds_global_dets(set, kp, policy);
    return g > 1 ? g : 1;
}
// Whether an LDS-staged variant is compiled: for the pointwise kernel wherever
// one detector's window fits; for the time-marginalised kernel only up to the
// 9-mode set in FP64 (beyond it the staged variant runs out of scalar
// registers and gains nothing over L1/L2).
constexpr bool lnl_lds_compiled(int set, int kp, int policy) { return lds_global_dets(set, kp, policy) < kp; }
constexpr bool tmarg_lds_compiled(int set, int kp, int policy) {
    return tmarg_global_dets(set, kp, policy) < kp && (set <= 1 || policy == kFP32);
}

constexpr int set_lmax(int s) {
    int L = 0;
    for (int a = 0; a < kSets[s].n; a++) L = kSets[s].l[a] > L ? kSets[s].l[a] : L;
    return L;
}
constexpr int iabs_c(int x) { return x < 0 ? -x : x; }

// Pairs a <= b of a set, ordered two ways:
//  U-order: grouped by |m_a - m_b| (0..2 lmax), group g = [u_start[g], u_start[g+1]);
//  V-order: grouped by m_a + m_b (-2 lmax..2 lmax), group g = s + 2 lmax.
constexpr int kMaxPairs = kMaxModes * (kMaxModes + 1) / 2;
struct PairTable {
    int P;
    int lmax;
    int a[kMaxPairs], b[kMaxPairs];
    int u_pair[kMaxPairs];
    int u_start[10];
    int v_pair[kMaxPairs];
    int v_start[18];
};

constexpr PairTable make_pairs(int s) {
    PairTable t{};
    const ModeList &ml = kSets[s];
    t.lmax = set_lmax(s);
    int P = 0;
    for (int a = 0; a < ml.n; a++)
        for (int b = a; b < ml.n; b++) {
            t.a[P] = a;
            t.b[P] = b;
            P++;
        }
    t.P = P;
    int ng = 2 * t.lmax + 1;
    int k = 0;
    for (int g = 0; g < ng; g++) {
        t.u_start[g] = k;
        for (int p = 0; p < P; p++)
            if (iabs_c(ml.m[t.a[p]] - ml.m[t.b[p]]) == g) t.u_pair[k++] = p;
    }
    t.u_start[ng] = k;
    int nv = 4 * t.lmax + 1;
    k = 0;
    for (int g = 0; g < nv; g++) {
        t.v_start[g] = k;
        for (int p = 0; p < P; p++)
            if (ml.m[t.a[p]] + ml.m[t.b[p]] + 2 * t.lmax == g) t.v_pair[k++] = p;
    }
    t.v_start[nv] = k;
    return t;
}

template <int S>
struct MSet {
    static constexpr int id = S;
    static constexpr int n = kSets[S].n;
    static constexpr int lmax = set_lmax(S);
    static constexpr PairTable pt = make_pairs(S);
    static constexpr int P = pt.P;
};

// ------------------------------------------------- -2Y_lm(iota,.) amplitudes
// -2Y_lm(iota, -phi) = y_lm(iota) e^{-i m phi} with
// y_lm = sqrt((2l+1)/4pi) d^l_{m,2}(iota), and d^l_{m,2} a sum of monomials
// c^p s^q in c = cos(iota/2), s = sin(iota/2) (Wigner's explicit formula).
constexpr double cx_fact(int n) {
    double r = 1.0;
    for (int i = 2; i <= n; i++) r *= i;
    return r;
}
constexpr double cx_sqrt(double x) {
    if (x <= 0) return 0.0;
    double g = x > 1 ? x : 1.0;
    for (int i = 0; i < 200; i++) g = 0.5 * (g + x / g);
    return g;
}
constexpr double kPiC = 3.14159265358979323846;
struct WTerm {
    int nt;
    double coef[5];
    int p[5], q[5];
};
constexpr WTerm wigner_terms(int l, int m) {
    WTerm w{};
    int kmin = (2 - m) > 0 ? 2 - m : 0;
    int kmax = (l + 2) < (l - m) ? (l + 2) : (l - m);
    double pref = cx_sqrt(cx_fact(l + m) * cx_fact(l - m) * cx_fact(l + 2) * cx_fact(l - 2)) *
                  cx_sqrt((2.0 * l + 1.0) / (4.0 * kPiC));
    for (int k = kmin; k <= kmax; k++) {
        int e = k - 2 + m;
        double sg = (e % 2 == 0) ? 1.0 : -1.0;
        double den = cx_fact(l + 2 - k) * cx_fact(k) * cx_fact(l - k - m) * cx_fact(k - 2 + m);
        w.coef[w.nt] = sg * pref / den;
        w.p[w.nt] = 2 * l - 2 * k + 2 - m;
        w.q[w.nt] = 2 * k - 2 + m;
        w.nt++;
    }
    return w;
}

// --------------------------------------------------------------- Philox
// Philox-4x32-10 (Salmon et al., SC'11), device implementation.
struct U4 {
    uint32_t x, y, z, w;
};
__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; r++) {
        // one 32x32->64 product per multiplier (a single v_mad_u64_u32)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        // three-input XOR in one v_bitop3_b32 (truth table 0x96: odd parity)
        const uint32_t x1 = (uint32_t)__builtin_amdgcn_bitop3_b32(hi1, c.y, k0, 0x96);
        const uint32_t x3 = (uint32_t)__builtin_amdgcn_bitop3_b32(hi0, c.w, k1, 0x96);
        U4 n{x1, lo1, x3, lo0};
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}
// Uniform in (0,1) with 53 random bits from two words.
__device__ __forceinline__ double u53(uint32_t w0, uint32_t w1) {
    return ((double)(w0 >> 5) * 67108864.0 + (double)(w1 >> 6) + 0.5) * (1.0 / 9007199254740992.0);
}

// ------------------------------------------------------------ device jobs
// Distance-marginal table geometry: nodes u_i = u0 + i du (a = asinh(u)-grid
// in T1/sqrt(T2)), b_j = b0 + j db (ln T2).
struct DistTable {
    const double *r;      // [nb][nu] residual ln L_D - a^2
    int nu, nb;
    double u0, du, b0, db;
    double s_min, s_max;  // d_ref/d_max, d_ref/d_min
    double a_scale;       // a = a_scale * sinh(u)
    double inv_du, inv_db, inv_a_scale;
};

struct EvalJob {
    const void *Q;        // [Kp][T][NM] complex, policy contraction type (FP32 in the mixed policy)
    const void *Ut;       // [P][Kp] complex, U-order, weighted; mixed policy: [Kp][NT] FP32 quadratic-form rows
    const void *Vt;       // [P][Kp] complex, V-order, weighted (unused by the mixed policy)
    // mixed policy: the reference terms (written on the device by k_ref_build)
    const float *ref_rg;  // r [Kp][NM] then G [Kp][NM], complex FP32
    const double *ref_R;  // [Kp][T] Re(r^+ Q)
    const double *ref_C0; // C0
    DistTable dt;
    double tau0, inv_dt, gmst, d_ref;
    double xc[3][3];      // detector position / c (seconds)
    double D[3][6];       // response tensor (xx, yy, zz, xy, xz, yz)
    // FP32 copies of the same constants for the FP32 parts of the policies
    float xcf[3][3];
    float Df[3][6];
    float gmstf, tau0f, inv_dtf, d_reff;
    int n_time;
    int tm_half;          // time-marginalised launches: nodes j = -tm_half..tm_half
    const void *theta;
    int64_t ld;
    const void *lnpmps;
    void *lnL;
    void *lw;
    int64_t n;            // samples of this job in the launch
    double tm_lnw;        // time-marginalised launches: ln(dt / (R 2 t_w)) per node
};

// Where the reference builder of a mixed-policy job reads and writes.
struct RefBuild {
    const double *theta_ref;  // [7]
    const double *Q64;        // [Kp][T][NM] complex FP64
    const double *U64, *V64;  // [Kp][NM][NM] complex FP64 (slot order)
    float *rg;                // -> EvalJob::ref_rg
    double *R;                // -> EvalJob::ref_R
    double *C0;               // -> EvalJob::ref_C0
};

struct Tile {
    int32_t job;
    int32_t pad_;
    int64_t begin, end;
};

// Pooled estimator state (device, FP64).
struct MargState {
    double m;        // max lw
    double s1, s2;   // sums of e^{lw-m}, e^{2(lw-m)}
    int64_t n, n_bad, argmax;
};
struct MargPartial {
    double m, s1, s2;
    int64_t n_bad, argmax;
};
// One job of a batched estimator launch: its tiles are [tile_begin, tile_end).
struct MargJob {
    const void *lw;
    int64_t n;
    int32_t tile_begin, tile_end;
    MargState *state;     // pooled state (device)
    int32_t out_idx;      // slot of the state copy in the launch's output array, or -1
    int32_t reset;
};

constexpr int kMaxComp = 16;
struct GmmDev {
    int n_comp, n_dim;
    int dims[7];
    int valid;
    int shear;                            // 0, or +-1: mixture column psi is (psi + shear phi_c) mod pi
    double eps_def;
    double w[kMaxComp];                   // pi_j
    double logw[kMaxComp];                // ln pi_j (-inf if pi_j = 0)
    double mean[kMaxComp][7];
    double cov[kMaxComp][7][7];
    double L[kMaxComp][7][7];             // Cholesky factor
    double Linv[kMaxComp][7][7];          // inverse of L (lower)
    double logdet_half[kMaxComp];         // sum ln L_dd
    double lnZ[kMaxComp];
    // density of a mixture draw (set with the in-support masses): component
    // j contributes e^{lnc_j} N_j(x) p_rest(x), the prior p(x) is weighted by
    // e^{ln_fb} (defensive draws plus components whose 64 attempts all failed)
    double lnc[kMaxComp];                 // ln[(1-eps) pi_j/sum pi (1 - (1-Z_j)^64) / Z_j]
    double ln_fb;                         // ln[eps + (1-eps) sum_j pi_j/sum pi (1-Z_j)^64]
};

struct PriorDev {
    double t_window, d_min, d_max, d_ref;
    int dist_marg;
};

// Phase shear of a mixture's coordinates: the psi column becomes
// y = (psi + s phi_c) mod pi (s = +-1), a shear of the (phi_c, psi) torus with
// unit Jacobian.  A face-on source's likelihood depends on the phases nearly
// only through psi + phi_c (face-off: psi - phi_c), a ridge along phi_c at
// fixed y that one elongated component covers.  shear_phase(y, phi, -s)
// maps back.
__device__ __forceinline__ double shear_phase(double psi, double phi, int s) {
    constexpr double kPiS = 3.14159265358979323846;
    const double y = psi + (double)s * phi;
    return y - kPiS * floor(y / kPiS);
}

// Mixture pool of an adaptive job after its round r: every sample of rounds
// 0..r taken as a draw of the equal-weight mixture of the rounds' proposals
// (round 0: the prior).  lmix[i] = ln sum_{q<=r} p_s,q(x_i)/p(x_i) is kept
// across rounds (old samples add the newest proposal's term, the new round's
// samples get every term), and lw[i] = lnL[i] - lmix[i] + ln(r + 1).
struct PoolJob {
    const void *theta;    // [7][ld] every round's samples (policy theta type)
    int64_t ld;
    const void *lnL;      // [(r+1) n_round] (policy output type)
    double *lmix;         // [(r+1) n_round]
    void *lw;             // [(r+1) n_round] (policy log-weight type)
    const GmmDev *hist;   // hist[q]: the proposal that drew round q (q = 1..r)
    PriorDev pr;
    int64_t n_round;
    int32_t round;
    int32_t pad_;
    int64_t tile_begin;   // first block of this job (blocks cover the jobs in order)
};
// Samples per tile of the pool update (one block each).
constexpr int64_t kPoolTileSamples = 512;
hipError_t launch_pool_mix(int policy, const PoolJob *d_jobs, int n_jobs, int64_t n_tiles, hipStream_t st);

// Inverse-CDF map of seven uniforms onto the prior: alpha ~ U[0, 2pi),
// p(dec) = cos(dec)/2, t ~ U[-t_w, t_w], p(D) = 3 D^2/(D_max^3 - D_min^3)
// (D = d_ref when the distance is marginalised), cos(iota) ~ U[-1, 1],
// phi_c ~ U[0, 2pi), psi ~ U[0, pi).
__device__ __forceinline__ void prior_map(const PriorDev &pr, const double u[7], double th[7]) {
    constexpr double kPiM = 3.14159265358979323846;
    th[0] = 2 * kPiM * u[0];
    th[1] = asin(2.0 * u[1] - 1.0);
    th[2] = -pr.t_window + 2.0 * pr.t_window * u[2];
    if (pr.dist_marg) {
        th[3] = pr.d_ref;
    } else {
        const double a3 = pr.d_min * pr.d_min * pr.d_min, b3 = pr.d_max * pr.d_max * pr.d_max;
        th[3] = cbrt(a3 + u[3] * (b3 - a3));
    }
    th[4] = 2.0 * u[4] - 1.0;
    th[5] = 2 * kPiM * u[5];
    th[6] = kPiM * u[6];
}

struct DrawJob {
    const GmmDev *gmm;    // null: prior draws
    PriorDev pr;
    uint64_t seed;
    uint32_t round;
    int64_t first;
    void *theta;
    int64_t ld;
    void *lnpmps;
    int64_t n;
};

// --------------------------------------------------------- launch wrappers
// Return hipSuccess or the launch error.  All enqueue on `st`.
// A device array of job descriptors with a tile list (one block per tile).
hipError_t launch_eval(int set, int kdet, int policy, bool dist_marg, size_t lds_bytes,
                       const EvalJob *d_jobs, const Tile *d_tiles, int n_tiles, int block, hipStream_t st);
size_t eval_lds_limit();
// Mixed policy: rebuild a job's reference terms (one block) from the
// reference point at rb.theta_ref; and set that point to the mean of the
// heaviest component of a mixture (non-mixture columns: prior midpoints).
hipError_t launch_ref_build(int set, int kdet, const EvalJob &job, const RefBuild &rb, hipStream_t st);
hipError_t launch_ref_from_gmm(const GmmDev *g, PriorDev pr, double *theta_ref, hipStream_t st);

hipError_t launch_marg_partials(int policy, const void *lw, int64_t n, int64_t tile,
                                MargPartial *d_part, hipStream_t st);
hipError_t launch_marg_combine(const MargPartial *d_part, int n_part, int64_t n, MargState *d_state,
                               int reset, hipStream_t st);
hipError_t launch_marg_batch(int policy, const MargJob *d_jobs, int n_jobs, const Tile *d_tiles, int n_tiles,
                             MargPartial *d_part, MargState *d_out, hipStream_t st);

// `mix`: some job carries a mixture proposal (otherwise the prior-only kernel).
hipError_t launch_draw(int policy, const DrawJob *d_jobs, const Tile *d_tiles, int n_tiles,
                       const DrawJob &single, int64_t tile, bool mix, hipStream_t st);

// One job of a batched mixture refit or mass estimate.  Every stage is one
// launch over all jobs of the batch (one sample type per launch).
struct EmJob {
    const void *theta;    // [7][ld] samples (policy theta type)
    int64_t ld;
    const void *lw;       // [n] log-weights (policy weight type)
    int64_t n;
    GmmDev *gmm;
    double *work;         // em_work_bytes(n) bytes
    uint32_t *zcount;     // [kMaxComp] in-support counters
    PriorDev pr;
    int n_comp;           // first fit: components
    int first;            // 1: first fit from the highest-weight samples
    int n_dim;            // first fit: mixture columns
    int dims[7];
    double eps_def;       // first fit: defensive prior fraction
    double temper;        // ESS fraction of the tempering rule (<= 0: beta = 1)
    int shear_auto;       // first fit: shear the phases, sign from the best sample's cos(iota)
    uint64_t z_seed;      // in-support mass: Philox key, round, number of draws
    uint32_t z_round;
    int64_t z_draws;
};

// Factor every job's mixture (Cholesky, inverse, log-weights).
hipError_t launch_gmm_factor(const EmJob *d_jobs, int n_jobs, hipStream_t st);
// In-support masses Z_j of every job's mixture from z_draws candidates each.
hipError_t launch_gmm_mass(const EmJob *d_jobs, int n_jobs, hipStream_t st);

// ------------------------------------------------------- adaptive volume
// Section "Adaptive volume integration": samples uniform over the active
// hypercubes of a grid of nb bins per sampled column, in the unit cube of the
// prior's CDF coordinates; after each round a likelihood threshold, a refined
// bin count (eq. nbins_V) and the cells holding the samples above it.
constexpr int kAvMaxBins = 511;
constexpr int kAvMassBits = 40;
struct AvDev {
    int32_t d;            // sampled columns
    int32_t dims[7];      // their theta columns (increasing)
    int32_t kcol[7];      // grid dimension of each theta column, -1: drawn from the prior
    int32_t nb;           // bins per dimension of the current grid
    int32_t nb_next;      // of the grid the last update built
    int32_t cur;          // which cell buffer holds the current grid
    int32_t valid;        // the last update found a finite sample
    int32_t pad_;
    int64_t n_cells, n_cells_next;
    double ln_vol;        // ln V = ln n_cells - d ln nb
    // last update
    double thr;           // threshold (log-weight)
    int64_t n_min, n_live;
    double vol_mc;        // V n_min / n_live
    // threshold selection (radix select over order-preserving keys): chain 0
    // follows the enclosed mass, chain 1 the count
    double vmax;
    unsigned long long key_max, n_fin, total;
    unsigned long long prefix[2], above_cnt[2], above_mass[2], target[2], last_cnt[2];
    unsigned long long thr_key;
};
struct AvBufs {
    AvDev *st;
    uint16_t *cells[2];           // [cap][8] cell coordinates, two buffers
    unsigned long long *hkey;     // [hcap] cell ids of the open-addressing set
    uint32_t *hidx;               // [hcap] first sample index of each cell
    uint64_t hmask;               // hcap - 1
    uint32_t *slot;               // [cap] set slot of each sample above the threshold
    uint32_t *bcnt;               // [cap / 256 + 1] per-block counts, then offsets
    unsigned long long *hist;     // [2 chains][256 digits][count, mass]
};
// One job of a batched AV draw or update (blockIdx.z selects the job).
struct AvJob {
    AvBufs b;
    PriorDev pr;          // draws
    uint64_t seed;
    uint32_t round;
    int64_t first;
    int64_t n;
    void *theta;          // draws: [7][ld] theta type, and [n] ln p - ln p_s (or null)
    int64_t ld;
    void *lnpmps;
    const void *lw;       // updates: [n] log-weights in the policy's output type
    double p_thr;
    int64_t n_min_live;
    int max_bins;
};
// ------------------------------------------------- adaptive Cartesian
// Product-form adaptive Cartesian sampler: one kAcBins-bin histogram marginal
// per sampled coordinate of the prior's CDF cube.
constexpr int kAcBins = 64;
struct AcDev {
    int32_t d;            // sampled columns
    int32_t dims[7];
    int32_t kcol[7];      // marginal of each theta column, -1: drawn from the prior
    int32_t pad_;
    double pi[7][kAcBins];      // bin probabilities
    double cum[7][kAcBins];     // sequential cumulative sums, cum[k][nb-1] = 1
    double lnbp[7][kAcBins];    // ln(nb pi)
    unsigned long long key_max, n_fin;
    unsigned long long hist[7][kAcBins];   // update: fixed-point masses per bin
};
struct AcJob {
    AcDev *st;
    PriorDev pr;          // draws
    uint64_t seed;
    uint32_t round;
    int64_t first;
    int64_t n;
    void *theta;          // draws: [7][ld] theta type; [n] ln p - ln p_s or null
    int64_t ld;
    void *lnpmps;
    const void *lw;       // updates: [n] log-weights (the policy's output type)
    double floor;         // updates: uniform fraction mixed into each marginal
};
hipError_t launch_ac_reset(AcDev *st, int d, const int *dims, hipStream_t st_);
hipError_t launch_ac_draw(int policy, const AcJob *d_jobs, const AcJob *h_jobs, int n_jobs, hipStream_t st);
hipError_t launch_ac_update(int policy, const AcJob *d_jobs, const AcJob *h_jobs, int n_jobs, hipStream_t st);

// Q, U, V of eq. (QUV) from modes and data (k_qv.hip).  h_band / h_msig:
// host lists of the band's grid indices and their signed frequency indices.
int qv_slices(int64_t n_band, int64_t cols, int n_time);
size_t qv_scratch_bytes(int64_t n, int64_t n_band, int64_t cols, int n_time, int n_slices);
hipError_t launch_qv(const void *hlm, const void *data, const double *inv_psd, int64_t n, int na, int nd, int np,
                     double df, const int64_t *h_band, const int64_t *h_msig, int64_t n_band, int n_time,
                     int win_half, void *Q, void *U, void *V, void *scratch, int n_slices, hipStream_t st);

// Order-preserving integer keys of finite values (key(a) < key(b) iff
// a < b; -0 is taken as +0), their inverse, and the fixed-point sample mass
// floor(exp(v - vmax) 2^40) shared by the AV threshold, the AC histograms and
// the fair draws.
__device__ __forceinline__ unsigned long long ord_key(float v) {
    const uint32_t bits = __float_as_uint(v + 0.0f);
    return (unsigned long long)((bits & 0x80000000u) ? ~bits : (bits | 0x80000000u));
}
__device__ __forceinline__ unsigned long long ord_key(double v) {
    const unsigned long long bits = (unsigned long long)__double_as_longlong(v + 0.0);
    return (bits >> 63) ? ~bits : (bits | (1ull << 63));
}
__device__ __forceinline__ double ord_value(unsigned long long k, int nbits) {
    if (nbits == 32) {
        const uint32_t kk = (uint32_t)k;
        return (double)__uint_as_float((kk & 0x80000000u) ? (kk & 0x7FFFFFFFu) : ~kk);
    }
    return __longlong_as_double((long long)((k >> 63) ? (k & ~(1ull << 63)) : ~k));
}
__device__ __forceinline__ unsigned long long mass_fx(double v, double vmax) {
    return (unsigned long long)floor(exp(v - vmax) * (double)(1ull << kAvMassBits));
}

// Fair draws from weighted samples (k_fair.hip): scratch of
// fair_scratch_bytes(n) bytes; lw in the policy's output type, theta in its
// theta type.
size_t fair_scratch_bytes(int64_t n);
hipError_t launch_fair_draw(int policy, const void *lw, int64_t n, uint64_t seed, uint32_t round, int64_t k,
                            int64_t *idx, const void *theta, int64_t ld, void *theta_out, int64_t ld_out,
                            void *scratch, hipStream_t st);

// Initial grid: one cell, nb = 1, over the given columns.
hipError_t launch_av_reset(const AvBufs &b, int d, const int *dims, hipStream_t st);
// d_jobs: device copy of h_jobs (all of one theta type for draws, of one
// log-weight type for updates: `policy` names it).
hipError_t launch_av_draw(int policy, const AvJob *d_jobs, const AvJob *h_jobs, int n_jobs, hipStream_t st);
hipError_t launch_av_update(int policy, const AvJob *d_jobs, const AvJob *h_jobs, int n_jobs, hipStream_t st);
// Weighted EM refit of every job: max and tempering exponent, first fit for
// jobs with `first`, then n_iter iterations.  h_jobs: host copy of d_jobs.
hipError_t launch_em_batch(int policy, const EmJob *d_jobs, const EmJob *h_jobs, int n_jobs, int n_iter,
                           hipStream_t st);
size_t em_work_bytes(int64_t n);

hipError_t build_dist_table(DistTable *tab, double *d_buf, PriorDev pr, hipStream_t st);
size_t dist_table_bytes();

}  // namespace ile
