/*
 * ile.h - C ABI of the MI355X (gfx950) extrinsic-marginalised likelihood (ILE).
 *
 * Paper: arXiv 2505.11655 ("Narrowing RIFT"), Section "Review of the RIFT
 * likelihood".  For one intrinsic point lambda the inputs are, per detector k,
 * the windowed inner-product series Q_k,lm(tau) and the mode overlaps
 * U_k,lm,l'm' = <h_lm|h_l'm'>, V_k,lm,l'm' = <h_lm^*|h_l'm'> of eq. (QUV).
 * The library evaluates, for Monte Carlo samples theta = (alpha, delta, t, D,
 * cos iota, phi_c, psi), the factored log-likelihood of eq.
 * (def:lnL:Decomposed) and integrates it with the estimator of eq.
 * (lnL:MonteCarlo) and the effective sample size of eq. (neff).
 *
 * Conventions (the paper is silent or self-inconsistent on these):
 *  - F_k = F+ + i Fx (with h = h+ - i hx and h_k = F+ h+ + Fx hx this makes
 *    the printed decomposition exact);
 *  - the sky vector points to the source, tau_k = t - x_k . n / c;
 *  - Y_lm = -2Y_lm(iota, -phi_c); psi only rotates the polarisation basis;
 *  - Q between window samples: 4-point Lagrange cubic on samples i-1..i+2,
 *    i = floor((tau - tau0)/dt), valid for 1 <= i <= n_time-3.
 *
 * Memory: the arrays of ile_problem are host memory, or device memory of the
 * context's GPU when mem_is_device = 1; either way ile_prepare and
 * ile_server_submit deep-copy them and the caller may free them on return.  Sample buffers passed to ile_eval_lnL / ile_draw /
 * ile_marginalize / ile_adapt_proposal are DEVICE memory owned by the caller
 * (e.g. torch tensors); the library never frees them.  Calls enqueue work on
 * the given HIP stream (NULL = the device's null stream) and return without
 * waiting, except where a host-side result is requested (then the stream is
 * synchronised before returning).
 *
 * Errors: every call returns an ile_status.  ILE_E_INVALID for bad shapes,
 * sizes, pointers, non-finite or non-Hermitian inputs; ILE_E_DEVICE for a
 * HIP error, after which the context is sticky-failed and every later call on
 * it returns ILE_E_DEVICE.  ile_last_error() gives a message for the last
 * failing call on the calling thread.  No exception crosses the ABI.
 */
#ifndef ILE_H
#define ILE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ILE_OK = 0,
    ILE_PENDING = 1,
    ILE_E_INVALID = -1,
    ILE_E_NOMEM = -2,
    ILE_E_TOO_BIG = -3,
    ILE_E_DEVICE = -4,
    ILE_E_STATE = -5,
    ILE_E_CANCELLED = -6,
    ILE_E_TIMEOUT = -7
} ile_status;

/* Arithmetic policy (eq. def:lnL:Decomposed).
 *  ILE_FP64          everything in FP64; theta, ln p - ln p_s, lnL, lw are double.
 *  ILE_FP32          FP32 contractions, FP32 accumulation; the sky direction and
 *                    detector delays are FP64 (an FP32 delay moves the phase of
 *                    Q by enough to move lnL by ~1e-4 at SNR 20); theta,
 *                    ln p - ln p_s, lnL, lw are float.
 *  ILE_FP32_CANCEL64 lnL written about a reference point (ile_set_reference):
 *                    the two rho^2-sized terms that cancel -- the reference
 *                    amplitudes against the interpolated Q, and their quadratic
 *                    form in U, V -- are FP64, as are the mode amplitudes
 *                    s F_k Y_lm; every term in a sample's offset from the
 *                    reference is an FP32 contraction with FP32 accumulation.
 *                    theta and ln p - ln p_s are float; lnL and lw are double. */
typedef enum { ILE_FP64 = 0, ILE_FP32 = 1, ILE_FP32_CANCEL64 = 2 } ile_precision;

typedef struct ile_ctx ile_ctx;
typedef struct ile_job ile_job;
typedef struct ile_server ile_server;
typedef void *ile_stream; /* hipStream_t */

/* Prior support (the sampled coordinates):
 * alpha ~ U[0,2pi), p(delta) = cos(delta)/2, t ~ U[-t_window, t_window],
 * p(D) = 3 D^2 / (d_max^3 - d_min^3) on [d_min, d_max] Mpc, cos iota ~ U[-1,1],
 * phi_c ~ U[0,2pi), psi ~ U[0,pi).  dist_marg = 1: the distance integral is
 * done inside the likelihood (2-D FP64 table over (T1, T2)) and D is not sampled. */
typedef struct {
    double t_window;
    double d_min, d_max;
    int32_t dist_marg;
} ile_prior;

typedef struct {
    int32_t n_det;            /* 1..3 */
    int32_t n_modes;          /* 1..21, every l in 2..4, |m| <= l, no duplicates */
    int32_t n_time;           /* window samples, >= 4 */
    int32_t mem_is_device;    /* 0: the arrays below are host memory; 1: device memory of
                                 the context's GPU (copied to the host for validation and
                                 packing, then uploaded as for host arrays) */
    const int32_t *mode_l;    /* [n_modes] */
    const int32_t *mode_m;    /* [n_modes] */
    const double *det_pos;    /* [n_det][3] metres, Earth-fixed */
    const double *det_resp;   /* [n_det][3][3] response tensor, symmetric */
    double gmst_rad;          /* Greenwich sidereal angle of the reference time */
    double tau0_s, dt_s;      /* window: tau_i = tau0_s + i dt_s, relative to the reference time */
    const double *Q;          /* [n_det][n_modes][n_time] complex128 (re, im) */
    const double *U;          /* [n_det][n_modes][n_modes] complex128, Hermitian */
    const double *V;          /* same, complex symmetric; NULL = zero (only if all m share a sign) */
    double d_ref_mpc;         /* distance at which Q, U, V were computed */
    double mode_filter_eps;   /* 0 = off (paper default); else keep (l,m) iff some
                                 |U_0[lm][l'm'] / U_0[22][22]| > eps (detector 0) */
    int32_t precision;        /* ile_precision */
    ile_prior prior;
} ile_problem;

typedef struct {
    double ln_L;              /* ln of the estimator (1/N) sum w_i */
    double ln_sigma;          /* ln of its standard error */
    double n_eff;             /* eq. (neff): sum w / max w */
    double n_ess;             /* (sum w)^2 / sum w^2 */
    double max_lw;            /* max log-weight */
    int64_t argmax;           /* index of max lw (lowest on ties; pooled index) */
    int64_t n;                /* samples pooled */
    int64_t n_nonfinite;      /* samples with non-finite lw (zero weight) */
} ile_marg;

typedef struct {
    int32_t n_modes_kept;     /* after the mode filter */
    int32_t mode_slots;       /* compiled mode-set size the job runs in (5, 9, 17, 21) */
    int32_t n_det_slots;      /* compiled detector count (2 or 3) */
    size_t device_bytes;      /* resident device memory of the job */
} ile_job_info;

/* Context: one per HIP device.  hbm_budget_bytes = 0 means the whole device.
 * (Library state, not a step of the paper's method.) */
ile_status ile_ctx_create(int hip_device, size_t hbm_budget_bytes, ile_ctx **out);
void ile_ctx_destroy(ile_ctx *ctx);
const char *ile_last_error(void);

/* Validate, filter modes, convert to the policy's precision and layout, upload:
 * the residency of Q, U, V for one intrinsic point (Section "Review of the
 * RIFT likelihood", eq. QUV).  U is Hermitian and V symmetric, so only the
 * pairs a <= b are kept (Section "Reduce duplication of inner products").
 * mode_filter_eps > 0 drops modes whose overlaps are negligible, as in
 * Section "Disable automatic mode filtering" (0 = off, the paper's choice). */
ile_status ile_prepare(ile_ctx *ctx, const ile_problem *problem, ile_job **out);
ile_status ile_job_info_get(const ile_job *job, ile_job_info *info);
void ile_job_release(ile_job *job);

/* Reference point of an ILE_FP32_CANCEL64 job (eq. def:lnL:Decomposed written
 * about a reference, Section "Review of the RIFT likelihood"): that policy
 * evaluates the two terms of size rho^2 that cancel in lnL -- Re of the
 * reference amplitudes against the interpolated Q, and the reference's
 * quadratic form in U, V -- in FP64, and everything that depends on a
 * sample's offset from the reference in FP32.  lnL does not depend on the
 * reference (up to rounding); its FP32 rounding shrinks with the samples'
 * distance from it, so the reference should sit near the samples that carry
 * the weight.  theta_ref: host [7] (alpha, delta, t, D, cos iota, phi_c, psi);
 * a point outside the support clears the reference (plain FP32 arithmetic,
 * the state after ile_prepare).  ile_set_proposal and ile_adapt_proposal set
 * it to the mean of the mixture's heaviest component.  Built on the device on
 * `stream` (the call waits for the small upload).  No effect for the other
 * policies. */
ile_status ile_set_reference(ile_job *job, const double *theta_ref, ile_stream stream);

/* Per-sample lnL, eq. (def:lnL:Decomposed).
 * theta: device [7][ld] (float or double by policy), columns (alpha, delta, t,
 * D, cos iota, phi_c, psi), ld >= n.  lnpmps: device [n] ln p - ln p_s in the
 * theta type, or NULL (0).  lnL_out: device [n] (float for ILE_FP32, else
 * double).  lw_out: device [n] lnL + lnpmps, or NULL.  Samples outside the
 * support (window stencil out of range, D <= 0, |cos iota| > 1) give -inf.
 * With prior.dist_marg the D column is ignored and lnL is the distance-
 * marginalised value. */
ile_status ile_eval_lnL(ile_job *job, int64_t n, const void *theta, int64_t ld,
                        const void *lnpmps, void *lnL_out, void *lw_out, ile_stream stream);

/* Several jobs of the same policy in one pass; arrays of length n_jobs. */
ile_status ile_eval_lnL_batch(ile_job *const *jobs, int32_t n_jobs, const int64_t *n,
                              const void *const *theta, const int64_t *ld,
                              const void *const *lnpmps, void *const *lnL_out,
                              void *const *lw_out, ile_stream stream);

/* Time-marginalised likelihood per extrinsic sample: the (time) x (extrinsic)
 * array of eq. (lnL:MatrixForm) integrated over the geocentric time prior
 * U[-t_window, t_window] by the rectangle rule on the nodes t_j = j dt / R,
 * |j| <= floor(R t_window / dt) (dt = the window's sample step), each weighted
 * dt / (R 2 t_window):
 *     lnL_t = ln sum_j (dt / (R 2 t_window)) exp lnL(theta with t = t_j).
 * The t column of theta is ignored; all other arguments are those of
 * ile_eval_lnL (lw_out = lnL_t + lnpmps).  oversample R: 1 or 4 (R = 4 resolves
 * a likelihood peak narrower than dt; the rule's error is O((dt/R)^2)).
 * With prior.dist_marg the D column is ignored too and each node's value is
 * the distance-marginalised one, ln L_D(T1(t_j), T2) from the distance table
 * (T1, T2 at D = d_ref): time and distance integrated together, as the paper's
 * timed runs integrate time (Appendix "Timing analysis") with distance
 * marginalisation (Section "Adaptive volume integration").
 * ILE_FP32 and ILE_FP64 jobs only; other jobs, or another R, give
 * ILE_E_INVALID.  A node whose stencil leaves the window contributes 0;
 * no valid node gives -inf. */
ile_status ile_eval_lnL_tmarg(ile_job *job, int64_t n, const void *theta, int64_t ld,
                              const void *lnpmps, void *lnL_out, void *lw_out, int32_t oversample,
                              ile_stream stream);

/* The same for several jobs in one pass per compiled kernel; arrays of length n_jobs. */
ile_status ile_eval_lnL_tmarg_batch(ile_job *const *jobs, int32_t n_jobs, const int64_t *n,
                                    const void *const *theta, const int64_t *ld,
                                    const void *const *lnpmps, void *const *lnL_out,
                                    void *const *lw_out, int32_t oversample, ile_stream stream);

/* Monte Carlo estimator of eq. (lnL:MonteCarlo) on log-weights lw (device [n],
 * the lw type of the policy).  The job keeps the pooled (max, S1, S2, N) state.
 * flags: ILE_MARG_RESET clears it first; ILE_MARG_POOL adds this batch to it.
 * out (host, may be NULL): the pooled result; the stream is synchronised when given. */
#define ILE_MARG_RESET 1u
#define ILE_MARG_POOL 2u
ile_status ile_marginalize(ile_job *job, int64_t n, const void *lw, uint32_t flags,
                           ile_marg *out, ile_stream stream);

/* The same for several jobs of one policy in two launches; arrays of length
 * n_jobs.  out: host [n_jobs] or NULL.  Each job's result is bitwise the one
 * ile_marginalize gives for it alone (same tiles, same order). */
ile_status ile_marginalize_batch(ile_job *const *jobs, int32_t n_jobs, const int64_t *n,
                                 const void *const *lw, uint32_t flags, ile_marg *out,
                                 ile_stream stream);

/* ile_marginalize for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same kernels, tiles and result (bitwise that of ile_marginalize), but
 * the per-tile partials live in a fixed 1 MiB device array that the library
 * holds on each GPU until the process ends, so this call allocates nothing.
 * n above ile_marginalize_noalloc_max() samples gives ILE_E_TOO_BIG.  All
 * calls on one GPU share that array: calls that overlap in time on one GPU
 * (other streams, other threads) race and must be serialised by the caller.
 * out (host, may be NULL): as for ile_marginalize (copied through the job's
 * pinned buffer; the stream is synchronised). */
ile_status ile_marginalize_noalloc(ile_job *job, int64_t n, const void *lw, uint32_t flags,
                                   ile_marg *out, ile_stream stream);
size_t ile_marginalize_noalloc_max(void);

/* Counter-based draws (Philox-4x32-10) of samples first_index .. first_index+n-1
 * of round `round` under key `seed`: from the prior while the job has no
 * proposal, else from the mixture proposal p_s -- the samples and the
 * ln p - ln p_s of the Monte Carlo estimator, eq. (lnL:MonteCarlo), with the
 * sampling priors of Section "Evaluating the marginalized likelihood".
 * theta_out: device [7][ld]; lnpmps_out: device [n] ln p - ln p_s (theta
 * type), or NULL. */
ile_status ile_draw(ile_job *job, uint64_t seed, uint32_t round, int64_t first_index, int64_t n,
                    void *theta_out, int64_t ld, void *lnpmps_out, ile_stream stream);

/* Mixture proposal p_s = (1 - eps) sum_j pi_j N_j / Z_j + eps p over the sampled
 * columns (all seven, or six with dist_marg); periodic alpha, phi_c (2pi) and
 * psi (pi) use differences wrapped into (-P/2, P/2].  The Gaussian-mixture
 * sampling prior of Section "Evaluating the marginalized likelihood" (its
 * details are not printed there; this is the library's reading). */
#define ILE_GMM_MAX_COMP 16
typedef struct {
    int32_t n_comp;           /* 1..16 */
    int32_t n_dim;            /* 6 or 7 (set by the library) */
    int32_t dims[7];          /* theta column of each dimension */
    double eps_def;           /* defensive prior weight */
    double weight[ILE_GMM_MAX_COMP];
    double mean[ILE_GMM_MAX_COMP][7];
    double cov[ILE_GMM_MAX_COMP][7][7];
    double ln_Z[ILE_GMM_MAX_COMP];  /* in-support mass (output of set/adapt) */
    int32_t shear;            /* 0, or +1 / -1: the mixture's psi column (mean, covariance) is
                                 y = (psi + shear phi_c) mod pi, a shear of the (phi_c, psi) torus
                                 with unit Jacobian; draws are mapped back to psi */
} ile_gmm_params;

typedef struct {
    int32_t n_comp;           /* default 8 */
    int32_t n_iter;           /* EM iterations per call, default 8 */
    double eps_def;           /* default 0.05 */
    uint64_t seed;            /* key for the in-support mass draws */
    uint32_t round;           /* counter word for the same */
    int64_t z_draws;          /* in-support mass draws per component, default 65536 */
    double temper_ess;        /* 0: EM on the weights w; f in (0,1]: EM on w^beta with beta
                                 the largest of 2^(-k/4), k = 0..47, whose effective sample
                                 size (sum w^beta)^2 / sum w^(2 beta) >= f * (finite samples) */
    int32_t phase_shear;      /* first fit only: 1 fits the mixture in sheared phases (see
                                 ile_gmm_params.shear), sign +1 if the highest-weight sample has
                                 cos(iota) >= 0 (face-on: the likelihood ridge runs along
                                 psi + phi_c = const), else -1; 0 (default) leaves them as they are.
                                 Later refits keep the first fit's shear. */
} ile_gmm_opts;

/* Install an explicit proposal (host parameters); the library factorises the
 * covariances and estimates ln Z on the device (opts may be NULL for defaults).
 * Section "Evaluating the marginalized likelihood" (GMM sampling prior).
 * ILE_FP32_CANCEL64 jobs also take the heaviest component's mean as their
 * reference point (ile_set_reference). */
ile_status ile_set_proposal(ile_job *job, const ile_gmm_params *params, const ile_gmm_opts *opts,
                            ile_stream stream);
ile_status ile_get_proposal(ile_job *job, ile_gmm_params *params, ile_stream stream);

/* Weighted EM refit of the proposal from samples (theta [7][ld], lw [n], device):
 * first call seeds the means at the highest-weight distinct samples with a
 * common weighted covariance; later calls warm-start.  Each component gets
 * Sigma += 1e-8 diag(range^2).  Host diagnostics (may be NULL): the new params.
 * The adaptive step of the GMM sampling prior (Section "Evaluating the
 * marginalized likelihood": the proposal is refitted to the weighted samples
 * until the effective sample size of eq. (neff) reaches its target).
 * ILE_FP32_CANCEL64 jobs move their reference point to the refitted mixture's
 * heaviest component. */
ile_status ile_adapt_proposal(ile_job *job, int64_t n, const void *theta, int64_t ld,
                              const void *lw, const ile_gmm_opts *opts,
                              ile_gmm_params *out, ile_stream stream);

/* ------------------------------------------------------- adaptive volume */
/* The adaptive-volume (AV) integrator of Section "Adaptive volume
 * integration": samples uniform over a set of active hypercubes of a grid of
 * n_bins bins per sampled column, in the unit cube of the prior's CDF
 * coordinates u (theta = the prior's inverse-CDF map of u), so that
 * ln p - ln p_s = ln V for every sample, V = n_cells / n_bins^n_dim the active
 * volume.  Each update takes one round's log-weights, sets a likelihood
 * threshold, refines the bin count by eq. (nbins_V) and keeps the cells that
 * hold a sample at or above the threshold.  The grid lives in device memory
 * with the job; draws and updates are asynchronous on the stream and read it
 * there (no host synchronisation). */
typedef struct {
    double p_thr;             /* enclosed probability the threshold keeps, (0, 1]; default 0.999 */
    int64_t n_min_live;       /* at least this many highest samples kept; default 1000 */
    int32_t max_bins;         /* cap on bins per dimension, 1..511; default 511 */
} ile_av_opts;

typedef struct {
    int32_t n_dim;            /* sampled columns */
    int32_t dims[7];          /* their theta columns (increasing), -1 beyond n_dim */
    int32_t n_bins;           /* current grid */
    int64_t n_cells;
    double ln_vol;            /* ln V = ln n_cells - n_dim ln n_bins */
    double lnL_thr;           /* last update: threshold (log-weight; -inf if none) */
    int64_t n_min;            /*   samples at or above it */
    int64_t n_live;           /*   samples of the round */
    double vol_mc;            /*   Monte Carlo estimate V n_min / n_live of the volume above it */
} ile_av_state;

/* Start over from the whole cube (one cell, n_bins = 1) over the given theta
 * columns (n_dim = 0: every sampled column, i.e. all seven, or six with
 * dist_marg).  Columns outside the grid are drawn from the prior.  Errors:
 * ILE_E_INVALID for columns not strictly increasing in 0..6 or column 3 with
 * dist_marg. */
ile_status ile_av_reset(ile_job *job, int32_t n_dim, const int32_t *dims, ile_stream stream);

/* Draws of samples first_index .. first_index+n-1 of round `round` under key
 * `seed`, uniform over the active cells (Philox-4x32-10 with the prior draw's
 * counters: on the one-cell grid the draws are the prior draws).
 * theta_out: device [7][ld] (theta type); lnpmps_out: device [n] = ln V, or
 * NULL.  The first AV call on a job resets it (n_dim = 0). */
ile_status ile_av_draw(ile_job *job, uint64_t seed, uint32_t round, int64_t first_index, int64_t n,
                       void *theta_out, int64_t ld, void *lnpmps_out, ile_stream stream);

/* Refine the grid from the samples of one ile_av_draw call (the same seed,
 * round, first_index and n, with the grid unchanged since): lw device [n]
 * log-weights (or log-likelihoods: only differences matter) in the policy's
 * output type.  The threshold is the largest lw value v such that the samples
 * at or above v hold at least min(ceil(p_thr total), total) of the fixed-point
 * masses floor(exp(lw - max lw) 2^40) and number at least
 * min(n_min_live, finite samples).  n_bins' = ceil((1/dV)^(1/n_dim)) clamped to
 * [1, max_bins], dV = V n_min / (n sqrt(n_min)); the new cells are those of
 * the n_bins' grid holding a sample at or above the threshold, in order of
 * their first such sample.  With no finite lw the grid is kept.  opts may be
 * NULL; out (host, may be NULL) synchronises the stream.  n < 2^31. */
ile_status ile_av_update(ile_job *job, uint64_t seed, uint32_t round, int64_t first_index, int64_t n,
                         const void *lw, const ile_av_opts *opts, ile_av_state *out, ile_stream stream);

/* Current grid and last update (synchronises the stream).  cells: host
 * [cap][n_dim] int32 cell coordinates in list order, or NULL; at most cap rows
 * are written. */
ile_status ile_av_get(ile_job *job, ile_av_state *out, int32_t *cells, int64_t cap, ile_stream stream);

/* ---------------------------------------------------- adaptive Cartesian */
/* Section "Evaluating the marginalized likelihood": a sampling prior that is a
 * product of one-dimensional distributions, each updated after a block of
 * evaluations to follow the integrand's support.
 * The product-form adaptive Cartesian (AC) sampling prior: one adaptive
 * 64-bin piecewise-constant marginal per sampled column of the prior's CDF
 * cube (all seven columns, or six with dist_marg, or a chosen subset; other
 * columns are drawn from the prior).  A draw inverts each marginal's CDF at
 * the prior draw's uniform for that column, so uniform marginals draw exactly
 * the prior; ln p - ln p_s = -sum_k ln(64 pi_k(bin)).  An update replaces each
 * marginal by the histogram, over its bins, of the round's fixed-point masses
 * floor(exp(lw - max lw) 2^40), mixed with the uniform:
 * pi = (1 - floor) h / total + floor / 64 (floor 0 means 0.1); with no finite
 * lw the marginals are kept.  The update must follow the draw it refers to
 * (same seed, round, first_index, n) with the marginals unchanged since.
 * The state lives in device memory with the job; draws and updates are
 * asynchronous on the stream. */
ile_status ile_ac_reset(ile_job *job, int32_t n_dim, const int32_t *dims, ile_stream stream);
ile_status ile_ac_draw(ile_job *job, uint64_t seed, uint32_t round, int64_t first_index, int64_t n,
                       void *theta_out, int64_t ld, void *lnpmps_out, ile_stream stream);
ile_status ile_ac_update(ile_job *job, uint64_t seed, uint32_t round, int64_t first_index, int64_t n,
                         const void *lw, double floor_frac, ile_stream stream);
/* Marginals (synchronises the stream): n_dim, dims[7] (-1 beyond n_dim) and
 * pi host [n_dim][64]; any output may be NULL. */
ile_status ile_ac_get(ile_job *job, int32_t *n_dim, int32_t *dims, double *pi, ile_stream stream);

/* ---------------------------------------------------- Q, U, V precompute */
/* The inner products of eq. (QUV) on the device, in FP64, for n_points
 * intrinsic points (mode sets) sharing one data set:
 *   Q[p][k][a][i] = 2 df sum_f e^{2 pi i f tau_i} conj(h_pa(f)) d_k(f) w_k(f),
 *   U[p][k][a][b] = 2 df sum_f conj(h_pa(f)) h_pb(f) w_k(f),
 *   V[p][k][a][b] = 2 df sum_f h_pa(-f) h_pb(f) w_k(f),
 * over f_lo <= |f| <= f_hi of the two-sided grid f_m = m' df (m' the signed
 * index in FFT order: 0..n/2-1, then -n/2..-1), tau_i = (i - win_half)/(n df)
 * with the phase taken exactly as 2 pi ((m' (i - win_half)) mod n)/n.  U is
 * formed for a <= b and mirrored (U_ba = conj U_ab, V_ba = V_ab).  The Q and
 * U, V layouts are those ile_problem takes, one block per point.  At most
 * 1000 modes (ILE_E_INVALID beyond).
 * Routes for Q (the same sums, rounded in a different order):
 *   ILE_QV_DIRECT: the window times x band bins product as written;
 *   ILE_QV_DECIMATED: the grid split once, n = R N2 (the first step of a
 *     decimation-in-frequency FFT, as Section "Reduce duplication of inner
 *     products" prefers FFTs to time-domain sums): radix-R partial sums over
 *     the R aliases m2 + N2 a of each bin, then the product over N2 bins at
 *     the decimated times floor((i - win_half) / R) only.  R is taken among
 *     2, 4, 8, 16 dividing n that put the window on at most 64 decimated
 *     times (one 32- or 64-row tile of the product), by estimated cost;
 *     ILE_E_INVALID when there is none;
 *   ILE_QV_AUTO: the decimated route when it applies and its estimated cost
 *     is lower, else the direct one; also the direct one when the decimated
 *     route's scratch (16 B per grid bin and column, against 16 B per band
 *     bin and column) cannot be allocated within the context's budget.
 * The band lists are staged in pinned memory, so the call does not wait on
 * the stream before its final synchronisation. */
#define ILE_QV_AUTO 0
#define ILE_QV_DIRECT 1
#define ILE_QV_DECIMATED 2
typedef struct {
    int32_t n_points, n_modes, n_det;
    int64_t n_freq;           /* grid length n */
    double df, f_lo, f_hi;
    int32_t n_time, win_half; /* Q window */
    int32_t route;            /* how Q is summed; ILE_QV_AUTO (0) picks the faster */
} ile_qv_shape;
/* hlm: device [n_points][n_modes][n_freq] complex128; data: device
 * [n_det][n_freq] complex128; inv_psd: device [n_det][n_freq] 1/S_k(|f|) or
 * NULL (flat, 1); Q: device [n_points][n_det][n_modes][n_time] complex128;
 * U, V: device [n_points][n_det][n_modes][n_modes] complex128.  Synchronises
 * the stream (its scratch is released on return). */
ile_status ile_overlaps(ile_ctx *ctx, const ile_qv_shape *shape, const void *hlm, const void *data,
                        const double *inv_psd, void *Q, void *U, void *V, ile_stream stream);

/* ------------------------------------------------------------ fair draws */
/* Section "Likelihood interpolation and posterior distributions" (the final
 * fair extrinsic draws; their before/after-resampling check is in Section
 * "Before and after extrinsic resampling").
 * Fair draws from weighted samples: the final extrinsic samples of an ILE run
 * are drawn fairly from its weighted Monte Carlo samples (and the posterior
 * from CIP's weighted samples the same way).  k independent draws with
 * replacement: index i with probability q_i / sum q, q_i =
 * floor(exp(lw_i - max lw) 2^40) (0 for non-finite lw).  Draw j uses Philox
 * counter (j lo, j hi, round, 80) under `seed`: r = w0 2^32 + w1, target =
 * floor(r total / 2^64), index = the first i whose cumulative mass exceeds
 * it; -1 when no sample has mass.  lw: device [n], the policy's output type.
 * idx_out: device [k] int64 or NULL.  theta (device [7][ld], theta type) and
 * theta_out (device [7][ld_out], ld_out >= k) are optional: theta_out gets the
 * drawn samples (NaN for index -1).  Asynchronous on the stream. */
ile_status ile_fair_draw(ile_job *job, int64_t n, const void *lw, uint64_t seed, uint32_t round, int64_t k,
                         int64_t *idx_out, const void *theta, int64_t ld, void *theta_out, int64_t ld_out,
                         ile_stream stream);

/* ---------------------------------------------------------------- serving */
/* A persistent loop that evaluates many intrinsic points' marginal
 * likelihoods at once, as one ILE process evaluates several points in turn
 * (Appendix "Timing analysis"): jobs are admitted by device footprint and
 * their draws, likelihoods, estimators and refits are batched per pass. */
typedef struct {
    int32_t max_active;       /* jobs evaluated per pass (default 64); up to as
                                 many more are admitted (prepared, uploaded,
                                 holding their footprint) while a pass runs */
    size_t hbm_budget_bytes;  /* 0: the context's budget */
    int64_t chunk_samples;    /* samples per job per scheduling pass (default 1<<20) */
    int32_t record_samples;   /* 0 */
} ile_server_opts;

typedef struct {
    int64_t n_samples;        /* fixed budget (plain mode) */
    int32_t adaptive;         /* 1: rounds + mixture refits until n_eff target */
    int64_t round_samples;    /* adaptive: samples per round (default 65536) */
    int32_t max_rounds;       /* adaptive: default 32 */
    double n_eff_target;      /* adaptive: default 1000 */
    uint64_t seed;
    int32_t tmarg_oversample; /* 0: pointwise lnL; 1 or 4: time-marginalised lnL (ile_eval_lnL_tmarg with
                                 this R, distance-marginalised too with dist_marg; plain ILE_FP32 /
                                 ILE_FP64 jobs only), with chunk_samples/16 samples per pass */
    int32_t integrator;       /* adaptive: ILE_INT_GMM (mixture refits), ILE_INT_AV (adaptive volume,
                                 ile_av_update with default options after each round) or ILE_INT_AC
                                 (adaptive Cartesian, ile_ac_update with floor 0.1 after each round) */
    int32_t pool;             /* adaptive ILE_INT_GMM: ILE_POOL_ROUNDS (default) or ILE_POOL_MIXTURE */
    int32_t phase_shear;      /* adaptive ILE_INT_GMM: 1 fits the mixture in sheared phases
                                 (ile_gmm_opts.phase_shear) */
} ile_job_opts;

#define ILE_INT_GMM 0
#define ILE_INT_AV 1
#define ILE_INT_AC 2

/* How an adaptive job's rounds form one Monte Carlo estimate, eq.
 * (lnL:MonteCarlo), with eq. (neff) on the pooled weights.
 * ILE_POOL_ROUNDS: each sample weighted by the proposal of its own round,
 *   w = L p / p_s,r.
 * ILE_POOL_MIXTURE: the R rounds (equal size) taken together as draws of the
 *   equal-weight mixture of their proposals, w = L p / ((1/R) sum_q p_s,q),
 *   recomputed for every sample after each round; the prior (round 0) is a
 *   member, so w <= R L.  A sample that an early proposal put where later
 *   proposals concentrate no longer dominates the pool.  The library keeps
 *   every round's samples (7 theta, lnL, ln sum and weight per sample) and
 *   proposals until the job ends. */
#define ILE_POOL_ROUNDS 0
#define ILE_POOL_MIXTURE 1

typedef struct {
    ile_marg marg;
    int32_t status;           /* ile_status of the job */
    int32_t rounds;
    int64_t samples;
    int64_t t_arrival_ns, t_admit_ns, t_start_ns, t_finish_ns;  /* steady clock */
} ile_result;

ile_status ile_server_create(ile_ctx *ctx, const ile_server_opts *opts, ile_server **out);
ile_status ile_server_submit(ile_server *srv, const ile_problem *problem, const ile_job_opts *opts,
                             uint64_t *job_id);
ile_status ile_server_poll(ile_server *srv, uint64_t job_id, ile_result *out);
ile_status ile_server_wait(ile_server *srv, uint64_t job_id, int64_t timeout_ms, ile_result *out);
ile_status ile_server_cancel(ile_server *srv, uint64_t job_id);
/* active: admitted jobs (those of the current pass and those prepared for
 * the next); queued: waiting for admission; done: finished. */
ile_status ile_server_stats(ile_server *srv, int64_t *active, int64_t *queued, int64_t *done);
void ile_server_destroy(ile_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* ILE_H */
