"""Plain FP64 CPU oracle for the ILE extrinsic-likelihood path.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product library.  It shares no
code with the HIP path.  ``ile_oracle.c`` holds the per-sample likelihood of
eq. (def:lnL:Decomposed), the Monte Carlo estimator of eq. (lnL:MonteCarlo)
with eq. (neff), the counter-based draws and the Gaussian-mixture density;
this module wraps it and adds definition-level numpy helpers:

  * ``exact_Q``          - Q_k,lm(tau) as the direct frequency sum of eq. (QUV);
  * ``lnL_exact``        - lnL with exact Q at the detector times (no window);
  * ``em_fit``           - weighted EM for the mixture proposal (see its docstring);
  * ``ln_dist_marg``     - the distance-marginalised likelihood by adaptive quadrature;
  * ``lnL_tmarg_dist``   - the time- and distance-marginalised likelihood;
  * ``draw_av``, ``av_threshold``, ``av_refine_bins``, ``av_cells``, ``av_update``
                         - the adaptive-volume integrator (its readings are listed there);
  * ``draw_ac``, ``ac_update`` - the product-form adaptive Cartesian sampler;
  * ``fair_draw``        - fair draws from weighted samples;
  * ``overlaps_qv``      - Q, U, V of eq. (QUV) from modes and data.

Pins: ``tests/test_oracle_pins.py``.  Parity unpinned: EM trajectories with
more than one component, the in-support mass estimates (Monte Carlo).
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

MAXC, MAXD = 16, 7
C_SI = 299792458.0


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP, no fast-math)."""
    import subprocess
    src = os.path.join(_HERE, "ile_oracle.c")
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-std=c11", "-fPIC", "-shared",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Problem(C.Structure):
    _fields_ = [("n_det", C.c_int), ("n_modes", C.c_int), ("n_time", C.c_int),
                ("mode_l", C.POINTER(C.c_int)), ("mode_m", C.POINTER(C.c_int)),
                ("det_pos", C.POINTER(C.c_double)), ("det_resp", C.POINTER(C.c_double)),
                ("gmst", C.c_double), ("tau0", C.c_double), ("dt", C.c_double),
                ("Q", C.POINTER(C.c_double)), ("U", C.POINTER(C.c_double)),
                ("V", C.POINTER(C.c_double)), ("d_ref", C.c_double)]


class _Marg(C.Structure):
    _fields_ = [("ln_L", C.c_double), ("ln_sigma", C.c_double), ("n_eff", C.c_double),
                ("n_ess", C.c_double), ("max_lw", C.c_double), ("argmax", C.c_int64),
                ("n", C.c_int64), ("n_nonfinite", C.c_int64)]


class _Prior(C.Structure):
    _fields_ = [("t_window", C.c_double), ("d_min", C.c_double), ("d_max", C.c_double),
                ("dist_marg", C.c_int), ("d_ref", C.c_double)]


class _Gmm(C.Structure):
    _fields_ = [("n_comp", C.c_int), ("n_dim", C.c_int), ("dims", C.c_int * MAXD),
                ("weight", C.c_double * MAXC), ("mean", (C.c_double * MAXD) * MAXC),
                ("cov", ((C.c_double * MAXD) * MAXD) * MAXC), ("ln_Z", C.c_double * MAXC),
                ("eps_def", C.c_double), ("shear", C.c_int)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"oracle library missing ({_LIB_PATH}); run oracle.build()")
        L = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.orc_antenna.argtypes = [dp, C.c_double, C.c_double, C.c_double, C.c_double, dp, dp]
        L.orc_delay.argtypes = [dp, C.c_double, C.c_double, C.c_double]
        L.orc_delay.restype = C.c_double
        L.orc_wigner_d.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double]
        L.orc_wigner_d.restype = C.c_double
        L.orc_lagrange4.argtypes = [C.c_double, dp]
        L.orc_sample_tau.argtypes = [C.POINTER(_Problem), dp, dp]
        L.orc_lnL_qhat.argtypes = [C.POINTER(_Problem), dp, dp, dp, dp, dp]
        L.orc_lnL.argtypes = [C.POINTER(_Problem), C.c_int64, dp, C.c_int64, dp, dp, dp, C.c_int]
        L.orc_marginalize.argtypes = [C.c_int64, dp, C.POINTER(_Marg)]
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                        C.POINTER(C.c_uint32)]
        L.orc_ln_prior.argtypes = [C.POINTER(_Prior), dp]
        L.orc_ln_prior.restype = C.c_double
        L.orc_draw_prior.argtypes = [C.POINTER(_Prior), C.c_uint64, C.c_uint32, C.c_int64,
                                     C.c_int64, dp, C.c_int64, dp]
        L.orc_draw_av.argtypes = [C.POINTER(_Prior), C.c_int, C.POINTER(C.c_int), C.c_int, C.c_int64,
                                  C.POINTER(C.c_int32), C.c_uint64, C.c_uint32, C.c_int64, C.c_int64, dp,
                                  C.c_int64, dp]
        L.orc_draw_ac.argtypes = [C.POINTER(_Prior), C.c_int, C.POINTER(C.c_int), C.c_int, dp, dp, dp,
                                  C.c_uint64, C.c_uint32, C.c_int64, C.c_int64, dp, C.c_int64, dp,
                                  C.POINTER(C.c_int32)]
        L.orc_gmm_comp_logpdf.argtypes = [C.POINTER(_Prior), C.POINTER(_Gmm), C.c_int, dp]
        L.orc_gmm_comp_logpdf.restype = C.c_double
        L.orc_gmm_ln_ps.argtypes = [C.POINTER(_Prior), C.POINTER(_Gmm), dp]
        L.orc_gmm_ln_ps.restype = C.c_double
        L.orc_gmm_ln_ps_n.argtypes = [C.POINTER(_Prior), C.POINTER(_Gmm), dp, C.c_int]
        L.orc_gmm_ln_ps_n.restype = C.c_double
        L.orc_draw_gmm.argtypes = [C.POINTER(_Prior), C.POINTER(_Gmm), C.c_uint64, C.c_uint32,
                                   C.c_int64, C.c_int64, dp, C.c_int64, dp]
        L.orc_gmm_inbox_mass.argtypes = [C.POINTER(_Prior), C.POINTER(_Gmm), C.c_int, C.c_uint64,
                                         C.c_uint32, C.c_int64]
        L.orc_gmm_inbox_mass.restype = C.c_double
        L.orc_gmm_ln_ps_batch.argtypes = [C.POINTER(_Prior), C.POINTER(_Gmm), C.c_int64, dp, C.c_int64, dp]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


# ------------------------------------------------------------------ geometry
def antenna(resp, ra, dec, psi, gmst):
    """(F+, Fx) of one detector by the tensor definition."""
    r = np.ascontiguousarray(resp, dtype=np.float64)
    fp, fx = C.c_double(), C.c_double()
    lib().orc_antenna(_dp(r), ra, dec, psi, gmst, C.byref(fp), C.byref(fx))
    return fp.value, fx.value


def delay(pos, ra, dec, gmst):
    """x . n_hat / c (s); the detector time is t - delay."""
    p = np.ascontiguousarray(pos, dtype=np.float64)
    return lib().orc_delay(_dp(p), ra, dec, gmst)


def wigner_d(l, mp, m, beta):
    return lib().orc_wigner_d(l, mp, m, beta)


def sylm(l, m, theta, phi):
    """-2Y_lm(theta, phi)."""
    return math.sqrt((2 * l + 1) / (4 * math.pi)) * wigner_d(l, m, 2, theta) * complex(
        math.cos(m * phi), math.sin(m * phi))


def lagrange4(f):
    w = np.zeros(4)
    lib().orc_lagrange4(f, _dp(w))
    return w


# ------------------------------------------------------------------ problem
class _Holder:
    """Keeps the numpy buffers behind an orc_problem alive."""

    def __init__(self, prob):
        K, n = prob.n_det, prob.n_modes
        if K > 8 or n > 32:
            raise ValueError("oracle supports at most 8 detectors and 32 modes")
        self.ml = np.array([l for l, _ in prob.modes], dtype=np.int32)
        self.mm = np.array([m for _, m in prob.modes], dtype=np.int32)
        self.pos = np.ascontiguousarray(prob.det_pos, dtype=np.float64)
        self.resp = np.ascontiguousarray(prob.det_resp, dtype=np.float64)
        self.Q = np.ascontiguousarray(np.asarray(prob.Q, dtype=np.complex128)).view(np.float64)
        self.U = np.ascontiguousarray(np.asarray(prob.U, dtype=np.complex128)).view(np.float64)
        self.V = None if prob.V is None else np.ascontiguousarray(
            np.asarray(prob.V, dtype=np.complex128)).view(np.float64)
        ip = C.POINTER(C.c_int)
        self.s = _Problem(K, n, prob.Q.shape[-1], self.ml.ctypes.data_as(ip),
                          self.mm.ctypes.data_as(ip), _dp(self.pos), _dp(self.resp),
                          prob.gmst, prob.tau0, prob.dt, _dp(self.Q), _dp(self.U),
                          _dp(self.V) if self.V is not None else C.POINTER(C.c_double)(),
                          prob.d_ref)


def lnL(prob, theta, threads=None, return_terms=False):
    """Per-sample lnL (window Q, Lagrange cubic).  theta: [7][n] (upcast to FP64)."""
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
    n = th.shape[1]
    h = _Holder(prob)
    out = np.empty(n)
    T1 = np.empty(n) if return_terms else None
    T2 = np.empty(n) if return_terms else None
    nt = threads if threads is not None else (os.cpu_count() or 1)
    lib().orc_lnL(C.byref(h.s), n, _dp(th), n, _dp(out),
                  _dp(T1) if T1 is not None else C.POINTER(C.c_double)(),
                  _dp(T2) if T2 is not None else C.POINTER(C.c_double)(), nt)
    if return_terms:
        return out, T1, T2
    return out


def tmarg_grid(prob, oversample=4):
    """Nodes of the time integral: t_j = j dt/R, |j| <= floor(R t_w / dt)
    (relative to the reference time), each with weight dt / (R 2 t_w) against
    the uniform time prior on [-t_w, t_w]."""
    R = int(oversample)
    J = int(math.floor(R * prob.t_window / prob.dt + 1e-9))
    j = np.arange(-J, J + 1)
    return j * (prob.dt / R), math.log(prob.dt / (R * 2.0 * prob.t_window))


def lnL_tmarg(prob, theta, oversample=4, threads=None):
    """Time-marginalised likelihood: the (time) x (extrinsic) array of
    eq. (lnL:MatrixForm) integrated over the geocentric time prior by the
    rectangle rule on the nodes of ``tmarg_grid``:
        ln L_t = ln sum_j (dt / (R 2 t_w)) exp lnL(theta with t = t_j).
    The t row of theta is ignored.  Every node is the pointwise oracle lnL."""
    th = np.asarray(theta, dtype=np.float64)
    n = th.shape[1]
    tj, lnw = tmarg_grid(prob, oversample)
    nt = len(tj)
    big = np.repeat(th, nt, axis=1)
    big[2] = np.tile(tj, n)
    L = lnL(prob, big, threads=threads).reshape(n, nt)
    m = np.max(L, axis=1)
    out = np.full(n, -np.inf)
    fin = np.isfinite(m)
    out[fin] = m[fin] + np.log(np.sum(np.exp(L[fin] - m[fin, None]), axis=1)) + lnw
    return out


def lnL_tmarg_dist(prob, theta, oversample=1, threads=None, d_min=None, d_max=None):
    """Time- and distance-marginalised likelihood: the time nodes of
    ``tmarg_grid`` with, at each node, the distance integral of
    ``ln_dist_marg`` (adaptive quadrature) in place of a fixed distance:
        ln L_{t,D} = ln sum_j (dt / (R 2 t_w)) L_D(T1(t_j), T2),
    T1, T2 at s = 1 (D = d_ref) from the pointwise oracle.  The t and D rows
    of theta are ignored.  Slow: one quadrature per node."""
    th = np.array(theta, dtype=np.float64, copy=True)
    th[3] = prob.d_ref
    n_s = th.shape[1]
    tj, lnw = tmarg_grid(prob, oversample)
    nt = len(tj)
    d_min = prob.d_min if d_min is None else d_min
    d_max = prob.d_max if d_max is None else d_max
    out = np.full(n_s, -np.inf)
    for i in range(n_s):
        big = np.repeat(th[:, i:i + 1], nt, axis=1)
        big[2] = tj
        L, T1, T2 = lnL(prob, big, threads=threads, return_terms=True)
        fin = np.isfinite(L)
        if not np.any(fin):
            continue
        t2 = float(T2[fin][0])
        vals = np.array([ln_dist_marg(a, t2, d_ref=prob.d_ref, d_min=d_min, d_max=d_max) for a in T1[fin]])
        m = np.max(vals)
        out[i] = m + math.log(np.sum(np.exp(vals - m))) + lnw
    return out


def sample_tau(prob, th7):
    h = _Holder(prob)
    t = np.ascontiguousarray(th7, dtype=np.float64)
    tau = np.zeros(prob.n_det)
    lib().orc_sample_tau(C.byref(h.s), _dp(t), _dp(tau))
    return tau


def exact_Q(f, df, hlm, data_k, tau, psd=1.0, f_lo=20.0, f_hi=1024.0):
    """Q_lm(tau) = 2 sum_f df e^{2 pi i f tau} conj(h~_lm(f)) d~(f) / S over the band (eq. QUV)."""
    band = (np.abs(f) >= f_lo) & (np.abs(f) <= f_hi)
    ph = np.exp(2j * np.pi * f[band] * tau)
    return 2.0 * df * (np.conj(hlm[:, band]) @ (ph * data_k[band])) / psd


def lnL_exact(prob, th7, f, df, hlm, data):
    """lnL at one sample with Q evaluated exactly at each detector time (no window)."""
    th = np.ascontiguousarray(th7, dtype=np.float64)
    tau = sample_tau(prob, th)
    qh = np.stack([exact_Q(f, df, hlm, data[k], tau[k]) for k in range(prob.n_det)])
    qri = np.ascontiguousarray(qh.astype(np.complex128)).view(np.float64)
    h = _Holder(prob)
    l, t1, t2 = C.c_double(), C.c_double(), C.c_double()
    lib().orc_lnL_qhat(C.byref(h.s), _dp(th), _dp(qri), C.byref(l), C.byref(t1), C.byref(t2))
    return l.value, t1.value, t2.value


# ------------------------------------------------------------- marginalise
def marginalize(lw):
    """Monte Carlo estimator of eq. (lnL:MonteCarlo) with eq. (neff) on given log-weights."""
    a = np.ascontiguousarray(np.asarray(lw, dtype=np.float64))
    m = _Marg()
    lib().orc_marginalize(len(a), _dp(a), C.byref(m))
    return {k: getattr(m, k) for k, _ in _Marg._fields_}


# ------------------------------------------------------------------- draws
def philox(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return list(o)


def make_prior(t_window=0.028, d_min=1.0, d_max=3000.0, dist_marg=False, d_ref=100.0):
    return _Prior(t_window, d_min, d_max, int(dist_marg), d_ref)


def ln_prior(prior, th7):
    t = np.ascontiguousarray(th7, dtype=np.float64)
    return lib().orc_ln_prior(C.byref(prior), _dp(t))


def draw_prior(prior, seed, rnd, i0, n):
    th = np.empty((7, n))
    lp = np.empty(n)
    lib().orc_draw_prior(C.byref(prior), seed, rnd, i0, n, _dp(th), n, _dp(lp))
    return th, lp


def make_gmm(weights, means, covs, dims, ln_Z=None, eps_def=0.05, shear=0):
    """Mixture over the theta columns ``dims``; with shear = +-1 (columns 5 and
    6 both in ``dims``) the means and covariances are in the coordinates of
    ``shear_theta``."""
    if shear and not (5 in dims and 6 in dims):
        raise ValueError("a sheared mixture needs both phase columns")
    g = _Gmm()
    g.shear = int(shear)
    nc, nd = len(weights), len(dims)
    g.n_comp, g.n_dim = nc, nd
    for a, d in enumerate(dims):
        g.dims[a] = d
    for j in range(nc):
        g.weight[j] = float(weights[j])
        for a in range(nd):
            g.mean[j][a] = float(means[j][a])
            for b in range(nd):
                g.cov[j][a][b] = float(covs[j][a][b])
        g.ln_Z[j] = 0.0 if ln_Z is None else float(ln_Z[j])
    g.eps_def = eps_def
    return g


def gmm_comp_logpdf(prior, g, j, th7):
    t = np.ascontiguousarray(th7, dtype=np.float64)
    return lib().orc_gmm_comp_logpdf(C.byref(prior), C.byref(g), j, _dp(t))


def gmm_ln_ps(prior, g, th7, attempts=64):
    """ln of the density of a ``draw_gmm`` draw: the mixture term of each
    component scaled by 1 - (1 - Z_j)^attempts, the prior term carrying the
    defensive weight plus the draws whose attempts all failed
    (attempts <= 0: unlimited attempts)."""
    t = np.ascontiguousarray(th7, dtype=np.float64)
    return lib().orc_gmm_ln_ps_n(C.byref(prior), C.byref(g), _dp(t), int(attempts))


def draw_gmm(prior, g, seed, rnd, i0, n):
    th = np.empty((7, n))
    lr = np.empty(n)
    lib().orc_draw_gmm(C.byref(prior), C.byref(g), seed, rnd, i0, n, _dp(th), n, _dp(lr))
    return th, lr


def gmm_ln_ps_batch(prior, g, theta):
    """``gmm_ln_ps`` of every column of theta [7][n]."""
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
    out = np.empty(th.shape[1])
    lib().orc_gmm_ln_ps_batch(C.byref(prior), C.byref(g), th.shape[1], _dp(th), th.shape[1], _dp(out))
    return out


def shear_theta(theta, shear):
    """Mixture coordinates: column 6 replaced by (psi + shear phi_c) mod pi.
    For a face-on source the likelihood depends on the two phases nearly only
    through psi + phi_c (face-off: psi - phi_c), a ridge along phi_c at fixed
    y.  The map is a shear of the (phi_c, psi) torus with unit Jacobian, so
    densities carry over unchanged."""
    th = np.array(theta, dtype=np.float64, copy=True)
    if shear:
        y = th[6] + shear * th[5]
        th[6] = y - math.pi * np.floor(y / math.pi)
    return th


PHASE_SHEAR_MIN_COS = 0.5


def phase_shear_sign(theta, lw):
    """Shear of a first fit, from the highest-weight sample (lowest index
    among ties): +1 if its cos iota >= 0.5 (face-on: the m = +2 end of each
    multiplet dominates, ((1 + cos i)/(1 - cos i))^2 >= 9, and the likelihood
    ridge runs along psi + phi_c = const), -1 if cos iota <= -0.5 (face-off),
    0 otherwise (no single ridge) or if no weight is finite."""
    lw = np.asarray(lw, dtype=np.float64)
    if not np.any(np.isfinite(lw)):
        return 0
    key = np.where(np.isfinite(lw), lw, -np.inf)
    i = int(np.argsort(-key, kind="stable")[0])
    c = float(np.asarray(theta)[4][i])
    return 1 if c >= PHASE_SHEAR_MIN_COS else (-1 if c <= -PHASE_SHEAR_MIN_COS else 0)


def pool_mixture_lw(prior, proposals, thetas, lnLs):
    """Log-weights of every sample of an adaptive run pooled as draws of the
    equal-weight mixture of the rounds' proposals: eq. (lnL:MonteCarlo) with
    p_s(x) = (1/R) sum_q p_s,q(x) for all R rounds of equal size.  Round q
    drew ``thetas[q]`` from ``proposals[q]`` (None: the prior) and has
    likelihoods ``lnLs[q]``; returns the concatenated
      lw = lnL + ln p - ln( (1/R) sum_q p_s,q ).
    Each sample's weight is at most R times its likelihood, since the prior
    is one of the mixture's members."""
    R = len(thetas)
    out = []
    for r in range(R):
        th = np.asarray(thetas[r], dtype=np.float64)
        lp = np.array([ln_prior(prior, th[:, i]) for i in range(th.shape[1])])
        terms = []
        for q in range(R):
            if proposals[q] is None:
                terms.append(np.zeros(th.shape[1]))
            else:
                terms.append(gmm_ln_ps_batch(prior, proposals[q], th) - lp)
        T = np.stack(terms)
        m = np.max(T, axis=0)
        lmix = m + np.log(np.sum(np.exp(T - m), axis=0)) - math.log(R)
        out.append(np.asarray(lnLs[r], dtype=np.float64) - lmix)
    return np.concatenate(out)


def gmm_inbox_mass(prior, g, j, seed, rnd, m=1 << 16):
    return lib().orc_gmm_inbox_mass(C.byref(prior), C.byref(g), j, seed, rnd, m)


# ---------------------------------------------------------- adaptive volume
# Section "Adaptive volume integration" (the AV integrator), in the prior's
# CDF coordinates u in [0,1)^d (theta = inverse-CDF map of u): a grid of nb
# bins per sampled dimension, a set of active cells, samples uniform over the
# active cells (so ln p - ln p_s = ln V, V the active volume), and after each
# round a likelihood threshold, a refined bin count (eq. nbins_V) and the new
# active cells.  Readings where the section is silent:
#   * the live points of an update are the n samples of the round just drawn;
#   * the enclosed probability is measured on the fixed-point masses
#     q_i = floor(exp(lnL_i - max lnL) 2^40) (integer sums, so the threshold
#     does not depend on summation order);
#   * the threshold is the largest lnL value at or above which both at least
#     min(ceil(p_thr * total), total) of the fixed-point mass (p_thr * total
#     is formed in FP64, whose rounding can exceed the integer total) and at
#     least min(n_min_live, n_finite) samples lie (the "fixed large number of
#     highest points" of early iterations);
#   * n_bins = ceil((1/dV)^(1/d)), clamped to [1, max_bins], with
#     dV = V n_min / (n sqrt(n_min)) the Monte Carlo error of the live volume;
#   * the new active cells are the cells of the refined grid holding a sample
#     at or above the threshold, in order of their first such sample.
AV_MASS_BITS = 40


class AvGrid:
    def __init__(self, nb, cells, dims):
        self.nb = int(nb)
        self.cells = np.ascontiguousarray(np.asarray(cells, dtype=np.int32).reshape(-1, len(dims)))
        self.dims = list(dims)

    @property
    def d(self):
        return len(self.dims)

    @property
    def n_cells(self):
        return self.cells.shape[0]

    @property
    def ln_vol(self):
        return math.log(self.n_cells) - self.d * math.log(self.nb)


def av_dims(dist_marg=False):
    return [0, 1, 2, 4, 5, 6] if dist_marg else list(range(7))


def av_init(dist_marg=False):
    """The whole cube: one cell of a one-bin grid."""
    dims = av_dims(dist_marg)
    return AvGrid(1, np.zeros((1, len(dims)), dtype=np.int32), dims)


def draw_av(prior, grid, seed, rnd, i0, n):
    """Samples uniform over the active cells (orc_draw_av): theta [7][n] and u [d][n]."""
    th = np.empty((7, n))
    u = np.empty((grid.d, n))
    dims = (C.c_int * grid.d)(*grid.dims)
    cells = np.ascontiguousarray(grid.cells, dtype=np.int32)
    lib().orc_draw_av(C.byref(prior), grid.d, dims, grid.nb, grid.n_cells,
                      cells.ctypes.data_as(C.POINTER(C.c_int32)), seed, rnd, i0, n, _dp(th), n, _dp(u))
    return th, u


def av_mass(lnL_finite):
    m = float(np.max(lnL_finite))
    return np.floor(np.exp(lnL_finite - m) * float(1 << AV_MASS_BITS)).astype(np.uint64)


def av_threshold(lnL, p_thr, n_min_live):
    """Likelihood threshold of one round: (lnL_thr, n_min), or None when no
    sample is finite.  Sorts the finite samples by lnL (descending) and takes
    the lower of the value where the cumulative fixed-point mass first reaches
    ceil(p_thr * total) and the k-th largest value, k = min(n_min_live, n)."""
    lnL = np.asarray(lnL, dtype=np.float64)
    x = lnL[np.isfinite(lnL)]
    if x.size == 0:
        return None
    q = av_mass(x)
    order = np.argsort(-x, kind="stable")
    cum = np.cumsum(q[order], dtype=np.uint64)
    target = min(np.uint64(math.ceil(p_thr * float(cum[-1]))), cum[-1])
    k_mass = int(np.argmax(cum >= target))
    k = min(int(n_min_live), x.size)
    thr = min(float(x[order[k_mass]]), float(x[order[k - 1]]))
    return thr, int(np.count_nonzero(x >= thr))


def av_refine_bins(n_min, n, ln_vol, d, max_bins):
    """eq. (nbins_V) with dV = V n_min / (n sqrt(n_min))."""
    ln_dv = ln_vol + 0.5 * math.log(n_min) - math.log(n)
    x = math.exp(-ln_dv / d)
    return int(min(max(math.ceil(x - 1e-9), 1), max_bins))


def av_cells(u_top, nb):
    """Cells of the nb-bin grid holding the points u_top [d][m] (index order),
    each once, in order of first appearance."""
    if u_top.shape[1] == 0:
        return np.zeros((0, u_top.shape[0]), dtype=np.int32)
    c = np.minimum(np.floor(u_top * nb), nb - 1).astype(np.int32).T
    _, first = np.unique(c, axis=0, return_index=True)
    return c[np.sort(first)]


def av_update(grid, u, lnL, p_thr=0.999, n_min_live=1000, max_bins=511):
    """One refinement from a round's n samples (u [d][n], lnL [n]).  Returns
    (new grid, info); the grid is unchanged when no sample is finite."""
    lnL = np.asarray(lnL, dtype=np.float64)
    n = lnL.size
    r = av_threshold(lnL, p_thr, n_min_live)
    if r is None:
        return grid, {"lnL_thr": -math.inf, "n_min": 0, "n_live": n, "vol_mc": 0.0}
    thr, n_min = r
    nb = av_refine_bins(n_min, n, grid.ln_vol, grid.d, max_bins)
    top = np.nonzero(np.isfinite(lnL) & (lnL >= thr))[0]
    cells = av_cells(np.asarray(u)[:, top], nb)
    info = {"lnL_thr": thr, "n_min": n_min, "n_live": n, "vol_mc": math.exp(grid.ln_vol) * n_min / n}
    return AvGrid(nb, cells, grid.dims), info


# ------------------------------------------------------ adaptive Cartesian
# The product-form adaptive Cartesian (AC) sampler: one adaptive histogram per
# sampled coordinate of the prior's CDF cube (nb = 64 equal bins), drawn by
# the inverse CDF of each piecewise-constant marginal, so p_s / p is the
# product of nb pi[k][b_k].  Readings (the paper only says each marginal is
# updated after a block of evaluations to follow the integrand's support):
#   * the update replaces every marginal by the histogram of the round's
#     fixed-point masses q_i (the AV/fair-draw masses) over that coordinate's
#     bins, mixed with the uniform: pi = (1 - floor) h / total + floor / nb,
#     floor = 0.1 (p_s stays positive everywhere, so every round is unbiased);
#   * cumulative sums are sequential in bin order with the last set to 1;
#   * with no finite sample the marginals are kept.
AC_BINS = 64


class AcState:
    def __init__(self, pi, dims):
        self.pi = np.ascontiguousarray(np.asarray(pi, dtype=np.float64).reshape(len(dims), AC_BINS))
        self.dims = list(dims)
        c = np.cumsum(self.pi, axis=1)
        c[:, -1] = 1.0
        self.cum = np.ascontiguousarray(c)
        self.lnbp = np.ascontiguousarray(np.log(AC_BINS * self.pi))

    @property
    def d(self):
        return len(self.dims)


def ac_init(dist_marg=False, dims=None):
    dims = av_dims(dist_marg) if dims is None else list(dims)
    return AcState(np.full((len(dims), AC_BINS), 1.0 / AC_BINS), dims)


def draw_ac(prior, st, seed, rnd, i0, n):
    """theta [7][n], ln p - ln p_s [n], bins [d][n]."""
    th = np.empty((7, n))
    lr = np.empty(n)
    bins = np.empty((st.d, n), dtype=np.int32)
    dims = (C.c_int * st.d)(*st.dims)
    lib().orc_draw_ac(C.byref(prior), st.d, dims, AC_BINS, _dp(st.pi), _dp(st.cum), _dp(st.lnbp), seed, rnd,
                      i0, n, _dp(th), n, _dp(lr), bins.ctypes.data_as(C.POINTER(C.c_int32)))
    return th, lr, bins


def ac_update(st, bins, lw, floor=0.1):
    """New marginals from one round's bins [d][n] and log-weights [n]."""
    lw = np.asarray(lw, dtype=np.float64)
    fin = np.isfinite(lw)
    if not fin.any():
        return st
    q = np.zeros(lw.size, dtype=np.uint64)
    q[fin] = av_mass(lw[fin])
    total = int(np.sum(q, dtype=np.uint64))
    pi = np.empty((st.d, AC_BINS))
    for k in range(st.d):
        h = np.zeros(AC_BINS, dtype=np.uint64)
        np.add.at(h, bins[k], q)
        pi[k] = (1.0 - floor) * (h.astype(np.float64) / float(total)) + floor / AC_BINS
    return AcState(pi, st.dims)


# ------------------------------------------------------ Q, U, V precompute
def overlaps_qv(hlm, data, inv_psd, df, f_lo, f_hi, n_time, win_half):
    """The inner products of eq. (QUV) from the modes and the data, by their
    definitions over the two-sided frequency grid f_m = m' df (m' the signed
    index of FFT order), restricted to f_lo <= |f| <= f_hi, with
    <a|b>_k = 2 df sum_f conj(a(f)) b(f) w_k(f), w_k = 1/S_k (None: 1):
      Q[k][a][i] = 2 df sum_f e^{2 pi i f tau_i} conj(h_a(f)) d_k(f) w_k(f),
                   tau_i = (i - win_half) / (n df), the phase taken as
                   2 pi ((m' (i - win_half)) mod n) / n;
      U[k][a][b] = <h_a|h_b>_k;
      V[k][a][b] = <h_a^*|h_b>_k = 2 df sum_f h_a(-f) h_b(f) w_k(f).
    hlm [n_modes][n], data [n_det][n] (complex), inv_psd [n_det][n] or None."""
    hlm = np.asarray(hlm, dtype=np.complex128)
    data = np.asarray(data, dtype=np.complex128)
    na, n = hlm.shape
    nd = data.shape[0]
    w = np.ones((nd, n)) if inv_psd is None else np.asarray(inv_psd, dtype=np.float64)
    ms = np.fft.fftfreq(n, d=1.0 / n).round().astype(np.int64)
    f = ms * df
    band = np.nonzero((np.abs(f) >= f_lo) & (np.abs(f) <= f_hi))[0]
    neg = (n - band) % n
    j = np.arange(n_time, dtype=np.int64) - win_half
    E = np.exp(2j * np.pi * ((np.outer(j, ms[band]) % n) / n))
    Q = np.empty((nd, na, n_time), dtype=np.complex128)
    U = np.empty((nd, na, na), dtype=np.complex128)
    V = np.empty((nd, na, na), dtype=np.complex128)
    hb = hlm[:, band]
    for k in range(nd):
        wk = w[k, band]
        x = 2.0 * df * np.conj(hb) * (data[k, band] * wk)[None, :]
        Q[k] = (E @ x.T).T
        U[k] = 2.0 * df * (np.conj(hb) * wk) @ hb.T
        V[k] = 2.0 * df * (hlm[:, neg] * wk) @ hb.T
    return Q, U, V


# --------------------------------------------------------------- fair draws
# A fair draw from weighted samples (the final step of an ILE run and of the
# posterior construction: sample locations with weights w, then a fair draw
# from them).  Reading: k independent draws with replacement, index i with
# probability q_i / sum q, q_i = floor(exp(lw_i - max lw) 2^40) the same
# fixed-point masses as the AV threshold (0 for non-finite lw).  Draw j uses
# the Philox words of counter (j lo, j hi, round, 16 * 5 + 0) under the key:
# r = w0 2^32 + w1 (64 bits), target = floor(r * total / 2^64), and the index
# is the first i whose inclusive cumulative mass exceeds the target.
FAIR_ATTEMPT = 5


def fair_draw(lw, seed, rnd, k):
    """Indices [k] (int64); -1 for every draw when no sample has mass."""
    lw = np.asarray(lw, dtype=np.float64)
    fin = np.isfinite(lw)
    q = np.zeros(lw.size, dtype=np.uint64)
    if fin.any():
        q[fin] = av_mass(lw[fin])
    cum = np.cumsum(q, dtype=np.uint64)
    total = int(cum[-1]) if cum.size else 0
    out = np.full(k, -1, dtype=np.int64)
    if total == 0:
        return out
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    for j in range(k):
        w = philox((j & 0xFFFFFFFF, (j >> 32) & 0xFFFFFFFF, rnd, 16 * FAIR_ATTEMPT), key)
        r = (w[0] << 32) | w[1]
        target = (r * total) >> 64
        out[j] = int(np.searchsorted(cum, np.uint64(target), side="right"))
    return out


# ----------------------------------------------------------------------- EM
PERIODS = {0: 2 * math.pi, 5: 2 * math.pi, 6: math.pi}


def col_range(col, t_window=0.028, d_min=1.0, d_max=3000.0):
    return {0: 2 * math.pi, 1: math.pi, 2: 2 * t_window, 3: d_max - d_min, 4: 2.0,
            5: 2 * math.pi, 6: math.pi}[col]


def wrap_diff(d, period):
    if period <= 0:
        return d
    r = d - period * np.floor(d / period)
    return np.where(r > 0.5 * period, r - period, r)


def _wrapped(X, mu, dims):
    return np.stack([wrap_diff(X[:, a] - mu[a], PERIODS.get(c, 0.0)) for a, c in enumerate(dims)],
                    axis=1)


def _logpdf_rows(D, cov):
    Lc = np.linalg.cholesky(cov)
    y = np.linalg.solve(Lc, D.T)
    return -0.5 * np.sum(y * y, axis=0) - np.sum(np.log(np.diag(Lc))) - 0.5 * D.shape[1] * math.log(2 * math.pi)


def first_fit_candidates(n_comp):
    """How many of the highest-weight samples the first fit scans for
    distinct means (a bounded top-k selection)."""
    return 2 * n_comp


def em_init(theta, lw, dims, n_comp=8, shear=0, **rng_kw):
    """First fit: means at the highest-weight distinct samples among the
    2 n_comp highest-weight ones (ties: lower index first), scanned in that
    order; if fewer than n_comp are distinct the last one found is repeated.
    Common weighted covariance (differences wrapped about the best sample),
    equal weights.  shear != 0: all of it in the coordinates of ``shear_theta``."""
    X = shear_theta(theta, shear)[dims].T
    lw = np.asarray(lw, dtype=np.float64)
    fin = np.isfinite(lw)
    w = np.where(fin, np.exp(np.where(fin, lw, -np.inf) - np.max(lw[fin])), 0.0)
    key = np.where(fin, lw, -np.inf)
    order = np.argsort(-key, kind="stable")[:first_fit_candidates(n_comp)]
    means = []
    for i in order:
        if not fin[i]:
            break
        if any(np.array_equal(X[i], m) for m in means):
            continue
        means.append(X[i].copy())
        if len(means) == n_comp:
            break
    while len(means) < n_comp:
        means.append(means[-1].copy())
    Dd = _wrapped(X, means[0], dims)
    wn = w / w.sum()
    mu = wn @ Dd
    cov = (Dd * wn[:, None]).T @ Dd - np.outer(mu, mu)
    cov = cov + np.diag([1e-8 * col_range(c, **rng_kw) ** 2 for c in dims])
    return (np.full(n_comp, 1.0 / n_comp), np.array(means), np.array([cov] * n_comp))


def em_step(theta, lw, dims, weights, means, covs, shear=0, **rng_kw):
    """One weighted EM iteration.

    w_i = e^{lw_i - max lw}; responsibilities r_ij from the untruncated
    components pi_j N(wrap(x_i - mu_j); 0, Sigma_j); M-step with differences
    wrapped about the current mu_j; Sigma_j += 1e-8 diag(range^2).  A component
    with zero total weight keeps its mean and covariance.  shear != 0: the
    samples are taken in the coordinates of ``shear_theta``.
    """
    X = shear_theta(theta, shear)[dims].T
    lw = np.asarray(lw, dtype=np.float64)
    fin = np.isfinite(lw)
    w = np.where(fin, np.exp(np.where(fin, lw, -np.inf) - np.max(lw[fin])), 0.0)
    nc = len(weights)
    logr = np.full((X.shape[0], nc), -np.inf)
    Ds = []
    for j in range(nc):
        Dj = _wrapped(X, means[j], dims)
        Ds.append(Dj)
        if weights[j] > 0:
            logr[:, j] = math.log(weights[j]) + _logpdf_rows(Dj, covs[j])
    mx = np.max(logr, axis=1, keepdims=True)
    r = np.exp(logr - mx)
    r /= r.sum(axis=1, keepdims=True)
    floor = np.diag([1e-8 * col_range(c, **rng_kw) ** 2 for c in dims])
    W = (w[:, None] * r).sum(axis=0)
    new_w, new_m, new_c = np.zeros(nc), np.array(means, dtype=float).copy(), np.array(covs, dtype=float).copy()
    tot = W.sum()
    for j in range(nc):
        new_w[j] = W[j] / tot
        if W[j] <= 0:
            continue
        g = w * r[:, j]
        mj = (g @ Ds[j]) / W[j]
        dd = Ds[j] - mj
        new_c[j] = (dd * g[:, None]).T @ dd / W[j] + floor
        mu = np.array(means[j], dtype=float) + mj
        for a, c in enumerate(dims):
            P = PERIODS.get(c, 0.0)
            if P > 0:
                mu[a] = mu[a] - P * math.floor(mu[a] / P)
        new_m[j] = mu
    return new_w, new_m, new_c


def temper_beta(lw, frac):
    """Largest beta = 2^(-k/4), k = 0..47, with (sum w^beta)^2 / sum w^(2 beta)
    >= frac * (finite samples), w = e^{lw - max lw}; frac <= 0 gives 1."""
    if not frac > 0:
        return 1.0
    lw = np.asarray(lw, dtype=np.float64)
    fin = np.isfinite(lw)
    x = lw[fin] - np.max(lw[fin])
    target = frac * fin.sum()
    for k in range(48):
        b = 2.0 ** (-k / 4.0)
        w = np.exp(b * x)
        if w.sum() ** 2 / (w * w).sum() >= target:
            return b
    return 2.0 ** (-47 / 4.0)


def em_fit(theta, lw, dims, state=None, n_iter=8, n_comp=8, temper_ess=0.0, shear=0, **rng_kw):
    """Warm-started EM: ``n_iter`` iterations from ``state`` (or the first fit),
    on the tempered log-weights beta * lw (beta from ``temper_beta``), in the
    mixture coordinates of ``shear_theta``."""
    lw = np.asarray(lw, dtype=np.float64) * temper_beta(lw, temper_ess)
    if state is None:
        state = em_init(theta, lw, dims, n_comp=n_comp, shear=shear, **rng_kw)
    w, m, c = state
    for _ in range(n_iter):
        w, m, c = em_step(theta, lw, dims, w, m, c, shear=shear, **rng_kw)
    return w, m, c


# ------------------------------------------------------ distance marginal
def ln_dist_marg(T1, T2, d_ref=100.0, d_min=1.0, d_max=3000.0, prior="volume"):
    """ln of the distance integral of exp(s T1 - s^2 T2 / 4), s = d_ref/D,
    against p(D) = 3 D^2/(Dmax^3 - Dmin^3) ("volume") or uniform in s ("uniform_s").
    Adaptive quadrature in s, with the exponent shifted by its maximum."""
    from scipy.integrate import quad
    s_lo, s_hi = d_ref / d_max, d_ref / d_min

    def expo(s):
        return s * T1 - s * s * T2 / 4.0

    if prior == "volume":
        cst = 3.0 * d_ref ** 3 / (d_max ** 3 - d_min ** 3)

        def lnw(s):
            return math.log(cst) - 4.0 * math.log(s)
    else:
        def lnw(s):
            return -math.log(s_hi - s_lo)
    grid = np.exp(np.linspace(math.log(s_lo), math.log(s_hi), 4001))
    vals = np.array([expo(s) + lnw(s) for s in grid])
    s_star = min(max(2.0 * T1 / T2, s_lo), s_hi) if T2 > 0 else s_hi
    cands = list(grid) + [s_star]
    m = max(max(vals), expo(s_star) + lnw(s_star))
    pts = sorted({s_star, grid[int(np.argmax(vals))]})
    width = 2.0 / math.sqrt(T2) if T2 > 0 else (s_hi - s_lo)
    brk = sorted({min(max(p + k * width, s_lo), s_hi) for p in pts for k in (-40, -10, -3, 0, 3, 10, 40)})
    brk = [b for b in brk if s_lo < b < s_hi]
    edges = [s_lo] + brk + [s_hi]
    tot = 0.0
    for a, b in zip(edges[:-1], edges[1:]):
        v, _ = quad(lambda s: math.exp(expo(s) + lnw(s) - m), a, b, epsabs=0.0, epsrel=1e-13,
                    limit=500)
        tot += v
    del cands
    return m + math.log(tot)
