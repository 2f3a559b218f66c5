"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the property it pins and the passage it comes from.  None of
them re-types an oracle formula: they use closed forms, invariances, a
brute-force sum, an independent library routine, or the data model.
"""
import math

import numpy as np
import pytest

import chirpgen

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


@pytest.fixture(scope="module")
def recs():
    return chirpgen.load_injections()


def _event(recs, key, dets, n, mc=30.0, q=2.0, snr=20.0, noise=False, seed=7):
    probs, ev = chirpgen.build_event(recs[key] if isinstance(key, str) else key, dets, n, mc, q,
                                     snr, noise_seed=seed, noise=noise)
    p = probs[0]
    hlm = chirpgen.modes_fd(ev["f"], p.modes, mc, q, amp0=ev["amp0"])
    return p, ev, hlm


# --------------------------------------------------------------------- P1
@pytest.mark.parametrize("key,dets,n,q", [("c1", ["H", "L"], 5, 2.0),
                                          ("c2", ["H", "L", "V"], 9, 3.0),
                                          ("c3", ["H", "L", "V"], 17, 20.0)])
def test_P1_injection_lnL_is_half_rho2(orc, recs, key, dets, n, q):
    """Noiseless injection, exact Q: lnL(theta_inj) = rho^2/2, and the best
    distance scale 2 T1/T2 equals D_ref/D_inj (eq. def:lnL:Decomposed with the
    strain model h_k = F+ h+ + Fx hx, h = h+ - i hx).  rho^2 comes from the
    detector strains alone (no U, no Y).  Fails for F+ - iFx, a dropped V
    term or a misplaced conjugate."""
    p, ev, hlm = _event(recs, key, dets, n, q=q)
    th = np.array(recs[key]["theta"])
    l, t1, t2 = orc.lnL_exact(p, th, ev["f"], ev["df"], hlm, ev["data"])
    rho2 = chirpgen.network_snr2(ev["f"], ev["df"], ev["strain"])
    assert abs(rho2 - 400.0) < 1e-9
    assert abs(l - rho2 / 2) <= 1e-9 * rho2 / 2
    assert abs(2 * t1 / t2 - 100.0 / th[3]) <= 1e-9


def test_P1_conjugated_response_fails(orc, recs):
    """A planted mistake in the oracle's inputs (V conjugated, i.e. the
    V-term written with conj(V)) breaks P1: the pin sees a wrong V term."""
    p, ev, hlm = _event(recs, "c3", ["H", "L", "V"], 17, q=20.0)
    th = np.array(recs["c3"]["theta"])
    rho2 = chirpgen.network_snr2(ev["f"], ev["df"], ev["strain"])
    bad = p.__class__(**{**p.__dict__})
    bad.V = np.conj(p.V)   # planted: V conjugated
    l_bad, _, _ = orc.lnL_exact(bad, th, ev["f"], ev["df"], hlm, ev["data"])
    assert abs(l_bad - rho2 / 2) > 1e-3


# --------------------------------------------------------------------- P2
def test_P2_interpolant_exact_on_cubics(orc):
    """Lagrange cubic weights reproduce samples at f = 0 and cubic polynomials."""
    w0 = orc.lagrange4(0.0)
    assert np.allclose(w0, [0, 1, 0, 0], atol=0, rtol=0)
    rng = np.random.default_rng(1)
    for _ in range(50):
        c = rng.normal(size=4)
        f = rng.uniform(0, 1)
        poly = lambda x: c[0] + c[1] * x + c[2] * x * x + c[3] * x ** 3  # noqa: E731
        w = orc.lagrange4(f)
        val = sum(w[j] * poly(j - 1) for j in range(4))
        assert abs(val - poly(f)) <= 1e-12 * (1 + abs(poly(f)))
    assert abs(orc.lagrange4(0.37).sum() - 1.0) < 1e-15


def test_P2_window_lnL_matches_interpolated_exact(orc, recs):
    """The window path equals lnL with Q from the exact sum at the four stencil
    times, combined with the Lagrange weights (definition of the interpolant)."""
    p, ev, hlm = _event(recs, "c1", ["H", "L"], 5, noise=True)
    rng = np.random.default_rng(3)
    th = chirpgen.prior_samples(rng, 4)
    win = orc.lnL(p, th)
    for i in range(4):
        t7 = th[:, i]
        tau = orc.sample_tau(p, t7)
        qh = []
        for k in range(p.n_det):
            u = (tau[k] - p.tau0) / p.dt
            i0 = math.floor(u)
            w = orc.lagrange4(u - i0)
            qs = [orc.exact_Q(ev["f"], ev["df"], hlm, ev["data"][k], p.tau0 + (i0 - 1 + j) * p.dt)
                  for j in range(4)]
            qh.append(sum(w[j] * qs[j] for j in range(4)))
        import ctypes as C
        qri = np.ascontiguousarray(np.stack(qh).astype(np.complex128)).view(np.float64)
        h = orc._Holder(p)
        l = C.c_double()
        d = C.c_double()
        orc.lib().orc_lnL_qhat(C.byref(h.s), orc._dp(np.ascontiguousarray(t7)), orc._dp(qri),
                               C.byref(l), C.byref(d), C.byref(C.c_double()))
        assert abs(l.value - win[i]) <= 1e-9 * (1 + abs(win[i]))


# --------------------------------------------------------------------- P3/P4
def test_P3_psi_plus_pi_invariance(orc, recs):
    p, ev, hlm = _event(recs, "c2", ["H", "L", "V"], 9, noise=True)
    rng = np.random.default_rng(4)
    th = chirpgen.prior_samples(rng, 2000)
    th2 = th.copy()
    th2[6] += math.pi
    a, b = orc.lnL(p, th), orc.lnL(p, th2)
    assert np.all(np.abs(a - b) <= 1e-12 * (1 + np.abs(a)))


def test_P4_mode_set_invariances(orc):
    rng = np.random.default_rng(5)
    # {(2,+-2)}: (psi + pi/2, phi + pi/2) leaves F Y unchanged
    p = chirpgen.random_problem(rng, 5, ["H", "L", "V"])
    keep = [0, 4]
    p.modes = [p.modes[a] for a in keep]
    p.Q = p.Q[:, keep]
    p.U = p.U[:, keep][:, :, keep]
    p.V = p.V[:, keep][:, :, keep]
    th = chirpgen.prior_samples(rng, 1000)
    th2 = th.copy()
    th2[6] += math.pi / 2
    th2[5] += math.pi / 2
    a, b = orc.lnL(p, th), orc.lnL(p, th2)
    assert np.all(np.abs(a - b) <= 1e-11 * (1 + np.abs(a)))
    # even-m only: phi + pi invariance
    p = chirpgen.random_problem(rng, 5, ["H", "L"])
    keep = [0, 2, 4]
    p.modes = [p.modes[a] for a in keep]
    p.Q, p.U, p.V = p.Q[:, keep], p.U[:, keep][:, :, keep], p.V[:, keep][:, :, keep]
    th2 = th.copy()
    th2[5] += math.pi
    a, b = orc.lnL(p, th), orc.lnL(p, th2)
    assert np.all(np.abs(a - b) <= 1e-11 * (1 + np.abs(a)))
    # and a set with odd m is NOT phi + pi invariant
    p = chirpgen.random_problem(rng, 5, ["H", "L"])
    a, b = orc.lnL(p, th), orc.lnL(p, th2)
    assert np.max(np.abs(a - b)) > 1e-3


# --------------------------------------------------------------------- P5
def test_P5_sylm_closed_forms(orc):
    """-2Y_2m closed forms (Appendix on frame conventions uses -2Y_lm)."""
    rng = np.random.default_rng(6)
    for _ in range(20):
        th, ph = rng.uniform(0, math.pi), rng.uniform(0, 2 * math.pi)
        c, s = math.cos(th), math.sin(th)
        e = lambda m: complex(math.cos(m * ph), math.sin(m * ph))  # noqa: E731
        ref = {2: math.sqrt(5 / (64 * math.pi)) * (1 + c) ** 2 * e(2),
               1: math.sqrt(5 / (16 * math.pi)) * s * (1 + c) * e(1),
               0: math.sqrt(15 / (32 * math.pi)) * s * s,
               -1: math.sqrt(5 / (16 * math.pi)) * s * (1 - c) * e(-1),
               -2: math.sqrt(5 / (64 * math.pi)) * (1 - c) ** 2 * e(-2)}
        for m, v in ref.items():
            assert abs(orc.sylm(2, m, th, ph) - v) <= 1e-14


def test_P5_sylm_sum_rule_and_pole(orc):
    rng = np.random.default_rng(7)
    for l in (2, 3, 4):
        for th in rng.uniform(0, math.pi, 10):
            tot = sum(abs(orc.sylm(l, m, th, 0.3)) ** 2 for m in range(-l, l + 1))
            assert abs(tot - (2 * l + 1) / (4 * math.pi)) <= 1e-13
        for m in range(-l, l + 1):
            v = orc.sylm(l, m, 0.0, 0.4)
            if m == 2:
                assert abs(v) > 0.1
            else:
                assert abs(v) <= 1e-15


def test_P5_sylm_orthonormal(orc):
    """Gauss-Legendre in cos(theta) x uniform phi quadrature."""
    x, w = np.polynomial.legendre.leggauss(24)
    phis = np.linspace(0, 2 * math.pi, 20, endpoint=False)
    lms = [(l, m) for l in (2, 3, 4) for m in range(-l, l + 1)]
    vals = np.array([[[orc.sylm(l, m, math.acos(xi), ph) for ph in phis] for xi in x] for l, m in lms])
    G = np.einsum("aij,bij,i->ab", np.conj(vals), vals, w) * (2 * math.pi / len(phis))
    assert np.allclose(G, np.eye(len(lms)), atol=1e-12)


# --------------------------------------------------------------------- P6
def test_P6_antenna_identities(orc):
    rng = np.random.default_rng(8)
    for name in ("H", "L", "V"):
        pos, resp = chirpgen.detector(name)
        assert abs(np.trace(resp)) < 1e-15 and np.allclose(resp, resp.T)
        for _ in range(20):
            ra, dec, psi, g = rng.uniform(0, 6.28), rng.uniform(-1.5, 1.5), rng.uniform(0, 3.14), rng.uniform(0, 6.28)
            f0 = complex(*orc.antenna(resp, ra, dec, 0.0, g))
            f1 = complex(*orc.antenna(resp, ra, dec, psi, g))
            f2 = complex(*orc.antenna(resp, ra, dec, psi + math.pi / 2, g))
            assert abs(abs(f1) - abs(f0)) < 1e-14
            assert abs(f2 + f1) < 1e-14
            assert abs(f1 - f0 * complex(math.cos(2 * psi), -math.sin(2 * psi))) < 1e-14


def test_P6_antenna_textbook_detector_frame(orc):
    """Detector at the pole, arms along x and y: F+^2 + Fx^2 equals the
    detector-frame closed form (1/4)(1+cos^2 th)^2 cos^2 2ph + cos^2 th sin^2 2ph."""
    resp = 0.5 * (np.outer([1, 0, 0], [1, 0, 0]) - np.outer([0, 1, 0], [0, 1, 0]))
    rng = np.random.default_rng(9)
    for _ in range(50):
        th, ph, psi = rng.uniform(0, math.pi), rng.uniform(0, 2 * math.pi), rng.uniform(0, math.pi)
        fp, fx = orc.antenna(resp, ph, math.pi / 2 - th, psi, 0.0)
        ref = 0.25 * (1 + math.cos(th) ** 2) ** 2 * math.cos(2 * ph) ** 2 + math.cos(th) ** 2 * math.sin(2 * ph) ** 2
        assert abs(fp * fp + fx * fx - ref) < 1e-14
    fp, fx = orc.antenna(resp, 0.3, math.pi / 2, 0.2, 0.0)   # zenith
    assert abs(math.hypot(fp, fx) - 1.0) < 1e-14


def test_A3_zenith_arrives_first(orc):
    """A source at detector k's zenith (geocentric direction of x_k) reaches it
    |x_k|/c before the geocentre: tau_k - t = -|x_k|/c."""
    for name in ("H", "L", "V"):
        pos, _ = chirpgen.detector(name)
        r = np.linalg.norm(pos)
        dec = math.asin(pos[2] / r)
        ra = math.atan2(pos[1], pos[0]) + 1.1
        d = orc.delay(pos, ra, dec, 1.1)
        assert abs(d - r / chirpgen.C_SI) < 1e-15


# --------------------------------------------------------------------- P7
def test_P7_exactly_quadratic_in_s(orc, recs):
    p, ev, hlm = _event(recs, "c2", ["H", "L", "V"], 9, noise=True)
    rng = np.random.default_rng(10)
    th = chirpgen.prior_samples(rng, 500)
    _, T1, T2 = orc.lnL(p, th, return_terms=True)
    assert np.all(T2 >= -1e-12 * np.abs(T2).max())
    Ds = [200.0, 700.0, 2500.0]
    L = []
    for D in Ds:
        t = th.copy()
        t[3] = D
        L.append(orc.lnL(p, t))
    s = np.array([100.0 / D for D in Ds])
    A = np.stack([s, -s * s / 4], axis=1)
    sol = np.linalg.solve(A[:2], np.stack(L[:2]))
    assert np.allclose(sol[0], T1, rtol=1e-11, atol=1e-9)
    assert np.allclose(sol[1], T2, rtol=1e-11, atol=1e-9)
    pred = s[2] * sol[0] - s[2] ** 2 * sol[1] / 4
    assert np.allclose(pred, L[2], rtol=1e-11, atol=1e-9)


# --------------------------------------------------------------------- P8
@pytest.mark.slow
def test_P8_noise_statistics(orc, recs):
    """Over noise realisations: E lnL(theta_inj) = rho^2/2, Var = rho^2;
    E |Q_noise|^2 = U_aa (eq. QUV with the stated noise model)."""
    rec = recs["c1"]
    th = np.array(rec["theta"])
    vals, qn = [], []
    for seed in range(160):
        p, ev, hlm = _event(recs, "c1", ["H", "L"], 5, noise=True, seed=1000 + seed)
        vals.append(orc.lnL_exact(p, th, ev["f"], ev["df"], hlm, ev["data"])[0])
        noise = ev["data"] - ev["strain"]
        qn.append(orc.exact_Q(ev["f"], ev["df"], hlm, noise[0], 0.0013))
    vals = np.array(vals)
    n = len(vals)
    rho2 = 400.0
    assert abs(vals.mean() - rho2 / 2) < 4 * math.sqrt(rho2 / n)
    assert abs(vals.var(ddof=1) / rho2 - 1) < 4 * math.sqrt(2 / (n - 1))
    e = np.mean(np.abs(np.array(qn)) ** 2, axis=0)
    U = np.real(np.diag(p.U[0]))
    assert np.all(np.abs(e / U - 1) < 4 * math.sqrt(1.0 / n) + 0.02)


# --------------------------------------------------------------------- P9
def test_P9_face_on_single_mode_matched_filter(orc, recs):
    """Mode set {(2,2)}, iota = 0, one detector: V_22,22 = 0 for a one-sided
    h_22 spectrum, and the maximum of lnL over (D, phi_c) equals the complex
    matched-filter value |Q|^2/U."""
    p, ev, hlm = _event(recs, "c1", ["H"], 5, noise=True)
    a = p.modes.index((2, 2))
    p.modes = [(2, 2)]
    p.Q, p.U, p.V = p.Q[:, [a]], p.U[:, [a]][:, :, [a]], p.V[:, [a]][:, :, [a]]
    assert abs(p.V[0, 0, 0]) < 1e-12 * abs(p.U[0, 0, 0])
    th = np.array(recs["c1"]["theta"])
    th[4] = 1.0
    tau = orc.sample_tau(p, th)[0]
    u = (tau - p.tau0) / p.dt
    i0 = math.floor(u)
    w = orc.lagrange4(u - i0)
    qh = sum(w[j] * p.Q[0, 0, i0 - 1 + j] for j in range(4))
    U = p.U[0, 0, 0].real
    target = abs(qh) ** 2 / U
    F = complex(*orc.antenna(p.det_resp[0], th[0], th[1], th[6], p.gmst))
    y = orc.sylm(2, 2, 0.0, 0.0)
    zstar = 2 * qh / U                       # optimal complex amplitude s F Y
    s = abs(zstar) / abs(F * y)
    # Y22(0, -phi) = y e^{-2 i phi}:  arg(F y) - 2 phi = arg(z*)
    phi = (np.angle(F * y) - np.angle(zstar)) / 2
    t = th.copy()
    t[3] = 100.0 / s
    t[5] = phi % (2 * math.pi)
    best = orc.lnL(p, t[:, None])[0]
    assert abs(best - target) <= 1e-10 * target
    for dphi, ds in [(0.01, 1.0), (0.0, 1.01), (-0.02, 0.99)]:
        t2 = t.copy()
        t2[5] = (phi + dphi) % (2 * math.pi)
        t2[3] = 100.0 / (s * ds)
        assert orc.lnL(p, t2[:, None])[0] < best


# --------------------------------------------------------------------- P10
def test_P10_logsumexp_vs_mpmath(orc):
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 50
    rng = np.random.default_rng(11)
    lw = rng.uniform(-1e5, 1e5, 3000)
    lw[:2000] = rng.uniform(9.99e4, 1e5, 2000)
    r = orc.marginalize(lw)
    s1 = mpmath.fsum(mpmath.exp(mpmath.mpf(float(x))) for x in lw)
    s2 = mpmath.fsum(mpmath.exp(2 * mpmath.mpf(float(x))) for x in lw)
    ref = mpmath.log(s1) - mpmath.log(len(lw))
    assert abs(r["ln_L"] - float(ref)) <= 1e-12 * abs(float(ref))
    m = mpmath.mpf(float(lw.max()))
    assert abs(r["n_eff"] - float(s1 / mpmath.exp(m))) <= 1e-12 * r["n_eff"]
    assert abs(r["n_ess"] - float(s1 * s1 / s2)) <= 1e-12 * r["n_ess"]
    N = len(lw)
    var = (N * s2 / (s1 * s1) - 1) / (N - 1)
    assert abs(r["ln_sigma"] - float(ref + mpmath.log(var) / 2)) <= 1e-10


def test_P10_neff_special_cases(orc):
    r = orc.marginalize(np.full(1000, -3.5))
    assert abs(r["n_eff"] - 1000) < 1e-9 and abs(r["n_ess"] - 1000) < 1e-9
    assert abs(r["ln_L"] + 3.5) < 1e-12
    lw = np.full(1000, -800.0)
    lw[17] = 0.0
    r = orc.marginalize(lw)
    assert abs(r["n_eff"] - 1.0) < 1e-12 and r["argmax"] == 17
    r = orc.marginalize(np.array([-np.inf] * 10))
    assert r["ln_L"] == -np.inf and r["n_eff"] == 0 and r["n_nonfinite"] == 10
    r = orc.marginalize(np.array([0.0, -np.inf, np.nan, 0.0]))
    assert r["n_nonfinite"] == 2 and abs(r["ln_L"] - math.log(2 / 4)) < 1e-15
    # ties go to the lowest index
    assert orc.marginalize(np.array([1.0, 3.0, 3.0]))["argmax"] == 1


# --------------------------------------------------------------------- P11
@pytest.mark.slow
def test_P11_brute_force_quadrature(orc, recs):
    """Fix (alpha, dec, psi, t) at the injection; the product-grid quadrature
    over (cos iota, phi_c, D) against the prior agrees with a Monte Carlo
    estimate of the same integral within 4 sigma, and feeding the grid nodes
    with ln(weight) as log-weights through the estimator reproduces the grid sum."""
    p, ev, hlm = _event(recs, "c1", ["H", "L"], 5, noise=True)
    th0 = np.array(recs["c1"]["theta"])
    nc, nphi, nD = 64, 64, 256
    xc, wc = np.polynomial.legendre.leggauss(nc)           # cos iota on [-1,1]
    phis = np.arange(nphi) * 2 * math.pi / nphi
    Dlo, Dhi = 100.0, 1500.0
    xd, wd = np.polynomial.legendre.leggauss(nD)
    Ds = 0.5 * (Dhi - Dlo) * xd + 0.5 * (Dhi + Dlo)
    wD = 0.5 * (Dhi - Dlo) * wd
    pD = 3 * Ds ** 2 / (Dhi ** 3 - Dlo ** 3)
    C_, P_, D_ = np.meshgrid(np.arange(nc), np.arange(nphi), np.arange(nD), indexing="ij")
    th = np.tile(th0[:, None], (1, C_.size))
    th[4] = xc[C_.ravel()]
    th[5] = phis[P_.ravel()]
    th[3] = Ds[D_.ravel()]
    L = orc.lnL(p, th)
    lnw = (np.log(wc[C_.ravel()] / 2) + math.log(1.0 / nphi) + np.log(wD[D_.ravel()] * pD[D_.ravel()]))
    grid = np.logaddexp.reduce(L + lnw)
    r = orc.marginalize(L + lnw)
    assert abs((r["ln_L"] + math.log(L.size)) - grid) <= 1e-12 * abs(grid)
    rng = np.random.default_rng(12)
    N = 400000
    ths = np.tile(th0[:, None], (1, N))
    ths[4] = rng.uniform(-1, 1, N)
    ths[5] = rng.uniform(0, 2 * math.pi, N)
    ths[3] = np.cbrt(rng.uniform(Dlo ** 3, Dhi ** 3, N))
    rm = orc.marginalize(orc.lnL(p, ths))
    sig = math.exp(rm["ln_sigma"] - rm["ln_L"])
    assert abs(rm["ln_L"] - grid) < 4 * sig + 1e-3


# --------------------------------------------------------------------- P12/P13
def test_P13_em_single_component_is_weighted_moments(orc):
    rng = np.random.default_rng(13)
    n = 5000
    th = chirpgen.prior_samples(rng, n)
    lw = rng.normal(size=n)
    dims = [1, 2, 3, 4]
    X = th[dims].T
    w = np.exp(lw - lw.max())
    mu0 = X[0].copy()
    cov0 = np.diag([0.3, 1e-4, 1e5, 0.2])
    nw, nm, nc = orc.em_step(th, lw, dims, [1.0], [mu0], [cov0])
    m = (w @ X) / w.sum()
    c = ((X - m) * w[:, None]).T @ (X - m) / w.sum()
    floor = np.diag([1e-8 * orc.col_range(cc) ** 2 for cc in dims])
    assert np.allclose(nm[0], m, rtol=1e-12, atol=1e-12)
    assert np.allclose(nc[0], c + floor, rtol=1e-11, atol=1e-14)
    assert nw[0] == 1.0


def _first_fit_case(orc, case):
    """Samples whose first fit has a closed form (dims dec, t, D; all
    non-periodic).  Every top sample has lw = 0 (equal weights, ties by
    index); the rest lw = -800, finite (so candidates) but of weight exactly
    zero in FP64.  Returns (theta, lw, expected means, expected covariance)."""
    dims = [1, 2, 3]
    c = np.array([0.1, 0.001, 1000.0])
    a, b, g = 0.05, 0.002, 100.0
    e = np.eye(3)
    if case == 0:
        # eight distinct points, each twice: found within the top 16
        pts = [c, c + a * e[0], c - a * e[0], c + b * e[1], c - b * e[1], c + g * e[2], c - g * e[2],
               c + a * e[0] + b * e[1]]
        top = [p for p in pts for _ in range(2)]
        means = pts
        cov = np.array([[23 * a * a / 64, 7 * a * b / 64, 0.0],
                        [7 * a * b / 64, 23 * b * b / 64, 0.0],
                        [0.0, 0.0, g * g / 4]])
    else:
        # five distinct points fill the top 16 (4 + 3 + 3 + 3 + 3): the rule
        # repeats the fifth and never reaches the lower samples
        pts = [c, c + a * e[0], c - a * e[0], c + b * e[1], c - b * e[1]]
        top = [pts[0]] * 4 + [p for p in pts[1:] for _ in range(3)]
        means = pts + [pts[-1]] * 3
        cov = np.diag([6 * a * a / 16, 6 * b * b / 16, 0.0])
    rng = np.random.default_rng(21 + case)
    low = [c + rng.normal(size=3) * np.array([0.3, 0.01, 300.0]) for _ in range(20)]
    X = np.array(top + low)
    lw = np.concatenate([np.zeros(len(top)), np.full(len(low), -800.0)])
    th = np.zeros((7, len(X)))
    th[dims] = X.T
    cov = cov + np.diag([1e-8 * orc.col_range(cc) ** 2 for cc in dims])
    return th, lw, dims, np.array(means), cov


def _first_fit_holds(orc, case):
    th, lw, dims, means, cov = _first_fit_case(orc, case)
    w, m, C = orc.em_init(th, lw, dims, n_comp=8)
    return (np.array_equal(m, means) and np.allclose(w, 1.0 / 8, rtol=0, atol=0)
            and all(np.allclose(C[j], cov, rtol=1e-12, atol=1e-18) for j in range(8)))


@pytest.mark.parametrize("case", [0, 1])
def test_P13_em_first_fit_closed_form(orc, case):
    """First fit on duplicate-heavy samples: the means are the distinct points
    among the 2 n_comp highest-weight samples in weight order (the last one
    repeated when fewer are distinct), the common covariance the weighted
    covariance of the differences about the best sample (closed form), the
    weights 1/n_comp."""
    assert _first_fit_holds(orc, case)


def test_P13_em_first_fit_pin_rejects_other_rules(orc, monkeypatch):
    """Planted mistakes in the oracle's candidate rule fail the pin: scanning
    only the top n_comp samples (case 0: four distinct means), or every
    sample (case 1: the lower samples become means)."""
    monkeypatch.setattr(orc, "first_fit_candidates", lambda nc: nc)
    assert not _first_fit_holds(orc, 0)
    monkeypatch.setattr(orc, "first_fit_candidates", lambda nc: 10 ** 9)
    assert _first_fit_holds(orc, 0)
    assert not _first_fit_holds(orc, 1)


def test_P13_component_logpdf_matches_scipy(orc):
    from scipy.stats import multivariate_normal
    rng = np.random.default_rng(14)
    prior = orc.make_prior()
    dims = [1, 2, 3, 4]
    A = rng.normal(size=(4, 4))
    R = A @ A.T + 4 * np.eye(4)
    sd = np.sqrt(np.diag(R))
    R = R / np.outer(sd, sd)                       # correlation matrix
    sig = np.array([0.3, 0.5, 2.0, 0.3])
    cov = R * np.outer(sig, sig)
    mean = [0.1, 0.001, 500.0, 0.2]  # theta[3] near 500 lies far out: exercises a large Mahalanobis value
    g = orc.make_gmm([1.0], [mean], [cov], dims)
    for _ in range(20):
        th = chirpgen.prior_samples(rng, 1)[:, 0]
        ref = multivariate_normal(mean=mean, cov=cov).logpdf(th[dims])
        assert abs(orc.gmm_comp_logpdf(prior, g, 0, th) - ref) <= 1e-10 * (1 + abs(ref))


def test_temper_beta_gaussian_closed_form(orc):
    """For log-weights ~ N(0, s^2), (sum w^b)^2 / sum w^(2b) / N -> e^{-b^2 s^2};
    the rule picks the largest grid value 2^(-k/4) meeting the target."""
    rng = np.random.default_rng(17)
    s = 10.0
    lw = rng.normal(0.0, s, 1 << 20)
    frac = 1.0 / 16.0
    b = orc.temper_beta(lw, frac)
    bstar = math.sqrt(math.log(1.0 / frac)) / s
    grid = [2.0 ** (-k / 4.0) for k in range(48)]
    expect = max(g for g in grid if g <= bstar)
    assert b == expect
    assert orc.temper_beta(lw, 0.0) == 1.0
    # all weights equal: beta = 1 already has full ESS
    assert orc.temper_beta(np.zeros(100), 0.5) == 1.0


def test_P13_periodic_wrap_logpdf(orc):
    """Periodic columns use the wrapped difference: a mean near 2 pi and a
    point near 0 are close."""
    from scipy.stats import multivariate_normal
    prior = orc.make_prior()
    g = orc.make_gmm([1.0], [[6.2, 0.05]], [np.diag([0.04, 0.01])], [0, 6])
    th = np.zeros(7)
    th[0], th[6] = 0.05, 3.1
    ref = multivariate_normal(mean=[0, 0], cov=np.diag([0.04, 0.01])).logpdf(
        [0.05 + 2 * math.pi - 6.2, 3.1 - math.pi - 0.05])
    assert abs(orc.gmm_comp_logpdf(prior, g, 0, th) - ref) < 1e-12


def test_P12_two_gaussian_recovery(orc):
    """Two Gaussians, sigma = sqrt(2), centres (+-4, 0, 0) (the hyperpipeline
    demonstration target): the fitted mixture covers both, and importance
    sampling from it integrates the normalised target to 1 within 4 sigma."""
    from scipy.stats import multivariate_normal
    rng = np.random.default_rng(15)
    dims = [1, 2, 3]           # three bounded columns used as a plain 3-D space
    sc = np.array([1.0, 1.0, 1.0])
    n = 60000
    X = rng.uniform(-12, 12, size=(n, 3))
    tgt = lambda Z: np.logaddexp(  # noqa: E731
        multivariate_normal([4, 0, 0], 2 * np.eye(3)).logpdf(Z),
        multivariate_normal([-4, 0, 0], 2 * np.eye(3)).logpdf(Z)) + math.log(0.5)
    lw = tgt(X) - math.log(1 / 24 ** 3)
    th = np.zeros((7, n))
    th[dims] = (X * sc).T
    w, m, c = orc.em_fit(th, lw, dims, n_iter=30, n_comp=8, t_window=100.0, d_min=-100, d_max=100)
    left = sum(w[j] for j in range(8) if m[j][0] < 0)
    assert 0.3 < left < 0.7
    # importance integral of the target under the fitted mixture
    comp = rng.choice(8, size=40000, p=w / w.sum())
    Z = np.array([rng.multivariate_normal(m[j], c[j]) for j in comp])
    lq = np.logaddexp.reduce([math.log(w[j]) + multivariate_normal(m[j], c[j]).logpdf(Z) for j in range(8) if w[j] > 0], axis=0)
    ratio = np.exp(tgt(Z) - lq)
    est, err = ratio.mean(), ratio.std() / math.sqrt(len(ratio))
    assert abs(est - 1) < 4 * err + 1e-3


# --------------------------------------------------------------------- P14
@pytest.mark.parametrize("T1,T2", [(30.0, 900.0), (5.0, 4.0), (-3.0, 50.0), (400.0, 1.6e5)])
def test_P14_distance_integral_closed_form(orc, T1, T2):
    """Prior uniform in s: int e^{s T1 - s^2 T2/4} ds has an erf closed form."""
    from scipy.special import erf, erfc
    slo, shi = 100 / 3000, 100.0
    ss = 2 * T1 / T2
    a = math.sqrt(T2) / 2
    x1, x2 = a * (slo - ss), a * (shi - ss)
    # erf(x2) - erf(x1), written with erfc when both arguments are positive
    diff = erfc(x1) - erfc(x2) if x1 > 0 else erf(x2) - erf(x1)
    # ln of e^{T1^2/T2} sqrt(pi/T2) diff / (s_hi - s_lo)
    ref = T1 * T1 / T2 + 0.5 * math.log(math.pi / T2) + math.log(diff) - math.log(shi - slo)
    got = orc.ln_dist_marg(T1, T2, prior="uniform_s")
    assert abs(got - ref) <= 1e-11 * max(1, abs(ref))


def test_P14_distance_integral_volume_prior_bruteforce(orc):
    """Volume prior: compare with a dense Simpson rule in log D."""
    from scipy.integrate import simpson
    for T1, T2 in [(30.0, 900.0), (2.0, 1.0), (150.0, 2.0e4)]:
        lD = np.linspace(math.log(1.0), math.log(3000.0), 400001)
        D = np.exp(lD)
        s = 100.0 / D
        e = s * T1 - s * s * T2 / 4
        m = e.max()
        integrand = np.exp(e - m) * 3 * D ** 2 / (3000 ** 3 - 1) * D
        ref = m + math.log(simpson(integrand, x=lD))
        assert abs(orc.ln_dist_marg(T1, T2) - ref) < 1e-8


# --------------------------------------------------------------------- P15
def test_P15_generator_matrices(recs):
    probs, _ = chirpgen.build_event(recs["c3"], ["H", "L", "V"], 17, 30.0, 20.0, 100.0, noise_seed=3)
    p = probs[0]
    for k in range(p.n_det):
        assert np.allclose(p.U[k], np.conj(p.U[k].T), atol=1e-12 * np.abs(p.U[k]).max())
        assert np.allclose(p.V[k], p.V[k].T, atol=1e-12 * np.abs(p.V[k]).max())
        ev = np.linalg.eigvalsh(p.U[k])
        assert ev.min() > -1e-10 * ev.max()


# --------------------------------------------------------------------- draws
def test_philox_known_answers(orc):
    """Philox-4x32-10 known-answer vectors published with the Random123 library
    (Salmon et al., SC'11); stored in tests/golden/philox_kat.txt."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "philox_kat.txt")
    n = 0
    for line in open(path):
        if not line.strip() or line.startswith("#"):
            continue
        v = [int(x, 16) for x in line.split()]
        assert orc.philox(v[0:4], v[4:6]) == v[6:10]
        n += 1
    assert n == 3


def test_prior_draws_distribution(orc):
    from scipy import stats
    prior = orc.make_prior()
    th, lp = orc.draw_prior(prior, 12345, 0, 0, 20000)
    assert stats.kstest(th[0] / (2 * math.pi), "uniform").pvalue > 1e-4
    assert stats.kstest((np.sin(th[1]) + 1) / 2, "uniform").pvalue > 1e-4
    assert stats.kstest((th[3] ** 3 - 1) / (3000 ** 3 - 1), "uniform").pvalue > 1e-4
    assert stats.kstest((th[4] + 1) / 2, "uniform").pvalue > 1e-4
    assert stats.kstest(th[6] / math.pi, "uniform").pvalue > 1e-4
    # ln p integrates: mean of exp(-lnp) over the box volume (importance identity)
    i = 7
    ref = (-math.log(2 * math.pi) + math.log(math.cos(th[1, i]) / 2) - math.log(0.056)
           + math.log(3 * th[3, i] ** 2 / (3000 ** 3 - 1)) - math.log(2) - math.log(2 * math.pi) - math.log(math.pi))
    assert abs(lp[i] - ref) < 1e-12
    # counter-based: a later window reproduces the same samples
    th2, _ = orc.draw_prior(prior, 12345, 0, 100, 50)
    assert np.array_equal(th2, th[:, 100:150])


def test_gmm_draws_follow_ps(orc):
    """E_{p_s}[p/p_s] = 1 for draws from the proposal (importance identity), and
    a one-dimensional in-support mass agrees with its erf closed form."""
    from scipy.special import erf
    prior = orc.make_prior()
    dims = [0, 1, 2, 3, 4, 5, 6]
    rng = np.random.default_rng(16)
    means = [[6.0, 0.3, 0.01, 500.0, 0.5, 0.1, 3.0], [1.0, -0.5, -0.02, 2500.0, -0.9, 3.0, 0.2]]
    covs = [np.diag([0.2, 0.1, 1e-4, 1e4, 0.1, 0.3, 0.2]) ** 1, np.diag([0.5, 0.05, 4e-4, 3e5, 0.05, 1.0, 0.5])]
    g = orc.make_gmm([0.6, 0.4], means, covs, dims)
    lz = [math.log(orc.gmm_inbox_mass(prior, g, j, 99, 0, 1 << 16)) for j in range(2)]
    g = orc.make_gmm([0.6, 0.4], means, covs, dims, ln_Z=lz)
    th, lr = orc.draw_gmm(prior, g, 99, 1, 0, 40000)
    r = np.exp(lr)
    assert abs(r.mean() - 1) < 4 * r.std() / math.sqrt(len(r)) + 2e-3
    del rng
    # 1-D mass: t column with mean 0.02, sd 0.01 on [-0.028, 0.028]
    g1 = orc.make_gmm([1.0], [[0.02]], [[[1e-4]]], [2])
    z = orc.gmm_inbox_mass(prior, g1, 0, 5, 0, 1 << 16)
    ref = 0.5 * (erf((0.028 - 0.02) / (0.01 * math.sqrt(2))) - erf((-0.028 - 0.02) / (0.01 * math.sqrt(2))))
    assert abs(z - ref) < 4 * math.sqrt(ref * (1 - ref) / (1 << 16))


def test_gmm_draw_density_counts_failed_attempts(orc):
    """A component that lies mostly outside the support (in-support mass
    Z ~ 0.012, so its 64 rejection attempts all fail ~46 % of the time) beside
    one inside it, on the t column alone (the other six columns come from the
    prior draw), unnormalised weights.  With the exact in-support masses
    (erf closed form) the importance identity E_{p_s}[p / p_s] = 1 must hold
    for the draws; a density without the failed-attempt mass (the oracle's
    own ln p_s with unlimited attempts) must fail it."""
    from scipy.special import erf
    prior = orc.make_prior()
    tw = 0.028
    comps = [(0.055, 0.012), (0.0, 0.006)]

    def zmass(mu, sd):
        return 0.5 * (erf((tw - mu) / (sd * math.sqrt(2))) - erf((-tw - mu) / (sd * math.sqrt(2))))

    lz = [math.log(zmass(mu, sd)) for mu, sd in comps]
    g = orc.make_gmm([3.0, 1.0], [[mu] for mu, _ in comps], [[[sd * sd]] for _, sd in comps], [2], ln_Z=lz)
    n = 40000
    th, lr = orc.draw_gmm(prior, g, 2024, 3, 0, n)
    r = np.exp(lr)
    assert abs(r.mean() - 1) < 4 * r.std() / math.sqrt(n)
    # the same draws scored without the failed-attempt mass
    lr0 = np.array([orc.ln_prior(prior, th[:, i]) - orc.gmm_ln_ps(prior, g, th[:, i], attempts=0)
                    for i in range(n)])
    r0 = np.exp(lr0)
    assert abs(r0.mean() - 1) > 10 * r0.std() / math.sqrt(n)


def _phase_gmm(orc, prior, shear, dims=(0, 1, 4, 5, 6)):
    """Two components over sky, inclination and the phases; the second is
    wide along phi_c (a ridge at fixed psi + shear phi_c)."""
    dims = list(dims)
    means = [[1.0, 0.3, 0.5, 2.0, 1.0], [4.0, -0.4, -0.7, 5.0, 2.5]]
    covs = [np.diag([0.05, 0.02, 0.01, 0.04, 0.01]), np.diag([0.2, 0.05, 0.02, 4.0, 0.003])]
    g = orc.make_gmm([0.5, 0.5], means, covs, dims, shear=shear)
    lz = [math.log(orc.gmm_inbox_mass(prior, g, j, 31, 0, 1 << 16)) for j in range(2)]
    return orc.make_gmm([0.5, 0.5], means, covs, dims, ln_Z=lz, shear=shear), means, covs


@pytest.mark.parametrize("shear", [1, -1])
def test_PS1_sheared_mixture_is_a_density_of_its_draws(orc, shear):
    """Phase-sheared mixture (column 6 of the mixture is (psi + s phi_c) mod pi):
    its draws satisfy the importance identity E_{p_s}[p / p_s] = 1, prior
    draws satisfy E_p[p_s / p] = 1 (p_s integrates to one over the support),
    and the draws of the ridge component have y = (psi + s phi_c) mod pi
    concentrated at the component's mean with its standard deviation while
    psi alone spreads over its range.  A density evaluated in the unsheared
    coordinates fails the first identity."""
    prior = orc.make_prior()
    g, means, covs = _phase_gmm(orc, prior, shear)
    n = 60000
    th, lr = orc.draw_gmm(prior, g, 77, 2, 0, n)
    r = np.exp(lr)
    assert abs(r.mean() - 1) < 4 * r.std() / math.sqrt(n)
    thp, _ = orc.draw_prior(prior, 78, 0, 0, n)
    q = np.exp(orc.gmm_ln_ps_batch(prior, g, thp) - np.array([orc.ln_prior(prior, thp[:, i]) for i in range(n)]))
    assert abs(q.mean() - 1) < 4 * q.std() / math.sqrt(n)
    # the ridge component: samples near its sky position (about 2 % of them
    # defensive prior draws, hence median and median absolute deviation)
    sel = np.abs(th[0] - means[1][0]) < 0.3
    y = np.mod(th[6, sel] + shear * th[5, sel], math.pi)
    med = np.median(y)
    assert abs(med - means[1][4]) < 0.005
    assert abs(1.4826 * np.median(np.abs(y - med)) - math.sqrt(covs[1][4][4])) < 0.005
    assert np.std(th[6, sel]) > 0.6          # psi alone is spread (uniform: pi/sqrt(12) = 0.91)
    # the same draws scored by a mixture with the same parameters but no shear
    g0 = orc.make_gmm([0.5, 0.5], means, covs, [0, 1, 4, 5, 6], ln_Z=[g.ln_Z[0], g.ln_Z[1]])
    lr0 = np.array([orc.ln_prior(prior, th[:, i]) for i in range(n)]) - orc.gmm_ln_ps_batch(prior, g0, th)
    r0 = np.exp(lr0)
    assert abs(r0.mean() - 1) > 10 * r0.std() / math.sqrt(n)


def test_PS2_shear_sign_and_round_trip(orc):
    """The shear follows the inclination of the best sample (none between
    cos iota = -1/2 and 1/2); shearing by s then by -s returns every phase
    pair (mod its period)."""
    th = np.zeros((7, 4))
    th[4] = [0.9, -0.2, 0.3, -0.8]
    assert orc.phase_shear_sign(th, [1.0, 5.0, 2.0, -np.inf]) == 0     # |cos iota| < 1/2: no shear
    assert orc.phase_shear_sign(th, [7.0, 5.0, 2.0, np.nan]) == 1
    assert orc.phase_shear_sign(th, [1.0, 5.0, 2.0, 6.0]) == -1
    assert orc.phase_shear_sign(th, [-np.inf] * 4) == 0
    rng = np.random.default_rng(3)
    t = np.zeros((7, 1000))
    t[5] = rng.uniform(0, 2 * math.pi, 1000)
    t[6] = rng.uniform(0, math.pi, 1000)
    for s in (1, -1):
        u = orc.shear_theta(t, s)
        assert np.all((u[6] >= 0) & (u[6] < math.pi))
        back = orc.shear_theta(u, -s)
        d = np.mod(back[6] - t[6] + math.pi / 2, math.pi) - math.pi / 2
        assert np.max(np.abs(d)) < 1e-12


def _von_mises_rounds(orc, prior, kappa, phi0, rounds, n, seed):
    """An adaptive-like run on L = exp(kappa cos(phi_c - phi0)): the prior,
    then mixtures over phi_c of growing accuracy (the other columns from the
    prior).  Returns proposals, thetas, lnLs."""
    props, ths, lls = [None], [], []
    for r in range(rounds):
        g = props[r]
        if g is None:
            th, _ = orc.draw_prior(prior, seed, r, 0, n)
        else:
            th, _ = orc.draw_gmm(prior, g, seed, r, 0, n)
        ths.append(th)
        lls.append(kappa * np.cos(th[5] - phi0))
        sd = 2.0 / math.sqrt(kappa) / (r + 1)     # proposals narrower than the target
        g = orc.make_gmm([1.0], [[phi0 + 0.1 * r]], [[[sd * sd]]], [5], eps_def=0.05)
        lz = [math.log(orc.gmm_inbox_mass(prior, g, 0, seed + 1, r, 1 << 15))]
        props.append(orc.make_gmm([1.0], [[phi0 + 0.1 * r]], [[[sd * sd]]], [5], ln_Z=lz, eps_def=0.05))
    return props[:rounds], ths, lls


def test_PP1_mixture_pool_closed_form_and_bounds(orc):
    """Samples pooled as draws of the equal-weight mixture of the rounds'
    proposals (eq. (lnL:MonteCarlo) with that mixture as p_s): on
    L = exp(kappa cos(phi_c - phi0)) with a uniform phi_c prior the integral is
    the modified Bessel value I0(kappa); the pooled estimate must match it
    within its Monte Carlo error, every weight must be at most R L (the prior
    is a member of the mixture), and one round from the prior gives lw = lnL.
    Scoring each sample by its own round's proposal alone also estimates I0,
    but with a larger spread; a pool that forgets the 1/R of the mixture is
    off by ln R."""
    from scipy.special import i0e
    prior = orc.make_prior()
    kappa, phi0, R, n = 40.0, 2.0, 4, 8000
    props, ths, lls = _von_mises_rounds(orc, prior, kappa, phi0, R, n, 404)
    lw = orc.pool_mixture_lw(prior, props, ths, lls)
    L = np.concatenate(lls)
    assert np.all(lw <= L + math.log(R) + 1e-12)
    w = np.exp(lw - kappa)
    est, err = w.mean(), w.std() / math.sqrt(len(w))
    exact = i0e(kappa)                       # I0(kappa) e^{-kappa}
    assert abs(est - exact) < 4 * err
    assert abs(math.log(est) - math.log(exact)) < 0.02
    # one prior round
    lw1 = orc.pool_mixture_lw(prior, props[:1], ths[:1], lls[:1])
    assert np.array_equal(lw1, np.asarray(lls[0], dtype=np.float64))
    # forgetting the 1/R: off by ln R, far outside the error
    assert abs(math.log(np.exp(lw + math.log(R) - kappa).mean()) - math.log(exact)) > 20 * err / exact


# ------------------------------------------------ time-marginalised lnL
def test_PT1_time_constant_Q_closed_form(orc):
    """Q constant in time makes lnL independent of t, so the time integral is
    lnL(t = 0) + ln(N_t dt / (R 2 t_w)) with N_t = 2 floor(R t_w/dt) + 1."""
    rng = np.random.default_rng(60)
    p = chirpgen.random_problem(rng, 5, ["H", "L"])
    p.Q = np.repeat(p.Q[:, :, 205:206], p.Q.shape[2], axis=2)
    th = chirpgen.prior_samples(rng, 300)
    t0 = th.copy()
    t0[2] = 0.0
    base = orc.lnL(p, t0)
    for R in (1, 4):
        nt = 2 * int(math.floor(R * p.t_window / p.dt + 1e-9)) + 1
        want = base + math.log(nt * p.dt / (R * 2 * p.t_window))
        got = orc.lnL_tmarg(p, th, oversample=R)
        assert np.allclose(got, want, rtol=1e-12, atol=1e-10)


def test_PT1_single_node(orc):
    """A time window shorter than one node spacing leaves the node t = 0."""
    rng = np.random.default_rng(61)
    p = chirpgen.random_problem(rng, 9, ["H", "L", "V"])
    p.t_window = 0.2 * p.dt / 4
    th = chirpgen.prior_samples(rng, 200)
    t0 = th.copy()
    t0[2] = 0.0
    want = orc.lnL(p, t0) + math.log(p.dt / (4 * 2 * p.t_window))
    assert np.allclose(orc.lnL_tmarg(p, th, oversample=4), want, rtol=1e-13, atol=1e-11)


def test_PTD2_time_and_distance_closed_forms(orc):
    """Q constant in time: every node has the same T1, so the time- and
    distance-marginalised value is ln L_D(T1, T2) + ln(N_t dt / (R 2 t_w)).
    A distance prior squeezed onto [D0, D0 (1 + 1e-7)] turns it into the
    time-marginalised likelihood at D = D0."""
    rng = np.random.default_rng(62)
    p = chirpgen.random_problem(rng, 5, ["H", "L"])
    pc = chirpgen.random_problem(rng, 5, ["H", "L"])
    pc.Q = np.repeat(pc.Q[:, :, 205:206], pc.Q.shape[2], axis=2)
    th = chirpgen.prior_samples(rng, 4)
    t0 = th.copy()
    t0[2], t0[3] = 0.0, pc.d_ref
    _, T1, T2 = orc.lnL(pc, t0, return_terms=True)
    nt = 2 * int(math.floor(pc.t_window / pc.dt + 1e-9)) + 1
    want = np.array([orc.ln_dist_marg(a, b) for a, b in zip(T1, T2)]) + math.log(nt * pc.dt / (2 * pc.t_window))
    assert np.allclose(orc.lnL_tmarg_dist(pc, th, oversample=1), want, rtol=1e-10, atol=1e-8)
    D0 = 400.0
    thd = th.copy()
    thd[3] = D0
    narrow = orc.lnL_tmarg_dist(p, th[:, :2], oversample=1, d_min=D0, d_max=D0 * (1 + 1e-7))
    assert np.allclose(narrow, orc.lnL_tmarg(p, thd[:, :2], oversample=1), rtol=1e-9, atol=1e-6)


def test_PT2_node_sum_converges_to_quadrature(orc, recs):
    """Near the likelihood peak of an SNR-20 event (width in t ~80 us) the
    node sum converges to the time integral of the same interpolated
    likelihood, computed by a trapezoid rule 16x finer than R = 4 over exactly
    [-t_w, t_w].  The integrand has derivative jumps where a detector time
    crosses a window sample, so the rule is O(h^2): measured 0.31 (R = 1),
    4e-3 (R = 4), 2e-4 (R = 16).  Fails for a wrong node weight (>= ln 2), a
    sum that uses the sample's own t, or a missing log/exp."""
    p, ev, _ = _event(recs, "c1", ["H", "L"], 5, noise=True)
    th0 = np.array(recs["c1"]["theta"])
    rng = np.random.default_rng(62)
    w = np.array([0.03, 0.03, 0.0, 0.05 * th0[3], 0.05, 0.1, 0.1])
    th = th0[:, None] + w[:, None] * rng.standard_normal((7, 12))
    th[4] = np.clip(th[4], -1, 1)
    th[2] = rng.uniform(-p.t_window, p.t_window, 12)     # ignored by the time integral
    got = orc.lnL_tmarg(p, th, oversample=4)
    M = 64 * int(2 * p.t_window / p.dt) + 1
    tf = np.linspace(-p.t_window, p.t_window, M)
    ref = np.empty(th.shape[1])
    for i in range(th.shape[1]):
        big = np.repeat(th[:, i:i + 1], M, axis=1)
        big[2] = tf
        L = orc.lnL(p, big)
        m = L.max()
        ref[i] = m + math.log(np.trapezoid(np.exp(L - m), tf) / (2 * p.t_window))
    assert np.max(got) > 150.0                         # a loud peak inside the window
    fine = orc.lnL_tmarg(p, th, oversample=16)
    assert np.max(np.abs(got - ref)) < 1e-2, np.max(np.abs(got - ref))
    assert np.max(np.abs(fine - ref)) < 1e-3, np.max(np.abs(fine - ref))


# ------------------------------------------------------------------ AV (f2)
# Section "Adaptive volume integration": hypercube refinement of the unit cube
# of the prior's CDF coordinates.
def test_PA1_av_one_cell_is_the_prior_draw(orc):
    """With the whole cube as the single active cell of a one-bin grid the
    sampler is the prior itself: the same draws, and ln p - ln p_s = ln V = 0."""
    pr = orc.make_prior()
    g = orc.av_init()
    th, u = orc.draw_av(pr, g, 0xABCDEF, 3, 1000, 5000)
    tp, _ = orc.draw_prior(pr, 0xABCDEF, 3, 1000, 5000)
    assert np.array_equal(th, tp)
    assert g.ln_vol == 0.0
    gd = orc.av_init(dist_marg=True)
    prd = orc.make_prior(dist_marg=True)
    th2, u2 = orc.draw_av(prd, gd, 5, 0, 0, 100)
    assert u2.shape == (6, 100) and np.all(th2[3] == 100.0)


def test_PA2_av_draws_uniform_over_active_cells(orc):
    """Every draw lies in an active cell, the cells are used equally often
    (chi-square) and positions inside a cell are uniform (Kolmogorov-Smirnov)."""
    from scipy import stats
    rng = np.random.default_rng(80)
    nb, d = 4, 7
    ids = rng.choice(nb ** d, size=37, replace=False)
    cells = np.array([[(i // nb ** k) % nb for k in range(d)] for i in ids], dtype=np.int32)
    g = orc.AvGrid(nb, cells, list(range(7)))
    n = 200000
    _, u = orc.draw_av(orc.make_prior(), g, 99, 1, 0, n)
    c = np.floor(u * nb).astype(np.int64)
    key = sum(c[k] * nb ** k for k in range(d))
    pos = {int(i): j for j, i in enumerate(ids)}
    assert all(int(x) in pos for x in np.unique(key))
    counts = np.bincount([pos[int(x)] for x in key], minlength=len(ids))
    assert stats.chisquare(counts).pvalue > 1e-4
    frac = (u * nb - c).ravel()
    assert stats.kstest(frac, "uniform").pvalue > 1e-4
    assert abs(g.ln_vol - math.log(37 / nb ** d)) < 1e-12


@pytest.mark.parametrize("case", range(6))
def test_PA3_av_threshold_is_the_largest_feasible_value(orc, case):
    """The threshold is the largest finite lnL value v such that the samples at
    or above v hold at least min(ceil(p_thr * total), total) of the fixed-point
    mass and
    number at least min(n_min_live, n_finite): found here by trying every
    distinct value, against the oracle's sorted cumulative sum."""
    rng = np.random.default_rng(81 + case)
    n = [50, 400, 3000, 3000, 17, 1000][case]
    x = rng.normal(0, [3.0, 10.0, 0.5, 30.0, 1.0, 5.0][case], n)
    x = np.round(x, [6, 1, 2, 3, 6, 0][case])          # ties
    x[rng.choice(n, n // 10, replace=False)] = -np.inf
    x[rng.choice(n, 2, replace=False)] = np.nan
    fin = x[np.isfinite(x)]
    m = fin.max()
    q = [int(math.floor(math.exp(v - m) * 2.0 ** 40)) for v in fin]
    total = sum(q)
    for p_thr, k in [(0.999, 1), (0.9, 10), (0.5, 100), (1.0, 5), (0.99, 10 ** 6), (1e-9, 1)]:
        target = min(math.ceil(p_thr * float(total)), total)
        kk = min(k, fin.size)
        best = None
        for v in np.unique(fin)[::-1]:
            sel = fin >= v
            if sum(qq for qq, s in zip(q, sel) if s) >= target and int(sel.sum()) >= kk:
                best = float(v)
                break
        thr, n_min = orc.av_threshold(x, p_thr, k)
        assert thr == best, (p_thr, k, thr, best)
        assert n_min == int(np.count_nonzero(fin >= best))
    assert orc.av_threshold(np.full(5, -np.inf), 0.9, 3) is None


def test_PA5_nbins_worked_examples(orc):
    """eq. (nbins_V) by hand: d = 2, V = 1, 100 of 10^4 live points above the
    threshold: V' = 0.01, dV = 0.001, (1/dV)^(1/2) = 31.6 -> 32 bins; d = 7,
    1000 of 2^16: dV = (1000/65536)/sqrt(1000) = 4.83e-4, 2071^(1/7) = 2.98 ->
    3 bins; every one of 10^6 points kept, d = 7: dV = 1e-3, 1000^(1/7) = 2.68
    -> 3; and the clamp at max_bins."""
    assert orc.av_refine_bins(100, 10000, 0.0, 2, 511) == 32
    assert orc.av_refine_bins(1000, 65536, 0.0, 7, 511) == 3
    assert orc.av_refine_bins(10 ** 6, 10 ** 6, 0.0, 7, 511) == 3
    assert orc.av_refine_bins(4, 10 ** 6, math.log(1e-3), 2, 511) == 511


def _gauss_cell_integral(cells, nb, mu, sig):
    """Exact integral of prod_k N(u_k; mu_k, sig_k) over a union of cells."""
    from scipy.special import ndtr
    lo = cells / nb
    hi = (cells + 1) / nb
    per = ndtr((hi - mu) / sig) - ndtr((lo - mu) / sig)
    return float(np.sum(np.prod(per, axis=1)))


def test_PA4_av_estimator_is_unbiased_on_the_active_volume(orc):
    """A product Gaussian over the seven unit-cube coordinates, integrated by
    rounds of AV draws: each round's samples weighted by the active volume V
    (ln p - ln p_s = ln V) estimate the exact integral over that round's active
    cells (a closed form per cell), so the pooled estimator agrees within 4
    sigma with the sample-weighted mean of those exact integrals; the active
    cells keep >= 99 % of the whole integral."""
    rng = np.random.default_rng(84)
    mu = rng.uniform(0.35, 0.65, 7)
    sig = np.full(7, 0.08)
    norm = -0.5 * 7 * math.log(2 * math.pi) - float(np.sum(np.log(sig)))
    full = _gauss_cell_integral(np.zeros((1, 7), dtype=np.int32), 1, mu, sig)
    pr = orc.make_prior()
    g = orc.av_init()
    n, lws, expect, vols = 40000, [], 0.0, []
    for r in range(5):
        _, u = orc.draw_av(pr, g, 2024, r, 0, n)
        lnL = norm - 0.5 * np.sum(((u.T - mu) / sig) ** 2, axis=1)
        lws.append(lnL + g.ln_vol)
        exact_r = _gauss_cell_integral(g.cells, g.nb, mu, sig)
        assert exact_r >= 0.99 * full
        expect += n * exact_r
        vols.append(g.ln_vol)
        g, _ = orc.av_update(g, u, lnL, p_thr=0.999, n_min_live=2000)
    o = orc.marginalize(np.concatenate(lws))
    expect = math.log(expect / (n * len(lws)))
    sigma = math.exp(o["ln_sigma"] - o["ln_L"])
    assert abs(o["ln_L"] - expect) <= 4 * sigma, (o["ln_L"], expect, sigma)
    assert vols[-1] < math.log(0.05)          # the active volume shrank around the peak


def test_PA6_av_rosenbrock_sampling_efficiency(orc):
    """The paper's Rosenbrock demonstration: a grid over two unit-cube
    coordinates (the other columns drawn from the prior, the volume counted
    over the grid's dimensions only); the AV rounds sample far more
    efficiently than the prior (n_eff/N of the last round vs the first)."""
    pr = orc.make_prior()
    g = orc.AvGrid(1, np.zeros((1, 2), dtype=np.int32), [0, 1])
    n, eff = 20000, []
    for r in range(5):
        _, u = orc.draw_av(pr, g, 77, r, 0, n)
        x, y = 4.0 * u[0] - 2.0, 4.0 * u[1] - 1.0
        lnL = -((1.0 - x) ** 2 + 100.0 * (y - x * x) ** 2)
        eff.append(orc.marginalize(lnL + g.ln_vol)["n_eff"] / n)
        g, _ = orc.av_update(g, u, lnL, p_thr=0.999, n_min_live=1000)
    assert eff[-1] > 5 * eff[0], eff


def test_PA7_av_new_cells_hold_exactly_the_top_samples(orc):
    """After an update every sample at or above the threshold lies in a listed
    cell of the refined grid, every listed cell holds one, no cell is listed
    twice, and the list follows the first such sample of each cell."""
    pr = orc.make_prior()
    g = orc.av_init()
    rng = np.random.default_rng(85)
    _, u = orc.draw_av(pr, g, 31, 0, 0, 30000)
    lnL = -np.sum(((u.T - 0.4) / 0.15) ** 2, axis=1) + rng.normal(0, 0.1, 30000)
    lnL[:100] = -np.inf
    g2, info = orc.av_update(g, u, lnL, p_thr=0.99, n_min_live=300)
    top = np.nonzero(lnL >= info["lnL_thr"])[0]
    assert top.size == info["n_min"] >= 300
    c = np.minimum(np.floor(u[:, top] * g2.nb), g2.nb - 1).astype(np.int64).T
    listed = {tuple(x) for x in g2.cells}
    assert len(listed) == g2.n_cells
    assert {tuple(x) for x in c} == listed
    first = []
    for x in map(tuple, c):
        if x not in first:
            first.append(x)
    assert [tuple(x) for x in g2.cells] == first


def test_PA3_av_threshold_total_beyond_double_precision(orc):
    """p_thr = 1 with a total fixed-point mass of 2^54 + 3 (2^14 samples of
    mass 2^40 and three of mass 1): in FP64 the total rounds up to 2^54 + 4,
    beyond every cumulative sum; the target is clamped to the total, so the
    threshold reaches the three light samples."""
    x = np.zeros((1 << 14) + 3)
    x[-3:] = -27.6                 # exp(-27.6) 2^40 = 1.1 -> mass 1
    assert int(np.sum(orc.av_mass(x))) == (1 << 54) + 3
    thr, n_min = orc.av_threshold(x, 1.0, 1)
    assert n_min == x.size and thr == -27.6


# ------------------------------------------------------------- fair draws (f3)
def test_PF1_fair_draw_frequencies_follow_the_weights(orc):
    """Draw counts over 40,000 fair draws match the normalised weights
    (chi-square over the indices with expected count >= 5); a sample with
    zero or non-finite weight is never drawn."""
    from scipy import stats
    rng = np.random.default_rng(86)
    lw = rng.normal(0, 2, 600)
    lw[:7] = -np.inf
    lw[7] = np.nan
    idx = orc.fair_draw(lw, 1234, 2, 40000)
    assert idx.min() >= 8
    w = np.where(np.isfinite(lw), np.exp(lw - np.nanmax(lw[np.isfinite(lw)])), 0.0)
    p = w / w.sum()
    cnt = np.bincount(idx, minlength=lw.size)
    m = p * idx.size >= 5
    assert stats.chisquare(cnt[m], p[m] / p[m].sum() * cnt[m].sum()).pvalue > 1e-4


def test_PF2_fair_draw_degenerate_cases(orc):
    """One finite sample is drawn every time; no finite sample gives -1."""
    lw = np.full(50, -np.inf)
    assert np.all(orc.fair_draw(lw, 1, 0, 10) == -1)
    lw[31] = -5.0
    assert np.all(orc.fair_draw(lw, 1, 0, 10) == 31)


def test_PF3_fair_draws_reproduce_the_target_distribution(orc):
    """Importance samples of a truncated normal on [0, 1] (uniform proposal,
    lw = ln of the density) fairly redrawn follow that truncated normal
    (Kolmogorov-Smirnov against scipy's CDF): the check that extrinsic
    samples resampled from an ILE run reproduce its posterior."""
    from scipy import stats
    rng = np.random.default_rng(87)
    u = rng.uniform(0, 1, 200000)
    mu, sig = 0.4, 0.05
    lw = -0.5 * ((u - mu) / sig) ** 2
    idx = orc.fair_draw(lw, 99, 0, 3000)
    tn = stats.truncnorm((0 - mu) / sig, (1 - mu) / sig, loc=mu, scale=sig)
    assert stats.kstest(u[idx], tn.cdf).pvalue > 1e-3


# ------------------------------------------------------ adaptive Cartesian (f3)
def test_PC1_ac_uniform_marginals_are_the_prior(orc):
    """Uniform marginals: the AC draw is the prior draw and ln p - ln p_s = 0."""
    pr = orc.make_prior()
    th, lr, _ = orc.draw_ac(pr, orc.ac_init(), 0xAC, 2, 500, 4000)
    tp, _ = orc.draw_prior(pr, 0xAC, 2, 500, 4000)
    assert np.allclose(th, tp, rtol=1e-15, atol=1e-15)
    assert np.all(np.abs(lr) < 1e-14)


def test_PC2_ac_draws_follow_the_product_density(orc):
    """Random marginals: bin frequencies per column follow pi (chi-square),
    positions inside a bin are uniform (KS), and the importance identity
    E_ps[p/p_s] = 1 holds for the returned ln p - ln p_s."""
    from scipy import stats
    rng = np.random.default_rng(88)
    dims = list(range(7))
    pi = rng.dirichlet(np.full(orc.AC_BINS, 0.7), size=7)
    pi = 0.9 * pi + 0.1 / orc.AC_BINS
    st = orc.AcState(pi, dims)
    n = 200000
    th, lr, bins = orc.draw_ac(orc.make_prior(), st, 7, 0, 0, n)
    for k in range(7):
        cnt = np.bincount(bins[k], minlength=orc.AC_BINS)
        assert stats.chisquare(cnt, st.pi[k] / st.pi[k].sum() * n).pvalue > 1e-4
    u0 = th[0] / (2 * math.pi) * orc.AC_BINS
    assert np.all(np.floor(u0).astype(int) == bins[0])
    assert stats.kstest(u0 - bins[0], "uniform").pvalue > 1e-4
    r = np.exp(lr)
    assert abs(r.mean() - 1.0) < 4 * r.std() / math.sqrt(n)


def test_PC3_ac_estimator_unbiased_and_adapts(orc):
    """The seven-dimensional product Gaussian of PA4 integrated by AC rounds:
    p_s > 0 everywhere, so the pooled estimate agrees with the closed form
    within 4 sigma; the adapted marginals raise n_eff per sample."""
    from scipy.special import ndtr
    rng = np.random.default_rng(89)
    mu = rng.uniform(0.35, 0.65, 7)
    sig = np.full(7, 0.08)
    exact = float(np.sum(np.log(ndtr((1 - mu) / sig) - ndtr(-mu / sig))))
    norm = -0.5 * 7 * math.log(2 * math.pi) - float(np.sum(np.log(sig)))
    pr = orc.make_prior()
    st = orc.ac_init()
    n, lws, eff = 40000, [], []
    for r in range(6):
        th, lr, bins = orc.draw_ac(pr, st, 2025, r, 0, n)
        u = np.stack([th[0] / (2 * math.pi), (np.sin(th[1]) + 1) / 2, (th[2] + 0.028) / 0.056,
                      (th[3] ** 3 - 1.0) / (3000.0 ** 3 - 1.0), (th[4] + 1) / 2, th[5] / (2 * math.pi),
                      th[6] / math.pi])
        lnL = norm - 0.5 * np.sum(((u.T - mu) / sig) ** 2, axis=1)
        lw = lnL + lr
        lws.append(lw)
        eff.append(orc.marginalize(lw)["n_eff"] / n)
        st = orc.ac_update(st, bins, lw)
    o = orc.marginalize(np.concatenate(lws))
    sigma = math.exp(o["ln_sigma"] - o["ln_L"])
    assert abs(o["ln_L"] - exact) <= 4 * sigma + 1e-6, (o["ln_L"], exact, sigma)
    assert eff[-1] > 5 * eff[0], eff


def test_PC4_ac_update_histogram_closed_form(orc):
    """All weight inside one bin of the first coordinate: that marginal
    becomes 0.9 + 0.1/64 there and 0.1/64 elsewhere; with no finite weight the
    marginals are kept."""
    pr = orc.make_prior()
    st = orc.ac_init()
    th, lr, bins = orc.draw_ac(pr, st, 3, 0, 0, 50000)
    lw = np.where(bins[0] == 10, 0.0, -np.inf)
    st2 = orc.ac_update(st, bins, lw)
    want = np.full(orc.AC_BINS, 0.1 / orc.AC_BINS)
    want[10] += 0.9
    assert np.allclose(st2.pi[0], want, rtol=1e-15, atol=1e-18)
    assert abs(st2.cum[0, -1] - 1.0) == 0.0
    st3 = orc.ac_update(st, bins, np.full(50000, -np.inf))
    assert np.array_equal(st3.pi, st.pi)


# ------------------------------------------------------- Q, U, V precompute (f4)
def test_PQ1_window_Q_is_the_exact_Q_at_the_sample_times(orc, recs):
    """The windowed Q of the precompute equals the direct frequency sum of
    eq. (QUV) at each window time tau_i = (i - 205)/4096 (exact_Q, pinned by
    P1), for every detector, mode and time."""
    p, ev, hlm = _event(recs, "c2", ["H", "L", "V"], 9, q=3.0, noise=True, seed=5)
    Q, U, V = orc.overlaps_qv(hlm, ev["data"], None, ev["df"], 20.0, 1024.0, 410, 205)
    for k in range(3):
        for i in (0, 1, 137, 205, 409):
            ref = orc.exact_Q(ev["f"], ev["df"], hlm, ev["data"][k], (i - 205) / 4096.0)
            assert np.allclose(Q[k, :, i], ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())


@pytest.mark.parametrize("key,dets,n,q", [("c1", ["H", "L"], 5, 2.0), ("c3", ["H", "L", "V"], 17, 20.0)])
def test_PQ2_precomputed_U_V_give_rho2_over_2(orc, recs, key, dets, n, q):
    """With U and V from the precompute, the noiseless injection's lnL (exact
    Q) is rho^2/2 from the strains alone (P1), and U is Hermitian positive
    semi-definite, V symmetric; V built without the frequency reversal (a
    planted mistake: <h_a|h_b> in place of <h_a^*|h_b>) fails."""
    p, ev, hlm = _event(recs, key, dets, n, q=q)
    th = np.array(recs[key]["theta"])
    rho2 = chirpgen.network_snr2(ev["f"], ev["df"], ev["strain"])
    Q, U, V = orc.overlaps_qv(hlm, ev["data"], None, ev["df"], 20.0, 1024.0, 410, 205)
    for k in range(len(dets)):
        assert np.allclose(U[k], np.conj(U[k]).T, rtol=0, atol=1e-12 * np.abs(U[k]).max())
        assert np.allclose(V[k], V[k].T, rtol=0, atol=1e-12 * np.abs(V[k]).max())
        assert np.linalg.eigvalsh(U[k]).min() > -1e-10 * np.abs(U[k]).max()
    p2 = p.__class__(**{**p.__dict__})
    p2.U, p2.V = U, V
    l, _, _ = orc.lnL_exact(p2, th, ev["f"], ev["df"], hlm, ev["data"])
    assert abs(l - rho2 / 2) <= 1e-9 * rho2 / 2
    bad = p.__class__(**{**p.__dict__})
    bad.U, bad.V = U, U.copy()
    lb, _, _ = orc.lnL_exact(bad, th, ev["f"], ev["df"], hlm, ev["data"])
    assert abs(lb - rho2 / 2) > 1e-3


def test_PQ3_single_frequency_closed_form(orc):
    """One mode and one detector with a single band frequency f0 (and its
    mirror for V): Q(tau) = 2 df conj(h) d e^{2 pi i f0 tau}, U = 2 df |h|^2,
    V = 2 df h(-f0) h(f0); a PSD weight scales all three."""
    n, df = 4096, 0.5
    m0 = 300                                   # f0 = 150 Hz
    h = np.zeros((1, n), complex)
    d = np.zeros((1, n), complex)
    h[0, m0] = 0.3 - 0.4j
    h[0, n - m0] = 0.1 + 0.2j
    d[0, m0] = 1.5 + 0.5j
    w = np.full((1, n), 2.0)
    Q, U, V = orc.overlaps_qv(h, d, w, df, 20.0, 1024.0, 64, 32)
    tau = (np.arange(64) - 32) / (n * df)
    want = 2 * df * np.conj(h[0, m0]) * d[0, m0] * 2.0 * np.exp(2j * np.pi * 150.0 * tau)
    assert np.allclose(Q[0, 0], want, rtol=1e-13, atol=1e-15)
    assert abs(U[0, 0, 0] - 2 * df * 2.0 * (abs(h[0, m0]) ** 2 + abs(h[0, n - m0]) ** 2)) < 1e-14
    assert abs(V[0, 0, 0] - 2 * df * 2.0 * 2 * h[0, n - m0] * h[0, m0]) < 1e-14


def _u_of_theta(pr, th):
    """The prior's CDF coordinates of theta (the inverse of its map from u)."""
    u = np.empty((7, th.shape[1]))
    u[0] = th[0] / (2 * math.pi)
    u[1] = (np.sin(th[1]) + 1.0) / 2.0
    u[2] = (th[2] + pr.t_window) / (2 * pr.t_window)
    a3, b3 = pr.d_min ** 3, pr.d_max ** 3
    u[3] = (th[3] ** 3 - a3) / (b3 - a3)
    u[4] = (th[4] + 1.0) / 2.0
    u[5] = th[5] / (2 * math.pi)
    u[6] = th[6] / math.pi
    return u


def _mixture_rounds(orc, pr, fn, dims, n, rounds, seed):
    """n_eff / N of each round of the adaptive mixture (prior first, then the
    tempered EM refit after every round) on the integrand fn(u)."""
    state, g, eff = None, None, []
    for r in range(rounds):
        if g is None:
            th, _ = orc.draw_prior(pr, seed, r, 0, n)
            lr = np.zeros(n)
        else:
            th, lr = orc.draw_gmm(pr, g, seed, r, 0, n)
        lw = fn(_u_of_theta(pr, th)) + lr
        eff.append(orc.marginalize(lw)["n_eff"] / n)
        state = orc.em_fit(th, lw, dims, state=state, n_iter=8, n_comp=8, temper_ess=1 / 16,
                           t_window=pr.t_window, d_min=pr.d_min, d_max=pr.d_max)
        w, m, c = state
        g0 = orc.make_gmm(w, m, c, dims, eps_def=0.05)
        lz = [math.log(max(orc.gmm_inbox_mass(pr, g0, j, seed ^ 0x55, r), 1e-300)) for j in range(len(w))]
        g = orc.make_gmm(w, m, c, dims, ln_Z=lz, eps_def=0.05)
    return eff


def _av_rounds(orc, pr, fn, dims, n, rounds, seed, n_min_live):
    g = orc.AvGrid(1, np.zeros((1, len(dims)), dtype=np.int32), dims)
    eff = []
    for r in range(rounds):
        _, u = orc.draw_av(pr, g, seed, r, 0, n)
        uu = np.full((7, n), 0.5)
        uu[dims] = u
        lnL = fn(uu)
        eff.append(orc.marginalize(lnL + g.ln_vol)["n_eff"] / n)
        g, _ = orc.av_update(g, u, lnL, p_thr=0.999, n_min_live=n_min_live)
    return eff


def test_PA8_av_and_mixture_on_the_test_problems(orc):
    """The two integrators side by side on the section's test problems (n_eff
    per sample of each round, six rounds): on the Rosenbrock banana over two
    columns the adaptive volume settles near 0.12 from the third round on,
    while the mixture's efficiency swings by an order of magnitude between
    rounds; on a seven-dimensional Gaussian in the CDF coordinates the
    mixture reaches about half while the volume's uniform cells stay near
    1e-3.  Both start from the prior (the same first round)."""
    pr = orc.make_prior()

    def rosen(u):
        x, y = 4.0 * u[0] - 2.0, 4.0 * u[1] - 1.0
        return -((1.0 - x) ** 2 + 100.0 * (y - x * x) ** 2)

    av = _av_rounds(orc, pr, rosen, [0, 1], 20000, 6, 77, 1000)
    mx = _mixture_rounds(orc, pr, rosen, [0, 1], 20000, 6, 77)
    assert abs(av[0] - mx[0]) <= 1e-9 * av[0]   # the same prior round (u read back from theta)
    assert min(av[2:]) > 0.1 and max(av[2:]) < 1.5 * min(av[2:])
    assert max(mx[1:]) > 4 * min(mx[1:])

    rng = np.random.default_rng(84)
    mu = rng.uniform(0.35, 0.65, 7)
    sig = np.full(7, 0.08)
    norm = -0.5 * 7 * math.log(2 * math.pi) - float(np.sum(np.log(sig)))

    def gauss(u):
        return norm - 0.5 * np.sum(((u.T - mu) / sig) ** 2, axis=1)

    dims = list(range(7))
    av7 = _av_rounds(orc, pr, gauss, dims, 40000, 6, 2024, 2000)
    mx7 = _mixture_rounds(orc, pr, gauss, dims, 40000, 6, 2024)
    assert max(av7) < 0.01
    assert min(mx7[3:]) > 0.3
