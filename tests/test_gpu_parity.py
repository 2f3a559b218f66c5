"""Parity of the HIP path (through the C ABI) with the CPU oracle on identical
seeded inputs: per-sample lnL for every precision policy and compiled mode set,
the Monte Carlo estimator, and the counter-based prior draws."""
import math

import numpy as np
import pytest

import chirpgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2505_11655_amd as ile  # noqa: E402
from tests import gpu_util as gu  # noqa: E402

POLICIES = [ile.ILE_FP64, ile.ILE_FP32, ile.ILE_FP32_CANCEL64]
PNAME = {0: "fp64", 1: "fp32", 2: "fp32c64"}


@pytest.fixture(scope="module")
def recs():
    return chirpgen.load_injections()


def _np_theta(th, policy):
    return np.ascontiguousarray(th.astype(np.float64 if policy == ile.ILE_FP64 else np.float32))


def _run(orc, prob, th, policy, lnpmps=None, eps=0.0, ref=None):
    ph = ile.ProblemHost(prob, precision=policy, mode_filter_eps=eps)
    job = ile.ile_prepare(gu.ctx(), ph)
    try:
        if ref is not None:
            ile.ile_set_reference(job, ref)
        L, W = gu.gpu_eval(job, th, policy, lnpmps)
    finally:
        ile.ile_job_release(job)
    ref, T1, T2 = orc.lnL(prob, th.astype(np.float64), return_terms=True)
    s = 100.0 / th[3].astype(np.float64)
    return L, W, ref, T1, T2, s


@pytest.mark.parametrize("policy", POLICIES, ids=[PNAME[p] for p in POLICIES])
@pytest.mark.parametrize("cfg", ["hl5", "hlv9", "hlv17"])
def test_eval_prior_samples(orc, recs, policy, cfg):
    """Prior-drawn samples (ragged count) on physical inputs, the three
    workload shapes: H,L with 5 modes; H,L,V with 9; H,L,V with 17 (q = 20)."""
    dets, n_modes, rec, mc, q, snr = {
        "hl5": (["H", "L"], 5, "c1", 30.0, 2.0, 20.0),
        "hlv9": (["H", "L", "V"], 9, "c2", 30.0, 2.0, 20.0),
        "hlv17": (["H", "L", "V"], 17, "c3", 30.0, 20.0, 20.0),
    }[cfg]
    probs, _ = chirpgen.build_event(recs[rec], dets, n_modes, mc, q, snr, noise_seed=11,
                                    templates=[(mc * 1.01, q)])
    rng = np.random.default_rng(21)
    th = _np_theta(chirpgen.prior_samples(rng, 40961), policy)
    L, W, ref, T1, T2, s = _run(orc, probs[0], th, policy)
    ok, ms, ma = gu.tol_check(L, ref, T1, T2, s, policy)
    print(f"{cfg} {PNAME[policy]} max|d| scoped={ms:.3e} all={ma:.3e}")
    assert ok
    assert np.array_equal(np.isfinite(W), np.isfinite(L))


@pytest.mark.parametrize("snr", [100.0, 400.0])
def test_eval_precision_strong_source(orc, recs, snr):
    """Loud edge-on q = 20 source, 17 modes, samples near the peak: the
    FP32 + FP64-cancellation policy, its reference at the box centre, meets
    1e-3 per sample (scoped); plain FP32 is reported for contrast."""
    probs, _ = chirpgen.build_event(recs["c3"], ["H", "L", "V"], 17, 30.0, 20.0, snr, noise_seed=5)
    th0 = np.array(recs["c3"]["theta"])
    sc = 100.0 / snr
    widths = np.array([0.01, 0.01, 1e-4, 0.05 * th0[3], 0.02, 0.05, 0.05]) * sc * 3
    rng = np.random.default_rng(22)
    thd = chirpgen.box_samples(rng, 30000, th0, widths)
    res = {}
    for policy in (ile.ILE_FP32_CANCEL64, ile.ILE_FP32):
        th = _np_theta(thd, policy)
        L, W, ref, T1, T2, s = _run(orc, probs[0], th, policy, ref=th0)
        ok, ms, ma = gu.tol_check(L, ref, T1, T2, s, policy)
        res[policy] = (ok, ms, ma, float(np.max(ref)))
        print(f"SNR {snr} {PNAME[policy]} max lnL={np.max(ref):.1f} max|d| scoped={ms:.3e} all={ma:.3e}")
    assert res[ile.ILE_FP32_CANCEL64][0]


@pytest.mark.parametrize("snr", [100.0, 400.0])
def test_c3_marginal_matches_oracle(orc, recs, snr):
    """The precision configuration end to end: H, L, V, 17 modes, q = 20,
    edge-on, SNR 100 and 400; 2^20 draws of a narrow 8-component Gaussian
    mixture over the 7 extrinsic parameters (means scattered by sigma/2
    about the injection, covariance diag(sigma^2), sigma shrinking as 1/SNR)
    with their ln p - ln p_s.  GPU lnL + estimator against the oracle on the
    same draws and weights, the mixture also set on the job (which places
    the reference of the FP32 + FP64-cancellation policy): that policy within
    1e-4 on the marginal ln L and 1e-3 per sample (scoped).  Plain FP32 is
    reported; its lw alone is quantised to ~1e-2 at lnL ~ 8e4."""
    probs, _ = chirpgen.build_event(recs["c3"], ["H", "L", "V"], 17, 30.0, 20.0, snr, noise_seed=5)
    prob = probs[0]
    th0 = np.array(recs["c3"]["theta"])
    sig = np.array([0.01, 0.01, 1e-4, 0.05 * th0[3], 0.02, 0.05, 0.05]) * (100.0 / snr)
    rng = np.random.default_rng(31)
    means = th0[None, :] + rng.normal(size=(8, 7)) * sig[None, :] / 2
    covs = [np.diag(sig ** 2)] * 8
    prior = orc.make_prior(t_window=prob.t_window, d_min=prob.d_min, d_max=prob.d_max)
    g = orc.make_gmm(np.full(8, 1.0 / 8), means, covs, list(range(7)))
    thd, lrd = orc.draw_gmm(prior, g, 0xC3C3, int(snr), 0, 1 << 20)
    out = {}
    for policy in (ile.ILE_FP32_CANCEL64, ile.ILE_FP32):
        th = _np_theta(thd, policy)
        lr = lrd.astype(th.dtype)
        job = ile.ile_prepare(gu.ctx(), ile.ProblemHost(prob, precision=policy))
        try:
            # the same mixture on the job: the FP32 + FP64-cancellation policy
            # takes its reference from it (the heaviest component's mean)
            ile.ile_set_proposal(job, ile.gmm_params(np.full(8, 1.0 / 8), means, covs))
            L, W = gu.gpu_eval(job, th, policy, lr)
            r = _gpu_marg(job, W, ile.ILE_FP64 if policy == ile.ILE_FP32_CANCEL64 else policy)
        finally:
            ile.ile_job_release(job)
        ref, T1, T2 = orc.lnL(prob, th.astype(np.float64), return_terms=True)
        o = orc.marginalize(ref + lr.astype(np.float64))
        ok, ms, ma = gu.tol_check(L, ref, T1, T2, 100.0 / th[3].astype(np.float64), policy)
        out[policy] = (abs(r["ln_L"] - o["ln_L"]), ok, ms)
        print(f"C3 SNR {snr} {PNAME[policy]}: ln L gpu {r['ln_L']:.6f} oracle {o['ln_L']:.6f} "
              f"|d| {out[policy][0]:.2e} n_eff {o['n_eff']:.1f} max|d lnL| scoped {ms:.2e}")
    d, ok, ms = out[ile.ILE_FP32_CANCEL64]
    assert d <= 1e-4 and ms <= 1e-3


@pytest.mark.parametrize("where", ["none", "near", "far", "outside"])
def test_reference_independence(orc, recs, where):
    """FP32 + FP64 cancellation: lnL does not depend on the reference point
    beyond rounding.  SNR-20 HLV 9-mode event, prior draws and a box about
    the injection; reference none, at the injection, at a far prior draw, and
    outside the support (clears it).  Every case within the per-sample bound."""
    probs, _ = chirpgen.build_event(recs["c2"], ["H", "L", "V"], 9, 30.0, 2.0, 20.0, noise_seed=7)
    th0 = np.array(recs["c2"]["theta"])
    rng = np.random.default_rng(41)
    thp = chirpgen.prior_samples(rng, 20000)
    thb = chirpgen.box_samples(rng, 20000, th0, np.array([0.03, 0.03, 3e-4, 0.1 * th0[3], 0.05, 0.2, 0.2]))
    thd = np.concatenate([thp, thb], axis=1)
    ref_pt = {"none": None, "near": th0, "far": thp[:, 17].copy(),
              "outside": np.array([1.0, 0.2, 0.0, -5.0, 0.3, 1.0, 1.0])}[where]
    th = _np_theta(thd, ile.ILE_FP32_CANCEL64)
    L, W, ref, T1, T2, s = _run(orc, probs[0], th, ile.ILE_FP32_CANCEL64, ref=ref_pt)
    ok, ms, ma = gu.tol_check(L, ref, T1, T2, s, ile.ILE_FP32_CANCEL64)
    print(f"reference {where}: max|d| scoped={ms:.3e} all={ma:.3e}")
    assert ok


@pytest.mark.parametrize("policy", POLICIES, ids=[PNAME[p] for p in POLICIES])
@pytest.mark.parametrize("case", ["all21_k3", "k1_pad", "subset_scrambled", "k2_set17", "set9_k2"])
def test_eval_random_inputs(orc, policy, case):
    """Random Hermitian/symmetric inputs over every compiled mode set, one
    detector (padded), and a scrambled mode subset placed in a larger set."""
    rng = np.random.default_rng(hash(case) % 2 ** 32)
    if case == "all21_k3":
        p = chirpgen.random_problem(rng, 21, ["H", "L", "V"])
    elif case == "k1_pad":
        p = chirpgen.random_problem(rng, 9, ["V"])
    elif case == "k2_set17":
        p = chirpgen.random_problem(rng, 17, ["L", "V"])
    elif case == "set9_k2":
        p = chirpgen.random_problem(rng, 9, ["H", "V"])
    else:
        p = chirpgen.random_problem(rng, 21, ["H", "L"])
        keep = [14, 4, 0, 20, 9]           # (4,-2),(2,2),(2,-2),(4,4),(3,1) in scrambled order
        p.modes = [p.modes[a] for a in keep]
        p.Q, p.U, p.V = p.Q[:, keep], p.U[:, keep][:, :, keep], p.V[:, keep][:, :, keep]
    th = _np_theta(chirpgen.prior_samples(rng, 9999), policy)
    L, W, ref, T1, T2, s = _run(orc, p, th, policy)
    ok, ms, ma = gu.tol_check(L, ref, T1, T2, s, policy)
    print(f"{case} {PNAME[policy]} max|d| scoped={ms:.3e} all={ma:.3e}")
    assert ok


@pytest.mark.parametrize("policy", POLICIES, ids=[PNAME[p] for p in POLICIES])
def test_eval_edge_cases(orc, policy):
    """Outside the support gives -inf exactly where the oracle does; n = 1,
    n = 0 and lw = lnL + (ln p - ln p_s)."""
    rng = np.random.default_rng(23)
    p = chirpgen.random_problem(rng, 5, ["H", "L"])
    th = chirpgen.prior_samples(rng, 600)
    th[3, 0:50] = -5.0                  # D <= 0
    th[3, 50:60] = 0.0
    th[4, 60:110] = 1.5                 # |cos iota| > 1
    th[2, 110:160] = 0.2                # far outside the window
    th[2, 160:170] = np.nan
    th = _np_theta(th, policy)
    lr = rng.normal(size=600).astype(th.dtype)
    L, W, ref, T1, T2, s = _run(orc, p, th, policy, lnpmps=lr)
    assert np.all(np.isneginf(L[:160]))
    assert np.all(np.isneginf(ref[:160]))
    ok, _, _ = gu.tol_check(L, ref, T1, T2, s, policy)
    assert ok
    fin = np.isfinite(L)
    tolw = 1e-12 if policy == ile.ILE_FP64 else 1e-5
    assert np.allclose(W[fin], L[fin] + lr[fin].astype(np.float64), rtol=tolw, atol=tolw)
    # single sample and empty launch
    ph = ile.ProblemHost(p, precision=policy)
    job = ile.ile_prepare(gu.ctx(), ph)
    try:
        L1, _ = gu.gpu_eval(job, np.ascontiguousarray(th[:, 200:201]), policy)
        ref1 = orc.lnL(p, th[:, 200:201].astype(np.float64))
        assert abs(L1[0] - ref1[0]) <= (1e-9 if policy == 0 else 1e-3) * (1 + abs(ref1[0]))
        L0, _ = gu.gpu_eval(job, np.zeros((7, 0), dtype=th.dtype), policy)
        assert L0.size == 0
    finally:
        ile.ile_job_release(job)


def test_mode_filter(orc, recs):
    """eps > 0 keeps (l,m) iff some |U_0[lm][l'm'] / U_0[22][22]| > eps; the
    result equals the oracle on the kept modes."""
    probs, _ = chirpgen.build_event(recs["c2"], ["H", "L", "V"], 17, 30.0, 1.2, 20.0, noise_seed=3)
    p = probs[0]
    U0 = p.U[0]
    a22 = p.modes.index((2, 2))
    eps = 0.02
    keep = [a for a in range(len(p.modes)) if np.max(np.abs(U0[a]) / abs(U0[a22, a22])) > eps]
    assert 0 < len(keep) < len(p.modes)
    pk = chirpgen.Problem(**{**p.__dict__})
    pk.modes = [p.modes[a] for a in keep]
    pk.Q, pk.U, pk.V = p.Q[:, keep], p.U[:, keep][:, :, keep], p.V[:, keep][:, :, keep]
    rng = np.random.default_rng(24)
    th = chirpgen.prior_samples(rng, 5000)
    ph = ile.ProblemHost(p, precision=ile.ILE_FP64, mode_filter_eps=eps)
    job = ile.ile_prepare(gu.ctx(), ph)
    try:
        assert ile.ile_job_info_get(job).n_modes_kept == len(keep)
        L, _ = gu.gpu_eval(job, th, ile.ILE_FP64)
    finally:
        ile.ile_job_release(job)
    ref, T1, T2 = orc.lnL(pk, th, return_terms=True)
    ok, _, _ = gu.tol_check(L, ref, T1, T2, 100.0 / th[3], ile.ILE_FP64)
    assert ok


def test_prepare_rejects_bad_inputs():
    rng = np.random.default_rng(25)
    p = chirpgen.random_problem(rng, 5, ["H", "L"])
    bad = chirpgen.Problem(**{**p.__dict__})
    bad.U = p.U.copy()
    bad.U[0, 0, 1] += 1.0              # not Hermitian
    with pytest.raises(ile.IleError) as e:
        ile.ile_prepare(gu.ctx(), ile.ProblemHost(bad))
    assert e.value.status == -1
    bad = chirpgen.Problem(**{**p.__dict__})
    bad.Q = p.Q.copy()
    bad.Q[1, 2, 3] = np.nan
    with pytest.raises(ile.IleError):
        ile.ile_prepare(gu.ctx(), ile.ProblemHost(bad))
    bad = chirpgen.Problem(**{**p.__dict__})
    bad.modes = [(2, 2), (2, 2), (2, 0), (2, 1), (2, -1)]
    with pytest.raises(ile.IleError):
        ile.ile_prepare(gu.ctx(), ile.ProblemHost(bad))
    # the context stays usable after rejected inputs
    job = ile.ile_prepare(gu.ctx(), ile.ProblemHost(p))
    ile.ile_job_release(job)


# ------------------------------------------------------------------ estimator
def _gpu_marg(job, lw, policy, flags=ile.ILE_MARG_RESET, offset=0):
    """`offset` > 0 places lw that many elements into its buffer (an input
    that is not 16-byte aligned)."""
    dt = np.float32 if policy == ile.ILE_FP32 else np.float64
    buf = np.zeros(len(lw) + offset, dtype=dt)
    buf[offset:] = lw
    t = torch.from_numpy(buf).to("cuda")
    return ile.ile_marginalize(job, len(lw), t[offset:], flags)


@pytest.mark.parametrize("policy", [ile.ILE_FP64, ile.ILE_FP32])
def test_marginalize_parity(orc, policy):
    rng = np.random.default_rng(26)
    p = chirpgen.random_problem(rng, 5, ["H", "L"])
    job = ile.ile_prepare(gu.ctx(), ile.ProblemHost(p, precision=policy))
    try:
        inner = rng.normal(size=40000) * 50
        inner[[100, 2049, 9000]] = [np.inf, np.nan, -np.inf]      # inside full vector steps
        inner[[777, 30000]] = 400.0                              # tied maxima: the lower index wins
        far = rng.normal(size=60000) - 200.0                     # most terms below the skip cut
        far[[5, 33333]] = [-150.0, 10.0]
        cases = [(rng.uniform(-1e5, 1e5, 100003), 0), (rng.normal(size=70001) * 30 - 500, 0),
                 (np.full(5000, -3.25), 0), (np.array([7.0]), 0), (np.array([-np.inf] * 17), 0),
                 (np.concatenate([rng.normal(size=4000), [np.inf, np.nan, -np.inf]]), 0),
                 (inner, 0), (far, 0), (rng.normal(size=50007) * 10, 1), (inner, 3)]
        for lw, off in cases:
            if policy == ile.ILE_FP32:
                lw = lw.astype(np.float32).astype(np.float64)
            r = _gpu_marg(job, lw, policy, offset=off)
            o = orc.marginalize(lw)
            assert r["n"] == o["n"] and r["n_nonfinite"] == o["n_nonfinite"] and r["argmax"] == o["argmax"]
            if o["ln_L"] == -np.inf:
                assert r["ln_L"] == -np.inf and r["n_eff"] == 0
                continue
            assert abs(r["ln_L"] - o["ln_L"]) <= 1e-12 * max(1, abs(o["ln_L"]))
            assert abs(r["n_eff"] - o["n_eff"]) <= 1e-11 * o["n_eff"]
            assert abs(r["n_ess"] - o["n_ess"]) <= 1e-11 * o["n_ess"]
            if len(lw) > 1:
                if np.isfinite(o["ln_sigma"]):
                    assert abs(r["ln_sigma"] - o["ln_sigma"]) <= 1e-9 * max(1, abs(o["ln_sigma"]))
                else:                      # equal weights: zero spread on both sides
                    assert r["ln_sigma"] == o["ln_sigma"]
        # pooling over batches equals one pass over the concatenation
        a, b = rng.normal(size=30000) * 5, rng.normal(size=20011) * 5 + 3
        _gpu_marg(job, a, policy, ile.ILE_MARG_RESET)
        r = _gpu_marg(job, b, policy, ile.ILE_MARG_POOL)
        cat = np.concatenate([a, b])
        if policy == ile.ILE_FP32:
            cat = cat.astype(np.float32).astype(np.float64)
        o = orc.marginalize(cat)
        assert r["n"] == o["n"] and r["argmax"] == o["argmax"]
        assert abs(r["ln_L"] - o["ln_L"]) <= 1e-12 * max(1, abs(o["ln_L"]))
        # empty call leaves the pooled state unchanged
        r2 = ile.ile_marginalize(job, 0, None, ile.ILE_MARG_POOL)
        assert r2["n"] == r["n"] and r2["ln_L"] == r["ln_L"]
    finally:
        ile.ile_job_release(job)


@pytest.mark.parametrize("policy", POLICIES, ids=[PNAME[p] for p in POLICIES])
def test_eval_batch_equals_single(policy):
    """The batched likelihood sizes its tiles from the batch total (256 to
    8192 samples); every sample's lnL and lw equal the single-job call's to
    the bit in every policy, for one-job batches of 1, 300, 2^17 + 5 and
    2^21 + 3 samples and for all four in one batch.  A batch of 64 copies of
    the 2^17 + 5 job (8.4M samples) runs the LDS-staged kernel, which the job
    alone never does: its results too equal the single-job call's to the bit.
    (Every compiled copy of the likelihood makes the same multiply-add
    fusions, so a sample's value does not depend on which copy ran it; a
    misplaced tile would show O(1) differences.)"""
    rng = np.random.default_rng(28)
    sizes = [1, 300, (1 << 17) + 5, (1 << 21) + 3]
    dt = torch.float64 if policy == ile.ILE_FP64 else torch.float32
    ot = gu.out_dtype(policy)
    p = chirpgen.random_problem(rng, 5, ["H", "L"])
    job = ile.ile_prepare(gu.ctx(), ile.ProblemHost(p, precision=policy))
    try:
        ths = [torch.from_numpy(np.ascontiguousarray(chirpgen.prior_samples(rng, n))).to(device="cuda", dtype=dt)
               for n in sizes]
        lrs = [torch.from_numpy(rng.normal(size=n)).to(device="cuda", dtype=dt) for n in sizes]
        single = []
        for n, th, lr in zip(sizes, ths, lrs):
            L = torch.empty(n, dtype=ot, device="cuda")
            W = torch.empty(n, dtype=ot, device="cuda")
            ile.ile_eval_lnL(job, n, th, n, lr, L, W)
            single.append((L, W))

        def batch(idx):
            Ls = [torch.empty(sizes[i], dtype=ot, device="cuda") for i in idx]
            Ws = [torch.empty(sizes[i], dtype=ot, device="cuda") for i in idx]
            ile.ile_eval_lnL_batch([job] * len(idx), [sizes[i] for i in idx], [ths[i] for i in idx],
                                   [sizes[i] for i in idx], [lrs[i] for i in idx], Ls, Ws)
            return Ls, Ws

        runs = [([i], batch([i])) for i in range(len(sizes))] + [(list(range(len(sizes))), batch(range(len(sizes))))]
        # LDS-staged regime: 64 copies of job 2 in one batch
        runs.append(([2] * 64, batch([2] * 64)))
        torch.cuda.synchronize()
        for idx, (Ls, Ws) in runs:
            for i, L, W in zip(idx, Ls, Ws):
                for got, ref in ((L, single[i][0]), (W, single[i][1])):
                    g, r = got.double().cpu().numpy(), ref.double().cpu().numpy()
                    assert np.array_equal(np.isfinite(g), np.isfinite(r)), (idx[:4], sizes[i])
                    f = np.isfinite(r)
                    d = np.abs(g[f] - r[f])
                    assert d.size == 0 or d.max() == 0.0, (PNAME[policy], len(idx), sizes[i], d.max())
    finally:
        ile.ile_job_release(job)


@pytest.mark.parametrize("policy", [ile.ILE_FP64, ile.ILE_FP32])
def test_marginalize_batch_equals_single(policy):
    """The batched estimator and the single-job one use the same tile for a
    job of n samples (2048 up to 16384, by n), so they agree to the bit: job
    sizes from one sample to 3 * 2^20 cover every tile size and ragged
    tails, all in one batch."""
    rng = np.random.default_rng(27)
    sizes = [1, 2047, 2048 * 64 + 5, (1 << 18) + 3, (1 << 20) + 7, 3 << 20]
    dt = torch.float32 if policy == ile.ILE_FP32 else torch.float64
    jobs, bufs = [], []
    try:
        for k, n in enumerate(sizes):
            p = chirpgen.random_problem(rng, 5, ["H", "L"])
            jobs.append(ile.ile_prepare(gu.ctx(), ile.ProblemHost(p, precision=policy)))
            lw = rng.normal(size=n) * 20 - 50 * k
            lw[rng.integers(0, n, size=min(n, 3))] = -np.inf
            bufs.append(torch.from_numpy(lw).to(device="cuda", dtype=dt))
        batch = ile.ile_marginalize_batch(jobs, sizes, bufs, ile.ILE_MARG_RESET)
        torch.cuda.synchronize()
        for job, n, buf, rb in zip(jobs, sizes, bufs, batch):
            rs = ile.ile_marginalize(job, n, buf, ile.ILE_MARG_RESET)
            for key in ("n", "n_nonfinite", "argmax", "ln_L", "n_eff", "n_ess", "max_lw"):
                assert rs[key] == rb[key], (n, key, rs[key], rb[key])
    finally:
        for j in jobs:
            ile.ile_job_release(j)


@pytest.mark.parametrize("noise_seed", [9, 1, 4])
def test_eval_then_marginalize_matches_oracle(orc, recs, noise_seed):
    """End to end on the small workload: GPU lnL + estimator vs oracle on the
    same samples over three noise realisations: |d ln L| <= 1e-10 (FP64) and
    <= 1e-4 (FP32, and FP32 with the FP64 cancellation term).  The
    realisations include n_eff = 1 cases (one dominant sample at lnL ~ 150),
    where the marginal's error is that sample's own error."""
    probs, _ = chirpgen.build_event(recs["c1"], ["H", "L"], 5, 30.0, 2.0, 20.0, noise_seed=noise_seed)
    rng = np.random.default_rng(27 + noise_seed)
    thd = chirpgen.prior_samples(rng, 1 << 17)
    for policy, tol in ((ile.ILE_FP64, 1e-10), (ile.ILE_FP32, 1e-4), (ile.ILE_FP32_CANCEL64, 1e-4)):
        th = _np_theta(thd, policy)
        job = ile.ile_prepare(gu.ctx(), ile.ProblemHost(probs[0], precision=policy))
        try:
            L, W = gu.gpu_eval(job, th, policy)
            r = _gpu_marg(job, W, policy if policy != ile.ILE_FP32_CANCEL64 else ile.ILE_FP64)
        finally:
            ile.ile_job_release(job)
        o = orc.marginalize(orc.lnL(probs[0], th.astype(np.float64)))
        print(PNAME[policy], "lnL_marg gpu", r["ln_L"], "oracle", o["ln_L"], "n_eff", o["n_eff"])
        assert abs(r["ln_L"] - o["ln_L"]) <= tol


# ---------------------------------------------------------------------- draws
@pytest.mark.parametrize("policy", [ile.ILE_FP64, ile.ILE_FP32])
def test_prior_draw_parity(orc, policy):
    rng = np.random.default_rng(28)
    p = chirpgen.random_problem(rng, 5, ["H", "L"])
    job = ile.ile_prepare(gu.ctx(), ile.ProblemHost(p, precision=policy))
    n, first, seed, rnd = 20011, 12345, 0xDEADBEEF12345678, 3
    th = torch.empty((7, n), dtype=gu.torch_dtype(policy), device="cuda")
    lr = torch.full((n,), 9.0, dtype=gu.torch_dtype(policy), device="cuda")
    try:
        ile.ile_draw(job, seed, rnd, first, n, th, n, lr)
        torch.cuda.synchronize()
    finally:
        ile.ile_job_release(job)
    g = th.double().cpu().numpy()
    o, _ = orc.draw_prior(orc.make_prior(), seed, rnd, first, n)
    if policy == ile.ILE_FP64:
        assert np.allclose(g, o, rtol=1e-14, atol=1e-15)
    else:
        assert np.allclose(g, o.astype(np.float32).astype(np.float64), rtol=2e-7, atol=1e-12)
    assert np.all(lr.cpu().numpy() == 0.0)


def test_prepare_from_device_arrays(orc, recs):
    """ile_problem arrays in device memory (mem_is_device = 1) give the same
    job as host arrays: identical lnL, bitwise, in every policy; the server
    takes them too."""
    import ctypes as C
    probs, _ = chirpgen.build_event(recs["c2"], ["H", "L", "V"], 9, 30.0, 2.0, 20.0, noise_seed=3)
    prob = probs[0]
    rng = np.random.default_rng(61)
    thd = chirpgen.prior_samples(rng, 5000)
    for policy in POLICIES:
        ph = ile.ProblemHost(prob, precision=policy)
        # the same arrays on the device
        keep = {}
        dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int32)

        def dev(a, ctype):
            t = torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
            keep[id(t)] = t
            return C.cast(C.c_void_p(t.data_ptr()), ctype)
        sd = ile.ile_problem.from_buffer_copy(ph.s)
        sd.mem_is_device = 1
        sd.mode_l, sd.mode_m = dev(ph.ml, ip), dev(ph.mm, ip)
        sd.det_pos, sd.det_resp = dev(ph.pos, dp), dev(ph.resp, dp)
        sd.Q, sd.U = dev(ph.Q, dp), dev(ph.U, dp)
        sd.V = dev(ph.V, dp)
        torch.cuda.synchronize()
        jh = ile.ile_prepare(gu.ctx(), ph)
        hd = ile.ile_prepare(gu.ctx(), sd)
        try:
            th = _np_theta(thd, policy)
            Lh, _ = gu.gpu_eval(jh, th, policy)
            Ld, _ = gu.gpu_eval(hd, th, policy)
        finally:
            ile.ile_job_release(jh)
            ile.ile_job_release(hd)
        f = np.isfinite(Lh)
        assert np.array_equal(f, np.isfinite(Ld)) and np.array_equal(Lh[f], Ld[f]), PNAME[policy]
    # the server copies device arrays as well
    srv = ile.ile_server_create(gu.ctx())
    try:
        r = ile.ile_server_wait(srv, ile.ile_server_submit(srv, sd, ile.job_opts(n_samples=4096, seed=5)), 60000)
        rh = ile.ile_server_wait(srv, ile.ile_server_submit(srv, ph, ile.job_opts(n_samples=4096, seed=5)), 60000)
    finally:
        ile.ile_server_destroy(srv)
    assert r.status == 0 and rh.status == 0 and r.marg.ln_L == rh.marg.ln_L
