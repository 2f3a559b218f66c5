"""Time-marginalised likelihood on the GPU vs the oracle: the (time) x
(extrinsic) array integrated over the time prior by the rectangle rule on
nodes j dt / R.  Per-sample tolerances as for the pointwise likelihood, with
the magnitude |s T1| + s^2 T2 / 4 taken at t = 0."""

import numpy as np
import pytest

import chirpgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2505_11655_amd as ile  # noqa: E402
from tests import gpu_util as gu  # noqa: E402

PNAME = {0: "fp64", 1: "fp32"}


@pytest.fixture(scope="module")
def recs():
    return chirpgen.load_injections()


def _gpu_tmarg(job, th_np, policy, R, lnpmps_np=None):
    n = th_np.shape[1]
    th = torch.from_numpy(np.ascontiguousarray(th_np)).to("cuda")
    lr = None if lnpmps_np is None else torch.from_numpy(np.ascontiguousarray(lnpmps_np)).to("cuda")
    L = torch.full((max(n, 1),), float("nan"), dtype=gu.out_dtype(policy), device="cuda")
    W = torch.full((max(n, 1),), float("nan"), dtype=gu.out_dtype(policy), device="cuda")
    ile.ile_eval_lnL_tmarg(job, n, th, n, lr, L, W, oversample=R)
    torch.cuda.synchronize()
    return L[:n].double().cpu().numpy(), W[:n].double().cpu().numpy()


def _check(orc, prob, th, got, policy, R):
    ref = orc.lnL_tmarg(prob, th.astype(np.float64), oversample=R)
    t0 = th.astype(np.float64).copy()
    t0[2] = 0.0
    _, T1, T2 = orc.lnL(prob, t0, return_terms=True)
    s = 100.0 / t0[3]
    return gu.tol_check(got, ref, T1, T2, s, policy), ref


def _samples(rng, th0, n_prior, n_peak, policy, widths):
    a = chirpgen.prior_samples(rng, n_prior)
    b = th0[:, None] + widths[:, None] * rng.standard_normal((7, n_peak))
    b[4] = np.clip(b[4], -1, 1)
    th = np.concatenate([a, b], axis=1)
    return np.ascontiguousarray(th.astype(np.float64 if policy == ile.ILE_FP64 else np.float32))


@pytest.mark.parametrize("R", [1, 4])
@pytest.mark.parametrize("policy", [ile.ILE_FP64, ile.ILE_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("cfg", ["hl5", "hlv9", "hlv17"])
def test_tmarg_matches_oracle(orc, recs, cfg, policy, R):
    """Prior samples (ragged count) plus samples near the peak of an SNR-20
    event; HL 5 modes (window staged in LDS), HLV 9 modes (FP32: LDS; FP64:
    L2) and HLV 17 modes (the strong-source mode set, q = 20)."""
    dets, n_modes, rec, q = {"hl5": (["H", "L"], 5, "c1", 2.0), "hlv9": (["H", "L", "V"], 9, "c2", 2.0),
                             "hlv17": (["H", "L", "V"], 17, "c3", 20.0)}[cfg]
    probs, _ = chirpgen.build_event(recs[rec], dets, n_modes, 30.0, q, 20.0, noise_seed=11)
    p = probs[0]
    th0 = np.array(recs[rec]["theta"])
    rng = np.random.default_rng(70)
    w = np.array([0.03, 0.03, 0.0, 0.05 * th0[3], 0.05, 0.1, 0.1])
    th = _samples(rng, th0, 1537, 300, policy, w)
    lr = rng.normal(size=th.shape[1]).astype(th.dtype)
    job = ile.ile_prepare(gu.ctx(), ile.ProblemHost(p, precision=policy))
    try:
        L, W = _gpu_tmarg(job, th, policy, R, lr)
    finally:
        ile.ile_job_release(job)
    (ok, ms, ma), ref = _check(orc, p, th, L, policy, R)
    print(f"{cfg} {PNAME[policy]} R={R} max lnL_t={np.max(ref):.2f} max|d| scoped={ms:.3e} all={ma:.3e}")
    assert ok
    fin = np.isfinite(L)
    tolw = 1e-12 if policy == ile.ILE_FP64 else 1e-5
    assert np.allclose(W[fin], L[fin] + lr[fin].astype(np.float64), rtol=tolw, atol=tolw)


def test_tmarg_window_edges_and_support(orc):
    """A time prior so wide that the outer nodes leave the window (those nodes
    contribute nothing, as the oracle's -inf), samples outside the support
    (D <= 0, |cos iota| > 1) give -inf, and n = 1 / n = 0 launches work."""
    rng = np.random.default_rng(71)
    p = chirpgen.random_problem(rng, 5, ["H", "L"])
    p.t_window = 0.0495
    th = chirpgen.prior_samples(rng, 700)
    th[3, :20] = -3.0
    th[4, 20:40] = 1.5
    th = np.ascontiguousarray(th)
    job = ile.ile_prepare(gu.ctx(), ile.ProblemHost(p, precision=ile.ILE_FP64))
    try:
        L, _ = _gpu_tmarg(job, th, ile.ILE_FP64, 4)
        L1, _ = _gpu_tmarg(job, np.ascontiguousarray(th[:, 100:101]), ile.ILE_FP64, 4)
        L0, _ = _gpu_tmarg(job, np.zeros((7, 0)), ile.ILE_FP64, 4)
    finally:
        ile.ile_job_release(job)
    ref = orc.lnL_tmarg(p, th, oversample=4)
    assert np.all(np.isneginf(L[:40])) and np.all(np.isneginf(ref[:40]))
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(L))
    assert np.allclose(L[fin], ref[fin], rtol=1e-9, atol=1e-9)
    assert abs(L1[0] - ref[100]) <= 1e-9 * (1 + abs(ref[100]))
    assert L0.size == 0


def test_tmarg_batch_equals_single(recs):
    """Several jobs in one launch: each result is bitwise the single-job one."""
    rng = np.random.default_rng(72)
    jobs, ths, singles = [], [], []
    try:
        for i, (n_modes, dets) in enumerate([(5, ["H", "L"]), (9, ["H", "L", "V"]), (5, ["H", "L"])]):
            p = chirpgen.random_problem(rng, n_modes, dets)
            job = ile.ile_prepare(gu.ctx(), ile.ProblemHost(p, precision=ile.ILE_FP32))
            th = np.ascontiguousarray(chirpgen.prior_samples(rng, 1000 + 333 * i).astype(np.float32))
            jobs.append(job)
            ths.append(th)
            singles.append(_gpu_tmarg(job, th, ile.ILE_FP32, 4)[0])
        tt = [torch.from_numpy(t).to("cuda") for t in ths]
        outs = [torch.empty(t.shape[1], dtype=torch.float32, device="cuda") for t in ths]
        ile.ile_eval_lnL_tmarg_batch(jobs, [t.shape[1] for t in ths], tt, [t.shape[1] for t in ths], None, outs,
                                     oversample=4)
        torch.cuda.synchronize()
        for k in range(len(jobs)):
            assert np.array_equal(outs[k].double().cpu().numpy(), singles[k])
    finally:
        for j in jobs:
            ile.ile_job_release(j)


def test_tmarg_rejects():
    rng = np.random.default_rng(73)
    p = chirpgen.random_problem(rng, 5, ["H", "L"])
    th = torch.zeros((7, 10), dtype=torch.float32, device="cuda")
    out = torch.zeros(10, dtype=torch.float32, device="cuda")
    job = ile.ile_prepare(gu.ctx(), ile.ProblemHost(p, precision=ile.ILE_FP32))
    try:
        with pytest.raises(ile.IleError):
            ile.ile_eval_lnL_tmarg(job, 10, th, 10, None, out, oversample=2)
    finally:
        ile.ile_job_release(job)
    for kw in ({"precision": ile.ILE_FP32_CANCEL64},):
        job = ile.ile_prepare(gu.ctx(), ile.ProblemHost(p, **kw))
        try:
            with pytest.raises(ile.IleError):
                ile.ile_eval_lnL_tmarg(job, 10, th, 10, None, out, oversample=4)
        finally:
            ile.ile_job_release(job)


@pytest.mark.parametrize("R,n_prior,n_peak", [(1, 8, 8), (4, 0, 4)])
@pytest.mark.parametrize("policy", [ile.ILE_FP64, ile.ILE_FP32], ids=["fp64", "fp32"])
def test_tmarg_with_distance_matches_oracle(orc, recs, policy, R, n_prior, n_peak):
    """Time and distance integrated together (a dist_marg job): every node's
    value is the distance table's ln L_D(T1(t_j), T2); the oracle takes the
    distance integral at every node by adaptive quadrature.  HL 5 modes,
    SNR 20; prior samples and samples near the peak (the D column ignored).
    FP64 agrees to the table's accuracy near the peak, FP32 to the FP32
    policy's per-sample bound."""
    probs, _ = chirpgen.build_event(recs["c1"], ["H", "L"], 5, 30.0, 2.0, 20.0, noise_seed=11)
    p = probs[0]
    th0 = np.array(recs["c1"]["theta"])
    rng = np.random.default_rng(72)
    w = np.array([0.03, 0.03, 0.0, 0.0, 0.05, 0.1, 0.1])
    th = _samples(rng, th0, n_prior, n_peak, policy, w)
    th[3] = p.d_ref
    job = ile.ile_prepare(gu.ctx(), ile.ProblemHost(p, precision=policy, dist_marg=True))
    try:
        L, _ = _gpu_tmarg(job, th, policy, R)
    finally:
        ile.ile_job_release(job)
    ref = orc.lnL_tmarg_dist(p, th.astype(np.float64), oversample=R)
    assert np.array_equal(np.isfinite(L), np.isfinite(ref))
    fin = np.isfinite(ref)
    d = np.abs(L[fin] - ref[fin])
    print(f"tmarg+dist {PNAME[policy]} R={R}: max lnL={np.max(ref):.2f} max|d|={d.max():.2e}")
    if policy == ile.ILE_FP64:
        assert np.all(d <= 1e-5 * (1 + np.abs(ref[fin])))
    else:
        assert np.all(d <= 1e-3 + 1e-6 * np.abs(ref[fin]))
