"""Fair draws from weighted samples on the GPU: indices bit-exact against the
oracle (integer masses and prefix sums on both sides) on a ragged sample
count with non-finite weights, the drawn samples copied out, the no-weight
case, and the resampling check on an ILE run: the fair draws reproduce the
weighted distribution of the run's samples in every column."""
import numpy as np
import pytest

import chirpgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2505_11655_amd as ile  # noqa: E402
from tests import gpu_util as gu  # noqa: E402


def _job(policy, seed=110):
    rng = np.random.default_rng(seed)
    p = chirpgen.random_problem(rng, 5, ["H", "L"])
    return ile.ile_prepare(gu.ctx(), ile.ProblemHost(p, precision=policy))


@pytest.mark.parametrize("policy", [ile.ILE_FP64, ile.ILE_FP32, ile.ILE_FP32_CANCEL64],
                         ids=["fp64", "fp32", "fp32c64"])
@pytest.mark.parametrize("n", [1, 4095, 100003])
def test_fair_draw_matches_oracle(orc, policy, n):
    rng = np.random.default_rng(111 + n)
    lw = rng.normal(0, 4, n)
    if n > 10:
        lw[rng.choice(n, n // 20, replace=False)] = -np.inf
        lw[rng.choice(n, 3, replace=False)] = np.nan
        lw[5] = lw[np.isfinite(lw)].max()          # a tie at the maximum
    odt = np.float32 if policy == ile.ILE_FP32 else np.float64
    tdt = np.float64 if policy == ile.ILE_FP64 else np.float32
    lw = lw.astype(odt)
    th = rng.normal(size=(7, n)).astype(tdt)
    k = 30011
    job = _job(policy)
    try:
        lw_d = torch.from_numpy(lw).to("cuda")
        th_d = torch.from_numpy(th).to("cuda")
        idx = torch.full((k,), -7, dtype=torch.int64, device="cuda")
        out = torch.zeros((7, k), dtype=th_d.dtype, device="cuda")
        ile.ile_fair_draw(job, n, lw_d, 0xFA1, 4, k, idx, th_d, n, out, k)
        torch.cuda.synchronize()
        g = idx.cpu().numpy()
    finally:
        ile.ile_job_release(job)
    o = orc.fair_draw(lw.astype(np.float64), 0xFA1, 4, k)
    assert np.array_equal(g, o)
    assert np.array_equal(out.cpu().numpy(), th[:, o])


def test_fair_draw_without_weight_and_errors():
    job = _job(ile.ILE_FP64, seed=112)
    try:
        lw = torch.full((100,), float("-inf"), dtype=torch.float64, device="cuda")
        th = torch.zeros((7, 100), dtype=torch.float64, device="cuda")
        idx = torch.zeros(50, dtype=torch.int64, device="cuda")
        out = torch.zeros((7, 50), dtype=torch.float64, device="cuda")
        ile.ile_fair_draw(job, 100, lw, 1, 0, 50, idx, th, 100, out, 50)
        torch.cuda.synchronize()
        assert np.all(idx.cpu().numpy() == -1) and torch.isnan(out).all().item()
        with pytest.raises(ile.IleError):
            ile.ile_fair_draw(job, 0, lw, 1, 0, 5, idx)
        with pytest.raises(ile.IleError):
            ile.ile_fair_draw(job, 100, lw, 1, 0, 5, None, th, 100, out, 4)
    finally:
        ile.ile_job_release(job)


def test_fair_draws_reproduce_the_weighted_run():
    """Before/after resampling: prior draws of an SNR-10 HL event weighted by
    the FP64 likelihood, then 20,000 fair draws; the draw counts of the
    samples follow their weights (chi-square over the samples with expected
    count >= 5, the rest pooled), and each column's mean over the draws
    agrees with the weighted mean within 5 standard errors."""
    from scipy import stats
    rec = chirpgen.load_injections()["pool"][7]
    probs, _ = chirpgen.build_event(rec, ["H", "L"], 5, 25.0, 1.5, 10.0, noise_seed=77)
    job = ile.ile_prepare(gu.ctx(), ile.ProblemHost(probs[0], precision=ile.ILE_FP64))
    n, k = 1 << 21, 20000
    try:
        th = torch.empty((7, n), dtype=torch.float64, device="cuda")
        lr = torch.empty((n,), dtype=torch.float64, device="cuda")
        L = torch.empty((n,), dtype=torch.float64, device="cuda")
        W = torch.empty((n,), dtype=torch.float64, device="cuda")
        ile.ile_draw(job, 31, 0, 0, n, th, n, lr)
        ile.ile_eval_lnL(job, n, th, n, lr, L, W)
        m = ile.ile_marginalize(job, n, W)
        idx = torch.empty(k, dtype=torch.int64, device="cuda")
        out = torch.empty((7, k), dtype=torch.float64, device="cuda")
        ile.ile_fair_draw(job, n, W, 32, 0, k, idx, th, n, out, k)
        torch.cuda.synchronize()
        w = W.cpu().numpy()
        x = th.cpu().numpy()
        d = out.cpu().numpy()
        ix = idx.cpu().numpy()
    finally:
        ile.ile_job_release(job)
    print("n_eff", m["n_eff"])
    w = np.exp(w - w.max())
    p = w / w.sum()
    big = np.nonzero(p * k >= 5)[0]
    cnt = np.array([np.count_nonzero(ix == i) for i in big] + [np.count_nonzero(~np.isin(ix, big))])
    exp_ = np.concatenate([p[big] * k, [k * (1 - p[big].sum())]])
    keep = exp_ > 0
    assert stats.chisquare(cnt[keep], exp_[keep] / exp_[keep].sum() * cnt[keep].sum()).pvalue > 1e-4
    assert np.array_equal(d, x[:, ix])
    for c in range(7):
        mu = float(np.sum(p * x[c]))
        sd = float(np.sqrt(np.sum(p * (x[c] - mu) ** 2)))
        assert abs(d[c].mean() - mu) <= 5 * sd / np.sqrt(k) + 1e-12, c
