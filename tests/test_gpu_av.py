"""The adaptive-volume integrator on the GPU against the oracle: draws from a
grid, the threshold / refinement / cell list of each update (bit-exact:
integer keys and fixed-point masses on both sides), edge cases of the
threshold, a grid over a subset of columns, buffer growth, and whole rounds of
draw -> likelihood -> update on an ILE problem in FP64.  The log-weights fed
to both sides come from the seeded generator or from each side's own
likelihood, never from the GPU into the oracle."""
import math

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


def _job(policy, seed=90, dist_marg=False, n_modes=5, dets=("H", "L")):
    rng = np.random.default_rng(seed)
    p = chirpgen.random_problem(rng, n_modes, list(dets))
    return p, ile.ile_prepare(gu.ctx(), ile.ProblemHost(p, precision=policy, dist_marg=dist_marg))


def _gpu_draw(job, policy, seed, rnd, first, n):
    dt = gu.torch_dtype(policy)
    th = torch.empty((7, n), dtype=dt, device="cuda")
    lr = torch.full((n,), 99.0, dtype=dt, device="cuda")
    ile.ile_av_draw(job, seed, rnd, first, n, th, n, lr)
    torch.cuda.synchronize()
    return th.double().cpu().numpy(), lr.double().cpu().numpy()


def _synthetic_lw(rng, u, kind, dtype):
    """Seeded log-weights of the unit-cube coordinates (generator side)."""
    d, n = u.shape
    mu = rng.uniform(0.3, 0.7, d)
    if kind == "gauss":
        lw = -0.5 * np.sum(((u.T - mu) / 0.12) ** 2, axis=1)
    elif kind == "ties":
        lw = np.round(-np.sum(((u.T - mu) / 0.2) ** 2, axis=1), 0)
    else:
        lw = rng.normal(0, 3, n)
    lw[rng.choice(n, n // 50, replace=False)] = -np.inf
    return lw.astype(dtype)


def _compare_grid(job, g, info=None, st=None, thr_rtol=0.0):
    """thr_rtol = 0: both sides thresholded the same log-weights, so the
    threshold is the same sample value; otherwise each side used its own
    likelihood and the values differ by that likelihood's rounding."""
    st_g, cells = ile.ile_av_get(job)
    assert st_g["n_bins"] == g.nb and st_g["n_cells"] == g.n_cells, (st_g, g.nb, g.n_cells)
    assert np.array_equal(cells, g.cells)
    assert abs(st_g["ln_vol"] - g.ln_vol) <= 1e-12 * max(1.0, abs(g.ln_vol))
    if info is not None:
        assert abs(st["lnL_thr"] - info["lnL_thr"]) <= thr_rtol * max(1.0, abs(info["lnL_thr"]))
        assert st["n_min"] == info["n_min"]
        assert st["n_live"] == info["n_live"]
        assert abs(st["vol_mc"] - info["vol_mc"]) <= 1e-12 * info["vol_mc"]


@pytest.mark.parametrize("policy", [ile.ILE_FP64, ile.ILE_FP32], ids=["fp64", "fp32"])
def test_av_draws_and_updates_match_oracle(orc, policy):
    """Three rounds on a ragged sample count: GPU draws equal the oracle's
    (FP64 to rounding, FP32 to the float of the FP64 value), ln p - ln p_s is
    ln V, and each update (on seeded log-weights of the oracle's own
    coordinates) gives the same threshold, n_min, bin count and cell list."""
    p, job = _job(policy)
    pr = orc.make_prior(t_window=p.t_window, d_min=p.d_min, d_max=p.d_max)
    g = orc.av_init()
    rng = np.random.default_rng(91)
    npdt = np.float32 if policy == ile.ILE_FP32 else np.float64
    seed, n = 0xC0FFEE, 20011
    opts = ile.av_opts(p_thr=0.99, n_min_live=400)
    try:
        ile.ile_av_reset(job)
        for rnd, kind in enumerate(["gauss", "ties", "noise"]):
            th_g, lr_g = _gpu_draw(job, policy, seed, rnd, 7, n)
            th_o, u_o = orc.draw_av(pr, g, seed, rnd, 7, n)
            if policy == ile.ILE_FP64:
                assert np.allclose(th_g, th_o, rtol=1e-14, atol=1e-15)
            else:
                assert np.allclose(th_g, th_o.astype(np.float32).astype(np.float64), rtol=2e-7, atol=1e-12)
            assert np.all(np.abs(lr_g - g.ln_vol) <= 1e-6 * max(1.0, abs(g.ln_vol)))
            lw = _synthetic_lw(rng, u_o, kind, npdt)
            st = ile.ile_av_update(job, seed, rnd, 7, n, torch.from_numpy(lw).to("cuda"), opts)
            g, info = orc.av_update(g, u_o, lw.astype(np.float64), p_thr=0.99, n_min_live=400)
            print(PNAME[policy], rnd, kind, st)
            _compare_grid(job, g, info, st)
    finally:
        ile.ile_job_release(job)


def test_av_threshold_edge_cases(orc):
    """No finite weight keeps the grid; a single finite sample; p_thr = 1 and
    n_min_live above n (every finite sample kept); NaN and +/-0 handled as the
    oracle does."""
    p, job = _job(ile.ILE_FP64, seed=92)
    g = orc.av_init()
    pr = orc.make_prior(t_window=p.t_window, d_min=p.d_min, d_max=p.d_max)
    try:
        n = 3001
        _, u = orc.draw_av(pr, g, 5, 0, 0, n)
        _gpu_draw(job, ile.ILE_FP64, 5, 0, 0, n)
        lw = np.full(n, -np.inf)
        st = ile.ile_av_update(job, 5, 0, 0, n, torch.from_numpy(lw).to("cuda"))
        assert st["n_bins"] == 1 and st["n_cells"] == 1 and st["n_min"] == 0 and st["lnL_thr"] == -np.inf
        lw[1234] = 3.5
        lw[17] = np.nan
        st = ile.ile_av_update(job, 5, 0, 0, n, torch.from_numpy(lw).to("cuda"), ile.av_opts(n_min_live=1))
        g1, info = orc.av_update(g, u, lw, n_min_live=1)
        _compare_grid(job, g1, info, st)
        assert st["n_min"] == 1 and st["n_cells"] == 1
        ile.ile_av_reset(job)
        rng = np.random.default_rng(93)
        lw = rng.normal(0, 1, n)
        lw[:10] = 0.0
        lw[10:20] = -0.0
        st = ile.ile_av_update(job, 5, 0, 0, n, torch.from_numpy(lw).to("cuda"),
                               ile.av_opts(p_thr=1.0, n_min_live=10 ** 6, max_bins=3))
        g2, info = orc.av_update(g, u, lw, p_thr=1.0, n_min_live=10 ** 6, max_bins=3)
        _compare_grid(job, g2, info, st)
        assert st["n_min"] == n and st["n_bins"] <= 3
        # total mass 2^54 + 3: p_thr * total rounds above the total in FP64
        ile.ile_av_reset(job)
        n = (1 << 14) + 3
        _, u = orc.draw_av(pr, g, 6, 0, 0, n)
        lw = np.zeros(n)
        lw[-3:] = -27.6
        st = ile.ile_av_update(job, 6, 0, 0, n, torch.from_numpy(lw).to("cuda"), ile.av_opts(p_thr=1.0, n_min_live=1))
        g3, info = orc.av_update(g, u, lw, p_thr=1.0, n_min_live=1)
        _compare_grid(job, g3, info, st)
        assert st["n_min"] == n
    finally:
        ile.ile_job_release(job)


def test_av_grid_over_two_columns(orc):
    """A grid over (alpha, dec) only (the other columns from the prior, the
    volume counted over the grid): the Rosenbrock rounds of the paper's
    demonstration, GPU and oracle, with the same grids."""
    p, job = _job(ile.ILE_FP64, seed=94)
    pr = orc.make_prior(t_window=p.t_window, d_min=p.d_min, d_max=p.d_max)
    g = orc.AvGrid(1, np.zeros((1, 2), dtype=np.int32), [0, 1])
    try:
        ile.ile_av_reset(job, dims=[0, 1])
        n = 20000
        for rnd in range(4):
            _gpu_draw(job, ile.ILE_FP64, 77, rnd, 0, n)
            _, u = orc.draw_av(pr, g, 77, rnd, 0, n)
            x, y = 4.0 * u[0] - 2.0, 4.0 * u[1] - 1.0
            lw = -((1.0 - x) ** 2 + 100.0 * (y - x * x) ** 2)
            st = ile.ile_av_update(job, 77, rnd, 0, n, torch.from_numpy(lw).to("cuda"))
            g, info = orc.av_update(g, u, lw)
            _compare_grid(job, g, info, st)
        assert g.nb > 10
    finally:
        ile.ile_job_release(job)


def test_av_rejects_bad_arguments():
    p, job = _job(ile.ILE_FP32, seed=95, dist_marg=True)
    try:
        for dims in ([3], [2, 1], [0, 7], [0, 0]):
            with pytest.raises(ile.IleError):
                ile.ile_av_reset(job, dims=dims)
        lw = torch.zeros(10, dtype=torch.float32, device="cuda")
        for o in (ile.av_opts(p_thr=1.5), ile.av_opts(n_min_live=-1), ile.av_opts(max_bins=600)):
            with pytest.raises(ile.IleError):
                ile.ile_av_update(job, 1, 0, 0, 10, lw, o)
        st, _ = ile.ile_av_get(job, cells=False)
        assert st["n_dim"] == 6 and st["dims"] == [0, 1, 2, 4, 5, 6]
    finally:
        ile.ile_job_release(job)


def test_av_buffer_growth_keeps_the_grid(orc):
    """An update larger than the buffers grows them; the grid built before
    carries over and later rounds still match the oracle."""
    p, job = _job(ile.ILE_FP64, seed=96)
    pr = orc.make_prior(t_window=p.t_window, d_min=p.d_min, d_max=p.d_max)
    g = orc.av_init()
    rng = np.random.default_rng(97)
    try:
        for rnd, n in enumerate([3000, 70001, 5000]):
            _gpu_draw(job, ile.ILE_FP64, 8, rnd, 0, n)
            _, u = orc.draw_av(pr, g, 8, rnd, 0, n)
            lw = _synthetic_lw(rng, u, "gauss", np.float64)
            st = ile.ile_av_update(job, 8, rnd, 0, n, torch.from_numpy(lw).to("cuda"), ile.av_opts(n_min_live=200))
            g, info = orc.av_update(g, u, lw, n_min_live=200)
            _compare_grid(job, g, info, st)
    finally:
        ile.ile_job_release(job)


def test_av_rounds_on_an_ile_problem_match_oracle(orc):
    """Rounds of AV draws, FP64 likelihood and updates on an SNR-20 HL event:
    the GPU loop (its own likelihood) and the oracle loop (the oracle's
    likelihood of its own draws) build the same grids, and the pooled
    estimates agree to 1e-9."""
    recs = chirpgen.load_injections()
    probs, _ = chirpgen.build_event(recs["c1"], ["H", "L"], 5, 30.0, 2.0, 20.0, noise_seed=31)
    p = probs[0]
    job = ile.ile_prepare(gu.ctx(), ile.ProblemHost(p, precision=ile.ILE_FP64))
    pr = orc.make_prior(t_window=p.t_window, d_min=p.d_min, d_max=p.d_max)
    g = orc.av_init()
    n, seed = 1 << 14, 4242
    lw_all = []
    th = torch.empty((7, n), dtype=torch.float64, device="cuda")
    lr = torch.empty((n,), dtype=torch.float64, device="cuda")
    L = torch.empty((n,), dtype=torch.float64, device="cuda")
    W = torch.empty((n,), dtype=torch.float64, device="cuda")
    try:
        ile.ile_av_reset(job)
        for rnd in range(5):
            ile.ile_av_draw(job, seed, rnd, 0, n, th, n, lr)
            ile.ile_eval_lnL(job, n, th, n, lr, L, W)
            res = ile.ile_marginalize(job, n, W, ile.ILE_MARG_RESET if rnd == 0 else ile.ILE_MARG_POOL)
            st = ile.ile_av_update(job, seed, rnd, 0, n, W)
            th_o, u_o = orc.draw_av(pr, g, seed, rnd, 0, n)
            lnL_o = orc.lnL(p, th_o)
            lw_o = lnL_o + g.ln_vol
            lw_all.append(lw_o)
            g, info = orc.av_update(g, u_o, lw_o)
            print(rnd, st, res["n_eff"])
            _compare_grid(job, g, info, st, thr_rtol=1e-12)
        o = orc.marginalize(np.concatenate(lw_all))
        assert abs(res["ln_L"] - o["ln_L"]) <= 1e-9 * max(1.0, abs(o["ln_L"]))
        assert abs(res["n_eff"] - o["n_eff"]) <= 1e-8 * o["n_eff"]
        assert g.ln_vol < -3.0
    finally:
        ile.ile_job_release(job)
