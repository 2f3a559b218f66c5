"""Parity at full size, in the launch configuration the benchmark times: 256
intrinsic points (H, L, V; 9 modes; M_c uniform 20-40, q 1-4; SNR 20) with
2^20 extrinsic samples each, drawn by the counter-based prior generator into
one array and evaluated by one batched launch per kernel (the LDS-staged lnL
kernel at this size).  The oracle recomputes sampled outputs one by one: the
draws at sampled indices, lnL of sampled draws of every point (each block
boundary of the kernels' tiles included), and the estimator of each point on
seeded log-weights of the full length, and the marginal ln L of the GPU's
own 2^20 draws of four points against the oracle on those draws."""
import numpy as np
import pytest

import chirpgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2505_11655_amd as ile  # noqa: E402
from tests import gpu_util as gu  # noqa: E402

N_POINTS = 256
N_PER = 1 << 20
PNAME = {0: "fp64", 1: "fp32", 2: "fp32c64"}


@pytest.fixture(scope="module")
def problems():
    recs = chirpgen.load_injections()
    rng = np.random.default_rng(2505)
    templates = [(float(rng.uniform(20, 40)), float(rng.uniform(1, 4))) for _ in range(N_POINTS)]
    probs, _ = chirpgen.build_event(recs["c2"], ["H", "L", "V"], 9, 30.0, 2.0, 20.0,
                                    noise_seed=chirpgen.BASE_SEED + 2, templates=templates)
    return probs


def _sample_index(rng, n_per):
    """Sampled positions within one point: both ends, every 65536-sample tile
    boundary, and random positions."""
    edges = np.arange(0, n_per, 65536)
    idx = np.concatenate([[0, n_per - 1], edges, edges - 1, rng.integers(0, n_per, 24)])
    return np.unique(idx[(idx >= 0) & (idx < n_per)])


@pytest.mark.parametrize("policy", [ile.ILE_FP32, ile.ILE_FP64, ile.ILE_FP32_CANCEL64], ids=["fp32", "fp64", "fp32c64"])
def test_fullsize_draw_and_lnL(orc, problems, policy):
    dt = gu.torch_dtype(policy)
    jobs = [ile.ile_prepare(gu.ctx(), ile.ProblemHost(p, precision=policy)) for p in problems]
    J, N = len(jobs), len(jobs) * N_PER
    seed, rnd = 0x5EED0000 + policy, 0
    try:
        th = torch.empty((7, N), dtype=dt, device="cuda")
        lr = torch.empty((N,), dtype=dt, device="cuda")
        L = torch.full((N,), float("nan"), dtype=gu.out_dtype(policy), device="cuda")
        W = torch.full((N,), float("nan"), dtype=gu.out_dtype(policy), device="cuda")
        esz, osz = th.element_size(), L.element_size()
        ile.ile_draw(jobs[0], seed, rnd, 0, N, th, N, lr)
        ile.ile_eval_lnL_batch(jobs, [N_PER] * J, [th.data_ptr() + j * N_PER * esz for j in range(J)], [N] * J,
                               [lr.data_ptr() + j * N_PER * esz for j in range(J)],
                               [L.data_ptr() + j * N_PER * osz for j in range(J)],
                               [W.data_ptr() + j * N_PER * osz for j in range(J)])
        torch.cuda.synchronize()
        rng = np.random.default_rng(26)
        worst_s, worst_a = 0.0, 0.0
        prior = orc.make_prior(t_window=problems[0].t_window, d_min=problems[0].d_min, d_max=problems[0].d_max)
        for j in range(J):
            loc = _sample_index(rng, N_PER)
            gidx = torch.from_numpy(j * N_PER + loc).to("cuda")
            g_th = th[:, gidx].double().cpu().numpy()
            g_L = L[gidx].double().cpu().numpy()
            g_W = W[gidx].double().cpu().numpy()
            g_lr = lr[gidx].double().cpu().numpy()
            # the draws at these global indices, one by one
            o_th = np.concatenate([orc.draw_prior(prior, seed, rnd, int(j * N_PER + i), 1)[0] for i in loc], axis=1)
            if policy == ile.ILE_FP64:
                assert np.allclose(g_th, o_th, rtol=1e-14, atol=1e-15)
            else:
                assert np.allclose(g_th, o_th.astype(np.float32).astype(np.float64), rtol=2e-7, atol=1e-12)
            assert np.all(g_lr == 0.0)
            # lnL of those draws (as the kernel read them) against the oracle
            ref, T1, T2 = orc.lnL(problems[j], g_th, return_terms=True)
            ok, ms, ma = gu.tol_check(g_L, ref, T1, T2, 100.0 / g_th[3], policy)
            assert ok, (j, ms, ma)
            fin = np.isfinite(g_L)
            assert np.array_equal(g_W[fin], g_L[fin])
            worst_s, worst_a = max(worst_s, ms), max(worst_a, ma)
        assert not torch.isnan(L).any().item()
        print(f"{PNAME[policy]} {J} x {N_PER}: max|d| scoped={worst_s:.3e} all={worst_a:.3e}")
        # the marginal ln L of four points from the GPU's own draws, the whole
        # 2^20 of each, against the oracle on the same draws: the two loudest
        # points and two seeded ones
        res = ile.ile_marginalize_batch(jobs, [N_PER] * J, [W.data_ptr() + j * N_PER * osz for j in range(J)],
                                        ile.ILE_MARG_RESET, want=True)
        torch.cuda.synchronize()
        loud = np.argsort([-r["ln_L"] for r in res])[:2]
        pick = list(dict.fromkeys([int(loud[0]), int(loud[1])] + [int(v) for v in rng.choice(J, 4, replace=False)]))[:4]
        tol = 1e-10 if policy == ile.ILE_FP64 else 1e-4
        worst = 0.0
        for j in pick:
            thj = th[:, j * N_PER:(j + 1) * N_PER].double().cpu().numpy()
            o = orc.marginalize(orc.lnL(problems[j], thj))
            d = abs(res[j]["ln_L"] - o["ln_L"])
            print(f"{PNAME[policy]} point {j}: ln L gpu {res[j]['ln_L']:.9f} oracle {o['ln_L']:.9f} "
                  f"n_eff {o['n_eff']:.1f} |d| {d:.2e}")
            assert d <= tol, (j, d)
            worst = max(worst, d)
        print(f"{PNAME[policy]} marginal of the draws, 4 points: max|d ln L| = {worst:.2e}")
    finally:
        for jb in jobs:
            ile.ile_job_release(jb)


@pytest.mark.parametrize("policy", [ile.ILE_FP32, ile.ILE_FP64], ids=["fp32", "fp64"])
def test_fullsize_marginalize(orc, problems, policy):
    """The batched estimator over 256 points of 2^20 seeded log-weights each
    (spread as a weighted sample's are, a few points with non-finite entries),
    per point against the oracle.  Both accumulate in FP64, so the bound is
    summation-order rounding over 2^20 terms."""
    jobs = [ile.ile_prepare(gu.ctx(), ile.ProblemHost(p, precision=policy)) for p in problems[:N_POINTS]]
    J = len(jobs)
    rng = np.random.default_rng(27)
    try:
        npdt = np.float32 if policy == ile.ILE_FP32 else np.float64
        lw = np.empty((J, N_PER), dtype=npdt)
        for j in range(J):
            lw[j] = (rng.normal(-40.0, 6.0, N_PER) + rng.uniform(0, 30)).astype(npdt)
        lw[3, 17] = -np.inf
        lw[5, 1000:1010] = np.nan
        Wt = torch.from_numpy(lw.reshape(-1)).to("cuda")
        esz = Wt.element_size()
        res = ile.ile_marginalize_batch(jobs, [N_PER] * J, [Wt.data_ptr() + j * N_PER * esz for j in range(J)],
                                        ile.ILE_MARG_RESET, want=True)
        torch.cuda.synchronize()
        for j in range(J):
            o = orc.marginalize(lw[j].astype(np.float64))
            r = res[j]
            assert r["n"] == o["n"] and r["n_nonfinite"] == o["n_nonfinite"] and r["argmax"] == o["argmax"]
            assert abs(r["ln_L"] - o["ln_L"]) <= 1e-12 * max(1, abs(o["ln_L"])), (j, r["ln_L"], o["ln_L"])
            assert abs(r["n_eff"] - o["n_eff"]) <= 1e-10 * o["n_eff"], (j, r["n_eff"], o["n_eff"])
    finally:
        for jb in jobs:
            ile.ile_job_release(jb)
