"""The product-form adaptive Cartesian sampler on the GPU against the oracle:
draws (theta and ln p - ln p_s) from adapted marginals, and each update's
marginals to 1e-12 (integer histograms of the fixed-point masses on both
sides; a mass can differ by one unit where the two sides' exp round
differently), for every column and for a chosen subset; a served AC job
equals the oracle's loop of draws, likelihood and updates."""
import numpy as np
import pytest

import chirpgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2505_11655_amd as ile  # noqa: E402
from tests import gpu_util as gu  # noqa: E402


def _lw_of(th, rng_seed, dtype):
    """Seeded synthetic log-weights of the drawn parameters (generator side)."""
    rng = np.random.default_rng(rng_seed)
    a, b = rng.uniform(1, 5), rng.uniform(-0.5, 0.5)
    lw = -0.5 * ((th[0] - a) / 0.3) ** 2 - 0.5 * ((th[4] - b) / 0.2) ** 2 - 0.5 * ((th[6] - 1.0) / 0.5) ** 2
    lw[rng.choice(th.shape[1], th.shape[1] // 40, replace=False)] = -np.inf
    return lw.astype(dtype)


@pytest.mark.parametrize("policy", [ile.ILE_FP64, ile.ILE_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("dims", [None, [0, 4, 6]], ids=["all", "subset"])
def test_ac_draws_and_updates_match_oracle(orc, policy, dims):
    rng = np.random.default_rng(120)
    p = chirpgen.random_problem(rng, 5, ["H", "L"])
    job = ile.ile_prepare(gu.ctx(), ile.ProblemHost(p, precision=policy))
    pr = orc.make_prior(t_window=p.t_window, d_min=p.d_min, d_max=p.d_max)
    st = orc.ac_init(dims=dims)
    dt = gu.torch_dtype(policy)
    odt = np.float32 if policy == ile.ILE_FP32 else np.float64
    n, seed = 30011, 0xACAC
    try:
        ile.ile_ac_reset(job, dims=dims)
        for rnd in range(4):
            th = torch.empty((7, n), dtype=dt, device="cuda")
            lr = torch.empty((n,), dtype=dt, device="cuda")
            ile.ile_ac_draw(job, seed, rnd, 3, n, th, n, lr)
            torch.cuda.synchronize()
            th_o, lr_o, bins = orc.draw_ac(pr, st, seed, rnd, 3, n)
            g = th.double().cpu().numpy()
            if policy == ile.ILE_FP64:
                # after an update the marginals agree to rounding; the inverse
                # CDFs of the prior (asin near the poles) magnify that slightly
                close = np.isclose(g, th_o, rtol=1e-14, atol=1e-15)
                assert close.mean() > 0.99, close.mean()
                assert np.allclose(g, th_o, rtol=1e-9, atol=1e-9), np.abs(g - th_o).max()
                assert np.allclose(lr.cpu().numpy(), lr_o, rtol=1e-12, atol=1e-12)
            else:
                assert np.allclose(g, th_o.astype(np.float32).astype(np.float64), rtol=2e-7, atol=1e-12)
                assert np.allclose(lr.double().cpu().numpy(), lr_o, rtol=2e-7, atol=1e-6)
            lw = _lw_of(th_o, 121 + rnd, odt)
            ile.ile_ac_update(job, seed, rnd, 3, n, torch.from_numpy(lw).to("cuda"), 0.1)
            st = orc.ac_update(st, bins, lw.astype(np.float64), floor=0.1)
            gdims, gpi = ile.ile_ac_get(job)
            assert gdims == st.dims
            # each side forms the fixed-point masses with its own exp: a mass can
            # differ by one unit, so the marginals agree to rounding, not bitwise
            assert np.allclose(gpi, st.pi, rtol=1e-12, atol=0.0), np.abs(gpi - st.pi).max()
        assert st.pi.max() > 0.1          # the marginals did adapt
    finally:
        ile.ile_job_release(job)


def test_ac_rejects_bad_arguments():
    rng = np.random.default_rng(122)
    p = chirpgen.random_problem(rng, 5, ["H", "L"])
    job = ile.ile_prepare(gu.ctx(), ile.ProblemHost(p, precision=ile.ILE_FP32, dist_marg=True))
    try:
        for dims in ([3], [5, 2], [7]):
            with pytest.raises(ile.IleError):
                ile.ile_ac_reset(job, dims=dims)
        lw = torch.zeros(10, dtype=torch.float32, device="cuda")
        with pytest.raises(ile.IleError):
            ile.ile_ac_update(job, 1, 0, 0, 10, lw, 1.5)
        dims, pi = ile.ile_ac_get(job)
        assert dims == [0, 1, 2, 4, 5, 6] and np.allclose(pi, 1.0 / 64)
    finally:
        ile.ile_job_release(job)


def test_ac_job_matches_oracle_loop(orc):
    """A served AC job (FP64, 6 rounds of 2^14): the same pooled estimate as
    the oracle's loop to 1e-9."""
    recs = chirpgen.load_injections()
    probs, _ = chirpgen.build_event(recs["c1"], ["H", "L"], 5, 30.0, 2.0, 20.0, noise_seed=41)
    p = probs[0]
    ph = ile.ProblemHost(p, precision=ile.ILE_FP64)
    n, seed, max_rounds, target = 1 << 14, 909, 6, 1e9
    jo = ile.job_opts(adaptive=True, round_samples=n, max_rounds=max_rounds, n_eff_target=target, seed=seed,
                      integrator=ile.ILE_INT_AC)
    srv = ile.ile_server_create(gu.ctx())
    try:
        r = ile.ile_server_wait(srv, ile.ile_server_submit(srv, ph, jo), 120000)
    finally:
        ile.ile_server_destroy(srv)
    assert r.status == 0 and r.rounds == max_rounds
    pr = orc.make_prior(t_window=p.t_window, d_min=p.d_min, d_max=p.d_max)
    st = orc.ac_init()
    lws = []
    for rnd in range(max_rounds):
        th, lr, bins = orc.draw_ac(pr, st, seed, rnd, 0, n)
        lw = orc.lnL(p, th) + lr
        lws.append(lw)
        st = orc.ac_update(st, bins, lw)
    o = orc.marginalize(np.concatenate(lws))
    print("AC job", r.marg.ln_L, r.marg.n_eff, "oracle", o["ln_L"], o["n_eff"])
    assert abs(r.marg.ln_L - o["ln_L"]) <= 1e-9 * max(1.0, abs(o["ln_L"]))
    assert abs(r.marg.n_eff - o["n_eff"]) <= 1e-8 * o["n_eff"]
