"""The continuous-batching server: every job's result is the same alone and in
a mix; plain jobs equal the oracle on the same (reproduced) draws; admission by
device footprint queues jobs under a small budget and rejects oversize ones;
cancellation; adaptive jobs stop at the n_eff target or the round cap."""
import math
import time

import numpy as np
import pytest

import chirpgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2505_11655_amd as ile  # noqa: E402
from tests import gpu_util as gu  # noqa: E402

FIELDS = ["ln_L", "ln_sigma", "n_eff", "n_ess", "max_lw", "argmax", "n", "n_nonfinite"]


@pytest.fixture(scope="module")
def pool():
    """A small pool of events of every (modes, detectors) class."""
    recs = chirpgen.load_injections()["pool"]
    out = []
    rng = np.random.default_rng(50)
    for i, (n, dets) in enumerate([(5, ["H", "L"]), (9, ["H", "L", "V"]), (17, ["H", "L", "V"]),
                                   (5, ["H", "L", "V"]), (9, ["H", "L"]), (17, ["L", "V"])]):
        snr = float(np.exp(rng.uniform(np.log(10), np.log(40))))
        probs, _ = chirpgen.build_event(recs[i], dets, n, float(rng.uniform(20, 40)), float(rng.uniform(1, 4)), snr,
                                        noise_seed=100 + i)
        out.append(probs[0])
    return out


def _specs(pool):
    rng = np.random.default_rng(51)
    specs = []
    for i in range(14):
        p = pool[i % len(pool)]
        policy = [ile.ILE_FP32, ile.ILE_FP64, ile.ILE_FP32_CANCEL64][i % 3]
        adaptive = i % 4 == 3
        tm = 4 if (i % 5 == 4 and not adaptive and policy != ile.ILE_FP32_CANCEL64) else 0
        n = int(2 ** rng.uniform(14, 17))
        specs.append((p, policy, adaptive, n, 1000 + i, tm))
    return specs


def _submit(srv, spec):
    p, policy, adaptive, n, seed, tm = spec
    ph = ile.ProblemHost(p, precision=policy)
    jo = ile.job_opts(n_samples=n, adaptive=adaptive, round_samples=1 << 14, max_rounds=6, n_eff_target=300.0,
                      seed=seed, tmarg_oversample=tm)
    return ile.ile_server_submit(srv, ph, jo), ph


def _res(r):
    return {f: getattr(r.marg, f) for f in FIELDS} | {"status": r.status, "rounds": r.rounds, "samples": r.samples}


def test_mixed_equals_alone(pool):
    specs = _specs(pool)
    srv = ile.ile_server_create(gu.ctx(), max_active=64, chunk_samples=1 << 15)
    try:
        ids = [_submit(srv, s)[0] for s in specs]
        mixed = [_res(ile.ile_server_wait(srv, i, 120000)) for i in ids]
    finally:
        ile.ile_server_destroy(srv)
    for k, s in enumerate(specs):
        solo = ile.ile_server_create(gu.ctx(), max_active=1, chunk_samples=1 << 15)
        try:
            jid, _ = _submit(solo, s)
            alone = _res(ile.ile_server_wait(solo, jid, 120000))
        finally:
            ile.ile_server_destroy(solo)
        assert mixed[k]["status"] == 0 and alone["status"] == 0
        for f in FIELDS + ["rounds", "samples"]:
            a, b = mixed[k][f], alone[f]
            assert a == b or (isinstance(a, float) and np.isnan(a) and np.isnan(b)), (k, f, a, b)


@pytest.mark.parametrize("policy", [ile.ILE_FP32, ile.ILE_FP64], ids=["fp32", "fp64"])
def test_mixed_equals_alone_lds_regime(pool, policy):
    """Ten 2^20-sample jobs of one class submitted together: a pass over them
    evaluates 10.5M samples of one compiled kernel, past the batched
    likelihood's LDS-staging threshold, while each job alone runs the
    unstaged kernel.  Each result equals the job's solo result to the bit."""
    specs = [(pool[1], policy, False, 1 << 20, 3000 + i, 0) for i in range(10)]
    srv = ile.ile_server_create(gu.ctx(), max_active=64, chunk_samples=1 << 20)
    try:
        ids = [_submit(srv, s)[0] for s in specs]
        mixed = [_res(ile.ile_server_wait(srv, i, 120000)) for i in ids]
    finally:
        ile.ile_server_destroy(srv)
    for k, s in enumerate(specs):
        solo = ile.ile_server_create(gu.ctx(), max_active=1, chunk_samples=1 << 20)
        try:
            jid, _ = _submit(solo, s)
            alone = _res(ile.ile_server_wait(solo, jid, 120000))
        finally:
            ile.ile_server_destroy(solo)
        assert mixed[k]["status"] == 0 and alone["status"] == 0
        for f in FIELDS + ["rounds", "samples"]:
            a, b = mixed[k][f], alone[f]
            assert a == b or (isinstance(a, float) and np.isnan(a) and np.isnan(b)), (k, f, a, b)


@pytest.mark.parametrize("policy,tol", [(ile.ILE_FP64, 1e-10), (ile.ILE_FP32_CANCEL64, 1e-4), (ile.ILE_FP32, 1e-4)])
def test_plain_job_matches_oracle(orc, pool, policy, tol):
    """The server's draws are reproduced by the oracle's generator (same key,
    round 0, indices 0..n-1); the served ln L equals the oracle estimator:
    1e-10 in FP64, 1e-4 in FP32 and with the FP64 cancellation terms (an
    SNR-39 source of the pool)."""
    p = pool[1]
    n, seed = 3 * (1 << 14) + 123, 777
    srv = ile.ile_server_create(gu.ctx(), chunk_samples=1 << 14)
    try:
        ph = ile.ProblemHost(p, precision=policy)
        jid = ile.ile_server_submit(srv, ph, ile.job_opts(n_samples=n, seed=seed))
        r = ile.ile_server_wait(srv, jid, 60000)
    finally:
        ile.ile_server_destroy(srv)
    th, _ = orc.draw_prior(orc.make_prior(), seed, 0, 0, n)
    if policy != ile.ILE_FP64:
        th = th.astype(np.float32).astype(np.float64)
    o = orc.marginalize(orc.lnL(p, th))
    assert r.status == 0 and r.marg.n == n
    assert abs(r.marg.ln_L - o["ln_L"]) <= tol, (r.marg.ln_L, o["ln_L"])


@pytest.mark.parametrize("policy,tol", [(ile.ILE_FP64, 1e-9), (ile.ILE_FP32, 2e-3)])
def test_tmarg_job_matches_oracle(orc, pool, policy, tol):
    """A time-marginalised job (R = 4): the served ln L equals the oracle
    estimator over the oracle's time-marginalised likelihood of the same
    draws (the t column of the draws is ignored on both sides)."""
    p = pool[0]
    n, seed = 2 * (1 << 12) + 77, 4242
    srv = ile.ile_server_create(gu.ctx(), chunk_samples=1 << 14)
    try:
        ph = ile.ProblemHost(p, precision=policy)
        jid = ile.ile_server_submit(srv, ph, ile.job_opts(n_samples=n, seed=seed, tmarg_oversample=4))
        r = ile.ile_server_wait(srv, jid, 60000)
    finally:
        ile.ile_server_destroy(srv)
    th, _ = orc.draw_prior(orc.make_prior(), seed, 0, 0, n)
    if policy != ile.ILE_FP64:
        th = th.astype(np.float32).astype(np.float64)
    o = orc.marginalize(orc.lnL_tmarg(p, th, oversample=4))
    assert r.status == 0 and r.marg.n == n
    assert abs(r.marg.ln_L - o["ln_L"]) <= tol, (r.marg.ln_L, o["ln_L"])


def test_tmarg_job_rejects(pool):
    p = pool[0]
    srv = ile.ile_server_create(gu.ctx())
    try:
        bad = [(ile.ProblemHost(p, precision=ile.ILE_FP32), ile.job_opts(n_samples=100, tmarg_oversample=2)),
               (ile.ProblemHost(p, precision=ile.ILE_FP32), ile.job_opts(adaptive=True, tmarg_oversample=4)),
               (ile.ProblemHost(p, precision=ile.ILE_FP32_CANCEL64), ile.job_opts(n_samples=100, tmarg_oversample=4))]
        for ph, jo in bad:
            with pytest.raises(ile.IleError) as e:
                ile.ile_server_submit(srv, ph, jo)
            assert e.value.status == -1
    finally:
        ile.ile_server_destroy(srv)


def test_budget_queueing_and_admission(pool):
    p = pool[0]
    ph = ile.ProblemHost(p, precision=ile.ILE_FP32)
    tiny = ile.ile_server_create(gu.ctx(), hbm_budget_bytes=256 << 10, chunk_samples=1 << 15)
    try:
        with pytest.raises(ile.IleError) as e:
            ile.ile_server_submit(tiny, ph, ile.job_opts(n_samples=1 << 16, seed=1))
        assert e.value.status == -3
    finally:
        ile.ile_server_destroy(tiny)
    srv = ile.ile_server_create(gu.ctx(), max_active=64, hbm_budget_bytes=3 << 20, chunk_samples=1 << 15)
    try:
        ids =[ile.ile_server_submit(srv, ph, ile.job_opts(n_samples=1 << 16, seed=10 + i)) for i in range(8)]
        seen_queue = 0
        for _ in range(200):
            a, q, d = ile.ile_server_stats(srv)
            seen_queue = max(seen_queue, q)
            if d >= 8:
                break
            time.sleep(0.005)
        res = [ile.ile_server_wait(srv, i, 60000) for i in ids]
    finally:
        ile.ile_server_destroy(srv)
    assert all(r.status == 0 for r in res)
    assert seen_queue > 0
    admits = [r.t_admit_ns for r in res]
    assert admits == sorted(admits)           # arrival order under memory pressure


def test_cancel(pool):
    p = pool[2]
    ph = ile.ProblemHost(p, precision=ile.ILE_FP64)
    srv = ile.ile_server_create(gu.ctx(), max_active=4, chunk_samples=1 << 14)
    try:
        big = ile.ile_server_submit(srv, ph, ile.job_opts(n_samples=1 << 26, seed=3))
        small = ile.ile_server_submit(srv, ph, ile.job_opts(n_samples=1 << 14, seed=4))
        time.sleep(0.05)
        ile.ile_server_cancel(srv, big)
        rb = ile.ile_server_wait(srv, big, 60000)
        rs = ile.ile_server_wait(srv, small, 60000)
    finally:
        ile.ile_server_destroy(srv)
    assert rb.status == -6 and rb.samples < (1 << 26)
    assert rs.status == 0


def test_cancel_admitted_during_pass(pool):
    """Jobs admitted while a long job's passes run (inputs uploaded beside the
    pass) and then cancelled before their first pass: their buffers go back
    to the pool only after those uploads, so the jobs that run on, and a later
    server on the same context, equal their solo results to the bit."""
    specs = [(pool[k % len(pool)], ile.ILE_FP32, False, 1 << 14, 4000 + k, 0) for k in range(12)]
    long_spec = (pool[2], ile.ILE_FP64, False, 1 << 22, 4100, 0)
    srv = ile.ile_server_create(gu.ctx(), max_active=2, chunk_samples=1 << 14)
    try:
        lid, _ = _submit(srv, long_spec)
        ids = [_submit(srv, s)[0] for s in specs]
        for i in ids[1::2]:
            ile.ile_server_cancel(srv, i)
        res = [ile.ile_server_wait(srv, i, 120000) for i in ids]
        ile.ile_server_cancel(srv, lid)
        ile.ile_server_wait(srv, lid, 120000)
    finally:
        ile.ile_server_destroy(srv)
    # a server destroyed with admitted jobs still waiting for their first pass
    srv = ile.ile_server_create(gu.ctx(), max_active=2, chunk_samples=1 << 14)
    try:
        _submit(srv, long_spec)
        for s in specs:
            _submit(srv, s)
        time.sleep(0.02)
    finally:
        ile.ile_server_destroy(srv)
    for k, s in enumerate(specs):
        if k % 2 == 1:
            assert res[k].status in (0, -6)
            continue
        solo = ile.ile_server_create(gu.ctx(), max_active=1, chunk_samples=1 << 14)
        try:
            jid, _ = _submit(solo, s)
            alone = _res(ile.ile_server_wait(solo, jid, 120000))
        finally:
            ile.ile_server_destroy(solo)
        got = _res(res[k])
        assert got["status"] == 0 and alone["status"] == 0
        for f in FIELDS + ["rounds", "samples"]:
            a, b = got[f], alone[f]
            assert a == b or (isinstance(a, float) and np.isnan(a) and np.isnan(b)), (k, f, a, b)


def test_adaptive_job():
    """Adaptive rounds: stops at n_eff >= target or at the round cap; the
    estimate agrees with a long plain prior run within the combined errors.
    The source is quiet (SNR 10) so that the plain run is a valid reference
    (its own relative error is checked first); a loud source's posterior is
    too small a fraction of the prior for 2^24 prior draws."""
    rec = chirpgen.load_injections()["pool"][7]
    probs, _ = chirpgen.build_event(rec, ["H", "L"], 5, 25.0, 1.5, 10.0, noise_seed=77)
    p = probs[0]
    ph = ile.ProblemHost(p, precision=ile.ILE_FP32)
    srv = ile.ile_server_create(gu.ctx())
    try:
        ja = ile.ile_server_submit(srv, ph, ile.job_opts(adaptive=True, round_samples=1 << 16, max_rounds=32,
                                                         n_eff_target=1000.0, seed=5))
        jp = ile.ile_server_submit(srv, ph, ile.job_opts(n_samples=1 << 24, seed=6))
        ra = ile.ile_server_wait(srv, ja, 120000)
        rp = ile.ile_server_wait(srv, jp, 120000)
    finally:
        ile.ile_server_destroy(srv)
    assert ra.status == 0 and rp.status == 0
    assert ra.rounds <= 32 and (ra.marg.n_eff >= 1000.0 or ra.rounds == 32)
    sa = np.exp(ra.marg.ln_sigma - ra.marg.ln_L)
    sp = np.exp(rp.marg.ln_sigma - rp.marg.ln_L)
    print("adaptive", ra.rounds, ra.marg.n_eff, ra.marg.ln_L, "+-", sa, "plain", rp.marg.ln_L, "+-", sp,
          "plain n_eff", rp.marg.n_eff)
    assert sp < 0.2, "reference run not converged"
    assert abs(ra.marg.ln_L - rp.marg.ln_L) < 5 * np.hypot(sa, sp) + 0.05


def test_av_job_matches_oracle_loop(orc, pool):
    """An adaptive-volume job (FP64) runs the same rounds as an oracle loop of
    AV draws, oracle likelihood and AV updates with the server's options
    (p_thr 0.999, 1000 highest samples, 511 bins): same round count, pooled
    estimate to 1e-9; alone and in a mix of other jobs it gives bitwise the
    same result."""
    p = pool[0]
    ph = ile.ProblemHost(p, precision=ile.ILE_FP64)
    n, seed, max_rounds, target = 1 << 14, 606, 6, 2000.0
    jo = ile.job_opts(adaptive=True, round_samples=n, max_rounds=max_rounds, n_eff_target=target, seed=seed,
                      integrator=ile.ILE_INT_AV)
    srv = ile.ile_server_create(gu.ctx())
    try:
        alone = ile.ile_server_wait(srv, ile.ile_server_submit(srv, ph, jo), 120000)
        others = [_submit(srv, s) for s in _specs(pool)[:6]]
        jid = ile.ile_server_submit(srv, ph, jo)
        mixed = ile.ile_server_wait(srv, jid, 120000)
        for j, _ in others:
            ile.ile_server_wait(srv, j, 120000)
    finally:
        ile.ile_server_destroy(srv)
    assert alone.status == 0 and mixed.status == 0
    assert _res(alone) == _res(mixed)
    pr = orc.make_prior(t_window=p.t_window, d_min=p.d_min, d_max=p.d_max)
    g = orc.av_init()
    lws = []
    for rnd in range(max_rounds):
        th, u = orc.draw_av(pr, g, seed, rnd, 0, n)
        lw = orc.lnL(p, th) + g.ln_vol
        lws.append(lw)
        o = orc.marginalize(np.concatenate(lws))
        if o["n_eff"] >= target or rnd + 1 == max_rounds:
            break
        g, _ = orc.av_update(g, u, lw)
    print("AV job", alone.rounds, alone.marg.ln_L, alone.marg.n_eff, "oracle", len(lws), o["ln_L"], o["n_eff"])
    assert alone.rounds == len(lws)
    assert abs(alone.marg.ln_L - o["ln_L"]) <= 1e-9 * max(1.0, abs(o["ln_L"]))
    assert abs(alone.marg.n_eff - o["n_eff"]) <= 1e-8 * o["n_eff"]


def test_mixture_job_matches_oracle_loop(orc, pool):
    """An adaptive mixture job (FP64) runs the same rounds as an oracle loop
    with the server's options: prior draws in round 0; after each round a
    warm-started EM refit of 8 components (8 iterations, tempered to an
    effective sample size of 1/16 of the round) on that round's samples, the
    in-support masses from the server's mass key, and the next round drawn
    from the refitted mixture (defensive weight 0.05).  Same round count,
    pooled estimate to 1e-8; alone and in a mix of other jobs it gives
    bitwise the same result."""
    p = pool[3]
    ph = ile.ProblemHost(p, precision=ile.ILE_FP64)
    n, seed, max_rounds, target = 1 << 14, 707, 4, 1e9
    jo = ile.job_opts(adaptive=True, round_samples=n, max_rounds=max_rounds, n_eff_target=target, seed=seed)
    srv = ile.ile_server_create(gu.ctx())
    try:
        alone = ile.ile_server_wait(srv, ile.ile_server_submit(srv, ph, jo), 120000)
        others = [_submit(srv, s) for s in _specs(pool)[:6]]
        jid = ile.ile_server_submit(srv, ph, jo)
        mixed = ile.ile_server_wait(srv, jid, 120000)
        for j, _ in others:
            ile.ile_server_wait(srv, j, 120000)
    finally:
        ile.ile_server_destroy(srv)
    assert alone.status == 0 and mixed.status == 0
    assert _res(alone) == _res(mixed)
    pr = orc.make_prior(t_window=p.t_window, d_min=p.d_min, d_max=p.d_max)
    dims = list(range(7))
    zseed, m = seed ^ 0x9E3779B97F4A7C15, 1 << 16
    g, state, lws = None, None, []
    for rnd in range(max_rounds):
        if g is None:
            th, lr = orc.draw_prior(pr, seed, rnd, 0, n)
            lr = np.zeros(n)
        else:
            th, lr = orc.draw_gmm(pr, g, seed, rnd, 0, n)
        lw = orc.lnL(p, th) + lr
        lws.append(lw)
        o = orc.marginalize(np.concatenate(lws))
        print(f"oracle round {rnd}: n_eff {o['n_eff']:.2f} ln L {o['ln_L']:.9f}")
        if o["n_eff"] >= target or rnd + 1 == max_rounds:
            break
        state = orc.em_fit(th, lw, dims, state=state, n_iter=8, n_comp=8, temper_ess=1.0 / 16.0)
        w, mu, cov = state
        g0 = orc.make_gmm(w, mu, cov, dims)
        lz = [math.log(max(orc.gmm_inbox_mass(pr, g0, j, zseed, rnd + 1, m), 0.5 / m)) for j in range(len(w))]
        g = orc.make_gmm(w, mu, cov, dims, ln_Z=lz, eps_def=0.05)
    print("mixture job", alone.rounds, alone.marg.ln_L, alone.marg.n_eff, "oracle", len(lws), o["ln_L"], o["n_eff"])
    assert alone.rounds == len(lws)
    assert abs(alone.marg.ln_L - o["ln_L"]) <= 1e-8 * max(1.0, abs(o["ln_L"]))
    assert abs(alone.marg.n_eff - o["n_eff"]) <= 1e-6 * o["n_eff"]


def test_pooled_sheared_mixture_job_matches_oracle_loop(orc, pool):
    """An adaptive mixture job with the mixture pool (every sample weighted by
    the equal-weight mixture of all rounds' proposals, the prior included) and
    the phase shear (first fit: sign from the best sample's inclination), FP64:
    the same rounds as an oracle loop -- draws from the last refit, lnL,
    pooled weights from ``pool_mixture_lw``, estimator over the whole pool,
    refit on the round's own weights in the sheared phases.  Same round
    count, estimate to 1e-8; alone and in a mix it is bitwise the same."""
    p = pool[3]
    ph = ile.ProblemHost(p, precision=ile.ILE_FP64)
    n, seed, max_rounds, target = 1 << 13, 909, 4, 1e9
    jo = ile.job_opts(adaptive=True, round_samples=n, max_rounds=max_rounds, n_eff_target=target, seed=seed,
                      pool=ile.ILE_POOL_MIXTURE, phase_shear=1)
    # a second pooled job with a ragged round size, in the same passes
    ph2 = ile.ProblemHost(pool[1], precision=ile.ILE_FP64)
    jo2 = ile.job_opts(adaptive=True, round_samples=3001, max_rounds=5, n_eff_target=target, seed=77,
                       pool=ile.ILE_POOL_MIXTURE, phase_shear=1)
    srv = ile.ile_server_create(gu.ctx())
    try:
        alone = ile.ile_server_wait(srv, ile.ile_server_submit(srv, ph, jo), 120000)
        alone2 = ile.ile_server_wait(srv, ile.ile_server_submit(srv, ph2, jo2), 120000)
        others = [_submit(srv, s) for s in _specs(pool)[:6]]
        jid = ile.ile_server_submit(srv, ph, jo)
        jid2 = ile.ile_server_submit(srv, ph2, jo2)
        mixed = ile.ile_server_wait(srv, jid, 120000)
        mixed2 = ile.ile_server_wait(srv, jid2, 120000)
        for j, _ in others:
            ile.ile_server_wait(srv, j, 120000)
    finally:
        ile.ile_server_destroy(srv)
    assert alone.status == 0 and mixed.status == 0 and alone2.status == 0 and mixed2.status == 0
    assert _res(alone) == _res(mixed)
    assert _res(alone2) == _res(mixed2) and alone2.rounds == 5
    pr = orc.make_prior(t_window=p.t_window, d_min=p.d_min, d_max=p.d_max)
    dims = list(range(7))
    zseed, m = seed ^ 0x9E3779B97F4A7C15, 1 << 16
    g, state, shear = None, None, 0
    props, ths, lls = [], [], []
    for rnd in range(max_rounds):
        if g is None:
            th, _ = orc.draw_prior(pr, seed, rnd, 0, n)
            lr = np.zeros(n)
        else:
            th, lr = orc.draw_gmm(pr, g, seed, rnd, 0, n)
        L = orc.lnL(p, th)
        props.append(g)
        ths.append(th)
        lls.append(L)
        o = orc.marginalize(orc.pool_mixture_lw(pr, props, ths, lls))
        print(f"oracle round {rnd}: n_eff {o['n_eff']:.2f} ln L {o['ln_L']:.9f}")
        if o["n_eff"] >= target or rnd + 1 == max_rounds:
            break
        lw = L + lr
        if state is None:
            shear = orc.phase_shear_sign(th, lw)
        state = orc.em_fit(th, lw, dims, state=state, n_iter=8, n_comp=8, temper_ess=1.0 / 16.0, shear=shear)
        w, mu, cov = state
        g0 = orc.make_gmm(w, mu, cov, dims, shear=shear)
        lz = [math.log(max(orc.gmm_inbox_mass(pr, g0, j, zseed, rnd + 1, m), 0.5 / m)) for j in range(len(w))]
        g = orc.make_gmm(w, mu, cov, dims, ln_Z=lz, eps_def=0.05, shear=shear)
    print("pooled job", alone.rounds, alone.marg.ln_L, alone.marg.n_eff, "oracle", len(ths), o["ln_L"], o["n_eff"])
    assert alone.rounds == len(ths)
    assert abs(alone.marg.ln_L - o["ln_L"]) <= 1e-8 * max(1.0, abs(o["ln_L"]))
    assert abs(alone.marg.n_eff - o["n_eff"]) <= 1e-6 * o["n_eff"]
