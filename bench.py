"""Benchmark of the ILE extrinsic-likelihood hot path on one MI355X.

Workload (default): 3 detectors (H, L, V), 9 harmonics (l = 2, 3), one
injected SNR-20 data set and 256 intrinsic template points (M_c ~ U[20, 40],
q ~ U[1, 4]) each with its own Q (410-sample windows), U and V; 2^20
extrinsic prior samples per point.  One step = the whole path over all 256
points: counter-based prior draws, batched lnL over every point, batched
log-sum-exp estimator.  Inputs (Q, U, V, the sample buffers) are resident in
HBM before timing starts.  `value` is FP32 samples/s; the FP64 policy is run
on the same workload and reported beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--points 256] [--log2n 20]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "extrinsic lnL samples/s (FP32 vs FP64 plain, |dlnL|<=1e-3) + p50/p99 latency"
# per-sample FLOP model of the fused likelihood for K = 3, n = 9 (Hermitian /
# symmetric pair form): trig 90 + F 40K + tau 20K + Y 6n + T1 24Kn + quadratic
# P + 18KP (P = n(n+1)/2) + combine 12K + 10
FLOP_PER_SAMPLE = {(3, 9): 3493, (2, 5): 1069, (3, 17): 10057}
PEAK = {"fp32": 157.3e12, "fp64": 78.6e12}
HBM_PEAK = 8.0e12
# algorithmic HBM bytes per sample of the lnL kernel: 7 theta + ln p - ln p_s
# read, lnL + lw written (FP32: 4 B each; FP64: 8 B)
LNL_BYTES = {"fp32": 40, "fp64": 80}
# Measured HBM traffic of the FP32 lnL kernel on this workload: two
# `rocprofv3 --pmc` runs of `bench.py --probe` (FETCH_SIZE, then WRITE_SIZE,
# KiB per dispatch), each scaled by the same counter's reading for the probe's
# 1 GiB device copy (FETCH_SIZE reads half the bytes: x2.000; WRITE_SIZE x1.000).
# The figures hold only for the kernel source they were taken on.
# SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_{F32,F64} of the same probe give the FLOPs
# the kernel executes (64 lanes x (add + mul + 2 fma + trans) per wave
# instruction): 2,437 FP32 + 108 FP64 (sky direction and delays).
LNL_TRAFFIC = {"fetch_B_per_sample": 32.720, "write_B_per_sample": 8.000, "executed_flop_per_sample": 2545.0,
               "src_sha256": "49ca0381430112c6fa838f49740150430a22f9c69e09be241f2642f5c0f3af6a"}
# algorithmic HBM bytes per sample of the draw (7 theta + ln p - ln p_s
# written) and estimator (lw read) kernels
DRAW_BYTES = {"fp32": 32, "fp64": 64}
MARG_BYTES = {"fp32": 4, "fp64": 8}
LNL_SOURCES = ["paper_2505_11655_amd/csrc/k_lnl_impl.h", "paper_2505_11655_amd/csrc/ile_internal.h",
               "paper_2505_11655_amd/csrc/k_lnl_s1_p1.hip"]


def lnl_src_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in LNL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_problems(n_points, seed):
    import chirpgen
    recs = chirpgen.load_injections()
    rng = np.random.default_rng(seed)
    templates = [(float(rng.uniform(20, 40)), float(rng.uniform(1, 4))) for _ in range(n_points)]
    probs, _ = chirpgen.build_event(recs["c2"], ["H", "L", "V"], 9, 30.0, 2.0, 20.0,
                                    noise_seed=chirpgen.BASE_SEED + 2, templates=templates)
    return probs


def config_problems(name, n_points=1, snr=None):
    """The other configurations of the workload: C1 (HL, 5 modes, SNR 20) and
    C3 (HLV, 17 modes, mass ratio 20, SNR 100 by default, the template at the
    injected parameters; one noise realisation per point)."""
    import chirpgen
    recs = chirpgen.load_injections()
    rng = np.random.default_rng(7)
    if name == "c1":
        templates = [(30.0, 2.0)] + [(float(rng.uniform(25, 35)), float(rng.uniform(1.5, 2.5)))
                                     for _ in range(n_points - 1)]
        probs, _ = chirpgen.build_event(recs["c1"], ["H", "L"], 5, 30.0, 2.0, 20.0 if snr is None else snr,
                                        noise_seed=chirpgen.BASE_SEED + 11, templates=templates)
    else:
        # the precision configuration has its template at the true parameters:
        # n_points independent noise realisations of that one event
        probs = []
        for i in range(n_points):
            pr, _ = chirpgen.build_event(recs["c3"], ["H", "L", "V"], 17, 30.0, 20.0, 100.0 if snr is None else snr,
                                         noise_seed=chirpgen.BASE_SEED + 13 + 101 * i, templates=[(30.0, 20.0)])
            probs += pr
    return probs


def c3_proposal(snr):
    """The precision configuration's proposal: a narrow 8-component mixture
    over the 7 extrinsic parameters, means scattered by sigma/2 about the
    injection, covariance diag(sigma^2), sigma shrinking as 1/SNR."""
    import chirpgen
    th0 = np.array(chirpgen.load_injections()["c3"]["theta"])
    sig = np.array([0.01, 0.01, 1e-4, 0.05 * th0[3], 0.02, 0.05, 0.05]) * (100.0 / snr)
    rng = np.random.default_rng(31)
    means = th0[None, :] + rng.normal(size=(8, 7)) * sig[None, :] / 2
    return np.full(8, 1.0 / 8), means, [np.diag(sig ** 2)] * 8


def configs_leg(ile, torch, ctx, stream):
    """Draw + lnL + estimator throughput of the C1 and C3 configurations, per
    precision policy (the same step as the C2 benchmark).  C3 draws from its
    narrow mixture proposal (set on every job; FP32 + FP64-cancellation jobs
    then move their reference to their best pilot sample), at SNR 100 and
    400, and compares every policy's marginal ln L with FP64's on one set of
    draws."""
    c1 = config_problems("c1")
    out = {}
    pols = (("fp32", ile.ILE_FP32), ("fp64", ile.ILE_FP64), ("fp32c64", ile.ILE_FP32_CANCEL64))
    legs = [("c1_hl5_1x2e17", c1, 1 << 17, 50, 5, None), ("c1_hl5_1x2e24", c1, 1 << 24, 5, 1, None)]
    for snr in (100.0, 400.0):
        legs.append((f"c3_hlv17_snr{int(snr)}_16x2e20_mixture", config_problems("c3", n_points=16, snr=snr),
                     1 << 20, 5, 1, c3_proposal(snr)))
    for label, probs, n_per, steps, warm, prop in legs:
        out[label] = {}
        for name, pol in pols:
            if label.startswith("c1") and name == "fp32c64":
                continue
            r = run_policy(ile, torch, ctx, probs, pol, n_per, steps, warm, stream, proposal=prop)
            out[label][name] = {"samples_per_s": r["samples_per_s"], "ms_per_step": r["ms_per_step"],
                                "kernel_ms": r["kernel_ms"], "samples": r["N"]}
            log(f"{label} {name} {out[label][name]}")
        if prop is not None:
            out[label]["marginal_comparison"] = same_draw_marginals(ile, torch, ctx, probs, n_per, 4343, stream,
                                                                    proposal=prop)
            log(f"{label} same draws {out[label]['marginal_comparison']}")
    return out


def references_at_best(ile, torch, jobs, n_per, stream, seed=777):
    """FP32 + FP64-cancellation jobs: one untimed pilot pass (draws, lnL,
    estimator), then each job's reference point at its highest-weight pilot
    sample, as a caller does before the timed evaluations.  Every template
    peaks at its own point, so one shared reference (the proposal's) would sit
    away from most templates' samples."""
    J = len(jobs)
    N = J * n_per
    th = torch.empty((7, N), dtype=torch.float32, device="cuda")
    lr = torch.empty((N,), dtype=torch.float32, device="cuda")
    W = torch.empty((N,), dtype=torch.float64, device="cuda")
    ile.ile_draw(jobs[0], seed, 0, 0, N, th, N, lr, stream=stream)
    esz, osz = th.element_size(), W.element_size()
    ile.ile_eval_lnL_batch(jobs, [n_per] * J, [th.data_ptr() + j * n_per * esz for j in range(J)], [N] * J,
                           [lr.data_ptr() + j * n_per * esz for j in range(J)],
                           [W.data_ptr() + j * n_per * osz for j in range(J)], [None] * J, stream=stream)
    res = ile.ile_marginalize_batch(jobs, [n_per] * J, [W.data_ptr() + j * n_per * osz for j in range(J)],
                                    ile.ILE_MARG_RESET, want=True, stream=stream)
    torch.cuda.synchronize()
    for j, (job, r) in enumerate(zip(jobs, res)):
        if r["argmax"] >= 0:
            ile.ile_set_reference(job, th[:, j * n_per + r["argmax"]].double().cpu().numpy(), stream=stream)
    torch.cuda.synchronize()
    del th, lr, W


def run_policy(ile, torch, ctx, probs, policy, n_per, steps, warmup, stream, tmarg_R=None, proposal=None):
    """One step = draws + batched lnL (time-marginalised when tmarg_R is set) + batched estimator.
    proposal = (weights, means, covs): a mixture set on every job (draws come from it)."""
    # theta (and ln p - ln p_s) in the policy's theta type; lnL and lw in its
    # output type (FP64 for the FP64 and the FP32 + FP64-cancellation policies)
    dt = torch.float64 if policy == ile.ILE_FP64 else torch.float32
    ot = torch.float32 if policy == ile.ILE_FP32 else torch.float64
    jobs = [ile.ile_prepare(ctx, ile.ProblemHost(p, precision=policy)) for p in probs]
    if proposal is not None:
        for j in jobs:
            ile.ile_set_proposal(j, ile.gmm_params(*proposal))
        if policy == ile.ILE_FP32_CANCEL64:
            references_at_best(ile, torch, jobs, n_per, stream)
    J = len(jobs)
    N = J * n_per
    th = torch.empty((7, N), dtype=dt, device="cuda")
    lr = torch.empty((N,), dtype=dt, device="cuda")
    L = torch.empty((N,), dtype=ot, device="cuda")
    W = torch.empty((N,), dtype=ot, device="cuda")
    esz, osz = th.element_size(), L.element_size()
    theta_ptrs = [th.data_ptr() + j * n_per * esz for j in range(J)]
    lr_ptrs = [lr.data_ptr() + j * n_per * esz for j in range(J)]
    L_ptrs = [L.data_ptr() + j * n_per * osz for j in range(J)]
    W_ptrs = [W.data_ptr() + j * n_per * osz for j in range(J)]
    ns = [n_per] * J
    lds = [N] * J
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    t_kernel = {"draw": 0.0, "eval": 0.0, "marg": 0.0}
    res = None

    def step(seed, timed):
        nonlocal res
        ev[0].record(stream)
        ile.ile_draw(jobs[0], seed, 0, 0, N, th, N, lr, stream=stream)
        ev[1].record(stream)
        if tmarg_R is None:
            ile.ile_eval_lnL_batch(jobs, ns, theta_ptrs, lds, lr_ptrs, L_ptrs, W_ptrs, stream=stream)
        else:
            ile.ile_eval_lnL_tmarg_batch(jobs, ns, theta_ptrs, lds, lr_ptrs, L_ptrs, W_ptrs, oversample=tmarg_R,
                                         stream=stream)
        ev[2].record(stream)
        res = ile.ile_marginalize_batch(jobs, ns, W_ptrs, ile.ILE_MARG_RESET, want=False, stream=stream)
        ev[3].record(stream)
        if timed:
            ev[3].synchronize()
            t_kernel["draw"] += ev[0].elapsed_time(ev[1])
            t_kernel["eval"] += ev[1].elapsed_time(ev[2])
            t_kernel["marg"] += ev[2].elapsed_time(ev[3])

    for w in range(warmup):
        step(1000 + w, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        step(2000 + k, True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = ile.ile_marginalize_batch(jobs, [0] * J, [None] * J, ile.ILE_MARG_POOL, want=True, stream=stream)
    torch.cuda.synchronize()
    ln_marg = [o["ln_L"] for o in out]
    del res
    for j in jobs:
        ile.ile_job_release(j)
    del th, lr, L, W
    torch.cuda.empty_cache()
    per = {k: v / steps for k, v in t_kernel.items()}
    return dict(samples_per_s=N * steps / wall, ms_per_step=1e3 * wall / steps, kernel_ms=per, N=N,
                lnL_marg_first=out[0]["ln_L"], n_eff_first=out[0]["n_eff"], lnL_marg=ln_marg)


def same_draw_marginals(ile, torch, ctx, probs, n_per, seed, stream, proposal=None):
    """ln L of every point under each policy on ONE set of draws: the FP32
    prior draws (float theta), upcast exactly to double for the FP64 policy,
    so the differences are the arithmetic's alone (the parity protocol:
    identical samples on both sides)."""
    J = len(probs)
    N = J * n_per
    th32 = torch.empty((7, N), dtype=torch.float32, device="cuda")
    lr32 = torch.empty((N,), dtype=torch.float32, device="cuda")
    out = {}
    for name, pol in (("fp32", ile.ILE_FP32), ("fp64", ile.ILE_FP64), ("fp32c64", ile.ILE_FP32_CANCEL64)):
        jobs = [ile.ile_prepare(ctx, ile.ProblemHost(p, precision=pol)) for p in probs]
        if proposal is not None:
            for j in jobs:
                ile.ile_set_proposal(j, ile.gmm_params(*proposal))
            if pol == ile.ILE_FP32_CANCEL64:
                references_at_best(ile, torch, jobs, n_per, stream)
        if name == "fp32":
            ile.ile_draw(jobs[0], seed, 0, 0, N, th32, N, lr32, stream=stream)
        th = th32.double() if pol == ile.ILE_FP64 else th32
        lr = lr32.double() if pol == ile.ILE_FP64 else lr32
        ot = torch.float32 if pol == ile.ILE_FP32 else torch.float64
        L = torch.empty((N,), dtype=ot, device="cuda")
        W = torch.empty((N,), dtype=ot, device="cuda")
        esz, osz = th.element_size(), L.element_size()
        ile.ile_eval_lnL_batch(jobs, [n_per] * J, [th.data_ptr() + j * n_per * esz for j in range(J)], [N] * J,
                               [lr.data_ptr() + j * n_per * esz for j in range(J)],
                               [L.data_ptr() + j * n_per * osz for j in range(J)],
                               [W.data_ptr() + j * n_per * osz for j in range(J)], stream=stream)
        res = ile.ile_marginalize_batch(jobs, [n_per] * J, [W.data_ptr() + j * n_per * osz for j in range(J)],
                                        ile.ILE_MARG_RESET, want=True, stream=stream)
        torch.cuda.synchronize()
        out[name] = np.array([r["ln_L"] for r in res])
        for j in jobs:
            ile.ile_job_release(j)
        del th, lr, L, W
    del th32, lr32
    torch.cuda.empty_cache()
    return {"max_abs_dlnL_marg_fp32_vs_fp64": float(np.max(np.abs(out["fp32"] - out["fp64"]))),
            "max_abs_dlnL_marg_fp32c64_vs_fp64": float(np.max(np.abs(out["fp32c64"] - out["fp64"]))),
            "points": J, "samples_per_point": n_per,
            "draws": "one set of FP32 prior draws; the FP64 policy evaluates them upcast exactly"}


def serving_pool(per_class, seed):
    """Events of every (modes, detectors) class; each job of the stream picks one."""
    import chirpgen
    recs = chirpgen.load_injections()["pool"]
    rng = np.random.default_rng(seed)
    pool = []
    classes = [(n, d) for n in (5, 9, 17) for d in (("H", "L"), ("H", "L", "V"))]
    for ci, (n, dets) in enumerate(classes):
        for e in range(per_class):
            rec = recs[(ci * per_class + e) % len(recs)]
            snr = float(np.exp(rng.uniform(np.log(10), np.log(100))))
            probs, _ = chirpgen.build_event(rec, list(dets), n, float(rng.uniform(20, 40)),
                                            float(rng.uniform(1, 4)), snr, noise_seed=int(rng.integers(1 << 30)))
            pool.append(probs[0])
    return pool


def serving_leg(ile, ctx, pool, n_jobs, adaptive, seed, policy, budget=0, rate=None, integrator=0):
    """Submit a job stream with Poisson arrivals; returns throughput and latency.
    rate=None: all jobs at once (saturated).  integrator: the adaptive jobs'
    proposal (0: mixture refits, 1: adaptive volume, 2: adaptive Cartesian,
    3: mixture refits in sheared phases with the rounds pooled as draws of
    the mixture of their proposals)."""
    pooled = integrator == 3
    integrator = 0 if pooled else integrator
    rng = np.random.default_rng(seed)
    hosts = {}
    srv = ile.ile_server_create(ctx, max_active=64, hbm_budget_bytes=budget, chunk_samples=1 << 20)
    sizes = np.exp(rng.uniform(np.log(2 ** 14), np.log(2 ** 20), n_jobs)).astype(np.int64)
    picks = rng.integers(0, len(pool), n_jobs)
    gaps = rng.exponential(1.0 / rate, n_jobs) if rate else np.zeros(n_jobs)
    ids = []
    t0 = time.perf_counter()
    t_next = t0
    for k in range(n_jobs):
        t_next += gaps[k]
        while rate and time.perf_counter() < t_next:
            pass
        pi = int(picks[k])
        if pi not in hosts:
            hosts[pi] = ile.ProblemHost(pool[pi], precision=policy, dist_marg=adaptive)
        jo = ile.job_opts(n_samples=int(sizes[k]), adaptive=adaptive, round_samples=1 << 16, max_rounds=32,
                          n_eff_target=1000.0, seed=int(seed * 100003 + k), integrator=integrator,
                          pool=ile.ILE_POOL_MIXTURE if pooled else ile.ILE_POOL_ROUNDS, phase_shear=int(pooled))
        ids.append(ile.ile_server_submit(srv, hosts[pi], jo))
    res = [ile.ile_server_wait(srv, i, -1) for i in ids]
    t1 = time.perf_counter()
    ile.ile_server_destroy(srv)
    lat = np.array([(r.t_finish_ns - r.t_arrival_ns) * 1e-6 for r in res])
    waits = np.array([(r.t_admit_ns - r.t_arrival_ns) * 1e-6 for r in res])
    # arrival -> first pass that includes the job, and first pass -> result
    to_start = np.array([(r.t_start_ns - r.t_arrival_ns) * 1e-6 for r in res])
    in_flight = np.array([(r.t_finish_ns - r.t_start_ns) * 1e-6 for r in res])
    samples = sum(r.samples for r in res)
    first = min(r.t_arrival_ns for r in res)
    last = max(r.t_finish_ns for r in res)
    out = {"jobs": n_jobs, "samples": int(samples), "samples_per_s": samples / ((last - first) * 1e-9),
           "wall_s": t1 - t0, "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "admit_wait_p99_ms": float(np.percentile(waits, 99)),
           "to_first_pass_p50_ms": float(np.percentile(to_start, 50)),
           "to_first_pass_p99_ms": float(np.percentile(to_start, 99)),
           "in_flight_p50_ms": float(np.percentile(in_flight, 50)),
           "in_flight_p99_ms": float(np.percentile(in_flight, 99)),
           "p99_jobs_samples_median": float(np.median(np.array([r.samples for r in res])[lat >= np.percentile(lat, 99)])),
           "failed": int(sum(r.status != 0 for r in res))}
    if adaptive:
        rounds = np.array([r.rounds for r in res])
        neff = np.array([r.marg.n_eff for r in res])
        name = {0: "mixture", 1: "adaptive volume", 2: "adaptive Cartesian"}[integrator]
        if pooled:
            name = "mixture, sheared phases, rounds pooled as the mixture of their proposals"
        out.update({"integrator": name,
                    "rounds_mean": float(rounds.mean()),
                    "frac_reached_neff": float(np.mean(neff >= 1000.0)),
                    "n_eff_median": float(np.median(neff)),
                    "n_eff_per_sample_median": float(np.median(neff / np.maximum(1, [r.samples for r in res])))})
    return out


def serving_warmup(ile, ctx, pool):
    """One untimed saturated stream before the timed legs, as a server that has
    been up for a while would be: it fills the context's buffer pool for every
    size class the streams use (about a thousand device and pinned allocations
    when cold) and loads every kernel the passes launch.  Its own rate is the
    cold one and is reported beside the timed legs."""
    out = {}
    for policy, name in ((ile.ILE_FP32, "fp32"), (ile.ILE_FP64, "fp64")):
        r = serving_leg(ile, ctx, pool, 1000, False, 7, policy)
        out[f"cold_samples_per_s_{name}"] = r["samples_per_s"]
    return out


def fair_leg(ile, torch, ctx, prob, stream, log2n=26, log2k=20, reps=5):
    """Fair draws of 2^log2k samples from 2^log2n weighted ones (FP32 weights
    of a spread like a prior run's, seeded), the drawn theta copied out: the
    final-draw step of an ILE run at the scale of one benchmark step."""
    n, k = 1 << log2n, 1 << log2k
    job = ile.ile_prepare(ctx, ile.ProblemHost(prob, precision=ile.ILE_FP32))
    g = torch.Generator(device="cuda").manual_seed(7)
    lw = torch.randn(n, device="cuda", generator=g) * 30.0
    th = torch.randn((7, n), device="cuda", generator=g)
    idx = torch.empty(k, dtype=torch.int64, device="cuda")
    out = torch.empty((7, k), device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ile.ile_fair_draw(job, n, lw, 1, 0, k, idx, th, n, out, k, stream=stream)
    torch.cuda.synchronize()
    ev[0].record(stream)
    for r in range(reps):
        ile.ile_fair_draw(job, n, lw, 1, r, k, idx, th, n, out, k, stream=stream)
    ev[1].record(stream)
    ev[1].synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    ile.ile_job_release(job)
    del lw, th, idx, out
    torch.cuda.empty_cache()
    # HBM: lw read twice (tile sums, prefix sums), the prefix sums written once;
    # each draw reads ~log2 n prefix entries and copies 7 theta values
    bytes_ = n * (4 + 4 + 8) + k * (7 * 4 * 2 + 8)
    return {"n": n, "k": k, "ms": ms, "samples_per_s": n / (ms * 1e-3), "draws_per_s": k / (ms * 1e-3),
            "hbm_GBps_algorithmic": bytes_ / (ms * 1e-3) / 1e9, "hbm_frac": bytes_ / (ms * 1e-3) / HBM_PEAK}


def overlaps_leg(ile, torch, ctx, stream, n_points=256, n_modes=9, n_det=3, reps=3):
    """Q, U, V of eq. (QUV) for the benchmark's 256 intrinsic points (9 modes,
    3 detectors, 4 s at 4096 Hz, band 20-1024 Hz, 410-sample window) in one
    call; modes and data are seeded random spectra of that shape.  Each route
    for Q is timed twice: the wall time of the synchronous call, and the GPU
    time of its work alone (HIP events on the call's stream, recorded after a
    matrix product that keeps the stream busy while the host prepares the
    call, so host setup falls outside; the second event also holds the
    synchronisation wake-up, some tens of microseconds)."""
    n, df = 16384, 0.25
    g = torch.Generator(device="cuda").manual_seed(11)
    hlm = torch.randn((n_points, n_modes, n), dtype=torch.complex128, device="cuda", generator=g)
    data = torch.randn((n_det, n), dtype=torch.complex128, device="cuda", generator=g)
    Q = torch.empty((n_points, n_det, n_modes, 410), dtype=torch.complex128, device="cuda")
    U = torch.empty((n_points, n_det, n_modes, n_modes), dtype=torch.complex128, device="cuda")
    V = torch.empty_like(U)
    busy_a = torch.randn((4096, 4096), dtype=torch.float32, device="cuda", generator=g)
    n_band = int(np.count_nonzero((np.abs(np.fft.fftfreq(n, 1.0 / (n * df))) >= 20.0)
                                  & (np.abs(np.fft.fftfreq(n, 1.0 / (n * df))) <= 1024.0)))
    cols = n_points * n_det * n_modes
    flop_direct = 8.0 * 410 * n_band * cols
    flop_uv = 2 * 8.0 * (n_modes * (n_modes + 1) // 2) * n_band * n_points * n_det
    out = {"points": n_points, "modes": n_modes, "detectors": n_det, "band_bins": n_band, "window": 410}
    Qs = {}
    for name, route in (("direct", ile.ILE_QV_DIRECT), ("decimated", ile.ILE_QV_DECIMATED)):
        ile.ile_overlaps(ctx, hlm, data, df, 20.0, 1024.0, 410, 205, Q, U, V, stream=stream, route=route)
        t0 = time.perf_counter()
        for _ in range(reps):
            ile.ile_overlaps(ctx, hlm, data, df, 20.0, 1024.0, 410, 205, Q, U, V, stream=stream, route=route)
        wall = (time.perf_counter() - t0) * 1e3 / reps
        gpu = []
        for _ in range(reps):
            with torch.cuda.stream(stream):
                for _ in range(4):
                    busy_a = busy_a @ busy_a * (1.0 / 64.0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            ile.ile_overlaps(ctx, hlm, data, df, 20.0, 1024.0, 410, 205, Q, U, V, stream=stream, route=route)
            e1.record(stream)
            e1.synchronize()
            gpu.append(e0.elapsed_time(e1))
        gms = float(np.median(gpu))
        Qs[name] = Q.clone()
        out[name] = {"ms_per_call_wall": wall, "ms_per_call_gpu": gms,
                     "direct_equivalent_TFLOPs": (flop_direct + flop_uv) / (gms * 1e-3) / 1e12}
    dq = (Qs["direct"] - Qs["decimated"]).abs().max().item() / Qs["direct"].abs().max().item()
    out["decimated_vs_direct_max_rel_diff"] = dq
    out["speedup_gpu"] = out["direct"]["ms_per_call_gpu"] / out["decimated"]["ms_per_call_gpu"]
    out["note"] = ("direct: 410 x 8034 bins per column on the FP64 matrix cores; decimated: radix-16 partial "
                   "sums, then 32 x 1024 bins per column (26 decimated times used); flop figures count the "
                   "direct sum's work")
    del hlm, data, Q, U, V, Qs, busy_a
    torch.cuda.empty_cache()
    return out


def cpu_baseline(probs, budget_s=15.0):
    """The oracle as it stands, on a bounded sample of the same workload."""
    import chirpgen
    import oracle
    threads = os.cpu_count() or 1
    rng = np.random.default_rng(5)
    oracle.lnL(probs[0], chirpgen.prior_samples(rng, 4096), threads=threads)   # thread start-up
    m = 1 << 17
    th = chirpgen.prior_samples(rng, m)
    t0 = time.perf_counter()
    oracle.lnL(probs[0], th, threads=threads)
    dt = time.perf_counter() - t0
    n = int(min(max(m, budget_s / max(dt, 1e-6) * m), 1 << 26))
    th = chirpgen.prior_samples(rng, n)
    t0 = time.perf_counter()
    lw = oracle.lnL(probs[1 % len(probs)], th, threads=threads)
    oracle.marginalize(lw)
    dt = time.perf_counter() - t0
    m_one = 1 << 13
    t0 = time.perf_counter()
    oracle.lnL(probs[1 % len(probs)], th[:, :m_one], threads=1)
    c2_one = m_one / (time.perf_counter() - t0)
    per_config = {}
    for label, cp, m1 in (("c1_hl5", config_problems("c1")[0], 1 << 20),
                          ("c3_hlv17_snr100", config_problems("c3")[0], 1 << 18)):
        thc = chirpgen.prior_samples(rng, m1)
        t1 = time.perf_counter()
        oracle.marginalize(oracle.lnL(cp, thc, threads=threads))
        d_all = time.perf_counter() - t1
        m_one = max(m1 >> 4, 1024)
        t1 = time.perf_counter()
        oracle.lnL(cp, thc[:, :m_one], threads=1)
        d_one = time.perf_counter() - t1
        per_config[label] = {"samples_per_s_all_cores": m1 / d_all, "samples_per_s_one_thread": m_one / d_one,
                             "samples": m1}
    host = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            host = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), host)
    except OSError:
        pass
    return {"value": n / dt, "unit": "samples/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} prior samples of one intrinsic point of the same workload (lnL + estimator), "
                      f"FP64, OpenMP {threads} threads, {dt:.1f} s",
            "samples_per_s_one_thread": c2_one, "host_cpu": host,
            "per_config": per_config}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--points", type=int, default=256)
    ap.add_argument("--log2n", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--serving-jobs", type=int, default=10000)
    ap.add_argument("--adaptive-jobs", type=int, default=500)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-tmarg", action="store_true")
    ap.add_argument("--tmarg-log2n", type=int, default=16,
                    help="extrinsic samples per point of the time-marginalised leg (log2)")
    ap.add_argument("--tmarg-steps", type=int, default=5)
    ap.add_argument("--probe", action="store_true",
                    help="counter probe: one 1 GiB device copy (known bytes) then one step")
    ap.add_argument("--probe-policy", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--probe-tmarg", action="store_true",
                    help="the probe's step uses the time-marginalised likelihood (R = 4, 2^tmarg-log2n per point)")
    ap.add_argument("--adaptive-only", action="store_true",
                    help="run only the adaptive serving leg (--adaptive-jobs jobs) and print its summary")
    ap.add_argument("--overlaps-only", action="store_true",
                    help="run only the Q, U, V precompute leg (256 points) and print its summary")
    ap.add_argument("--adaptive-integrator", choices=["gmm", "av", "ac", "gmm_pool", "all"], default="all",
                    help="proposal of the adaptive serving leg(s)")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the saturated plain serving leg (FP32, --serving-jobs up to 2000) and print it")
    ap.add_argument("--configs-only", action="store_true",
                    help="run only the C1 / C3 configuration legs and print their summary")
    ap.add_argument("--no-configs", action="store_true")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {a.gpus} is not supported (the path shards by "
              "intrinsic point with no exchange between GPUs)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2505_11655_amd as ile
    assert torch.cuda.is_available(), "bench needs a GPU"
    log("building inputs ...")
    probs = make_problems(a.points, 250511655)
    n_per = 1 << a.log2n
    ctx = ile.ile_ctx_create(0, 0)
    stream = torch.cuda.current_stream()
    if a.probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)                      # reference kernel: reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del src, dst
        pol = ile.ILE_FP32 if a.probe_policy == "fp32" else ile.ILE_FP64
        if a.probe_tmarg:
            r = run_policy(ile, torch, ctx, probs, pol, 1 << a.tmarg_log2n, 1, 0, stream, tmarg_R=4)
        else:
            r = run_policy(ile, torch, ctx, probs, pol, n_per, 1, 0, stream)
        print(json.dumps({"probe": True, "policy": a.probe_policy, "samples": r["N"], "kernel_ms": r["kernel_ms"],
                          "lnl_src_sha256": lnl_src_sha256()}), flush=True)
        return
    if a.overlaps_only:
        print(json.dumps({"overlaps": overlaps_leg(ile, torch, ctx, stream)}), flush=True)
        return
    if a.configs_only:
        print(json.dumps({"configs": configs_leg(ile, torch, ctx, stream)}), flush=True)
        return
    integrators = {"gmm": [0], "av": [1], "ac": [2], "gmm_pool": [3], "all": [0, 1, 2, 3]}[a.adaptive_integrator]
    leg_name = {0: "adaptive_saturated", 1: "adaptive_av_saturated", 2: "adaptive_ac_saturated",
                3: "adaptive_pooled_saturated"}
    if a.serving_only:
        pool = serving_pool(64, 250511655 + 4)
        warm = serving_warmup(ile, ctx, pool)
        sat = serving_leg(ile, ctx, pool, min(2000, a.serving_jobs), False, 11, ile.ILE_FP32)
        print(json.dumps({"serving_warmup": warm, "plain_saturated": sat}), flush=True)
        return
    if a.adaptive_only:
        pool = serving_pool(8, 250511655 + 4)
        out = {}
        for it in integrators:
            out[leg_name[it]] = serving_leg(
                ile, ctx, pool, a.adaptive_jobs, True, 13, ile.ILE_FP32, integrator=it)
        print(json.dumps(out), flush=True)
        return
    log("fp32 ...")
    r32 = run_policy(ile, torch, ctx, probs, ile.ILE_FP32, n_per, a.steps, a.warmup, stream)
    log(f"fp32 {dict((k, v) for k, v in r32.items() if k != 'lnL_marg')}")
    r64 = None
    if not a.no_fp64:
        log("fp64 ...")
        r64 = run_policy(ile, torch, ctx, probs, ile.ILE_FP64, n_per, a.steps, a.warmup, stream)
        log(f"fp64 {dict((k, v) for k, v in r64.items() if k != 'lnL_marg')}")
    rmx = None
    if not a.no_fp64:
        log("fp32 + fp64 cancellation ...")
        rmx = run_policy(ile, torch, ctx, probs, ile.ILE_FP32_CANCEL64, n_per, a.steps, a.warmup, stream)
        log(f"fp32c64 {dict((k, v) for k, v in rmx.items() if k != 'lnL_marg')}")
    same = None
    if not a.no_fp64:
        log("marginals of all policies on one set of draws ...")
        same = same_draw_marginals(ile, torch, ctx, probs, n_per, 4242, stream)
        log(f"same draws {same}")
    tmarg = None
    if not a.no_tmarg:
        R = 4
        tw = probs[0].t_window
        nodes = 2 * int(math.floor(R * tw / probs[0].dt + 1e-9)) + 1
        tmarg = {"oversample": R, "nodes_per_sample": nodes, "samples_per_point": 1 << a.tmarg_log2n}
        for name, pol in (("fp32", ile.ILE_FP32), ("fp64", ile.ILE_FP64)):
            if name == "fp64" and a.no_fp64:
                continue
            log(f"time-marginalised {name} ...")
            rt = run_policy(ile, torch, ctx, probs, pol, 1 << a.tmarg_log2n, a.tmarg_steps, 1, stream, tmarg_R=R)
            log(f"tmarg {name} {dict((k, v) for k, v in rt.items() if k != 'lnL_marg')}")
            tmarg[name] = {"samples_per_s": rt["samples_per_s"], "nodes_per_s": rt["samples_per_s"] * nodes,
                           "ms_per_step": rt["ms_per_step"], "kernel_ms": rt["kernel_ms"],
                           "lnL_marg_first": rt["lnL_marg_first"]}
    configs = None
    if not a.no_configs:
        log("configurations C1, C3 ...")
        configs = configs_leg(ile, torch, ctx, stream)
    log("fair draws ...")
    fair = fair_leg(ile, torch, ctx, probs[0], stream)
    log(f"fair {fair}")
    log("overlaps ...")
    qv = overlaps_leg(ile, torch, ctx, stream)
    log(f"overlaps {qv}")
    serving = None
    if not a.no_serving:
        log("serving pool ...")
        pool = serving_pool(64, 250511655 + 4)
        warm = serving_warmup(ile, ctx, pool)
        log(f"serving warm-up {warm}")
        sat = serving_leg(ile, ctx, pool, min(2000, a.serving_jobs), False, 11, ile.ILE_FP32)
        log(f"saturated {sat}")
        e_n = (2 ** 20 - 2 ** 14) / math.log(2 ** 6)
        serving = {"plain_saturated": sat, "warmup": warm,
                   "pool": f"{len(pool)} events (64 per (modes, detectors) class, SNR log-uniform 10-100), reused",
                   "arrival_rates_per_s": {}}
        for frac in (0.5, 0.7, 0.9):
            rate = frac * sat["samples_per_s"] / e_n
            leg = serving_leg(ile, ctx, pool, a.serving_jobs, False, 12, ile.ILE_FP32, rate=rate)
            log(f"poisson {frac} {leg}")
            serving[f"plain_poisson_{frac}"] = leg
            serving["arrival_rates_per_s"][str(frac)] = rate
        # admission by footprint: the saturated stream under small budgets queues
        for gib, label in ((2.0, "2GiB"), (0.25, "256MiB")):
            leg = serving_leg(ile, ctx, pool, min(2000, a.serving_jobs), False, 11, ile.ILE_FP32,
                              budget=int(gib * (1 << 30)))
            log(f"saturated budget {label} {leg}")
            serving[f"plain_saturated_budget_{label}"] = leg
        # FP64 serving for comparison: saturated, and Poisson at 0.7 of its own saturated rate
        sat64 = serving_leg(ile, ctx, pool, min(2000, a.serving_jobs), False, 11, ile.ILE_FP64)
        log(f"saturated fp64 {sat64}")
        serving["plain_saturated_fp64"] = sat64
        rate64 = 0.7 * sat64["samples_per_s"] / e_n
        serving["plain_poisson_0.7_fp64"] = serving_leg(ile, ctx, pool, a.serving_jobs, False, 12, ile.ILE_FP64,
                                                        rate=rate64)
        serving["arrival_rates_per_s"]["0.7_fp64"] = rate64
        log(f"poisson fp64 {serving['plain_poisson_0.7_fp64']}")
        if a.adaptive_jobs > 0:
            for it in integrators:
                ada = serving_leg(ile, ctx, pool, a.adaptive_jobs, True, 13, ile.ILE_FP32, integrator=it)
                log(f"{leg_name[it]} {ada}")
                serving[leg_name[it]] = ada
    N = r32["N"]
    flop = FLOP_PER_SAMPLE[(3, 9)]
    t_eval = r32["kernel_ms"]["eval"] * 1e-3
    achieved = flop * N / t_eval
    bytes_eval = LNL_BYTES["fp32"] * N
    traffic = None
    executed = None
    if LNL_TRAFFIC["src_sha256"] is not None and LNL_TRAFFIC["src_sha256"] == lnl_src_sha256():
        traffic = (LNL_TRAFFIC["fetch_B_per_sample"] + LNL_TRAFFIC["write_B_per_sample"]) * N
        executed = LNL_TRAFFIC["executed_flop_per_sample"] * N / t_eval / 1e12
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK["fp32"] / 1e12, "unit": "TFLOP/s",
            "frac": achieved / PEAK["fp32"], "traffic": traffic, "traffic_unit": "bytes per launch",
            "algorithmic_bytes_per_launch": bytes_eval,
            "kernel": "k_lnl (fused lnL, FP32, K=3, 9 modes)", "flop_per_sample": flop,
            "samples_per_launch": N, "avg_launch_ms": r32["kernel_ms"]["eval"],
            "hbm_algorithmic_GBps": bytes_eval / t_eval / 1e9,
            "hbm_frac": bytes_eval / t_eval / HBM_PEAK,
            "executed_TFLOPs": executed,
            "executed_frac_of_nonpacked_fp32": None if executed is None else executed / 78.6}

    def hbm(per_sample, r, key):
        t = r["kernel_ms"][key] * 1e-3
        return {"ms": r["kernel_ms"][key], "bytes": per_sample * r["N"],
                "GBps": per_sample * r["N"] / t / 1e9, "hbm_frac": per_sample * r["N"] / t / HBM_PEAK}
    kernels = {"fp32": {"draw": hbm(DRAW_BYTES["fp32"], r32, "draw"),
                        "lnl": hbm(LNL_BYTES["fp32"], r32, "eval"),
                        "marg": hbm(MARG_BYTES["fp32"], r32, "marg")}}
    if r64 is not None:
        kernels["fp64"] = {"draw": hbm(DRAW_BYTES["fp64"], r64, "draw"),
                           "lnl": hbm(LNL_BYTES["fp64"], r64, "eval"),
                           "marg": hbm(MARG_BYTES["fp64"], r64, "marg")}
    line = {
        "metric": METRIC, "value": r32["samples_per_s"], "unit": "samples/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": r32["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"HLV, 9 modes (l=2,3), {a.points} intrinsic points x 2^{a.log2n} prior "
                               "samples, SNR 20, 410-sample Q windows, draw+lnL+estimator per step",
                   "points": a.points, "samples_per_point": n_per, "detectors": 3, "modes": 9},
        "roofline": roof,
        "kernel_ms": r32["kernel_ms"],
        "kernels_hbm": kernels,
        "fp64": None if r64 is None else {"value": r64["samples_per_s"], "ms_per_step": r64["ms_per_step"],
                                          "kernel_ms": r64["kernel_ms"],
                                          "fp32_over_fp64": r32["samples_per_s"] / r64["samples_per_s"],
                                          # the arithmetic's error: every policy on the same draws
                                          "max_abs_dlnL_marg_fp32_vs_fp64": same["max_abs_dlnL_marg_fp32_vs_fp64"],
                                          "marginal_comparison": same,
                                          # the timed steps' own draws: the FP64 run's draws are the FP32
                                          # run's before rounding to float, so these differ by where the
                                          # samples sit as well as by the arithmetic
                                          "max_abs_dlnL_marg_fp32_vs_fp64_own_draws": float(np.max(np.abs(
                                              np.array(r32["lnL_marg"]) - np.array(r64["lnL_marg"]))))},
        "fp32_cancel64": None if rmx is None else {
            "value": rmx["samples_per_s"], "ms_per_step": rmx["ms_per_step"], "kernel_ms": rmx["kernel_ms"],
            "max_abs_dlnL_marg_vs_fp64": same["max_abs_dlnL_marg_fp32c64_vs_fp64"]},
        "time_marginalised": tmarg,
        "configs": configs,
        "fair_draws": fair,
        "overlaps": qv,
        "serving": serving,
        "cpu_baseline": None if a.no_cpu else cpu_baseline(probs),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
