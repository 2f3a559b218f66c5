"""The estimator entry point that allocates nothing (ile_marginalize_noalloc)
against ile_marginalize: the same result to the bit, on two calls in a row
(the second with fewer samples, so stale partials of the first call in the
shared scratch would show), with reset and with pooling, in FP64 and FP32;
sizes beyond the scratch are rejected on the host."""
import numpy as np
import pytest

import chirpgen
import paper_2505_11655_amd as ile
from tests import gpu_util as gu

torch = pytest.importorskip("torch")

KEYS = ("n", "n_nonfinite", "argmax", "ln_L", "ln_sigma", "n_eff", "n_ess", "max_lw")


def _same(a, b):
    for k in KEYS:
        assert a[k] == b[k] or (np.isnan(a[k]) and np.isnan(b[k])), (k, a[k], b[k])


@pytest.mark.gpu
@pytest.mark.parametrize("policy", [ile.ILE_FP64, ile.ILE_FP32])
def test_noalloc_equals_marginalize(orc, policy):
    rng = np.random.default_rng(71)
    p = chirpgen.random_problem(rng, 5, ["H", "L"])
    dt = torch.float32 if policy == ile.ILE_FP32 else torch.float64
    ja = ile.ile_prepare(gu.ctx(), ile.ProblemHost(p, precision=policy))
    jb = ile.ile_prepare(gu.ctx(), ile.ProblemHost(p, precision=policy))
    try:
        sizes = [3 * (1 << 20) + 7, 5000]
        bufs = []
        for k, n in enumerate(sizes):
            lw = rng.normal(size=n) * 15 - 40 * k
            lw[rng.integers(0, n, size=4)] = -np.inf
            bufs.append(torch.from_numpy(lw).to(device="cuda", dtype=dt))
        # two calls in a row, each reset (the second smaller), then a pooled one
        for n, buf in zip(sizes, bufs):
            print("noalloc reset n =", n, "policy", policy, flush=True)
            ra = ile.ile_marginalize_noalloc(ja, n, buf, ile.ILE_MARG_RESET)
            rb = ile.ile_marginalize(jb, n, buf, ile.ILE_MARG_RESET)
            _same(ra, rb)
            o = orc.marginalize(buf.double().cpu().numpy())
            assert abs(ra["ln_L"] - o["ln_L"]) <= 1e-10 * max(1.0, abs(o["ln_L"]))
            assert ra["argmax"] == o["argmax"]
        print("noalloc pool", flush=True)
        ra = ile.ile_marginalize_noalloc(ja, sizes[0], bufs[0], ile.ILE_MARG_POOL)
        rb = ile.ile_marginalize(jb, sizes[0], bufs[0], ile.ILE_MARG_POOL)
        _same(ra, rb)
        assert ra["n"] == sizes[0] + sizes[1]
        # empty input
        ra = ile.ile_marginalize_noalloc(ja, 0, None, ile.ILE_MARG_RESET)
        rb = ile.ile_marginalize(jb, 0, None, ile.ILE_MARG_RESET)
        _same(ra, rb)
        # more samples than the fixed scratch holds: rejected before any launch
        big = ile.ile_marginalize_noalloc_max() + 1
        with pytest.raises(ile.IleError) as ei:
            ile.ile_marginalize_noalloc(ja, big, bufs[1], ile.ILE_MARG_RESET)
        assert ei.value.status == -3  # ILE_E_TOO_BIG
        # the job still works after the rejection
        ra = ile.ile_marginalize_noalloc(ja, sizes[1], bufs[1], ile.ILE_MARG_RESET)
        rb = ile.ile_marginalize(jb, sizes[1], bufs[1], ile.ILE_MARG_RESET)
        _same(ra, rb)
        torch.cuda.synchronize()
    finally:
        ile.ile_job_release(ja)
        ile.ile_job_release(jb)
