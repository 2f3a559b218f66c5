"""Q, U, V of eq. (QUV) computed on the GPU from modes and data, against the
oracle's definition: one event (H, L, V; 9 modes; noise), several intrinsic
points in one call with a per-detector PSD weight, an odd grid length, and the
precomputed inputs used for the likelihood; both routes for Q (the direct
windowed sum and the decimated one) on the same inputs, every radix of the
decimated route, and its refusal where no radix applies."""
import numpy as np
import pytest

import chirpgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2505_11655_amd as ile  # noqa: E402
from tests import gpu_util as gu  # noqa: E402


def _gpu(hlm, data, df, f_lo, f_hi, n_time, win_half, inv_psd=None, route=0):
    h = torch.from_numpy(np.ascontiguousarray(hlm)).to("cuda")
    d = torch.from_numpy(np.ascontiguousarray(data)).to("cuda")
    w = None if inv_psd is None else torch.from_numpy(np.ascontiguousarray(inv_psd)).to("cuda")
    npnt = 1 if hlm.ndim == 2 else hlm.shape[0]
    na, nd = hlm.shape[-2], data.shape[0]
    Q = torch.zeros((npnt, nd, na, n_time), dtype=torch.complex128, device="cuda")
    U = torch.zeros((npnt, nd, na, na), dtype=torch.complex128, device="cuda")
    V = torch.zeros((npnt, nd, na, na), dtype=torch.complex128, device="cuda")
    ile.ile_overlaps(gu.ctx(), h, d, df, f_lo, f_hi, n_time, win_half, Q, U, V, inv_psd=w, route=route)
    torch.cuda.synchronize()
    return Q.cpu().numpy(), U.cpu().numpy(), V.cpu().numpy()


def _close(g, o, tol=1e-12):
    scale = np.abs(o).max()
    assert np.abs(g - o).max() <= tol * scale, np.abs(g - o).max() / scale


def test_overlaps_one_event_matches_oracle(orc):
    recs = chirpgen.load_injections()
    probs, ev = chirpgen.build_event(recs["c2"], ["H", "L", "V"], 9, 30.0, 2.0, 20.0, noise_seed=12)
    hlm = chirpgen.modes_fd(ev["f"], probs[0].modes, 30.0, 2.0, amp0=ev["amp0"])
    Qg, Ug, Vg = _gpu(hlm, ev["data"], ev["df"], 20.0, 1024.0, 410, 205)
    Qo, Uo, Vo = orc.overlaps_qv(hlm, ev["data"], None, ev["df"], 20.0, 1024.0, 410, 205)
    _close(Qg[0], Qo)
    _close(Ug[0], Uo)
    _close(Vg[0], Vo)
    # U Hermitian and V symmetric exactly (mirrored halves)
    assert np.array_equal(Ug[0], np.conj(np.transpose(Ug[0], (0, 2, 1))))
    assert np.array_equal(Vg[0], np.transpose(Vg[0], (0, 2, 1)))


def test_overlaps_several_points_with_psd(orc):
    """Three intrinsic points (different chirp masses and mass ratios) in one
    call with a coloured PSD weight per detector; each block equals the
    oracle for that point."""
    rng = np.random.default_rng(130)
    f, df = chirpgen.freq_grid()
    modes = chirpgen.mode_set(5)
    hl = np.stack([chirpgen.modes_fd(f, modes, mc, q) for mc, q in ((25.0, 1.5), (31.0, 2.5), (38.0, 3.7))])
    data = rng.normal(size=(2, f.size)) + 1j * rng.normal(size=(2, f.size))
    w = 1.0 / (1.0 + (np.abs(f)[None, :] / 200.0) ** 2 + rng.uniform(0, 0.1, (2, f.size)))
    w = 0.5 * (w + w[:, (f.size - np.arange(f.size)) % f.size])     # w(-f) = w(f)
    Qg, Ug, Vg = _gpu(hl, data, df, 20.0, 1024.0, 410, 205, inv_psd=w)
    for p in range(3):
        Qo, Uo, Vo = orc.overlaps_qv(hl[p], data, w, df, 20.0, 1024.0, 410, 205)
        _close(Qg[p], Qo)
        _close(Ug[p], Uo)
        _close(Vg[p], Vo)


def test_overlaps_odd_grid_and_window(orc):
    """An odd grid length (n = 3001, df = 1.25 Hz), a 77-sample window
    centred off the middle, random modes."""
    rng = np.random.default_rng(131)
    n, df = 3001, 1.25
    hl = rng.normal(size=(4, n)) + 1j * rng.normal(size=(4, n))
    data = rng.normal(size=(3, n)) + 1j * rng.normal(size=(3, n))
    Qg, Ug, Vg = _gpu(hl, data, df, 30.0, 900.0, 77, 20)
    Qo, Uo, Vo = orc.overlaps_qv(hl, data, None, df, 30.0, 900.0, 77, 20)
    _close(Qg[0], Qo)
    _close(Ug[0], Uo)
    _close(Vg[0], Vo)


def test_overlaps_feed_the_likelihood(orc):
    """The GPU-precomputed Q, U, V of an event, prepared as a job, give the
    oracle's likelihood (on the oracle's own precompute) on prior samples."""
    recs = chirpgen.load_injections()
    probs, ev = chirpgen.build_event(recs["c1"], ["H", "L"], 5, 30.0, 2.0, 20.0, noise_seed=13)
    p = probs[0]
    hlm = chirpgen.modes_fd(ev["f"], p.modes, 30.0, 2.0, amp0=ev["amp0"])
    Qg, Ug, Vg = _gpu(hlm, ev["data"], ev["df"], 20.0, 1024.0, 410, 205)
    Qo, Uo, Vo = orc.overlaps_qv(hlm, ev["data"], None, ev["df"], 20.0, 1024.0, 410, 205)
    pg = p.__class__(**{**p.__dict__})
    pg.Q, pg.U, pg.V = Qg[0], Ug[0], Vg[0]
    po = p.__class__(**{**p.__dict__})
    po.Q, po.U, po.V = Qo, Uo, Vo
    rng = np.random.default_rng(132)
    th = chirpgen.prior_samples(rng, 4001)
    job = ile.ile_prepare(gu.ctx(), ile.ProblemHost(pg, precision=ile.ILE_FP64))
    try:
        L, _ = gu.gpu_eval(job, np.ascontiguousarray(th), ile.ILE_FP64)
    finally:
        ile.ile_job_release(job)
    ref = orc.lnL(po, th)
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(L))
    assert np.allclose(L[fin], ref[fin], rtol=1e-9, atol=1e-9)


def test_overlaps_one_slice_and_short_window(orc):
    """A one-sample window over a short band (102 bins, fewer than one band
    slice): U and V come from a single slice written directly, Q from a
    single time tile."""
    rng = np.random.default_rng(133)
    n, df = 200, 1.0
    hl = rng.normal(size=(2, 4, n)) + 1j * rng.normal(size=(2, 4, n))
    data = rng.normal(size=(2, n)) + 1j * rng.normal(size=(2, n))
    Qg, Ug, Vg = _gpu(hl, data, df, 10.0, 60.0, 1, 0)
    for p in range(2):
        Qo, Uo, Vo = orc.overlaps_qv(hl[p], data, None, df, 10.0, 60.0, 1, 0)
        _close(Qg[p], Qo)
        _close(Ug[p], Uo)
        _close(Vg[p], Vo)


def test_overlaps_many_modes_and_detectors(orc):
    """24 modes (300 pairs: two pair groups of U, V blocks) and 5 detectors
    (two detector groups) with a PSD weight; several band slices."""
    rng = np.random.default_rng(134)
    n, df = 1024, 2.0
    hl = rng.normal(size=(24, n)) + 1j * rng.normal(size=(24, n))
    data = rng.normal(size=(5, n)) + 1j * rng.normal(size=(5, n))
    f = np.fft.fftfreq(n, 1.0 / (n * df))
    w = 1.0 / (1.0 + (np.abs(f)[None, :] / 300.0) ** 2) * rng.uniform(0.5, 1.5, (5, 1))
    Qg, Ug, Vg = _gpu(hl, data, df, 20.0, 900.0, 33, 16, inv_psd=w)
    Qo, Uo, Vo = orc.overlaps_qv(hl, data, w, df, 20.0, 900.0, 33, 16)
    _close(Qg[0], Qo)
    _close(Ug[0], Uo)
    _close(Vg[0], Vo)
    assert np.array_equal(Ug[0], np.conj(np.transpose(Ug[0], (0, 2, 1))))
    assert np.array_equal(Vg[0], np.transpose(Vg[0], (0, 2, 1)))


@pytest.mark.parametrize("route", [ile.ILE_QV_DIRECT, ile.ILE_QV_DECIMATED])
def test_overlaps_both_routes_event_shape(orc, route):
    """The benchmark's shape (4 s at 4096 Hz: 16384 bins, 20-1024 Hz, the
    410-sample window centred) for two points with a PSD weight, forced
    through each route; the decimated one takes radix 16 here (26 decimated
    times in a 32-row tile)."""
    rng = np.random.default_rng(135)
    f, df = chirpgen.freq_grid()
    modes = chirpgen.mode_set(5)
    hl = np.stack([chirpgen.modes_fd(f, modes, mc, q) for mc, q in ((27.0, 1.3), (35.0, 3.1))])
    data = rng.normal(size=(3, f.size)) + 1j * rng.normal(size=(3, f.size))
    w = 1.0 / (1.0 + (np.abs(f)[None, :] / 150.0) ** 2) * rng.uniform(0.5, 1.5, (3, 1))
    Qg, Ug, Vg = _gpu(hl, data, df, 20.0, 1024.0, 410, 205, inv_psd=w, route=route)
    for p in range(2):
        Qo, Uo, Vo = orc.overlaps_qv(hl[p], data, w, df, 20.0, 1024.0, 410, 205)
        _close(Qg[p], Qo)
        _close(Ug[p], Uo)
        _close(Vg[p], Vo)


def _dec_choice(n, n_time, win_half):
    """The radix and tile height the decimated route takes: of R in 2..16
    dividing n whose decimated window fits one 32- or 64-row tile, the lowest
    tile + 49 + 2R."""
    best = None
    for r in (2, 4, 8, 16):
        if n % r:
            continue
        nt = (n_time - 1 - win_half) // r - (-win_half) // r + 1
        tile = 32 if nt <= 32 else 64 if nt <= 64 else 0
        if tile and (best is None or tile + 49 + 2 * r < best[0]):
            best = (tile + 49 + 2 * r, r, tile)
    return best[1:]


@pytest.mark.parametrize("n,df,n_time,win_half,radix,tile", [
    (200, 1.0, 1, 0, 2, 32),         # one window time, N2 = 100 (one band slice)
    (1002, 1.0, 100, 50, 2, 64),
    (3000, 1.25, 77, 20, 4, 32),     # off-centre window: decimated times -5 .. 14
    (1004, 2.0, 200, 100, 4, 64),
    (1024, 2.0, 200, 150, 8, 32),    # window mostly before the reference time
    (3000, 1.0, 400, 200, 8, 64),
    (2048, 1.0, 500, 250, 16, 32),
    (4096, 0.5, 1000, 499, 16, 64),  # 64 decimated times, -32 .. 31
])
def test_overlaps_decimated_every_radix(orc, n, df, n_time, win_half, radix, tile):
    """The decimated route forced on random modes and data for every radix
    and both tile heights of its matrix-core product, against the oracle."""
    assert _dec_choice(n, n_time, win_half) == (radix, tile)
    rng = np.random.default_rng(136 + radix + tile)
    hl = rng.normal(size=(3, n)) + 1j * rng.normal(size=(3, n))
    data = rng.normal(size=(2, n)) + 1j * rng.normal(size=(2, n))
    f_hi = 0.45 * n * df
    Qg, Ug, Vg = _gpu(hl, data, df, 3.0 * df, f_hi, n_time, win_half, route=ile.ILE_QV_DECIMATED)
    Qo, Uo, Vo = orc.overlaps_qv(hl, data, None, df, 3.0 * df, f_hi, n_time, win_half)
    _close(Qg[0], Qo)
    _close(Ug[0], Uo)
    _close(Vg[0], Vo)


def test_overlaps_decimated_refused_without_radix():
    """A prime grid length has no radix: the forced decimated route is an
    error (ILE_E_INVALID), and the automatic route still answers."""
    rng = np.random.default_rng(140)
    n = 3001
    hl = rng.normal(size=(2, n)) + 1j * rng.normal(size=(2, n))
    data = rng.normal(size=(1, n)) + 1j * rng.normal(size=(1, n))
    with pytest.raises(Exception, match="decimated route"):
        _gpu(hl, data, 1.0, 5.0, 900.0, 41, 20, route=ile.ILE_QV_DECIMATED)
    _gpu(hl, data, 1.0, 5.0, 900.0, 41, 20, route=ile.ILE_QV_AUTO)


def test_overlaps_auto_falls_back_to_direct_within_budget(orc):
    """A context whose device budget holds the direct route's scratch but not
    the decimated route's: 96 points x 9 modes x 3 detectors on the
    16384-bin event grid need about 480 MiB through the direct sum (X over
    8034 band bins, 10 band slices) and about 700 MiB through the decimated
    one (the partial sums over all 16384 bins), allocated in power-of-two
    classes of 512 MiB and 1 GiB; the budget is 768 MiB.  The forced
    decimated route reports the budget; the automatic route answers through
    the direct sum (two points checked against the oracle)."""
    rng = np.random.default_rng(141)
    f, df = chirpgen.freq_grid()
    n = f.size
    npt, na, nd = 96, 9, 3
    hl = rng.normal(size=(npt, na, n)) + 1j * rng.normal(size=(npt, na, n))
    data = rng.normal(size=(nd, n)) + 1j * rng.normal(size=(nd, n))
    ctx = ile.ile_ctx_create(0, 768 * 2 ** 20)
    try:
        h = torch.from_numpy(hl).to("cuda")
        d = torch.from_numpy(data).to("cuda")
        Q = torch.zeros((npt, nd, na, 410), dtype=torch.complex128, device="cuda")
        U = torch.zeros((npt, nd, na, na), dtype=torch.complex128, device="cuda")
        V = torch.zeros_like(U)
        with pytest.raises(Exception, match="budget"):
            ile.ile_overlaps(ctx, h, d, df, 20.0, 1024.0, 410, 205, Q, U, V, route=ile.ILE_QV_DECIMATED)
        with pytest.raises(Exception, match="bad overlap route"):
            ile.ile_overlaps(ctx, h, d, df, 20.0, 1024.0, 410, 205, Q, U, V, route=7)
        before = ile.lib().ile_last_error()
        ile.ile_overlaps(ctx, h, d, df, 20.0, 1024.0, 410, 205, Q, U, V, route=ile.ILE_QV_AUTO)
        # the fallback's failed first allocation is not reported as an error:
        # the last failing call is still the one with the bad route
        assert ile.lib().ile_last_error() == before == b"bad overlap route"
        torch.cuda.synchronize()
        Qg, Ug, Vg = Q.cpu().numpy(), U.cpu().numpy(), V.cpu().numpy()
    finally:
        ile.ile_ctx_destroy(ctx)
    for p in (0, npt - 1):
        Qo, Uo, Vo = orc.overlaps_qv(hl[p], data, None, df, 20.0, 1024.0, 410, 205)
        _close(Qg[p], Qo)
        _close(Ug[p], Uo)
        _close(Vg[p], Vo)


def test_overlaps_full_size_sampled(orc):
    """The benchmark's launch shape: 256 points x 9 modes x 3 detectors on
    the 16384-bin grid (20-1024 Hz, the centred 410-sample window), seeded
    random spectra made on the host.  Both routes run at full size and agree
    everywhere to 1e-12 of max |Q| (U, V are shared), and the automatic
    route's output equals the oracle at sampled points (first, a middle
    one, last) for every detector, mode and window time."""
    rng = np.random.default_rng(142)
    n, df = 16384, 0.25
    npt, na, nd = 256, 9, 3
    hl = rng.standard_normal((npt, na, n)) + 1j * rng.standard_normal((npt, na, n))
    data = rng.standard_normal((nd, n)) + 1j * rng.standard_normal((nd, n))
    h = torch.from_numpy(hl).to("cuda")
    d = torch.from_numpy(data).to("cuda")
    out = {}
    for route in (ile.ILE_QV_AUTO, ile.ILE_QV_DIRECT):
        Q = torch.empty((npt, nd, na, 410), dtype=torch.complex128, device="cuda")
        U = torch.empty((npt, nd, na, na), dtype=torch.complex128, device="cuda")
        V = torch.empty_like(U)
        ile.ile_overlaps(gu.ctx(), h, d, df, 20.0, 1024.0, 410, 205, Q, U, V, route=route)
        torch.cuda.synchronize()
        out[route] = (Q.cpu().numpy(), U.cpu().numpy(), V.cpu().numpy())
    del h, d
    torch.cuda.empty_cache()
    Qa, Ua, Va = out[ile.ILE_QV_AUTO]
    Qd, Ud, Vd = out[ile.ILE_QV_DIRECT]
    _close(Qa, Qd)
    assert np.array_equal(Ua, Ud) and np.array_equal(Va, Vd)
    for p in (0, 131, npt - 1):
        Qo, Uo, Vo = orc.overlaps_qv(hl[p], data, None, df, 20.0, 1024.0, 410, 205)
        _close(Qa[p], Qo)
        _close(Ua[p], Uo)
        _close(Va[p], Vo)
