"""Seeded synthetic inputs for the ILE extrinsic-likelihood path.

This module builds the *inputs* of the likelihood: detector descriptors,
leading-order chirp harmonics h_lm(f), Gaussian noise, the data d_k, and the
precomputed overlaps Q_k,lm(tau), U_k and V_k of eq. (QUV).  It also draws
extrinsic samples from the prior with numpy's generator (random numbers the
method would draw, handed in as inputs).

It holds none of the likelihood arithmetic itself: no antenna pattern, no
spin-weighted harmonic, no interpolation, no quadratic form, no reduction.
The injected signal is assembled from per-detector projection numbers
(F+, Fx, arrival-time offset and the complex harmonic weights) that the
caller supplies; the stored injections under ``tests/golden`` were written
by a script that calls only the oracle.

Conventions (paper, Section "Review of the RIFT likelihood"):
  * complex strain h = h+ - i hx, h = (D_ref/D) sum_lm h_lm Y_lm;
  * detector strain h_k = F+ h+ + Fx hx, delayed to the detector time;
  * <a|b> = 2 sum_f df conj(a~) b~ / S(|f|) over f_low <= |f| <= f_high.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 250511655
C_SI = 299792458.0
MSUN_S = 4.925490947641267e-06          # G Msun / c^3 in seconds
D_REF_MPC = 100.0

FS = 4096.0                             # sample rate (Hz)
SEG_S = 4.0                             # segment length (s)
F_LO, F_HI = 20.0, 1024.0               # band (Hz)
N_WIN = 410                             # Q window samples
WIN_HALF = 205                          # tau_i = (i - 205)/fs
T_WINDOW = 0.028                        # geocentric time prior half-width (s)
D_MIN, D_MAX = 1.0, 3000.0              # distance prior (Mpc)

# Approximate public site values: geodetic latitude, longitude (deg), arm
# azimuths (deg, clockwise from local North).  Placed on WGS-84 at h = 0.
SITES = {
    "H": (46.455, -119.408, 324.0, 234.0),
    "L": (30.563, -90.774, 252.3, 162.3),
    "V": (43.631, 10.504, 19.4, 289.4),
}
WGS84_A = 6378137.0
WGS84_F = 1.0 / 298.257223563


def detector(name: str):
    """Earth-fixed position (m) and response tensor D = (a a^T - b b^T)/2."""
    lat, lon, az_a, az_b = SITES[name]
    p, l = math.radians(lat), math.radians(lon)
    e2 = WGS84_F * (2.0 - WGS84_F)
    n_curv = WGS84_A / math.sqrt(1.0 - e2 * math.sin(p) ** 2)
    pos = np.array([n_curv * math.cos(p) * math.cos(l),
                    n_curv * math.cos(p) * math.sin(l),
                    n_curv * (1.0 - e2) * math.sin(p)])
    east = np.array([-math.sin(l), math.cos(l), 0.0])
    north = np.array([-math.sin(p) * math.cos(l), -math.sin(p) * math.sin(l), math.cos(p)])

    def arm(az):
        a = math.radians(az)
        return math.cos(a) * north + math.sin(a) * east

    a, b = arm(az_a), arm(az_b)
    resp = 0.5 * (np.outer(a, a) - np.outer(b, b))
    return pos, resp


def detectors(names):
    pos = np.stack([detector(n)[0] for n in names])
    resp = np.stack([detector(n)[1] for n in names])
    return pos, resp


# ---------------------------------------------------------------- mode sets
def mode_set(n: int):
    """Mode lists used by the workloads (l <= 4).

    5  = l=2 all m;  9 = 5 + (3,+-3),(3,+-2);
    17 = l=2 all, l=3 m != 0, l=4 |m| >= 2;  21 = every (l,m) with l <= 4.
    """
    l2 = [(2, m) for m in range(-2, 3)]
    if n == 5:
        return l2
    if n == 9:
        return l2 + [(3, -3), (3, -2), (3, 2), (3, 3)]
    if n == 17:
        return l2 + [(3, m) for m in (-3, -2, -1, 1, 2, 3)] + [(4, m) for m in (-4, -3, -2, 2, 3, 4)]
    if n == 21:
        return [(l, m) for l in (2, 3, 4) for m in range(-l, l + 1)]
    raise ValueError(f"no mode set of size {n}")


def mode_amplitude(l: int, m: int, q: float) -> float:
    """Synthetic relative harmonic amplitudes (q = m1/m2 >= 1)."""
    d = (q - 1.0) / (q + 1.0)
    eta = q / (1.0 + q) ** 2
    am = abs(m)
    table = {
        (2, 2): 1.0, (2, 1): 0.3 * d, (2, 0): 0.05,
        (3, 3): 0.4 * d, (3, 2): 0.1 * (1 - 3 * eta), (3, 1): 0.05 * d, (3, 0): 0.02,
        (4, 4): 0.15 * (1 - 3 * eta), (4, 3): 0.05 * d, (4, 2): 0.03 * (1 - 3 * eta),
        (4, 1): 0.02 * d, (4, 0): 0.01,
    }
    return table[(l, am)]


def freq_grid(fs: float = FS, seg: float = SEG_S):
    n = int(round(fs * seg))
    f = np.fft.fftfreq(n, d=1.0 / fs)
    return f, 1.0 / seg


def _psi22(f, mc_s):
    return -math.pi / 4.0 + (3.0 / 128.0) * (math.pi * mc_s * f) ** (-5.0 / 3.0)


def modes_fd(f, modes, mc_msun, q, amp0=1.0):
    """h~_lm(f) on the FFT grid (zero outside the band).

    m > 0 modes live at f < 0 with phase +Psi_m(|f|); m < 0 modes follow from
    h_{l,-m}(t) = (-1)^l conj(h_lm(t)); m = 0 modes are real in time.
    Psi_m(f) = (m/2) Psi_22(2f/m) (leading-order stationary phase, t_c = 0).
    """
    mc_s = mc_msun * MSUN_S
    af = np.abs(f)
    band = (af >= F_LO) & (af <= F_HI)
    afb = np.where(band, af, 1.0)
    out = np.zeros((len(modes), len(f)), dtype=np.complex128)
    for a, (l, m) in enumerate(modes):
        amp = amp0 * mode_amplitude(l, m, q) * mc_s ** (5.0 / 6.0) * afb ** (-7.0 / 6.0)
        mm = abs(m) if m != 0 else 2
        phase = (mm / 2.0) * _psi22(2.0 * afb / mm, mc_s)
        neg = band & (f < 0)
        pos = band & (f > 0)
        if m > 0:
            out[a, neg] = amp[neg] * np.exp(1j * phase[neg])
        elif m < 0:
            out[a, pos] = (-1) ** l * amp[pos] * np.exp(-1j * phase[pos])
        else:
            out[a, neg] = amp[neg] * np.exp(1j * phase[neg])
            out[a, pos] = amp[pos] * np.exp(-1j * phase[pos])
    return out


def _reverse(x):
    """x(-f) on the FFT index grid."""
    return np.roll(x[..., ::-1], 1, axis=-1)


def project_strain(f, hlm, coeff_Y, fplus, fcross, dt_arrival, s_inj):
    """Detector strain h~_k(f) from the definitions, for given projection numbers.

    H(f) = s_inj * sum_lm Y_lm h~_lm(f) is the complex strain h+ - i hx;
    h_k(t) = F+ Re h(t - dt) - Fx Im h(t - dt).
    """
    H = s_inj * np.tensordot(coeff_Y, hlm, axes=(0, 0))
    Hr = _reverse(H)
    re_part = 0.5 * (H + np.conj(Hr))
    im_part = (H - np.conj(Hr)) / 2j
    out = []
    for Fp, Fx, dt in zip(fplus, fcross, dt_arrival):
        out.append(np.exp(-2j * np.pi * f * dt) * (Fp * re_part - Fx * im_part))
    return np.stack(out)


def network_snr2(f, df, hk, psd=1.0):
    """rho^2 = sum_k 4 sum_{f>0} |h~_k|^2 df / S, from the detector strains alone."""
    band = (f >= F_LO) & (f <= F_HI)
    return float(np.sum(4.0 * np.abs(hk[:, band]) ** 2 * df / psd))


def white_noise(rng, f, df, n_det, psd=1.0):
    """Hermitian white noise with Re, Im ~ N(0, S/(4 df)) at f > 0."""
    n = len(f)
    sig = math.sqrt(psd / (4.0 * df))
    out = np.zeros((n_det, n), dtype=np.complex128)
    pos = np.where(f > 0)[0]
    for k in range(n_det):
        z = rng.normal(0.0, sig, size=len(pos)) + 1j * rng.normal(0.0, sig, size=len(pos))
        out[k, pos] = z
        out[k, (n - pos) % n] = np.conj(z)
    return out


def overlaps(f, df, hlm, data, psd=1.0, n_win=N_WIN, win_half=WIN_HALF):
    """Q_k,lm(tau_i), U_k, V_k of eq. (QUV) by FFT, band-limited, flat PSD.

    Q[k][a][i] at tau_i = (i - win_half)/fs;  U[k][a][b] = <h_a|h_b>;
    V[k][a][b] = <h_a^*|h_b>.
    """
    n = len(f)
    nd = data.shape[0]
    na = hlm.shape[0]
    band = ((np.abs(f) >= F_LO) & (np.abs(f) <= F_HI)).astype(float)
    Q = np.empty((nd, na, n_win), dtype=np.complex128)
    idx = (np.arange(n_win) - win_half) % n
    for k in range(nd):
        x = 2.0 * np.conj(hlm) * data[k][None, :] * band / psd
        q = np.fft.ifft(x, axis=-1) * n * df
        Q[k] = q[:, idx]
    hb = hlm * band
    U1 = 2.0 * df * (np.conj(hb) @ hb.T) / psd
    V1 = 2.0 * df * (_reverse(hb) @ hb.T) / psd
    U = np.broadcast_to(U1, (nd, na, na)).copy()
    V = np.broadcast_to(V1, (nd, na, na)).copy()
    return Q, U, V


# ------------------------------------------------------------ injections
_INJ_FILE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                         "tests", "golden", "injections.json")


def load_injections(path: str = _INJ_FILE):
    """Projection numbers of the stored injections (written by the oracle)."""
    with open(path) as fh:
        return json.load(fh)


def injection_theta(rng, iota=None, t_half=0.005):
    """Seeded injection parameters (alpha, dec, t, D, cos iota, phi_c, psi)."""
    alpha = rng.uniform(0, 2 * math.pi)
    dec = math.asin(rng.uniform(-1, 1))
    t = rng.uniform(-t_half, t_half)
    D = 400.0
    ci = math.cos(iota) if iota is not None else rng.uniform(-1, 1)
    phi = rng.uniform(0, 2 * math.pi)
    psi = rng.uniform(0, math.pi)
    return [alpha, dec, t, D, ci, phi, psi]


# ------------------------------------------------------------ problems
@dataclass
class Problem:
    """One intrinsic point: the host-side inputs of ile_prepare."""
    modes: list
    det_names: list
    det_pos: np.ndarray
    det_resp: np.ndarray
    gmst: float
    Q: np.ndarray          # [K][n][T] complex128
    U: np.ndarray          # [K][n][n] complex128
    V: np.ndarray          # [K][n][n] complex128
    tau0: float = -WIN_HALF / FS
    dt: float = 1.0 / FS
    d_ref: float = D_REF_MPC
    t_window: float = T_WINDOW
    d_min: float = D_MIN
    d_max: float = D_MAX
    meta: dict = field(default_factory=dict)

    @property
    def n_det(self):
        return len(self.det_names)

    @property
    def n_modes(self):
        return len(self.modes)


def _inj_projection(rec, det_names, modes):
    fp = [rec["det"][d]["Fp"] for d in det_names]
    fx = [rec["det"][d]["Fx"] for d in det_names]
    dtk = [rec["theta"][2] - rec["det"][d]["delay"] for d in det_names]
    yl = {tuple(int(v) for v in key.split(",")): complex(*val) for key, val in rec["Y"].items()}
    coeffY = np.array([yl[lm] for lm in modes])
    return fp, fx, dtk, coeffY


def build_event(rec, det_names, n_modes, mc, q, snr, noise_seed, templates=None,
                noise=True):
    """Data for one injection record and the overlaps of one or more templates.

    The injection uses (mc, q) and is scaled so the noiseless network SNR is
    exactly ``snr``.  ``templates`` is a list of (mc, q) (default: the
    injected one); returns one Problem per template, all against the same data.
    """
    modes = mode_set(n_modes)
    f, df = freq_grid()
    pos, resp = detectors(det_names)
    inj_modes = mode_set(21)
    h_inj = modes_fd(f, inj_modes, mc, q)
    fp, fx, dtk, coeffY = _inj_projection(rec, det_names, inj_modes)
    s_inj = D_REF_MPC / rec["theta"][3]
    # restrict the injection to the analysed harmonics so lnL(theta_inj) = rho^2/2
    keep = np.array([lm in modes for lm in inj_modes], dtype=float)
    hk = project_strain(f, h_inj * keep[:, None], coeffY, fp, fx, dtk, s_inj)
    rho2 = network_snr2(f, df, hk)
    amp0 = snr / math.sqrt(rho2)
    hk = hk * amp0
    data = hk.copy()
    if noise:
        rng = np.random.default_rng(noise_seed)
        data = data + white_noise(rng, f, df, len(det_names))
    out = []
    for (tmc, tq) in (templates or [(mc, q)]):
        hlm = modes_fd(f, modes, tmc, tq, amp0=amp0)
        Q, U, V = overlaps(f, df, hlm, data)
        out.append(Problem(modes=modes, det_names=list(det_names), det_pos=pos, det_resp=resp,
                           gmst=rec["gmst"], Q=Q, U=U, V=V,
                           meta={"theta_inj": list(rec["theta"]), "snr": snr, "mc": tmc, "q": tq,
                                 "amp0": amp0, "inj_mc": mc, "inj_q": q}))
    return out, dict(f=f, df=df, data=data, strain=hk, amp0=amp0)


def prior_samples(rng, n, t_window=T_WINDOW, d_min=D_MIN, d_max=D_MAX, dtype=np.float64):
    """Extrinsic samples [7][n] from the prior, drawn with numpy's generator."""
    th = np.empty((7, n), dtype=np.float64)
    th[0] = rng.uniform(0, 2 * math.pi, n)
    th[1] = np.arcsin(rng.uniform(-1, 1, n))
    th[2] = rng.uniform(-t_window, t_window, n)
    th[3] = np.cbrt(rng.uniform(d_min ** 3, d_max ** 3, n))
    th[4] = rng.uniform(-1, 1, n)
    th[5] = rng.uniform(0, 2 * math.pi, n)
    th[6] = rng.uniform(0, math.pi, n)
    return np.ascontiguousarray(th.astype(dtype))


def box_samples(rng, n, theta_c, widths, t_window=T_WINDOW, d_min=D_MIN, d_max=D_MAX,
                dtype=np.float64):
    """Samples uniform in a box around theta_c, clipped to the support."""
    th = np.empty((7, n), dtype=np.float64)
    for c in range(7):
        th[c] = theta_c[c] + rng.uniform(-1, 1, n) * widths[c]
    th[0] %= 2 * math.pi
    th[1] = np.clip(th[1], -math.pi / 2, math.pi / 2)
    th[2] = np.clip(th[2], -t_window, t_window)
    th[3] = np.clip(th[3], d_min, d_max)
    th[4] = np.clip(th[4], -1, 1)
    th[5] %= 2 * math.pi
    th[6] %= math.pi
    return np.ascontiguousarray(th.astype(dtype))


def random_problem(rng, n_modes, det_names, q=2.0, gmst=None):
    """Valid but non-physical inputs: random Q windows and random Gram U, V.

    U is built as a Gram matrix (Hermitian PSD) and V as a complex symmetric
    matrix; used for fast parity cases that need no waveform.
    """
    modes = mode_set(n_modes)
    K, n = len(det_names), len(modes)
    pos, resp = detectors(det_names)
    Q = (rng.normal(size=(K, n, N_WIN)) + 1j * rng.normal(size=(K, n, N_WIN))) * 5.0
    A = rng.normal(size=(K, n, 2 * n)) + 1j * rng.normal(size=(K, n, 2 * n))
    U = np.einsum("kai,kbi->kab", np.conj(A), A) * 2.0
    B = rng.normal(size=(K, n, n)) + 1j * rng.normal(size=(K, n, n))
    V = 0.3 * (B + np.transpose(B, (0, 2, 1)))
    g = rng.uniform(0, 2 * math.pi) if gmst is None else gmst
    return Problem(modes=modes, det_names=list(det_names), det_pos=pos, det_resp=resp,
                   gmst=g, Q=Q, U=U, V=V, meta={"random": True})
