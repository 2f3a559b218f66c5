"""Python binding of libile.so, the gfx950 ILE extrinsic-likelihood library.

Argument marshalling only: every step of the likelihood path runs in the HIP
kernels behind the C ABI of ``include/ile.h``.  Functions keep the C names.
Device buffers are passed as integers (``tensor.data_ptr()``) or torch
tensors; streams as ``torch.cuda.Stream`` / raw handles / None (null stream).
Loading fails loudly if the library has not been built
(``python -m paper_2505_11655_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libile.so")

ILE_FP64, ILE_FP32, ILE_FP32_CANCEL64 = 0, 1, 2
ILE_MARG_RESET, ILE_MARG_POOL = 1, 2
STATUS = {0: "OK", 1: "PENDING", -1: "E_INVALID", -2: "E_NOMEM", -3: "E_TOO_BIG", -4: "E_DEVICE",
          -5: "E_STATE", -6: "E_CANCELLED", -7: "E_TIMEOUT"}


class IleError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"ile status {status} ({STATUS.get(status, '?')}): {msg}")
        self.status = status


class ile_prior(C.Structure):
    _fields_ = [("t_window", C.c_double), ("d_min", C.c_double), ("d_max", C.c_double),
                ("dist_marg", C.c_int32)]


class ile_problem(C.Structure):
    _fields_ = [("n_det", C.c_int32), ("n_modes", C.c_int32), ("n_time", C.c_int32), ("mem_is_device", C.c_int32),
                ("mode_l", C.POINTER(C.c_int32)), ("mode_m", C.POINTER(C.c_int32)),
                ("det_pos", C.POINTER(C.c_double)), ("det_resp", C.POINTER(C.c_double)),
                ("gmst_rad", C.c_double), ("tau0_s", C.c_double), ("dt_s", C.c_double),
                ("Q", C.POINTER(C.c_double)), ("U", C.POINTER(C.c_double)), ("V", C.POINTER(C.c_double)),
                ("d_ref_mpc", C.c_double), ("mode_filter_eps", C.c_double), ("precision", C.c_int32),
                ("prior", ile_prior)]


class ile_marg(C.Structure):
    _fields_ = [("ln_L", C.c_double), ("ln_sigma", C.c_double), ("n_eff", C.c_double),
                ("n_ess", C.c_double), ("max_lw", C.c_double), ("argmax", C.c_int64),
                ("n", C.c_int64), ("n_nonfinite", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ile_job_info(C.Structure):
    _fields_ = [("n_modes_kept", C.c_int32), ("mode_slots", C.c_int32), ("n_det_slots", C.c_int32),
                ("device_bytes", C.c_size_t)]


MAXC = 16


class ile_gmm_params(C.Structure):
    _fields_ = [("n_comp", C.c_int32), ("n_dim", C.c_int32), ("dims", C.c_int32 * 7),
                ("eps_def", C.c_double), ("weight", C.c_double * MAXC),
                ("mean", (C.c_double * 7) * MAXC), ("cov", ((C.c_double * 7) * 7) * MAXC),
                ("ln_Z", C.c_double * MAXC), ("shear", C.c_int32)]


class ile_gmm_opts(C.Structure):
    _fields_ = [("n_comp", C.c_int32), ("n_iter", C.c_int32), ("eps_def", C.c_double),
                ("seed", C.c_uint64), ("round", C.c_uint32), ("z_draws", C.c_int64),
                ("temper_ess", C.c_double), ("phase_shear", C.c_int32)]


class ile_server_opts(C.Structure):
    _fields_ = [("max_active", C.c_int32), ("hbm_budget_bytes", C.c_size_t),
                ("chunk_samples", C.c_int64), ("record_samples", C.c_int32)]


class ile_job_opts(C.Structure):
    _fields_ = [("n_samples", C.c_int64), ("adaptive", C.c_int32), ("round_samples", C.c_int64),
                ("max_rounds", C.c_int32), ("n_eff_target", C.c_double), ("seed", C.c_uint64),
                ("tmarg_oversample", C.c_int32), ("integrator", C.c_int32), ("pool", C.c_int32),
                ("phase_shear", C.c_int32)]


ILE_INT_GMM, ILE_INT_AV, ILE_INT_AC = 0, 1, 2
ILE_POOL_ROUNDS, ILE_POOL_MIXTURE = 0, 1
ILE_QV_AUTO, ILE_QV_DIRECT, ILE_QV_DECIMATED = 0, 1, 2
AC_BINS = 64


class ile_qv_shape(C.Structure):
    _fields_ = [("n_points", C.c_int32), ("n_modes", C.c_int32), ("n_det", C.c_int32), ("n_freq", C.c_int64),
                ("df", C.c_double), ("f_lo", C.c_double), ("f_hi", C.c_double), ("n_time", C.c_int32),
                ("win_half", C.c_int32), ("route", C.c_int32)]


class ile_av_opts(C.Structure):
    _fields_ = [("p_thr", C.c_double), ("n_min_live", C.c_int64), ("max_bins", C.c_int32)]


class ile_av_state(C.Structure):
    _fields_ = [("n_dim", C.c_int32), ("dims", C.c_int32 * 7), ("n_bins", C.c_int32), ("n_cells", C.c_int64),
                ("ln_vol", C.c_double), ("lnL_thr", C.c_double), ("n_min", C.c_int64), ("n_live", C.c_int64),
                ("vol_mc", C.c_double)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "dims"}
        d["dims"] = [self.dims[k] for k in range(self.n_dim)]
        return d


class ile_result(C.Structure):
    _fields_ = [("marg", ile_marg), ("status", C.c_int32), ("rounds", C.c_int32), ("samples", C.c_int64),
                ("t_arrival_ns", C.c_int64), ("t_admit_ns", C.c_int64), ("t_start_ns", C.c_int64),
                ("t_finish_ns", C.c_int64)]


EXPORTS = {
    # name: (restype, argtypes)
    "ile_ctx_create": (C.c_int, [C.c_int, C.c_size_t, C.POINTER(C.c_void_p)]),
    "ile_ctx_destroy": (None, [C.c_void_p]),
    "ile_last_error": (C.c_char_p, []),
    "ile_prepare": (C.c_int, [C.c_void_p, C.POINTER(ile_problem), C.POINTER(C.c_void_p)]),
    "ile_job_info_get": (C.c_int, [C.c_void_p, C.POINTER(ile_job_info)]),
    "ile_job_release": (None, [C.c_void_p]),
    "ile_eval_lnL": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_void_p]),
    "ile_eval_lnL_batch": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_int64),
                                     C.POINTER(C.c_void_p), C.POINTER(C.c_int64), C.POINTER(C.c_void_p),
                                     C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_void_p]),
    "ile_eval_lnL_tmarg": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_int32, C.c_void_p]),
    "ile_eval_lnL_tmarg_batch": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_int64),
                                           C.POINTER(C.c_void_p), C.POINTER(C.c_int64), C.POINTER(C.c_void_p),
                                           C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_int32, C.c_void_p]),
    "ile_set_reference": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_void_p]),
    "ile_marginalize": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_uint32, C.POINTER(ile_marg),
                                  C.c_void_p]),
    "ile_marginalize_noalloc": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_uint32, C.POINTER(ile_marg),
                                          C.c_void_p]),
    "ile_marginalize_noalloc_max": (C.c_size_t, []),
    "ile_marginalize_batch": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_int64),
                                        C.POINTER(C.c_void_p), C.c_uint32, C.POINTER(ile_marg), C.c_void_p]),
    "ile_draw": (C.c_int, [C.c_void_p, C.c_uint64, C.c_uint32, C.c_int64, C.c_int64, C.c_void_p, C.c_int64,
                           C.c_void_p, C.c_void_p]),
    "ile_set_proposal": (C.c_int, [C.c_void_p, C.POINTER(ile_gmm_params), C.POINTER(ile_gmm_opts),
                                   C.c_void_p]),
    "ile_get_proposal": (C.c_int, [C.c_void_p, C.POINTER(ile_gmm_params), C.c_void_p]),
    "ile_adapt_proposal": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                     C.POINTER(ile_gmm_opts), C.POINTER(ile_gmm_params), C.c_void_p]),
    "ile_av_reset": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.c_void_p]),
    "ile_av_draw": (C.c_int, [C.c_void_p, C.c_uint64, C.c_uint32, C.c_int64, C.c_int64, C.c_void_p, C.c_int64,
                              C.c_void_p, C.c_void_p]),
    "ile_av_update": (C.c_int, [C.c_void_p, C.c_uint64, C.c_uint32, C.c_int64, C.c_int64, C.c_void_p,
                                C.POINTER(ile_av_opts), C.POINTER(ile_av_state), C.c_void_p]),
    "ile_av_get": (C.c_int, [C.c_void_p, C.POINTER(ile_av_state), C.POINTER(C.c_int32), C.c_int64,
                             C.c_void_p]),
    "ile_ac_reset": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.c_void_p]),
    "ile_ac_draw": (C.c_int, [C.c_void_p, C.c_uint64, C.c_uint32, C.c_int64, C.c_int64, C.c_void_p, C.c_int64,
                              C.c_void_p, C.c_void_p]),
    "ile_ac_update": (C.c_int, [C.c_void_p, C.c_uint64, C.c_uint32, C.c_int64, C.c_int64, C.c_void_p, C.c_double,
                                C.c_void_p]),
    "ile_ac_get": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_double),
                             C.c_void_p]),
    "ile_overlaps": (C.c_int, [C.c_void_p, C.POINTER(ile_qv_shape), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_void_p, C.c_void_p]),
    "ile_fair_draw": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_uint64, C.c_uint32, C.c_int64, C.c_void_p,
                                C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p]),
    "ile_server_create": (C.c_int, [C.c_void_p, C.POINTER(ile_server_opts), C.POINTER(C.c_void_p)]),
    "ile_server_submit": (C.c_int, [C.c_void_p, C.POINTER(ile_problem), C.POINTER(ile_job_opts),
                                    C.POINTER(C.c_uint64)]),
    "ile_server_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(ile_result)]),
    "ile_server_wait": (C.c_int, [C.c_void_p, C.c_uint64, C.c_int64, C.POINTER(ile_result)]),
    "ile_server_cancel": (C.c_int, [C.c_void_p, C.c_uint64]),
    "ile_server_stats": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                   C.POINTER(C.c_int64)]),
    "ile_server_destroy": (None, [C.c_void_p]),
}

_lib = None


def lib():
    """Load libile.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libile.so not built ({LIB_PATH}); run python -m paper_2505_11655_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            if not hasattr(L, name):
                continue
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _chk(status):
    if status < 0:
        raise IleError(status, (lib().ile_last_error() or b"").decode())
    return status


def _p(x):
    """Device pointer of a torch tensor / int / None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _s(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ------------------------------------------------------------------ context
def ile_ctx_create(device=0, hbm_budget_bytes=0):
    h = C.c_void_p()
    _chk(lib().ile_ctx_create(device, hbm_budget_bytes, C.byref(h)))
    return h


def ile_ctx_destroy(ctx):
    lib().ile_ctx_destroy(ctx)


def ile_last_error():
    return (lib().ile_last_error() or b"").decode()


# ------------------------------------------------------------------ problems
class ProblemHost:
    """An ile_problem with the host arrays it points to kept alive."""

    def __init__(self, prob, precision=ILE_FP64, dist_marg=False, mode_filter_eps=0.0):
        self.ml = np.ascontiguousarray([l for l, _ in prob.modes], dtype=np.int32)
        self.mm = np.ascontiguousarray([m for _, m in prob.modes], dtype=np.int32)
        self.pos = np.ascontiguousarray(prob.det_pos, dtype=np.float64)
        self.resp = np.ascontiguousarray(prob.det_resp, dtype=np.float64)
        self.Q = np.ascontiguousarray(np.asarray(prob.Q, dtype=np.complex128)).view(np.float64)
        self.U = np.ascontiguousarray(np.asarray(prob.U, dtype=np.complex128)).view(np.float64)
        self.V = None if prob.V is None else np.ascontiguousarray(
            np.asarray(prob.V, dtype=np.complex128)).view(np.float64)
        ip, dp = C.POINTER(C.c_int32), C.POINTER(C.c_double)
        self.s = ile_problem(
            len(prob.det_pos), len(prob.modes), prob.Q.shape[-1], 0,
            self.ml.ctypes.data_as(ip), self.mm.ctypes.data_as(ip),
            self.pos.ctypes.data_as(dp), self.resp.ctypes.data_as(dp),
            prob.gmst, prob.tau0, prob.dt,
            self.Q.ctypes.data_as(dp), self.U.ctypes.data_as(dp),
            self.V.ctypes.data_as(dp) if self.V is not None else dp(),
            prob.d_ref, mode_filter_eps, precision,
            ile_prior(prob.t_window, prob.d_min, prob.d_max, int(dist_marg)))


def _problem_struct(problem):
    """A ProblemHost's ile_problem, or an ile_problem given directly (e.g. one
    whose arrays are device memory, mem_is_device = 1)."""
    return problem.s if isinstance(problem, ProblemHost) else problem


def ile_prepare(ctx, problem):
    h = C.c_void_p()
    _chk(lib().ile_prepare(ctx, C.byref(_problem_struct(problem)), C.byref(h)))
    return h


def ile_job_info_get(job):
    info = ile_job_info()
    _chk(lib().ile_job_info_get(job, C.byref(info)))
    return info


def ile_job_release(job):
    lib().ile_job_release(job)


# ------------------------------------------------------------------ compute
def ile_eval_lnL(job, n, theta, ld, lnpmps, lnL_out, lw_out=None, stream=None):
    _chk(lib().ile_eval_lnL(job, n, _p(theta), ld, _p(lnpmps), _p(lnL_out), _p(lw_out), _s(stream)))


def ile_eval_lnL_batch(jobs, n, theta, ld, lnpmps, lnL_out, lw_out=None, stream=None):
    k = len(jobs)
    VP = C.c_void_p * k
    I64 = C.c_int64 * k
    _chk(lib().ile_eval_lnL_batch(
        VP(*[j.value if isinstance(j, C.c_void_p) else j for j in jobs]), k, I64(*n),
        VP(*[_p(t) for t in theta]), I64(*ld),
        VP(*[_p(t) for t in lnpmps]) if lnpmps is not None else None,
        VP(*[_p(t) for t in lnL_out]),
        VP(*[_p(t) for t in lw_out]) if lw_out is not None else None, _s(stream)))


def ile_eval_lnL_tmarg(job, n, theta, ld, lnpmps, lnL_out, lw_out=None, oversample=4, stream=None):
    _chk(lib().ile_eval_lnL_tmarg(job, n, _p(theta), ld, _p(lnpmps), _p(lnL_out), _p(lw_out), oversample,
                                  _s(stream)))


def ile_eval_lnL_tmarg_batch(jobs, n, theta, ld, lnpmps, lnL_out, lw_out=None, oversample=4, stream=None):
    k = len(jobs)
    VP = C.c_void_p * k
    I64 = C.c_int64 * k
    _chk(lib().ile_eval_lnL_tmarg_batch(
        VP(*[j.value if isinstance(j, C.c_void_p) else j for j in jobs]), k, I64(*n),
        VP(*[_p(t) for t in theta]), I64(*ld),
        VP(*[_p(t) for t in lnpmps]) if lnpmps is not None else None,
        VP(*[_p(t) for t in lnL_out]),
        VP(*[_p(t) for t in lw_out]) if lw_out is not None else None, oversample, _s(stream)))


def ile_set_reference(job, theta_ref, stream=None):
    t = (C.c_double * 7)(*[float(v) for v in theta_ref])
    _chk(lib().ile_set_reference(job, t, _s(stream)))


def ile_marginalize(job, n, lw, flags=ILE_MARG_RESET, want=True, stream=None):
    out = ile_marg() if want else None
    _chk(lib().ile_marginalize(job, n, _p(lw), flags, C.byref(out) if out is not None else None, _s(stream)))
    return out.as_dict() if out is not None else None


def ile_marginalize_noalloc(job, n, lw, flags=ILE_MARG_RESET, want=True, stream=None):
    out = ile_marg() if want else None
    _chk(lib().ile_marginalize_noalloc(job, n, _p(lw), flags, C.byref(out) if out is not None else None,
                                       _s(stream)))
    return out.as_dict() if out is not None else None


def ile_marginalize_noalloc_max():
    return int(lib().ile_marginalize_noalloc_max())


def ile_marginalize_batch(jobs, n, lw, flags=ILE_MARG_RESET, want=True, stream=None):
    k = len(jobs)
    VP = C.c_void_p * k
    out = (ile_marg * k)() if want else None
    _chk(lib().ile_marginalize_batch(
        VP(*[j.value if isinstance(j, C.c_void_p) else j for j in jobs]), k, (C.c_int64 * k)(*n),
        VP(*[_p(t) for t in lw]), flags, out, _s(stream)))
    return [o.as_dict() for o in out] if want else None


def ile_draw(job, seed, rnd, first_index, n, theta_out, ld, lnpmps_out=None, stream=None):
    _chk(lib().ile_draw(job, seed, rnd, first_index, n, _p(theta_out), ld, _p(lnpmps_out), _s(stream)))


def gmm_params(weights, means, covs, eps_def=0.05, shear=0):
    p = ile_gmm_params()
    p.n_comp = len(weights)
    p.eps_def = eps_def
    p.shear = int(shear)
    for j in range(len(weights)):
        p.weight[j] = float(weights[j])
        d = len(means[j])
        for a in range(d):
            p.mean[j][a] = float(means[j][a])
            for b in range(d):
                p.cov[j][a][b] = float(covs[j][a][b])
    return p


def gmm_opts(n_comp=8, n_iter=8, eps_def=0.05, seed=0x243F6A8885A308D3, rnd=0, z_draws=65536, temper_ess=0.0,
             phase_shear=0):
    return ile_gmm_opts(n_comp, n_iter, eps_def, seed, rnd, z_draws, temper_ess, int(phase_shear))


def ile_set_proposal(job, params, opts=None, stream=None):
    _chk(lib().ile_set_proposal(job, C.byref(params), C.byref(opts) if opts is not None else None, _s(stream)))


def ile_get_proposal(job, stream=None):
    p = ile_gmm_params()
    _chk(lib().ile_get_proposal(job, C.byref(p), _s(stream)))
    return p


def ile_adapt_proposal(job, n, theta, ld, lw, opts=None, want=True, stream=None):
    p = ile_gmm_params() if want else None
    _chk(lib().ile_adapt_proposal(job, n, _p(theta), ld, _p(lw), C.byref(opts) if opts is not None else None,
                                  C.byref(p) if p is not None else None, _s(stream)))
    return p


# ---------------------------------------------------------- adaptive volume
def av_opts(p_thr=0.999, n_min_live=1000, max_bins=511):
    return ile_av_opts(p_thr, n_min_live, max_bins)


def ile_av_reset(job, dims=None, stream=None):
    if dims is None:
        _chk(lib().ile_av_reset(job, 0, None, _s(stream)))
    else:
        arr = (C.c_int32 * max(len(dims), 1))(*dims)
        _chk(lib().ile_av_reset(job, len(dims), arr, _s(stream)))


def ile_av_draw(job, seed, rnd, first_index, n, theta_out, ld, lnpmps_out=None, stream=None):
    _chk(lib().ile_av_draw(job, seed, rnd, first_index, n, _p(theta_out), ld, _p(lnpmps_out), _s(stream)))


def ile_av_update(job, seed, rnd, first_index, n, lw, opts=None, want=True, stream=None):
    out = ile_av_state() if want else None
    _chk(lib().ile_av_update(job, seed, rnd, first_index, n, _p(lw), C.byref(opts) if opts is not None else None,
                             C.byref(out) if out is not None else None, _s(stream)))
    return out.as_dict() if out is not None else None


def ile_av_get(job, cells=True, stream=None):
    """(state dict, cells [n_cells][n_dim] int32 numpy array or None)."""
    import numpy as np
    st = ile_av_state()
    _chk(lib().ile_av_get(job, C.byref(st), None, 0, _s(stream)))
    if not cells:
        return st.as_dict(), None
    arr = np.zeros((max(st.n_cells, 1), max(st.n_dim, 1)), dtype=np.int32)
    _chk(lib().ile_av_get(job, C.byref(st), arr.ctypes.data_as(C.POINTER(C.c_int32)), st.n_cells, _s(stream)))
    return st.as_dict(), arr[:st.n_cells, :st.n_dim]


def ile_ac_reset(job, dims=None, stream=None):
    if dims is None:
        _chk(lib().ile_ac_reset(job, 0, None, _s(stream)))
    else:
        arr = (C.c_int32 * max(len(dims), 1))(*dims)
        _chk(lib().ile_ac_reset(job, len(dims), arr, _s(stream)))


def ile_ac_draw(job, seed, rnd, first_index, n, theta_out, ld, lnpmps_out=None, stream=None):
    _chk(lib().ile_ac_draw(job, seed, rnd, first_index, n, _p(theta_out), ld, _p(lnpmps_out), _s(stream)))


def ile_ac_update(job, seed, rnd, first_index, n, lw, floor=0.1, stream=None):
    _chk(lib().ile_ac_update(job, seed, rnd, first_index, n, _p(lw), floor, _s(stream)))


def ile_ac_get(job, stream=None):
    """(dims list, pi [n_dim][64] numpy array)."""
    import numpy as np
    nd = C.c_int32()
    dims = (C.c_int32 * 7)()
    pi = np.zeros((7, AC_BINS))
    _chk(lib().ile_ac_get(job, C.byref(nd), dims, pi.ctypes.data_as(C.POINTER(C.c_double)), _s(stream)))
    return [dims[k] for k in range(nd.value)], pi[:nd.value]


def ile_overlaps(ctx, hlm, data, df, f_lo, f_hi, n_time, win_half, Q, U, V, inv_psd=None, stream=None,
                 route=0):
    """hlm: device [n_points][n_modes][n] complex128 (a 2-D [n_modes][n] array is one point);
    route: ILE_QV_AUTO, ILE_QV_DIRECT or ILE_QV_DECIMATED."""
    n_points, n_modes, n = (1,) + tuple(hlm.shape) if hlm.dim() == 2 else tuple(hlm.shape)
    sh = ile_qv_shape(n_points, n_modes, data.shape[0], n, df, f_lo, f_hi, n_time, win_half, route)
    _chk(lib().ile_overlaps(ctx, C.byref(sh), _p(hlm), _p(data), _p(inv_psd), _p(Q), _p(U), _p(V), _s(stream)))


def ile_fair_draw(job, n, lw, seed, rnd, k, idx_out=None, theta=None, ld=0, theta_out=None, ld_out=0, stream=None):
    _chk(lib().ile_fair_draw(job, n, _p(lw), seed, rnd, k, _p(idx_out), _p(theta), ld, _p(theta_out), ld_out,
                             _s(stream)))


# ------------------------------------------------------------------ serving
def ile_server_create(ctx, max_active=64, hbm_budget_bytes=0, chunk_samples=1 << 20):
    h = C.c_void_p()
    o = ile_server_opts(max_active, hbm_budget_bytes, chunk_samples, 0)
    _chk(lib().ile_server_create(ctx, C.byref(o), C.byref(h)))
    return h


def job_opts(n_samples=1 << 16, adaptive=False, round_samples=1 << 16, max_rounds=32, n_eff_target=1000.0,
             seed=1, tmarg_oversample=0, integrator=ILE_INT_GMM, pool=ILE_POOL_ROUNDS, phase_shear=0):
    return ile_job_opts(n_samples, int(adaptive), round_samples, max_rounds, n_eff_target, seed, tmarg_oversample,
                        integrator, int(pool), int(phase_shear))


def ile_server_submit(srv, problem, opts):
    jid = C.c_uint64()
    _chk(lib().ile_server_submit(srv, C.byref(_problem_struct(problem)), C.byref(opts), C.byref(jid)))
    return jid.value


def ile_server_poll(srv, job_id):
    r = ile_result()
    st = _chk(lib().ile_server_poll(srv, job_id, C.byref(r)))
    return st, r


def ile_server_wait(srv, job_id, timeout_ms=-1):
    r = ile_result()
    _chk(lib().ile_server_wait(srv, job_id, timeout_ms, C.byref(r)))
    return r


def ile_server_cancel(srv, job_id):
    _chk(lib().ile_server_cancel(srv, job_id))


def ile_server_stats(srv):
    a, q, d = C.c_int64(), C.c_int64(), C.c_int64()
    _chk(lib().ile_server_stats(srv, C.byref(a), C.byref(q), C.byref(d)))
    return a.value, q.value, d.value


def ile_server_destroy(srv):
    lib().ile_server_destroy(srv)
