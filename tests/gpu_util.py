"""Shared helpers for the GPU tests: device context, problem upload, and the
per-sample tolerance used to compare the HIP path with the oracle."""
import numpy as np

import paper_2505_11655_amd as ile

_CTX = None


def ctx():
    global _CTX
    if _CTX is None:
        _CTX = ile.ile_ctx_create(0, 0)
    return _CTX


def torch_dtype(policy):
    import torch
    return torch.float64 if policy == ile.ILE_FP64 else torch.float32


def out_dtype(policy):
    import torch
    return torch.float32 if policy == ile.ILE_FP32 else torch.float64


def gpu_eval(job, theta_np, policy, lnpmps_np=None, stream=None):
    """Upload theta [7][n] (numpy, already in the policy dtype), run ile_eval_lnL,
    return (lnL, lw) as float64 numpy arrays."""
    import torch
    n = theta_np.shape[1]
    th = torch.from_numpy(np.ascontiguousarray(theta_np)).to("cuda")
    lr = None if lnpmps_np is None else torch.from_numpy(np.ascontiguousarray(lnpmps_np)).to("cuda")
    L = torch.full((max(n, 1),), float("nan"), dtype=out_dtype(policy), device="cuda")
    W = torch.full((max(n, 1),), float("nan"), dtype=out_dtype(policy), device="cuda")
    ile.ile_eval_lnL(job, n, th, n, lr, L, W, stream=stream)
    torch.cuda.synchronize()
    return L[:n].double().cpu().numpy(), W[:n].double().cpu().numpy()


def tol_check(got, ref, T1, T2, s, policy, scope_abs=1e-3):
    """Per-sample agreement, as stated for each policy:
      FP64: |d| <= 1e-9 (1 + |s T1| + |s^2 T2 / 4|);
      FP32 and FP32+FP64-cancellation: |d| <= scope_abs for every sample with
      lnL >= max lnL - 50, and |d| <= scope_abs + 1e-6 (|s T1| + |s^2 T2/4|)
      elsewhere (those carry weight below e^-50).
    -inf (outside the support) must match exactly.  Returns (ok, max_scoped, max_all)."""
    inf_ref = ~np.isfinite(ref)
    assert np.array_equal(inf_ref, ~np.isfinite(got)), "support mismatch"
    g, r = got[~inf_ref], ref[~inf_ref]
    mag = np.abs(s * T1) + np.abs(s * s * T2 / 4)
    mag = mag[~inf_ref]
    d = np.abs(g - r)
    if d.size == 0:
        return True, 0.0, 0.0
    if policy == ile.ILE_FP64:
        ok = np.all(d <= 1e-9 * (1 + mag))
        return ok, float(d.max()), float(d.max())
    top = r >= r.max() - 50
    ok = np.all(d[top] <= scope_abs) and np.all(d <= scope_abs + 1e-6 * mag)
    if not ok:
        w = int(np.argmax(d / (scope_abs + 1e-6 * mag)))
        print(f"tol_check worst: |d|={d[w]:.3e} lnL={r[w]:.6g} mag={mag[w]:.6g} "
              f"sT1={float((s * T1)[~inf_ref][w]):.6g} s2T2/4={float((s * s * T2 / 4)[~inf_ref][w]):.6g} "
              f"scoped={bool(top[w])}")
    return ok, float(d[top].max()), float(d.max())
