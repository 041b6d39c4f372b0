"""Shared helpers of the GPU parity tests: seeded workloads and error measures."""
import numpy as np
import torch

import p2o_synth as S


# Tolerances of the comparisons with the FP64 oracle, (normwise per
# right-hand side, element-wise against the largest output of the
# right-hand side).  FP64: the method's target.  16-bit hi+lo tiers: the
# stated bound 1e-5 normwise.  Element-wise, a bfloat16 hi+lo entry (and, on
# the matrix cores, a vector entry split the same way) carries up to 2^-16 ~
# 1.5e-5 relative error, so one output's error is bounded by ~3e-5 of
# sum |F^||x^|, not of |y|; where an output is a short sum (Nt = 1, a few
# sensors or columns) the largest output can be well below that sum, hence
# 2e-5 element-wise for bfloat16.  binary16 entries carry 2^-22 and stay
# far inside 1e-5.  The hi-only tier: 2e-2 (its error is ~1e-3).
TOL_VS_FP64 = {"fp64": (1e-10, 1e-10), "mixed_fp16": (1e-5, 1e-5),
               "mixed_bf16": (1e-5, 2e-5), "fast_bf16": (2e-2, 2e-2)}


def check_tier(y, ref, prec, label=""):
    """check_close with the tier's tolerances against the FP64 oracle."""
    tn, te = TOL_VS_FP64[prec]
    return check_close(y, ref, tn, label, elem_tol=te)


def _batched(y, ref):
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if ref.ndim == 2:
        y, ref = y[None], ref[None]
    return y.reshape(ref.shape), ref


def rel_err(y, ref):
    """Max over right-hand sides of ||y - ref||_2 / ||ref||_2 (arrays [.., Nt, n])."""
    y, ref = _batched(y, ref)
    num = np.sqrt(((y - ref) ** 2).reshape(ref.shape[0], -1).sum(1))
    den = np.sqrt((ref ** 2).reshape(ref.shape[0], -1).sum(1))
    return float((num / den).max())


def elem_err(y, ref):
    """Element-wise error: max over right-hand sides b of
    max_{t,n} |y[b,t,n] - ref[b,t,n]| / max_{t,n} |ref[b,t,n]|,
    with the (b, t) of the worst element."""
    y, ref = _batched(y, ref)
    B = ref.shape[0]
    den = np.abs(ref).reshape(B, -1).max(1)
    den = np.where(den > 0, den, 1.0)
    e = np.abs(y - ref) / den[:, None, None]
    b, t, _ = np.unravel_index(int(np.argmax(e)), e.shape)
    return float(e.max()), (int(b), int(t))


def check_close(y, ref, tol, label="", elem_tol=None):
    """Assert both the normwise (per right-hand side) and the element-wise
    error are within tolerance; print both and the worst (rhs, step)."""
    en = rel_err(y, ref)
    ee, (b, t) = elem_err(y, ref)
    et = tol if elem_tol is None else elem_tol
    print(f"  {label}: normwise {en:.2e}, element-wise {ee:.2e} (worst at rhs {b}, step {t})",
          flush=True)
    assert en <= tol, f"{label}: normwise error {en:.3e} > {tol:.1e}"
    assert ee <= et, f"{label}: element-wise error {ee:.3e} > {et:.1e} at rhs {b}, step {t}"
    return en, ee


def workload(seed, Nd, Nm, Nt, tau, amp=None, nrhs=None):
    """Host blocks and parameter/data vectors of one seeded workload."""
    amp = 1.0 / np.sqrt(Nm) if amp is None else amp
    env = S.envelope(Nt, tau, amp)
    blocks = S.blocks(seed, Nd, Nm, Nt, env)
    shape_m = (Nt, Nm) if nrhs is None else (nrhs, Nt, Nm)
    shape_d = (Nt, Nd) if nrhs is None else (nrhs, Nt, Nd)
    m = S.vector(seed, S.ARRAY_M, int(np.prod(shape_m))).reshape(shape_m)
    d = S.vector(seed, S.ARRAY_D, int(np.prod(shape_d))).reshape(shape_d)
    return blocks, m, d


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()
