"""Shared helpers of the GPU parity tests: seeded workloads and error measures."""
import numpy as np
import torch

import p2o_synth as S


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
