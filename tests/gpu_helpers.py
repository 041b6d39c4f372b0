"""Shared helpers of the GPU parity tests: seeded workloads and error norms."""
import numpy as np
import torch

import p2o_synth as S


def rel_err(y, ref):
    """Max over right-hand sides of ||y - ref||_2 / ||ref||_2 (arrays [.., Nt, n])."""
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if ref.ndim == 2:
        y, ref = y[None], ref[None]
    y = y.reshape(ref.shape)
    num = np.sqrt(((y - ref) ** 2).reshape(ref.shape[0], -1).sum(1))
    den = np.sqrt((ref ** 2).reshape(ref.shape[0], -1).sum(1))
    return float((num / den).max())


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
