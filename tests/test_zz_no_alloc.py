"""The allocation-free online posterior mean (p2o_posterior_mean_kinv_noalloc)
through the C ABI against p2o_posterior_mean_kinv, the entry point it is a
variant of: the same kernels on a fixed device scratch, so the results must
be equal bit for bit, on consecutive calls whose inputs shrink (fewer
right-hand sides, then a smaller plan), with and without a spatial prior;
also against the oracle's posterior mean (1e-10), and a request beyond the
fixed scratch is refused with P2O_ENOMEM."""
import numpy as np
import pytest
import torch

import oracle
import p2o_synth as S
import paper_2504_16344_amd as P
from gpu_helpers import dev, host, rel_err, workload

pytestmark = pytest.mark.gpu


def _noise(seed, n, lo=0.05, hi=0.5):
    u = (S.vector(seed, S.ARRAY_NOISE, n) + 10.0) / 20.0
    return lo + (hi - lo) * np.clip(u, 0.0, 1.0)


def _prepared(plan, blocks, Nt, Nd, seed, prior=None):
    """K assembled and factored on the device, K^{-1} from the factor, and
    the oracle's K for the same plan (with the prior's C if any)."""
    n = Nt * Nd
    nv = _noise(seed, n)
    C = None
    if prior is not None:
        (nx, ny), r, ell, delta = prior
        plan.set_prior((nx, ny), radius=r, length=ell, delta=delta)
        C = oracle.prior_grid_matrix(nx, ny, r, ell, delta)
    K = plan.hessian(0.25, dev(nv))
    plan.posterior(K, dev(np.zeros((Nt, Nd))), 0.25, refine_steps=0)
    Kinv = plan.posterior_invert(K)
    K_ref = oracle.hessian_gram(blocks, 0.25, nv, C)
    return Kinv, nv, K_ref, C


def _check_call(plan, Kinv, d, blocks, nv, K_ref, C, label):
    """One call of each entry point on the same inputs; equal bit for bit,
    and both within 1e-10 of the oracle."""
    nrhs = d.shape[0]
    out_ref = torch.empty((nrhs, plan.Nt, plan.Nm), dtype=torch.float64, device="cuda")
    out_na = torch.full_like(out_ref, float("nan"))
    plan.posterior_mean_kinv(Kinv, dev(d), 0.25, out=out_ref)
    plan.posterior_mean_kinv_noalloc(Kinv, dev(d), 0.25, out=out_na)
    torch.cuda.synchronize()
    m_ref = np.stack([oracle.posterior_mean(blocks, 0.25, nv, d[r], K=K_ref, prior_C=C)
                      for r in range(nrhs)])
    e = rel_err(host(out_na), m_ref)
    print(f"  {label}: nrhs={nrhs} vs oracle {e:.2e}", flush=True)
    assert torch.equal(out_na, out_ref), label
    assert e <= 1e-10, label


def test_noalloc_matches_allocating_entry_point():
    print("\n[noalloc] consecutive calls, shrinking inputs", flush=True)
    shape_a, shape_b = (5, 300, 29), (3, 40, 7)
    ba, _, _ = workload(41, *shape_a, tau=29 / 3)
    bb, _, _ = workload(42, *shape_b, tau=7 / 3)
    with P.Plan(dev(ba), "fp64") as pa, P.Plan(dev(bb), "fp64") as pb:
        Nd, Nm, Nt = shape_a
        Kinv_a, nv_a, K_a, _ = _prepared(pa, ba, Nt, Nd, 41)
        d = S.vector(41, S.ARRAY_D, 3 * Nt * Nd).reshape(3, Nt, Nd)
        _check_call(pa, Kinv_a, d, ba, nv_a, K_a, None, "call 1 (5x300x29)")
        _check_call(pa, Kinv_a, d[1:2], ba, nv_a, K_a, None, "call 2 (fewer RHS)")
        Nd, Nm, Nt = shape_b
        Kinv_b, nv_b, K_b, _ = _prepared(pb, bb, Nt, Nd, 42)
        d = S.vector(42, S.ARRAY_D, 2 * Nt * Nd).reshape(2, Nt, Nd)
        _check_call(pb, Kinv_b, d, bb, nv_b, K_b, None, "call 3 (smaller plan)")


def test_noalloc_with_spatial_prior():
    print("\n[noalloc] spatial prior", flush=True)
    Nd, nx, ny, Nt = 6, 10, 6, 24
    blocks, _, _ = workload(43, Nd, nx * ny, Nt, tau=Nt / 3)
    with P.Plan(dev(blocks), "fp64") as plan:
        Kinv, nv, K_ref, C = _prepared(plan, blocks, Nt, Nd, 43, prior=((nx, ny), 1, 0.8, 0.3))
        d = S.vector(43, S.ARRAY_D, 2 * Nt * Nd).reshape(2, Nt, Nd)
        _check_call(plan, Kinv, d, blocks, nv, K_ref, C, "prior, 2 RHS")
        _check_call(plan, Kinv, d[:1], blocks, nv, K_ref, C, "prior, 1 RHS")


def test_noalloc_refuses_beyond_fixed_scratch():
    """5 x 300 x 29 needs ~147 KB per right-hand side: 500 exceed 64 MiB."""
    Nd, Nm, Nt = 5, 300, 29
    blocks, _, _ = workload(44, Nd, Nm, Nt, tau=5.0)
    lib = P.load_library()
    n = Nt * Nd
    with P.Plan(dev(blocks), "fp64") as plan:
        Kinv = torch.eye(n, dtype=torch.float64, device="cuda")
        d = torch.zeros((500, Nt, Nd), dtype=torch.float64, device="cuda")
        m = torch.zeros((500, Nt, Nm), dtype=torch.float64, device="cuda")
        assert lib.p2o_posterior_mean_kinv_noalloc(plan._handle(), Kinv.data_ptr(), d.data_ptr(),
                                                   m.data_ptr(), 500, 0.25, None) == 2
        assert lib.p2o_posterior_mean_kinv_noalloc(plan._handle(), None, d.data_ptr(),
                                                   m.data_ptr(), 1, 0.25, None) == 1
        torch.cuda.synchronize()
        assert torch.count_nonzero(m) == 0  # refused calls do nothing
