"""Spatial prior covariance Gamma_prior = prior_var (I (x) C) through the C
ABI (p2o_set_prior): K, the posterior mean and the QoI maps against the
oracle at small and ragged grids, restoring C = I, and the argument checks."""
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


@pytest.mark.parametrize("case", [
    # Nd, Nq, nx, ny, Nt, radius, length, delta, nrhs
    (3, 2, 5, 8, 24, 2, 1.5, 0.1, 1),
    (6, 3, 10, 6, 24, 1, 0.8, 0.3, 3),
    (20, 5, 15, 20, 48, 3, 2.0, 0.05, 20),
])
def test_prior_inversion_matches_oracle(case):
    Nd, Nq, nx, ny, Nt, r, ell, delta, nrhs = case
    Nm = nx * ny
    print(f"\n[prior] case={case}", flush=True)
    blocks, _, _ = workload(31, Nd, Nm, Nt, tau=Nt / 3)
    env = S.envelope(Nt, Nt / 3, 1.0 / np.sqrt(Nm))
    blocks_q = S.blocks(31 + S.QOI_SEED_OFFSET, Nq, Nm, Nt, env)
    n = Nt * Nd
    nv = _noise(31, n)
    d = S.vector(31, S.ARRAY_D, nrhs * n).reshape(nrhs, Nt, Nd)
    C = oracle.prior_grid_matrix(nx, ny, r, ell, delta)
    K_ref = oracle.hessian_gram(blocks, 0.25, nv, C)
    m_ref = np.stack([oracle.posterior_mean(blocks, 0.25, nv, d[i], K=K_ref, prior_C=C)
                      for i in range(nrhs)])
    Q_ref, G_ref = oracle.qoi_maps(blocks, blocks_q, 0.25, nv, C)
    with P.Plan(dev(blocks), "fp64") as plan, P.Plan(dev(blocks_q), "fp64") as planq:
        plan.set_prior((nx, ny), radius=r, length=ell, delta=delta)
        K = plan.hessian(0.25, dev(nv))
        Kh = host(K)
        m = host(plan.posterior(K, dev(d), 0.25, refine_steps=1))
        Q, G = plan.qoi_precompute(planq, K, 0.25)
        Qh, Gh = host(Q), host(G)
    eK = np.abs(Kh - K_ref).max() / np.abs(K_ref).max()
    em = rel_err(m, m_ref)
    eQ = np.abs(Qh - Q_ref).max() / np.abs(Q_ref).max()
    eG = np.abs(Gh - G_ref).max() / np.abs(G_ref).max()
    print(f"  K {eK:.2e}  m {em:.2e}  Q {eQ:.2e}  Gq {eG:.2e}", flush=True)
    assert eK <= 1e-12
    assert em <= 1e-10
    assert eQ <= 1e-9
    assert eG <= 1e-9


def test_prior_reset_restores_identity():
    blocks, _, _ = workload(32, 3, 24, 16, tau=5.0)
    nv = np.full(48, 0.1)
    with P.Plan(dev(blocks), "fp64") as plan:
        K0 = host(plan.hessian(0.25, dev(nv)))
        plan.set_prior((4, 6), radius=2, length=1.0, delta=0.1)
        K1 = host(plan.hessian(0.25, dev(nv)))
        plan.set_prior(None)
        K2 = host(plan.hessian(0.25, dev(nv)))
    assert np.abs(K1 - K0).max() > 1e-3 * np.abs(K0).max()
    assert np.array_equal(K0, K2)


def test_prior_argument_checks():
    blocks, _, _ = workload(33, 2, 24, 8, tau=3.0)
    with P.Plan(dev(blocks), "fp64") as plan:
        for grid, kw in (((5, 5), {}), ((4, 6), {"radius": 33}), ((4, 6), {"radius": -1}),
                         ((4, 6), {"length": 0.0}), ((4, 6), {"delta": 0.0}),
                         ((0, 24), {})):
            with pytest.raises(P.P2OError) as e:
                plan.set_prior(grid, **kw)
            assert e.value.status == 1
        # a rejected prior leaves the plan's identity prior in place
        K = host(plan.hessian(0.25, dev(np.full(16, 0.1))))
        K_ref = oracle.hessian_gram(blocks, 0.25, np.full(16, 0.1))
        assert np.abs(K - K_ref).max() <= 1e-12 * np.abs(K_ref).max()
