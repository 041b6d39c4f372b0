"""QoI posterior (section "Real-time Bayesian inference and prediction
framework", Phases 3 and 4) through the C ABI: the data-to-QoI map Q and the
QoI posterior covariance against the oracle at small and ragged sizes
(several triangular-solve blocks with a ragged tail, several matrix-core
GEMM tiles), the online prediction Q d against the p2q map applied to the
MAP point, the many-right-hand-side solve path of the posterior mean, the
100 x 5000 x 200 inversion workload with 21 QoI locations, and the error
paths."""
import numpy as np
import pytest
import torch

import oracle
import p2o_synth as S
import paper_2504_16344_amd as P
from gpu_helpers import dev, host, rel_err, workload

pytestmark = pytest.mark.gpu


def _noise(seed, n, lo=0.05, hi=0.5):
    u = (S.vector(seed, S.ARRAY_NOISE, n) + 10.0) / 20.0  # deterministic, positive
    return lo + (hi - lo) * np.clip(u, 0.0, 1.0)


def _qoi_blocks(seed, Nq, Nm, Nt, tau):
    env = S.envelope(Nt, tau, 1.0 / np.sqrt(Nm))
    return S.blocks(seed + S.QOI_SEED_OFFSET, Nq, Nm, Nt, env)


@pytest.mark.parametrize("shape", [(3, 2, 40, 24), (6, 3, 60, 24), (20, 5, 300, 48)])
def test_qoi_maps_match_oracle(shape):
    Nd, Nq, Nm, Nt = shape
    print(f"\n[qoi] shape={shape}", flush=True)
    blocks, _, d = workload(11, Nd, Nm, Nt, tau=Nt / 3)
    blocks_q = _qoi_blocks(11, Nq, Nm, Nt, Nt / 3)
    n = Nt * Nd
    nv = _noise(11, n)
    Q_ref, G_ref = oracle.qoi_maps(blocks, blocks_q, 0.25, nv)
    with P.Plan(dev(blocks), "fp64") as plan, P.Plan(dev(blocks_q), "fp64") as planq:
        K = plan.hessian(0.25, dev(nv))
        m = plan.posterior(K, dev(d), 0.25, refine_steps=1)
        Q, G = plan.qoi_precompute(planq, K, 0.25)
        q = P.qoi_predict(Q, dev(d))
        q_map = host(planq.F(m))
        Qh, Gh, qh = host(Q), host(G), host(q)
    eQ = np.abs(Qh - Q_ref).max() / np.abs(Q_ref).max()
    eG = np.abs(Gh - G_ref).max() / np.abs(G_ref).max()
    eq = rel_err(qh.reshape(Nt, Nq), q_map)
    print(f"  Q err {eQ:.2e}  Gq err {eG:.2e}  Qd vs Fq m_map {eq:.2e}", flush=True)
    assert eQ <= 1e-9
    assert eG <= 1e-9
    assert np.array_equal(Gh, Gh.T)
    assert eq <= 1e-9
    assert rel_err(qh, Q_ref @ d.reshape(-1)) <= 1e-9


def test_posterior_many_rhs_path_matches_oracle():
    """nrhs >= 16 takes the blocked matrix-core solve."""
    Nd, Nm, Nt, nrhs = 5, 300, 29, 20
    print(f"\n[qoi] posterior nrhs={nrhs}", flush=True)
    blocks, _, _ = workload(12, Nd, Nm, Nt, tau=Nt / 3)
    n = Nt * Nd
    nv = _noise(12, n)
    d = S.vector(12, S.ARRAY_D, nrhs * n).reshape(nrhs, Nt, Nd)
    K_ref = oracle.hessian_gram(blocks, 0.25, nv)
    m_ref = np.stack([oracle.posterior_mean(blocks, 0.25, nv, d[r], K=K_ref) for r in range(nrhs)])
    for refine in (0, 1):
        with P.Plan(dev(blocks), "fp64") as plan:
            K = plan.hessian(0.25, dev(nv))
            m = host(plan.posterior(K, dev(d), 0.25, refine_steps=refine))
        e = rel_err(m, m_ref)
        print(f"  refine={refine}: m err {e:.2e}", flush=True)
        assert e <= 1e-10


def test_qoi_predict_ragged_and_many_rhs():
    """q = Q d for row and column counts off the wavefront width and 1..9
    right-hand sides, against a float64 host product."""
    rng = np.random.default_rng(5)
    for nq, n, nrhs in ((1, 1, 1), (7, 129, 3), (37, 1000, 9), (64, 4097, 5)):
        Qm = rng.standard_normal((nq, n))
        dm = rng.standard_normal((nrhs, n))
        q = host(P.qoi_predict(dev(Qm), dev(dm)))
        ref = dm @ Qm.T
        assert np.abs(q - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_qoi_inversion_workload_100x5000x200():
    """Nd = 100, Nm = 5000, Nt = 200 with the paper's 21 QoI locations:
    Q (4200 x 20000) and Gq (4200 x 4200) through the full pipeline; checked
    by Phase 4's identity Q d_obs = Fq m_map, symmetry and positive
    diagonal of Gq, and Gq below the prior QoI covariance on sampled
    diagonal entries."""
    Nd, Nq, Nm, Nt = 100, 21, 5000, 200
    print("\n[qoi] 100x5000x200, Nq = 21", flush=True)
    blocks, m_true, _ = workload(5, Nd, Nm, Nt, tau=40.0)
    blocks_q = _qoi_blocks(5, Nq, Nm, Nt, 40.0)
    n = Nt * Nd
    d_clean = oracle.apply_F(blocks, m_true)
    s2 = 1e-2 * float(np.mean(d_clean ** 2))
    d_obs = d_clean + np.sqrt(s2) * S.vector(5, S.ARRAY_NOISE, n).reshape(Nt, Nd)
    nv = np.full(n, s2)
    with P.Plan(dev(blocks), "fp64") as plan, P.Plan(dev(blocks_q), "fp64") as planq:
        K = plan.hessian(0.25, dev(nv))
        m = plan.posterior(K, dev(d_obs), 0.25, refine_steps=1)
        Q, G = plan.qoi_precompute(planq, K, 0.25)
        q = host(P.qoi_predict(Q, dev(d_obs)))
        q_map = host(planq.F(m)).reshape(-1)
        Gh = host(G)
    e = np.linalg.norm(q - q_map) / np.linalg.norm(q_map)
    print(f"  Q d vs Fq m_map {e:.2e}", flush=True)
    assert e <= 1e-8
    assert np.array_equal(Gh, Gh.T)
    diag = np.diag(Gh)
    assert (diag > 0).all()
    for j in (0, 20, 21 * 100 + 7, Nt * Nq - 1):
        t, qi = divmod(j, Nq)
        rows = blocks_q[:t + 1, qi, :]                 # Fq_k[qi, :] for k <= t
        prior_jj = 0.25 * float((rows ** 2).sum())     # (Fq Gp Fq^T)_jj
        assert 0 < diag[j] <= prior_jj


def test_qoi_errors():
    blocks, _, _ = workload(13, 2, 40, 8, tau=3.0)
    bq6, _, _ = workload(14, 1, 40, 6, tau=3.0)   # different Nt
    bq, _, _ = workload(14, 1, 40, 8, tau=3.0)
    with P.Plan(dev(blocks), "fp64") as plan, P.Plan(dev(bq6), "fp64") as p6, \
            P.Plan(dev(bq), "fp64") as pq:
        K = plan.hessian(0.25, dev(np.full(16, 0.1)))
        plan.posterior(K, dev(np.ones((8, 2))), 0.25)
        with pytest.raises(P.P2OError) as e:
            plan.qoi_precompute(p6, K, 0.25)
        assert e.value.status == 1
        Q, G = plan.qoi_precompute(pq, K, 0.25)
        assert torch.isfinite(Q).all() and torch.isfinite(G).all()
    bq256, _, _ = workload(15, 1, 256, 8, tau=3.0)
    b256, _, _ = workload(15, 2, 256, 8, tau=3.0)
    with P.Plan(dev(b256), "fp64") as plan, P.Plan(dev(bq256), "mixed_bf16") as pm:
        K = torch.eye(16, dtype=torch.float64, device="cuda")
        with pytest.raises(P.P2OError) as e:
            plan.qoi_precompute(pm, K, 0.25)
        assert e.value.status == 6
