"""Data-space Hessian K = Gn + F Gp F* (Phase 2) and the posterior mean
m = Gp F* K^{-1} d (Phase 4) through the C ABI, against the oracle: full K
at small and ragged sizes (Cholesky blocks of 64 with a ragged tail, several
right-hand sides, 0-2 refinement steps), sampled K columns and the MAP
optimality condition at the 100 x 5000 x 200 inversion workload, and the
error paths."""
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


@pytest.mark.parametrize("shape,nrhs,refine", [
    ((3, 40, 7), 1, 1),
    ((5, 300, 29), 3, 0),
    ((5, 300, 29), 2, 2),
    ((10, 500, 60), 1, 1),
    ((20, 300, 55), 2, 1),
    ((12, 200, 110), 2, 1),  # n = 1320: trailing updates on 128 x 128 tiles, ragged edges
])
def test_hessian_and_posterior_match_oracle(shape, nrhs, refine):
    Nd, Nm, Nt = shape
    print(f"\n[inverse] shape={shape} nrhs={nrhs} refine={refine}", flush=True)
    blocks, _, _ = workload(6, Nd, Nm, Nt, tau=Nt / 3)
    n = Nt * Nd
    nv = _noise(6, n)
    d = S.vector(6, S.ARRAY_D, nrhs * n).reshape(nrhs, Nt, Nd)
    K_ref = oracle.hessian_gram(blocks, 0.25, nv)
    m_ref = np.stack([oracle.posterior_mean(blocks, 0.25, nv, d[r], K=K_ref) for r in range(nrhs)])
    with P.Plan(dev(blocks), "fp64") as plan:
        K = plan.hessian(0.25, dev(nv))
        Kh = host(K)
        m = host(plan.posterior(K, dev(d), 0.25, refine_steps=refine))
        L = np.tril(host(K))
    eK = np.abs(Kh - K_ref).max() / np.abs(K_ref).max()
    em = rel_err(m, m_ref)
    print(f"  K err {eK:.2e}  m err {em:.2e}", flush=True)
    assert np.array_equal(Kh, Kh.T)
    assert eK <= 1e-12
    assert em <= 1e-10
    # the factor left in the lower triangle reproduces K
    assert np.abs(L @ L.T - K_ref).max() / np.abs(K_ref).max() <= 1e-12


def test_posterior_many_right_hand_sides():
    """520 right-hand sides at n = 1100: the blocked many-right-hand-side
    solve, whose backward rank-256 updates (C += A B with B the row-major
    factor) run on the 128 x 128 matrix-core tiles, against the oracle's
    posterior mean for a sample of right-hand sides and against the same
    solve one right-hand side at a time (the substitution kernels)."""
    Nd, Nm, Nt, nrhs = 20, 300, 55, 520
    print(f"\n[inverse] many right-hand sides nrhs={nrhs}", flush=True)
    blocks, _, _ = workload(12, Nd, Nm, Nt, tau=Nt / 3)
    n = Nt * Nd
    nv = _noise(12, n)
    d = S.vector(12, S.ARRAY_D, nrhs * n).reshape(nrhs, Nt, Nd)
    K_ref = oracle.hessian_gram(blocks, 0.25, nv)
    with P.Plan(dev(blocks), "fp64") as plan:
        K = plan.hessian(0.25, dev(nv))
        m_all = host(plan.posterior(K, dev(d), 0.25, refine_steps=0))  # factors K
        sample = [0, 1, 255, 256, 511, 519]
        m_one = np.stack([host(plan.posterior_mean(K, dev(d[r:r + 1]), 0.25))[0] for r in sample])
    m_ref = np.stack([oracle.posterior_mean(blocks, 0.25, nv, d[r], K=K_ref) for r in sample])
    e_ref = rel_err(m_all[sample], m_ref)
    e_one = rel_err(m_all[sample], m_one)
    print(f"  m err vs oracle {e_ref:.2e}, vs one at a time {e_one:.2e}", flush=True)
    assert e_ref <= 1e-10
    assert e_one <= 1e-12


def test_inversion_workload_100x5000x200():
    """Full-size K (20000 x 20000): sampled columns against the paper's
    unit-vector definition in the oracle, then the posterior mean checked by
    the MAP optimality condition F* Gn^-1 (F m - d) + m / Gp = 0."""
    Nd, Nm, Nt = 100, 5000, 200
    print("\n[inverse] 100x5000x200", flush=True)
    blocks, m_true, _ = workload(5, Nd, Nm, Nt, tau=40.0)
    n = Nt * Nd
    d_clean = oracle.apply_F(blocks, m_true)
    s2 = 1e-2 * float(np.mean(d_clean ** 2))
    d_obs = d_clean + np.sqrt(s2) * S.vector(5, S.ARRAY_NOISE, n).reshape(Nt, Nd)
    nv = np.full(n, s2)
    with P.Plan(dev(blocks), "fp64") as plan:
        K = plan.hessian(0.25, dev(nv))
        torch.cuda.synchronize()
        for col in (0, 1, 99, 5050, 12345, n - 1):
            ref = oracle.hessian_column(blocks, 0.25, nv, col)
            got = host(K[:, col])
            e = np.abs(got - ref).max() / np.abs(ref).max()
            print(f"  K column {col}: err {e:.2e}", flush=True)
            assert e <= 1e-12
        m_dev = plan.posterior(K, dev(d_obs), 0.25, refine_steps=1)
        m = host(m_dev)
        # Phase 4 online, from the factor and from K^{-1}, against the refined m
        m_fac = host(plan.posterior_mean(K, dev(d_obs), 0.25))
        Kinv = plan.posterior_invert(K)
        m_inv = host(plan.posterior_mean_kinv(Kinv, dev(d_obs), 0.25))
        del Kinv
    e_fac, e_inv = rel_err(m_fac, m), rel_err(m_inv, m)
    print(f"  online m vs refined: from the factor {e_fac:.2e}, from K^-1 {e_inv:.2e}", flush=True)
    assert e_fac <= 1e-12 and e_inv <= 1e-12
    g = oracle.map_objective_gradient(blocks, 0.25, nv, d_obs, m)
    scale = np.linalg.norm(m / 0.25)
    print(f"  MAP gradient rel {np.linalg.norm(g) / scale:.2e}", flush=True)
    assert np.linalg.norm(g) / scale <= 1e-9


def test_not_positive_definite_reports_pivot():
    Nd, Nm, Nt = 4, 30, 50  # n = 200: pivot in the fourth Cholesky block
    blocks, _, _ = workload(7, Nd, Nm, Nt, tau=5.0)
    n = Nt * Nd
    with P.Plan(dev(blocks), "fp64") as plan:
        K = torch.eye(n, dtype=torch.float64, device="cuda")
        K[137, 137] = -1.0
        with pytest.raises(P.P2OError) as e:
            plan.posterior(K, dev(np.ones((Nt, Nd))), 0.25)
        assert e.value.status == 4 and e.value.failed_pivot == 137
        # the plan is still usable afterwards
        K2 = plan.hessian(0.25, dev(np.full(n, 0.1)))
        assert torch.isfinite(K2).all()


def test_inversion_needs_fp64_plan():
    blocks, _, _ = workload(8, 2, 256, 4, tau=2.0)
    with P.Plan(dev(blocks), "mixed_bf16") as plan:
        with pytest.raises(P.P2OError) as e:
            plan.hessian(0.25, dev(np.ones(8)))
        assert e.value.status == 6


@pytest.mark.parametrize("shape,nrhs", [((3, 40, 7), 1), ((5, 300, 29), 3), ((5, 300, 29), 20),
                                        ((20, 300, 55), 2), ((5, 60, 13), 2), ((4, 60, 32), 1)])
def test_posterior_mean_from_factor(shape, nrhs):
    """Phase 4 online: m = Gp F* K^{-1} d from the factor left by posterior()
    (single- and many-right-hand-side sweeps), against the oracle; K is not
    modified by the call.  n = Nt Nd covers one ragged block (21), the
    forward sweep's block pairs with and without a ragged second block and
    a single last block (145, 1100), a pair whose second block is one row
    (65) and a pair with no rows below it (128)."""
    Nd, Nm, Nt = shape
    print(f"\n[inverse] online shape={shape} nrhs={nrhs}", flush=True)
    blocks, _, _ = workload(9, Nd, Nm, Nt, tau=Nt / 3)
    n = Nt * Nd
    nv = _noise(9, n)
    d = S.vector(9, S.ARRAY_D, nrhs * n).reshape(nrhs, Nt, Nd)
    K_ref = oracle.hessian_gram(blocks, 0.25, nv)
    m_ref = np.stack([oracle.posterior_mean(blocks, 0.25, nv, d[r], K=K_ref) for r in range(nrhs)])
    with P.Plan(dev(blocks), "fp64") as plan:
        K = plan.hessian(0.25, dev(nv))
        plan.posterior(K, dev(np.zeros((Nt, Nd))), 0.25, refine_steps=0)  # factor K
        K_before = K.clone()
        m = host(plan.posterior_mean(K, dev(d), 0.25))
        assert torch.equal(K, K_before)
    e = rel_err(m, m_ref)
    print(f"  m err {e:.2e}", flush=True)
    assert e <= 1e-10


def test_posterior_mean_errors():
    blocks, _, _ = workload(10, 2, 24, 8, tau=3.0)
    with P.Plan(dev(blocks), "fp64") as plan:
        K = torch.eye(16, dtype=torch.float64, device="cuda")
        with pytest.raises(ValueError):
            plan.posterior_mean(K, dev(np.ones((7, 2))), 0.25)
        lib = P.load_library()
        d = dev(np.ones((8, 2)))
        m = torch.empty((8, 24), dtype=torch.float64, device="cuda")
        assert lib.p2o_posterior_mean(plan._handle(), None, d.data_ptr(), m.data_ptr(), 1,
                                      0.25, None) == 1
        assert lib.p2o_posterior_mean(plan._handle(), K.data_ptr(), d.data_ptr(),
                                      m.data_ptr(), 0, 0.25, None) == 1
    b256, _, _ = workload(10, 2, 256, 8, tau=3.0)
    with P.Plan(dev(b256), "mixed_bf16") as plan:
        with pytest.raises(P.P2OError) as e:
            plan.posterior_mean(torch.eye(16, dtype=torch.float64, device="cuda"),
                                dev(np.ones((8, 2))), 0.25)
        assert e.value.status == 6


@pytest.mark.parametrize("shape,nrhs", [((3, 40, 7), 1), ((5, 300, 29), 3), ((5, 300, 29), 20),
                                        ((4, 60, 32), 2), ((20, 300, 55), 1), ((8, 100, 70), 2)])
def test_posterior_mean_from_inverse(shape, nrhs):
    """Phase 4 online from K^{-1}: posterior_invert() forms K^{-1} from the
    factor (checked by K K^{-1} = I against the oracle's K, and exact
    symmetry; n = 1100 and 560 take the forward sweep and the in-place
    product L^-T L^-1, the smaller ones both sweeps), then
    m = Gp F* (K^{-1} d) against the oracle's posterior mean;
    a second call with one right-hand side reuses the plan's temporaries and
    gives the same first result (bit for bit when both calls take the
    vector-unit F* kernels)."""
    Nd, Nm, Nt = shape
    print(f"\n[inverse] explicit inverse shape={shape} nrhs={nrhs}", flush=True)
    blocks, _, _ = workload(11, Nd, Nm, Nt, tau=Nt / 3)
    n = Nt * Nd
    nv = _noise(11, n)
    d = S.vector(11, S.ARRAY_D, nrhs * n).reshape(nrhs, Nt, Nd)
    K_ref = oracle.hessian_gram(blocks, 0.25, nv)
    m_ref = np.stack([oracle.posterior_mean(blocks, 0.25, nv, d[r], K=K_ref) for r in range(nrhs)])
    with P.Plan(dev(blocks), "fp64") as plan:
        K = plan.hessian(0.25, dev(nv))
        plan.posterior(K, dev(np.zeros((Nt, Nd))), 0.25, refine_steps=0)  # factor K
        K_before = K.clone()
        Kinv = plan.posterior_invert(K)
        assert torch.equal(K, K_before)
        m = plan.posterior_mean_kinv(Kinv, dev(d), 0.25)
        m1 = plan.posterior_mean_kinv(Kinv, dev(d[:1]), 0.25)
        torch.cuda.synchronize()
        Ki, m, m1 = host(Kinv), host(m), host(m1)
    assert np.array_equal(Ki, Ki.T)
    eI = np.abs(K_ref @ Ki - np.eye(n)).max()
    e = rel_err(m, m_ref)
    print(f"  |K K^-1 - I| {eI:.2e}  m err {e:.2e}", flush=True)
    assert eI <= 1e-12
    assert e <= 1e-10
    if nrhs < 8:  # same product kernels (vector units) for both calls
        assert np.array_equal(m1[0], m[0])
    else:         # 20 right-hand sides: F* on the float64 matrix cores
        assert rel_err(m1[0], m[0]) <= 1e-13


def test_posterior_mean_from_inverse_with_prior():
    """The explicit-inverse path with a spatial prior C (Gp = 0.25 (I (x) C))."""
    Nd, nx, ny, Nt, nrhs = 6, 10, 6, 24, 2
    Nm = nx * ny
    blocks, _, _ = workload(12, Nd, Nm, Nt, tau=Nt / 3)
    n = Nt * Nd
    nv = _noise(12, n)
    d = S.vector(12, S.ARRAY_D, nrhs * n).reshape(nrhs, Nt, Nd)
    C = oracle.prior_grid_matrix(nx, ny, 1, 0.8, 0.3)
    K_ref = oracle.hessian_gram(blocks, 0.25, nv, C)
    m_ref = np.stack([oracle.posterior_mean(blocks, 0.25, nv, d[i], K=K_ref, prior_C=C)
                      for i in range(nrhs)])
    with P.Plan(dev(blocks), "fp64") as plan:
        plan.set_prior((nx, ny), radius=1, length=0.8, delta=0.3)
        K = plan.hessian(0.25, dev(nv))
        plan.posterior(K, dev(np.zeros((Nt, Nd))), 0.25, refine_steps=0)
        m = host(plan.posterior_mean_kinv(plan.posterior_invert(K), dev(d), 0.25))
    e = rel_err(m, m_ref)
    print(f"\n[inverse] explicit inverse with prior: m err {e:.2e}", flush=True)
    assert e <= 1e-10


def test_posterior_inverse_errors():
    blocks, _, _ = workload(10, 2, 24, 8, tau=3.0)
    lib = P.load_library()
    with P.Plan(dev(blocks), "fp64") as plan:
        K = torch.eye(16, dtype=torch.float64, device="cuda")
        with pytest.raises(ValueError):
            plan.posterior_invert(torch.eye(15, dtype=torch.float64, device="cuda"))
        d = dev(np.ones((8, 2)))
        m = torch.empty((8, 24), dtype=torch.float64, device="cuda")
        assert lib.p2o_posterior_invert(plan._handle(), K.data_ptr(), None, None) == 1
        assert lib.p2o_posterior_mean_kinv(plan._handle(), None, d.data_ptr(), m.data_ptr(), 1,
                                           0.25, None) == 1
        assert lib.p2o_posterior_mean_kinv(plan._handle(), K.data_ptr(), d.data_ptr(),
                                           m.data_ptr(), 0, 0.25, None) == 1
    b256, _, _ = workload(10, 2, 256, 8, tau=3.0)
    with P.Plan(dev(b256), "mixed_bf16") as plan:
        K = torch.eye(16, dtype=torch.float64, device="cuda")
        with pytest.raises(P.P2OError) as e:
            plan.posterior_invert(K)
        assert e.value.status == 6
        with pytest.raises(P.P2OError) as e:
            plan.posterior_mean_kinv(K, dev(np.ones((8, 2))), 0.25)
        assert e.value.status == 6
