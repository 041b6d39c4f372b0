"""Gram-form assembly (p2o_set_assembly(P2O_ASSEMBLE_GRAM)) through the C
ABI: K = Gn + F Gp F* against the oracle's dense definition at small and
ragged sizes (several 64-wide GEMM tiles with ragged tails, contraction
lengths off the 32-entry chunk, a single time step), against the unit-vector
method, with a spatial prior, the QoI maps (rectangular block-diagonal sums
with different row and column steps), sampled columns at the
100 x 5000 x 200 inversion workload, and the argument checks."""
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


@pytest.mark.parametrize("shape", [(3, 40, 7), (4, 33, 1), (5, 300, 29), (20, 300, 55),
                                   (7, 129, 40)])
def test_gram_hessian_matches_dense_definition(shape):
    Nd, Nm, Nt = shape
    print(f"\n[gram] K shape={shape}", flush=True)
    blocks, _, _ = workload(41, Nd, Nm, Nt, tau=max(Nt / 3, 1.0))
    n = Nt * Nd
    nv = _noise(41, n)
    K_ref = oracle.hessian_dense(blocks, 0.25, nv)
    with P.Plan(dev(blocks), "fp64") as plan:
        Kg = host(plan.hessian(0.25, dev(nv), method="gram"))
        Km = host(plan.hessian(0.25, dev(nv), method="matvec"))
    scale = np.abs(K_ref).max()
    eg = np.abs(Kg - K_ref).max() / scale
    em = np.abs(Kg - Km).max() / scale
    print(f"  gram vs dense {eg:.2e}  gram vs unit vectors {em:.2e}", flush=True)
    assert np.array_equal(Kg, Kg.T)
    assert eg <= 1e-12
    assert em <= 1e-12


@pytest.mark.parametrize("Nd,Nq", [(6, 3), (3, 7)])
def test_gram_posterior_and_qoi_match_oracle(Nd, Nq):
    """Both row-step orders of the rectangular block-diagonal sums (N_q below
    and above N_d)."""
    Nm, Nt, nrhs = 200, 30, 2
    print(f"\n[gram] posterior + QoI Nd={Nd} Nq={Nq}", flush=True)
    blocks, _, _ = workload(42, Nd, Nm, Nt, tau=10.0)
    env = S.envelope(Nt, 10.0, 1.0 / np.sqrt(Nm))
    blocks_q = S.blocks(42 + S.QOI_SEED_OFFSET, Nq, Nm, Nt, env)
    n = Nt * Nd
    nv = _noise(42, n)
    d = S.vector(42, S.ARRAY_D, nrhs * n).reshape(nrhs, Nt, Nd)
    K_ref = oracle.hessian_dense(blocks, 0.25, nv)
    m_ref = np.stack([oracle.posterior_mean(blocks, 0.25, nv, d[i], K=K_ref)
                      for i in range(nrhs)])
    Q_ref, G_ref = oracle.qoi_maps(blocks, blocks_q, 0.25, nv)
    with P.Plan(dev(blocks), "fp64") as plan, P.Plan(dev(blocks_q), "fp64") as planq:
        plan.set_assembly("gram")
        K = plan.hessian(0.25, dev(nv))
        m = host(plan.posterior(K, dev(d), 0.25, refine_steps=1))
        Q, G = plan.qoi_precompute(planq, K, 0.25)
        Qh, Gh = host(Q), host(G)
    em = rel_err(m, m_ref)
    eQ = np.abs(Qh - Q_ref).max() / np.abs(Q_ref).max()
    eG = np.abs(Gh - G_ref).max() / np.abs(G_ref).max()
    print(f"  m {em:.2e}  Q {eQ:.2e}  Gq {eG:.2e}", flush=True)
    assert em <= 1e-10
    assert eQ <= 1e-9
    assert eG <= 1e-9
    assert np.array_equal(Gh, Gh.T)


@pytest.mark.parametrize("case", [
    # Nd, Nq, nx, ny, Nt, radius, length, delta
    (3, 2, 5, 8, 24, 2, 1.5, 0.1),
    (20, 5, 15, 20, 48, 3, 2.0, 0.05),
])
def test_gram_with_spatial_prior(case):
    Nd, Nq, nx, ny, Nt, r, ell, delta = case
    Nm = nx * ny
    print(f"\n[gram] prior case={case}", flush=True)
    blocks, _, _ = workload(43, Nd, Nm, Nt, tau=Nt / 3)
    env = S.envelope(Nt, Nt / 3, 1.0 / np.sqrt(Nm))
    blocks_q = S.blocks(43 + S.QOI_SEED_OFFSET, Nq, Nm, Nt, env)
    n = Nt * Nd
    nv = _noise(43, n)
    C = oracle.prior_grid_matrix(nx, ny, r, ell, delta)
    K_ref = oracle.hessian_dense(blocks, 0.25, nv, C)
    Q_ref, G_ref = oracle.qoi_maps(blocks, blocks_q, 0.25, nv, C)
    with P.Plan(dev(blocks), "fp64") as plan, P.Plan(dev(blocks_q), "fp64") as planq:
        plan.set_prior((nx, ny), radius=r, length=ell, delta=delta)
        K = plan.hessian(0.25, dev(nv), method="gram")
        Kh = host(K)
        plan.posterior(K, dev(np.ones((Nt, Nd))), 0.25)
        Q, G = plan.qoi_precompute(planq, K, 0.25)
        Qh, Gh = host(Q), host(G)
    eK = np.abs(Kh - K_ref).max() / np.abs(K_ref).max()
    eQ = np.abs(Qh - Q_ref).max() / np.abs(Q_ref).max()
    eG = np.abs(Gh - G_ref).max() / np.abs(G_ref).max()
    print(f"  K {eK:.2e}  Q {eQ:.2e}  Gq {eG:.2e}", flush=True)
    assert eK <= 1e-12
    assert eQ <= 1e-9
    assert eG <= 1e-9


def test_gram_inversion_workload_100x5000x200():
    """Full-size K by the Gram form: sampled columns against the oracle's
    unit-vector definition, and the whole matrix against the unit-vector
    method on the GPU."""
    Nd, Nm, Nt = 100, 5000, 200
    print("\n[gram] 100x5000x200", flush=True)
    blocks, _, _ = workload(5, Nd, Nm, Nt, tau=40.0)
    n = Nt * Nd
    nv = np.full(n, 0.01)
    with P.Plan(dev(blocks), "fp64") as plan:
        Kg = plan.hessian(0.25, dev(nv), method="gram")
        torch.cuda.synchronize()
        for col in (0, 1, 99, 5050, 12345, n - 1):
            ref = oracle.hessian_column(blocks, 0.25, nv, col)
            got = host(Kg[:, col])
            e = np.abs(got - ref).max() / np.abs(ref).max()
            print(f"  K column {col}: err {e:.2e}", flush=True)
            assert e <= 1e-12
        Km = plan.hessian(0.25, dev(nv), method="matvec")
        diff = ((Kg - Km).abs().max() / Km.abs().max()).item()
    print(f"  gram vs unit vectors {diff:.2e}", flush=True)
    assert diff <= 1e-12


def test_set_assembly_checks():
    blocks, _, _ = workload(44, 2, 24, 8, tau=3.0)
    with P.Plan(dev(blocks), "fp64") as plan:
        with pytest.raises(ValueError):
            plan.set_assembly("cholesky")
        lib = P.load_library()
        assert lib.p2o_set_assembly(plan._handle(), 2) == 1
        assert lib.p2o_set_assembly(None, 0) == 1


def test_unit_vector_assembly_in_step_runs(monkeypatch):
    """Temporary budgets below one sensor's spectra split the unit-vector
    assembly into runs of time steps (the running sum restarted per run,
    with a ragged last run); a budget of two sensors gives passes of 2 and 1
    sensors.  K must not change."""
    Nd, Nm, Nt = 3, 500, 40
    blocks, _, _ = workload(45, Nd, Nm, Nt, tau=12.0)
    n = Nt * Nd
    nv = _noise(45, n)
    K_ref = oracle.hessian_dense(blocks, 0.25, nv)
    with P.Plan(dev(blocks), "fp64") as plan:
        K_all = host(plan.hessian(0.25, dev(nv), method="matvec"))
        # one unit vector's spectra: nf * Nm * 16 bytes = 41 * 500 * 16 = 0.33 MB
        monkeypatch.setenv("P2O_WORKSPACE_MB", "3")  # ~9 unit vectors a pass
        K_run = host(plan.hessian(0.25, dev(nv)))
        monkeypatch.setenv("P2O_WORKSPACE_MB", "27")  # two sensors (80 unit vectors)
        K_two = host(plan.hessian(0.25, dev(nv)))
    scale = np.abs(K_ref).max()
    print(f"\n[gram] step runs: {np.abs(K_run - K_ref).max() / scale:.2e}", flush=True)
    assert np.abs(K_run - K_ref).max() <= 1e-12 * scale
    assert np.abs(K_run - K_all).max() <= 1e-13 * scale
    assert np.abs(K_two - K_all).max() <= 1e-13 * scale
