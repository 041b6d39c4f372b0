"""Pins of the oracle with a spatial prior covariance Gamma_prior =
prior_var (I (x) C): the grid covariance's closed forms and invariants, the
Gram-recurrence K against the dense product, and the data-space (SMW)
posterior mean and QoI maps against the parameter-space normal equations
with Gamma_prior^{-1} (a wrong placement of C in either route fails these)."""
import numpy as np
import pytest

import oracle
import p2o_synth as S


def test_grid_covariance_closed_forms():
    # radius 0: B = I, C = (delta + 1) I
    C = oracle.prior_grid_matrix(3, 4, 0, 0.7, 0.2)
    assert np.allclose(C, 1.2 * np.eye(12))
    # window covering the grid with unit weights: B = 1 1^T, C = delta I + n 1 1^T
    C = oracle.prior_grid_matrix(2, 3, 5, 1e9, 0.5)
    assert np.allclose(C, 0.5 * np.eye(6) + 6.0 * np.ones((6, 6)))
    # one axis of length 1 reduces to the 1-D window along the other
    C1 = oracle.prior_grid_matrix(1, 5, 1, 1.0, 0.0)
    w1 = np.exp(-0.5)
    W = np.eye(5) + w1 * (np.eye(5, k=1) + np.eye(5, k=-1))
    assert np.allclose(C1, W @ W)


@pytest.mark.parametrize("grid", [(3, 4, 1, 1.0, 0.1), (4, 4, 2, 1.5, 0.05), (2, 5, 3, 0.8, 0.3)])
def test_grid_covariance_is_spd(grid):
    C = oracle.prior_grid_matrix(*grid)
    assert np.array_equal(C, C.T)
    assert np.linalg.eigvalsh(C).min() >= grid[4] * (1 - 1e-12)


def _setup(Nd=3, Nq=2, nx=2, ny=4, Nt=5, seed=23):
    Nm = nx * ny
    env = S.envelope(Nt, Nt / 2.0)
    blocks = S.blocks(seed, Nd, Nm, Nt, env)
    blocks_q = S.blocks(seed + S.QOI_SEED_OFFSET, Nq, Nm, Nt, env)
    nv = 0.05 + 0.1 * np.arange(Nt * Nd) / (Nt * Nd)
    C = oracle.prior_grid_matrix(nx, ny, 1, 1.2, 0.2)
    d = S.vector(seed, S.ARRAY_D, Nt * Nd).reshape(Nt, Nd)
    return blocks, blocks_q, nv, C, d


def test_gram_recurrence_with_prior_matches_dense():
    blocks, _, nv, C, _ = _setup()
    K1 = oracle.hessian_gram(blocks, 0.3, nv, C)
    K2 = oracle.hessian_dense(blocks, 0.3, nv, C)
    assert np.abs(K1 - K2).max() <= 1e-13 * np.abs(K2).max()


def test_posterior_with_prior_matches_normal_equations():
    blocks, _, nv, C, d = _setup()
    m1 = oracle.posterior_mean(blocks, 0.3, nv, d, prior_C=C)
    m2 = oracle.posterior_mean_normal_eq(blocks, 0.3, nv, d, prior_C=C)
    assert np.abs(m1 - m2).max() <= 1e-10 * np.abs(m2).max()
    # and differs from the identity-prior answer (C matters)
    m0 = oracle.posterior_mean(blocks, 0.3, nv, d)
    assert np.abs(m0 - m2).max() > 1e-3 * np.abs(m2).max()


def test_qoi_with_prior_matches_parameter_space():
    blocks, blocks_q, nv, C, d = _setup()
    Q, G = oracle.qoi_maps(blocks, blocks_q, 0.3, nv, C)
    Qp, Gp = oracle.qoi_maps_parameter_space(blocks, blocks_q, 0.3, nv, C)
    assert np.abs(Q - Qp).max() <= 1e-10 * np.abs(Qp).max()
    assert np.abs(G - Gp).max() <= 1e-10 * np.abs(Gp).max()
    m = oracle.posterior_mean_normal_eq(blocks, 0.3, nv, d, prior_C=C)
    assert np.allclose(Q @ d.reshape(-1), oracle.apply_F(blocks_q, m).reshape(-1),
                       rtol=1e-10, atol=1e-12)
