"""Pins of the oracle's QoI posterior (section "Real-time Bayesian inference
and prediction framework", Phase 3): the Sherman-Morrison-Woodbury route
the oracle takes, checked against the parameter-space definitions
Q = Fq Gamma_post F^* Gamma_noise^{-1}, Gamma_post(q) = Fq Gamma_post Fq^*
with Gamma_post = (F^* Gn^{-1} F + Gp^{-1})^{-1}, against Phase 4's
identity Q d = Fq m_map, and the cross Gram product against dense
matrices."""
import numpy as np
import pytest

import oracle
import p2o_synth as S


def _setup(Nd=3, Nq=2, Nm=7, Nt=5, seed=21):
    env = S.envelope(Nt, Nt / 2.0)
    blocks = S.blocks(seed, Nd, Nm, Nt, env)
    blocks_q = S.blocks(seed + S.QOI_SEED_OFFSET, Nq, Nm, Nt, env)
    nv = 0.05 + 0.1 * np.arange(Nt * Nd) / (Nt * Nd)
    return blocks, blocks_q, nv


def test_cross_gram_is_dense_product():
    blocks, blocks_q, _ = _setup()
    ref = 0.3 * oracle.dense_F(blocks) @ oracle.dense_F(blocks_q).T
    assert np.allclose(oracle.cross_gram(blocks, blocks_q, 0.3), ref, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("shape", [(3, 2, 7, 5), (4, 3, 5, 6), (2, 1, 9, 4)])
def test_qoi_maps_match_parameter_space_definitions(shape):
    Nd, Nq, Nm, Nt = shape
    blocks, blocks_q, nv = _setup(Nd, Nq, Nm, Nt)
    Q, G = oracle.qoi_maps(blocks, blocks_q, 0.25, nv)
    Qp, Gp = oracle.qoi_maps_parameter_space(blocks, blocks_q, 0.25, nv)
    assert Q.shape == (Nt * Nq, Nt * Nd) and G.shape == (Nt * Nq, Nt * Nq)
    assert np.abs(Q - Qp).max() <= 1e-10 * np.abs(Qp).max()
    assert np.abs(G - Gp).max() <= 1e-10 * np.abs(Gp).max()
    # a covariance: symmetric, positive definite, below the prior covariance
    assert np.abs(G - G.T).max() <= 1e-12 * np.abs(G).max()
    assert np.linalg.eigvalsh((G + G.T) / 2).min() > 0
    prior = oracle.cross_gram(blocks_q, blocks_q, 0.25)
    assert np.linalg.eigvalsh(prior - (G + G.T) / 2).min() > -1e-12


def test_q_times_data_is_qoi_of_map_point():
    blocks, blocks_q, nv = _setup()
    Nt, Nd = blocks.shape[:2]
    d = S.vector(21, S.ARRAY_D, Nt * Nd).reshape(Nt, Nd)
    Q, _ = oracle.qoi_maps(blocks, blocks_q, 0.25, nv)
    m = oracle.posterior_mean_normal_eq(blocks, 0.25, nv, d)
    q_ref = oracle.apply_F(blocks_q, m).reshape(-1)
    assert np.allclose(Q @ d.reshape(-1), q_ref, rtol=1e-10, atol=1e-12)


def test_qoi_pin_fails_on_planted_sign_error():
    """A dropped minus sign in the covariance update is caught."""
    blocks, blocks_q, nv = _setup()
    Q, G = oracle.qoi_maps(blocks, blocks_q, 0.25, nv)
    B = oracle.cross_gram(blocks, blocks_q, 0.25)
    wrong = oracle.cross_gram(blocks_q, blocks_q, 0.25) + Q @ B
    _, Gp = oracle.qoi_maps_parameter_space(blocks, blocks_q, 0.25, nv)
    assert np.abs(wrong - Gp).max() > 1e-3 * np.abs(Gp).max()
    assert np.abs(G - Gp).max() <= 1e-10 * np.abs(Gp).max()
