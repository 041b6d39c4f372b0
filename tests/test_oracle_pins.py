"""Pins for the FP64 oracle, against facts other than the oracle itself:
a hand-worked example, textbook special cases (causal convolution, a plain
matrix-vector product, a pure delay), the adjoint identity, linearity, shift
invariance, the exactness of the circulant/FFT embedding (checked with
numpy.fft, a different algorithm), two independent routes to K and two to
the posterior mean, closed forms for the scalar problem, and finite
differences.  Each pin is also run against a copy of the oracle with one
planted mistake, to show the pin would catch it.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import p2o_oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


def rand_blocks(rng, Nt, Nd, Nm, tau=None):
    b = rng.standard_normal((Nt, Nd, Nm))
    if tau:
        b *= np.exp(-np.arange(Nt) / tau)[:, None, None]
    return b


def load_golden(name):
    vals = {}
    with open(os.path.join(HERE, "golden", name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *rest = line.split()
            vals[key] = np.array([float(x) for x in rest])
    return vals


# --------------------------------------------------------------------------
# Pin checks, parameterised by the implementation under test.
# --------------------------------------------------------------------------
def check_golden(F, Fadj, hess):
    g = load_golden("hand_example.txt")
    Nd, Nm, Nt = int(g["Nd"][0]), int(g["Nm"][0]), int(g["Nt"][0])
    blocks = np.stack([g[f"F{k}"].reshape(Nd, Nm) for k in range(Nt)])
    m = np.stack([g[f"m{j}"] for j in range(Nt)])
    d = F(blocks, m)
    np.testing.assert_array_equal(d.reshape(-1), g["d"])
    np.testing.assert_array_equal(Fadj(blocks, d).reshape(-1), g["Ftd"])
    K = hess(blocks, g["prior_var"][0], g["noise_var"][0])
    np.testing.assert_array_equal(K.reshape(-1), g["K"])


def check_convolve(F, rng):
    """Nd = Nm = 1: F is causal convolution, np.convolve(f, m)[:Nt]."""
    for Nt in (1, 2, 7, 33):
        f = rng.standard_normal(Nt)
        m = rng.standard_normal(Nt)
        d = F(f.reshape(Nt, 1, 1), m.reshape(Nt, 1)).reshape(-1)
        ref = np.convolve(f, m)[:Nt]
        np.testing.assert_allclose(d, ref, rtol=0, atol=1e-13 * (1 + np.abs(ref).max()))


def check_single_step(F, Fadj, rng):
    """Nt = 1: F is the matrix-vector product F_0 m_0, F* is F_0^T d_0."""
    A = rng.standard_normal((5, 9))
    m = rng.standard_normal(9)
    d = rng.standard_normal(5)
    np.testing.assert_allclose(F(A[None], m[None])[0], A @ m, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(Fadj(A[None], d[None])[0], A.T @ d, rtol=1e-14, atol=1e-14)


def check_delay(F, Fadj, rng):
    """F_k = I for k = s only: F delays m by s steps, F* advances d by s."""
    Nt, n = 9, 4
    m = rng.standard_normal((Nt, n))
    for s in (0, 1, 5, Nt - 1):
        blocks = np.zeros((Nt, n, n))
        blocks[s] = np.eye(n)
        ref = np.zeros_like(m)
        ref[s:] = m[: Nt - s]
        np.testing.assert_array_equal(F(blocks, m), ref)
        refa = np.zeros_like(m)
        refa[: Nt - s] = m[s:]
        np.testing.assert_array_equal(Fadj(blocks, m), refa)


def check_adjoint(F, Fadj, rng):
    """<F m, d> = <m, F* d> for the Euclidean inner product."""
    for (Nt, Nd, Nm) in ((6, 3, 5), (11, 4, 2), (1, 2, 3)):
        b = rand_blocks(rng, Nt, Nd, Nm)
        m = rng.standard_normal((Nt, Nm))
        d = rng.standard_normal((Nt, Nd))
        lhs = np.vdot(F(b, m), d)
        rhs = np.vdot(m, Fadj(b, d))
        assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0)


def check_fft_route(F, Fadj, rng):
    """The block-circulant embedding of length L = 2Nt, diagonalised by the
    DFT, gives F exactly up to rounding (section "FFT-based Hessian matvecs",
    items (ii)-(iii)); numpy.fft is an independent FFT implementation."""
    Nt, Nd, Nm = 13, 3, 4
    b = rand_blocks(rng, Nt, Nd, Nm, tau=5)
    m = rng.standard_normal((Nt, Nm))
    d = rng.standard_normal((Nt, Nd))
    L = 2 * Nt
    Bh = np.fft.rfft(b, n=L, axis=0)
    mh = np.fft.rfft(m, n=L, axis=0)
    dh = np.fft.rfft(d, n=L, axis=0)
    yF = np.fft.irfft(np.einsum("ksp,kp->ks", Bh, mh), n=L, axis=0)[:Nt]
    yA = np.fft.irfft(np.einsum("ksp,ks->kp", Bh.conj(), dh), n=L, axis=0)[:Nt]
    np.testing.assert_allclose(F(b, m), yF, rtol=0, atol=1e-12)
    np.testing.assert_allclose(Fadj(b, d), yA, rtol=0, atol=1e-12)


def check_hessian(hess_a, hess_b, rng):
    Nt, Nd, Nm = 5, 3, 7
    b = rand_blocks(rng, Nt, Nd, Nm)
    nv = rng.uniform(0.1, 1.0, Nt * Nd)
    Ka = hess_a(b, 0.25, nv)
    Kb = hess_b(b, 0.25, nv)
    np.testing.assert_allclose(Ka, Kb, rtol=1e-13, atol=1e-13)


def check_posterior(post, rng):
    """Data-space formula (Sherman-Morrison-Woodbury, Phase 2/4) against the
    parameter-space normal equations, eq. mmap-problem."""
    Nt, Nd, Nm = 4, 2, 5
    b = rand_blocks(rng, Nt, Nd, Nm)
    nv = rng.uniform(0.05, 0.5, Nt * Nd)
    d = rng.standard_normal((Nt, Nd))
    ma = post(b, 0.25, nv, d)
    mb = O.posterior_mean_normal_eq(b, 0.25, nv, d)
    np.testing.assert_allclose(ma, mb, rtol=1e-11, atol=1e-12)


# --------------------------------------------------------------------------
# The oracle passes every pin.
# --------------------------------------------------------------------------
def test_golden_hand_example():
    check_golden(O.apply_F, O.apply_Fadj, O.hessian_gram)
    check_golden(O.apply_F, O.apply_Fadj, O.hessian_dense)
    check_golden(lambda b, m: O.apply_F_loops(b, m), lambda b, d: O.apply_Fadj_loops(b, d),
                 O.hessian_dense)


def test_scalar_case_is_causal_convolution():
    check_convolve(O.apply_F, np.random.default_rng(1))
    check_convolve(O.apply_F_loops, np.random.default_rng(1))


def test_single_step_is_plain_gemv():
    check_single_step(O.apply_F, O.apply_Fadj, np.random.default_rng(2))


def test_pure_delay():
    check_delay(O.apply_F, O.apply_Fadj, np.random.default_rng(3))


def test_adjoint_identity():
    check_adjoint(O.apply_F, O.apply_Fadj, np.random.default_rng(4))
    check_adjoint(O.apply_F_loops, O.apply_Fadj_loops, np.random.default_rng(4))


def test_fft_embedding_route():
    check_fft_route(O.apply_F, O.apply_Fadj, np.random.default_rng(5))


def test_fft_embedding_too_short_aliases():
    """L = 2Nt - 1 is the shortest exact embedding; L = 2Nt - 2 wraps the last
    block around and must disagree with the oracle at O(1)."""
    rng = np.random.default_rng(6)
    Nt, Nd, Nm = 9, 2, 3
    b = rand_blocks(rng, Nt, Nd, Nm)
    m = rng.standard_normal((Nt, Nm))
    ref = O.apply_F(b, m)
    for L, exact in ((2 * Nt - 1, True), (2 * Nt - 2, False)):
        y = np.fft.irfft(np.einsum("ksp,kp->ks", np.fft.rfft(b, n=L, axis=0),
                                   np.fft.rfft(m, n=L, axis=0)), n=L, axis=0)[:Nt]
        err = np.abs(y - ref).max() / np.abs(ref).max()
        assert (err < 1e-13) == exact, (L, err)


def test_dense_matrix_agrees():
    rng = np.random.default_rng(7)
    Nt, Nd, Nm = 6, 3, 4
    b = rand_blocks(rng, Nt, Nd, Nm)
    A = O.dense_F(b)
    m = rng.standard_normal((Nt, Nm))
    d = rng.standard_normal((Nt, Nd))
    np.testing.assert_allclose(O.apply_F(b, m).reshape(-1), A @ m.reshape(-1), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(O.apply_Fadj(b, d).reshape(-1), A.T @ d.reshape(-1), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(O.apply_F_loops(b, m), O.apply_F(b, m), rtol=1e-13, atol=1e-13)


def test_linearity_and_multi_rhs():
    rng = np.random.default_rng(8)
    Nt, Nd, Nm = 7, 3, 5
    b = rand_blocks(rng, Nt, Nd, Nm)
    m1, m2 = rng.standard_normal((2, Nt, Nm))
    lhs = O.apply_F(b, 2.5 * m1 - 0.75 * m2)
    rhs = 2.5 * O.apply_F(b, m1) - 0.75 * O.apply_F(b, m2)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-13, atol=1e-13)
    batch = O.apply_F(b, np.stack([m1, m2]))
    np.testing.assert_array_equal(batch[0], O.apply_F(b, m1))
    np.testing.assert_array_equal(batch[1], O.apply_F(b, m2))


def test_shift_invariance_bitwise():
    """Delaying m by s delays d by s (truncated at Nt); only exact zeros are
    added, so the oracle reproduces it bit for bit."""
    rng = np.random.default_rng(9)
    Nt, Nd, Nm = 10, 3, 4
    b = rand_blocks(rng, Nt, Nd, Nm)
    m = rng.standard_normal((Nt, Nm))
    d = O.apply_F(b, m)
    for s in (1, 3, 9):
        ms = np.zeros_like(m)
        ms[s:] = m[: Nt - s]
        ds = O.apply_F(b, ms)
        assert np.array_equal(ds[s:], d[: Nt - s])
        assert np.all(ds[:s] == 0)


def test_hessian_routes_agree():
    rng = np.random.default_rng(10)
    check_hessian(O.hessian_dense, O.hessian_gram, rng)
    Nt, Nd, Nm = 4, 2, 6
    b = rand_blocks(rng, Nt, Nd, Nm)
    nv = rng.uniform(0.1, 1.0, Nt * Nd)
    K = O.hessian_gram(b, 0.25, nv)
    for col in range(Nt * Nd):
        np.testing.assert_allclose(O.hessian_column(b, 0.25, nv, col), K[:, col],
                                   rtol=1e-13, atol=1e-13)
    assert np.array_equal(K, K.T) or np.abs(K - K.T).max() < 1e-14 * np.abs(K).max()
    assert np.linalg.eigvalsh(K).min() >= nv.min() * (1 - 1e-12)


def test_posterior_two_formulas():
    check_posterior(O.posterior_mean, np.random.default_rng(11))


def test_posterior_scalar_closed_form():
    """Nt = Nd = Nm = 1: m = p f d / (sigma^2 + p f^2)."""
    f, p, s2, d = 1.7, 0.25, 0.3, -0.9
    m = O.posterior_mean(np.array([[[f]]]), p, s2, np.array([[d]]))
    assert abs(m[0, 0] - p * f * d / (s2 + p * f * f)) < 1e-15


def test_posterior_is_stationary_point():
    rng = np.random.default_rng(12)
    Nt, Nd, Nm = 6, 3, 4
    b = rand_blocks(rng, Nt, Nd, Nm)
    nv = rng.uniform(0.05, 0.5, Nt * Nd)
    d = rng.standard_normal((Nt, Nd))
    m = O.posterior_mean(b, 0.25, nv, d)
    g = O.map_objective_gradient(b, 0.25, nv, d, m)
    assert np.abs(g).max() < 1e-11 * (1 + np.abs(m).max() / 0.25)


def test_misfit_gradient_central_differences():
    rng = np.random.default_rng(13)
    Nt, Nd, Nm = 5, 2, 3
    b = rand_blocks(rng, Nt, Nd, Nm)
    m = rng.standard_normal((Nt, Nm))
    d = rng.standard_normal((Nt, Nd))
    v = rng.standard_normal((Nt, Nm))
    f = lambda x: 0.5 * np.sum((O.apply_F(b, x) - d) ** 2)
    h = 1e-3
    fd = (f(m + h * v) - f(m - h * v)) / (2 * h)
    g = np.vdot(O.misfit_gradient(b, m, d), v)
    assert abs(fd - g) <= 1e-9 * (abs(g) + 1)


# --------------------------------------------------------------------------
# Planted mistakes: each mutant copy of an oracle function must fail a pin.
# --------------------------------------------------------------------------
def _F_drop_diagonal(blocks, m):          # forgets the j = i term (F_0)
    Nt = blocks.shape[0]
    d = np.zeros(m.shape[:-2] + (Nt, blocks.shape[1]))
    for k in range(1, Nt):
        d[..., k:, :] += m[..., : Nt - k, :] @ blocks[k].T
    return d


def _F_off_by_one(blocks, m):             # uses F_{i-j-1}: shifted one step
    Nt = blocks.shape[0]
    d = np.zeros(m.shape[:-2] + (Nt, blocks.shape[1]))
    for k in range(Nt - 1):
        d[..., k + 1:, :] += m[..., : Nt - k - 1, :] @ blocks[k].T
    return d


def _Fadj_lower(blocks, d):               # adjoint built as lower triangular
    Nt = blocks.shape[0]
    m = np.zeros(d.shape[:-2] + (Nt, blocks.shape[2]))
    for k in range(Nt):
        m[..., k:, :] += d[..., : Nt - k, :] @ blocks[k]
    return m


def _Fadj_wrong_sign(blocks, d):
    return -O.apply_Fadj(blocks, d)


def _hess_no_recurrence(blocks, prior_var, noise_var):
    Nt, Nd, Nm = blocks.shape
    S = blocks.reshape(Nt * Nd, Nm)
    G = prior_var * (S @ S.T)
    G[np.diag_indices_from(G)] += np.broadcast_to(noise_var, (Nt * Nd,))
    return G


def _hess_no_noise(blocks, prior_var, noise_var):
    return O.hessian_gram(blocks, prior_var, 0.0)


def _post_missing_prior(blocks, prior_var, noise_var, d):
    return O.posterior_mean(blocks, prior_var, noise_var, d) / prior_var


def _post_transposed_solve(blocks, prior_var, noise_var, d):
    return prior_var * O.apply_Fadj(blocks, d / np.broadcast_to(noise_var, d.size).reshape(d.shape))


@pytest.mark.parametrize("mutant", [_F_drop_diagonal, _F_off_by_one])
def test_mutant_forward_is_caught(mutant):
    rng = np.random.default_rng(20)
    with pytest.raises(AssertionError):
        check_convolve(mutant, rng)
    with pytest.raises(AssertionError):
        check_golden(mutant, O.apply_Fadj, O.hessian_gram)


@pytest.mark.parametrize("mutant", [_Fadj_lower, _Fadj_wrong_sign])
def test_mutant_adjoint_is_caught(mutant):
    with pytest.raises(AssertionError):
        check_adjoint(O.apply_F, mutant, np.random.default_rng(21))
    with pytest.raises(AssertionError):
        check_fft_route(O.apply_F, mutant, np.random.default_rng(21))


@pytest.mark.parametrize("mutant", [_hess_no_recurrence, _hess_no_noise])
def test_mutant_hessian_is_caught(mutant):
    with pytest.raises(AssertionError):
        check_hessian(O.hessian_dense, mutant, np.random.default_rng(22))
    with pytest.raises(AssertionError):
        check_golden(O.apply_F, O.apply_Fadj, mutant)


@pytest.mark.parametrize("mutant", [_post_missing_prior, _post_transposed_solve])
def test_mutant_posterior_is_caught(mutant):
    with pytest.raises(AssertionError):
        check_posterior(mutant, np.random.default_rng(23))
