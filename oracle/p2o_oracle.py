"""FP64 CPU oracle: the p2o map F, its adjoint F*, the data-space Hessian K,
the posterior mean and the QoI posterior (data-to-QoI map Q and covariance
Gamma_post(q)), each written as the plain definition from the paper.

TEST INFRASTRUCTURE ONLY (see the package docstring).  No FFT, no blocking,
no reordering beyond what the definitions state: the FFT method the product
path uses must reproduce these results up to rounding, because the paper
states that its Fourier-space matvecs are exact.

Notation (section "FFT-based Hessian matvecs", eq. ShiftInvariance):
the paper's 1-based blocks F_{i1} (i = 1..Nt) are stored 0-based as
``blocks[k] = F_{k+1,1}``, an Nd x Nm matrix, for k = 0..Nt-1.  Parameters
m are [..., Nt, Nm] (time block j holds m_j), data d are [..., Nt, Nd].
Leading dimensions are independent right-hand sides.

Readings where the paper is silent (all listed in the design notes):
* F* is the Euclidean transpose F^T (the blocks are given matrices; no mass
  or quadrature weights are named).
* The prior mean is zero, as the paper takes it in its online phase.
* Gamma_prior = prior_var * (I_Nt (x) C), the same spatial covariance C on
  every time step (C = I unless given; prior_grid_matrix builds the
  synthetic smooth one), and Gamma_noise = diag(noise_var).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

__all__ = [
    "apply_F", "apply_Fadj", "apply_F_loops", "apply_Fadj_loops", "dense_F",
    "F_entry", "Fadj_entry", "hessian_dense", "hessian_gram",
    "hessian_column", "posterior_mean", "posterior_mean_normal_eq",
    "misfit_gradient", "map_objective_gradient", "cross_gram", "qoi_maps",
    "qoi_maps_parameter_space", "prior_grid_matrix",
]


def _dims(blocks: np.ndarray):
    if blocks.ndim != 3:
        raise ValueError("blocks must be [Nt][Nd][Nm]")
    return blocks.shape  # Nt, Nd, Nm


def apply_F(blocks: np.ndarray, m: np.ndarray) -> np.ndarray:
    """d = F m, eq. ShiftInvariance: d_i = sum_{j<=i} F_{i-j} m_j.

    Grouped by the block index k = i - j: every output step i >= k receives
    F_k m_{i-k}, i.e. d[k:] += m[:Nt-k] F_k^T.  Same terms as the double sum.
    """
    Nt, Nd, Nm = _dims(blocks)
    m = np.asarray(m, dtype=np.float64)
    if m.shape[-2:] != (Nt, Nm):
        raise ValueError(f"m must end in ({Nt}, {Nm}), got {m.shape}")
    d = np.zeros(m.shape[:-2] + (Nt, Nd), dtype=np.float64)
    for k in range(Nt):
        d[..., k:, :] += m[..., : Nt - k, :] @ blocks[k].T
    return d


def apply_Fadj(blocks: np.ndarray, d: np.ndarray) -> np.ndarray:
    """m = F* d with F* = F^T: (F^T d)_j = sum_{i>=j} F_{i-j}^T d_i.

    Transpose of eq. ShiftInvariance (block upper-triangular Toeplitz).
    Grouped by k = i - j: m[:Nt-k] += d[k:] F_k.
    """
    Nt, Nd, Nm = _dims(blocks)
    d = np.asarray(d, dtype=np.float64)
    if d.shape[-2:] != (Nt, Nd):
        raise ValueError(f"d must end in ({Nt}, {Nd}), got {d.shape}")
    m = np.zeros(d.shape[:-2] + (Nt, Nm), dtype=np.float64)
    for k in range(Nt):
        m[..., : Nt - k, :] += d[..., k:, :] @ blocks[k]
    return m


def apply_F_loops(blocks: np.ndarray, m: np.ndarray) -> np.ndarray:
    """Scalar-loop form of eq. ShiftInvariance for one right-hand side (tiny sizes)."""
    Nt, Nd, Nm = _dims(blocks)
    d = np.zeros((Nt, Nd))
    for i in range(Nt):
        for j in range(i + 1):
            for s in range(Nd):
                acc = 0.0
                for p in range(Nm):
                    acc += blocks[i - j, s, p] * m[j, p]
                d[i, s] += acc
    return d


def apply_Fadj_loops(blocks: np.ndarray, d: np.ndarray) -> np.ndarray:
    """Scalar-loop form of F^T for one right-hand side (tiny sizes)."""
    Nt, Nd, Nm = _dims(blocks)
    m = np.zeros((Nt, Nm))
    for j in range(Nt):
        for i in range(j, Nt):
            for p in range(Nm):
                acc = 0.0
                for s in range(Nd):
                    acc += blocks[i - j, s, p] * d[i, s]
                m[j, p] += acc
    return m


def dense_F(blocks: np.ndarray) -> np.ndarray:
    """The (Nt Nd) x (Nt Nm) block lower-triangular Toeplitz matrix of eq.
    ShiftInvariance: block (i, j) is F_{i-j} for j <= i and 0 above."""
    Nt, Nd, Nm = _dims(blocks)
    A = np.zeros((Nt * Nd, Nt * Nm))
    for i in range(Nt):
        for j in range(i + 1):
            A[i * Nd:(i + 1) * Nd, j * Nm:(j + 1) * Nm] = blocks[i - j]
    return A


def F_entry(rows_s: np.ndarray, m: np.ndarray, i: int) -> float:
    """One output d_i[s] = sum_{j<=i} F_{i-j}[s, :] . m_j.

    rows_s: [Nt][Nm], rows_s[k] = F_k[s, :] (only k <= i is read).  Lets a test
    check single outputs of workloads whose blocks do not fit in host memory.
    """
    acc = 0.0
    for j in range(i + 1):
        acc += float(rows_s[i - j] @ m[j])
    return acc


def Fadj_entry(cols_p: np.ndarray, d: np.ndarray, j: int) -> float:
    """One output (F^T d)_j[p] = sum_{i>=j} F_{i-j}[:, p] . d_i.

    cols_p: [Nt][Nd], cols_p[k] = F_k[:, p].
    """
    Nt = d.shape[0]
    acc = 0.0
    for i in range(j, Nt):
        acc += float(cols_p[i - j] @ d[i])
    return acc


def _noise_diag(noise_var, n: int) -> np.ndarray:
    v = np.broadcast_to(np.asarray(noise_var, dtype=np.float64), (n,))
    return np.array(v)


def hessian_dense(blocks: np.ndarray, prior_var: float, noise_var,
                  prior_C: np.ndarray | None = None) -> np.ndarray:
    """K = Gamma_noise + F Gamma_prior F^*  (section "Real-time Bayesian
    inference and prediction framework", Phase 2, with G^* = Gamma_prior F^*),
    from the explicit dense F; Gamma_prior = prior_var (I_Nt (x) C), C = I
    unless prior_C is given.  Row/column index (i, s) -> i*Nd + s."""
    Nt, Nd, _ = _dims(blocks)
    A = dense_F(blocks)
    if prior_C is None:
        K = prior_var * (A @ A.T)
    else:
        K = prior_var * (A @ np.kron(np.eye(Nt), prior_C) @ A.T)
    K[np.diag_indices_from(K)] += _noise_diag(noise_var, Nt * Nd)
    return K


def hessian_gram(blocks: np.ndarray, prior_var: float, noise_var,
                 prior_C: np.ndarray | None = None) -> np.ndarray:
    """The same K without forming F: block (i, j) of F (I (x) C) F^T is
    sum_{l<=min(i,j)} F_{i-l} C F_{j-l}^T, which satisfies
    (F (I (x) C) F^T)_{ij} = F_i C F_j^T + (...)_{i-1, j-1} (terms with a
    negative index are zero).  One Gram product of the stacked blocks plus
    that recurrence; independent of the matvec route the product path uses."""
    Nt, Nd, Nm = _dims(blocks)
    S = blocks.reshape(Nt * Nd, Nm)
    G = S @ (S.T if prior_C is None else prior_C @ S.T)  # block (a, b) = F_a C F_b^T
    for i in range(1, Nt):           # row block i uses the finished row block i-1
        G[i * Nd:(i + 1) * Nd, Nd:] += G[(i - 1) * Nd:i * Nd, :-Nd]
    G *= prior_var
    G[np.diag_indices_from(G)] += _noise_diag(noise_var, Nt * Nd)
    return G


def hessian_column(blocks: np.ndarray, prior_var: float, noise_var, col: int) -> np.ndarray:
    """Column `col` = (i, s) of K as the paper forms it: K e = Gamma_noise e +
    F(Gamma_prior F^* e) for the unit vector e (Phase 2)."""
    Nt, Nd, _ = _dims(blocks)
    e = np.zeros((Nt, Nd))
    e.flat[col] = 1.0
    out = apply_F(blocks, prior_var * apply_Fadj(blocks, e)).reshape(-1)
    out[col] += _noise_diag(noise_var, Nt * Nd)[col]
    return out


def cross_gram(blocks_a: np.ndarray, blocks_b: np.ndarray, prior_var: float,
               prior_C: np.ndarray | None = None) -> np.ndarray:
    """Fa Gamma_prior Fb^T for two block-Toeplitz maps on the same parameter
    grid (same Nm, Nt), e.g. F Gamma_prior Fq^* of Phase 3: block (i, j) is
    prior_var sum_{l<=min(i,j)} Fa_{i-l} C Fb_{j-l}^T, by the recurrence of
    hessian_gram applied to the Gram product of the two stacked block sets."""
    Nt, Nda, Nm = _dims(blocks_a)
    Ntb, Ndb, Nmb = _dims(blocks_b)
    assert (Nt, Nm) == (Ntb, Nmb)
    Sb = blocks_b.reshape(Nt * Ndb, Nm).T
    G = blocks_a.reshape(Nt * Nda, Nm) @ (Sb if prior_C is None else prior_C @ Sb)
    for i in range(1, Nt):
        G[i * Nda:(i + 1) * Nda, Ndb:] += G[(i - 1) * Nda:i * Nda, :-Ndb]
    return prior_var * G


def qoi_maps(blocks: np.ndarray, blocks_q: np.ndarray, prior_var: float,
             noise_var, prior_C: np.ndarray | None = None) -> tuple[np.ndarray, np.ndarray]:
    """Phase 3 of section "Real-time Bayesian inference and prediction
    framework" (zero prior mean, Gamma_prior = prior_var I): the data-to-QoI
    map Q = Fq Gamma_post F^* Gamma_noise^{-1} and the QoI posterior
    covariance Gamma_post(q) = Fq Gamma_post Fq^*, both written through the
    Sherman-Morrison-Woodbury form Gamma_post = Gamma_prior -
    G^* K^{-1} G (G^* = Gamma_prior F^*): Q = Fq G^* K^{-1},
    Gamma_post(q) = Fq Gamma_prior Fq^* - Q F Gamma_prior Fq^*.
    Q: [(Nt Nq)][(Nt Nd)], Gamma_post(q): [(Nt Nq)]^2 (index t*N + s)."""
    K = hessian_gram(blocks, prior_var, noise_var, prior_C)
    B = cross_gram(blocks, blocks_q, prior_var, prior_C)   # F Gp Fq^*, (Nt Nd) x (Nt Nq)
    KinvB = scipy.linalg.cho_solve(scipy.linalg.cho_factor(K, lower=True), B)
    Q = KinvB.T                                            # K symmetric
    Gq = cross_gram(blocks_q, blocks_q, prior_var, prior_C) - B.T @ KinvB
    return Q, Gq


def qoi_maps_parameter_space(blocks: np.ndarray, blocks_q: np.ndarray, prior_var: float,
                             noise_var, prior_C: np.ndarray | None = None
                             ) -> tuple[np.ndarray, np.ndarray]:
    """The same two matrices from the parameter-space posterior covariance,
    eq. Hessian: Gamma_post = (F^* Gn^{-1} F + Gp^{-1})^{-1}, then
    Q = Fq Gamma_post F^* Gn^{-1} and Gamma_post(q) = Fq Gamma_post Fq^*
    (dense F and Fq; tiny only)."""
    Nt, Nd, Nm = _dims(blocks)
    A, Aq = dense_F(blocks), dense_F(blocks_q)
    ninv = 1.0 / _noise_diag(noise_var, Nt * Nd)
    H = A.T @ (ninv[:, None] * A) + _prior_inverse(Nt, Nm, prior_var, prior_C)
    post = np.linalg.inv(H)
    return Aq @ post @ A.T * ninv[None, :], Aq @ post @ Aq.T


def posterior_mean(blocks: np.ndarray, prior_var: float, noise_var,
                   d: np.ndarray, K: np.ndarray | None = None,
                   prior_C: np.ndarray | None = None) -> np.ndarray:
    """m_map = Gamma_prior F^* K^{-1} d (zero prior mean; Phases 2 and 4),
    with K^{-1} d from a Cholesky factorisation (LAPACK potrf/potrs) and
    Gamma_prior = prior_var (I (x) C): C on every time slice."""
    Nt, Nd, _ = _dims(blocks)
    if K is None:
        K = hessian_gram(blocks, prior_var, noise_var, prior_C)
    d = np.asarray(d, dtype=np.float64)
    rhs = d.reshape(-1, Nt * Nd).T
    x = scipy.linalg.cho_solve(scipy.linalg.cho_factor(K, lower=True), rhs)
    x = x.T.reshape(d.shape)
    m = prior_var * apply_Fadj(blocks, x)
    return m if prior_C is None else m @ prior_C.T


def _prior_inverse(Nt: int, Nm: int, prior_var: float, prior_C) -> np.ndarray:
    """Gamma_prior^{-1} = (I_Nt (x) C^{-1}) / prior_var, dense."""
    Ci = np.eye(Nm) if prior_C is None else np.linalg.inv(prior_C)
    return np.kron(np.eye(Nt), Ci) / prior_var


def prior_grid_matrix(nx: int, ny: int, radius: int, length: float,
                      delta: float) -> np.ndarray:
    """The spatial prior covariance C on an nx x ny parameter grid
    (p = ix ny + iy): C = delta I + B B with B x[ix, iy] =
    sum_{|a|,|b|<=radius} w_a w_b x[ix+a, iy+b], w_a = exp(-a^2/(2 length^2)),
    zero outside the grid (a synthetic smooth SPD stand-in for the paper's
    Matern-type prior, which needs a mesh)."""
    w = np.exp(-np.arange(radius + 1) ** 2 / (2.0 * length ** 2))

    def window(n):
        Wn = np.zeros((n, n))
        for i in range(n):
            for j in range(max(0, i - radius), min(n, i + radius + 1)):
                Wn[i, j] = w[abs(i - j)]
        return Wn
    B = np.kron(window(nx), window(ny))
    return delta * np.eye(nx * ny) + B @ B


def posterior_mean_normal_eq(blocks: np.ndarray, prior_var: float, noise_var,
                             d: np.ndarray, prior_C: np.ndarray | None = None) -> np.ndarray:
    """m_map from the parameter-space normal equations, eq. mmap-problem:
    (F^* Gn^{-1} F + Gp^{-1}) m = F^* Gn^{-1} d (zero prior mean).  Tiny only."""
    Nt, Nd, Nm = _dims(blocks)
    A = dense_F(blocks)
    ninv = 1.0 / _noise_diag(noise_var, Nt * Nd)
    H = A.T @ (ninv[:, None] * A) + _prior_inverse(Nt, Nm, prior_var, prior_C)
    rhs = A.T @ (ninv * np.asarray(d, dtype=np.float64).reshape(-1))
    return np.linalg.solve(H, rhs).reshape(Nt, Nm)


def misfit_gradient(blocks: np.ndarray, m: np.ndarray, d: np.ndarray) -> np.ndarray:
    """Gradient of 0.5 ||F m - d||^2 with respect to m: F^*(F m - d)."""
    return apply_Fadj(blocks, apply_F(blocks, m) - d)


def map_objective_gradient(blocks: np.ndarray, prior_var: float, noise_var,
                           d: np.ndarray, m: np.ndarray) -> np.ndarray:
    """Gradient of the MAP objective of section "State of the art" with zero
    prior mean: F^* Gn^{-1}(F m - d) + Gp^{-1} m.  Zero at m_map."""
    Nt, Nd, _ = _dims(blocks)
    ninv = 1.0 / _noise_diag(noise_var, Nt * Nd).reshape(Nt, Nd)
    return apply_Fadj(blocks, ninv * (apply_F(blocks, m) - d)) + m / prior_var
