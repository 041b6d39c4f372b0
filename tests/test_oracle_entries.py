"""Pins for the oracle's one-output forms F_entry and Fadj_entry, which are
the checkers of the full-size GPU tests (where the blocks do not fit in host
memory and outputs are computed one at a time).

They are pinned against facts other than themselves: the hand-worked
integer example (exact), the scalar case (textbook causal convolution,
np.convolve) and, at every output (t, s) / (t, p) of three shapes including
t = 0 and t = Nt - 1, the whole-vector oracle apply_F / apply_Fadj, which
carries its own pins (dense matrix, golden, convolution, adjoint identity,
FFT route).  Planted mistakes (a dropped diagonal block, an off-by-one
delay, a missing last term) must fail these pins.
"""
import os

import numpy as np
import pytest

from oracle import p2o_oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
SHAPES = [(1, 2, 3), (7, 3, 5), (13, 4, 2), (6, 1, 1)]  # (Nt, Nd, Nm)


def _golden():
    vals = {}
    with open(os.path.join(HERE, "golden", "hand_example.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                key, *rest = line.split()
                vals[key] = np.array([float(x) for x in rest])
    return vals


def check_entries_golden(F_entry, Fadj_entry):
    """Hand-worked integer example (section "FFT-based Hessian matvecs", eq.
    ShiftInvariance): every entry of d = F m and of F^T d exactly."""
    g = _golden()
    Nd, Nm, Nt = int(g["Nd"][0]), int(g["Nm"][0]), int(g["Nt"][0])
    blocks = np.stack([g[f"F{k}"].reshape(Nd, Nm) for k in range(Nt)])
    m = np.stack([g[f"m{j}"] for j in range(Nt)])
    d = g["d"].reshape(Nt, Nd)
    ftd = g["Ftd"].reshape(Nt, Nm)
    for t in range(Nt):
        for s in range(Nd):
            assert F_entry(blocks[:, s, :], m, t) == d[t, s], (t, s)
        for p in range(Nm):
            assert Fadj_entry(blocks[:, :, p], d, t) == ftd[t, p], (t, p)


def check_entries_convolve(F_entry, Fadj_entry, rng):
    """Nd = Nm = 1: d = np.convolve(f, m)[:Nt]; F^T d is the correlation
    (F^T d)_j = sum_{i>=j} f_{i-j} d_i = np.correlate(d, f, 'full') read at
    lag j."""
    for Nt in (1, 2, 9):
        f = rng.standard_normal(Nt)
        m = rng.standard_normal(Nt)
        d = rng.standard_normal(Nt)
        conv = np.convolve(f, m)[:Nt]
        corr = np.correlate(d, f, "full")[Nt - 1:]
        for t in range(Nt):
            got = F_entry(f.reshape(Nt, 1), m.reshape(Nt, 1), t)
            assert abs(got - conv[t]) <= 1e-13 * (1 + abs(conv[t])), (Nt, t)
            gota = Fadj_entry(f.reshape(Nt, 1), d.reshape(Nt, 1), t)
            assert abs(gota - corr[t]) <= 1e-13 * (1 + abs(corr[t])), (Nt, t)


def check_entries_everywhere(F_entry, Fadj_entry, rng):
    """Every output of three shapes against the whole-vector oracle."""
    for Nt, Nd, Nm in SHAPES:
        b = rng.standard_normal((Nt, Nd, Nm)) * np.exp(-np.arange(Nt) / 4.0)[:, None, None]
        m = rng.standard_normal((Nt, Nm))
        d = rng.standard_normal((Nt, Nd))
        yF = O.apply_F(b, m)
        yA = O.apply_Fadj(b, d)
        for t in range(Nt):
            for s in range(Nd):
                ref = yF[t, s]
                assert abs(F_entry(b[:, s, :], m, t) - ref) <= 1e-13 * (1 + abs(ref)), (t, s)
            for p in range(Nm):
                ref = yA[t, p]
                assert abs(Fadj_entry(b[:, :, p], d, t) - ref) <= 1e-13 * (1 + abs(ref)), (t, p)


def test_entries_golden():
    check_entries_golden(O.F_entry, O.Fadj_entry)


def test_entries_scalar_convolution():
    check_entries_convolve(O.F_entry, O.Fadj_entry, np.random.default_rng(31))


def test_entries_match_whole_vector_oracle():
    check_entries_everywhere(O.F_entry, O.Fadj_entry, np.random.default_rng(32))


# ----------------------------------------------------- planted mistakes
def _F_entry_no_diagonal(rows_s, m, i):        # forgets F_0 (j = i)
    return sum(float(rows_s[i - j] @ m[j]) for j in range(i))


def _F_entry_delayed(rows_s, m, i):            # uses F_{i-j-1}
    return sum(float(rows_s[i - j - 1] @ m[j]) for j in range(i))


def _Fadj_entry_no_last(cols_p, d, j):         # stops one step early
    Nt = d.shape[0]
    return sum(float(cols_p[i - j] @ d[i]) for i in range(j, Nt - 1))


def _Fadj_entry_lower(cols_p, d, j):           # sums i <= j (a lower-triangular "adjoint")
    return sum(float(cols_p[j - i] @ d[i]) for i in range(j + 1))


@pytest.mark.parametrize("mutant", [_F_entry_no_diagonal, _F_entry_delayed])
def test_mutant_F_entry_is_caught(mutant):
    with pytest.raises(AssertionError):
        check_entries_golden(mutant, O.Fadj_entry)
    with pytest.raises(AssertionError):
        check_entries_convolve(mutant, O.Fadj_entry, np.random.default_rng(33))
    with pytest.raises(AssertionError):
        check_entries_everywhere(mutant, O.Fadj_entry, np.random.default_rng(34))


@pytest.mark.parametrize("mutant", [_Fadj_entry_no_last, _Fadj_entry_lower])
def test_mutant_Fadj_entry_is_caught(mutant):
    with pytest.raises(AssertionError):
        check_entries_golden(O.F_entry, mutant)
    with pytest.raises(AssertionError):
        check_entries_convolve(O.F_entry, mutant, np.random.default_rng(35))
    with pytest.raises(AssertionError):
        check_entries_everywhere(O.F_entry, mutant, np.random.default_rng(36))
