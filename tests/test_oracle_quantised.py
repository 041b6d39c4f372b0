"""Pins for the quantised-spectrum oracle (oracle/quantised.py), against facts
other than itself:
  * the rounding to binary16 equals numpy's float16 conversion (a library
    routine, round to nearest even, subnormals included); the rounding to
    bfloat16 equals a brute-force nearest search over all finite bfloat16
    values (ties to the even bit pattern);
  * the scale of every (frequency, 256-column) sub-block puts its largest
    component in the documented range;
  * spectra that are exactly representable as s (hi + c lo) come back bit
    for bit;
  * every decoded entry is within the encoding's rounding bound of the
    input: 2^-16 |v| (bfloat16 hi+lo), 2^-22 |v| (binary16 hi+lo), 2^-8 |v|
    (bfloat16 hi only), up to the float32 and subnormal terms derived below;
  * the spectral route with unquantised spectra equals the time-domain
    definition (eq. ShiftInvariance) for every exact embedding length and
    aliases for a short one.
Each pin is also run against a copy with one planted mistake.
"""
import numpy as np
import pytest

from oracle import p2o_oracle as O
from oracle import quantised as Q


def _blocks(rng, Nt, Nd, Nm, tau):
    return rng.standard_normal((Nt, Nd, Nm)) * np.exp(-np.arange(Nt) / tau)[:, None, None]


# ------------------------------------------------------------------ rounding
def check_round_fp16(round_fn, rng):
    """float32 inputs over the binary16 range (normal, subnormal, exact ties)."""
    x = np.concatenate([
        rng.standard_normal(20000) * 10.0 ** rng.uniform(-8, 4, 20000),
        rng.uniform(-6.1e-5, 6.1e-5, 5000),                    # subnormal range
    ]).astype(np.float32)
    h = rng.standard_normal(5000).astype(np.float16)            # exact midpoints
    up = np.nextafter(h, np.float16(np.inf))
    ties = ((h.astype(np.float64) + up.astype(np.float64)) / 2).astype(np.float32)
    x = np.concatenate([x, ties, -ties]).astype(np.float64)
    x = x[np.abs(x) < 65000]
    ref = x.astype(np.float16).astype(np.float64)
    np.testing.assert_array_equal(round_fn(x, "fp16"), ref)


def _bf16_grid():
    bits = np.arange(0, 0x7f80, dtype=np.uint32)               # finite non-negative
    return (bits << 16).view(np.float32).astype(np.float64), bits


def check_round_bf16(round_fn, rng):
    grid, bits = _bf16_grid()
    x = np.concatenate([
        rng.standard_normal(20000) * 10.0 ** rng.uniform(-30, 30, 20000),
        (grid[1000:6000] + grid[1001:6001]) / 2,               # exact midpoints
        grid[20000:20500],                                     # representable values
    ]).astype(np.float32).astype(np.float64)
    a = np.abs(x)
    j = np.clip(np.searchsorted(grid, a), 1, len(grid) - 1)
    lo, hi = grid[j - 1], grid[j]
    pick_hi = (hi - a < a - lo) | ((hi - a == a - lo) & (bits[j] % 2 == 0))
    ref = np.where(pick_hi, hi, lo) * np.sign(x)
    exact = a == hi
    ref[exact] = x[exact]
    np.testing.assert_array_equal(round_fn(x, "bf16"), ref)


def test_round_fp16_matches_numpy_float16():
    check_round_fp16(Q.r16, np.random.default_rng(41))


def test_round_bf16_matches_brute_force_nearest():
    check_round_bf16(Q.r16, np.random.default_rng(42))


def _r16_truncating(x, fmt):          # planted: chops instead of rounding
    p, emin = Q.FORMATS[fmt]
    f32 = np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)
    _, E = np.frexp(f32)
    sp = np.ldexp(1.0, np.maximum(E - 1, emin) - (p - 1))
    return np.trunc(f32 / sp) * sp


def _r16_ties_away(x, fmt):           # planted: ties away from zero
    p, emin = Q.FORMATS[fmt]
    f32 = np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)
    _, E = np.frexp(f32)
    sp = np.ldexp(1.0, np.maximum(E - 1, emin) - (p - 1))
    return np.sign(f32) * np.floor(np.abs(f32) / sp + 0.5) * sp


@pytest.mark.parametrize("mutant", [_r16_truncating, _r16_ties_away])
def test_mutant_rounding_is_caught(mutant):
    with pytest.raises(AssertionError):
        check_round_fp16(mutant, np.random.default_rng(43))
    with pytest.raises(AssertionError):
        check_round_bf16(mutant, np.random.default_rng(44))


# ------------------------------------------------------------------ encoding
def check_scale_rule(scale_fn, rng):
    """Largest component of each sub-block in [0.5, 1) (bfloat16) or
    [2^14, 2^15) (binary16) after division by its scale."""
    fhat = Q.spectra(_blocks(rng, 9, 3, 700, 3.0), 18)
    fhat[2, :, 256:512] *= 1e-9                                # tiles of very different size
    fhat[4, :, 512:] = 0                                       # an all-zero ragged tile
    mag = np.maximum(np.abs(fhat.real), np.abs(fhat.imag))
    for fmt, (lo, hi) in (("bf16", (0.5, 1.0)), ("fp16", (2.0 ** 14, 2.0 ** 15))):
        e = scale_fn(fhat, fmt)
        assert e.shape == (fhat.shape[0], 3)
        for k in range(fhat.shape[0]):
            for t in range(3):
                M = mag[k, :, t * 256:(t + 1) * 256].max()
                if M == 0:
                    assert e[k, t] == np.clip(Q.SCALE_SHIFT[fmt], -120, 120)
                else:
                    assert lo <= M / 2.0 ** e[k, t] < hi, (fmt, k, t)


def _scale_per_frequency(fhat, fmt, tile=Q.TILE):   # planted: one scale per frequency
    nt = (fhat.shape[2] + tile - 1) // tile
    M = np.maximum(np.abs(fhat.real), np.abs(fhat.imag)).max(axis=(1, 2))
    _, E = np.frexp(M)
    return np.repeat((E + Q.SCALE_SHIFT[fmt])[:, None], nt, axis=1)


def test_scale_rule():
    check_scale_rule(Q.scale_exponents, np.random.default_rng(45))


def test_mutant_scale_rule_is_caught():
    with pytest.raises(AssertionError):
        check_scale_rule(_scale_per_frequency, np.random.default_rng(46))


def _representable(rng, fmt, nf=3, Nd=4, Nm=300):
    """Spectra exactly of the form s (hi + c lo): 16-bit hi with the
    sub-block maximum in the scale's range, lo at least 2 binades below hi's
    last bit (so r16(hi + c lo) = hi) and within float32's 24 bits of it."""
    p, _ = Q.FORMATS[fmt]
    c = Q.LO_FACTOR[fmt]
    top = {"bf16": 0.0, "fp16": 15.0}[fmt]
    out = np.zeros((nf, Nd, Nm), dtype=complex)
    for part in (1.0, 1j):
        ehi = rng.integers(-6, 0, (nf, Nd, Nm)) + top                 # hi in [2^(ehi-1), 2^ehi)
        hi = np.ldexp(rng.integers(2 ** (p - 1), 2 ** p, (nf, Nd, Nm)), (ehi - p).astype(int))
        hi *= rng.choice([-1.0, 1.0], (nf, Nd, Nm))
        elo = ehi - p - 1 - rng.integers(0, 24 - 2 * p, (nf, Nd, Nm))  # lo's leading bit
        lo = np.ldexp(rng.integers(2 ** (p - 1), 2 ** p, (nf, Nd, Nm)), (elo - p).astype(int))
        lo *= rng.choice([-1.0, 1.0], (nf, Nd, Nm))
        out += part * (hi + lo)
    out[:, 0, ::Q.TILE] = (2.0 ** top * (1 - 2.0 ** -p)) * (1 + 1j)   # pins each tile's maximum
    e = rng.integers(-30, 30, (nf, (Nm + Q.TILE - 1) // Q.TILE))
    s = np.repeat(np.ldexp(1.0, e), Q.TILE, axis=1)[:, :Nm]
    del c
    return out * s[:, None, :]


def check_exact_when_representable(qs_fn, rng):
    for fmt in ("bf16", "fp16"):
        v = _representable(rng, fmt)
        np.testing.assert_array_equal(qs_fn(v, fmt, True), v)


def check_error_bounds(qs_fn, rng):
    """Derivation (x = v/s, exact; u = 2^-p of the 16-bit format):
    hi = r16(x) with |hi - x| <= (u + 2^-24)|x|; r = x - hi is exact in
    float64 (hi and x within a factor of 2, Sterbenz); lo = r16(r / c) and
    the decoded x' = hi + c lo has |x' - x| = c |lo - r/c| <= (u + 2^-24)|r|
    plus half the 16-bit subnormal spacing.  So
      |v' - v| <= (u + 2^-24)^2 |v| + s c 2^(emin - p)."""
    b = _blocks(rng, 11, 5, 600, 4.0)
    fhat = Q.spectra(b, 22)
    for fmt in ("bf16", "fp16"):
        p, emin = Q.FORMATS[fmt]
        u = 2.0 ** -p
        e = Q.scale_exponents(fhat, fmt)
        s = np.repeat(np.ldexp(1.0, e), Q.TILE, axis=1)[:, :600][:, None, :]
        deq = qs_fn(fhat, fmt, True)
        for a, r in ((deq.real, fhat.real), (deq.imag, fhat.imag)):
            bound = (u + 2.0 ** -24) ** 2 * np.abs(r) + s * Q.LO_FACTOR[fmt] * 2.0 ** (emin - p)
            assert np.all(np.abs(a - r) <= bound), fmt
            assert np.abs(a - r).max() > 0                       # the encoding is not the identity
    # hi only (bfloat16): |v' - v| <= (2^-8 + 2^-24)|v| + s 2^-134
    e = Q.scale_exponents(fhat, "bf16")
    s = np.repeat(np.ldexp(1.0, e), Q.TILE, axis=1)[:, :600][:, None, :]
    deq = qs_fn(fhat, "bf16", False)
    for a, r in ((deq.real, fhat.real), (deq.imag, fhat.imag)):
        assert np.all(np.abs(a - r) <= (2.0 ** -8 + 2.0 ** -24) * np.abs(r) + s * 2.0 ** -134)


def _qs_no_residual(fhat, fmt, use_lo=True):        # planted: lo encodes v/s, not v/s - hi
    e = Q.scale_exponents(fhat, fmt)
    s = np.repeat(np.ldexp(1.0, e), Q.TILE, axis=1)[:, : fhat.shape[2]][:, None, :]
    x = fhat / s
    out = 0
    for part, comp in ((1.0, x.real), (1j, x.imag)):
        hi = Q.r16(comp, fmt)
        lo = Q.r16(comp / Q.LO_FACTOR[fmt], fmt) if use_lo else 0.0
        out = out + part * (hi + Q.LO_FACTOR[fmt] * lo)
    return s * out


def _qs_wrong_lo_factor(fhat, fmt, use_lo=True):    # planted: binary16 lo without its 2^11
    if fmt != "fp16":
        return Q.quantised_spectra(fhat, fmt, use_lo)
    hi, lo, e = Q.encode(fhat, fmt, use_lo)
    s = np.repeat(np.ldexp(1.0, e), Q.TILE, axis=1)[:, : fhat.shape[2]][:, None, :]
    return s * (hi + lo)


def _qs_dropped_imag_lo(fhat, fmt, use_lo=True):    # planted: lo of the imaginary part lost
    hi, lo, e = Q.encode(fhat, fmt, use_lo)
    return Q.decode(hi, lo.real + 0j, e, fmt)


def test_encoding_exact_when_representable():
    check_exact_when_representable(Q.quantised_spectra, np.random.default_rng(47))


def test_encoding_error_bounds():
    check_error_bounds(Q.quantised_spectra, np.random.default_rng(48))


@pytest.mark.parametrize("mutant", [_qs_no_residual, _qs_wrong_lo_factor, _qs_dropped_imag_lo])
def test_mutant_encoding_is_caught(mutant):
    caught = 0
    for check, seed in ((check_exact_when_representable, 49), (check_error_bounds, 50)):
        try:
            check(mutant, np.random.default_rng(seed))
        except AssertionError:
            caught += 1
    assert caught >= 1


# ------------------------------------------------------------ spectral route
def check_spectral_route(FS, FAS, rng):
    """Unquantised spectra: equal to the time-domain definition for L = 2Nt,
    2Nt - 1 and a 7-smooth length; L = 2Nt - 2 aliases (O(1) error)."""
    Nt, Nd, Nm = 11, 3, 5
    b = _blocks(rng, Nt, Nd, Nm, 4.0)
    m = rng.standard_normal((2, Nt, Nm))
    d = rng.standard_normal((2, Nt, Nd))
    refF, refA = O.apply_F(b, m), O.apply_Fadj(b, d)
    for L in (2 * Nt, 2 * Nt - 1, 28):
        fh = Q.spectra(b, L)
        np.testing.assert_allclose(FS(fh, m, L), refF, rtol=0, atol=1e-13 * np.abs(refF).max())
        np.testing.assert_allclose(FAS(fh, d, L), refA, rtol=0, atol=1e-13 * np.abs(refA).max())
    L = 2 * Nt - 2
    fh = Q.spectra(b, L)
    assert np.abs(FS(fh, m, L) - refF).max() > 1e-3 * np.abs(refF).max()


def _FAS_no_conj(fhat, d, L):                      # planted: F^_k^T instead of F^_k^H
    return Q.apply_Fadj_spectral(fhat.conj(), d, L)


def test_spectral_route_equals_time_domain():
    check_spectral_route(Q.apply_F_spectral, Q.apply_Fadj_spectral, np.random.default_rng(51))


def test_mutant_spectral_adjoint_is_caught():
    with pytest.raises(AssertionError):
        check_spectral_route(Q.apply_F_spectral, _FAS_no_conj, np.random.default_rng(52))


def test_quantised_route_error_sizes():
    """The quantised route differs from the exact map by about the encoding's
    relative error: ~1e-6 (bfloat16 hi+lo), ~1e-8 (binary16 hi+lo), ~1e-3
    (bfloat16 hi only); all well inside the mixed tiers' stated bound 1e-5
    except the hi-only tier."""
    rng = np.random.default_rng(53)
    Nt, Nd, Nm = 16, 6, 700
    b = _blocks(rng, Nt, Nd, Nm, 5.0) / np.sqrt(Nm)
    m = rng.standard_normal((Nt, Nm))
    ref = O.apply_F(b, m)
    fh = Q.spectra(b, 2 * Nt)
    err = {}
    for name, fmt, lo in (("bf16", "bf16", True), ("fp16", "fp16", True), ("bf16_hi", "bf16", False)):
        y = Q.apply_F_spectral(Q.quantised_spectra(fh, fmt, lo), m, 2 * Nt)
        err[name] = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    assert 1e-7 < err["bf16"] < 1e-5
    assert 1e-10 < err["fp16"] < 1e-7
    assert 1e-4 < err["bf16_hi"] < 1e-2
