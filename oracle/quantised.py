"""Quantised-spectrum oracle for the mixed-precision tiers.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The mixed tiers store the frequency blocks F^_k (section "FFT-based Hessian
matvecs": the DFT of the block-circulant embedding block-diagonalises F) as
16-bit terms with a power-of-two scale per sub-block, and then compute in
float32.  This module computes, in float64, what those tiers would return
if their only error were the encoding of F^: the encoded-then-decoded
spectra applied exactly, through the same embedding.  Comparing the GPU's
mixed tiers with it separates the encoding error (fixed by the storage
format) from the float32 arithmetic of the transforms and products.

The encoding written out here is the one the library's C ABI documents for
its mixed precisions (reading R8/R9 of the design notes):
  * one scale s = 2^e per (frequency k, 256 consecutive columns) sub-block,
    over all sensors, chosen from the largest component magnitude M of the
    sub-block (M in [2^(E-1), 2^E)): e = E for bfloat16 (so |v/s| < 1) and
    e = E - 15 for binary16 (so |v/s| < 2^15); e clamped to [-120, 120];
    E = 0 when the sub-block is all zero;
  * each real component v (real and imaginary part separately):
        hi = r16(v / s),   lo = r16((v / s - hi) / c),
        stored value = s (hi + c lo),
    with c = 1 (bfloat16) or 2^-11 (binary16), and r16 rounding to nearest,
    ties to even, first to float32 and then to the 16-bit format;
  * the hi-only tier keeps s hi.

Steps that are library primitives: numpy's float64 -> float32 conversion
(round to nearest even) and numpy.fft for the length-L real transforms.
"""
from __future__ import annotations

import numpy as np

__all__ = ["FORMATS", "round_sig", "r16", "spectra", "scale_exponents",
           "encode", "decode", "quantised_spectra", "apply_F_spectral",
           "apply_Fadj_spectral", "TILE"]

# significand bits (implicit bit included) and smallest normal exponent
FORMATS = {"bf16": (8, -126), "fp16": (11, -14)}
LO_FACTOR = {"bf16": 1.0, "fp16": 2.0 ** -11}
SCALE_SHIFT = {"bf16": 0, "fp16": -15}
TILE = 256


def round_sig(x: np.ndarray, p: int, emin: int) -> np.ndarray:
    """Round float64 values to the nearest number with p significant bits
    whose binary exponent is at least emin (spacing 2^(emin - p + 1) below
    2^emin: the format's subnormal grid), ties to the even multiple of the
    spacing.  No overflow handling: callers keep values in range."""
    x = np.asarray(x, dtype=np.float64)
    _, E = np.frexp(x)                       # |x| in [2^(E-1), 2^E)
    lead = np.maximum(E - 1, emin)           # exponent of the leading bit
    spacing = np.ldexp(1.0, lead - (p - 1))
    return np.rint(x / spacing) * spacing    # rint: half to even; division exact (power of two)


def r16(x: np.ndarray, fmt: str) -> np.ndarray:
    """Round to nearest even: float64 -> float32 -> the 16-bit format."""
    f32 = np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)
    return round_sig(f32, *FORMATS[fmt])


def spectra(blocks: np.ndarray, L: int) -> np.ndarray:
    """F^_k = sum_j F_j exp(-2 pi i j k / L), k = 0 .. L/2: the DFT over time
    of the zero-padded first block column, [L/2 + 1][Nd][Nm] complex."""
    return np.fft.rfft(np.asarray(blocks, dtype=np.float64), n=L, axis=0)


def scale_exponents(fhat: np.ndarray, fmt: str, tile: int = TILE) -> np.ndarray:
    """e[k, t] of the scale 2^e of sub-block (k, columns t*tile .. t*tile+tile-1)."""
    nf, Nd, Nm = fhat.shape
    nt = (Nm + tile - 1) // tile
    e = np.zeros((nf, nt), dtype=np.int64)
    mag = np.maximum(np.abs(fhat.real), np.abs(fhat.imag))
    for t in range(nt):
        M = mag[:, :, t * tile:(t + 1) * tile].max(axis=(1, 2))
        _, E = np.frexp(M)                   # frexp(0) gives E = 0
        e[:, t] = np.clip(E + SCALE_SHIFT[fmt], -120, 120)
    return e


def encode(fhat: np.ndarray, fmt: str, use_lo: bool = True, tile: int = TILE):
    """(hi, lo, e): hi and lo complex arrays of 16-bit values (real and
    imaginary parts encoded separately), e the scale exponents [nf][tiles]."""
    e = scale_exponents(fhat, fmt, tile)
    s = np.repeat(np.ldexp(1.0, e), tile, axis=1)[:, : fhat.shape[2]]  # [nf][Nm]
    x = fhat / s[:, None, :]
    c = LO_FACTOR[fmt]
    parts = []
    for comp in (x.real, x.imag):
        hi = r16(comp, fmt)
        lo = r16((comp - hi) / c, fmt) if use_lo else np.zeros_like(hi)
        parts.append((hi, lo))
    hi = parts[0][0] + 1j * parts[1][0]
    lo = parts[0][1] + 1j * parts[1][1]
    return hi, lo, e


def decode(hi: np.ndarray, lo: np.ndarray, e: np.ndarray, fmt: str, tile: int = TILE):
    """s (hi + c lo) per entry."""
    s = np.repeat(np.ldexp(1.0, e), tile, axis=1)[:, : hi.shape[2]]
    return s[:, None, :] * (hi + LO_FACTOR[fmt] * lo)


def quantised_spectra(fhat: np.ndarray, fmt: str, use_lo: bool = True) -> np.ndarray:
    """The spectra a mixed tier stores, decoded to float64."""
    hi, lo, e = encode(fhat, fmt, use_lo)
    return decode(hi, lo, e, fmt)


def apply_F_spectral(fhat: np.ndarray, m: np.ndarray, L: int) -> np.ndarray:
    """d = F m through the embedding: the length-L DFT of each parameter
    series, one block product per frequency, the inverse DFT truncated to
    the first Nt steps.  m [..., Nt, Nm] -> d [..., Nt, Nd]."""
    m = np.asarray(m, dtype=np.float64)
    Nt = m.shape[-2]
    mh = np.fft.rfft(m, n=L, axis=-2)                      # [..., nf, Nm]
    yh = np.einsum("ksp,...kp->...ks", fhat, mh)
    return np.fft.irfft(yh, n=L, axis=-2)[..., :Nt, :]


def apply_Fadj_spectral(fhat: np.ndarray, d: np.ndarray, L: int) -> np.ndarray:
    """m = F^T d through the embedding: block products with the conjugate
    transposes F^_k^H (the blocks are real).  d [..., Nt, Nd] -> [..., Nt, Nm]."""
    d = np.asarray(d, dtype=np.float64)
    Nt = d.shape[-2]
    dh = np.fft.rfft(d, n=L, axis=-2)
    yh = np.einsum("ksp,...ks->...kp", fhat.conj(), dh)
    return np.fft.irfft(yh, n=L, axis=-2)[..., :Nt, :]
