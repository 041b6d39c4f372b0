"""Seeded synthetic inputs for the p2o map: the only code the oracle and the
HIP product path both use.

Nothing here computes any part of the method (no transform, no block
product, no Hessian): it only draws numbers.  Every value is a pure function
of (seed, array id, flat index), so any single entry of a huge array can be
regenerated on the host without materialising the array.

Generator (counter-based, from published definitions):

* SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
  generators", OOPSLA 2014).  The stream key is
  ``K = mix64(seed * G + array_id)`` and draw ``n`` of the stream is
  ``mix64(K + (n + 1) * G)`` with ``G = 0x9E3779B97F4A7C15`` and ``mix64``
  the SplitMix64 output finaliser; all arithmetic is modulo 2**64.
* Box-Muller (1958), cosine branch only: entry ``n`` takes draws ``2n`` and
  ``2n+1``; ``u1 = ((a >> 11) + 1) * 2**-53`` lies in (0, 1],
  ``u2 = (b >> 11) * 2**-53`` in [0, 1), and
  ``z = sqrt(-2 ln u1) * cos(2 pi u2)``.

The device implementation (``csrc/synth.hip``) evaluates the same
definition; the two may differ in the last bit of ``log``/``cos``
(host libm versus the device math library), i.e. by about 1e-16 relative.

Input recipes (seed = workload index; array ids blocks=1, m=2, d=3, noise=4,
direction=5, instance shapes=6):

* blocks ``F_k[s, p] = z((k*Nd + s)*Nm + p) * env[k]`` with
  ``env[k] = exp(-k / tau) * amp``.  The envelope table is computed once on
  the host and shipped to the device, so both sides scale by the same
  doubles.
* vectors ``v[n] = z(offset + n) * scale``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

ARRAY_BLOCKS = 1
ARRAY_M = 2
ARRAY_D = 3
ARRAY_NOISE = 4
ARRAY_DIRECTION = 5
ARRAY_SHAPES = 6
# The p2q map's blocks are drawn like the p2o map's (array id ARRAY_BLOCKS)
# under the workload seed plus this offset.
QOI_SEED_OFFSET = 7919


_CHUNK = 1 << 20


def _mix64_inplace(z: np.ndarray, t: np.ndarray) -> None:
    """SplitMix64 output finaliser applied in place (t: scratch of same size)."""
    np.right_shift(z, np.uint64(30), out=t)
    np.bitwise_xor(z, t, out=z)
    np.multiply(z, _M1, out=z)
    np.right_shift(z, np.uint64(27), out=t)
    np.bitwise_xor(z, t, out=z)
    np.multiply(z, _M2, out=z)
    np.right_shift(z, np.uint64(31), out=t)
    np.bitwise_xor(z, t, out=z)


def stream_key(seed: int, array_id: int) -> np.uint64:
    z = np.array([(seed * 0x9E3779B97F4A7C15 + array_id) % (1 << 64)],
                 dtype=np.uint64)
    _mix64_inplace(z, np.empty_like(z))
    return z[0]


def _normals_flat(key: np.uint64, idx: np.ndarray, out: np.ndarray) -> None:
    """out[i] = z(idx[i]) for 1-D uint64 idx; works in chunks to limit temporaries."""
    n = idx.shape[0]
    a = np.empty(min(n, _CHUNK), dtype=np.uint64)
    b = np.empty_like(a)
    t = np.empty_like(a)
    u1 = np.empty(a.shape, dtype=np.float64)
    u2 = np.empty_like(u1)
    for c0 in range(0, n, _CHUNK):
        c1 = min(n, c0 + _CHUNK)
        m = c1 - c0
        A, B, T, U1, U2 = a[:m], b[:m], t[:m], u1[:m], u2[:m]
        # draw 2n is mix64(key + (2n+1)G), draw 2n+1 is mix64(key + (2n+2)G)
        np.multiply(idx[c0:c1], np.uint64(2), out=A)
        np.add(A, np.uint64(1), out=A)
        np.multiply(A, GOLDEN, out=A)
        np.add(A, key, out=A)
        np.add(A, GOLDEN, out=B)
        _mix64_inplace(A, T)
        _mix64_inplace(B, T)
        np.right_shift(A, np.uint64(11), out=A)
        np.add(A, np.uint64(1), out=A)
        np.right_shift(B, np.uint64(11), out=B)
        U1[:] = A
        U2[:] = B
        np.multiply(U1, 2.0**-53, out=U1)
        np.multiply(U2, 2.0**-53, out=U2)
        np.log(U1, out=U1)
        np.multiply(U1, -2.0, out=U1)
        np.sqrt(U1, out=U1)
        np.multiply(U2, 2.0 * np.pi, out=U2)
        np.cos(U2, out=U2)
        np.multiply(U1, U2, out=out[c0:c1])


def normals(seed: int, array_id: int, idx) -> np.ndarray:
    """Standard normals for flat entry indices ``idx`` (any int array shape)."""
    idx = np.asarray(idx)
    flat = np.ascontiguousarray(idx.reshape(-1)).astype(np.uint64, copy=False)
    out = np.empty(flat.shape[0], dtype=np.float64)
    _normals_flat(stream_key(seed, array_id), flat, out)
    return out.reshape(idx.shape)


def uniform_ints(seed: int, array_id: int, n: int, lo: int, hi: int,
                 offset: int = 0) -> np.ndarray:
    """Integers uniform on lo..hi inclusive from draws offset..offset+n-1:
    draw mod (hi - lo + 1), plus lo."""
    key = stream_key(seed, array_id)
    z = (np.arange(offset, offset + n, dtype=np.uint64) + np.uint64(1)) * GOLDEN + key
    _mix64_inplace(z, np.empty_like(z))
    return (z % np.uint64(hi - lo + 1)).astype(np.int64) + lo


def envelope(Nt: int, tau: float, amp: float = 1.0) -> np.ndarray:
    """Per-step amplitude ``exp(-k/tau) * amp`` of the synthetic blocks."""
    return np.exp(-np.arange(Nt, dtype=np.float64) / tau) * amp


def blocks(seed: int, Nd: int, Nm: int, Nt: int, env: np.ndarray,
           k=None, s=None, p=None) -> np.ndarray:
    """Block entries ``F_k[s, p]`` as a [len(k)][len(s)][len(p)] float64 array.

    ``k``, ``s``, ``p`` select index subsets (default: all), so single rows
    or columns of a workload far larger than host memory can be drawn.
    """
    k = np.arange(Nt) if k is None else np.atleast_1d(np.asarray(k))
    s = np.arange(Nd) if s is None else np.atleast_1d(np.asarray(s))
    p = np.arange(Nm) if p is None else np.atleast_1d(np.asarray(p))
    out = np.empty((len(k), len(s), len(p)), dtype=np.float64)
    for a, kk in enumerate(k):
        flat = ((np.int64(kk) * Nd + s.astype(np.int64))[:, None] * Nm
                + p.astype(np.int64)[None, :])
        out[a] = normals(seed, ARRAY_BLOCKS, flat) * env[kk]
    return out


def vector(seed: int, array_id: int, n: int, offset: int = 0,
           scale: float = 1.0) -> np.ndarray:
    """``n`` consecutive normals starting at flat index ``offset``, times ``scale``."""
    return normals(seed, array_id, np.arange(offset, offset + n, dtype=np.int64)) * scale


# ----------------------------------------------------------------------------
# Device generator (for workloads too large to draw on the host).
# ----------------------------------------------------------------------------
_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libp2o_synth.so")
_lib = None


def load_device_library():
    """Load the device generator; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} missing: run __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        lib.synth_blocks_f64.restype = ctypes.c_int
        lib.synth_blocks_f64.argtypes = [
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
            ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p,
            ctypes.c_void_p]
        lib.synth_normals_f64.restype = ctypes.c_int
        lib.synth_normals_f64.argtypes = [
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
            ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p]
        _lib = lib
    return _lib


def device_blocks(out_ptr: int, Nt: int, Nd: int, Nm: int, p0: int, p1: int,
                  seed: int, env_dev_ptr: int, stream: int) -> None:
    """Write blocks F_k[s, p0:p1] into device buffer [Nt][Nd][p1-p0]."""
    rc = load_device_library().synth_blocks_f64(
        out_ptr, Nt, Nd, Nm, p0, p1, seed, env_dev_ptr, stream)
    if rc != 0:
        raise RuntimeError(f"synth_blocks_f64 failed with HIP error {rc}")


def device_normals(out_ptr: int, n: int, offset: int, seed: int, array_id: int,
                   scale: float, stream: int) -> None:
    rc = load_device_library().synth_normals_f64(
        out_ptr, n, offset, seed, array_id, scale, stream)
    if rc != 0:
        raise RuntimeError(f"synth_normals_f64 failed with HIP error {rc}")
