// Setup-time encoding of the frequency blocks for the mixed-precision
// paths.  Each real component v of a block entry is stored as two 16-bit
// terms with a shared power-of-two float32 scale s per sub-block
// (frequency k, 256 consecutive columns p, all rows s):
//
//   v ~= s * (hi + lo * c),   hi = round16(v / s),
//                             lo = round16((v / s - hi) / c),
//
// with c = 2^-11 for binary16 (so lo uses the full binary16 range) and c = 1
// for bfloat16 (whose exponent range needs no rescaling).  s is chosen so
// that the largest |v / s| of the sub-block lies in [2^14, 2^15) for
// binary16 (in range with head room for the rounding of hi) and in
// [0.5, 1) for bfloat16.  Because s is a power of two, dividing by it is
// exact and the stored pair differs from v only by the rounding of lo:
// about 2^-22 |v| (binary16) or 2^-16 |v| (bfloat16).  Rounding is to
// nearest even at each narrowing (float64 -> float32 -> 16 bit).
#include <cmath>

#include "p2o_internal.h"

namespace p2o {
namespace {

__device__ __forceinline__ uint32_t to_fp16_bits(double v) {
  const _Float16 h = (_Float16)(float)v;
  unsigned short u;
  __builtin_memcpy(&u, &h, 2);
  return u;
}

__device__ __forceinline__ uint32_t to_bf16_bits(double v) {
  const uint32_t u = __float_as_uint((float)v);
  // round to nearest even on the 16 dropped bits (finite inputs)
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ double from_fp16_bits(uint32_t u) {
  _Float16 h;
  const unsigned short s = (unsigned short)u;
  __builtin_memcpy(&h, &s, 2);
  return (double)(float)h;
}

__device__ __forceinline__ double from_bf16_bits(uint32_t u) {
  return (double)__uint_as_float(u << 16);
}

// grid: (tiles in this chunk, nf); block 256 threads.
__global__ void __launch_bounds__(256)
quantise_kernel(const cpx<double>* __restrict__ chunk, int64_t nf, int64_t Nd,
                int64_t Nm, int64_t p0, int64_t pc, void* __restrict__ Araw,
                float* __restrict__ scales, int fmt, int use_lo) {
  __shared__ double red[256];
  const int64_t tile = blockIdx.x;  // tile within the chunk
  const int64_t k = blockIdx.y;
  const int64_t q0 = tile * kScaleTile;           // column offset in chunk
  const int64_t qn = min((int64_t)kScaleTile, pc - q0);
  const int tid = threadIdx.x;

  // thread tid owns column q0 + tid of the tile and walks the rows
  double mx = 0.0;
  if (tid < qn)
    for (int64_t s = 0; s < Nd; ++s) {
      const cpx<double> v = chunk[(k * Nd + s) * pc + q0 + tid];
      mx = fmax(mx, fmax(fabs(v.x), fabs(v.y)));
    }
  red[tid] = mx;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) red[tid] = fmax(red[tid], red[tid + off]);
    __syncthreads();
  }
  mx = red[0];
  int e = 0;
  if (mx > 0.0) frexp(mx, &e);  // mx in [2^(e-1), 2^e)
  int se = (fmt == (int)Fmt16::FP16) ? e - 15 : e;
  se = max(-120, min(120, se));
  const double inv_s = ldexp(1.0, -se);
  const double lo_mul = (fmt == (int)Fmt16::FP16) ? 2048.0 : 1.0;
  const int64_t ntiles = (Nm + kScaleTile - 1) / kScaleTile;
  if (tid == 0) scales[k * ntiles + (p0 + q0) / kScaleTile] = ldexpf(1.0f, se);

  if (tid >= qn) return;
  const int64_t q = tid;
  for (int64_t s = 0; s < Nd; ++s) {
    const cpx<double> v = chunk[(k * Nd + s) * pc + q0 + q];
    const double vr = v.x * inv_s, vi = v.y * inv_s;
    uint32_t hr, hi, lr = 0, li = 0;
    double rr, ri;
    if (fmt == (int)Fmt16::FP16) {
      hr = to_fp16_bits(vr);
      hi = to_fp16_bits(vi);
      rr = vr - from_fp16_bits(hr);
      ri = vi - from_fp16_bits(hi);
      if (use_lo) {
        lr = to_fp16_bits(rr * lo_mul);
        li = to_fp16_bits(ri * lo_mul);
      }
    } else {
      hr = to_bf16_bits(vr);
      hi = to_bf16_bits(vi);
      rr = vr - from_bf16_bits(hr);
      ri = vi - from_bf16_bits(hi);
      if (use_lo) {
        lr = to_bf16_bits(rr * lo_mul);
        li = to_bf16_bits(ri * lo_mul);
      }
    }
    const int64_t idx = (k * Nd + s) * Nm + p0 + q0 + q;
    const uint32_t hw = hr | (hi << 16);
    if (use_lo)
      static_cast<uint2*>(Araw)[idx] = make_uint2(hw, lr | (li << 16));
    else
      static_cast<uint32_t*>(Araw)[idx] = hw;
  }
}

}  // namespace

hipError_t launch_quantise(const cpx<double>* chunk, int64_t nf, int64_t Nd,
                           int64_t Nm, int64_t p0, int64_t pc, void* A,
                           float* scales, Fmt16 fmt, bool use_lo,
                           hipStream_t s) {
  if (pc < 1) return hipSuccess;
  const int64_t tiles = (pc + kScaleTile - 1) / kScaleTile;
  if (nf > 65535) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(quantise_kernel, dim3((unsigned)tiles, (unsigned)nf), dim3(256), 0, s,
                     chunk, nf, Nd, Nm, p0, pc, (void*)A, scales, (int)fmt,
                     use_lo ? 1 : 0);
  return hipGetLastError();
}

}  // namespace p2o
