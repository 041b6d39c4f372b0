// Per-frequency complex block products for many right-hand sides on the
// bfloat16 matrix cores (v_mfma_f32_16x16x32_bf16, float32 accumulation),
// for plans whose frequency blocks are stored as bfloat16 hi (+ lo) terms.
//
// Operand precision.  A block entry is s * (H + Lo) (hi + lo bfloat16 with a
// power-of-two sub-block scale s); a vector entry x (float32) is split as
// x = xh + xl with xh = bf16(x), xl = bf16(x - xh), both rounded to nearest
// even.  Each real product is formed as H xh + H xl + Lo xh (the dropped
// Lo xl is below the representation error of either factor), so a complex
// product costs 12 instructions (8 for the hi-only tier) and keeps about 16
// significant bits in both operands, as the vector-unit kernels do.
//
// MFMA operand layout (16x16x32, bfloat16): lane l supplies the contraction
// slots A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16] (j = 0..7,
// bfloat16x8), accumulator element i of lane l is D[4 (l / 16) + i][l % 16]
// (float32).  Slots map to block entries of a 32-entry chunk, identically
// for both operands: F* uses sensors 8 (l / 16) + j; F interleaves them so
// the 4 lane groups of a block row read one contiguous 64-byte span per
// load, and stages the vector planes in LDS in the same slot order.
//
// F  ("rows"): workgroup = 128 sensors x (16 NT) right-hand sides of one
//    frequency and one column chunk; the column sub-block scales are folded
//    into the vector planes (exact: powers of two), so the chunk accumulates
//    in float32 on the matrix cores.
// F* ("cols"): X^T = Dhat^T conj(Fhat): workgroup = (16 MT) right-hand
//    sides x 128 columns; contraction over all sensors; the column scale is
//    applied to the float32 result.
// Vector operands come pre-split in four bfloat16 planes per (rhs, k):
// [re hi][re lo][im hi][im lo], each padded to a multiple of 8 entries.
#include "product_units.h"

namespace p2o {
namespace {

template <int NT, bool LO, bool VEC>
__global__ void __launch_bounds__(kBf16Threads)
gemm_rows_bf16(const uint32_t* __restrict__ A, const uint16_t* __restrict__ Xs,
               cpx<double>* __restrict__ P, GemvShape g, int64_t n8, int64_t b0, int nb) {
  __shared__ __align__(16) char lds[stage_bytes_bf16(NT)];
  const int64_t tile = xcd_local_tile(blockIdx.x, gridDim.x);
  const int64_t nmt = (g.Nd + kBf16Tile - 1) / kBf16Tile;
  const int64_t rest = tile / nmt;
  const int64_t pc = rest / g.nf;
  if (pc >= g.n_pc) return;  // grid padding: the whole workgroup leaves
  mfma_rows_bf16_wg<NT, LO, VEC>(A, Xs, P, g, n8, b0, nb, rest % g.nf, tile % nmt, pc, lds);
}

template <int MT, bool LO>
__global__ void __launch_bounds__(kBf16Threads)
gemm_cols_bf16(const uint32_t* __restrict__ A, const float* __restrict__ scales,
               const uint16_t* __restrict__ Ds, cpx<float>* __restrict__ Y, GemvShape g,
               int64_t nd8, int64_t b0, int nb) {
  __shared__ __align__(16) char lds[stage_bytes_bf16(MT)];
  const int64_t tile = xcd_local_tile(blockIdx.x, gridDim.x);
  const int64_t npt = (g.Nm + kBf16Tile - 1) / kBf16Tile;
  const int64_t k = tile / npt;
  if (k >= g.nf) return;
  mfma_cols_bf16_wg<MT, LO>(A, scales, Ds, Y, g, nd8, b0, nb, k, tile % npt, lds);
}

__device__ __forceinline__ uint16_t bf16_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// in: [count][n] complex float32 -> out: [count][4][n8] bfloat16 planes
// (re hi, re lo, im hi, im lo), zero in the padding n..n8-1.  With `scales`
// (F's operand), entry e of row c = b * nf + k is first multiplied by the
// power-of-two scale of sub-block (k, e / 256), which is exact.
__global__ void __launch_bounds__(256)
split_bf16(const cpx<float>* __restrict__ in, uint16_t* __restrict__ out, int64_t count,
           int64_t n, int64_t n8, const float* __restrict__ scales, int64_t nf) {
  const int64_t total = count * n8;
  const int64_t ntiles = (n + kScaleTile - 1) / kScaleTile;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = idx / n8, e = idx % n8;
    cpx<float> v = {0.f, 0.f};
    if (e < n) {
      v = in[c * n + e];
      if (scales) {
        const float sc = scales[(c % nf) * ntiles + e / kScaleTile];
        v.x *= sc;
        v.y *= sc;
      }
    }
    const uint16_t rh = bf16_rne(v.x), ih = bf16_rne(v.y);
    const uint16_t rl = bf16_rne(v.x - __uint_as_float((uint32_t)rh << 16));
    const uint16_t il = bf16_rne(v.y - __uint_as_float((uint32_t)ih << 16));
    uint16_t* o = out + c * 4 * n8 + e;
    o[0] = rh;
    o[n8] = rl;
    o[2 * n8] = ih;
    o[3 * n8] = il;
  }
}

unsigned padded_grid(int64_t tiles) { return (unsigned)((tiles + kXcds - 1) / kXcds * kXcds); }

template <bool LO, bool VEC>
hipError_t rows_passes(const uint32_t* A, const uint16_t* Xs, cpx<double>* P,
                       const GemvShape& g, int64_t n8, hipStream_t s) {
  const unsigned grid = padded_grid(((g.Nd + kBf16Tile - 1) / kBf16Tile) * g.nf * g.n_pc);
  for (int64_t b0 = 0; b0 < g.nrhs; b0 += 64) {
    const int nb = (int)std::min<int64_t>(64, g.nrhs - b0);
    if (nb > 32)
      hipLaunchKernelGGL((gemm_rows_bf16<4, LO, VEC>), dim3(grid), dim3(kBf16Threads), 0, s, A, Xs, P, g, n8, b0, nb);
    else if (nb > 16)
      hipLaunchKernelGGL((gemm_rows_bf16<2, LO, VEC>), dim3(grid), dim3(kBf16Threads), 0, s, A, Xs, P, g, n8, b0, nb);
    else
      hipLaunchKernelGGL((gemm_rows_bf16<1, LO, VEC>), dim3(grid), dim3(kBf16Threads), 0, s, A, Xs, P, g, n8, b0, nb);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <bool LO>
hipError_t cols_passes(const uint32_t* A, const float* sc, const uint16_t* Ds,
                       cpx<float>* Y, const GemvShape& g, int64_t nd8, hipStream_t s) {
  const unsigned grid = padded_grid(((g.Nm + kBf16Tile - 1) / kBf16Tile) * g.nf);
  for (int64_t b0 = 0; b0 < g.nrhs; b0 += 64) {
    const int nb = (int)std::min<int64_t>(64, g.nrhs - b0);
    if (nb > 32)
      hipLaunchKernelGGL((gemm_cols_bf16<4, LO>), dim3(grid), dim3(kBf16Threads), 0, s, A, sc, Ds, Y, g, nd8, b0, nb);
    else if (nb > 16)
      hipLaunchKernelGGL((gemm_cols_bf16<2, LO>), dim3(grid), dim3(kBf16Threads), 0, s, A, sc, Ds, Y, g, nd8, b0, nb);
    else
      hipLaunchKernelGGL((gemm_cols_bf16<1, LO>), dim3(grid), dim3(kBf16Threads), 0, s, A, sc, Ds, Y, g, nd8, b0, nb);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

hipError_t launch_split_bf16(const cpx<float>* in, uint16_t* out, int64_t count, int64_t n,
                             int64_t n8, const float* scales, int64_t nf, hipStream_t s) {
  const int64_t total = count * n8;
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 1 << 20));
  hipLaunchKernelGGL(split_bf16, dim3(g), dim3(256), 0, s, in, out, count, n, n8, scales, nf);
  return hipGetLastError();
}

hipError_t launch_gemm_rows_bf16(const void* A, const float* scales, const uint16_t* Xs,
                                 cpx<double>* P, const GemvShape& g, int64_t n8, bool lo,
                                 hipStream_t s) {
  const auto* a = static_cast<const uint32_t*>(A);
  // 16-byte loads need every row start aligned: Nm even (hi+lo), Nm % 4 == 0 (hi only)
  const bool vec = lo ? (g.Nm % 2 == 0) : (g.Nm % 4 == 0);
  (void)scales;  // folded into the vector planes by launch_split_bf16
  if (lo) return vec ? rows_passes<true, true>(a, Xs, P, g, n8, s)
                     : rows_passes<true, false>(a, Xs, P, g, n8, s);
  return vec ? rows_passes<false, true>(a, Xs, P, g, n8, s)
             : rows_passes<false, false>(a, Xs, P, g, n8, s);
}

hipError_t launch_gemm_cols_bf16(const void* A, const float* scales, const uint16_t* Ds,
                                 cpx<float>* Y, const GemvShape& g, int64_t nd8, bool lo,
                                 hipStream_t s) {
  const auto* a = static_cast<const uint32_t*>(A);
  return lo ? cols_passes<true>(a, scales, Ds, Y, g, nd8, s)
            : cols_passes<false>(a, scales, Ds, Y, g, nd8, s);
}

}  // namespace p2o
