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
// Vector operands arrive as four bfloat16 planes per (rhs, k), written by
// the forward transform: [re hi][re lo][im hi][im lo], each padded to a
// multiple of 8 entries.
#include "matrix_units.h"

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

hipError_t launch_gemm_rows_bf16(const void* A, const float* scales, const uint16_t* Xs,
                                 cpx<double>* P, const GemvShape& g, int64_t n8, bool lo,
                                 hipStream_t s) {
  const auto* a = static_cast<const uint32_t*>(A);
  // 16-byte loads need every row start aligned: Nm even (hi+lo), Nm % 4 == 0 (hi only)
  const bool vec = lo ? (g.Nm % 2 == 0) : (g.Nm % 4 == 0);
  (void)scales;  // folded into the vector planes by the forward transform
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
