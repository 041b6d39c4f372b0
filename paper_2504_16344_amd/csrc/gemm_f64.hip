// Per-frequency complex block products for many right-hand sides on the
// float64 matrix cores (v_mfma_f64_16x16x4_f64): the block-diagonal
// Fourier-space matvec of section "FFT-based Hessian matvecs" applied to B
// vectors at once, so each frequency block is streamed once per 64
// right-hand sides instead of once per vector.
//
// MFMA operand layout (16x16x4, float64, checked on the device): lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator element i
// of lane l is D[(l / 16) + 4 i][l % 16] (rows interleave, unlike the
// 16-bit 16x16 shapes, where it is D[4 (l / 16) + i][l % 16]).  Within a
// 32-entry chunk, the contraction index l / 16 of the j-th instruction is
// mapped to a block entry, the same one for both operands, so the sum over
// the chunk is unchanged: F takes entry base + 4 j + l / 16 (the 4 lanes of
// a sensor row read 64 contiguous bytes per load), F* takes sensor
// base + 8 (l / 16) + j (16 lanes read 16 neighbouring columns of a row).
//
// F  ("rows"): workgroup = 64 sensors s x (16 NT) right-hand sides of one
//    frequency k and one column chunk; D = Fhat_k[s, chunk] X_k[chunk, b];
//    partial spectra per chunk, summed in fixed order by the inverse
//    transform.
// F* ("cols"): workgroup = (16 MT) right-hand sides x 64 columns p; the
//    transposed product X^T = Dhat^T conj(Fhat) with the contraction over
//    all sensors s, written straight to the transformed parameter vector.
// Complex products use four real products each: re = ar br - ai bi,
// im = ar bi + ai br (the minus sign is folded into an operand).
#include "matrix_units.h"

namespace p2o {
namespace {

template <int NT>
__global__ void __launch_bounds__(256)
gemm_rows_f64(const cpx<double>* __restrict__ A, const cpx<double>* __restrict__ X,
              cpx<double>* __restrict__ P, GemvShape g, int64_t b0, int nb) {
  __shared__ __align__(16) char lds[stage_bytes_f64(NT)];
  const int64_t tile = xcd_local_tile(blockIdx.x, gridDim.x);
  const int64_t nmt = (g.Nd + kWgTile - 1) / kWgTile;
  const int64_t rest = tile / nmt;
  const int64_t pc = rest / g.nf;
  if (pc >= g.n_pc) return;  // grid padding: the whole workgroup leaves
  mfma_rows_f64_wg<NT>(A, X, P, g, b0, nb, rest % g.nf, tile % nmt, pc, lds);
}

template <int MT>
__global__ void __launch_bounds__(256)
gemm_cols_f64(const cpx<double>* __restrict__ A, const cpx<double>* __restrict__ D,
              cpx<double>* __restrict__ Y, GemvShape g, int64_t b0, int nb) {
  __shared__ __align__(16) char lds[stage_bytes_f64(MT)];
  const int64_t tile = xcd_local_tile(blockIdx.x, gridDim.x);
  const int64_t npt = (g.Nm + kWgTile - 1) / kWgTile;
  const int64_t k = tile / npt;
  if (k >= g.nf) return;
  mfma_cols_f64_wg<MT>(A, D, Y, g, b0, nb, k, tile % npt, lds);
}

unsigned padded_grid(int64_t tiles) { return (unsigned)((tiles + kXcds - 1) / kXcds * kXcds); }

}  // namespace

hipError_t launch_gemm_rows_f64(const cpx<double>* A, const cpx<double>* X,
                                cpx<double>* P, const GemvShape& g, hipStream_t s) {
  const unsigned grid = padded_grid(((g.Nd + kWgTile - 1) / kWgTile) * g.nf * g.n_pc);
  for (int64_t b0 = 0; b0 < g.nrhs; b0 += 64) {
    const int nb = (int)std::min<int64_t>(64, g.nrhs - b0);
    if (nb > 32)
      hipLaunchKernelGGL(gemm_rows_f64<4>, dim3(grid), dim3(256), 0, s, A, X, P, g, b0, nb);
    else if (nb > 16)
      hipLaunchKernelGGL(gemm_rows_f64<2>, dim3(grid), dim3(256), 0, s, A, X, P, g, b0, nb);
    else
      hipLaunchKernelGGL(gemm_rows_f64<1>, dim3(grid), dim3(256), 0, s, A, X, P, g, b0, nb);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_gemm_cols_f64(const cpx<double>* A, const cpx<double>* D,
                                cpx<double>* Y, const GemvShape& g, hipStream_t s) {
  const unsigned grid = padded_grid(((g.Nm + kWgTile - 1) / kWgTile) * g.nf);
  for (int64_t b0 = 0; b0 < g.nrhs; b0 += 64) {
    const int nb = (int)std::min<int64_t>(64, g.nrhs - b0);
    if (nb > 32)
      hipLaunchKernelGGL(gemm_cols_f64<4>, dim3(grid), dim3(256), 0, s, A, D, Y, g, b0, nb);
    else if (nb > 16)
      hipLaunchKernelGGL(gemm_cols_f64<2>, dim3(grid), dim3(256), 0, s, A, D, Y, g, b0, nb);
    else
      hipLaunchKernelGGL(gemm_cols_f64<1>, dim3(grid), dim3(256), 0, s, A, D, Y, g, b0, nb);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace p2o
