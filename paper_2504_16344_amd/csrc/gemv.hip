// Per-frequency complex block products, the step through which every
// frequency block streams from HBM once per apply (section "FFT-based
// Hessian matvecs", item (iii): after the DFT the p2o matvec is a
// block-diagonal matvec in Fourier space).
//
//   F : Yhat_k = Fhat_k Xhat_k        (Nd x Nm times Nm)
//   F*: Xhat_k = Fhat_k^H Dhat_k      (Nm x Nd times Nd)
//
// One copy of Fhat, layout [k][s][p] with p contiguous, serves both.
// F   ("rows"): a wavefront owns R consecutive rows s of one frequency k and
//     one column chunk; lane l walks columns p = p0 + V*l + 64*V*j, so each
//     row load of the wavefront is one contiguous segment, and Xhat_k[p] is
//     loaded once and reused for the R rows.  Lane partial sums are reduced
//     across the wavefront at the end and written per chunk; the chunks are
//     summed in fixed order by the inverse transform, so the result does not
//     depend on scheduling.
// F*  ("cols"): a wavefront owns 64*J*V consecutive columns of one k and
//     walks all rows s; Dhat_k[s] is wave-uniform, each lane keeps its own
//     columns' sums, so no cross-lane reduction is needed.
// The blocks are read with non-temporal loads: they are touched once per
// apply, and keeping them out of the caches leaves L2 to the reused vector.
// R, J and the vector width V are the tuning knobs (see the candidate
// tables at the end of this file).
#include "product_units.h"

namespace p2o {
namespace {

template <int R, int B>
__global__ void __launch_bounds__(256)
gemv_rows_f64_kernel(const cpx<double>* __restrict__ A, const cpx<double>* __restrict__ X,
                     cpx<double>* __restrict__ P, GemvShape g, int64_t b0, int nb) {
  const int64_t wave = (int64_t)blockIdx.x * 4 + wave_id_in_block();
  const int64_t nsg = (g.Nd + R - 1) / R;
  const int64_t rest = wave / nsg;
  const int64_t pc = rest / g.nf;
  if (pc >= g.n_pc) return;
  rows_f64_unit<R, B>(A, X, P, g, b0, nb, rest % g.nf, wave % nsg, pc);
}

template <int J, int B>
__global__ void __launch_bounds__(256)
gemv_cols_f64_kernel(const cpx<double>* __restrict__ A, const cpx<double>* __restrict__ D,
                     cpx<double>* __restrict__ Y, GemvShape g, int64_t b0, int nb) {
  const int64_t wave = (int64_t)blockIdx.x * 4 + wave_id_in_block();
  const int64_t npg = (g.Nm + 64 * J - 1) / (64 * J);
  const int64_t k = wave / npg;
  if (k >= g.nf) return;
  cols_f64_unit<J, B>(A, D, Y, g, b0, nb, k, wave % npg);
}

template <int R, int V, Fmt16 FMT, bool LO>
__global__ void __launch_bounds__(256)
gemv_rows_mixed_kernel(const void* __restrict__ A, const float* __restrict__ scales,
                       const cpx<float>* __restrict__ X, cpx<double>* __restrict__ P,
                       GemvShape g, int64_t b) {
  const int64_t wave = (int64_t)blockIdx.x * 4 + wave_id_in_block();
  const int64_t nsg = (g.Nd + R - 1) / R;
  const int64_t rest = wave / nsg;
  const int64_t pc = rest / g.nf;
  if (pc >= g.n_pc) return;
  rows_mixed_unit<R, V, FMT, LO>(A, scales, X, P, g, b, rest % g.nf, wave % nsg, pc);
}

template <int J, int V, Fmt16 FMT, bool LO>
__global__ void __launch_bounds__(256)
gemv_cols_mixed_kernel(const void* __restrict__ A, const float* __restrict__ scales,
                       const cpx<float>* __restrict__ D, cpx<float>* __restrict__ Y,
                       GemvShape g, int64_t b) {
  const int64_t wave = (int64_t)blockIdx.x * 4 + wave_id_in_block();
  const int64_t npg = (g.Nm + 64 * J * V - 1) / (64 * J * V);
  const int64_t k = wave / npg;
  if (k >= g.nf) return;
  cols_mixed_unit<J, V, FMT, LO>(A, scales, D, Y, g, b, k, wave % npg);
}

inline unsigned blocks_for_waves(int64_t waves) {
  return (unsigned)((waves + 3) / 4);  // 4 wavefronts per 256-thread block
}

// ------------------------------------------------------------ dispatching
template <int R, int B>
hipError_t rows_f64_pass(const cpx<double>* A, const cpx<double>* X,
                         cpx<double>* P, const GemvShape& g, int64_t b0, int nb,
                         hipStream_t s) {
  const int64_t waves = g.nf * ((g.Nd + R - 1) / R) * g.n_pc;
  hipLaunchKernelGGL((gemv_rows_f64_kernel<R, B>), dim3(blocks_for_waves(waves)),
                     dim3(256), 0, s, A, X, P, g, b0, nb);
  return hipGetLastError();
}

template <int J, int B>
hipError_t cols_f64_pass(const cpx<double>* A, const cpx<double>* D,
                         cpx<double>* Y, const GemvShape& g, int64_t b0, int nb,
                         hipStream_t s) {
  const int64_t waves = g.nf * ((g.Nm + 64 * J - 1) / (64 * J));
  hipLaunchKernelGGL((gemv_cols_f64_kernel<J, B>), dim3(blocks_for_waves(waves)),
                     dim3(256), 0, s, A, D, Y, g, b0, nb);
  return hipGetLastError();
}

template <int T>
hipError_t rows_f64_all(const cpx<double>* A, const cpx<double>* X,
                        cpx<double>* P, const GemvShape& g, hipStream_t s) {
  for (int64_t b0 = 0; b0 < g.nrhs;) {
    const int64_t left = g.nrhs - b0;
    hipError_t e;
    int step;
    if (left >= 4) { e = rows_f64_pass<T, 4>(A, X, P, g, b0, 4, s); step = 4; }
    else if (left >= 2) { e = rows_f64_pass<T, 2>(A, X, P, g, b0, 2, s); step = 2; }
    else { e = rows_f64_pass<T, 1>(A, X, P, g, b0, 1, s); step = 1; }
    if (e != hipSuccess) return e;
    b0 += step;
  }
  return hipSuccess;
}

template <int T>
hipError_t cols_f64_all(const cpx<double>* A, const cpx<double>* D,
                        cpx<double>* Y, const GemvShape& g, hipStream_t s) {
  for (int64_t b0 = 0; b0 < g.nrhs;) {
    const int64_t left = g.nrhs - b0;
    hipError_t e;
    int step;
    if (left >= 4) { e = cols_f64_pass<T, 4>(A, D, Y, g, b0, 4, s); step = 4; }
    else if (left >= 2) { e = cols_f64_pass<T, 2>(A, D, Y, g, b0, 2, s); step = 2; }
    else { e = cols_f64_pass<T, 1>(A, D, Y, g, b0, 1, s); step = 1; }
    if (e != hipSuccess) return e;
    b0 += step;
  }
  return hipSuccess;
}

template <int R, int V, Fmt16 FMT, bool LO>
hipError_t rows_mixed_all(const void* A, const float* sc, const cpx<float>* X,
                          cpx<double>* P, const GemvShape& g, hipStream_t s) {
  const int64_t waves = g.nf * ((g.Nd + R - 1) / R) * g.n_pc;
  for (int64_t b = 0; b < g.nrhs; ++b) {
    hipLaunchKernelGGL((gemv_rows_mixed_kernel<R, V, FMT, LO>), dim3(blocks_for_waves(waves)),
                       dim3(256), 0, s, A, sc, X, P, g, b);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int J, int V, Fmt16 FMT, bool LO>
hipError_t cols_mixed_all(const void* A, const float* sc, const cpx<float>* D,
                          cpx<float>* Y, const GemvShape& g, hipStream_t s) {
  const int64_t waves = g.nf * ((g.Nm + 64 * J * V - 1) / (64 * J * V));
  for (int64_t b = 0; b < g.nrhs; ++b) {
    hipLaunchKernelGGL((gemv_cols_mixed_kernel<J, V, FMT, LO>), dim3(blocks_for_waves(waves)),
                       dim3(256), 0, s, A, sc, D, Y, g, b);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Candidate tables.  Each row is one configuration the autotuner may pick;
// index 0 of every table is the default used before any tuning.
struct F64Rows { int R; hipError_t (*fn)(const cpx<double>*, const cpx<double>*, cpx<double>*, const GemvShape&, hipStream_t); };
struct F64Cols { int J; hipError_t (*fn)(const cpx<double>*, const cpx<double>*, cpx<double>*, const GemvShape&, hipStream_t); };
const F64Rows kF64Rows[] = {{4, rows_f64_all<4>}, {2, rows_f64_all<2>}, {8, rows_f64_all<8>}};
const F64Cols kF64Cols[] = {{2, cols_f64_all<2>}, {1, cols_f64_all<1>}, {4, cols_f64_all<4>}};

using RowsMixedFn = hipError_t (*)(const void*, const float*, const cpx<float>*, cpx<double>*,
                                   const GemvShape&, hipStream_t);
using ColsMixedFn = hipError_t (*)(const void*, const float*, const cpx<float>*, cpx<float>*,
                                   const GemvShape&, hipStream_t);
struct MixedRows { int R, V; RowsMixedFn fn[3]; };  // FP16 hi+lo, BF16 hi+lo, BF16 hi
struct MixedCols { int J, V; ColsMixedFn fn[3]; };

#define ROWS_SET(R, V) {R, V, {rows_mixed_all<R, V, Fmt16::FP16, true>, \
    rows_mixed_all<R, V, Fmt16::BF16, true>, rows_mixed_all<R, V, Fmt16::BF16, false>}}
#define COLS_SET(J, V) {J, V, {cols_mixed_all<J, V, Fmt16::FP16, true>, \
    cols_mixed_all<J, V, Fmt16::BF16, true>, cols_mixed_all<J, V, Fmt16::BF16, false>}}
// Candidate 0 of every table has vector width 1, so it is valid for any Nm.
const MixedRows kMixedRows[] = {ROWS_SET(4, 1), ROWS_SET(2, 1), ROWS_SET(8, 1),
                                ROWS_SET(4, 2), ROWS_SET(2, 2), ROWS_SET(8, 2)};
const MixedCols kMixedCols[] = {COLS_SET(2, 1), COLS_SET(1, 1), COLS_SET(4, 1),
                                COLS_SET(2, 2), COLS_SET(1, 2), COLS_SET(4, 2)};

int mixed_slot(Fmt16 fmt, bool lo) {
  if (!lo) return 2;
  return fmt == Fmt16::FP16 ? 0 : 1;
}

}  // namespace

int gemv_candidates(bool mixed, p2o_op op) {
  if (!mixed) return op == P2O_F ? 3 : 3;
  return op == P2O_F ? 6 : 6;
}

int gemv_vec_width(bool mixed, bool lo, p2o_op op, int cfg) {
  (void)lo;
  if (!mixed) return 1;
  return (op == P2O_F) ? kMixedRows[cfg].V : kMixedCols[cfg].V;
}

int gemv_rows_per_wave(bool mixed, int cfg) {
  return mixed ? kMixedRows[cfg].R : kF64Rows[cfg].R;
}

hipError_t launch_gemv_rows_f64(const cpx<double>* A, const cpx<double>* X,
                                cpx<double>* P, const GemvShape& g, int cfg,
                                hipStream_t s) {
  return kF64Rows[cfg].fn(A, X, P, g, s);
}

hipError_t launch_gemv_cols_f64(const cpx<double>* A, const cpx<double>* D,
                                cpx<double>* Y, const GemvShape& g, int cfg,
                                hipStream_t s) {
  return kF64Cols[cfg].fn(A, D, Y, g, s);
}

hipError_t launch_gemv_rows_mixed(const void* A, const float* scales,
                                  const cpx<float>* X, cpx<double>* P,
                                  const GemvShape& g, Fmt16 fmt, bool use_lo,
                                  int cfg, hipStream_t s) {
  return kMixedRows[cfg].fn[mixed_slot(fmt, use_lo)](A, scales, X, P, g, s);
}

hipError_t launch_gemv_cols_mixed(const void* A, const float* scales,
                                  const cpx<float>* D, cpx<float>* Y,
                                  const GemvShape& g, Fmt16 fmt, bool use_lo,
                                  int cfg, hipStream_t s) {
  return kMixedCols[cfg].fn[mixed_slot(fmt, use_lo)](A, scales, D, Y, g, s);
}

}  // namespace p2o
