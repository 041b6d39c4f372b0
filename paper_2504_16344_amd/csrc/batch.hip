// Persistent product kernel for a batch of independent p2o instances of
// uneven shape (section "FFT-based Hessian matvecs": every instance is its
// own block-diagonal Fourier-space product).  One launch covers the
// frequency-block products of every instance: the workgroup units of all
// instances are numbered consecutively, each workgroup takes units w,
// w + W, w + 2W, ... (W = workgroups in the grid, sized to the chip's
// resident capacity), finds the owning instance by binary search over the
// instances' first units, and runs that instance's path — four vector-unit
// wavefront units for few right-hand sides, one float64 matrix-core
// workgroup tile for many (FP64 instances) — through the same code as the
// single-plan kernels.  bfloat16 instances on the matrix-core path are not
// in the table: each gets its own warp-specialised launch (gemm_bf16.hip).
// Interleaving keeps every workgroup's mix of large and small instances
// alike, and neighbouring workgroups on neighbouring tiles of one instance,
// which share the vector operand in L2.
#include "matrix_units.h"

namespace p2o {
namespace {

// Tunable configurations of the persistent kernel: vector-unit rows per
// wavefront (F) and vector-unit column groups per wavefront (F*).
// p2o_batch_autotune times them on the batch itself.
struct BatchCfg {
  int rows_v, cols_v;
};
constexpr BatchCfg kBatchCfgs[] = {{4, 2}, {2, 1}, {8, 4}};
constexpr int kBatchCfgCount = sizeof(kBatchCfgs) / sizeof(kBatchCfgs[0]);

template <int CLS>
struct ClassTraits;
template <>
struct ClassTraits<kClassMixedFp16> { static constexpr Fmt16 fmt = Fmt16::FP16; static constexpr bool lo = true; };
template <>
struct ClassTraits<kClassMixedBf16> { static constexpr Fmt16 fmt = Fmt16::BF16; static constexpr bool lo = true; };
template <>
struct ClassTraits<kClassFastBf16> { static constexpr Fmt16 fmt = Fmt16::BF16; static constexpr bool lo = false; };

// LDS of the float64 matrix-core stage (FP64 class only).
template <int CLS>
constexpr int stage_bytes() {
  return CLS == kClassF64 ? stage_bytes_f64(4) : 16;
}

constexpr int kBatchThreads = 256;  // 4 wavefronts: 4 vector-unit wave units, or one 64-row tile

// Vector-path wave units of one instance (a workgroup unit is
// threads / 64 of them).
__host__ __device__ __forceinline__ int64_t vector_wave_units(p2o_op op, const GemvShape& g,
                                                              int rows_v, int cols_v) {
  if (op == P2O_F) return g.nf * ((g.Nd + rows_v - 1) / rows_v) * g.n_pc;
  return g.nf * ((g.Nm + 64 * cols_v - 1) / (64 * cols_v));
}

template <int CLS, int CFG>
__device__ __forceinline__ void rows_unit(const BatchInst& I, int64_t u, void* lds) {
  constexpr int kRowsV = kBatchCfgs[CFG].rows_v;
  const GemvShape& g = I.g;
  if constexpr (CLS == kClassF64) {
    if (I.path == kPathMatrix) {
      const int64_t nmt = (g.Nd + kWgTile - 1) / kWgTile, rest = u / nmt;
      const int64_t mt = u % nmt, k = rest % g.nf, pc = rest / g.nf;
      const auto* A = static_cast<const cpx<double>*>(I.fhat);
      const auto* X = static_cast<const cpx<double>*>(I.in);
      auto* P = static_cast<cpx<double>*>(I.out);
      for (int64_t b0 = 0; b0 < g.nrhs; b0 += 64) {
        const int nb = (int)min((int64_t)64, g.nrhs - b0);
        if (nb > 32) mfma_rows_f64_wg<4>(A, X, P, g, b0, nb, k, mt, pc, lds);
        else if (nb > 16) mfma_rows_f64_wg<2>(A, X, P, g, b0, nb, k, mt, pc, lds);
        else mfma_rows_f64_wg<1>(A, X, P, g, b0, nb, k, mt, pc, lds);
      }
      return;
    }
  }
  const int64_t wu = u * (kBatchThreads / 64) + wave_id_in_block();
  if (wu >= vector_wave_units(P2O_F, g, kRowsV, 1)) return;
  const int64_t nsg = (g.Nd + kRowsV - 1) / kRowsV, rest = wu / nsg;
  const int64_t sg = wu % nsg, k = rest % g.nf, pc = rest / g.nf;
  if constexpr (CLS == kClassF64) {
    const auto* A = static_cast<const cpx<double>*>(I.fhat);
    const auto* X = static_cast<const cpx<double>*>(I.in);
    auto* P = static_cast<cpx<double>*>(I.out);
    for (int64_t b0 = 0; b0 < g.nrhs;) {
      const int64_t left = g.nrhs - b0;
      if (left >= 4) { rows_f64_unit<kRowsV, 4>(A, X, P, g, b0, 4, k, sg, pc); b0 += 4; }
      else if (left >= 2) { rows_f64_unit<kRowsV, 2>(A, X, P, g, b0, 2, k, sg, pc); b0 += 2; }
      else { rows_f64_unit<kRowsV, 1>(A, X, P, g, b0, 1, k, sg, pc); b0 += 1; }
    }
  } else {
    constexpr Fmt16 FMT = ClassTraits<CLS>::fmt;
    constexpr bool LO = ClassTraits<CLS>::lo;
    for (int64_t b = 0; b < g.nrhs; ++b)
      rows_mixed_unit<kRowsV, 1, FMT, LO>(I.fhat, I.scales, static_cast<const cpx<float>*>(I.in),
                                          static_cast<cpx<double>*>(I.out), g, b, k, sg, pc);
  }
}

template <int CLS, int CFG>
__device__ __forceinline__ void cols_unit(const BatchInst& I, int64_t u, void* lds) {
  constexpr int kColsV = kBatchCfgs[CFG].cols_v;
  const GemvShape& g = I.g;
  if constexpr (CLS == kClassF64) {
    if (I.path == kPathMatrix) {
      const int64_t npt = (g.Nm + kWgTile - 1) / kWgTile;
      const int64_t pt = u % npt, k = u / npt;
      const auto* A = static_cast<const cpx<double>*>(I.fhat);
      const auto* D = static_cast<const cpx<double>*>(I.in);
      auto* Y = static_cast<cpx<double>*>(I.out);
      for (int64_t b0 = 0; b0 < g.nrhs; b0 += 64) {
        const int nb = (int)min((int64_t)64, g.nrhs - b0);
        if (nb > 32) mfma_cols_f64_wg<4>(A, D, Y, g, b0, nb, k, pt, lds);
        else if (nb > 16) mfma_cols_f64_wg<2>(A, D, Y, g, b0, nb, k, pt, lds);
        else mfma_cols_f64_wg<1>(A, D, Y, g, b0, nb, k, pt, lds);
      }
      return;
    }
  }
  const int64_t wu = u * (kBatchThreads / 64) + wave_id_in_block();
  if (wu >= vector_wave_units(P2O_FADJ, g, 1, kColsV)) return;
  const int64_t npg = (g.Nm + 64 * kColsV - 1) / (64 * kColsV);
  const int64_t pg = wu % npg, k = wu / npg;
  if constexpr (CLS == kClassF64) {
    const auto* A = static_cast<const cpx<double>*>(I.fhat);
    const auto* D = static_cast<const cpx<double>*>(I.in);
    auto* Y = static_cast<cpx<double>*>(I.out);
    for (int64_t b0 = 0; b0 < g.nrhs;) {
      const int64_t left = g.nrhs - b0;
      if (left >= 4) { cols_f64_unit<kColsV, 4>(A, D, Y, g, b0, 4, k, pg); b0 += 4; }
      else if (left >= 2) { cols_f64_unit<kColsV, 2>(A, D, Y, g, b0, 2, k, pg); b0 += 2; }
      else { cols_f64_unit<kColsV, 1>(A, D, Y, g, b0, 1, k, pg); b0 += 1; }
    }
  } else {
    constexpr Fmt16 FMT = ClassTraits<CLS>::fmt;
    constexpr bool LO = ClassTraits<CLS>::lo;
    for (int64_t b = 0; b < g.nrhs; ++b)
      cols_mixed_unit<kColsV, 1, FMT, LO>(I.fhat, I.scales, static_cast<const cpx<float>*>(I.in),
                                          static_cast<cpx<float>*>(I.out), g, b, k, pg);
  }
}

// The grid is a multiple of 8 workgroups; each XCD takes a contiguous range
// of units per round, so neighbouring tiles of one instance share its L2.
template <int CLS, int OP, int CFG>
__global__ void __launch_bounds__(kBatchThreads)
batch_product_kernel(const BatchInst* __restrict__ insts, int n, int64_t total) {
  __shared__ __align__(16) char lds[stage_bytes<CLS>()];
  const int64_t grid = gridDim.x;
  for (int64_t u = xcd_local_tile(blockIdx.x, grid); u < total; u += grid) {
    int lo = 0, hi = n - 1;  // last instance with unit_begin <= u
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (insts[mid].unit_begin <= u) lo = mid;
      else hi = mid - 1;
    }
    const BatchInst I = insts[lo];
    if constexpr (OP == P2O_F) rows_unit<CLS, CFG>(I, u - I.unit_begin, lds);
    else cols_unit<CLS, CFG>(I, u - I.unit_begin, lds);
  }
}

template <int CLS, int OP, int CFG>
hipError_t launch_one(const BatchInst* insts, int n, int64_t total, hipStream_t s) {
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_product_kernel<CLS, OP, CFG>,
                                                     kBatchThreads, 0);
  if (e != hipSuccess) return e;
  int64_t blocks = (int64_t)std::max(1, cus) * std::max(1, per_cu);
  blocks = std::min<int64_t>(blocks, total);
  if (blocks < 1) return hipSuccess;
  blocks = (blocks + kXcds - 1) / kXcds * kXcds;
  hipLaunchKernelGGL((batch_product_kernel<CLS, OP, CFG>), dim3((unsigned)blocks),
                     dim3(kBatchThreads), 0, s, insts, n, total);
  return hipGetLastError();
}

template <int CLS, int CFG>
hipError_t launch_cls(p2o_op op, const BatchInst* insts, int n, int64_t total, hipStream_t s) {
  return op == P2O_F ? launch_one<CLS, P2O_F, CFG>(insts, n, total, s)
                     : launch_one<CLS, P2O_FADJ, CFG>(insts, n, total, s);
}

template <int CFG>
hipError_t launch_cfg(BatchClass cls, p2o_op op, const BatchInst* insts, int n, int64_t total,
                      hipStream_t s) {
  switch (cls) {
    case kClassF64: return launch_cls<kClassF64, CFG>(op, insts, n, total, s);
    case kClassMixedFp16: return launch_cls<kClassMixedFp16, CFG>(op, insts, n, total, s);
    case kClassMixedBf16: return launch_cls<kClassMixedBf16, CFG>(op, insts, n, total, s);
    case kClassFastBf16: return launch_cls<kClassFastBf16, CFG>(op, insts, n, total, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

int batch_config_count() { return kBatchCfgCount; }

int64_t batch_units(BatchClass cls, p2o_op op, int path, const GemvShape& g, int cfg) {
  if (path == kPathMatrix) {  // float64 tiles (bfloat16 matrix-core instances have own launches)
    if (cls != kClassF64) return -1;
    if (op == P2O_F) return g.nf * ((g.Nd + kWgTile - 1) / kWgTile) * g.n_pc;
    return g.nf * ((g.Nm + kWgTile - 1) / kWgTile);
  }
  const BatchCfg& c = kBatchCfgs[cfg];
  const int64_t waves = vector_wave_units(op, g, c.rows_v, c.cols_v);
  const int64_t per = kBatchThreads / 64;
  return (waves + per - 1) / per;
}

hipError_t launch_batch_product(BatchClass cls, p2o_op op, const BatchInst* insts, int n,
                                int64_t total_units, int cfg, hipStream_t s) {
  static_assert(kBatchCfgCount == 3, "one launch_cfg case per configuration");
  switch (cfg) {
    case 0: return launch_cfg<0>(cls, op, insts, n, total_units, s);
    case 1: return launch_cfg<1>(cls, op, insts, n, total_units, s);
    case 2: return launch_cfg<2>(cls, op, insts, n, total_units, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace p2o
