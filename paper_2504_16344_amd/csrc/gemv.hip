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
#include "p2o_internal.h"

namespace p2o {
namespace {

typedef double d2v __attribute__((ext_vector_type(2)));
typedef unsigned u2v __attribute__((ext_vector_type(2)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ int wave_id_in_block() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

__device__ __forceinline__ cpx<double> ld_block(const cpx<double>* p) {
  const d2v v = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(p));
  return {v.x, v.y};
}

// ----------------------------------------------------------------- float64
template <int R, int B>
__global__ void __launch_bounds__(256)
gemv_rows_f64_kernel(const cpx<double>* __restrict__ A,
                     const cpx<double>* __restrict__ X,
                     cpx<double>* __restrict__ P, GemvShape g, int64_t b0,
                     int nb) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave_id_in_block();
  const int64_t nsg = (g.Nd + R - 1) / R;
  const int64_t sg = wave % nsg;
  const int64_t rest = wave / nsg;
  const int64_t k = rest % g.nf;
  const int64_t pc = rest / g.nf;
  if (pc >= g.n_pc) return;
  const int64_t s0 = sg * R;
  const int64_t p0 = pc * g.pc_len;
  const int64_t p1 = min(p0 + g.pc_len, g.Nm);

  const cpx<double>* Ar[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t s = min(s0 + r, g.Nd - 1);  // rows past Nd: computed, dropped
    Ar[r] = A + (k * g.Nd + s) * g.Nm;
  }
  const cpx<double>* Xb[B];
#pragma unroll
  for (int bb = 0; bb < B; ++bb)
    Xb[bb] = X + ((b0 + min(bb, nb - 1)) * g.nf + k) * g.Nm;

  double ar[R][B], ai[R][B];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int bb = 0; bb < B; ++bb) ar[r][bb] = ai[r][bb] = 0.0;

#pragma unroll 2
  for (int64_t p = p0 + lane; p < p1; p += 64) {
    cpx<double> x[B];
#pragma unroll
    for (int bb = 0; bb < B; ++bb) x[bb] = Xb[bb][p];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const cpx<double> a = ld_block(Ar[r] + p);
#pragma unroll
      for (int bb = 0; bb < B; ++bb) {
        ar[r][bb] += a.x * x[bb].x - a.y * x[bb].y;
        ai[r][bb] += a.x * x[bb].y + a.y * x[bb].x;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int bb = 0; bb < B; ++bb) {
      ar[r][bb] = wave_sum(ar[r][bb]);
      ai[r][bb] = wave_sum(ai[r][bb]);
    }
  if (lane == 0) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (s0 + r >= g.Nd) break;
#pragma unroll
      for (int bb = 0; bb < B; ++bb) {
        if (bb >= nb) break;
        P[(((b0 + bb) * g.n_pc + pc) * g.nf + k) * g.Nd + s0 + r] = {ar[r][bb], ai[r][bb]};
      }
    }
  }
}

template <int J, int B>
__global__ void __launch_bounds__(256)
gemv_cols_f64_kernel(const cpx<double>* __restrict__ A,
                     const cpx<double>* __restrict__ D,
                     cpx<double>* __restrict__ Y, GemvShape g, int64_t b0,
                     int nb) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave_id_in_block();
  const int64_t npg = (g.Nm + 64 * J - 1) / (64 * J);
  const int64_t pg = wave % npg;
  const int64_t k = wave / npg;
  if (k >= g.nf) return;
  int64_t pj[J];
#pragma unroll
  for (int j = 0; j < J; ++j) pj[j] = min(pg * 64 * J + j * 64 + lane, g.Nm - 1);
  const cpx<double>* Ak = A + k * g.Nd * g.Nm;
  const cpx<double>* Db[B];
#pragma unroll
  for (int bb = 0; bb < B; ++bb)
    Db[bb] = D + ((b0 + min(bb, nb - 1)) * g.nf + k) * g.Nd;

  double yr[J][B], yi[J][B];
#pragma unroll
  for (int j = 0; j < J; ++j)
#pragma unroll
    for (int bb = 0; bb < B; ++bb) yr[j][bb] = yi[j][bb] = 0.0;

#pragma unroll 4
  for (int64_t s = 0; s < g.Nd; ++s) {
    cpx<double> dv[B];
#pragma unroll
    for (int bb = 0; bb < B; ++bb) dv[bb] = Db[bb][s];
    const cpx<double>* As = Ak + s * g.Nm;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const cpx<double> a = ld_block(As + pj[j]);
#pragma unroll
      for (int bb = 0; bb < B; ++bb) {  // conj(a) * d
        yr[j][bb] += a.x * dv[bb].x + a.y * dv[bb].y;
        yi[j][bb] += a.x * dv[bb].y - a.y * dv[bb].x;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int64_t p = pg * 64 * J + j * 64 + lane;
    if (p >= g.Nm) break;
#pragma unroll
    for (int bb = 0; bb < B; ++bb) {
      if (bb >= nb) break;
      Y[((b0 + bb) * g.nf + k) * g.Nm + p] = {yr[j][bb], yi[j][bb]};
    }
  }
}

// ------------------------------------------------------------------- mixed
// Packed entry: word 0 = hi (real part in the low 16 bits, imaginary in the
// high 16 bits), word 1 = lo (same), absent for the hi-only tier.  Value =
// s * (hi + lo * kLoScale) with s the (k, 256-column tile) scale.
template <Fmt16 FMT>
struct Dec;
template <>
struct Dec<Fmt16::FP16> {
  static constexpr float kLoScale = 1.0f / 2048.0f;
  __device__ static __forceinline__ float lo16(uint32_t w) {
    _Float16 h;
    const unsigned short u = (unsigned short)(w & 0xffffu);
    __builtin_memcpy(&h, &u, 2);
    return (float)h;
  }
  __device__ static __forceinline__ float hi16(uint32_t w) {
    _Float16 h;
    const unsigned short u = (unsigned short)(w >> 16);
    __builtin_memcpy(&h, &u, 2);
    return (float)h;
  }
};
template <>
struct Dec<Fmt16::BF16> {
  static constexpr float kLoScale = 1.0f;
  __device__ static __forceinline__ float lo16(uint32_t w) {
    return __uint_as_float(w << 16);
  }
  __device__ static __forceinline__ float hi16(uint32_t w) {
    return __uint_as_float(w & 0xffff0000u);
  }
};

// V consecutive entries loaded with one instruction (4, 8 or 16 bytes).
template <bool LO, int V>
struct Pack {
  static constexpr int kWords = (LO ? 2 : 1) * V;
  using T = typename std::conditional<kWords == 1, uint32_t,
            typename std::conditional<kWords == 2, u2v, u4v>::type>::type;
  __device__ static __forceinline__ void load(const void* base, int64_t entry,
                                              uint32_t (&w)[kWords]) {
    const T v = __builtin_nontemporal_load(
        reinterpret_cast<const T*>(static_cast<const uint32_t*>(base) + entry * (LO ? 2 : 1)));
    if constexpr (kWords == 1) {
      w[0] = v;
    } else {
#pragma unroll
      for (int i = 0; i < kWords; ++i) w[i] = v[i];
    }
  }
};

template <Fmt16 FMT, bool LO>
__device__ __forceinline__ cpx<float> decode(const uint32_t* w) {
  cpx<float> v = {Dec<FMT>::lo16(w[0]), Dec<FMT>::hi16(w[0])};
  if constexpr (LO) {
    v.x = fmaf(Dec<FMT>::lo16(w[1]), Dec<FMT>::kLoScale, v.x);
    v.y = fmaf(Dec<FMT>::hi16(w[1]), Dec<FMT>::kLoScale, v.y);
  }
  return v;
}

template <int R, int V, Fmt16 FMT, bool LO>
__global__ void __launch_bounds__(256)
gemv_rows_mixed_kernel(const void* __restrict__ A,
                       const float* __restrict__ scales,
                       const cpx<float>* __restrict__ X,
                       cpx<double>* __restrict__ P, GemvShape g, int64_t b) {
  using PK = Pack<LO, V>;
  constexpr int WPE = LO ? 2 : 1;  // words per entry
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave_id_in_block();
  const int64_t nsg = (g.Nd + R - 1) / R;
  const int64_t sg = wave % nsg;
  const int64_t rest = wave / nsg;
  const int64_t k = rest % g.nf;
  const int64_t pc = rest / g.nf;
  if (pc >= g.n_pc) return;
  const int64_t s0 = sg * R;
  const int64_t p0 = pc * g.pc_len;
  const int64_t p1 = min(p0 + g.pc_len, g.Nm);
  const int64_t ntiles = (g.Nm + kScaleTile - 1) / kScaleTile;
  const float* __restrict__ sk = scales + k * ntiles;

  int64_t Ar[R];
#pragma unroll
  for (int r = 0; r < R; ++r) Ar[r] = (k * g.Nd + min(s0 + r, g.Nd - 1)) * g.Nm;
  const cpx<float>* Xk = X + (b * g.nf + k) * g.Nm;

  float ar[R], ai[R];
#pragma unroll
  for (int r = 0; r < R; ++r) ar[r] = ai[r] = 0.0f;

  // V consecutive columns per lane; Nm and the chunk bounds are multiples
  // of V whenever V > 1 is selected, so no partial vector occurs.
#pragma unroll 2
  for (int64_t p = p0 + (int64_t)V * lane; p < p1; p += 64 * V) {
    const float sc = sk[p / kScaleTile];
    cpx<float> x[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      x[v] = Xk[p + v];
      x[v].x *= sc;
      x[v].y *= sc;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      uint32_t w[PK::kWords];
      PK::load(A, Ar[r] + p, w);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const cpx<float> a = decode<FMT, LO>(w + WPE * v);
        ar[r] = fmaf(a.x, x[v].x, fmaf(-a.y, x[v].y, ar[r]));
        ai[r] = fmaf(a.x, x[v].y, fmaf(a.y, x[v].x, ai[r]));
      }
    }
  }
  double dr[R], di[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    dr[r] = wave_sum((double)ar[r]);
    di[r] = wave_sum((double)ai[r]);
  }
  if (lane == 0) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (s0 + r >= g.Nd) break;
      P[((b * g.n_pc + pc) * g.nf + k) * g.Nd + s0 + r] = {dr[r], di[r]};
    }
  }
}

template <int J, int V, Fmt16 FMT, bool LO>
__global__ void __launch_bounds__(256)
gemv_cols_mixed_kernel(const void* __restrict__ A,
                       const float* __restrict__ scales,
                       const cpx<float>* __restrict__ D,
                       cpx<float>* __restrict__ Y, GemvShape g, int64_t b) {
  using PK = Pack<LO, V>;
  constexpr int WPE = LO ? 2 : 1;
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave_id_in_block();
  constexpr int kCols = 64 * J * V;  // columns per wavefront
  const int64_t npg = (g.Nm + kCols - 1) / kCols;
  const int64_t pg = wave % npg;
  const int64_t k = wave / npg;
  if (k >= g.nf) return;
  int64_t pj[J];
#pragma unroll
  for (int j = 0; j < J; ++j)
    pj[j] = min(pg * kCols + (int64_t)j * 64 * V + (int64_t)V * lane, g.Nm - V);
  const int64_t Ak = k * g.Nd * g.Nm;
  const cpx<float>* Dk = D + (b * g.nf + k) * g.Nd;

  float yr[J][V], yi[J][V];
#pragma unroll
  for (int j = 0; j < J; ++j)
#pragma unroll
    for (int v = 0; v < V; ++v) yr[j][v] = yi[j][v] = 0.0f;

#pragma unroll 4
  for (int64_t s = 0; s < g.Nd; ++s) {
    const cpx<float> dv = Dk[s];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      uint32_t w[PK::kWords];
      PK::load(A, Ak + s * g.Nm + pj[j], w);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const cpx<float> a = decode<FMT, LO>(w + WPE * v);
        yr[j][v] = fmaf(a.x, dv.x, fmaf(a.y, dv.y, yr[j][v]));
        yi[j][v] = fmaf(a.x, dv.y, fmaf(-a.y, dv.x, yi[j][v]));
      }
    }
  }
  const int64_t ntiles = (g.Nm + kScaleTile - 1) / kScaleTile;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int64_t pbase = pg * kCols + (int64_t)j * 64 * V + (int64_t)V * lane;
    if (pbase >= g.Nm) break;
    const float sc = scales[k * ntiles + pbase / kScaleTile];
#pragma unroll
    for (int v = 0; v < V; ++v)
      Y[(b * g.nf + k) * g.Nm + pbase + v] = {yr[j][v] * sc, yi[j][v] * sc};
  }
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
