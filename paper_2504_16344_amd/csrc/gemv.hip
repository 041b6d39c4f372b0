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
//     one column chunk; lane l walks columns p = p0 + l + 64 j, so each row
//     load of the wavefront is one contiguous 1 KB (float64) segment, and
//     Xhat_k[p] is loaded once and reused for the R rows.  Lane partial sums
//     are reduced across the wavefront at the end and written per chunk;
//     the chunks are summed in fixed order by the inverse transform, so the
//     result does not depend on scheduling.
// F*  ("cols"): a wavefront owns 64*J consecutive columns of one k and walks
//     all rows s; Dhat_k[s] is wave-uniform (scalar loads), each lane keeps
//     its own columns' sums, so no cross-lane reduction is needed.
#include "p2o_internal.h"

namespace p2o {
namespace {

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ int wave_id_in_block() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
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
      const cpx<double> a = Ar[r][p];
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
      const cpx<double> a = As[pj[j]];
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
// Entry e of the packed layout: e.x = hi (re low half, im high half),
// e.y = lo (same).  Value = s * (hi + lo * kLoScale) with s the
// (k, 256-column tile) scale.
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

template <Fmt16 FMT, bool LO>
struct Entry {
  using type = typename std::conditional<LO, uint2, uint32_t>::type;
  __device__ static __forceinline__ cpx<float> value(uint2 e) {
    cpx<float> v = {Dec<FMT>::lo16(e.x), Dec<FMT>::hi16(e.x)};
    v.x = fmaf(Dec<FMT>::lo16(e.y), Dec<FMT>::kLoScale, v.x);
    v.y = fmaf(Dec<FMT>::hi16(e.y), Dec<FMT>::kLoScale, v.y);
    return v;
  }
  __device__ static __forceinline__ cpx<float> value(uint32_t e) {
    return {Dec<FMT>::lo16(e), Dec<FMT>::hi16(e)};
  }
};

template <int R, Fmt16 FMT, bool LO>
__global__ void __launch_bounds__(256)
gemv_rows_mixed_kernel(const void* __restrict__ Araw,
                       const float* __restrict__ scales,
                       const cpx<float>* __restrict__ X,
                       cpx<double>* __restrict__ P, GemvShape g, int64_t b) {
  using E = typename Entry<FMT, LO>::type;
  const E* __restrict__ A = static_cast<const E*>(Araw);
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

  const E* Ar[R];
#pragma unroll
  for (int r = 0; r < R; ++r) Ar[r] = A + (k * g.Nd + min(s0 + r, g.Nd - 1)) * g.Nm;
  const cpx<float>* Xk = X + (b * g.nf + k) * g.Nm;

  float ar[R], ai[R];
#pragma unroll
  for (int r = 0; r < R; ++r) ar[r] = ai[r] = 0.0f;

#pragma unroll 2
  for (int64_t p = p0 + lane; p < p1; p += 64) {
    cpx<float> x = Xk[p];
    const float sc = sk[p / kScaleTile];
    x.x *= sc;
    x.y *= sc;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const cpx<float> a = Entry<FMT, LO>::value(Ar[r][p]);
      ar[r] = fmaf(a.x, x.x, fmaf(-a.y, x.y, ar[r]));
      ai[r] = fmaf(a.x, x.y, fmaf(a.y, x.x, ai[r]));
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

template <int J, Fmt16 FMT, bool LO>
__global__ void __launch_bounds__(256)
gemv_cols_mixed_kernel(const void* __restrict__ Araw,
                       const float* __restrict__ scales,
                       const cpx<float>* __restrict__ D,
                       cpx<float>* __restrict__ Y, GemvShape g, int64_t b) {
  using E = typename Entry<FMT, LO>::type;
  const E* __restrict__ A = static_cast<const E*>(Araw);
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave_id_in_block();
  const int64_t npg = (g.Nm + 64 * J - 1) / (64 * J);
  const int64_t pg = wave % npg;
  const int64_t k = wave / npg;
  if (k >= g.nf) return;
  int64_t pj[J];
#pragma unroll
  for (int j = 0; j < J; ++j) pj[j] = min(pg * 64 * J + j * 64 + lane, g.Nm - 1);
  const E* Ak = A + k * g.Nd * g.Nm;
  const cpx<float>* Dk = D + (b * g.nf + k) * g.Nd;

  float yr[J], yi[J];
#pragma unroll
  for (int j = 0; j < J; ++j) yr[j] = yi[j] = 0.0f;

#pragma unroll 4
  for (int64_t s = 0; s < g.Nd; ++s) {
    const cpx<float> dv = Dk[s];
    const E* As = Ak + s * g.Nm;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const cpx<float> a = Entry<FMT, LO>::value(As[pj[j]]);
      yr[j] = fmaf(a.x, dv.x, fmaf(a.y, dv.y, yr[j]));
      yi[j] = fmaf(a.x, dv.y, fmaf(-a.y, dv.x, yi[j]));
    }
  }
  const int64_t ntiles = (g.Nm + kScaleTile - 1) / kScaleTile;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int64_t p = pg * 64 * J + j * 64 + lane;
    if (p >= g.Nm) break;
    const float sc = scales[k * ntiles + p / kScaleTile];
    Y[(b * g.nf + k) * g.Nm + p] = {yr[j] * sc, yi[j] * sc};
  }
}

inline unsigned blocks_for_waves(int64_t waves) {
  return (unsigned)((waves + 3) / 4);  // 4 wavefronts per 256-thread block
}

constexpr int kRowsF64 = 4;
constexpr int kColsF64 = 2;
constexpr int kRowsMixed = 4;
constexpr int kColsMixed = 2;

template <int B>
hipError_t rows_f64_pass(const cpx<double>* A, const cpx<double>* X,
                         cpx<double>* P, const GemvShape& g, int64_t b0, int nb,
                         hipStream_t s) {
  const int64_t waves = g.nf * ((g.Nd + kRowsF64 - 1) / kRowsF64) * g.n_pc;
  hipLaunchKernelGGL((gemv_rows_f64_kernel<kRowsF64, B>), dim3(blocks_for_waves(waves)),
                     dim3(256), 0, s, A, X, P, g, b0, nb);
  return hipGetLastError();
}

template <int B>
hipError_t cols_f64_pass(const cpx<double>* A, const cpx<double>* D,
                         cpx<double>* Y, const GemvShape& g, int64_t b0, int nb,
                         hipStream_t s) {
  const int64_t waves = g.nf * ((g.Nm + 64 * kColsF64 - 1) / (64 * kColsF64));
  hipLaunchKernelGGL((gemv_cols_f64_kernel<kColsF64, B>), dim3(blocks_for_waves(waves)),
                     dim3(256), 0, s, A, D, Y, g, b0, nb);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gemv_rows_f64(const cpx<double>* A, const cpx<double>* X,
                                cpx<double>* P, const GemvShape& g,
                                hipStream_t s) {
  for (int64_t b0 = 0; b0 < g.nrhs;) {
    const int64_t left = g.nrhs - b0;
    hipError_t e;
    int step;
    if (left >= 4) { e = rows_f64_pass<4>(A, X, P, g, b0, 4, s); step = 4; }
    else if (left >= 2) { e = rows_f64_pass<2>(A, X, P, g, b0, 2, s); step = 2; }
    else { e = rows_f64_pass<1>(A, X, P, g, b0, 1, s); step = 1; }
    if (e != hipSuccess) return e;
    b0 += step;
  }
  return hipSuccess;
}

hipError_t launch_gemv_cols_f64(const cpx<double>* A, const cpx<double>* D,
                                cpx<double>* Y, const GemvShape& g,
                                hipStream_t s) {
  for (int64_t b0 = 0; b0 < g.nrhs;) {
    const int64_t left = g.nrhs - b0;
    hipError_t e;
    int step;
    if (left >= 4) { e = cols_f64_pass<4>(A, D, Y, g, b0, 4, s); step = 4; }
    else if (left >= 2) { e = cols_f64_pass<2>(A, D, Y, g, b0, 2, s); step = 2; }
    else { e = cols_f64_pass<1>(A, D, Y, g, b0, 1, s); step = 1; }
    if (e != hipSuccess) return e;
    b0 += step;
  }
  return hipSuccess;
}

hipError_t launch_gemv_rows_mixed(const uint2* A, const float* scales,
                                  const cpx<float>* X, cpx<double>* P,
                                  const GemvShape& g, Fmt16 fmt, bool use_lo,
                                  hipStream_t s) {
  const int64_t waves = g.nf * ((g.Nd + kRowsMixed - 1) / kRowsMixed) * g.n_pc;
  for (int64_t b = 0; b < g.nrhs; ++b) {
    if (fmt == Fmt16::FP16 && use_lo)
      hipLaunchKernelGGL((gemv_rows_mixed_kernel<kRowsMixed, Fmt16::FP16, true>),
                         dim3(blocks_for_waves(waves)), dim3(256), 0, s, A, scales, X, P, g, b);
    else if (fmt == Fmt16::BF16 && use_lo)
      hipLaunchKernelGGL((gemv_rows_mixed_kernel<kRowsMixed, Fmt16::BF16, true>),
                         dim3(blocks_for_waves(waves)), dim3(256), 0, s, A, scales, X, P, g, b);
    else if (fmt == Fmt16::BF16)
      hipLaunchKernelGGL((gemv_rows_mixed_kernel<kRowsMixed, Fmt16::BF16, false>),
                         dim3(blocks_for_waves(waves)), dim3(256), 0, s, A, scales, X, P, g, b);
    else
      hipLaunchKernelGGL((gemv_rows_mixed_kernel<kRowsMixed, Fmt16::FP16, false>),
                         dim3(blocks_for_waves(waves)), dim3(256), 0, s, A, scales, X, P, g, b);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_gemv_cols_mixed(const uint2* A, const float* scales,
                                  const cpx<float>* D, cpx<float>* Y,
                                  const GemvShape& g, Fmt16 fmt, bool use_lo,
                                  hipStream_t s) {
  const int64_t waves = g.nf * ((g.Nm + 64 * kColsMixed - 1) / (64 * kColsMixed));
  for (int64_t b = 0; b < g.nrhs; ++b) {
    if (fmt == Fmt16::FP16 && use_lo)
      hipLaunchKernelGGL((gemv_cols_mixed_kernel<kColsMixed, Fmt16::FP16, true>),
                         dim3(blocks_for_waves(waves)), dim3(256), 0, s, A, scales, D, Y, g, b);
    else if (fmt == Fmt16::BF16 && use_lo)
      hipLaunchKernelGGL((gemv_cols_mixed_kernel<kColsMixed, Fmt16::BF16, true>),
                         dim3(blocks_for_waves(waves)), dim3(256), 0, s, A, scales, D, Y, g, b);
    else if (fmt == Fmt16::BF16)
      hipLaunchKernelGGL((gemv_cols_mixed_kernel<kColsMixed, Fmt16::BF16, false>),
                         dim3(blocks_for_waves(waves)), dim3(256), 0, s, A, scales, D, Y, g, b);
    else
      hipLaunchKernelGGL((gemv_cols_mixed_kernel<kColsMixed, Fmt16::FP16, false>),
                         dim3(blocks_for_waves(waves)), dim3(256), 0, s, A, scales, D, Y, g, b);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace p2o
