// Bodies of the vector-unit frequency-block product kernels (section
// "FFT-based Hessian matvecs", item (iii): one complex block product per
// frequency) and the helpers shared with the matrix-core units
// (matrix_units.h).  Every unit function here is executed by one 64-lane
// wavefront with uniform arguments naming one unit of work (frequency k, a
// tile of sensors or columns, a column chunk, a range of right-hand sides);
// the per-kernel launchers (gemv.hip) decode those from the grid, and the
// persistent multi-instance kernel (batch.hip) from its work ranges, so
// both run the same code.
#pragma once

#include "p2o_internal.h"

namespace p2o {
namespace {

typedef double d2v __attribute__((ext_vector_type(2)));
typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
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

// Block entries are streamed once per apply: non-temporal loads keep them
// out of the caches, which stay with the reused vector operands.
__device__ __forceinline__ cpx<double> ld_block(const cpx<double>* p) {
  const d2v v = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(p));
  return {v.x, v.y};
}

__device__ __forceinline__ d4v mfma64(double a, double b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
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

__device__ __forceinline__ f4v mma(u4v a, u4v b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8v, a),
                                                 __builtin_bit_cast(bf8v, b), c, 0, 0, 0);
}

// Pack the low (real) or high (imaginary) 16-bit halves of 8 words into a
// bfloat16x8 operand.
__device__ __forceinline__ u4v lows(const uint32_t* w) {
  u4v r;
#pragma unroll
  for (int q = 0; q < 4; ++q) r[q] = __builtin_amdgcn_perm(w[2 * q + 1], w[2 * q], 0x05040100u);
  return r;
}
__device__ __forceinline__ u4v highs(const uint32_t* w) {
  u4v r;
#pragma unroll
  for (int q = 0; q < 4; ++q) r[q] = __builtin_amdgcn_perm(w[2 * q + 1], w[2 * q], 0x07060302u);
  return r;
}
__device__ __forceinline__ u4v neg(u4v v) {
  return v ^ (u4v){0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
}

__device__ __forceinline__ u4v ld16(const uint16_t* p) {
  return *reinterpret_cast<const u4v*>(p);
}

// ------------------------------------------------- vector-unit units, float64
template <int R, int B>
__device__ __forceinline__ void rows_f64_unit(const cpx<double>* __restrict__ A,
                     const cpx<double>* __restrict__ X,
                     cpx<double>* __restrict__ P, GemvShape g, int64_t b0,
                     int nb, int64_t k, int64_t sg, int64_t pc) {
  const int lane = threadIdx.x & 63;
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
__device__ __forceinline__ void cols_f64_unit(const cpx<double>* __restrict__ A,
                     const cpx<double>* __restrict__ D,
                     cpx<double>* __restrict__ Y, GemvShape g, int64_t b0,
                     int nb, int64_t k, int64_t pg) {
  const int lane = threadIdx.x & 63;
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

// -------------------------------------------------- vector-unit units, mixed
template <int R, int V, Fmt16 FMT, bool LO>
__device__ __forceinline__ void rows_mixed_unit(const void* __restrict__ A,
                       const float* __restrict__ scales,
                       const cpx<float>* __restrict__ X,
                       cpx<double>* __restrict__ P, GemvShape g, int64_t b, int64_t k, int64_t sg, int64_t pc) {
  using PK = Pack<LO, V>;
  constexpr int WPE = LO ? 2 : 1;  // words per entry
  const int lane = threadIdx.x & 63;
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
__device__ __forceinline__ void cols_mixed_unit(const void* __restrict__ A,
                       const float* __restrict__ scales,
                       const cpx<float>* __restrict__ D,
                       cpx<float>* __restrict__ Y, GemvShape g, int64_t b, int64_t k, int64_t pg) {
  using PK = Pack<LO, V>;
  constexpr int kCols = 64 * J * V;  // columns per wavefront
  constexpr int WPE = LO ? 2 : 1;
  const int lane = threadIdx.x & 63;
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

}  // namespace
}  // namespace p2o
