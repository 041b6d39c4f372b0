// Wave-level bodies of the frequency-block product kernels (section
// "FFT-based Hessian matvecs", item (iii): one complex block product per
// frequency).  Every function here is executed by a whole 64-lane wavefront
// with wave-uniform arguments naming one unit of work (frequency k, a tile
// of sensors or columns, a column chunk, a range of right-hand sides); the
// per-kernel launchers decode those from the grid, and the persistent
// multi-instance kernel decodes them from its work ranges, so both run the
// same code.  See gemv.hip, gemm_f64.hip and gemm_bf16.hip for the design
// of each family.
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

// --------------------------------------------------- matrix-core units, f64
template <int NT>
__device__ __forceinline__ void mfma_rows_f64_unit(const cpx<double>* __restrict__ A, const cpx<double>* __restrict__ X,
              cpx<double>* __restrict__ P, GemvShape g, int64_t b0, int nb, int64_t k, int64_t mt, int64_t pc) {
  const int lane = threadIdx.x & 63;
  const int64_t p0 = pc * g.pc_len;
  const int64_t p1 = min(p0 + g.pc_len, g.Nm);
  const int col = lane & 15, kg = lane >> 4;
  const int64_t srow = min(mt * 16 + col, g.Nd - 1);  // A row this lane supplies
  const cpx<double>* __restrict__ Arow = A + (k * g.Nd + srow) * g.Nm;
  const cpx<double>* Xrow[NT];
  bool xok[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int b = t * 16 + col;
    xok[t] = b < nb;
    Xrow[t] = X + ((b0 + (xok[t] ? b : 0)) * g.nf + k) * g.Nm;
  }
  d4v accr[NT], acci[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) accr[t] = acci[t] = (d4v){0, 0, 0, 0};

  for (int64_t base = p0; base < p1; base += 32) {
    const int64_t q = base + 8 * kg;
    cpx<double> a[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = (q + j < p1) ? ld_block(Arow + q + j) : cpx<double>{0, 0};
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      cpx<double> x[8];
#pragma unroll
      for (int j = 0; j < 8; ++j)
        x[j] = (xok[t] && q + j < p1) ? Xrow[t][q + j] : cpx<double>{0, 0};
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        accr[t] = mfma64(a[j].x, x[j].x, accr[t]);
        accr[t] = mfma64(a[j].y, -x[j].y, accr[t]);
        acci[t] = mfma64(a[j].x, x[j].y, acci[t]);
        acci[t] = mfma64(a[j].y, x[j].x, acci[t]);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int b = t * 16 + col;
    if (b >= nb) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t s = mt * 16 + kg + 4 * i;  // float64 accumulator rows interleave
      if (s < g.Nd)
        P[(((b0 + b) * g.n_pc + pc) * g.nf + k) * g.Nd + s] = {accr[t][i], acci[t][i]};
    }
  }
}

template <int MT>
__device__ __forceinline__ void mfma_cols_f64_unit(const cpx<double>* __restrict__ A, const cpx<double>* __restrict__ D,
              cpx<double>* __restrict__ Y, GemvShape g, int64_t b0, int nb, int64_t k, int64_t pt) {
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, kg = lane >> 4;
  const int64_t pcol = min(pt * 16 + col, g.Nm - 1);  // Fhat column this lane supplies
  const cpx<double>* __restrict__ Ak = A + k * g.Nd * g.Nm + pcol;
  const cpx<double>* Drow[MT];
  bool dok[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) {
    const int b = t * 16 + col;
    dok[t] = b < nb;
    Drow[t] = D + ((b0 + (dok[t] ? b : 0)) * g.nf + k) * g.Nd;
  }
  d4v accr[MT], acci[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) accr[t] = acci[t] = (d4v){0, 0, 0, 0};

  for (int64_t base = 0; base < g.Nd; base += 32) {
    const int64_t q = base + 8 * kg;
    cpx<double> f[8];
#pragma unroll
    for (int j = 0; j < 8; ++j)
      f[j] = (q + j < g.Nd) ? ld_block(Ak + (q + j) * g.Nm) : cpx<double>{0, 0};
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      cpx<double> d[8];
#pragma unroll
      for (int j = 0; j < 8; ++j)
        d[j] = (dok[t] && q + j < g.Nd) ? Drow[t][q + j] : cpx<double>{0, 0};
#pragma unroll
      for (int j = 0; j < 8; ++j) {  // x += conj(f) d
        accr[t] = mfma64(d[j].x, f[j].x, accr[t]);
        accr[t] = mfma64(d[j].y, f[j].y, accr[t]);
        acci[t] = mfma64(d[j].y, f[j].x, acci[t]);
        acci[t] = mfma64(-d[j].x, f[j].y, acci[t]);
      }
    }
  }
  const int64_t p = pt * 16 + col;
  if (p >= g.Nm) return;
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int b = t * 16 + kg + 4 * i;  // float64 accumulator rows interleave
      if (b < nb) Y[((b0 + b) * g.nf + k) * g.Nm + p] = {accr[t][i], acci[t][i]};
    }
}

// ------------------------------------------------ matrix-core units, bf16
template <int NT, bool LO, bool VEC>
__device__ __forceinline__ void mfma_rows_bf16_unit(const uint32_t* __restrict__ A, const float* __restrict__ scales,
               const uint16_t* __restrict__ Xs, cpx<double>* __restrict__ P, GemvShape g,
               int64_t n8, int64_t b0, int nb, int64_t k, int64_t mt, int64_t pc) {
  constexpr int WPE = LO ? 2 : 1;  // words per entry
  const int lane = threadIdx.x & 63;
  const int64_t p0 = pc * g.pc_len;
  const int64_t p1 = min(p0 + g.pc_len, g.Nm);
  const int col = lane & 15, kg = lane >> 4;
  const int64_t srow = min(mt * 16 + col, g.Nd - 1);
  const uint32_t* __restrict__ Arow = A + (k * g.Nd + srow) * g.Nm * WPE;
  const int64_t ntiles = (g.Nm + kScaleTile - 1) / kScaleTile;
  const float* __restrict__ sk = scales + k * ntiles;
  const uint16_t* Xb[NT];
  bool xok[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int b = t * 16 + col;
    xok[t] = b < nb;
    Xb[t] = Xs + ((b0 + (xok[t] ? b : 0)) * g.nf + k) * 4 * n8;
  }
  double accr[NT][4], acci[NT][4];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) accr[t][i] = acci[t][i] = 0.0;

  // walk the chunk in pieces that never straddle a 256-column scale tile
  for (int64_t tb = p0, te; tb < p1; tb = te) {
    te = min((tb / kScaleTile + 1) * kScaleTile, p1);
    f4v tr[NT], ti[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) tr[t] = ti[t] = (f4v){0, 0, 0, 0};
    for (int64_t base = tb; base < te; base += 32) {
      const int64_t q = base + 8 * kg;
      uint32_t w0[8], w1[8];
      if (VEC && q + 8 <= te) {
        if constexpr (LO) {
#pragma unroll
          for (int h = 0; h < 4; ++h) {
            const u4v v = __builtin_nontemporal_load(reinterpret_cast<const u4v*>(Arow + 2 * (q + 2 * h)));
            w0[2 * h] = v[0];
            w1[2 * h] = v[1];
            w0[2 * h + 1] = v[2];
            w1[2 * h + 1] = v[3];
          }
        } else {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const u4v v = __builtin_nontemporal_load(reinterpret_cast<const u4v*>(Arow + q + 4 * h));
#pragma unroll
            for (int e = 0; e < 4; ++e) w0[4 * h + e] = v[e];
          }
        }
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const bool ok = q + j < te;
          w0[j] = ok ? Arow[(q + j) * WPE] : 0u;
          w1[j] = (LO && ok) ? Arow[(q + j) * WPE + 1] : 0u;
        }
      }
      const u4v hr = lows(w0), hi = highs(w0);
      const u4v nhi = neg(hi);
      u4v lr = {0, 0, 0, 0}, li = {0, 0, 0, 0}, nli = {0, 0, 0, 0};
      if constexpr (LO) {
        lr = lows(w1);
        li = highs(w1);
        nli = neg(li);
      }
      const bool qok = q < te;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        u4v xrh = {0, 0, 0, 0}, xrl = xrh, xih = xrh, xil = xrh;
        if (xok[t] && qok) {
          xrh = ld16(Xb[t] + 0 * n8 + q);
          xrl = ld16(Xb[t] + 1 * n8 + q);
          xih = ld16(Xb[t] + 2 * n8 + q);
          xil = ld16(Xb[t] + 3 * n8 + q);
        }
        // re: Hr xr - Hi xi ; im: Hr xi + Hi xr   (each with hi/lo splits)
        tr[t] = mma(hr, xrh, tr[t]);
        tr[t] = mma(hr, xrl, tr[t]);
        tr[t] = mma(nhi, xih, tr[t]);
        tr[t] = mma(nhi, xil, tr[t]);
        ti[t] = mma(hr, xih, ti[t]);
        ti[t] = mma(hr, xil, ti[t]);
        ti[t] = mma(hi, xrh, ti[t]);
        ti[t] = mma(hi, xrl, ti[t]);
        if constexpr (LO) {
          tr[t] = mma(lr, xrh, tr[t]);
          tr[t] = mma(nli, xih, tr[t]);
          ti[t] = mma(lr, xih, ti[t]);
          ti[t] = mma(li, xrh, ti[t]);
        }
      }
    }
    const double sc = (double)sk[tb / kScaleTile];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        accr[t][i] += sc * (double)tr[t][i];
        acci[t][i] += sc * (double)ti[t][i];
      }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int b = t * 16 + col;
    if (b >= nb) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t s = mt * 16 + 4 * kg + i;
      if (s < g.Nd)
        P[(((b0 + b) * g.n_pc + pc) * g.nf + k) * g.Nd + s] = {accr[t][i], acci[t][i]};
    }
  }
}

template <int MT, bool LO>
__device__ __forceinline__ void mfma_cols_bf16_unit(const uint32_t* __restrict__ A, const float* __restrict__ scales,
               const uint16_t* __restrict__ Ds, cpx<float>* __restrict__ Y, GemvShape g,
               int64_t nd8, int64_t b0, int nb, int64_t k, int64_t pt) {
  constexpr int WPE = LO ? 2 : 1;
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, kg = lane >> 4;
  const int64_t pcol = min(pt * 16 + col, g.Nm - 1);
  const uint32_t* __restrict__ Ak = A + (k * g.Nd * g.Nm + pcol) * WPE;
  const uint16_t* Db[MT];
  bool dok[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) {
    const int b = t * 16 + col;
    dok[t] = b < nb;
    Db[t] = Ds + ((b0 + (dok[t] ? b : 0)) * g.nf + k) * 4 * nd8;
  }
  f4v xr[MT], xi[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) xr[t] = xi[t] = (f4v){0, 0, 0, 0};

  for (int64_t base = 0; base < g.Nd; base += 32) {
    const int64_t q = base + 8 * kg;
    uint32_t w0[8], w1[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const bool ok = q + j < g.Nd;
      if constexpr (LO) {
        const u2v v = ok ? __builtin_nontemporal_load(
                               reinterpret_cast<const u2v*>(Ak + (q + j) * g.Nm * 2))
                         : (u2v){0u, 0u};
        w0[j] = v[0];
        w1[j] = v[1];
      } else {
        w0[j] = ok ? __builtin_nontemporal_load(Ak + (q + j) * g.Nm) : 0u;
        w1[j] = 0u;
      }
    }
    const u4v fr = lows(w0), fi = highs(w0);
    const u4v nfi = neg(fi);
    u4v lr = {0, 0, 0, 0}, nli = {0, 0, 0, 0};
    if constexpr (LO) {
      lr = lows(w1);
      nli = neg(highs(w1));
    }
    const u4v li = neg(nli);
    const bool qok = q < g.Nd;
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      u4v drh = {0, 0, 0, 0}, drl = drh, dih = drh, dil = drh;
      if (dok[t] && qok) {
        drh = ld16(Db[t] + 0 * nd8 + q);
        drl = ld16(Db[t] + 1 * nd8 + q);
        dih = ld16(Db[t] + 2 * nd8 + q);
        dil = ld16(Db[t] + 3 * nd8 + q);
      }
      // x += conj(f) d: re = dr fr + di fi ; im = di fr - dr fi
      xr[t] = mma(drh, fr, xr[t]);
      xr[t] = mma(drl, fr, xr[t]);
      xr[t] = mma(dih, fi, xr[t]);
      xr[t] = mma(dil, fi, xr[t]);
      xi[t] = mma(dih, fr, xi[t]);
      xi[t] = mma(dil, fr, xi[t]);
      xi[t] = mma(drh, nfi, xi[t]);
      xi[t] = mma(drl, nfi, xi[t]);
      if constexpr (LO) {
        xr[t] = mma(drh, lr, xr[t]);
        xr[t] = mma(dih, li, xr[t]);
        xi[t] = mma(dih, lr, xi[t]);
        xi[t] = mma(drh, nli, xi[t]);
      }
    }
  }
  const int64_t p = pt * 16 + col;
  if (p >= g.Nm) return;
  const int64_t ntiles = (g.Nm + kScaleTile - 1) / kScaleTile;
  const float sc = scales[k * ntiles + p / kScaleTile];
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int b = t * 16 + 4 * kg + i;
      if (b < nb) Y[((b0 + b) * g.nf + k) * g.Nm + p] = {xr[t][i] * sc, xi[t][i] * sc};
    }
}

}  // namespace
}  // namespace p2o
