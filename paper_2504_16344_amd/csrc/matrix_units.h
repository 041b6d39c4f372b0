// Bodies of the matrix-core (MFMA) frequency-block product kernels for many
// right-hand sides (section "FFT-based Hessian matvecs", item (iii), applied
// to a block of vectors): workgroup-level functions shared by the
// per-plan launchers (gemm_f64.hip, gemm_bf16.hip) and the persistent
// multi-instance kernel (batch.hip).
#pragma once

#include "product_units.h"

namespace p2o {
namespace {

// ------------------------------------------------------ matrix-core units
// Workgroup-cooperative: the 4 wavefronts of a 256-thread workgroup cover 64
// rows (F) or 64 columns (F*) of one frequency and walk the contraction in
// 32-entry chunks.  Each chunk of the vector operand (all right-hand sides
// of the pass) is staged in LDS once per workgroup and read by all 4
// wavefronts, so vector traffic per block byte is a quarter of what one
// wavefront alone would fetch; block entries stream from HBM straight into
// the matrix-core operands.  The loop is software-pipelined over a double
// LDS buffer: a wavefront first issues the next chunk's vector loads, then
// its block loads, then runs the current chunk's products, and only then
// waits for the vector loads (which were issued first, so the block loads
// stay in flight) to store them into the other buffer; one barrier per
// chunk.  All wavefronts of the workgroup must call a unit together.
constexpr int kWgTile = 64;       // float64 units: rows (F) / columns (F*) per workgroup
constexpr int kBf16Threads = 512;  // bfloat16 units: 8 wavefronts per workgroup
constexpr int kBf16Tile = 128;     // bfloat16 units: rows (F) / columns (F*) per workgroup
constexpr int kXcds = 8;

// LDS bytes of the double stage buffer for 16 NT right-hand sides.
__host__ __device__ constexpr int stage_bytes_f64(int nt) { return 2 * 32 * (16 * nt + 1) * 16; }
__host__ __device__ constexpr int stage_bytes_bf16(int nt) { return 2 * 16 * (16 * nt + 1) * 16; }

// Workgroups are handed to the 8 XCDs round-robin by workgroup index, and
// each XCD has its own L2.  For a grid padded to a multiple of 8, this maps
// the workgroup index so every XCD runs a contiguous range of tiles:
// neighbouring tiles (same frequency, same vector chunks) then meet in one
// L2 instead of being spread over all eight.
__device__ __forceinline__ int64_t xcd_local_tile(int64_t bid, int64_t grid) {
  return (bid % kXcds) * (grid / kXcds) + bid / kXcds;
}

// ---- vector-operand staging: global -> registers (issued early) -> LDS.
// The loads fetch raw values from clamped, valid addresses; the stores
// (which wait for the loads anyway) zero the positions past `end` or past
// the nb right-hand sides of the pass, so nothing between the two has to
// wait for the data.
// float64 vectors: entries [base, base + 32) of vector rows b0 .. b0 + 16 NT - 1
// (row b at src + ((b0 + b) nf + k) len), stored as s[entry * (16 NT + 1) + b].
template <int NT>
__device__ __forceinline__ void stage_f64_load(const cpx<double>* __restrict__ src, int64_t nf,
                                               int64_t k, int64_t len, int64_t b0, int nb,
                                               int64_t base, int64_t end,
                                               cpx<double> (&v)[2 * NT]) {
#pragma unroll
  for (int i = 0; i < 2 * NT; ++i) {
    const int e = threadIdx.x + 256 * i, ent = e & 31, b = e >> 5;
    const bool ok = b < nb && base + ent < end;
    v[i] = src[ok ? ((b0 + b) * nf + k) * len + base + ent : 0];
  }
}

template <int NT>
__device__ __forceinline__ void stage_f64_store(const cpx<double> (&v)[2 * NT], int nb,
                                                int64_t base, int64_t end, cpx<double>* s) {
  constexpr int PP = NT * 16 + 1;
#pragma unroll
  for (int i = 0; i < 2 * NT; ++i) {
    const int e = threadIdx.x + 256 * i, ent = e & 31, b = e >> 5;
    const bool ok = b < nb && base + ent < end;
    s[ent * PP + b] = ok ? v[i] : cpx<double>{0, 0};
  }
}

// bfloat16 planes: 8-entry parts of the 4 planes of each vector row
// (256 NT parts per chunk), spread over TH threads, PER parts each.
template <int NT, int TH>
constexpr int parts_per_thread() { return (256 * NT + TH - 1) / TH; }

// SLOTS: F's planes, stored per 32-entry chunk in slot order (part kg of a
// chunk holds slots 0..7 of lane group kg, and the planes are zero past the
// contraction up to a multiple of 32), so a chunk is valid as a whole; F*'s
// planes are in sensor order and a part is valid if it starts before `end`.
template <int NT, int TH, bool SLOTS>
__device__ __forceinline__ void stage_planes_load(const uint16_t* __restrict__ planes,
                                                  int64_t nf, int64_t k, int64_t n8, int64_t b0,
                                                  int nb, int64_t base, int64_t end,
                                                  u4v (&v)[parts_per_thread<NT, TH>()]) {
#pragma unroll
  for (int i = 0; i < parts_per_thread<NT, TH>(); ++i) {
    const int e = threadIdx.x + TH * i;
    const int part = e & 3, plane = (e >> 2) & 3, b = e >> 4;
    const int64_t q = base + 8 * part;
    const bool ok = e < 256 * NT && b < nb && (SLOTS ? base : q) < end;
    v[i] = ld16(planes + (ok ? (((b0 + b) * nf + k) * 4 + plane) * n8 + q : 0));
  }
}

template <bool SLOTS>
__device__ __forceinline__ u4v stage_part(const u4v& v, int e, int nb, int64_t base,
                                          int64_t end) {
  const bool ok = (e >> 4) < nb && (SLOTS ? base : base + 8 * (e & 3)) < end;
  return ok ? v : (u4v){0, 0, 0, 0};
}

// Stage layout: s[(plane * 4 + part) * (16 NT + 1) + b] holds part `part`
// of one plane (F*: sensors base + 8 part .. + 7; F: slots 0..7 of lane
// group `part`).
template <int NT, int TH, bool SLOTS>
__device__ __forceinline__ void stage_planes_store(const u4v (&v)[parts_per_thread<NT, TH>()],
                                                   int nb, int64_t base, int64_t end, u4v* s) {
  constexpr int PP = NT * 16 + 1;
#pragma unroll
  for (int i = 0; i < parts_per_thread<NT, TH>(); ++i) {
    const int e = threadIdx.x + TH * i;
    if (256 * NT % TH == 0 || e < 256 * NT)
      s[(((e >> 2) & 3) * 4 + (e & 3)) * PP + (e >> 4)] = stage_part<SLOTS>(v[i], e, nb, base, end);
  }
}

// ---- block-operand loads (non-temporal, straight into registers).
// Every load here and in the staging helpers is issued unconditionally, so
// the loop bodies stay straight-line and the compiler's wait before the LDS
// store counts only the vector loads, leaving the block loads in flight.  A
// block lane past the end of the contraction reads a clamped, valid address;
// its value is a finite block entry and meets the zero that the stage
// stores for that vector position, so it adds exactly nothing.
// F, float64: instruction j takes entry base + 4 j + kg, so the 4 lane
// groups of a row read 64 contiguous bytes per load.
__device__ __forceinline__ void load_row_f64(const cpx<double>* __restrict__ Arow, int64_t base,
                                             int kg, int64_t end, cpx<double> (&a)[8]) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int64_t e = base + 4 * j + kg;
    a[j] = ld_block(Arow + (e < end ? e : 0));
  }
}

// F*, float64: sensors q .. q + 7 of one column.
__device__ __forceinline__ void load_col_f64(const cpx<double>* __restrict__ Acol, int64_t q,
                                             int64_t Nd, int64_t Nm, cpx<double> (&f)[8]) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    f[j] = ld_block(Acol + (q + j < Nd ? (q + j) * Nm : 0));
  }
}

// F, bfloat16 words (hi, lo) of slots 0..7 of lane group kg, chunk at
// `base`; entries at or past `end` read the row's first entry instead.  With
// VEC the row is 16-byte aligned and `end` a multiple of the entries per
// load, so each 16-byte load is wholly in or out.
template <bool LO, bool VEC>
__device__ __forceinline__ void load_row_slots(const uint32_t* __restrict__ Arow, int64_t base,
                                               int kg, int64_t end, uint32_t (&w0)[8],
                                               uint32_t (&w1)[8]) {
  constexpr int WPE = LO ? 2 : 1;
  if constexpr (VEC && LO) {
#pragma unroll
    for (int h = 0; h < 4; ++h) {  // entries base + 8 h + 2 kg + {0, 1}
      const int64_t e = base + 8 * h + 2 * kg;
      const u4v v = __builtin_nontemporal_load(reinterpret_cast<const u4v*>(Arow + 2 * (e < end ? e : 0)));
      w0[2 * h] = v[0];
      w1[2 * h] = v[1];
      w0[2 * h + 1] = v[2];
      w1[2 * h + 1] = v[3];
    }
  } else if constexpr (VEC) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {  // entries base + 16 h + 4 kg + {0..3}
      const int64_t e = base + 16 * h + 4 * kg;
      const u4v v = __builtin_nontemporal_load(reinterpret_cast<const u4v*>(Arow + (e < end ? e : 0)));
#pragma unroll
      for (int c = 0; c < 4; ++c) w0[4 * h + c] = v[c];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) w1[j] = 0u;
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int64_t e = base + row_slot_entry(LO, kg, j);
      const uint32_t* at = Arow + (e < end ? e : 0) * WPE;
      w0[j] = __builtin_nontemporal_load(at);
      w1[j] = LO ? __builtin_nontemporal_load(at + 1) : 0u;
    }
  }
}

// F*, bfloat16 words of sensors q .. q + 7 of one column.
template <bool LO>
__device__ __forceinline__ void load_col8(const uint32_t* __restrict__ Acol, int64_t q,
                                          int64_t Nd, int64_t Nm, uint32_t (&w0)[8],
                                          uint32_t (&w1)[8]) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int64_t r = q + j < Nd ? q + j : 0;
    if constexpr (LO) {
      const u2v x = __builtin_nontemporal_load(reinterpret_cast<const u2v*>(Acol + r * Nm * 2));
      w0[j] = x[0];
      w1[j] = x[1];
    } else {
      w0[j] = __builtin_nontemporal_load(Acol + r * Nm);
      w1[j] = 0u;
    }
  }
}

// ---- units
// F, float64: rows mt*64 + 16 w .. of frequency k, column chunk pc, right-hand
// sides b0 .. b0 + nb - 1 (nb <= 16 NT).
template <int NT>
__device__ __forceinline__ void mfma_rows_f64_wg(const cpx<double>* __restrict__ A,
                                                 const cpx<double>* __restrict__ X,
                                                 cpx<double>* __restrict__ P, GemvShape g,
                                                 int64_t b0, int nb, int64_t k, int64_t mt,
                                                 int64_t pc, void* lds) {
  constexpr int PP = NT * 16 + 1, BUF = 32 * PP;
  cpx<double>* sx = static_cast<cpx<double>*>(lds);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, kg = lane >> 4;
  const int64_t p0 = pc * g.pc_len;
  const int64_t p1 = min(p0 + g.pc_len, g.Nm);
  const int64_t row0 = mt * kWgTile + 16 * wave;
  const cpx<double>* __restrict__ Arow = A + (k * g.Nd + min(row0 + col, g.Nd - 1)) * g.Nm;
  d4v accr[NT], acci[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) accr[t] = acci[t] = (d4v){0, 0, 0, 0};
  cpx<double> a[8];
  {
    cpx<double> v[2 * NT];
    stage_f64_load<NT>(X, g.nf, k, g.Nm, b0, nb, p0, p1, v);
    load_row_f64(Arow, p0, kg, p1, a);
    stage_f64_store<NT>(v, nb, p0, p1, sx);
  }
  __syncthreads();
  int cur = 0;
  for (int64_t base = p0; base < p1; base += 32) {
    const int64_t nend = base + 32 < p1 ? p1 : 0;  // 0: past the last chunk, all lanes off
    cpx<double> v[2 * NT], an[8];
    stage_f64_load<NT>(X, g.nf, k, g.Nm, b0, nb, base + 32, nend, v);
    __builtin_amdgcn_sched_barrier(0);  // vector loads first, then block loads
    load_row_f64(Arow, base + 32, kg, nend, an);
    __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the products
    const cpx<double>* xs = sx + cur * BUF;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {  // re / im chains alternate
        const cpx<double> x = xs[(4 * j + kg) * PP + t * 16 + col];
        accr[t] = mfma64(a[j].x, x.x, accr[t]);
        acci[t] = mfma64(a[j].x, x.y, acci[t]);
        accr[t] = mfma64(a[j].y, -x.y, accr[t]);
        acci[t] = mfma64(a[j].y, x.x, acci[t]);
      }
    }
    __builtin_amdgcn_sched_barrier(0);  // the store waits for the vector loads: after the products
    stage_f64_store<NT>(v, nb, base + 32, nend, sx + (cur ^ 1) * BUF);
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = an[j];
    __syncthreads();
    cur ^= 1;
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int b = t * 16 + col;
    if (b >= nb) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t s = row0 + kg + 4 * i;  // float64 accumulator rows interleave
      if (s < g.Nd)
        P[(((b0 + b) * g.n_pc + pc) * g.nf + k) * g.Nd + s] = {accr[t][i], acci[t][i]};
    }
  }
}

// F*, float64: columns pt*64 + 16 w .., X^T = Dhat^T conj(Fhat) over all sensors.
template <int MT>
__device__ __forceinline__ void mfma_cols_f64_wg(const cpx<double>* __restrict__ A,
                                                 const cpx<double>* __restrict__ D,
                                                 cpx<double>* __restrict__ Y, GemvShape g,
                                                 int64_t b0, int nb, int64_t k, int64_t pt,
                                                 void* lds) {
  constexpr int PP = MT * 16 + 1, BUF = 32 * PP;
  cpx<double>* sd = static_cast<cpx<double>*>(lds);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, kg = lane >> 4;
  const int64_t col0 = pt * kWgTile + 16 * wave;
  const cpx<double>* __restrict__ Ak = A + k * g.Nd * g.Nm + min(col0 + col, g.Nm - 1);
  d4v accr[MT], acci[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) accr[t] = acci[t] = (d4v){0, 0, 0, 0};
  cpx<double> f[8];
  {
    cpx<double> v[2 * MT];
    stage_f64_load<MT>(D, g.nf, k, g.Nd, b0, nb, 0, g.Nd, v);
    load_col_f64(Ak, 8 * kg, g.Nd, g.Nm, f);
    stage_f64_store<MT>(v, nb, 0, g.Nd, sd);
  }
  __syncthreads();
  int cur = 0;
  for (int64_t base = 0; base < g.Nd; base += 32) {
    const int64_t nend = base + 32 < g.Nd ? g.Nd : 0;  // 0: past the last chunk
    cpx<double> v[2 * MT], fn[8];
    stage_f64_load<MT>(D, g.nf, k, g.Nd, b0, nb, base + 32, nend, v);
    __builtin_amdgcn_sched_barrier(0);  // vector loads first, then block loads
    load_col_f64(Ak, base + 32 + 8 * kg, nend, g.Nm, fn);
    __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the products
    const cpx<double>* ds = sd + cur * BUF;
#pragma unroll
    for (int t = 0; t < MT; ++t) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {  // x += conj(f) d; re / im chains alternate
        const cpx<double> d = ds[(8 * kg + j) * PP + t * 16 + col];
        accr[t] = mfma64(d.x, f[j].x, accr[t]);
        acci[t] = mfma64(d.y, f[j].x, acci[t]);
        accr[t] = mfma64(d.y, f[j].y, accr[t]);
        acci[t] = mfma64(-d.x, f[j].y, acci[t]);
      }
    }
    __builtin_amdgcn_sched_barrier(0);  // the store waits for the vector loads: after the products
    stage_f64_store<MT>(v, nb, base + 32, nend, sd + (cur ^ 1) * BUF);
#pragma unroll
    for (int j = 0; j < 8; ++j) f[j] = fn[j];
    __syncthreads();
    cur ^= 1;
  }
  const int64_t p = col0 + col;
  if (p >= g.Nm) return;
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int b = t * 16 + kg + 4 * i;  // float64 accumulator rows interleave
      if (b < nb) Y[((b0 + b) * g.nf + k) * g.Nm + p] = {accr[t][i], acci[t][i]};
    }
}

// ---- bfloat16 matrix-core units.  The block loads run RING chunks ahead of
// the products through a ring of registers (unrolled, so every ring slot is
// a fixed register set): with a 32-entry chunk per step, one chunk in
// flight per wavefront is far too little to cover loaded HBM latency at
// these tile sizes, while the LDS vector stage is prefetched one chunk
// ahead (it hits in L2).

// Unpacked block operands of one chunk: real / imaginary hi parts, their
// negations where a product needs them, and the lo parts.
struct BlockOps {
  u4v hr, hi, nhi, lr, li, nli;
};

template <bool LO>
__device__ __forceinline__ BlockOps unpack_block(const uint32_t (&w0)[8], const uint32_t (&w1)[8]) {
  BlockOps o;
  o.hr = lows(w0);
  o.hi = highs(w0);
  o.nhi = neg(o.hi);
  o.lr = o.li = o.nli = (u4v){0, 0, 0, 0};
  if constexpr (LO) {
    o.lr = lows(w1);
    o.li = highs(w1);
    o.nli = neg(o.li);
  }
  return o;
}

// F chunk: t[b] += Fhat[rows, chunk] X[chunk, b] for the 16 NT right-hand
// sides; re: Hr xr - Hi xi, im: Hr xi + Hi xr, each with hi/lo splits.  The
// hi x hi products go to tr / ti, the hi x lo and lo x hi products (about
// 2^-8 of them) to their own accumulators sr / si: added to an accumulator
// 2^8 and more times larger, the matrix cores lose their low bits with a
// bias toward minus infinity (measured on gfx950), which over thousands of
// steps adds up coherently; summed among themselves they do not.
// xop(plane, t) returns this lane's operand of vector plane `plane` (re hi,
// re lo, im hi, im lo) for right-hand-side tile t.
template <int NT, bool LO, typename XOp>
__device__ __forceinline__ void rows_bf16_products(const BlockOps& a, XOp xop, f4v (&tr)[NT],
                                                   f4v (&ti)[NT], f4v (&sr)[NT],
                                                   f4v (&si)[NT]) {
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const u4v xrh = xop(0, t), xrl = xop(1, t);
    const u4v xih = xop(2, t), xil = xop(3, t);
    tr[t] = mma(a.hr, xrh, tr[t]);
    ti[t] = mma(a.hr, xih, ti[t]);
    sr[t] = mma(a.hr, xrl, sr[t]);
    si[t] = mma(a.hr, xil, si[t]);
    tr[t] = mma(a.nhi, xih, tr[t]);
    ti[t] = mma(a.hi, xrh, ti[t]);
    sr[t] = mma(a.nhi, xil, sr[t]);
    si[t] = mma(a.hi, xrl, si[t]);
    if constexpr (LO) {
      sr[t] = mma(a.lr, xrh, sr[t]);
      si[t] = mma(a.lr, xih, si[t]);
      sr[t] = mma(a.nli, xih, sr[t]);
      si[t] = mma(a.li, xrh, si[t]);
    }
  }
}

// The F chunk for U row sub-tiles that share the vector operands: the
// operands of tile t are read once, and each sub-tile's accumulators get
// exactly the sequence of rows_bf16_products.
template <int NT, bool LO, int U, typename XOp>
__device__ __forceinline__ void rows_bf16_products_sub(const BlockOps (&a)[U], XOp xop,
                                                       f4v (&tr)[U][NT], f4v (&ti)[U][NT],
                                                       f4v (&sr)[U][NT], f4v (&si)[U][NT]) {
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const u4v x0 = xop(0, t), x1 = xop(1, t), x2 = xop(2, t), x3 = xop(3, t);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      f4v r1[1] = {tr[u][t]}, i1[1] = {ti[u][t]}, s1[1] = {sr[u][t]}, j1[1] = {si[u][t]};
      rows_bf16_products<1, LO>(
          a[u], [&](int pl, int) { return pl == 0 ? x0 : pl == 1 ? x1 : pl == 2 ? x2 : x3; },
          r1, i1, s1, j1);
      tr[u][t] = r1[0];
      ti[u][t] = i1[0];
      sr[u][t] = s1[0];
      si[u][t] = j1[0];
    }
  }
}

// F* chunk: x[b] += conj(f) d[b]: re = dr fr + di fi, im = di fr - dr fi.
// As in the F chunk, the hi x hi products go to xr / xi and the hi x lo and
// lo x hi products to their own accumulators sr / si (the matrix cores'
// biased rounding of small addends would otherwise add up over the sensor
// contraction; F* contractions are as long as N_d).
template <int MT, bool LO, typename DOp>
__device__ __forceinline__ void cols_bf16_products(const BlockOps& f, DOp dop, f4v (&xr)[MT],
                                                   f4v (&xi)[MT], f4v (&sr)[MT],
                                                   f4v (&si)[MT]) {
#pragma unroll
  for (int t = 0; t < MT; ++t) {
    const u4v drh = dop(0, t), drl = dop(1, t);
    const u4v dih = dop(2, t), dil = dop(3, t);
    xr[t] = mma(drh, f.hr, xr[t]);
    xi[t] = mma(dih, f.hr, xi[t]);
    sr[t] = mma(drl, f.hr, sr[t]);
    si[t] = mma(dil, f.hr, si[t]);
    xr[t] = mma(dih, f.hi, xr[t]);
    xi[t] = mma(drh, f.nhi, xi[t]);
    sr[t] = mma(dil, f.hi, sr[t]);
    si[t] = mma(drl, f.nhi, si[t]);
    if constexpr (LO) {
      sr[t] = mma(drh, f.lr, sr[t]);
      si[t] = mma(dih, f.lr, si[t]);
      sr[t] = mma(dih, f.li, sr[t]);
      si[t] = mma(drh, f.nli, si[t]);
    }
  }
}

// Output of F's bfloat16 unit: rows row0 + 4 kg + i of right-hand sides
// b0 + 16 t + col, the two accumulator parts added in float64.
template <int NT>
__device__ __forceinline__ void rows_bf16_store(cpx<double>* __restrict__ P, const GemvShape& g,
                                                int64_t b0, int nb, int64_t k, int64_t pc,
                                                int64_t row0, int kg, int col,
                                                const f4v (&tr)[NT], const f4v (&ti)[NT],
                                                const f4v (&sr)[NT], const f4v (&si)[NT]) {
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int b = t * 16 + col;
    if (b >= nb) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t s = row0 + 4 * kg + i;
      if (s < g.Nd)
        P[(((b0 + b) * g.n_pc + pc) * g.nf + k) * g.Nd + s] = {
            (double)tr[t][i] + (double)sr[t][i], (double)ti[t][i] + (double)si[t][i]};
    }
  }
}

// Output of F*'s bfloat16 unit: column p for right-hand sides b0 + 16 t +
// 4 kg + i; the two parts added in float64, scaled by the column's
// sub-block scale sc (a power of two), rounded once.
__device__ __forceinline__ float col_scale(const float* __restrict__ scales, const GemvShape& g,
                                           int64_t k, int64_t p) {
  const int64_t ntiles = (g.Nm + kScaleTile - 1) / kScaleTile;
  return p < g.Nm ? scales[k * ntiles + p / kScaleTile] : 0.0f;
}

template <int MT>
__device__ __forceinline__ void cols_bf16_store(float sc, cpx<float>* __restrict__ Y,
                                                const GemvShape& g, int64_t b0, int nb, int64_t k,
                                                int64_t p, int kg, const f4v (&xr)[MT],
                                                const f4v (&xi)[MT], const f4v (&sr)[MT],
                                                const f4v (&si)[MT]) {
  if (p >= g.Nm) return;
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int b = t * 16 + 4 * kg + i;
      if (b < nb)
        Y[((b0 + b) * g.nf + k) * g.Nm + p] = {
            (float)(((double)xr[t][i] + (double)sr[t][i]) * sc),
            (float)(((double)xi[t][i] + (double)si[t][i]) * sc)};
    }
}

// The F* chunk for U column sub-tiles sharing the data operands (see
// rows_bf16_products_sub).
template <int MT, bool LO, int U, typename DOp>
__device__ __forceinline__ void cols_bf16_products_sub(const BlockOps (&f)[U], DOp dop,
                                                       f4v (&xr)[U][MT], f4v (&xi)[U][MT],
                                                       f4v (&sr)[U][MT], f4v (&si)[U][MT]) {
#pragma unroll
  for (int t = 0; t < MT; ++t) {
    const u4v d0 = dop(0, t), d1 = dop(1, t), d2 = dop(2, t), d3 = dop(3, t);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      f4v r1[1] = {xr[u][t]}, i1[1] = {xi[u][t]}, s1[1] = {sr[u][t]}, j1[1] = {si[u][t]};
      cols_bf16_products<1, LO>(
          f[u], [&](int pl, int) { return pl == 0 ? d0 : pl == 1 ? d1 : pl == 2 ? d2 : d3; },
          r1, i1, s1, j1);
      xr[u][t] = r1[0];
      xi[u][t] = i1[0];
      sr[u][t] = s1[0];
      si[u][t] = j1[0];
    }
  }
}

// Default load ring depth (chunks in flight per wavefront).
constexpr int kRing = 3;

// F on the bfloat16 matrix cores.  The vector planes carry the column
// sub-block scales already (folded in by the forward transform), so the whole
// column chunk accumulates in float32 matrix-core accumulators.
template <int NT, bool LO, bool VEC, int RING = kRing>
__device__ __forceinline__ void mfma_rows_bf16_wg(const uint32_t* __restrict__ A,
                                                  const uint16_t* __restrict__ Xs,
                                                  cpx<double>* __restrict__ P, GemvShape g,
                                                  int64_t n8, int64_t b0, int nb, int64_t k,
                                                  int64_t mt, int64_t pc, void* lds) {
  constexpr int WPE = LO ? 2 : 1;
  constexpr int PP = NT * 16 + 1, BUF = 16 * PP;
  u4v* sx = static_cast<u4v*>(lds);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, kg = lane >> 4;
  const int64_t p0 = pc * g.pc_len;
  const int64_t p1 = min(p0 + g.pc_len, g.Nm);
  const int64_t nch = (p1 - p0 + 31) / 32;
  const int64_t row0 = mt * kBf16Tile + 16 * wave;
  const uint32_t* __restrict__ Arow = A + (k * g.Nd + min(row0 + col, g.Nd - 1)) * g.Nm * WPE;
  f4v tr[NT], ti[NT], sr[NT], si[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) tr[t] = ti[t] = sr[t] = si[t] = (f4v){0, 0, 0, 0};
  // chunk c uses ring slot c % RING for its block words and for its vector
  // stage; both are loaded RING chunks ahead, vector part first, so every
  // wait (in-order load counter) targets loads issued RING steps earlier.
  uint32_t r0[RING][8], r1[RING][8];
  constexpr int PER = parts_per_thread<NT, kBf16Threads>();
  u4v xv[RING][PER];
#pragma unroll
  for (int d = 0; d < RING; ++d)
    stage_planes_load<NT, kBf16Threads, true>(Xs, g.nf, k, n8, b0, nb, p0 + 32 * d, d < nch ? p1 : 0, xv[d]);
#pragma unroll
  for (int d = 0; d < RING; ++d)
    load_row_slots<LO, VEC>(Arow, p0 + 32 * d, kg, d < nch ? p1 : 0, r0[d], r1[d]);
  stage_planes_store<NT, kBf16Threads, true>(xv[0], nb, p0, p1, sx);
  __syncthreads();
  // the main loop runs whole ring turns (straight-line, so the compiler's
  // waits track each slot exactly), the tail the remaining chunks
  auto step = [&](int64_t c, int d) {
    const int64_t base = p0 + 32 * c;
    const BlockOps a = unpack_block<LO>(r0[d], r1[d]);
    const int64_t ahead = base + 32 * RING, aend = c + RING < nch ? p1 : 0;
    stage_planes_load<NT, kBf16Threads, true>(Xs, g.nf, k, n8, b0, nb, ahead, aend, xv[d]);
    load_row_slots<LO, VEC>(Arow, ahead, kg, aend, r0[d], r1[d]);
    __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the products
    const u4v* xs = sx + (c & 1) * BUF;
    rows_bf16_products<NT, LO>(
        a, [&](int pl, int t) { return xs[(pl * 4 + kg) * PP + t * 16 + col]; }, tr, ti, sr, si);
    __builtin_amdgcn_sched_barrier(0);  // the store waits for its loads: after the products
    stage_planes_store<NT, kBf16Threads, true>(xv[(d + 1) % RING], nb, base + 32,
                                               c + 1 < nch ? p1 : 0, sx + ((c + 1) & 1) * BUF);
    __syncthreads();
  };
  const int64_t nfull = nch / RING * RING;
  for (int64_t c0 = 0; c0 < nfull; c0 += RING) {
#pragma unroll
    for (int d = 0; d < RING; ++d) step(c0 + d, d);
  }
#pragma unroll
  for (int d = 0; d < RING - 1; ++d)
    if (nfull + d < nch) step(nfull + d, d);
  rows_bf16_store<NT>(P, g, b0, nb, k, pc, row0, kg, col, tr, ti, sr, si);
}

// F* on the bfloat16 matrix cores: X^T = Dhat^T conj(Fhat), contraction over
// all sensors; the column scale is applied to the float32 result.
template <int MT, bool LO, int RING = kRing>
__device__ __forceinline__ void mfma_cols_bf16_wg(const uint32_t* __restrict__ A,
                                                  const float* __restrict__ scales,
                                                  const uint16_t* __restrict__ Ds,
                                                  cpx<float>* __restrict__ Y, GemvShape g,
                                                  int64_t nd8, int64_t b0, int nb, int64_t k,
                                                  int64_t pt, void* lds) {
  constexpr int WPE = LO ? 2 : 1;
  constexpr int PP = MT * 16 + 1, BUF = 16 * PP;
  u4v* sd = static_cast<u4v*>(lds);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, kg = lane >> 4;
  const int64_t nch = (g.Nd + 31) / 32;
  const int64_t col0 = pt * kBf16Tile + 16 * wave;
  const uint32_t* __restrict__ Ak = A + (k * g.Nd * g.Nm + min(col0 + col, g.Nm - 1)) * WPE;
  f4v xr[MT], xi[MT], sr[MT], si[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) xr[t] = xi[t] = sr[t] = si[t] = (f4v){0, 0, 0, 0};
  // ring and loop structure as in the F unit
  uint32_t r0[RING][8], r1[RING][8];
  constexpr int PER = parts_per_thread<MT, kBf16Threads>();
  u4v dv[RING][PER];
#pragma unroll
  for (int d = 0; d < RING; ++d)
    stage_planes_load<MT, kBf16Threads, false>(Ds, g.nf, k, nd8, b0, nb, 32 * d, d < nch ? g.Nd : 0, dv[d]);
#pragma unroll
  for (int d = 0; d < RING; ++d)
    load_col8<LO>(Ak, 32 * d + 8 * kg, d < nch ? g.Nd : 0, g.Nm, r0[d], r1[d]);
  stage_planes_store<MT, kBf16Threads, false>(dv[0], nb, 0, g.Nd, sd);
  __syncthreads();
  auto step = [&](int64_t c, int d) {
    const int64_t base = 32 * c;
    const BlockOps f = unpack_block<LO>(r0[d], r1[d]);
    const int64_t ahead = base + 32 * RING, aend = c + RING < nch ? g.Nd : 0;
    stage_planes_load<MT, kBf16Threads, false>(Ds, g.nf, k, nd8, b0, nb, ahead, aend, dv[d]);
    load_col8<LO>(Ak, ahead + 8 * kg, aend, g.Nm, r0[d], r1[d]);
    __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the products
    const u4v* ds = sd + (c & 1) * BUF;
    cols_bf16_products<MT, LO>(
        f, [&](int pl, int t) { return ds[(pl * 4 + kg) * PP + t * 16 + col]; }, xr, xi, sr, si);
    __builtin_amdgcn_sched_barrier(0);  // the store waits for its loads: after the products
    stage_planes_store<MT, kBf16Threads, false>(dv[(d + 1) % RING], nb, base + 32,
                                                c + 1 < nch ? g.Nd : 0, sd + ((c + 1) & 1) * BUF);
    __syncthreads();
  };
  const int64_t nfull = nch / RING * RING;
  for (int64_t c0 = 0; c0 < nfull; c0 += RING) {
#pragma unroll
    for (int d = 0; d < RING; ++d) step(c0 + d, d);
  }
#pragma unroll
  for (int d = 0; d < RING - 1; ++d)
    if (nfull + d < nch) step(nfull + d, d);
  cols_bf16_store<MT>(col_scale(scales, g, k, col0 + col), Y, g, b0, nb, k, col0 + col, kg, xr,
                      xi, sr, si);
}

}  // namespace
}  // namespace p2o
