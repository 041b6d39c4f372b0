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
// for both operands: F* uses sensors 8 (l / 16) + j; F interleaves them
// (row_slot_entry) so the 4 lane groups of a block row read one contiguous
// 64-byte span per load, and the forward transform writes F's vector planes
// in that slot order, so the 8 slots of a lane group are one 16-byte run.
//
// F  ("rows"): workgroup = 128 sensors x (16 NT) right-hand sides of one
//    frequency and one column chunk; the column sub-block scales are folded
//    into the vector planes (exact: powers of two), so the chunk accumulates
//    in float32 on the matrix cores.
// F* ("cols"): X^T = Dhat^T conj(Fhat): workgroup = (16 MT) right-hand
//    sides x 128 columns; contraction over all sensors; the column scale is
//    applied to the float32 result.
// Vector operands arrive as four bfloat16 planes per (rhs, k), written by
// the forward transform: [re hi][re lo][im hi][im lo], each zero-padded to a
// multiple of 32 entries.
//
// Two kernel families: the single-role kernels below (every wavefront loads
// and multiplies; also the units of the persistent multi-instance kernel,
// and the fallback when tile numbers or lane offsets exceed 32 bits) and the
// warp-specialised kernels further down, used otherwise, at any row
// alignment.  Both give bitwise equal results.
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

// ------------------------------------------------- warp-specialised kernels
// The kernels above issue block loads, vector stage, LDS reads and
// matrix-core products from every wavefront.  A wavefront issues in order,
// so when the memory system pushes back on a load, the matrix-core
// instructions behind it wait too: measured at 600 x 40000 x 420 with 64
// right-hand sides, the kernel time is about the sum of the memory-only
// (12.5 ms) and matrix-core-only (7.8 ms) times.  Here the roles are split.
// kWsProducers wavefronts load every chunk of block entries and vector
// planes into a ring of their own registers, kWsRegRing chunks ahead, and
// write each chunk into one of two LDS slots just before it is needed;
// kWsConsumers wavefronts only read LDS and issue products, so a producer
// stalled on memory holds up no product.  The loads in flight per CU are
// bounded by the producers' registers (3 chunks, ~144 KB) instead of by
// LDS: a ring of LDS slots filled by direct global-to-LDS copies keeps
// only ~1.5 chunks in flight in 160 KB and measured 18.5 ms for the copy
// stream alone.  One workgroup per CU, persistent over tiles so the ring
// runs on across tile boundaries; each XCD walks a contiguous range of
// tiles (tiles of one frequency share its vector chunks in that L2).
//
// Step protocol (one s_barrier per chunk): after barrier s, consumers
// compute chunk s from LDS slot s mod 2 while producers write chunk s + 1
// into the other slot (finished by every consumer before barrier s) and
// issue the loads of chunk s + 1 + kWsRegRing into the registers it came
// from.  Every wavefront runs the same number of steps (the workgroup's
// chunk count padded to whole register-ring turns; padding steps load
// valid bytes and compute nothing), so the barrier counts agree.  Consumers run
// the same per-chunk products, in the same order, as the units in
// matrix_units.h, so results are bitwise equal to theirs.
constexpr int kWsConsumers = 4;
constexpr int kWsSub = 2;  // 16-row (F) or 16-column (F*) sub-tiles per consumer: 128 per workgroup
constexpr int kWsProducers = 4;
constexpr int kWsThreads = 64 * (kWsConsumers + kWsProducers);
constexpr int kWsTile = 16 * kWsSub * kWsConsumers;  // columns of an F* tile
static_assert(kWsTile == kBf16Tile, "F*'s slot layout assumes 1 KB sensor rows (128 columns)");
// F's kernel: its own role counts (its tile rows follow from them) and
// workgroups per CU.
constexpr int kWsRowConsumers = kWsConsumers;
constexpr int kWsRowProducers = kWsProducers;
constexpr int kWsRowThreads = 64 * (kWsRowConsumers + kWsRowProducers);
constexpr int kWsRowTile = 16 * kWsSub * kWsRowConsumers;
constexpr int kWsRowPerCu = 1;
constexpr int kWsRegRing = 3;  // chunks in flight in each producer's registers

// This wavefront's LDS writes have completed.
__device__ __forceinline__ void wait_lds() {
  __builtin_amdgcn_s_waitcnt(15 | (7 << 4) | (0 << 8) | (3 << 14));
}

// Workgroup barrier without the memory fences of __syncthreads; the
// compiler may move no memory access across it.
__device__ __forceinline__ void ws_barrier() {
  __asm__ volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  __asm__ volatile("" ::: "memory");
}

// Tiles of this workgroup: XCD x = blockIdx % 8 owns the contiguous range
// [x span, (x + 1) span); its workgroups take every (grid / 8)-th tile of it.
struct WsTiles {
  int64_t tile, end, step;
  __device__ explicit WsTiles(int64_t total) {
    const int64_t span = (total + kXcds - 1) / kXcds;
    const int64_t x = blockIdx.x % kXcds;
    tile = x * span + blockIdx.x / kXcds;
    end = min(total, (x + 1) * span);
    step = gridDim.x / kXcds;
  }
  __device__ int64_t count() const { return end > tile ? (end - tile + step - 1) / step : 0; }
  // how many of this workgroup's tiles are >= thr
  __device__ int64_t count_from(int64_t thr) const {
    const int64_t n = count();
    const int64_t i0 = thr <= tile ? 0 : (thr - tile + step - 1) / step;
    return n > i0 ? n - i0 : 0;
  }
};

__device__ __forceinline__ int64_t ws_padded(int64_t n) {
  return (n + kWsRegRing - 1) / kWsRegRing * kWsRegRing;
}

// A 16-byte granule of block words at an address aligned to AL bytes: row
// starts are 16-byte aligned only when a row's byte length is a multiple
// of 16 (hi+lo: N_m even; hi-only: N_m a multiple of 4), else the granule
// is loaded in 8- or 4-byte parts (same bytes, more instructions).
template <int AL>
__device__ __forceinline__ u4v ld_granule(const char* p) {
  if constexpr (AL == 16) {
    return __builtin_nontemporal_load(reinterpret_cast<const u4v*>(p));
  } else if constexpr (AL == 8) {
    const u2v x = __builtin_nontemporal_load(reinterpret_cast<const u2v*>(p));
    const u2v y = __builtin_nontemporal_load(reinterpret_cast<const u2v*>(p + 8));
    return (u4v){x[0], x[1], y[0], y[1]};
  } else {
    static_assert(AL == 4, "granule alignment 16, 8 or 4 bytes");
    u4v r;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      r[i] = __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(p) + i);
    return r;
  }
}

// The granule that starts at entry e of a row (`row` points at entry 0, BPE
// bytes an entry) when only entries below r exist: it is loaded in AL-byte
// parts (each a whole number of entries, as r is a multiple of AL / BPE)
// and a part past r re-reads the last part below r, so no byte beyond entry
// r - 1 is read.
template <int AL, int BPE>
__device__ __forceinline__ u4v ld_granule_clamped(const char* row, int64_t e, int64_t r) {
  constexpr int EPP = AL / BPE;  // entries a part
  static_assert(EPP >= 1 && AL % BPE == 0, "a part holds whole entries");
  auto at = [&](int i) { return row + min<int64_t>(e + i * EPP, r - EPP) * BPE; };
  if constexpr (AL == 16) {
    return __builtin_nontemporal_load(reinterpret_cast<const u4v*>(at(0)));
  } else if constexpr (AL == 8) {
    const u2v x = __builtin_nontemporal_load(reinterpret_cast<const u2v*>(at(0)));
    const u2v y = __builtin_nontemporal_load(reinterpret_cast<const u2v*>(at(1)));
    return (u4v){x[0], x[1], y[0], y[1]};
  } else {
    static_assert(AL == 4, "granule alignment 16, 8 or 4 bytes");
    u4v v;
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(at(i)));
    return v;
  }
}

// F: tile = (row tile mt, frequency k, column chunk pc), mt fastest.
struct RowsStep {
  int64_t tile, end, stride, mt, k, pc, p0, p1, nch, c;
  __device__ void decode(const GemvShape& g) {  // 32-bit divisions: tile counts < 2^31
    const uint32_t nmt = (uint32_t)((g.Nd + kWsRowTile - 1) / kWsRowTile);
    const uint32_t t = (uint32_t)tile, rest = t / nmt;
    mt = t - rest * nmt;
    k = rest % (uint32_t)g.nf;
    pc = rest / (uint32_t)g.nf;
    p0 = pc * g.pc_len;
    p1 = min(p0 + g.pc_len, g.Nm);
    nch = (p1 - p0 + 31) / 32;
    c = 0;
  }
  __device__ bool valid() const { return tile < end; }
  __device__ void next(const GemvShape& g) {
    if (++c < nch) return;
    tile += stride;
    if (tile < end) decode(g);
  }
};

// Chunks of all of this workgroup's F tiles (the last column chunk is shorter).
__device__ __forceinline__ int64_t ws_rows_steps(const WsTiles& wt, const GemvShape& g) {
  const int64_t nmt = (g.Nd + kWsRowTile - 1) / kWsRowTile;
  const int64_t full = (g.pc_len + 31) / 32;
  const int64_t last = (g.Nm - (g.n_pc - 1) * g.pc_len + 31) / 32;
  return wt.count() * full - wt.count_from((g.n_pc - 1) * nmt * g.nf) * (full - last);
}

template <int NT, bool LO>
struct WsRowsLds {
  static constexpr int kBlock = kWsRowTile * 32 * 4 * (LO ? 2 : 1);  // 32 KB | 16 KB
  static constexpr int kVec = 16 * NT * 256;                        // 16 NT rhs x 16 granules
  static constexpr int kSlot = kBlock + kVec;
  static constexpr int kBlockIns = kBlock / 1024 / kWsRowProducers;   // per producer and chunk
  static constexpr int kVecIns = kVec / 1024 / kWsRowProducers;
  static constexpr int kIns = kBlockIns + kVecIns;
  static_assert(kBlock % (1024 * kWsRowProducers) == 0 && kVec % (1024 * kWsRowProducers) == 0,
                "whole 1 KB load instructions per producer");
};

// Slot layout (16-byte granules; each producer load instruction fills one
// KB, lane i granule i).  Block: row r of the tile, granule g (LO: entries
// 2g, 2g + 1 of the chunk; hi-only: 4g .. 4g + 3) at [r][g ^ swz(r)] (LO 16
// granules a row, swz = r mod 16; hi-only 8, swz = (r / 2) mod 8).  Vector:
// right-hand side b, granule L = plane * 4 + kg (slots 0..7 of lane group
// kg) at [b][L ^ (b mod 16)].  The XOR puts the 16 lanes of a lane group,
// which read 16 rows (or right-hand sides) at one granule, on 16 different
// bank groups.
// A producer's loads address memory as a wave-uniform 64-bit base (scalar
// arithmetic, per chunk) plus a 32-bit lane offset that is fixed for a
// tile: the vector units then spend almost nothing on addresses, which
// measurably competes with the consumers' products on the shared SIMD.
template <int NT, bool LO>
struct WsRowsOff {
  uint32_t blk[WsRowsLds<NT, LO>::kBlockIns];     // lane offsets (vector registers)
  uint32_t vec[WsRowsLds<NT, LO>::kVecIns];
  const char* bbase[WsRowsLds<NT, LO>::kBlockIns];  // chunk-0 bases of the tile (uniform)
  const char* vbase[WsRowsLds<NT, LO>::kVecIns];
};

// Block rows per load instruction and the granule of lane `lane`.
template <bool LO>
__device__ __forceinline__ void ws_rows_lane(int qi, int lane, int& rl, int& gr) {
  if constexpr (LO) {
    rl = qi * 4 + (lane >> 4);
    gr = (lane & 15) ^ (rl & 15);
  } else {
    rl = qi * 8 + (lane >> 3);
    gr = (lane & 7) ^ ((rl >> 1) & 7);
  }
}

// Offsets and bases of tile st (valid) for producer p.
template <int NT, bool LO>
__device__ __forceinline__ void ws_rows_offsets(const uint32_t* __restrict__ A,
                                                const uint16_t* __restrict__ Xs,
                                                const GemvShape& g, int64_t n8, int64_t b0, int nb,
                                                const RowsStep& st, int p, int lane,
                                                WsRowsOff<NT, LO>& o) {
  using Lay = WsRowsLds<NT, LO>;
  constexpr int WPE = LO ? 2 : 1, RPI = LO ? 4 : 8;
#pragma unroll
  for (int q = 0; q < Lay::kBlockIns; ++q) {
    const int qi = p * Lay::kBlockIns + q;
    int rl, gr;
    ws_rows_lane<LO>(qi, lane, rl, gr);
    const int64_t r0 = min(st.mt * kWsRowTile + qi * RPI, g.Nd - 1);
    const int64_t row = min(st.mt * kWsRowTile + rl, g.Nd - 1);  // rows past Nd: dropped
    o.blk[q] = (uint32_t)(((row - r0) * g.Nm + (LO ? 2 : 4) * gr) * WPE * 4);
    o.bbase[q] = reinterpret_cast<const char*>(A) + ((st.k * g.Nd + r0) * g.Nm + st.p0) * WPE * 4;
  }
#pragma unroll
  for (int q = 0; q < Lay::kVecIns; ++q) {  // right-hand sides past nb: a copy of the last (dropped)
    const int qx = p * Lay::kVecIns + q;
    const int b = qx * 4 + (lane >> 4);
    const int L = (lane & 15) ^ (b & 15);
    const int rb0 = min(qx * 4, nb - 1), rb = min(b, nb - 1) - rb0;
    o.vec[q] = (uint32_t)((((int64_t)rb * g.nf * 4 + (L >> 2)) * n8 + 8 * (L & 3)) * 2);
    o.vbase[q] = reinterpret_cast<const char*>(Xs) +
                 (((b0 + rb0) * g.nf + st.k) * 4 * n8 + st.p0) * 2;
  }
}

// Loads of chunk st (or, when !live, of any valid bytes: a padding step);
// block granules aligned to AL bytes.
template <int NT, bool LO, int AL>
__device__ __forceinline__ void ws_rows_load(const uint32_t* __restrict__ A,
                                             const uint16_t* __restrict__ Xs, const GemvShape& g,
                                             int64_t n8, int64_t b0, int nb, const RowsStep& st,
                                             bool live, const WsRowsOff<NT, LO>& o, int p,
                                             int lane, u4v (&v)[WsRowsLds<NT, LO>::kIns]) {
  using Lay = WsRowsLds<NT, LO>;
  constexpr int WPE = LO ? 2 : 1, RPI = LO ? 4 : 8, EPG = LO ? 2 : 4;  // entries a granule
  const int64_t base = st.p0 + 32 * st.c;
  const bool tail = live && base + 32 > st.p1;
  const int64_t bstep = live ? 32 * st.c * WPE * 4 : 0, vstep = live ? 32 * st.c * 2 : 0;
#pragma unroll
  for (int q = 0; q < Lay::kBlockIns; ++q) {
    const char* ub = (live ? o.bbase[q] : reinterpret_cast<const char*>(A)) + bstep;
    if (tail) {  // parts past the contraction re-read its last part (their vector entries are 0)
      const int qi = p * Lay::kBlockIns + q;
      int rl, gr;
      ws_rows_lane<LO>(qi, lane, rl, gr);
      const int64_t r0 = min(st.mt * kWsRowTile + qi * RPI, g.Nd - 1);
      const int64_t row = min(st.mt * kWsRowTile + rl, g.Nd - 1);
      v[q] = ld_granule_clamped<AL, WPE * 4>(ub + (uint32_t)((row - r0) * g.Nm * WPE * 4),
                                             EPG * gr, st.p1 - base);
    } else {
      v[q] = ld_granule<AL>(ub + o.blk[q]);
    }
  }
#pragma unroll
  for (int q = 0; q < Lay::kVecIns; ++q) {
    const char* ub = (live ? o.vbase[q] : reinterpret_cast<const char*>(Xs)) + vstep;
    v[Lay::kBlockIns + q] = *reinterpret_cast<const u4v*>(ub + o.vec[q]);
  }
}

template <int NT, bool LO>
__device__ __forceinline__ void ws_rows_store(char* slot, int p, int lane,
                                              const u4v (&v)[WsRowsLds<NT, LO>::kIns]) {
  using Lay = WsRowsLds<NT, LO>;
#pragma unroll
  for (int q = 0; q < Lay::kBlockIns; ++q)
    reinterpret_cast<u4v*>(slot + (p * Lay::kBlockIns + q) * 1024)[lane] = v[q];
#pragma unroll
  for (int q = 0; q < Lay::kVecIns; ++q)
    reinterpret_cast<u4v*>(slot + Lay::kBlock + (p * Lay::kVecIns + q) * 1024)[lane] =
        v[Lay::kBlockIns + q];
}

template <int NT, bool LO, int AL>
__global__ void __launch_bounds__(kWsRowThreads, 2)  // 2 wavefronts a SIMD: 256 registers each
gemm_rows_bf16_ws(const uint32_t* __restrict__ A, const uint16_t* __restrict__ Xs,
                  cpx<double>* __restrict__ P, GemvShape g, int64_t n8, int64_t b0, int nb) {
  using Lay = WsRowsLds<NT, LO>;
  __shared__ __align__(16) char lds[2 * Lay::kSlot];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const WsTiles wt(((g.Nd + kWsRowTile - 1) / kWsRowTile) * g.nf * g.n_pc);
  const int64_t nsteps = ws_rows_steps(wt, g), npad = ws_padded(nsteps);
  RowsStep st{wt.tile, wt.end, wt.step};
  if (st.valid()) st.decode(g);
  if (wave >= kWsRowConsumers) {  // producer
    const int p = wave - kWsRowConsumers;
    u4v ring[kWsRegRing][Lay::kIns];
    WsRowsOff<NT, LO> off{};  // zeros: a workgroup without tiles loads from the bases
    if (st.valid()) ws_rows_offsets<NT, LO>(A, Xs, g, n8, b0, nb, st, p, lane, off);
    auto load = [&](u4v(&v)[Lay::kIns]) {  // the next chunk of the sequence
      const bool live = st.valid();
      if (live && st.c == 0) ws_rows_offsets<NT, LO>(A, Xs, g, n8, b0, nb, st, p, lane, off);
      ws_rows_load<NT, LO, AL>(A, Xs, g, n8, b0, nb, st, live, off, p, lane, v);
      if (live) st.next(g);
    };
#pragma unroll
    for (int d = 0; d < kWsRegRing; ++d) load(ring[d]);
    ws_rows_store<NT, LO>(lds, p, lane, ring[0]);
    // chunk kWsRegRing into ring[0]: the loop is entered with the loads of
    // chunks 1 .. kWsRegRing pending in the order the loop leaves them, so
    // the compiler's load-counter waits stay exact (a chunk's registers are
    // waited for with the two later chunks still in flight)
    load(ring[0]);
    for (int64_t s0 = 0; s0 < npad; s0 += kWsRegRing) {
#pragma unroll
      for (int d = 0; d < kWsRegRing; ++d) {  // step s0 + d; chunk s0 + d + 1 is in ring[(d + 1) % R]
        wait_lds();
        ws_barrier();
        u4v(&r)[Lay::kIns] = ring[(d + 1) % kWsRegRing];
        ws_rows_store<NT, LO>(lds + ((s0 + d + 1) & 1) * Lay::kSlot, p, lane, r);
        load(r);
      }
    }
    return;
  }
  // consumer: rows 32 wave + 16 u .. + 15 (u < kWsSub) of each tile
  const int r = lane & 15, kg = lane >> 4;
  f4v tr[kWsSub][NT], ti[kWsSub][NT], sr[kWsSub][NT], si[kWsSub][NT];
  for (int64_t s = 0; s < npad; ++s) {
    const bool live = s < nsteps;
    if (live && st.c == 0) {
#pragma unroll
      for (int u = 0; u < kWsSub; ++u)
#pragma unroll
        for (int t = 0; t < NT; ++t) tr[u][t] = ti[u][t] = sr[u][t] = si[u][t] = (f4v){0, 0, 0, 0};
    }
    ws_barrier();
    if (!live) continue;
    const char* slot = lds + (s & 1) * Lay::kSlot;
    const u4v* blk = reinterpret_cast<const u4v*>(slot);
    const u4v* xs = reinterpret_cast<const u4v*>(slot + Lay::kBlock);
    const int64_t row0 = st.mt * kWsRowTile + 16 * kWsSub * wave;
    if (row0 < g.Nd) {  // rows past Nd in a live wavefront: computed, dropped
      BlockOps a[kWsSub];
#pragma unroll
      for (int u = 0; u < kWsSub; ++u) {
        const int rl = 16 * (kWsSub * wave + u) + r;
        uint32_t w0[8], w1[8];
        if constexpr (LO) {
#pragma unroll
          for (int h = 0; h < 4; ++h) {  // granule 4 h + kg: entries 8 h + 2 kg + {0, 1}
            const u4v v = blk[rl * 16 + ((4 * h + kg) ^ r)];
            w0[2 * h] = v[0];
            w1[2 * h] = v[1];
            w0[2 * h + 1] = v[2];
            w1[2 * h + 1] = v[3];
          }
        } else {
#pragma unroll
          for (int h = 0; h < 2; ++h) {  // granule 4 h + kg: entries 16 h + 4 kg + {0..3}
            const u4v v = blk[rl * 8 + ((4 * h + kg) ^ ((rl >> 1) & 7))];
#pragma unroll
            for (int c = 0; c < 4; ++c) w0[4 * h + c] = v[c];
          }
#pragma unroll
          for (int j = 0; j < 8; ++j) w1[j] = 0u;
        }
        a[u] = unpack_block<LO>(w0, w1);
      }
      rows_bf16_products_sub<NT, LO, kWsSub>(
          a, [&](int pl, int t) { return xs[(16 * t + r) * 16 + ((pl * 4 + kg) ^ r)]; }, tr, ti,
          sr, si);
      if (st.c + 1 == st.nch) {
#pragma unroll
        for (int u = 0; u < kWsSub; ++u)
          rows_bf16_store<NT>(P, g, b0, nb, st.k, st.pc, row0 + 16 * u, kg, r, tr[u], ti[u],
                              sr[u], si[u]);
      }
    }
    st.next(g);
  }
}

// F*: tile = (column tile pt, frequency k), pt fastest; chunks of 32 sensors.
struct ColsStep {
  int64_t tile, end, stride, pt, k, nch, c;
  __device__ void decode(const GemvShape& g) {  // 32-bit divisions: tile counts < 2^31
    const uint32_t npt = (uint32_t)((g.Nm + kWsTile - 1) / kWsTile);
    const uint32_t t = (uint32_t)tile;
    k = t / npt;
    pt = t - (uint32_t)k * npt;
    nch = (g.Nd + 31) / 32;
    c = 0;
  }
  __device__ bool valid() const { return tile < end; }
  __device__ void next(const GemvShape& g) {
    if (++c < nch) return;
    tile += stride;
    if (tile < end) decode(g);
  }
};

template <int MT, bool LO>
struct WsColsLds {
  static constexpr int kRow = kWsTile * 4 * (LO ? 2 : 1);  // bytes of one sensor row: 1 KB | 512
  static constexpr int kBlock = 32 * kRow;
  static constexpr int kVec = 16 * MT * 256;
  static constexpr int kSlot = kBlock + kVec;
  static constexpr int kBlockIns = kBlock / 1024 / kWsProducers;
  static constexpr int kIns = kBlockIns + MT;
  static_assert(kVec == 1024 * kWsProducers * MT, "MT vector load instructions per producer");
};

// Block slot layout: sensor row sl of the chunk, granule g (LO: columns 2g,
// 2g + 1 of the tile; hi-only: 4g .. 4g + 3) at [sl][g ^ swz(sl)] with swz
// = 8 ((sl / 8) mod 2) (LO) or 4 ((sl / 8) mod 4) (hi-only): the lane
// groups of a read (sensors 8 kg + j) land on different bank groups.
// Vector (data planes) as in F's layout.
template <bool LO>
__device__ __forceinline__ int ws_cols_swz(int sl) {
  return LO ? ((sl >> 3) & 1) << 3 : ((sl >> 3) & 3) << 2;
}

template <int MT, bool LO>
struct WsColsOff {
  uint32_t blk[WsColsLds<MT, LO>::kBlockIns];   // first (LO: only) row of the instruction
  uint32_t blk2[WsColsLds<MT, LO>::kBlockIns];  // hi-only: lanes 32..63 on the second row
  uint32_t vec[MT];
  const char* tbase;  // the tile's first column in sensor row 0 (uniform)
  const char* vbase[MT];
};

template <int MT, bool LO>
__device__ __forceinline__ void ws_cols_offsets(const uint32_t* __restrict__ A,
                                                const uint16_t* __restrict__ Ds,
                                                const GemvShape& g, int64_t nd32, int64_t b0,
                                                int nb, const ColsStep& st, int p, int lane,
                                                WsColsOff<MT, LO>& o) {
  const int64_t pt = st.pt;
  o.tbase = reinterpret_cast<const char*>(A) + (st.k * g.Nd * g.Nm + pt * kWsTile) * (LO ? 8 : 4);
  using Lay = WsColsLds<MT, LO>;
  constexpr int EPG = LO ? 2 : 4;  // columns a granule
#pragma unroll
  for (int q = 0; q < Lay::kBlockIns; ++q) {
    const int qi = p * Lay::kBlockIns + q;
    const int sl = LO ? qi : 2 * qi + (lane >> 5);
    const int gr = (LO ? lane : (lane & 31)) ^ ws_cols_swz<LO>(sl);
    // granules wholly past Nm: the row's last granule (dropped).  When Nm is
    // not a multiple of EPG the last granule runs up to EPG - 1 entries past
    // the row (into the next row, or the block array's tail padding): those
    // columns are dropped too.
    const int64_t col = min<int64_t>(EPG * gr, (g.Nm - 1 - pt * kWsTile) / EPG * EPG);
    o.blk[q] = (uint32_t)(col * (LO ? 8 : 4));
    o.blk2[q] = o.blk[q] + (LO ? 0u : (uint32_t)((lane >> 5) * g.Nm * 4));
  }
#pragma unroll
  for (int q = 0; q < MT; ++q) {
    const int qx = p * MT + q;
    const int b = qx * 4 + (lane >> 4);
    const int L = (lane & 15) ^ (b & 15);
    const int rb0 = min(qx * 4, nb - 1), rb = min(b, nb - 1) - rb0;
    o.vec[q] = (uint32_t)((((int64_t)rb * g.nf * 4 + (L >> 2)) * nd32 + 8 * (L & 3)) * 2);
    o.vbase[q] = reinterpret_cast<const char*>(Ds) + ((b0 + rb0) * g.nf + st.k) * 4 * nd32 * 2;
  }
}

// Loads of chunk st (or, when !live, of any valid bytes).  Sensors past Nd
// re-read row Nd - 1; their data planes are zero there (pitch a multiple
// of 32, zero-padded).
template <int MT, bool LO, int AL>
__device__ __forceinline__ void ws_cols_load(const uint32_t* __restrict__ A,
                                             const uint16_t* __restrict__ Ds, const GemvShape& g,
                                             int64_t nd32, int64_t b0, int nb, const ColsStep& st,
                                             bool live, const WsColsOff<MT, LO>& o, int p,
                                             u4v (&v)[WsColsLds<MT, LO>::kIns]) {
  using Lay = WsColsLds<MT, LO>;
  constexpr int WPE = LO ? 2 : 1;
  const int64_t base = 32 * st.c;
  const int64_t row_bytes = g.Nm * WPE * 4;
#pragma unroll
  for (int q = 0; q < Lay::kBlockIns; ++q) {
    const int qi = p * Lay::kBlockIns + q;
    const int64_t s0 = base + (LO ? qi : 2 * qi);
    const char* ub = live ? o.tbase + min(s0, g.Nd - 1) * row_bytes
                          : reinterpret_cast<const char*>(A);
    const uint32_t off = (LO || s0 + 1 >= g.Nd) ? o.blk[q] : o.blk2[q];
    v[q] = ld_granule<AL>(ub + off);
  }
#pragma unroll
  for (int q = 0; q < MT; ++q) {
    const char* ub = live ? o.vbase[q] + base * 2 : reinterpret_cast<const char*>(Ds);
    v[Lay::kBlockIns + q] = *reinterpret_cast<const u4v*>(ub + o.vec[q]);
  }
}

template <int MT, bool LO>
__device__ __forceinline__ void ws_cols_store(char* slot, int p, int lane,
                                              const u4v (&v)[WsColsLds<MT, LO>::kIns]) {
  using Lay = WsColsLds<MT, LO>;
#pragma unroll
  for (int q = 0; q < Lay::kBlockIns; ++q)
    reinterpret_cast<u4v*>(slot + (p * Lay::kBlockIns + q) * 1024)[lane] = v[q];
#pragma unroll
  for (int q = 0; q < MT; ++q)
    reinterpret_cast<u4v*>(slot + Lay::kBlock + (p * MT + q) * 1024)[lane] = v[Lay::kBlockIns + q];
}

template <int MT, bool LO, int AL>
__global__ void __launch_bounds__(kWsThreads)
gemm_cols_bf16_ws(const uint32_t* __restrict__ A, const float* __restrict__ scales,
                  const uint16_t* __restrict__ Ds, cpx<float>* __restrict__ Y, GemvShape g,
                  int64_t nd8, int64_t b0, int nb) {
  using Lay = WsColsLds<MT, LO>;
  __shared__ __align__(16) char lds[2 * Lay::kSlot];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const WsTiles wt(((g.Nm + kWsTile - 1) / kWsTile) * g.nf);
  const int64_t nsteps = wt.count() * ((g.Nd + 31) / 32), npad = ws_padded(nsteps);
  ColsStep st{wt.tile, wt.end, wt.step};
  if (st.valid()) st.decode(g);
  if (wave >= kWsConsumers) {  // producer
    const int p = wave - kWsConsumers;
    u4v ring[kWsRegRing][Lay::kIns];
    WsColsOff<MT, LO> off{};  // zeros: a workgroup without tiles loads from the bases
    if (st.valid()) ws_cols_offsets<MT, LO>(A, Ds, g, nd8, b0, nb, st, p, lane, off);
    auto load = [&](u4v(&v)[Lay::kIns]) {  // as for F
      const bool live = st.valid();
      if (live && st.c == 0) ws_cols_offsets<MT, LO>(A, Ds, g, nd8, b0, nb, st, p, lane, off);
      ws_cols_load<MT, LO, AL>(A, Ds, g, nd8, b0, nb, st, live, off, p, v);
      if (live) st.next(g);
    };
#pragma unroll
    for (int d = 0; d < kWsRegRing; ++d) load(ring[d]);
    ws_cols_store<MT, LO>(lds, p, lane, ring[0]);
    load(ring[0]);
    for (int64_t s0 = 0; s0 < npad; s0 += kWsRegRing) {
#pragma unroll
      for (int d = 0; d < kWsRegRing; ++d) {
        wait_lds();
        ws_barrier();
        u4v(&r)[Lay::kIns] = ring[(d + 1) % kWsRegRing];
        ws_cols_store<MT, LO>(lds + ((s0 + d + 1) & 1) * Lay::kSlot, p, lane, r);
        load(r);
      }
    }
    return;
  }
  // consumer: columns 32 wave + 16 u .. + 15 (u < kWsSub) of each tile
  const int n = lane & 15, kg = lane >> 4;
  f4v xr[kWsSub][MT], xi[kWsSub][MT], sr[kWsSub][MT], si[kWsSub][MT];
  float sc[kWsSub];
  for (int64_t s = 0; s < npad; ++s) {
    const bool live = s < nsteps;
    if (live && st.c == 0) {
#pragma unroll
      for (int u = 0; u < kWsSub; ++u) {
#pragma unroll
        for (int t = 0; t < MT; ++t) xr[u][t] = xi[u][t] = sr[u][t] = si[u][t] = (f4v){0, 0, 0, 0};
        // the output scale, fetched a tile ahead of its use
        sc[u] = col_scale(scales, g, st.k, st.pt * kWsTile + 16 * (kWsSub * wave + u) + n);
      }
    }
    ws_barrier();
    if (!live) continue;
    const char* slot = lds + (s & 1) * Lay::kSlot;
    const u4v* ds = reinterpret_cast<const u4v*>(slot + Lay::kBlock);
    const int64_t col0 = st.pt * kWsTile + 16 * kWsSub * wave;
    if (col0 < g.Nm) {
      BlockOps f[kWsSub];
#pragma unroll
      for (int u = 0; u < kWsSub; ++u) {
        const int cl = 16 * (kWsSub * wave + u) + n;
        uint32_t w0[8], w1[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {  // sensor 8 kg + j of the chunk, column cl
          const int sl = 8 * kg + j;
          if constexpr (LO) {
            const int gr = (cl >> 1) ^ ws_cols_swz<true>(sl);
            const u2v x = *reinterpret_cast<const u2v*>(slot + sl * Lay::kRow + gr * 16 +
                                                        (cl & 1) * 8);
            w0[j] = x[0];
            w1[j] = x[1];
          } else {
            const int gr = (cl >> 2) ^ ws_cols_swz<false>(sl);
            w0[j] = *reinterpret_cast<const uint32_t*>(slot + sl * Lay::kRow + gr * 16 +
                                                       (cl & 3) * 4);
            w1[j] = 0u;
          }
        }
        f[u] = unpack_block<LO>(w0, w1);
      }
      cols_bf16_products_sub<MT, LO, kWsSub>(
          f, [&](int pl, int t) { return ds[(16 * t + n) * 16 + ((pl * 4 + kg) ^ n)]; }, xr, xi,
          sr, si);
      if (st.c + 1 == st.nch) {
#pragma unroll
        for (int u = 0; u < kWsSub; ++u)
          cols_bf16_store<MT>(sc[u], Y, g, b0, nb, st.k, col0 + 16 * u + n, kg, xr[u], xi[u],
                              sr[u], si[u]);
      }
    }
    st.next(g);
  }
}

// The producers' 32-bit lane offsets: up to 3 right-hand sides of planes
// (pitch `pitch`) and up to 7 block rows.
bool ws_offsets_fit(const GemvShape& g, int64_t pitch) {
  const int64_t lim = int64_t{1} << 32;
  return (4 * g.nf * 4 + 4) * pitch * 2 < lim && 8 * g.Nm * 8 < lim;
}

int ws_grid(int64_t tiles, int per_cu) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  const int64_t g = std::min<int64_t>(tiles, (int64_t)cus * per_cu);
  return (int)std::max<int64_t>(kXcds, (g + kXcds - 1) / kXcds * kXcds);
}

// Alignment of the block rows' granules: 16 bytes when a row's byte length
// is a multiple of 16, else 8 or (hi only, 4-byte entries) 4.
template <bool LO>
int ws_align(int64_t Nm) {
  const int64_t row_bytes = Nm * (LO ? 8 : 4);
  return row_bytes % 16 == 0 ? 16 : (row_bytes % 8 == 0 ? 8 : 4);
}

template <bool LO, int AL>
void rows_ws_launch(unsigned grid, int nb, const uint32_t* A, const uint16_t* Xs,
                    cpx<double>* P, const GemvShape& g, int64_t n8, int64_t b0, hipStream_t s) {
  if (nb > 32)
    hipLaunchKernelGGL((gemm_rows_bf16_ws<4, LO, AL>), dim3(grid), dim3(kWsRowThreads), 0, s, A, Xs, P, g, n8, b0, nb);
  else if (nb > 16)
    hipLaunchKernelGGL((gemm_rows_bf16_ws<2, LO, AL>), dim3(grid), dim3(kWsRowThreads), 0, s, A, Xs, P, g, n8, b0, nb);
  else
    hipLaunchKernelGGL((gemm_rows_bf16_ws<1, LO, AL>), dim3(grid), dim3(kWsRowThreads), 0, s, A, Xs, P, g, n8, b0, nb);
}

template <bool LO, int AL>
void cols_ws_launch(unsigned grid, int nb, const uint32_t* A, const float* sc,
                    const uint16_t* Ds, cpx<float>* Y, const GemvShape& g, int64_t nd8,
                    int64_t b0, hipStream_t s) {
  if (nb > 32)
    hipLaunchKernelGGL((gemm_cols_bf16_ws<4, LO, AL>), dim3(grid), dim3(kWsThreads), 0, s, A, sc, Ds, Y, g, nd8, b0, nb);
  else if (nb > 16)
    hipLaunchKernelGGL((gemm_cols_bf16_ws<2, LO, AL>), dim3(grid), dim3(kWsThreads), 0, s, A, sc, Ds, Y, g, nd8, b0, nb);
  else
    hipLaunchKernelGGL((gemm_cols_bf16_ws<1, LO, AL>), dim3(grid), dim3(kWsThreads), 0, s, A, sc, Ds, Y, g, nd8, b0, nb);
}

template <bool LO, bool VEC>
hipError_t rows_passes(const uint32_t* A, const uint16_t* Xs, cpx<double>* P,
                       const GemvShape& g, int64_t n8, hipStream_t s) {
  const unsigned grid = padded_grid(((g.Nd + kBf16Tile - 1) / kBf16Tile) * g.nf * g.n_pc);
  // 32-bit tile numbers and lane offsets: the warp-specialised kernel, its
  // block loads at the rows' alignment
  const int64_t wtiles = ((g.Nd + kWsRowTile - 1) / kWsRowTile) * g.nf * g.n_pc;
  const bool ws = wtiles < (int64_t{1} << 31) && ws_offsets_fit(g, n8);
  const unsigned wgrid = ws ? (unsigned)ws_grid(wtiles, kWsRowPerCu) : 0u;
  const int al = ws_align<LO>(g.Nm);
  for (int64_t b0 = 0; b0 < g.nrhs; b0 += 64) {
    const int nb = (int)std::min<int64_t>(64, g.nrhs - b0);
    if (ws) {
      if (al == 16) rows_ws_launch<LO, 16>(wgrid, nb, A, Xs, P, g, n8, b0, s);
      else if (LO || al == 8) rows_ws_launch<LO, 8>(wgrid, nb, A, Xs, P, g, n8, b0, s);
      else rows_ws_launch<LO, LO ? 8 : 4>(wgrid, nb, A, Xs, P, g, n8, b0, s);  // hi only
    } else if (nb > 32)
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
  const int64_t tiles = ((g.Nm + kBf16Tile - 1) / kBf16Tile) * g.nf;
  const unsigned grid = padded_grid(tiles);
  // 32-bit tile numbers and lane offsets: the warp-specialised kernel, its
  // block loads at the rows' alignment
  const bool ws = tiles < (int64_t{1} << 31) && ws_offsets_fit(g, nd8);
  const unsigned wgrid = ws ? (unsigned)ws_grid(tiles, 1) : 0u;
  const int al = ws_align<LO>(g.Nm);
  for (int64_t b0 = 0; b0 < g.nrhs; b0 += 64) {
    const int nb = (int)std::min<int64_t>(64, g.nrhs - b0);
    if (ws) {
      if (al == 16) cols_ws_launch<LO, 16>(wgrid, nb, A, sc, Ds, Y, g, nd8, b0, s);
      else if (LO || al == 8) cols_ws_launch<LO, 8>(wgrid, nb, A, sc, Ds, Y, g, nd8, b0, s);
      else cols_ws_launch<LO, LO ? 8 : 4>(wgrid, nb, A, sc, Ds, Y, g, nd8, b0, s);  // hi only
    } else if (nb > 32)
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
