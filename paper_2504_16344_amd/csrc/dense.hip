// Dense float64 linear algebra on the data and QoI spaces (section "Real-time
// Bayesian inference and prediction framework", Phases 2-4): a matrix-core
// GEMM, triangular solves with the Cholesky factor of K for many
// right-hand sides at once (the N_q N_t unit vectors of the QoI
// precomputation), and the online QoI prediction q = Q d.
#include "matrix_units.h"

namespace p2o {
namespace {

constexpr int kGemmK = 32;     // contraction chunk staged in LDS
constexpr int kTriNb = 64;     // triangular-solve block (the Cholesky block size)
constexpr int64_t kSolvePanel = 256;  // columns per rank-k update of the solves

// C[i][j] += alpha sum_k A[i][k] op(B)[k][j] for i < M, j < N, row-major,
// op(B)[k][j] = B[j][k] (TRANSB) or B[k][j].  A workgroup owns a TM x TM
// tile of C, each of its 4 wavefronts a quarter (TM/32 x TM/32
// v_mfma_f64_16x16x4 tiles); 32-entry chunks of the contraction are staged
// in LDS as [k][row] for both operands.
// Triangle modes: kTriGrid (a symmetric rank-k update of a lower triangle,
// M == N) enumerates only the tiles I >= J and leaves the entries above the
// diagonal untouched; kTriMask keeps the rectangular grid and only masks
// the entries above the diagonal (a panel whose top square straddles it).
// Without ACC, C is overwritten (C = alpha A op(B)) and never read.
// kFullCols is kFull with the grid's x index running over row tiles, so
// that consecutive work-groups share a column tile of op(B) (for an A small
// enough to stay in the last-level cache while B streams once).
// A and C may be the same matrix when N <= TM (one column tile): a
// work-group reads all of its rows of A before it writes its rows of C, and
// no other work-group touches those rows (the Cholesky's in-place panel
// solve L21 = A21 W^T).
enum { kFull = 0, kTriGrid = 1, kTriMask = 2, kFullCols = 3, kTriUpperSq = 4 };
template <bool TRANSB, int TRI, bool ACC, int TM>
__global__ void __launch_bounds__(256)
dgemm_kernel(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
             const double* __restrict__ B, int64_t ldb, double* C, int64_t ldc) {
  constexpr int MT = TM / 32;  // MFMA tiles per wavefront and dimension
  __shared__ double sa[kGemmK][TM + 1];
  __shared__ double sb[kGemmK][TM + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, kq = lane >> 4;
  int64_t ti_ = blockIdx.y, tj_ = blockIdx.x;
  if constexpr (TRI == kFullCols) {
    ti_ = blockIdx.x;
    tj_ = blockIdx.y;
  }
  if constexpr (TRI == kTriGrid) {  // linear index t -> (I, J), J <= I
    const int64_t t = blockIdx.x;
    int64_t I = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) / 2.0);
    while (I * (I + 1) / 2 > t) --I;
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    ti_ = I;
    tj_ = t - I * (I + 1) / 2;
  }
  const int64_t i0 = ti_ * TM, j0 = tj_ * TM;
  const int wr = (wave >> 1) * (TM / 2), wc = (wave & 1) * (TM / 2);
  d4v acc[MT][MT];
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int b = 0; b < MT; ++b) acc[a][b] = (d4v){0, 0, 0, 0};
  // Each thread stages kPer entries of A and of op(B) per chunk: the next
  // chunk's loads are issued into registers before the current chunk's
  // matrix-core work, at clamped addresses (out-of-range entries are zeroed
  // when stored to LDS).
  constexpr int kPer = kGemmK * TM / 256;
  const int ra = tid / (kGemmK / kPer), ka = (tid % (kGemmK / kPer)) * kPer;  // A, B^T
  const int kb = tid / (TM / kPer), cb = (tid % (TM / kPer)) * kPer;  // B
  double va[kPer], vb[kPer];
  auto load = [&](int64_t k0) {
    const int64_t gi = min(i0 + ra, M - 1);
#pragma unroll
    for (int e = 0; e < kPer; ++e) va[e] = A[gi * lda + min(k0 + ka + e, K - 1)];
    if constexpr (TRANSB) {
      const int64_t gj = min(j0 + ra, N - 1);
#pragma unroll
      for (int e = 0; e < kPer; ++e) vb[e] = B[gj * ldb + min(k0 + ka + e, K - 1)];
    } else {
      const int64_t gk = min(k0 + kb, K - 1);
#pragma unroll
      for (int e = 0; e < kPer; ++e) vb[e] = B[gk * ldb + min(j0 + cb + e, N - 1)];
    }
  };
  auto store = [&](int64_t k0) {
    const bool ia = i0 + ra < M;
#pragma unroll
    for (int e = 0; e < kPer; ++e) sa[ka + e][ra] = (ia && k0 + ka + e < K) ? va[e] : 0.0;
    if constexpr (TRANSB) {
      const bool jb = j0 + ra < N;
#pragma unroll
      for (int e = 0; e < kPer; ++e) sb[ka + e][ra] = (jb && k0 + ka + e < K) ? vb[e] : 0.0;
    } else {
      const bool kin = k0 + kb < K;
#pragma unroll
      for (int e = 0; e < kPer; ++e) sb[kb][cb + e] = (kin && j0 + cb + e < N) ? vb[e] : 0.0;
    }
  };
  load(0);
  for (int64_t k0 = 0; k0 < K; k0 += kGemmK) {
    __syncthreads();  // the previous chunk's reads of sa, sb are done
    store(k0);
    __syncthreads();
    if (k0 + kGemmK < K) load(k0 + kGemmK);
#pragma unroll
    for (int ks = 0; ks < kGemmK; ks += 4) {
      double bf[MT];
#pragma unroll
      for (int tj = 0; tj < MT; ++tj) bf[tj] = sb[ks + kq][wc + 16 * tj + col];
#pragma unroll
      for (int ti = 0; ti < MT; ++ti) {
        const double a = sa[ks + kq][wr + 16 * ti + col];
#pragma unroll
        for (int tj = 0; tj < MT; ++tj) acc[ti][tj] = mfma64(a, bf[tj], acc[ti][tj]);
      }
    }
  }
  // C: all reads (clamped addresses) before the masked writes, so a lane
  // waits for one round trip, not one per entry.  (C is read only when
  // accumulating; the in-place use, A aliasing C, overwrites.)
  double cv[MT][MT][4];
  if constexpr (ACC) {
#pragma unroll
    for (int ti = 0; ti < MT; ++ti)
#pragma unroll
      for (int tj = 0; tj < MT; ++tj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t gi = min(i0 + wr + 16 * ti + kq + 4 * r, M - 1);
          const int64_t gj = min(j0 + wc + 16 * tj + col, N - 1);
          cv[ti][tj][r] = C[gi * ldc + gj];
        }
  }
#pragma unroll
  for (int ti = 0; ti < MT; ++ti)
#pragma unroll
    for (int tj = 0; tj < MT; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gi = i0 + wr + 16 * ti + kq + 4 * r;  // accumulator rows interleave
        const int64_t gj = j0 + wc + 16 * tj + col;
        if (gi < M && gj < N && (TRI == kFull || TRI == kFullCols || gj <= gi))
          C[gi * ldc + gj] = ACC ? cv[ti][tj][r] + alpha * acc[ti][tj][r] : alpha * acc[ti][tj][r];
      }
}

// ------------------------------------------ C (+)= alpha A B^T, large shapes
// For the big contractions with both operands row-major along the
// contraction (the Cholesky's trailing rank-512 updates, the Gram matrix,
// the solves' rank-256 updates): a 128 x 128 tile of C a work-group, each
// of its 4 wavefronts a 64 x 64 quarter (4 x 4 v_mfma_f64_16x16x4 tiles,
// 128 accumulator registers), so every operand value read from LDS feeds 4
// products and every byte staged feeds twice as many flops as on 64 x 64
// tiles.  The contraction is cut into 16-entry chunks: one 128-byte line of
// each operand row, loaded as 16-byte vectors and stored unchanged into
// LDS (granule G = entries 2G, 2G + 1 of row r at granule G ^ ((r / 2) mod
// 8), so the 16 rows a lane group reads at one granule fall on 16
// different bank groups).  Lane group q takes contraction entries 4q .. 4q
// + 3 of a chunk (one ds_read_b128 for two products), in the same order for
// both operands, so the chunk's sum is complete.  Two LDS stages and one
// barrier (without memory fences) per chunk: while the products of chunk c
// run, chunk c + 1 is already in the other stage and chunk c + 2 is in
// flight into registers.  Rows past M (N) re-read row M - 1 (N - 1) and are
// dropped; entries past K are zero in both operands.
constexpr int kNtTile = 128;
constexpr int kNtK = 16;
constexpr int kNtStage = kNtTile * kNtK;  // doubles of one operand in one stage
constexpr int kNtBRow = 130;              // row pitch (doubles) of a row-major B chunk

__device__ __forceinline__ int nt_lds_pos(int r, int g) { return r * kNtK + 2 * (g ^ ((r >> 1) & 7)); }

// This wavefront's LDS accesses have completed.
__device__ __forceinline__ void nt_wait_lds() {
  __builtin_amdgcn_s_waitcnt(15 | (7 << 4) | (0 << 8) | (3 << 14));
}

// Work-group barrier without the memory fences of __syncthreads (which
// would also wait for the next chunk's global loads); the compiler moves no
// memory access across it.
__device__ __forceinline__ void nt_barrier() {
  __asm__ volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  __asm__ volatile("" ::: "memory");
}

// TRI: kFull (tile t = I tc + J), kTriGrid (tiles I >= J, entries above
// the diagonal untouched) or kTriUpperSq: C = alpha Y Y^T in place for an
// upper-triangular Y (A = B = C = Y, n x n, entries below the diagonal
// zero): tiles I >= J, contraction from column i0 on (row i of Y is zero
// before column i); every operand entry below the diagonal is taken as
// zero (this launch may already have overwritten it), only the strict
// lower triangle of C is written and the diagonal goes to diag[], so no
// entry that any work-group reads as non-zero is ever written.  Both
// operands 16-byte aligned with even leading dimensions (the launcher
// checks).  No __restrict__: the in-place form aliases A, B and C.
// BROW: C (+)= alpha A B with B row-major along the contraction ([K][N],
// kFull only): its chunk is kept in LDS as 16 rows of kNtBRow doubles (the
// 130-double pitch puts the 4 lane groups of a read on distinct banks) and
// each product takes its two contraction entries from two 8-byte reads.
template <int TRI, bool ACC, bool BROW = false>
__global__ void __launch_bounds__(256, 2)
dgemm_nt128_kernel(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                   const double* B, int64_t ldb, double* C, int64_t ldc, int64_t tiles,
                   double* diag) {
  static_assert(!BROW || TRI == kFull, "row-major B on the full grid only");
  __shared__ __align__(16) double lds[2][2][kNtStage + (BROW ? kNtK * (kNtBRow - kNtTile) : 0)];
  // kTriUpperSq: a tile's contraction shrinks with its row band, so the
  // tiles are dealt to the XCDs round-robin in grid order (long ones first)
  // rather than in contiguous ranges, which would leave one XCD the bulk
  const int64_t t = TRI == kTriUpperSq ? (int64_t)blockIdx.x : xcd_local_tile(blockIdx.x, gridDim.x);
  if (t >= tiles) return;  // grid padding
  int64_t ti_, tj_;
  if constexpr (TRI == kTriGrid || TRI == kTriUpperSq) {
    // 8 x 8 super-blocks of tiles, in row-major order over the lower
    // triangle of super-blocks, tiles row-major inside a super-block: the
    // tiles an XCD runs at once share 8 row and 8 column bands of the
    // operands in its L2 (row-major tiles share one row band and stream a
    // new column band each)
    constexpr int64_t S = 8;
    const int64_t tr = (M + kNtTile - 1) / kNtTile;
    int64_t rem = t, IB = 0, h = 0;
    for (;; ++IB) {
      h = min(S, tr - IB * S);
      const int64_t cnt = IB * h * S + h * (h + 1) / 2;
      if (rem < cnt) break;
      rem -= cnt;
    }
    const int64_t JB = rem / (h * S);
    if (JB < IB) {
      const int64_t l = rem - JB * h * S;
      ti_ = IB * S + l / S;
      tj_ = JB * S + l % S;
    } else {
      const int64_t l = rem - IB * h * S;
      int64_t r = (int64_t)((sqrt(8.0 * (double)l + 1.0) - 1.0) / 2.0);
      while (r * (r + 1) / 2 > l) --r;
      while ((r + 1) * (r + 2) / 2 <= l) ++r;
      ti_ = IB * S + r;
      tj_ = IB * S + (l - r * (r + 1) / 2);
    }
  } else {
    const int64_t tc = (N + kNtTile - 1) / kNtTile;
    ti_ = t / tc;
    tj_ = t - ti_ * tc;
  }
  const int64_t i0 = ti_ * kNtTile, j0 = tj_ * kNtTile;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
  // loader: granule lg of rows lr + 32 u (u < 4) of both operands
  const int lg = tid & 7, lr = tid >> 3;
  const double* pa[4];
  const double* pb[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    pa[u] = A + min(i0 + lr + 32 * u, M - 1) * lda + 2 * lg;
    // BROW: row wave + 4 u of the chunk, columns j0 + 2 lane, + 1 (N even;
    // columns past N re-read the last pair and are dropped)
    pb[u] = BROW ? B + min(j0 + 2 * lane, N - 2) : B + min(j0 + lr + 32 * u, N - 1) * ldb + 2 * lg;
  }
  d2v ra[4], rb[4];
  // kTriUpperSq: the contraction starts at i0 (>= j0)
  const int64_t kbeg = TRI == kTriUpperSq ? i0 : 0;
  auto load = [&](int64_t k0) {
    if (k0 + kNtK <= K) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        ra[u] = *reinterpret_cast<const d2v*>(pa[u] + k0);
        rb[u] = BROW ? *reinterpret_cast<const d2v*>(pb[u] + (k0 + wave + 4 * u) * ldb)
                     : *reinterpret_cast<const d2v*>(pb[u] + k0);
      }
      if constexpr (TRI == kTriUpperSq) {  // entries below the diagonal are zero
        // entry k0 + 2 lg + h of row i0 + lr + 32 u: k - row = (k0 - i0) + h - thr
        const int da = (int)(k0 - i0), db = (int)(k0 - j0), thr = lr - 2 * lg;
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            ra[u][h] = da + h >= thr + 32 * u ? ra[u][h] : 0.0;
            rb[u][h] = db + h >= thr + 32 * u ? rb[u][h] : 0.0;
          }
      }
    } else {  // the contraction's ragged end
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int64_t e = k0 + 2 * lg + h;  // contraction index of this entry
          const int64_t ec = min(e, K - 1) - 2 * lg;
          const double x = pa[u][ec];
          const bool la = TRI != kTriUpperSq || (int)(e - i0) >= lr + 32 * u;
          ra[u][h] = e < K && la ? x : 0.0;
          if constexpr (!BROW) {
            const double y = pb[u][ec];
            const bool lb = TRI != kTriUpperSq || (int)(e - j0) >= lr + 32 * u;
            rb[u][h] = e < K && lb ? y : 0.0;
          }
        }
      if constexpr (BROW) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int64_t r = k0 + wave + 4 * u;  // contraction row of B
          const d2v y = *reinterpret_cast<const d2v*>(pb[u] + min(r, K - 1) * ldb);
          rb[u] = r < K ? y : (d2v){0.0, 0.0};
        }
      }
    }
  };
  auto store = [&](int st) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      *reinterpret_cast<d2v*>(&lds[st][0][nt_lds_pos(lr + 32 * u, lg)]) = ra[u];
      if constexpr (BROW) {  // row wave + 4 u, two 8-byte stores (the pitch is not 16-aligned)
        double* q = &lds[st][1][(wave + 4 * u) * kNtBRow + 2 * lane];
        q[0] = rb[u][0];
        q[1] = rb[u][1];
      } else {
        *reinterpret_cast<d2v*>(&lds[st][1][nt_lds_pos(lr + 32 * u, lg)]) = rb[u];
      }
    }
  };
  d4v acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = (d4v){0, 0, 0, 0};
  const int64_t nc = (K - kbeg + kNtK - 1) / kNtK;
  load(kbeg);
  store(0);
  if (nc > 1) load(kbeg + kNtK);
  nt_wait_lds();
  nt_barrier();
  for (int64_t c = 0; c < nc; ++c) {
    const int cur = (int)(c & 1);
    if (c + 1 < nc) {  // chunk c + 1 into the other stage (read by chunk c - 1's products, done)
      store(cur ^ 1);
      if (c + 2 < nc) load(kbeg + (c + 2) * kNtK);
    }
    const double* sa = lds[cur][0];
    const double* sb = lds[cur][1];
#pragma unroll
    for (int h = 0; h < 2; ++h) {  // contraction entries 4 kq + 2 h + {0, 1}
      d2v a[4], b[4];
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        a[f] = *reinterpret_cast<const d2v*>(&sa[nt_lds_pos(wr + 16 * f + col, 2 * kq + h)]);
        if constexpr (BROW) {
          const double* q = &sb[(4 * kq + 2 * h) * kNtBRow + wc + 16 * f + col];
          b[f] = (d2v){q[0], q[kNtBRow]};
        } else {
          b[f] = *reinterpret_cast<const d2v*>(&sb[nt_lds_pos(wc + 16 * f + col, 2 * kq + h)]);
        }
      }
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int fi = 0; fi < 4; ++fi)
#pragma unroll
          for (int fj = 0; fj < 4; ++fj) acc[fi][fj] = mfma64(a[fi][e], b[fj][e], acc[fi][fj]);
    }
    nt_wait_lds();
    nt_barrier();
  }
  // C: per 16-row group, all reads (clamped addresses) before the masked
  // writes, so a lane waits for one round trip per group, not per entry
#pragma unroll
  for (int fi = 0; fi < 4; ++fi) {
    double cv[4][4];
    if constexpr (ACC) {
#pragma unroll
      for (int fj = 0; fj < 4; ++fj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t gi = min(i0 + wr + 16 * fi + kq + 4 * r, M - 1);
          const int64_t gj = min(j0 + wc + 16 * fj + col, N - 1);
          cv[fj][r] = C[gi * ldc + gj];
        }
    }
#pragma unroll
    for (int fj = 0; fj < 4; ++fj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gi = i0 + wr + 16 * fi + kq + 4 * r;  // accumulator rows interleave
        const int64_t gj = j0 + wc + 16 * fj + col;
        if constexpr (TRI == kTriUpperSq) {
          if (gi < M && gj < N && gj < gi) C[gi * ldc + gj] = alpha * acc[fi][fj][r];
          if (gi < M && gj == gi) diag[gi] = alpha * acc[fi][fj][r];
        } else if (gi < M && gj < N && (TRI == kFull || gj <= gi)) {
          C[gi * ldc + gj] = ACC ? cv[fj][r] + alpha * acc[fi][fj][r] : alpha * acc[fi][fj][r];
        }
      }
  }
}

// Prefix sums along the block diagonals of X (rows (a, i) = a P + i, columns
// (b, j) = b Q + j, a, b < T):
//   X[(a, i)][(b, j)] <- sum_{l = 0 .. min(a, b)} X[(a - l, i)][(b - l, j)].
// One thread walks one chain (r, c), (r + P, c + Q), ... from its first
// entry (a = 0 or b = 0); chains are disjoint, so the sums are formed in
// place.  Lanes take consecutive columns of a chain start row, so every step
// of a wavefront reads a contiguous run.  With LOWER (P == Q, a symmetric
// matrix of which only the lower triangle is kept) chains that start above
// the diagonal are skipped and every other chain stays on or below it.
constexpr int kScanGroup = 8;  // chain entries loaded ahead of their sums
__global__ void __launch_bounds__(256)
block_diag_scan(double* __restrict__ X, int64_t ld, int64_t T, int64_t P, int64_t Q, int lower) {
  const int64_t R = T * P, Cn = T * Q;
  const int64_t nA = lower ? 0 : P * Cn;               // chains from block row 0
  const int64_t nB = lower ? R * Q : (R - P) * Q;      // chains from block column 0
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nA + nB;
       e += (int64_t)gridDim.x * 256) {
    int64_t r0, c0;
    if (e < nA) {
      r0 = e / Cn;
      c0 = e - r0 * Cn;
    } else {
      const int64_t f = e - nA;
      r0 = (lower ? 0 : P) + f / Q;
      c0 = f % Q;
    }
    if (lower && c0 > r0) continue;
    const int64_t steps = std::min((R - 1 - r0) / P, (Cn - 1 - c0) / Q) + 1;
    const int64_t stride = P * ld + Q;
    double* __restrict__ p = X + r0 * ld + c0;
    double acc = 0.0;
    for (int64_t l = 0; l < steps; l += kScanGroup) {
      double v[kScanGroup];
#pragma unroll
      for (int g = 0; g < kScanGroup; ++g)  // clamped: every load in bounds
        v[g] = p[std::min(l + g, steps - 1) * stride];
#pragma unroll
      for (int g = 0; g < kScanGroup; ++g) {
        if (l + g < steps) {
          acc += v[g];
          p[(l + g) * stride] = acc;
        }
      }
    }
  }
}

// Diagonal blocks of the triangular solves for many right-hand sides.  Y is
// [nrhs][n]; a wavefront owns one right-hand side at a time (lane = row of
// the block), the block of the factor sits in LDS for the workgroup (loaded
// coalesced, all loads issued first, clamped addresses), and each lane keeps
// the reciprocal of its diagonal entry, so a step is one multiply and one
// cross-lane broadcast.
__device__ __forceinline__ double load_tri_block(const double* __restrict__ K, int64_t n,
                                                 int64_t j0, int bs, double (*l)[kTriNb + 1]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cl = min(lane, bs - 1);
  double v[kTriNb / 4];
#pragma unroll
  for (int u = 0; u < kTriNb / 4; ++u) v[u] = K[(j0 + min(4 * u + wave, bs - 1)) * n + j0 + cl];
#pragma unroll
  for (int u = 0; u < kTriNb / 4; ++u) {
    const int row = 4 * u + wave;
    l[row][lane] = (row < bs && lane <= row) ? v[u] : 0.0;
  }
  __syncthreads();
  return 1.0 / l[cl][cl];
}

// Forward: y[j0 : j0 + bs] = L11^{-1} y[j0 : j0 + bs].
__global__ void __launch_bounds__(256)
trsm_lower_diag_many(const double* __restrict__ K, double* __restrict__ Y, int64_t n,
                     int64_t nrhs, int64_t j0, int bs) {
  __shared__ double l[kTriNb][kTriNb + 1];
  const double rl = load_tri_block(K, n, j0, bs, l);
  const int lane = threadIdx.x & 63;
  const int cl = min(lane, bs - 1);
  for (int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < nrhs;
       r += (int64_t)gridDim.x * 4) {
    double* y = Y + r * n + j0;
    double v = y[cl];
    if (lane >= bs) v = 0.0;
    for (int c = 0; c < bs; ++c) {
      const double yc = __shfl(v * rl, c, 64);
      if (lane == c) v = yc;
      else if (lane > c) v -= l[lane][c] * yc;
    }
    if (lane < bs) y[lane] = v;
  }
}

// Backward: x[j0 : j0 + bs] = L11^{-T} y[j0 : j0 + bs].
__global__ void __launch_bounds__(256)
trsm_upper_diag_many(const double* __restrict__ K, double* __restrict__ Y, int64_t n,
                     int64_t nrhs, int64_t j0, int bs) {
  __shared__ double l[kTriNb][kTriNb + 1];
  const double rl = load_tri_block(K, n, j0, bs, l);
  const int lane = threadIdx.x & 63;
  const int cl = min(lane, bs - 1);
  for (int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < nrhs;
       r += (int64_t)gridDim.x * 4) {
    double* y = Y + r * n + j0;
    double v = y[cl];
    if (lane >= bs) v = 0.0;
    for (int t = bs - 1; t >= 0; --t) {
      const double xt = __shfl(v * rl, t, 64);
      if (lane == t) v = xt;
      else if (lane < t) v -= l[t][lane] * xt;
    }
    if (lane < bs) y[lane] = v;
  }
}

// q[r][i] = sum_j Q[i][j] d[r][j] for RB right-hand sides at a time: one
// work-group of W wavefronts per RQ rows of Q, wavefront w summing the w-th
// of W contiguous column ranges of all RQ rows (each d entry loaded once
// serves RQ rows); each lane takes 2 consecutive entries per 128-entry step
// and U steps per loop turn, all loads issued before any product
// (unconditional, clamped addresses; entries past the range are zeroed at
// the consumer).  The W partial sums are added in LDS in a fixed order.  Q
// is streamed once per pass with non-temporal loads.  V16 (cols even, Q and
// D 16-byte aligned): a lane's 2 entries are one 16-byte load (measured
// 152 -> 110 us for a 4200 x 20000 Q; the 8-byte pairs left it at 0.55 of
// the HBM peak); the per-lane order of the additions is the same either
// way, so the results are identical.
template <int RB, int U, int W, int RQ, bool V16>
__global__ void __launch_bounds__(64 * W)
qoi_gemv(const double* __restrict__ Q, const double* __restrict__ D, double* __restrict__ q,
         int64_t rows, int64_t cols, int64_t r0, int nb) {
  __shared__ double red[W][RQ][RB];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * RQ;
  const double* __restrict__ Qr[RQ];
#pragma unroll
  for (int w = 0; w < RQ; ++w) Qr[w] = Q + min(i0 + w, rows - 1) * cols;
  const int64_t span = (cols + 128 * W - 1) / (128 * W) * 128;
  const int64_t c0 = wave * span, c1 = min(cols, c0 + span);
  double acc[RQ][RB];
#pragma unroll
  for (int w = 0; w < RQ; ++w)
#pragma unroll
    for (int b = 0; b < RB; ++b) acc[w][b] = 0.0;
  for (int64_t j0 = c0 + 2 * lane; j0 < c1; j0 += 128 * U) {
    double qv[RQ][2 * U], dv[RB][2 * U];
    if constexpr (V16) {  // j0 is even, so the pair is 16-byte aligned
#pragma unroll
      for (int u = 0; u < 2 * U; u += 2) {
        const int64_t j = min(j0 + 128 * (u >> 1), cols - 2);
#pragma unroll
        for (int w = 0; w < RQ; ++w) {
          const d2v x = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(Qr[w] + j));
          qv[w][u] = x.x;
          qv[w][u + 1] = x.y;
        }
#pragma unroll
        for (int b = 0; b < RB; ++b) {
          const d2v y = *reinterpret_cast<const d2v*>(D + (r0 + min(b, nb - 1)) * cols + j);
          dv[b][u] = y.x;
          dv[b][u + 1] = y.y;
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < 2 * U; ++u) {
        const int64_t j = min(j0 + 128 * (u >> 1) + (u & 1), cols - 1);
#pragma unroll
        for (int w = 0; w < RQ; ++w) qv[w][u] = __builtin_nontemporal_load(Qr[w] + j);
#pragma unroll
        for (int b = 0; b < RB; ++b) dv[b][u] = D[(r0 + min(b, nb - 1)) * cols + j];
      }
    }
#pragma unroll
    for (int u = 0; u < 2 * U; ++u) {
      const bool in = j0 + 128 * (u >> 1) + (u & 1) < c1;
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        const double du = in ? dv[b][u] : 0.0;
#pragma unroll
        for (int w = 0; w < RQ; ++w) acc[w][b] += qv[w][u] * du;
      }
    }
  }
#pragma unroll
  for (int w = 0; w < RQ; ++w)
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const double s = wave_sum(acc[w][b]);
      if (lane == 0) red[wave][w][b] = s;
    }
  __syncthreads();
  if (threadIdx.x < RQ * RB) {
    const int w = threadIdx.x / RB, b = threadIdx.x % RB;
    if (b < nb && i0 + w < rows) {
      double s = 0.0;
#pragma unroll
      for (int v = 0; v < W; ++v) s += red[v][w][b];
      q[(r0 + b) * rows + i0 + w] = s;
    }
  }
}

unsigned grid_rhs(int64_t nrhs) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((nrhs + 3) / 4, 2048));
}

}  // namespace

// One GEMM launch on 64 x 64 tiles (128 x 128 tiles need ~224 VGPRs, one
// wavefront per SIMD, and measured slower).
template <bool TRANSB, int TRI, bool ACC>
hipError_t launch_gemm(int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                       int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
                       hipStream_t s) {
  if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
  constexpr int64_t tm = 64;
  const int64_t tr = (M + tm - 1) / tm, tc = (N + tm - 1) / tm;
  dim3 grid;
  if (TRI == kTriGrid) {
    if (tr * (tr + 1) / 2 > 0x7fffffff) return hipErrorInvalidConfiguration;
    grid = dim3((unsigned)(tr * (tr + 1) / 2));
  } else if (TRI == kFullCols) {
    if (tc > 65535) return hipErrorInvalidConfiguration;
    grid = dim3((unsigned)tr, (unsigned)tc);
  } else {
    if (tr > 65535) return hipErrorInvalidConfiguration;
    grid = dim3((unsigned)tc, (unsigned)tr);
  }
  hipLaunchKernelGGL((dgemm_kernel<TRANSB, TRI, ACC, tm>), grid, dim3(256), 0, s, M, N, K, alpha,
                     A, lda, B, ldb, C, ldc);
  return hipGetLastError();
}

// The 128 x 128 kernel: both operands 16-byte aligned with even leading
// dimensions, and C large enough that its fewer, larger tiles still fill
// the chip.
bool nt128_fits(int64_t M, int64_t N, const double* A, int64_t lda, const double* B,
                int64_t ldb) {
  const uintptr_t al = reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B);
  return al % 16 == 0 && lda % 2 == 0 && ldb % 2 == 0 && std::min(M, N) >= 512;
}

template <int TRI, bool ACC, bool BROW = false>
hipError_t launch_gemm_nt128(int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                             int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
                             hipStream_t s, double* diag = nullptr) {
  const int64_t tr = (M + kNtTile - 1) / kNtTile, tc = (N + kNtTile - 1) / kNtTile;
  const int64_t tiles = TRI == kFull ? tr * tc : tr * (tr + 1) / 2;
  const int64_t grid = (tiles + kXcds - 1) / kXcds * kXcds;
  if (grid > 0x7fffffff) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((dgemm_nt128_kernel<TRI, ACC, BROW>), dim3((unsigned)grid), dim3(256), 0, s, M, N,
                     K, alpha, A, lda, B, ldb, C, ldc, tiles, diag);
  return hipGetLastError();
}

hipError_t launch_dgemm(bool transb, int64_t M, int64_t N, int64_t K, double alpha,
                        const double* A, int64_t lda, const double* B, int64_t ldb, double* C,
                        int64_t ldc, hipStream_t s) {
  if (transb && M > 0 && N > 0 && K > 0 && nt128_fits(M, N, A, lda, B, ldb))
    return launch_gemm_nt128<kFull, true>(M, N, K, alpha, A, lda, B, ldb, C, ldc, s);
  if (transb) return launch_gemm<true, kFull, true>(M, N, K, alpha, A, lda, B, ldb, C, ldc, s);
  if (M > 0 && N > 0 && K > 0 && N % 2 == 0 && nt128_fits(M, N, A, lda, B, ldb))
    return launch_gemm_nt128<kFull, true, true>(M, N, K, alpha, A, lda, B, ldb, C, ldc, s);
  return launch_gemm<false, kFull, true>(M, N, K, alpha, A, lda, B, ldb, C, ldc, s);
}

hipError_t launch_dgemm_nt_set(bool lower, int64_t M, int64_t N, int64_t K, double alpha,
                               const double* A, int64_t lda, const double* B, int64_t ldb,
                               double* C, int64_t ldc, hipStream_t s) {
  if (M <= 0 || N <= 0 || K <= 0 || (lower && M != N)) return hipErrorInvalidValue;
  if (lower && nt128_fits(M, N, A, lda, B, ldb))
    return launch_gemm_nt128<kTriGrid, false>(M, N, K, alpha, A, lda, B, ldb, C, ldc, s);
  if (lower)
    return launch_gemm<true, kTriGrid, false>(M, N, K, alpha, A, lda, B, ldb, C, ldc, s);
  // row tiles along x: A stays cached while B streams once
  return launch_gemm<true, kFullCols, false>(M, N, K, alpha, A, lda, B, ldb, C, ldc, s);
}

hipError_t launch_dgemm_nt_lower(int64_t n, int64_t K, double alpha, const double* A,
                                 int64_t lda, const double* B, int64_t ldb, double* C,
                                 int64_t ldc, hipStream_t s) {
  if (n > 0 && K > 0 && nt128_fits(n, n, A, lda, B, ldb))
    return launch_gemm_nt128<kTriGrid, true>(n, n, K, alpha, A, lda, B, ldb, C, ldc, s);
  return launch_gemm<true, kTriGrid, true>(n, n, K, alpha, A, lda, B, ldb, C, ldc, s);
}

hipError_t launch_dgemm_nt_lower_mask(int64_t M, int64_t N, int64_t K, double alpha,
                                      const double* A, int64_t lda, const double* B,
                                      int64_t ldb, double* C, int64_t ldc, hipStream_t s) {
  return launch_gemm<true, kTriMask, true>(M, N, K, alpha, A, lda, B, ldb, C, ldc, s);
}

hipError_t launch_block_diag_scan(double* X, int64_t ld, int64_t T, int64_t P, int64_t Q,
                                  bool lower, hipStream_t s) {
  if (T <= 0 || P <= 0 || Q <= 0 || (lower && P != Q)) return hipErrorInvalidValue;
  const int64_t chains = lower ? T * P * Q : P * T * Q + (T - 1) * P * Q;
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((chains + 255) / 256, 1 << 20));
  hipLaunchKernelGGL(block_diag_scan, dim3(g), dim3(256), 0, s, X, ld, T, P, Q, lower ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_dsyrk_lower(int64_t n, int64_t K, double alpha, const double* A, int64_t lda,
                              double* C, int64_t ldc, hipStream_t s) {
  if (n > 0 && K > 0 && nt128_fits(n, n, A, lda, A, lda))
    return launch_gemm_nt128<kTriGrid, true>(n, n, K, alpha, A, lda, A, lda, C, ldc, s);
  return launch_gemm<true, kTriGrid, true>(n, n, K, alpha, A, lda, A, lda, C, ldc, s);
}

// K holds the Cholesky factor L in its lower triangle.  Y ([nrhs][n]) is
// overwritten by K^{-1} Y = L^{-T} L^{-1} Y: block by block, the diagonal
// solve of every right-hand side, then the update of the others as
// matrix-core GEMMs (forward: Y[:, rest] -= Y[:, blk] L[rest, blk]^T;
// backward: Y[:, 0 : j0] -= Y[:, blk] L[blk, 0 : j0]), the updates beyond
// the current panel of kSolvePanel columns deferred and done as one.
namespace {
// The sweeps below for all nrhs right-hand sides, or (INV, Y = I, nrhs = n)
// only for the rows whose result is needed: row r of L^{-1} I is zero before
// column r, so a forward step on columns below c1 touches rows r < c1 only;
// of X = K^{-1} (symmetric) only the entries c >= r are kept, so a backward
// step that updates columns below c0 needs rows r < c0 only.  About half the
// work of the full solve.
hipError_t solve_many_sweeps(const double* K, double* Y, int64_t n, int64_t nrhs, bool inv,
                             bool backward, hipStream_t s) {
  hipError_t e = hipSuccess;
  auto rows = [&](int64_t c) { return inv ? std::min(nrhs, c) : nrhs; };
  // forward, L Z = Y: panels of kSolvePanel columns; inside a panel block by
  // block (diagonal solve, update of the panel's later columns), then one
  // rank-kSolvePanel update of all later columns
  for (int64_t p0 = 0; p0 < n; p0 += kSolvePanel) {
    const int64_t p1 = std::min(n, p0 + kSolvePanel);
    for (int64_t j0 = p0; j0 < p1; j0 += kTriNb) {
      const int bs = (int)std::min<int64_t>(kTriNb, p1 - j0);
      const int64_t j1 = j0 + bs;
      hipLaunchKernelGGL(trsm_lower_diag_many, dim3(grid_rhs(rows(j1))), dim3(256), 0, s, K, Y, n,
                         rows(j1), j0, bs);
      if (j1 < p1 && (e = launch_dgemm(true, rows(j1), p1 - j1, bs, -1.0, Y + j0, n,
                                       K + j1 * n + j0, n, Y + j1, n, s)) != hipSuccess)
        return e;
    }
    if (p1 < n && (e = launch_dgemm(true, rows(p1), n - p1, p1 - p0, -1.0, Y + p0, n,
                                    K + p1 * n + p0, n, Y + p1, n, s)) != hipSuccess)
      return e;
  }
  if (!backward) return hipGetLastError();
  // backward, L^T X = Z: the same from the last panel down
  for (int64_t p0 = ((n - 1) / kSolvePanel) * kSolvePanel; p0 >= 0; p0 -= kSolvePanel) {
    const int64_t p1 = std::min(n, p0 + kSolvePanel);
    for (int64_t j0 = p0 + ((p1 - 1 - p0) / kTriNb) * kTriNb; j0 >= p0; j0 -= kTriNb) {
      const int bs = (int)std::min<int64_t>(kTriNb, p1 - j0);
      hipLaunchKernelGGL(trsm_upper_diag_many, dim3(grid_rhs(rows(j0 + bs))), dim3(256), 0, s, K,
                         Y, n, rows(j0 + bs), j0, bs);
      if (j0 > p0 && (e = launch_dgemm(false, rows(j0), j0 - p0, bs, -1.0, Y + j0, n,
                                       K + j0 * n + p0, n, Y + p0, n, s)) != hipSuccess)
        return e;
    }
    if (p0 > 0 && (e = launch_dgemm(false, rows(p0), p0, p1 - p0, -1.0, Y + p0, n, K + p0 * n, n,
                                    Y, n, s)) != hipSuccess)
      return e;
  }
  return hipGetLastError();
}
}  // namespace

hipError_t launch_cholesky_solve_many(const double* K, double* Y, int64_t n, int64_t nrhs,
                                      hipStream_t s) {
  return solve_many_sweeps(K, Y, n, nrhs, false, true, s);
}

hipError_t launch_cholesky_inverse_upper(const double* K, double* Y, int64_t n, hipStream_t s) {
  return solve_many_sweeps(K, Y, n, n, true, true, s);
}

bool cholesky_inverse_by_square_fits(const double* Y, int64_t n) {
  return nt128_fits(n, n, Y, n, Y, n);
}

hipError_t launch_cholesky_inverse_by_square(const double* K, double* Y, double* diag, int64_t n,
                                             hipStream_t s) {
  if (!cholesky_inverse_by_square_fits(Y, n)) return hipErrorInvalidValue;
  // forward sweep only: row r of Y becomes L^{-1} e_r, so Y = L^{-T}
  // (upper triangular)
  hipError_t e = solve_many_sweeps(K, Y, n, n, true, false, s);
  if (e != hipSuccess) return e;
  // K^{-1} = L^{-T} L^{-1} = Y Y^T: strict lower triangle in place, the
  // diagonal into diag
  return launch_gemm_nt128<kTriUpperSq, false>(n, n, n, 1.0, Y, n, Y, n, Y, n, s, diag);
}

namespace {
template <bool V16>
hipError_t qoi_gemv_passes(const double* Q, const double* D, double* q, int64_t rows,
                           int64_t cols, int64_t nrhs, hipStream_t s) {
  // wavefronts per work-group, 128-entry steps per turn, rows of Q per work-group
  constexpr int W = 8, U = 4, RQ = 2;
  const int64_t g = (rows + RQ - 1) / RQ;
  if (g > 0x7fffffff) return hipErrorInvalidConfiguration;
  for (int64_t r0 = 0; r0 < nrhs; r0 += 4) {
    const int nb = (int)std::min<int64_t>(4, nrhs - r0);
    if (nb == 1)
      hipLaunchKernelGGL((qoi_gemv<1, U, W, RQ, V16>), dim3((unsigned)g), dim3(64 * W), 0, s, Q, D,
                         q, rows, cols, r0, nb);
    else if (nb == 2)
      hipLaunchKernelGGL((qoi_gemv<2, U, W, RQ, V16>), dim3((unsigned)g), dim3(64 * W), 0, s, Q, D,
                         q, rows, cols, r0, nb);
    else
      hipLaunchKernelGGL((qoi_gemv<4, U, W, RQ, V16>), dim3((unsigned)g), dim3(64 * W), 0, s, Q, D,
                         q, rows, cols, r0, nb);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
}  // namespace

hipError_t launch_qoi_gemv(const double* Q, const double* D, double* q, int64_t rows,
                           int64_t cols, int64_t nrhs, hipStream_t s) {
  const uintptr_t al = reinterpret_cast<uintptr_t>(Q) | reinterpret_cast<uintptr_t>(D);
  if (cols % 2 == 0 && al % 16 == 0) return qoi_gemv_passes<true>(Q, D, q, rows, cols, nrhs, s);
  return qoi_gemv_passes<false>(Q, D, q, rows, cols, nrhs, s);
}

}  // namespace p2o
