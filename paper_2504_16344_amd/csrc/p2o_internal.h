// Internal declarations of the p2o library: plan object, transform
// descriptors, and the kernel launchers each .hip file provides.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "p2o.h"

namespace p2o {

// ---------------------------------------------------------------- complex
template <typename T>
struct cpx {
  T x, y;
};

// ------------------------------------------------------------- transforms
// Real transforms of length L along the time axis, computed as a complex
// DFT of length N = L/2 on z[n] = x[2n] + i x[2n+1] (in-place mixed-radix
// decimation in frequency, radices 4, 2, 3, 5, 7), with the even/odd split
// undone on the way out.  Output bins are 0..N (nf = N + 1).
constexpr int kMaxStages = 24;

// float32 -> bfloat16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t bf16_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

struct FftDesc {
  int N;    // complex length L/2
  int L;    // real embedding length
  int Nt;   // real samples read (forward) / written (inverse)
  int nst;  // number of radix stages
  int radix[kMaxStages];
};

// Column-batched layout of one transform call.  Columns are contiguous in
// memory; the transformed axis (time or frequency) has its own stride; a
// second grid axis walks independent batches (right-hand sides, or sensors
// during setup).
struct FftIo {
  const void* in;
  void* out;
  int64_t ncols;       // columns per batch
  int64_t in_row;      // element stride between consecutive rows of `in`
  int64_t in_batch;    // element stride between batches of `in`
  int64_t out_row;
  int64_t out_batch;
  int nparts;          // inverse only: number of partial spectra summed
  int64_t part_stride; // inverse only: element stride between partials
  double scale;        // inverse only: output multiplier (1/L folded in)
  // Forward float32 only: when `planes` is set, the bins are written as the
  // four bfloat16 planes of the matrix-core products instead of to `out`:
  // planes[((b nbins + k) 4 + q) n8 + c], q = re hi, re lo, im hi, im lo
  // (x = hi + lo, each rounded to nearest even), optionally multiplied by
  // the column sub-block scales first; padding columns ncols..n8-1 are zero.
  uint16_t* planes;
  int64_t n8;            // plane pitch (ncols rounded up to 8, or to 32 in slot order)
  int64_t nbins;         // frequency bins per batch (nf)
  const float* col_scales;  // [nbins][ceil(ncols / kScaleTile)] or nullptr
  int slot_order;        // 0: columns in order; 1 / 2: each 32-column chunk in the
                         // matrix-core slot order of F's hi+lo / hi-only products
};

// Matrix-core slot order of F's bfloat16 products.  A 32-entry contraction
// chunk feeds slots j = 0..7 of lane groups kg = 0..3; slot j of group kg
// takes chunk entry row_slot_entry(kg, j), chosen so the 4 groups of a block
// row read one contiguous 64-byte span per 16-byte load (hi+lo entries are 8
// bytes, hi-only 4).  The forward transform stores F's vector planes with
// entry e of each chunk at position row_slot_position(e) = 8 kg + j, so the
// 8 slots of a group are one 16-byte run.
__host__ __device__ constexpr int row_slot_entry(bool lo, int kg, int j) {
  return lo ? 8 * (j >> 1) + 2 * kg + (j & 1) : 16 * (j >> 2) + 4 * kg + (j & 3);
}
__host__ __device__ constexpr int row_slot_position(bool lo, int e) {
  return lo ? 8 * ((e >> 1) & 3) + 2 * (e >> 3) + (e & 1)
            : 8 * ((e >> 2) & 3) + 4 * (e >> 4) + (e & 3);
}
__host__ __device__ constexpr bool row_slots_are_inverse() {
  for (int lo = 0; lo < 2; ++lo)
    for (int kg = 0; kg < 4; ++kg)
      for (int j = 0; j < 8; ++j)
        if (row_slot_position(lo, row_slot_entry(lo, kg, j)) != 8 * kg + j) return false;
  return true;
}
static_assert(row_slots_are_inverse(), "slot order and plane positions must match");

int64_t smooth_length(int64_t Nt);  // L: smallest even 7-smooth >= 2*Nt
bool make_fft_desc(int64_t Nt, FftDesc* d);
std::vector<int> make_perm(const FftDesc& d);

// Launchers (return hipError_t of the launch).
// Forward: real float64 rows [Nt] -> complex bins [N+1] of type TC.
hipError_t launch_rfft_fwd_f64(const FftDesc& d, const cpx<double>* tw,
                               const int* perm, const FftIo& io, int64_t nbatch,
                               hipStream_t s);
hipError_t launch_rfft_fwd_f32(const FftDesc& d, const cpx<float>* tw,
                               const int* perm, const FftIo& io, int64_t nbatch,
                               hipStream_t s);
// Inverse: complex bins (sum of nparts partials) -> first Nt real samples,
// times io.scale, written as float64.  in_f64 selects the input type.
hipError_t launch_rfft_inv_f64(const FftDesc& d, const cpx<double>* tw,
                               const int* perm, const FftIo& io, int64_t nbatch,
                               hipStream_t s);
hipError_t launch_rfft_inv_f32(const FftDesc& d, const cpx<float>* tw,
                               const int* perm, const FftIo& io, bool in_f64,
                               int64_t nbatch, hipStream_t s);

// ----------------------------------------------------------- block products
// Frequency-block layout: [nf][Nd][Nm], column p contiguous.
struct GemvShape {
  int64_t nf, Nd, Nm;
  int64_t nrhs;
  int n_pc;       // F only: number of column chunks (partial sums)
  int64_t pc_len; // F only: columns per chunk (multiple of 64)
};

// Mixed storage: 16-bit terms packed per complex entry, word 0 = hi (real
// part in the low half), word 1 = lo (absent for the hi-only tier).
constexpr int kScaleTile = 256;  // columns per scale sub-block
constexpr int kMaxPriorRadius = 32;  // largest half-width of the prior's window
enum class Fmt16 { FP16 = 0, BF16 = 1 };

// Candidate configurations of the product kernels (rows per wavefront for
// F, column groups per wavefront for F*, vector width).  `cfg` indexes the
// candidate table of the kernel family; 0 is the untuned default.
int gemv_candidates(bool mixed, p2o_op op);
int gemv_vec_width(bool mixed, bool lo, p2o_op op, int cfg);
int gemv_rows_per_wave(bool mixed, int cfg);

// F, float64: P[b][pc][k][s] = sum_{p in chunk pc} A[k][s][p] X[b][k][p]
hipError_t launch_gemv_rows_f64(const cpx<double>* A, const cpx<double>* X,
                                cpx<double>* P, const GemvShape& g, int cfg,
                                hipStream_t s);
// F*, float64: Y[b][k][p] = sum_s conj(A[k][s][p]) D[b][k][s]
hipError_t launch_gemv_cols_f64(const cpx<double>* A, const cpx<double>* D,
                                cpx<double>* Y, const GemvShape& g, int cfg,
                                hipStream_t s);
hipError_t launch_gemv_rows_mixed(const void* A, const float* scales,
                                  const cpx<float>* X, cpx<double>* P,
                                  const GemvShape& g, Fmt16 fmt, bool use_lo,
                                  int cfg, hipStream_t s);
hipError_t launch_gemv_cols_mixed(const void* A, const float* scales,
                                  const cpx<float>* D, cpx<float>* Y,
                                  const GemvShape& g, Fmt16 fmt, bool use_lo,
                                  int cfg, hipStream_t s);
// Quantise a float64 frequency chunk [nf][Nd][pc] into the packed layout at
// column offset p0 of [nf][Nd][Nm], with one scale per (k, 256-col tile).
hipError_t launch_quantise(const cpx<double>* chunk, int64_t nf, int64_t Nd,
                           int64_t Nm, int64_t p0, int64_t pc, void* A,
                           float* scales, Fmt16 fmt, bool use_lo,
                           hipStream_t s);

// Many right-hand sides on the float64 matrix cores (same operands and
// outputs as the row / column kernels above, all nrhs in passes of 64).
hipError_t launch_gemm_rows_f64(const cpx<double>* A, const cpx<double>* X,
                                cpx<double>* P, const GemvShape& g, hipStream_t s);
hipError_t launch_gemm_cols_f64(const cpx<double>* A, const cpx<double>* D,
                                cpx<double>* Y, const GemvShape& g, hipStream_t s);

// Many right-hand sides on the bfloat16 matrix cores (bfloat16 block
// storage).  Vector operands are the four bfloat16 planes per (rhs, k)
// written by the forward transform (FftIo::planes), each of
// n8 = roundup(n, 8) entries; F's planes carry the column scales.

hipError_t launch_gemm_rows_bf16(const void* A, const float* scales, const uint16_t* Xs,
                                 cpx<double>* P, const GemvShape& g, int64_t n8, bool lo,
                                 hipStream_t s);
hipError_t launch_gemm_cols_bf16(const void* A, const float* scales, const uint16_t* Ds,
                                 cpx<float>* Y, const GemvShape& g, int64_t nd8, bool lo,
                                 hipStream_t s);

// ---------------------------------------------------- batched instances
// One instance of a batched product: its frequency blocks, operands and
// shape, the kernel path it takes, and its range of work units in the
// batch (units are wavefront-sized pieces: a frequency and a tile of
// sensors or columns, with all of the instance's right-hand sides).
enum BatchPath : int { kPathVector = 0, kPathMatrix = 1 };
enum BatchClass : int { kClassF64 = 0, kClassMixedFp16 = 1, kClassMixedBf16 = 2, kClassFastBf16 = 3 };

struct BatchInst {
  const void* fhat;
  const float* scales;
  const void* in;      // transformed input, or its bfloat16 planes (matrix path, mixed)
  void* out;           // F: partial spectra, F*: transformed output
  GemvShape g;
  int64_t n8;          // bfloat16 plane pitch
  int64_t unit_begin;  // first unit of this instance in the batch
  int path;
};

// Configurations of the persistent kernel (batch.hip: vector-unit tiles);
// the work units of an instance depend on it (-1: a path the persistent
// kernel does not run, the bfloat16 matrix-core one).
int batch_config_count();
int64_t batch_units(BatchClass cls, p2o_op op, int path, const GemvShape& g, int cfg);
// One persistent launch over all instances' units (instances sorted by
// unit_begin, device array), in configuration `cfg`.
hipError_t launch_batch_product(BatchClass cls, p2o_op op, const BatchInst* insts, int n,
                                int64_t total_units, int cfg, hipStream_t s);

// ------------------------------------------------------- inversion kernels
// xh[(s - s0) ni + i - i0][k][p] (k < nf, p < Nm): spectra of the
// truncated, zero-padded adjoint unit vectors e_(i,s), s0 <= s < s0 + ns,
// i0 <= i < i0 + ni, times scale, from the time-domain rows A[(i Nd + s)][Nm]
// by a running sum over i.
hipError_t launch_unit_spectra(const double* A, int64_t Nd, int64_t Nm, int64_t nf, int64_t L,
                               const cpx<double>* tw, int64_t s0, int ns, int64_t i0, int64_t ni,
                               double scale, cpx<double>* xh, hipStream_t s);
hipError_t launch_add_diagonal(double* K, const double* v, int64_t n, hipStream_t s);
hipError_t launch_symmetrize(double* K, int64_t n, hipStream_t s);    // (K + K^T) / 2
hipError_t launch_mirror_lower(double* K, int64_t n, hipStream_t s);  // upper <- lower
hipError_t launch_mirror_upper(double* K, int64_t n, hipStream_t s);  // lower <- upper
hipError_t launch_set_diagonal(double* K, const double* d, int64_t n, hipStream_t s);
// Cholesky factor of K's lower triangle in place; scratch of
// cholesky_scratch_bytes(n) device bytes.
hipError_t launch_cholesky(double* K, int64_t n, int64_t* info_dev, double* scratch,
                           hipStream_t s);
size_t cholesky_scratch_bytes(int64_t n);
// Y[nrhs][n] <- K^{-1} Y with K's Cholesky factor in the lower triangle of K;
// scratch: cholesky_solve_scratch(n, nrhs) bytes of device memory (the
// forward solution and the inverted 64 x 64 diagonal blocks, two layouts).
hipError_t launch_cholesky_solve(const double* K, double* Y, double* scratch, int64_t n,
                                 int64_t nrhs, hipStream_t s);
size_t cholesky_solve_scratch(int64_t n, int64_t nrhs);
hipError_t launch_copy_diagonal(const double* K, double* d, int64_t n, hipStream_t s);
hipError_t launch_residual(const double* K, const double* diag, const double* D,
                           const double* X, double* R, double* rows, double* part, int64_t n,
                           int64_t nrhs, hipStream_t s);
hipError_t launch_axpy(double* y, const double* x, double a, int64_t n, hipStream_t s);
hipError_t launch_identity(double* X, int64_t n, hipStream_t s);  // X = I (n x n)
// Streaming-read ceiling: reads `bytes` (a multiple of 16) of `buf` once.
hipError_t launch_read_stream(const void* buf, int64_t bytes, double* sink, hipStream_t s);

// ------------------------------------------------- dense float64 (dense.hip)
// C[M x N] += alpha A[M x K] op(B), row-major; op(B) = B^T ([N x K]) when
// transb, else B ([K x N]); float64 matrix cores.
hipError_t launch_dgemm(bool transb, int64_t M, int64_t N, int64_t K, double alpha,
                        const double* A, int64_t lda, const double* B, int64_t ldb, double* C,
                        int64_t ldc, hipStream_t s);
// Lower triangle of C[n x n] += alpha A A^T (A [n x K]); entries above the
// diagonal untouched.
hipError_t launch_dsyrk_lower(int64_t n, int64_t K, double alpha, const double* A, int64_t lda,
                              double* C, int64_t ldc, hipStream_t s);
// C[M x N] = alpha A[M x K] B[N x K]^T, row-major, C overwritten (not read);
// with lower (M == N) only the lower triangle of C is written.
hipError_t launch_dgemm_nt_set(bool lower, int64_t M, int64_t N, int64_t K, double alpha,
                               const double* A, int64_t lda, const double* B, int64_t ldb,
                               double* C, int64_t ldc, hipStream_t s);
// In place prefix sums along the block diagonals of X [T P][T Q] (leading
// dimension ld): X[(a, i)][(b, j)] <- sum_{l <= min(a, b)} X[(a - l, i)][(b - l, j)];
// with lower (P == Q) only the lower triangle is read and written.
hipError_t launch_block_diag_scan(double* X, int64_t ld, int64_t T, int64_t P, int64_t Q,
                                  bool lower, hipStream_t s);
// Lower triangle of C[n x n] += alpha A B^T (A, B [n x K]); entries above
// the diagonal untouched.
hipError_t launch_dgemm_nt_lower(int64_t n, int64_t K, double alpha, const double* A,
                                 int64_t lda, const double* B, int64_t ldb, double* C,
                                 int64_t ldc, hipStream_t s);
// C[i][j] += alpha sum_k A[i][k] B[j][k] for i < M, j < N with j <= i only
// (C's origin on the diagonal of a symmetric matrix kept in its lower
// triangle; the entries above it are not touched).
hipError_t launch_dgemm_nt_lower_mask(int64_t M, int64_t N, int64_t K, double alpha,
                                      const double* A, int64_t lda, const double* B,
                                      int64_t ldb, double* C, int64_t ldc, hipStream_t s);
// Y[nrhs][n] <- K^{-1} Y with K's Cholesky factor in the lower triangle of K
// (no scratch; any nrhs, efficient from a few tens of right-hand sides on).
hipError_t launch_cholesky_solve_many(const double* K, double* Y, int64_t n, int64_t nrhs,
                                      hipStream_t s);
// Y = I (n x n) on entry; on return row r holds K^{-1} e_r in its entries
// c >= r (the upper triangle); the entries below the diagonal are not
// meaningful.  The many-right-hand-side sweeps restricted to the rows whose
// result is needed.
hipError_t launch_cholesky_inverse_upper(const double* K, double* Y, int64_t n, hipStream_t s);
// Y = I (n x n) on entry; on return the strict lower triangle of Y holds
// that of K^{-1} and diag[0 .. n) its diagonal (the upper triangle holds
// L^{-T}): the forward sweep only, then K^{-1} = L^{-T} L^{-1} as one
// symmetric product on the matrix cores.  Needs Y 16-byte aligned and
// n even, n >= 512 (cholesky_inverse_by_square_fits).
bool cholesky_inverse_by_square_fits(const double* Y, int64_t n);
hipError_t launch_cholesky_inverse_by_square(const double* K, double* Y, double* diag, int64_t n,
                                             hipStream_t s);
// Spatial prior covariance C on an nx x ny parameter grid (prior.hip):
// x[count][nx ny] <- C x in place; t1, t2 scratch of the same size; w the
// r + 1 window weights (device).
hipError_t launch_apply_prior(double* x, double* t1, double* t2, int64_t count, int64_t nx,
                              int64_t ny, const double* w, int r, double delta, hipStream_t s);
// q[r][rows] = Q[rows][cols] d[r][cols] for r < nrhs.
hipError_t launch_qoi_gemv(const double* Q, const double* D, double* q, int64_t rows,
                           int64_t cols, int64_t nrhs, hipStream_t s);

}  // namespace p2o

// ------------------------------------------------------------------ plan
struct p2o_plan_s {
  int64_t Nd = 0, Nm = 0, Nt = 0, L = 0, N = 0, nf = 0;
  p2o_prec prec = P2O_FP64;
  int device = 0;
  p2o::FftDesc fft{};
  p2o::cpx<double>* tw64 = nullptr;  // [L] exp(-2 pi i m / L)
  p2o::cpx<float>* tw32 = nullptr;
  int* perm = nullptr;               // [N] digit-reversal positions
  void* fhat = nullptr;              // frequency blocks
  float* scales = nullptr;           // [nf][ntiles] (mixed only)
  int64_t ntiles = 0;
  int64_t n_pc = 1;                  // F product: column chunks
  int64_t pc_len = 0;                // F product: columns per chunk
  int64_t cols_done = 0;             // setup progress
  int cfg[2] = {0, 0};               // product-kernel candidate per op
  int64_t mfma_min_rhs[2] = {8, 8};  // from this many RHS on, matrix cores (set per precision at setup)
  // spatial prior covariance C (p2o_set_prior); identity when prior_w is null
  double* prior_w = nullptr;         // [prior_r + 1] window weights (device)
  int64_t prior_nx = 0, prior_ny = 0;
  int prior_r = 0;
  double prior_delta = 0.0;
  int assembly = 0;                  // p2o_assembly of the inversion calls
  bool ready = false;
  void* scratch = nullptr;           // setup chunk staging (mixed)
  size_t scratch_bytes = 0;
  void* ws = nullptr;                // apply workspace
  size_t ws_bytes = 0;
  void* aux = nullptr;               // temporaries of the online posterior mean
  size_t aux_bytes = 0;
  bool timing = false;
  hipEvent_t ev_begin[2] = {nullptr, nullptr};
  hipEvent_t ev_end[2] = {nullptr, nullptr};
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[2];
  double kernel_ms[2] = {0, 0};
  int64_t kernel_launches[2] = {0, 0};
};
