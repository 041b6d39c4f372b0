// Data-space Hessian and posterior mean (section "Real-time Bayesian
// inference and prediction framework", Phases 2 and 4), float64 only:
//
//   K = Gamma_noise + F Gamma_prior F*,   formed one unit vector of data
//       space at a time (Phase 2), in batches of right-hand sides;
//   K = L L^T (blocked Cholesky), x = K^{-1} d with iterative refinement,
//   m = Gamma_prior F* x.
//
// F* of the unit vector e_(i,s) (sensor s, step i) is row s of F_(i-t) at
// step t <= i and zero after it, so the spectrum of its truncated,
// zero-padded series is W_L^(ik) sum_(u <= i) F_u[s, :] W_L^(-uk): a running
// sum over the shifts i, which gives the spectra of all Nt unit vectors of
// a sensor in one pass over the time-domain blocks (no transform per unit
// vector).  Those spectra then go through the F product and its inverse
// transform exactly as in an F apply.
#include <cmath>

#include "p2o_internal.h"

namespace p2o {
namespace {

constexpr int kNb = 64;  // Cholesky / triangular-solve block size

// ------------------------------------------------------------ assembly
// Spectra of the adjoint unit vectors e_(i,s), steps i0 <= i < i0 + ni of
// sensors s0 .. s0 + ns - 1 (batch b = (s - s0) ni + i - i0), already
// truncated to Nt steps and zero padded to L.  The time-domain F^* e_(i,s)
// is row s of F_(i-t) at step t <= i and zero after, so its spectrum is
//   xh_b[k][p] = scale W^(ik) P_i(k, p),  P_i = P_(i-1) + A[(i, s)][p] W^(-ik),
// a running sum over the steps (A: the time-domain rows, row i Nd + s =
// row s of F_i, with the prior's spatial factor already applied); the sum
// starts at step 0 whatever i0 is.  One thread per (k, p) walks the steps;
// tw holds W^m = exp(-2 pi i m / L).
__global__ void __launch_bounds__(256)
unit_spectra(const double* __restrict__ A, int64_t Nd, int64_t Nm, int64_t nf, int64_t L,
             const cpx<double>* __restrict__ tw, int64_t s0, int ns, int64_t i0, int64_t ni,
             double scale, cpx<double>* __restrict__ xh) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t k = blockIdx.y;
  if (p >= Nm) return;
  for (int j = 0; j < ns; ++j) {
    const double* __restrict__ a = A + (s0 + j) * Nm + p;
    cpx<double>* __restrict__ o = xh + ((int64_t)j * ni * nf + k) * Nm + p;
    double pr = 0.0, pi = 0.0;
    int64_t m = 0;  // i k mod L
    const int64_t iend = i0 + ni;
    constexpr int G = 8;  // steps whose block entries are loaded ahead
    for (int64_t ib = 0; ib < iend; ib += G) {
      double v[G];
#pragma unroll
      for (int g = 0; g < G; ++g) v[g] = a[min(ib + g, iend - 1) * Nd * Nm];  // clamped
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int64_t i = ib + g;
        if (i < iend) {
          const cpx<double> w = tw[m];
          pr += v[g] * w.x;  // v W^(-ik) = v conj(W^(ik))
          pi -= v[g] * w.y;
          if (i >= i0)
            o[(i - i0) * nf * Nm] = {scale * (w.x * pr - w.y * pi), scale * (w.x * pi + w.y * pr)};
          m += k;
          if (m >= L) m -= L;
        }
      }
    }
  }
}

__global__ void add_diagonal(double* __restrict__ K, const double* __restrict__ v,
                             int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) K[i * n + i] += v[i];
}

// K <- (K + K^T) / 2 (mirror 0), the lower triangle copied onto the upper
// one (mirror 1) or the upper onto the lower (mirror 2), on 32 x 32 tile
// pairs (I, J), I <= J.
__global__ void __launch_bounds__(256)
symmetrize(double* __restrict__ K, int64_t n, int64_t T, int mirror) {
  __shared__ double a[32][33], b[32][33];
  // linear index over the upper triangle of tiles: t -> (I, J), I <= J
  const int64_t t = blockIdx.x;
  int64_t J = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) / 2.0);
  while (J * (J + 1) / 2 > t) --J;
  while ((J + 1) * (J + 2) / 2 <= t) ++J;
  const int64_t I = t - J * (J + 1) / 2;
  (void)T;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int64_t gi = I * 32 + r, gj = J * 32 + tx;
    a[r][tx] = (gi < n && gj < n) ? K[gi * n + gj] : 0.0;   // tile (I, J)
    const int64_t hi = J * 32 + r, hj = I * 32 + tx;
    b[r][tx] = (hi < n && hj < n) ? K[hi * n + hj] : 0.0;   // tile (J, I)
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    // element (I*32+r, J*32+tx) pairs with (J*32+tx, I*32+r) = b[tx][r]
    const int64_t gi = I * 32 + r, gj = J * 32 + tx;
    const double v = mirror == 0   ? 0.5 * (a[r][tx] + b[tx][r])
                     : mirror == 1 ? (gj > gi ? b[tx][r] : a[r][tx])
                                   : (gj >= gi ? a[r][tx] : b[tx][r]);
    if (gi < n && gj < n) K[gi * n + gj] = v;
    const int64_t hi = J * 32 + tx, hj = I * 32 + r;
    if (hi < n && hj < n) K[hi * n + hj] = v;
  }
}

// ------------------------------------------------------------ Cholesky
// Diagonal step of the blocked Cholesky, once per block: the bs x bs
// diagonal block at (j0, j0) is factored in place (lower triangle) and its
// inverse W = L11^{-1} written to W[64][64] (row-major, zero above the
// diagonal and outside bs x bs), so that the column panel below becomes a
// matrix product L21 = A21 W^T on the matrix cores instead of a serial
// substitution per row.  One work-group of 256 threads, the block in LDS
// (padded with the identity, so padded entries stay finite), worked in
// 16 x 16 sub-blocks so the serial chains are 16 steps long:
//   for each sub-block column kb: wavefront 0 factors the diagonal
//   sub-block (lane r keeps row r in registers; column k goes through LDS)
//   and inverts it (lane c forms column c by substitution); then all
//   threads form the sub-blocks below it as products with that inverse and
//   update the trailing lower triangle;
//   then the off-diagonal sub-blocks of the inverse, block row by block row:
//   W_ij = -W_ii (sum_{j <= k < i} L_ik W_kj).
// The first non-positive (or NaN) pivot goes to *info.
// sqrt(d) and 1 / sqrt(d) for d > 0, for the factorisation's serial chain:
// the hardware reciprocal square root refined by three Newton steps on
// y = 1 / sqrt(d) (y <- y + y (1/2 - d y^2 / 2); each doubles the correct
// bits, enough from any start better than 2^-8), then g = d y corrected
// once by the residual d - g^2 (exact in a fused multiply-add): both within
// a unit or two in the last place, at the cost of a few multiply-adds
// instead of a rounded square root and a division.  NaN for d <= 0 (the
// caller reports the pivot).
__device__ __forceinline__ void sqrt_and_rsqrt(double d, double& g, double& y) {
  y = __builtin_amdgcn_rsq(d);
#pragma unroll
  for (int it = 0; it < 3; ++it) y = __builtin_fma(y, __builtin_fma(-0.5 * d * y, y, 0.5), y);
  g = d * y;
  g = __builtin_fma(0.5 * y, __builtin_fma(-g, g, d), g);
}

constexpr int kSb = 16;               // sub-block
constexpr int kNsb = kNb / kSb;       // sub-blocks per side

// 16 x 16 sub-block products on the float64 matrix cores
// (v_mfma_f64_16x16x4: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] of each 4-deep step; accumulator element q of lane l is
// C[l / 16 + 4 q][l % 16]).  Sub-blocks live in LDS arrays of row pitch
// kNb + 1; (r0, c0) is a sub-block's first row and column.
typedef double sub_d4 __attribute__((ext_vector_type(4)));
typedef double (*sub_lds)[kNb + 1];

__device__ __forceinline__ sub_d4 sub_load(sub_lds m, int r0, int c0, int lane) {
  sub_d4 c;
#pragma unroll
  for (int q = 0; q < 4; ++q) c[q] = m[r0 + (lane >> 4) + 4 * q][c0 + (lane & 15)];
  return c;
}

__device__ __forceinline__ void sub_store(sub_lds m, int r0, int c0, sub_d4 c, int lane) {
#pragma unroll
  for (int q = 0; q < 4; ++q) m[r0 + (lane >> 4) + 4 * q][c0 + (lane & 15)] = c[q];
}

// c += sign A B^T with A, B the 16 x 16 sub-blocks at (ar, ac) and (br, bc).
__device__ __forceinline__ void sub_mul_abt(sub_d4& c, sub_lds A, int ar, int ac, sub_lds B,
                                            int br, int bc, double sign, int lane) {
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int k = 4 * st + (lane >> 4);
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(sign * A[ar + (lane & 15)][ac + k],
                                             B[br + (lane & 15)][bc + k], c, 0, 0, 0);
  }
}

// c += sign A B with A, B the 16 x 16 sub-blocks at (ar, ac) and (br, bc).
__device__ __forceinline__ void sub_mul_ab(sub_d4& c, sub_lds A, int ar, int ac, sub_lds B,
                                           int br, int bc, double sign, int lane) {
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int k = 4 * st + (lane >> 4);
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(sign * A[ar + (lane & 15)][ac + k],
                                             B[br + k][bc + (lane & 15)], c, 0, 0, 0);
  }
}

__global__ void __launch_bounds__(256)
potrf_diag_inv(double* __restrict__ K, int64_t n, int64_t j0, int bs, double* __restrict__ W,
               int64_t* __restrict__ info) {
  __shared__ double a[kNb][kNb + 1];   // the block, then L
  __shared__ double w[kNb][kNb + 1];   // L^{-1}
  __shared__ double colk[kSb];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int idx = tid; idx < kNb * kNb; idx += 256) {
    const int u = idx / kNb, v = idx % kNb;
    const double x = K[(j0 + min(u, bs - 1)) * n + j0 + min(v, bs - 1)];
    a[u][v] = (u < bs && v < bs) ? (v <= u ? x : 0.0) : (u == v ? 1.0 : 0.0);
    w[u][v] = 0.0;
  }
  __syncthreads();
  for (int kb = 0; kb < kNsb; ++kb) {
    const int o = kb * kSb;
    if (wave == 0 && lane < kSb) {
      double r[kSb];     // row `lane` of the diagonal sub-block
      double dinv[kSb];  // 1 / L_kk, the same in every lane
#pragma unroll
      for (int j = 0; j < kSb; ++j) r[j] = a[o + lane][o + j];
#pragma unroll
      for (int k = 0; k < kSb; ++k) {
        // column k as updated so far, the pivot included, goes through LDS
        // once; every lane scales the entries it needs itself (the same
        // product the owning lane forms), so a step waits for one round trip
        colk[lane] = r[k];
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        const double d = colk[k];
        double col[kSb];
#pragma unroll
        for (int t = k + 1; t < kSb; ++t) col[t] = colk[t];
        if (lane == 0 && !(d > 0.0) && o + k < bs && *info < 0) *info = j0 + o + k;
        double piv, pinv;
        sqrt_and_rsqrt(d, piv, pinv);
        dinv[k] = pinv;
        r[k] = (lane == k) ? piv : (lane > k ? r[k] * pinv : r[k]);
        const double lik = (lane > k) ? r[k] : 0.0;
#pragma unroll
        for (int t = k + 1; t < kSb; ++t) r[t] -= lik * (col[t] * pinv);
        // this step's reads of colk precede the next step's write (one
        // wavefront: LDS accesses complete in issue order)
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      }
#pragma unroll
      for (int j = 0; j < kSb; ++j) a[o + lane][o + j] = (j <= lane) ? r[j] : 0.0;
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      // column `lane` of the sub-block's inverse, by a column sweep: x_k is
      // final once scaled by 1 / L_kk, then removed from the rows below
      // (independent updates, so the serial chain is one multiply and one
      // fused multiply-add a step)
      double x[kSb];
#pragma unroll
      for (int i = 0; i < kSb; ++i) x[i] = (i == lane) ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < kSb; ++k) {
        x[k] *= dinv[k];
#pragma unroll
        for (int i = k + 1; i < kSb; ++i) x[i] -= a[o + i][o + k] * x[k];
      }
#pragma unroll
      for (int i = 0; i < kSb; ++i) w[o + i][o + lane] = x[i];
    }
    __syncthreads();
    // panel: L_ik = A_ik W_kk^T for the sub-blocks i below, one a wavefront
    {
      const int i = kb + 1 + wave;
      if (i < kNsb) {
        sub_d4 acc = {0.0, 0.0, 0.0, 0.0};
        sub_mul_abt(acc, a, i * kSb, o, w, o, o, 1.0, lane);
        sub_store(a, i * kSb, o, acc, lane);
      }
    }
    __syncthreads();
    // trailing sub-blocks (i, j), kb < j <= i: A_ij -= L_ik L_jk^T (the upper
    // triangle of a diagonal sub-block takes garbage that the factorisation
    // never reads and overwrites with zeros).  The next diagonal sub-block
    // goes to wavefront 0, which factors it straight after, with no
    // work-group barrier in between: the others, dealt round-robin to
    // wavefronts 1..3, touch neither it nor its inverse, and the barrier
    // after that factorisation orders them before the next panel products.
    int t = 0;
    for (int i = kb + 1; i < kNsb; ++i)
      for (int jj = kb + 1; jj <= i; ++jj) {
        const int owner = (i == kb + 1 && jj == kb + 1) ? 0 : 1 + (t++ % 3);
        if (owner != wave) continue;
        sub_d4 acc = sub_load(a, i * kSb, jj * kSb, lane);
        sub_mul_abt(acc, a, i * kSb, o, a, jj * kSb, o, -1.0, lane);
        sub_store(a, i * kSb, jj * kSb, acc, lane);
      }
    // wavefront 0's lanes 0..15 read the sub-block its 64 lanes just stored
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  // off-diagonal sub-blocks of the inverse, block row by block row:
  // T_ij = sum_{j <= k < i} L_ik W_kj, parked where W_ij goes, then
  // W_ij = -W_ii T_ij; the j of a block row one a wavefront
  for (int i = 1; i < kNsb; ++i) {
    const int jj = wave;
    if (jj < i) {
      sub_d4 acc = {0.0, 0.0, 0.0, 0.0};
      for (int k = jj; k < i; ++k) sub_mul_ab(acc, a, i * kSb, k * kSb, w, k * kSb, jj * kSb, 1.0, lane);
      sub_store(w, i * kSb, jj * kSb, acc, lane);
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // T read back by other lanes
      __builtin_amdgcn_wave_barrier();
      sub_d4 acc2 = {0.0, 0.0, 0.0, 0.0};
      sub_mul_ab(acc2, w, i * kSb, i * kSb, w, i * kSb, jj * kSb, -1.0, lane);
      sub_store(w, i * kSb, jj * kSb, acc2, lane);
    }
    __syncthreads();
  }
  for (int idx = tid; idx < kNb * kNb; idx += 256) {
    const int u = idx / kNb, v = idx % kNb;
    if (u < bs && v <= u) K[(j0 + u) * n + j0 + v] = a[u][v];
    W[idx] = (u < bs && v < bs) ? w[u][v] : 0.0;
  }
}

// ------------------------------------------------------ triangular solves
// Y is [nrhs][n].  The diagonal blocks L_jj (64 x 64, the last one ragged)
// are inverted first, all in one launch, into two copies: column-major
// (for L_jj^{-1} z) and row-major (for L_jj^{-T} x).  Then one kernel per
// 64-block and direction (two blocks per kernel in the forward sweep, see
// trsv_fwd_pair): every work-group forms the block's solution as a
// 64 x 64 matrix-vector product with the inverse (no serial substitution on
// the sweep's critical path) and applies that block's update to its own
// share of the rest; work-group 0 stores the block's solution.  The block's
// right-hand side is read from one buffer and its solution written to
// another, so no work-group can see a block already solved by another:
//   forward  (L z = y): reads Y[:, blk], writes Z[:, blk], updates Y rows
//            i >= j1 (y_i -= L[i, blk] z_blk);
//   backward (L^T x = z): reads Z[:, blk], writes Y[:, blk], updates Z
//            entries c < j0 (z_c -= L[blk, c]^T x_blk).
constexpr int kFwdRows = 64;    // forward: rows updated per work-group
constexpr int kBwdCols = 256;   // backward: entries updated per work-group
constexpr int kQuarter = kNb / 4;  // inverse columns per wavefront in a product

__device__ __forceinline__ double wave_total(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One work-group (one wavefront) per diagonal block: lane c computes column
// c of L_jj^{-1} by forward substitution, x_c = 1 / l_cc and
// x_i = -(sum_{c <= k < i} l_ik x_k) / l_ii for i > c, with the column in
// registers (static indices: the loops are unrolled) and L_jj in LDS.  The
// block is padded to 64 with the identity so padded lanes stay finite;
// entries outside bs x bs are stored as zeros.
__global__ void __launch_bounds__(64)
invert_diag_blocks(const double* __restrict__ K, int64_t n, double* __restrict__ Dcm,
                   double* __restrict__ Drm) {
  __shared__ double a[kNb][kNb + 1];
  const int lane = threadIdx.x;
  const int64_t j0 = (int64_t)blockIdx.x * kNb;
  const int bs = (int)min<int64_t>(kNb, n - j0);
  const int cl = min(lane, bs - 1);
#pragma unroll 16
  for (int u = 0; u < kNb; ++u) {
    const double v = K[(j0 + min(u, bs - 1)) * n + j0 + cl];
    a[u][lane] = (u < bs && lane < bs) ? (lane <= u ? v : 0.0) : (lane == u ? 1.0 : 0.0);
  }
  __syncthreads();
  double x[kNb];
#pragma unroll
  for (int i = 0; i < kNb; ++i) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < i; ++k) s += a[i][k] * x[k];
    const double d = a[i][i];
    x[i] = (i < lane) ? 0.0 : (i == lane ? 1.0 / d : -s / d);
  }
  __syncthreads();  // a is reused for the transpose
#pragma unroll
  for (int i = 0; i < kNb; ++i) a[i][lane] = (i < bs && lane < bs) ? x[i] : 0.0;
  __syncthreads();
  double* cm = Dcm + (int64_t)blockIdx.x * kNb * kNb;
  double* rm = Drm + (int64_t)blockIdx.x * kNb * kNb;
#pragma unroll 16
  for (int u = 0; u < kNb; ++u) {
    rm[u * kNb + lane] = a[u][lane];  // (u, lane): row-major
    cm[u * kNb + lane] = a[lane][u];  // (lane, u): column-major
  }
}

// Both sweeps issue every global load of a right-hand side (the block's
// entries, the entries they update) and the wavefront's quarter of the
// inverse before the first barrier; the block's solution is the sum of four
// wavefront partial products (lane = output entry).
__global__ void __launch_bounds__(256)
trsv_fwd_step(const double* __restrict__ K, const double* __restrict__ Dcm,
              double* __restrict__ Y, double* __restrict__ Z, int64_t n, int64_t nrhs,
              int64_t j0, int bs) {
  __shared__ double part[4][kNb];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double* M = Dcm + (j0 / kNb) * kNb * kNb;
  double mv[kQuarter];  // mv[u] = (L_jj^{-1})[lane][wave kQuarter + u]
#pragma unroll
  for (int u = 0; u < kQuarter; ++u) mv[u] = M[(wave * kQuarter + u) * kNb + lane];
  const int64_t j1 = j0 + bs;
  const int64_t rbeg = j1 + (int64_t)blockIdx.x * kFwdRows;
  // this work-group's rows of the column panel, 16 a wavefront
  constexpr int kPer = kFwdRows / 4;
  double lr[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int64_t i = min(rbeg + wave * kPer + u, n - 1);
    lr[u] = K[i * n + j0 + min(lane, bs - 1)];
  }
  const int64_t my_row = min(rbeg + wave * kPer + min(lane, kPer - 1), n - 1);
  double yv[kQuarter];  // the block's right-hand side, this wavefront's quarter
#pragma unroll
  for (int u = 0; u < kQuarter; ++u) {
    const int k = wave * kQuarter + u;
    yv[u] = (k < bs) ? Y[j0 + k] : 0.0;
  }
  double yo = Y[my_row];  // right-hand side 0
  for (int64_t r = 0; r < nrhs; ++r) {
    double p = 0.0;
#pragma unroll
    for (int u = 0; u < kQuarter; ++u) p += mv[u] * yv[u];
    part[wave][lane] = p;
    __syncthreads();
    // zero at lanes >= bs (the inverse's padding), so the clamped panel
    // columns there add nothing
    const double zl = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
    if (blockIdx.x == 0 && wave == 0 && lane < bs) Z[r * n + j0 + lane] = zl;
    double mine = 0.0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const double s = wave_total(lr[u] * zl);
      if (lane == u) mine = s;
    }
    if (lane < kPer && rbeg + wave * kPer + lane < n) Y[r * n + my_row] = yo - mine;
    if (r + 1 < nrhs) {
#pragma unroll
      for (int u = 0; u < kQuarter; ++u) {
        const int k = wave * kQuarter + u;
        yv[u] = (k < bs) ? Y[(r + 1) * n + j0 + k] : 0.0;
      }
      yo = Y[(r + 1) * n + my_row];
    }
    __syncthreads();  // part is rewritten for the next right-hand side
  }
}

// Two blocks in one launch (half the launches of the forward sweep): block
// A = [j0, j0 + 64), always full, and block C = [j0 + 64, j0 + 64 + bs2).
// Every work-group forms z_A = L_AA^{-1} y_A, then y_C - L_CA z_A from the
// first rows of A's column panel and z_C = L_CC^{-1} of it, and updates its
// own rows below C with the columns of both blocks; work-group 0 stores z_A
// and z_C.  Y rows of C are consumed here and not written back (nothing
// reads them after this step).
__global__ void __launch_bounds__(256)
trsv_fwd_pair(const double* __restrict__ K, const double* __restrict__ Dcm,
              double* __restrict__ Y, double* __restrict__ Z, int64_t n, int64_t nrhs,
              int64_t j0, int bs2) {
  __shared__ double part[4][kNb];
  __shared__ double yc[kNb];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t jc = j0 + kNb;  // first row and column of block C
  const double* MA = Dcm + (j0 / kNb) * kNb * kNb;
  const double* MC = MA + kNb * kNb;
  double ma[kQuarter], mc[kQuarter], lb[kQuarter];
#pragma unroll
  for (int u = 0; u < kQuarter; ++u) {
    ma[u] = MA[(wave * kQuarter + u) * kNb + lane];
    mc[u] = MC[(wave * kQuarter + u) * kNb + lane];
    lb[u] = K[(jc + min(wave * kQuarter + u, bs2 - 1)) * n + j0 + lane];  // L_CA
  }
  const int64_t rbeg = jc + bs2 + (int64_t)blockIdx.x * kFwdRows;
  constexpr int kPer = kFwdRows / 4;
  double la[kPer], lc[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int64_t i = min(rbeg + wave * kPer + u, n - 1);
    la[u] = K[i * n + j0 + lane];
    lc[u] = K[i * n + jc + min(lane, bs2 - 1)];
  }
  const int64_t my_row = min(rbeg + wave * kPer + min(lane, kPer - 1), n - 1);
  const int crow = wave * kQuarter + min(lane, kQuarter - 1);  // lanes < 16: a row of C
  double yv[kQuarter];
#pragma unroll
  for (int u = 0; u < kQuarter; ++u) yv[u] = Y[j0 + wave * kQuarter + u];
  double ycv = (crow < bs2) ? Y[jc + crow] : 0.0;
  double yo = Y[my_row];  // right-hand side 0
  for (int64_t r = 0; r < nrhs; ++r) {
    double p = 0.0;
#pragma unroll
    for (int u = 0; u < kQuarter; ++u) p += ma[u] * yv[u];
    part[wave][lane] = p;
    __syncthreads();
    const double za = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
    if (blockIdx.x == 0 && wave == 0) Z[r * n + j0 + lane] = za;
    double mine = 0.0;
#pragma unroll
    for (int u = 0; u < kQuarter; ++u) {
      const double s = wave_total(lb[u] * za);
      if (lane == u) mine = s;
    }
    if (lane < kQuarter) yc[crow] = (crow < bs2) ? ycv - mine : 0.0;
    __syncthreads();  // yc complete; every read of part above is done
    p = 0.0;
#pragma unroll
    for (int u = 0; u < kQuarter; ++u) p += mc[u] * yc[wave * kQuarter + u];
    part[wave][lane] = p;
    __syncthreads();
    // zero at lanes >= bs2 (the inverse's padding)
    const double zc = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
    if (blockIdx.x == 0 && wave == 0 && lane < bs2) Z[r * n + jc + lane] = zc;
    mine = 0.0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const double s = wave_total(la[u] * za + lc[u] * zc);
      if (lane == u) mine = s;
    }
    if (lane < kPer && rbeg + wave * kPer + lane < n) Y[r * n + my_row] = yo - mine;
    if (r + 1 < nrhs) {
#pragma unroll
      for (int u = 0; u < kQuarter; ++u) yv[u] = Y[(r + 1) * n + j0 + wave * kQuarter + u];
      ycv = (crow < bs2) ? Y[(r + 1) * n + jc + crow] : 0.0;
      yo = Y[(r + 1) * n + my_row];
    }
    __syncthreads();  // part and yc are rewritten for the next right-hand side
  }
}

__global__ void __launch_bounds__(256)
trsv_bwd_step(const double* __restrict__ K, const double* __restrict__ Drm,
              double* __restrict__ Y, double* __restrict__ Z, int64_t n, int64_t nrhs,
              int64_t j0, int bs) {
  __shared__ double part[4][kNb];
  __shared__ double xb[kNb];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double* M = Drm + (j0 / kNb) * kNb * kNb;
  double mv[kQuarter];  // mv[u] = (L_jj^{-T})[lane][wave kQuarter + u]
#pragma unroll
  for (int u = 0; u < kQuarter; ++u) mv[u] = M[(wave * kQuarter + u) * kNb + lane];
  // this work-group's entries c < j0: column c of the block's row panel
  const int64_t c = (int64_t)blockIdx.x * kBwdCols + threadIdx.x;
  const bool own = c < j0;
  const int64_t cc = own ? c : 0;
  double lc[kNb];
#pragma unroll
  for (int t = 0; t < kNb; ++t) lc[t] = K[(j0 + min(t, bs - 1)) * n + cc];
  double zv[kQuarter];
#pragma unroll
  for (int u = 0; u < kQuarter; ++u) {
    const int k = wave * kQuarter + u;
    zv[u] = (k < bs) ? Z[j0 + k] : 0.0;
  }
  double zo = Z[cc];  // right-hand side 0
  for (int64_t r = 0; r < nrhs; ++r) {
    double p = 0.0;
#pragma unroll
    for (int u = 0; u < kQuarter; ++u) p += mv[u] * zv[u];
    part[wave][lane] = p;
    __syncthreads();
    if (wave == 0) {
      const double v = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
      xb[lane] = v;
      if (blockIdx.x == 0 && lane < bs) Y[r * n + j0 + lane] = v;
    }
    __syncthreads();
    double acc = 0.0;
#pragma unroll
    for (int t = 0; t < kNb; ++t) acc += (t < bs ? lc[t] : 0.0) * xb[t];
    if (own) Z[r * n + c] = zo - acc;
    if (r + 1 < nrhs) {
#pragma unroll
      for (int u = 0; u < kQuarter; ++u) {
        const int k = wave * kQuarter + u;
        zv[u] = (k < bs) ? Z[(r + 1) * n + j0 + k] : 0.0;
      }
      zo = Z[(r + 1) * n + cc];
    }
    __syncthreads();  // part and xb are rewritten for the next right-hand side
  }
}

// ------------------------------------------------- residual r = d - K x
// K x from the strict upper triangle U (untouched by the factorisation) and
// the saved diagonal: K x = U x + U^T x + diag x.
// U x: one wavefront per row, lanes over columns j > i.
__global__ void __launch_bounds__(256)
symv_upper_rows(const double* __restrict__ K, const double* __restrict__ X,
                double* __restrict__ out, int64_t n, int64_t nrhs) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  for (int64_t r = 0; r < nrhs; ++r) {
    double acc = 0.0;
    for (int64_t j = i + 1 + lane; j < n; j += 64) acc += K[i * n + j] * X[r * n + j];
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) out[r * n + i] = acc;
  }
}

// U^T x over a chunk of 1024 rows: part[c][r][i] = sum_{j in chunk, j < i} K[j][i] x[j].
__global__ void __launch_bounds__(256)
symv_upper_cols(const double* __restrict__ K, const double* __restrict__ X,
                double* __restrict__ part, int64_t n, int64_t nrhs) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t c = blockIdx.y;
  const int64_t jbeg = c * 1024, jend = min(jbeg + 1024, n);
  if (i >= n) return;
  for (int64_t r = 0; r < nrhs; ++r) {
    double acc = 0.0;
    const int64_t je = min(jend, i);
    for (int64_t j = jbeg; j < je; ++j) acc += K[j * n + i] * X[r * n + j];
    part[(c * nrhs + r) * n + i] = acc;
  }
}

__global__ void residual(const double* __restrict__ D, const double* __restrict__ X,
                         const double* __restrict__ diag, const double* __restrict__ rows,
                         const double* __restrict__ part, int nparts, double* __restrict__ R,
                         int64_t n, int64_t nrhs) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * nrhs) return;
  const int64_t i = idx % n;
  double kx = diag[i] * X[idx] + rows[idx];
  for (int c = 0; c < nparts; ++c) kx += part[(int64_t)c * n * nrhs + idx];
  R[idx] = D[idx] - kx;
}

__global__ void copy_diagonal(const double* __restrict__ K, double* __restrict__ d, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = K[i * n + i];
}

__global__ void set_diagonal(double* __restrict__ K, const double* __restrict__ d, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) K[i * n + i] = d[i];
}

// X = I (n x n, row-major): one thread per entry, grid-stride.
__global__ void identity(double* __restrict__ X, int64_t n) {
  const int64_t total = n * n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x)
    X[i] = (i / n == i % n) ? 1.0 : 0.0;
}

__global__ void axpy(double* __restrict__ y, const double* __restrict__ x, double a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}

unsigned grid1(int64_t n, int per = 256) {
  int64_t g = (n + per - 1) / per;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 1 << 30));
}

}  // namespace

hipError_t launch_unit_spectra(const double* A, int64_t Nd, int64_t Nm, int64_t nf, int64_t L,
                               const cpx<double>* tw, int64_t s0, int ns, int64_t i0, int64_t ni,
                               double scale, cpx<double>* xh, hipStream_t s) {
  if (Nm <= 0 || nf <= 0 || ns <= 0 || ni <= 0) return hipSuccess;
  if (nf > 65535) return hipErrorInvalidConfiguration;
  const dim3 grid((unsigned)((Nm + 255) / 256), (unsigned)nf);
  hipLaunchKernelGGL(unit_spectra, grid, dim3(256), 0, s, A, Nd, Nm, nf, L, tw, s0, ns, i0, ni,
                     scale, xh);
  return hipGetLastError();
}

hipError_t launch_add_diagonal(double* K, const double* v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(add_diagonal, dim3(grid1(n)), dim3(256), 0, s, K, v, n);
  return hipGetLastError();
}

hipError_t launch_symmetrize(double* K, int64_t n, hipStream_t s) {
  const int64_t T = (n + 31) / 32;
  const int64_t pairs = T * (T + 1) / 2;
  if (pairs > 0x7fffffff) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(symmetrize, dim3((unsigned)pairs), dim3(256), 0, s, K, n, T, 0);
  return hipGetLastError();
}

hipError_t launch_mirror_lower(double* K, int64_t n, hipStream_t s) {
  const int64_t T = (n + 31) / 32;
  const int64_t pairs = T * (T + 1) / 2;
  if (pairs > 0x7fffffff) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(symmetrize, dim3((unsigned)pairs), dim3(256), 0, s, K, n, T, 1);
  return hipGetLastError();
}

hipError_t launch_mirror_upper(double* K, int64_t n, hipStream_t s) {
  const int64_t T = (n + 31) / 32;
  const int64_t pairs = T * (T + 1) / 2;
  if (pairs > 0x7fffffff) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(symmetrize, dim3((unsigned)pairs), dim3(256), 0, s, K, n, T, 2);
  return hipGetLastError();
}

// Blocked right-looking Cholesky of the lower triangle, two levels: panels
// of kPanel columns, each factored as kNb-wide blocks: the diagonal block
// factored and inverted (potrf_diag_inv), the column below it formed in
// place as the product A21 L11^{-T} on the float64 matrix cores, and the
// panel's remaining columns updated by a masked product; after the panel
// one rank-kPanel update of the trailing
// lower triangle on the matrix cores.  The wide trailing update reads and
// writes the trailing matrix kPanel / kNb times less often than
// block-by-block updates.  scratch: cholesky_scratch_bytes(n).
constexpr int64_t kPanel = 512;
size_t cholesky_scratch_bytes(int64_t n) {
  (void)n;
  return (size_t)kNb * kNb * sizeof(double);  // the inverse of the current diagonal block
}

hipError_t launch_cholesky(double* K, int64_t n, int64_t* info_dev, double* scratch,
                           hipStream_t s) {
  double* W = scratch;  // [64][64] inverse of the diagonal block
  for (int64_t p0 = 0; p0 < n; p0 += kPanel) {
    const int64_t p1 = std::min(n, p0 + kPanel);
    for (int64_t j0 = p0; j0 < p1; j0 += kNb) {
      const int bs = (int)std::min<int64_t>(kNb, p1 - j0);
      const int64_t j1 = j0 + bs, m = n - j1;
      hipLaunchKernelGGL(potrf_diag_inv, dim3(1), dim3(256), 0, s, K, n, j0, bs, W, info_dev);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      if (m > 0) {
        // L21 = A21 W^T in place (rows j1 .. n-1 of the block's columns)
        e = launch_dgemm_nt_set(false, m, bs, bs, 1.0, K + j1 * n + j0, n, W, kNb,
                                K + j1 * n + j0, n, s);
        if (e != hipSuccess) return e;
        // the panel's columns j1 .. p1 - 1, rows j1 .. n - 1 (lower part only)
        e = launch_dgemm_nt_lower_mask(m, p1 - j1, bs, -1.0, K + j1 * n + j0, n,
                                       K + j1 * n + j0, n, K + j1 * n + j1, n, s);
        if (e != hipSuccess) return e;
      }
    }
    const int64_t mt = n - p1;
    if (mt > 0) {  // trailing lower triangle -= panel panel^T
      const hipError_t e = launch_dsyrk_lower(mt, p1 - p0, -1.0, K + p1 * n + p0, n,
                                              K + p1 * n + p1, n, s);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

// In place: Y <- (L L^T)^{-1} Y; scratch: cholesky_solve_scratch(n, nrhs)
// bytes (the forward solution, then both copies of the inverted diagonal
// blocks).
namespace {
int64_t solve_inverse_offset(int64_t n, int64_t nrhs) {  // doubles, 256-byte aligned
  return (n * nrhs + 31) / 32 * 32;
}
}  // namespace

hipError_t launch_cholesky_solve(const double* K, double* Y, double* scratch, int64_t n,
                                 int64_t nrhs, hipStream_t s) {
  const int64_t nb = (n + kNb - 1) / kNb;
  double* Z = scratch;
  double* Dcm = scratch + solve_inverse_offset(n, nrhs);
  double* Drm = Dcm + nb * kNb * kNb;
  hipLaunchKernelGGL(invert_diag_blocks, dim3((unsigned)nb), dim3(64), 0, s, K, n, Dcm, Drm);
  for (int64_t j0 = 0; j0 < n;) {
    const int64_t rest = n - j0;
    if (rest > kNb) {  // a full block and the next one
      const int bs2 = (int)std::min<int64_t>(kNb, rest - kNb);
      const int64_t m = rest - kNb - bs2;
      const unsigned g = (unsigned)std::max<int64_t>(1, (m + kFwdRows - 1) / kFwdRows);
      hipLaunchKernelGGL(trsv_fwd_pair, dim3(g), dim3(256), 0, s, K, Dcm, Y, Z, n, nrhs, j0,
                         bs2);
      j0 += kNb + bs2;
    } else {
      hipLaunchKernelGGL(trsv_fwd_step, dim3(1), dim3(256), 0, s, K, Dcm, Y, Z, n, nrhs, j0,
                         (int)rest);
      j0 = n;
    }
  }
  for (int64_t j0 = ((n - 1) / kNb) * kNb; j0 >= 0; j0 -= kNb) {
    const int bs = (int)std::min<int64_t>(kNb, n - j0);
    const unsigned g = (unsigned)std::max<int64_t>(1, (j0 + kBwdCols - 1) / kBwdCols);
    hipLaunchKernelGGL(trsv_bwd_step, dim3(g), dim3(256), 0, s, K, Drm, Y, Z, n, nrhs, j0, bs);
  }
  return hipGetLastError();
}

size_t cholesky_solve_scratch(int64_t n, int64_t nrhs) {
  const int64_t nb = (n + kNb - 1) / kNb;
  return (size_t)(solve_inverse_offset(n, nrhs) + 2 * nb * kNb * kNb) * sizeof(double);
}

hipError_t launch_set_diagonal(double* K, const double* d, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(set_diagonal, dim3(grid1(n)), dim3(256), 0, s, K, d, n);
  return hipGetLastError();
}

hipError_t launch_copy_diagonal(const double* K, double* d, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(copy_diagonal, dim3(grid1(n)), dim3(256), 0, s, K, d, n);
  return hipGetLastError();
}

// R = D - K X with K given by its strict upper triangle and `diag`.
// rows: [nrhs][n] scratch; part: [ceil(n/1024)][nrhs][n] scratch.
hipError_t launch_residual(const double* K, const double* diag, const double* D,
                           const double* X, double* R, double* rows, double* part, int64_t n,
                           int64_t nrhs, hipStream_t s) {
  hipLaunchKernelGGL(symv_upper_rows, dim3(grid1(n, 4)), dim3(256), 0, s, K, X, rows, n, nrhs);
  const int64_t nc = (n + 1023) / 1024;
  hipLaunchKernelGGL(symv_upper_cols, dim3(grid1(n), (unsigned)nc), dim3(256), 0, s, K, X,
                     part, n, nrhs);
  hipLaunchKernelGGL(residual, dim3(grid1(n * nrhs)), dim3(256), 0, s, D, X, diag, rows, part,
                     (int)nc, R, n, nrhs);
  return hipGetLastError();
}

hipError_t launch_identity(double* X, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(identity, dim3(std::min<unsigned>(grid1(n * n), 65536u)), dim3(256), 0, s,
                     X, n);
  return hipGetLastError();
}

hipError_t launch_axpy(double* y, const double* x, double a, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(axpy, dim3(grid1(n)), dim3(256), 0, s, y, x, a, n);
  return hipGetLastError();
}

}  // namespace p2o
