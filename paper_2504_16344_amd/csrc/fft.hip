// Batched real transforms along the time axis for the block-circulant
// embedding of the p2o map (section "FFT-based Hessian matvecs", items
// (ii)-(iii)): the Toeplitz matrix is embedded in a block circulant of
// length L >= 2*Nt - 1 that the DFT block-diagonalises.
//
// Each work-group owns C adjacent columns (C a power of two) of one batch.
// A column is a length-L real series whose first Nt samples are read and
// whose remaining samples are the zero padding.  The series is packed as
// z[n] = x[2n] + i x[2n+1] (n < N = L/2) into LDS laid out [n][C] so that
// lanes with consecutive column indices touch consecutive LDS words, then
// transformed in place by a mixed-radix decimation-in-frequency FFT (every
// butterfly reads and writes the same R slots, so a stage needs no second
// buffer), leaving Z in digit-reversed order; `perm[k]` is the LDS row
// holding Z[k].  The even/odd split is undone while storing:
//   X[k] = (Z[k] + conj Z[N-k]) / 2 - i W_L^k (Z[k] - conj Z[N-k]) / 2.
// The inverse runs the same steps backwards and writes only the first Nt
// real samples, which is the truncation back to the Toeplitz block.
#include <cmath>
#include <type_traits>

#include "p2o_internal.h"

namespace p2o {

int64_t smooth_length(int64_t Nt) {
  for (int64_t L = 2 * Nt;; L += 2) {
    int64_t n = L;
    for (int p : {2, 3, 5, 7})
      while (n % p == 0) n /= p;
    if (n == 1) return L;
  }
}

bool make_fft_desc(int64_t Nt, FftDesc* d) {
  if (Nt < 1 || Nt > (1 << 22)) return false;
  const int64_t L = smooth_length(Nt);
  d->L = (int)L;
  d->N = (int)(L / 2);
  d->Nt = (int)Nt;
  d->nst = 0;
  int64_t n = d->N;
  auto push = [&](int r) {
    if (d->nst >= kMaxStages) return false;
    d->radix[d->nst++] = r;
    n /= r;
    return true;
  };
  while (n % 4 == 0)
    if (!push(4)) return false;
  while (n % 2 == 0)
    if (!push(2)) return false;
  for (int p : {3, 5, 7})
    while (n % p == 0)
      if (!push(p)) return false;
  return n == 1;
}

// Z[k] sits at LDS row sum_s u_s * (M_s / r_s), where k = u_1 + r_1 u_2 +
// r_1 r_2 u_3 + ... and M_s is the sub-transform length entering stage s.
std::vector<int> make_perm(const FftDesc& d) {
  std::vector<int> perm(d.N);
  for (int k = 0; k < d.N; ++k) {
    int kk = k, pos = 0, M = d.N;
    for (int s = 0; s < d.nst; ++s) {
      const int r = d.radix[s];
      M /= r;
      pos += (kk % r) * M;
      kk /= r;
    }
    perm[k] = pos;
  }
  return perm;
}

namespace {

constexpr int kLoadGroup = 8;  // loads in flight per thread in the load stages

// Work-groups go to the 8 XCDs round-robin by linear index (x fastest),
// and each XCD has its own L2.  This renumbers the grid's (column tile,
// batch) pairs in groups of 8 kXcdChunk: XCD x runs tiles
// x kXcdChunk .. x kXcdChunk + kXcdChunk - 1 of each group, so adjacent
// column tiles share an L2, where the partial cache lines of their output
// rows merge before they reach HBM, while the chip as a whole still sweeps
// one contiguous range.
// A bijection on 0 .. total-1 (a last partial group keeps its order).
constexpr int64_t kXcdCount = 8, kXcdChunk = 4;
__device__ __forceinline__ int64_t xcd_chunked(int64_t lin, int64_t total) {
  constexpr int64_t g = kXcdCount * kXcdChunk;
  if (lin >= total / g * g) return lin;
  const int64_t w = lin % g;
  return lin - w + (w % kXcdCount) * kXcdChunk + w / kXcdCount;
}

template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) {
  return {a.x + b.x, a.y + b.y};
}
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) {
  return {a.x - b.x, a.y - b.y};
}

// Length-R DFT y[u] = sum_q x[q] w^(q u); w = exp(-+2 pi i / R) is held in
// wr[1] (wr[m] = w^m, already conjugated for the inverse).
template <int R, typename T>
__device__ __forceinline__ void dft(const cpx<T>* x, cpx<T>* y,
                                    const cpx<T>* wr, bool inv) {
  if constexpr (R == 2) {
    y[0] = cadd(x[0], x[1]);
    y[1] = csub(x[0], x[1]);
  } else if constexpr (R == 4) {
    const cpx<T> a = cadd(x[0], x[2]), b = csub(x[0], x[2]);
    const cpx<T> c = cadd(x[1], x[3]), e = csub(x[1], x[3]);
    y[0] = cadd(a, c);
    y[2] = csub(a, c);
    // forward: y1 = b - i e, y3 = b + i e; inverse swaps the signs of i.
    const cpx<T> mie = {e.y, -e.x};  // -i e
    if (!inv) {
      y[1] = cadd(b, mie);
      y[3] = csub(b, mie);
    } else {
      y[1] = csub(b, mie);
      y[3] = cadd(b, mie);
    }
  } else {
#pragma unroll
    for (int u = 0; u < R; ++u) {
      cpx<T> acc = x[0];
#pragma unroll
      for (int q = 1; q < R; ++q) {
        const cpx<T> w = wr[(q * u) % R];
        acc.x += x[q].x * w.x - x[q].y * w.y;
        acc.y += x[q].x * w.y + x[q].y * w.x;
      }
      y[u] = acc;
    }
  }
}

// One decimation-in-frequency stage of radix R on every column.  Sub-arrays
// of length M start at multiples of M; butterfly (g, n') combines the R
// values at g*M + n' + q*M/R, applies the DFT over q and the twiddle
// W_M^(n' u) to output u, and writes output u back to slot g*M + n' + u*M/R.
template <int R, typename T>
__device__ __forceinline__ void dif_stage(cpx<T>* buf, int N, int M, int L,
                                          const cpx<T>* __restrict__ tw,
                                          bool inv, int logC, int tid,
                                          int nthr) {
  const int Mr = M / R;
  const int nbf = N / R;
  const int twstep = 2 * (N / M);  // W_M = W_L^(2N/M)
  const int C = 1 << logC;
  cpx<T> wr[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    wr[m] = tw[(L / R) * m];
    if (inv) wr[m].y = -wr[m].y;
  }
  const float rMr = 1.0f / (float)Mr;
  for (int idx = tid; idx < (nbf << logC); idx += nthr) {
    const int bf = idx >> logC;
    const int c = idx & (C - 1);
    int g = (int)((float)bf * rMr);  // bf / Mr: float estimate, one correction step
    if (g * Mr > bf) --g;
    else if ((g + 1) * Mr <= bf) ++g;
    const int np = bf - g * Mr;
    const int base = g * M + np;
    cpx<T> x[R], y[R];
#pragma unroll
    for (int q = 0; q < R; ++q) x[q] = buf[((base + q * Mr) << logC) + c];
    dft<R, T>(x, y, wr, inv);
    buf[(base << logC) + c] = y[0];
#pragma unroll
    for (int u = 1; u < R; ++u) {
      cpx<T> w = tw[twstep * np * u];  // index < L: np < M/R, u < R
      if (inv) w.y = -w.y;
      buf[((base + u * Mr) << logC) + c] = cmul(y[u], w);
    }
  }
}

template <typename T>
__device__ void dif_all_stages(cpx<T>* buf, const FftDesc& d,
                               const cpx<T>* __restrict__ tw, bool inv,
                               int logC, int tid, int nthr) {
  int M = d.N;
  for (int s = 0; s < d.nst; ++s) {
    __syncthreads();
    const int R = d.radix[s];
    switch (R) {
      case 4: dif_stage<4, T>(buf, d.N, M, d.L, tw, inv, logC, tid, nthr); break;
      case 2: dif_stage<2, T>(buf, d.N, M, d.L, tw, inv, logC, tid, nthr); break;
      case 3: dif_stage<3, T>(buf, d.N, M, d.L, tw, inv, logC, tid, nthr); break;
      case 5: dif_stage<5, T>(buf, d.N, M, d.L, tw, inv, logC, tid, nthr); break;
      default: dif_stage<7, T>(buf, d.N, M, d.L, tw, inv, logC, tid, nthr); break;
    }
    M /= R;
  }
  __syncthreads();
}

// Forward: x (float64 rows 0..Nt-1 of each column) -> X[k], k = 0..N.
// Twiddle table (L entries) and digit-reversal table (N entries) copied to
// LDS after the N x C transform tile; visible after the next barrier.
template <typename T>
__device__ __forceinline__ void tables_to_lds(cpx<T>* buf, const FftDesc& d,
                                              const cpx<T>* __restrict__ tw,
                                              const int* __restrict__ perm, int logC, int tid,
                                              int nthr) {
  cpx<T>* stw = buf + (d.N << logC);
  int* sperm = reinterpret_cast<int*>(stw + d.L);
  for (int i = tid; i < d.L; i += nthr) stw[i] = tw[i];
  for (int i = tid; i < d.N; i += nthr) sperm[i] = perm[i];
}

// Bin k of the real transform from the half-length complex transform in
// `buf`: X = a/2 - i w e / 2 with a = Zk + conj Zn, e = Zk - conj Zn.
template <typename T>
__device__ __forceinline__ cpx<T> split_bin(const cpx<T>* buf, const cpx<T>* __restrict__ tw,
                                            const int* __restrict__ perm, int N, int logC,
                                            int k, int c, T half) {
  const int k1 = (k == N) ? 0 : k;
  const int k2 = (k == 0) ? 0 : N - k;
  const cpx<T> zk = buf[(perm[k1] << logC) + c];
  const cpx<T> zn = buf[(perm[k2] << logC) + c];
  const cpx<T> w = tw[k];
  const T ar = zk.x + zn.x, ai = zk.y - zn.y;
  const T er = zk.x - zn.x, ei = zk.y + zn.y;
  const T wer = w.x * er - w.y * ei, wei = w.x * ei + w.y * er;
  return {half * (ar + wei), half * (ai - wer)};
}

// Bins written as four bfloat16 planes per (batch, bin): re hi, re lo,
// im hi, im lo (x = hi + lo, each rounded to nearest even), after the
// optional power-of-two column scale (exact).  The block holding the last
// columns also zeroes the padding columns ncols..n8-1.  In slot order
// (io.slot_order), column c of each 32-column chunk goes to position
// row_slot_position(c % 32) of that chunk.
__device__ __forceinline__ int64_t plane_pos(int slot_order, int64_t c) {
  if (slot_order == 0) return c;
  return (c & ~(int64_t)31) + row_slot_position(slot_order == 1, (int)(c & 31));
}

__device__ __forceinline__ void write_planes(const cpx<float>* buf, const cpx<float>* __restrict__ tw,
                                             const int* __restrict__ perm, const FftIo& io,
                                             int logC, int N, int ncol, int64_t c0, int64_t b,
                                             int tid, int nthr) {
  const int C = 1 << logC;
  uint16_t* __restrict__ pl = io.planes + b * io.nbins * 4 * io.n8;
  const int64_t tiles = (io.ncols + kScaleTile - 1) / kScaleTile;
  for (int idx = tid; idx < ((N + 1) << logC); idx += nthr) {
    const int k = idx >> logC, c = idx & (C - 1);
    if (c >= ncol) continue;
    cpx<float> v = split_bin<float>(buf, tw, perm, N, logC, k, c, 0.5f);
    if (io.col_scales) {
      const float sc = io.col_scales[k * tiles + (c0 + c) / kScaleTile];
      v.x *= sc;
      v.y *= sc;
    }
    const uint16_t rh = bf16_rne(v.x), ih = bf16_rne(v.y);
    const uint16_t rl = bf16_rne(v.x - __uint_as_float((uint32_t)rh << 16));
    const uint16_t il = bf16_rne(v.y - __uint_as_float((uint32_t)ih << 16));
    uint16_t* o = pl + (int64_t)k * 4 * io.n8 + plane_pos(io.slot_order, c0 + c);
    o[0] = rh;
    o[io.n8] = rl;
    o[2 * io.n8] = ih;
    o[3 * io.n8] = il;
  }
  if (c0 + C >= io.ncols) {
    const int pad = (int)(io.n8 - io.ncols);
    for (int idx = tid; idx < (N + 1) * 4 * pad; idx += nthr) {
      const int row = idx / pad;  // k * 4 + plane
      pl[(int64_t)row * io.n8 + plane_pos(io.slot_order, io.ncols + idx % pad)] = 0;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(512)
rfft_fwd_kernel(FftDesc d, const cpx<T>* __restrict__ tw_g,
                const int* __restrict__ perm_g, FftIo io, int logC) {
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  const int C = 1 << logC;
  const int tid = threadIdx.x, nthr = blockDim.x;
  // bfloat16 planes are written in 2-byte runs of C columns: their tiles
  // are renumbered so the partial lines merge in one L2 (measured: the other
  // outputs, full 128-byte runs, gain nothing and the inverse loses)
  const int64_t lin = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
  const int64_t wg = io.planes ? xcd_chunked(lin, (int64_t)gridDim.x * gridDim.y) : lin;
  const int64_t c0 = (wg % gridDim.x) << logC;
  const int64_t b = wg / gridDim.x;
  const double* __restrict__ in =
      static_cast<const double*>(io.in) + b * io.in_batch + c0;
  cpx<T>* __restrict__ out = static_cast<cpx<T>*>(io.out) + b * io.out_batch + c0;
  const int ncol = (int)min((int64_t)C, io.ncols - c0);
  const int N = d.N, Nt = d.Nt;
  tables_to_lds(buf, d, tw_g, perm_g, logC, tid, nthr);
  const cpx<T>* tw = buf + (N << logC);
  const int* perm = reinterpret_cast<const int*>(tw + d.L);

  // groups of kLoadGroup elements a thread: all their loads are issued
  // before the first LDS store, so their latencies overlap
  const int total = N << logC;
  for (int base = tid; base < total; base += kLoadGroup * nthr) {
    double re[kLoadGroup], im[kLoadGroup];
#pragma unroll
    for (int g = 0; g < kLoadGroup; ++g) {  // unconditional: clamped addresses
      const int idx = base + g * nthr;
      const int n = idx >> logC, c = idx & (C - 1);
      const int t0 = 2 * n;
      const bool ok = idx < total && c < ncol;
      re[g] = in[(ok && t0 < Nt) ? (int64_t)t0 * io.in_row + c : 0];
      im[g] = in[(ok && t0 + 1 < Nt) ? (int64_t)(t0 + 1) * io.in_row + c : 0];
    }
#pragma unroll
    for (int g = 0; g < kLoadGroup; ++g) {
      const int idx = base + g * nthr;
      const int n = idx >> logC, c = idx & (C - 1);
      const bool ok = idx < total && c < ncol;
      if (idx < total)
        buf[idx] = {(ok && 2 * n < Nt) ? (T)re[g] : (T)0, (ok && 2 * n + 1 < Nt) ? (T)im[g] : (T)0};
    }
  }
  dif_all_stages<T>(buf, d, tw, false, logC, tid, nthr);

  const T half = (T)0.5;
  if constexpr (std::is_same<T, float>::value) {
    if (io.planes) {
      write_planes(buf, tw, perm, io, logC, N, ncol, c0, b, tid, nthr);
      return;
    }
  }
  for (int idx = tid; idx < ((N + 1) << logC); idx += nthr) {
    const int k = idx >> logC, c = idx & (C - 1);
    if (c >= ncol) continue;
    out[(int64_t)k * io.out_row + c] = split_bin<T>(buf, tw, perm, N, logC, k, c, half);
  }
}

// Partial spectra 1 .. nparts-1 (F's column chunks) added, in a fixed
// order, to the first ones sa (bins k) and sb (bins N - k) of the
// G elements of a load group; one part at a time for all elements,
// so the loads of a part are in flight together.  Sums stay in TIN
// (float64 for F's partials) until the caller narrows them.
template <int G, typename TIN>
__device__ __forceinline__ void add_partials(const cpx<TIN>* __restrict__ in, const FftIo& io,
                                             int base, int total, int nthr, int logC, int ncol,
                                             int N, cpx<TIN> (&sa)[G], cpx<TIN> (&sb)[G]) {
  const int C = 1 << logC;
  for (int q = 1; q < io.nparts; ++q) {
    cpx<TIN> va[G], vb[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int idx = base + g * nthr;
      const bool ok = idx < total && (idx & (C - 1)) < ncol;
      const int k = ok ? idx >> logC : 0, c = ok ? idx & (C - 1) : 0;
      va[g] = in[q * io.part_stride + (int64_t)k * io.in_row + c];
      vb[g] = in[q * io.part_stride + (int64_t)(N - k) * io.in_row + c];
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      sa[g].x += va[g].x;
      sa[g].y += va[g].y;
      sb[g].x += vb[g].x;
      sb[g].y += vb[g].y;
    }
  }
}

// Z[k] = (Xa + conj Xb) + i conj(W_L^k) (Xa - conj Xb) with Xa = X[k],
// Xb = X[N-k]; the 1/2 of the split and the 1/N of the inverse DFT are
// folded into io.scale (= 1/L).
template <typename T>
__device__ __forceinline__ cpx<T> unsplit(cpx<T> xa, cpx<T> xb, cpx<T> w) {
  const T ar = xa.x + xb.x, ai = xa.y - xb.y;
  const T er = xa.x - xb.x, ei = xa.y + xb.y;
  // conj(w) * e
  const T cr = w.x * er + w.y * ei, ci = w.x * ei - w.y * er;
  return {ar - ci, ai + cr};
}

// Inverse: X[k], k = 0..N (sum of io.nparts partial spectra) -> first Nt
// real samples of the length-L inverse DFT, times io.scale, as float64.
template <typename TIN, typename T>
__global__ void __launch_bounds__(512)
rfft_inv_kernel(FftDesc d, const cpx<T>* __restrict__ tw_g,
                const int* __restrict__ perm_g, FftIo io, int logC) {
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  const int C = 1 << logC;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int64_t c0 = (int64_t)blockIdx.x << logC;
  const int64_t b = blockIdx.y;
  const cpx<TIN>* __restrict__ in =
      static_cast<const cpx<TIN>*>(io.in) + b * io.in_batch + c0;
  double* __restrict__ out = static_cast<double*>(io.out) + b * io.out_batch + c0;
  const int ncol = (int)min((int64_t)C, io.ncols - c0);
  const int N = d.N, Nt = d.Nt;
  const int half = N / 2;
  tables_to_lds(buf, d, tw_g, perm_g, logC, tid, nthr);
  const cpx<T>* tw = buf + (N << logC);
  const int* perm = reinterpret_cast<const int*>(tw + d.L);
  __syncthreads();  // the load stage below reads the twiddles

  // groups of G bin pairs a thread, loads first (see the forward); half the
  // group when any side is float64 keeps the kernel within 128 VGPRs (two
  // work-groups a CU)
  constexpr int G = (std::is_same<T, double>::value || std::is_same<TIN, double>::value)
                        ? kLoadGroup / 2
                        : kLoadGroup;
  const int total = (half + 1) << logC;
  for (int base = tid; base < total; base += G * nthr) {
    cpx<T> xa[G], xb[G];
    {
      cpx<TIN> sa[G], sb[G];
#pragma unroll
      for (int g = 0; g < G; ++g) {  // first partial spectrum
        const int idx = base + g * nthr;
        const bool ok = idx < total && (idx & (C - 1)) < ncol;
        const int k = ok ? idx >> logC : 0, c = ok ? idx & (C - 1) : 0;
        sa[g] = in[(int64_t)k * io.in_row + c];
        sb[g] = in[(int64_t)(N - k) * io.in_row + c];
      }
      if (io.nparts > 1) add_partials<G>(in, io, base, total, nthr, logC, ncol, N, sa, sb);
#pragma unroll
      for (int g = 0; g < G; ++g) {
        xa[g] = {(T)sa[g].x, (T)sa[g].y};
        xb[g] = {(T)sb[g].x, (T)sb[g].y};
      }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int idx = base + g * nthr;
      if (idx >= total) continue;
      const int k = idx >> logC, c = idx & (C - 1);
      if (c >= ncol) xa[g] = xb[g] = cpx<T>{0, 0};
      if (k == 0) {  // bins 0 and N of a real series are real
        xa[g].y = 0;
        xb[g].y = 0;
      }
      buf[(k << logC) + c] = unsplit(xa[g], xb[g], tw[k]);
      const int k2 = N - k;
      if (k2 != k && k2 < N) buf[(k2 << logC) + c] = unsplit(xb[g], xa[g], tw[k2]);
    }
  }
  dif_all_stages<T>(buf, d, tw, true, logC, tid, nthr);

  const double scale = io.scale;
  for (int idx = tid; idx < (Nt << logC); idx += nthr) {
    const int t = idx >> logC, c = idx & (C - 1);
    if (c >= ncol) continue;
    const cpx<T> z = buf[(perm[t >> 1] << logC) + c];
    out[(int64_t)t * io.out_row + c] = (double)((t & 1) ? z.y : z.x) * scale;
  }
}

// LDS bytes of one work-group: the N x C transform tile, then the twiddle
// and digit-reversal tables.
template <typename T>
size_t fft_lds_bytes(const FftDesc& d, int logC) {
  return ((size_t)d.N << logC) * sizeof(cpx<T>) + (size_t)d.L * sizeof(cpx<T>) +
         (size_t)d.N * sizeof(int);
}

// Columns per work-group: the largest power of two <= 64 whose LDS fits the
// budget (two work-groups per compute unit at 80 KB).
constexpr size_t kFftLdsBudget = 81920;
template <typename T>
int pick_logC(const FftDesc& d) {
  int logC = 0;
  while (logC < 6 && fft_lds_bytes<T>(d, logC + 1) <= kFftLdsBudget) ++logC;
  return logC;
}

template <typename T, typename K>
hipError_t launch_common(K kernel, const FftDesc& d, const cpx<T>* tw,
                         const int* perm, const FftIo& io, int64_t nbatch,
                         hipStream_t s) {
  if (nbatch < 1 || io.ncols < 1) return hipSuccess;
  if (nbatch > 65535) return hipErrorInvalidConfiguration;
  const int logC = pick_logC<T>(d);
  const size_t lds = fft_lds_bytes<T>(d, logC);
  if (lds > 163840) return hipErrorInvalidConfiguration;
  const int64_t gx = (io.ncols + (1 << logC) - 1) >> logC;
  if (gx > 0x7fffffff) return hipErrorInvalidConfiguration;
  const int threads = 512;
  hipLaunchKernelGGL(kernel, dim3((unsigned)gx, (unsigned)nbatch), dim3(threads),
                     lds, s, d, tw, perm, io, logC);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_rfft_fwd_f64(const FftDesc& d, const cpx<double>* tw,
                               const int* perm, const FftIo& io, int64_t nbatch,
                               hipStream_t s) {
  return launch_common<double>(rfft_fwd_kernel<double>, d, tw, perm, io, nbatch, s);
}
hipError_t launch_rfft_fwd_f32(const FftDesc& d, const cpx<float>* tw,
                               const int* perm, const FftIo& io, int64_t nbatch,
                               hipStream_t s) {
  return launch_common<float>(rfft_fwd_kernel<float>, d, tw, perm, io, nbatch, s);
}
hipError_t launch_rfft_inv_f64(const FftDesc& d, const cpx<double>* tw,
                               const int* perm, const FftIo& io, int64_t nbatch,
                               hipStream_t s) {
  return launch_common<double>(rfft_inv_kernel<double, double>, d, tw, perm, io,
                               nbatch, s);
}
hipError_t launch_rfft_inv_f32(const FftDesc& d, const cpx<float>* tw,
                               const int* perm, const FftIo& io, bool in_f64,
                               int64_t nbatch, hipStream_t s) {
  if (in_f64)
    return launch_common<float>(rfft_inv_kernel<double, float>, d, tw, perm, io,
                                nbatch, s);
  return launch_common<float>(rfft_inv_kernel<float, float>, d, tw, perm, io,
                              nbatch, s);
}

}  // namespace p2o
