// Host runtime behind include/p2o.h: plan lifetime, setup (time-domain
// blocks -> frequency blocks), and p2o_apply, which chains
//   forward transform of x  ->  per-frequency block product  ->  inverse
//   transform with truncation to the first Nt steps
// on the caller's stream (section "FFT-based Hessian matvecs").
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <new>
#include <sstream>
#include <string>

#include "p2o_internal.h"

using namespace p2o;

namespace {

thread_local int g_last_hip = 0;

void load_tuned(p2o_plan_s* h);

p2o_status hip_fail(hipError_t e) {
  g_last_hip = (int)e;
  (void)hipGetLastError();  // do not leave the error for the next launch check
  return e == hipErrorOutOfMemory ? P2O_ENOMEM : P2O_EHIP;
}

#define TRY_HIP(expr)                         \
  do {                                        \
    const hipError_t e_ = (expr);             \
    if (e_ != hipSuccess) return hip_fail(e_); \
  } while (0)

#define TRY_ST(expr)                     \
  do {                                   \
    const p2o_status s_ = (expr);        \
    if (s_ != P2O_OK) return s_;         \
  } while (0)

bool valid_prec(int p) { return p >= P2O_FP64 && p <= P2O_MIXED_FP16; }
bool is_mixed(p2o_prec p) { return p != P2O_FP64; }
int64_t entry_bytes(p2o_prec p) {
  switch (p) {
    case P2O_FP64: return 16;
    case P2O_MIXED_FP16:
    case P2O_MIXED_BF16: return 8;
    case P2O_FAST_BF16: return 4;
  }
  return 0;
}
Fmt16 fmt_of(p2o_prec p) { return p == P2O_MIXED_FP16 ? Fmt16::FP16 : Fmt16::BF16; }
bool uses_lo(p2o_prec p) { return p != P2O_FAST_BF16; }

bool mul3(int64_t a, int64_t b, int64_t c, int64_t* r) {
  int64_t t;
  return !__builtin_mul_overflow(a, b, &t) && !__builtin_mul_overflow(t, c, r);
}

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

constexpr int kRowsPerWave = 4;        // must match the row kernels
constexpr int64_t kTargetWaves = 16384;

// Column chunking of the F product: enough wavefronts to fill the chip,
// chunks of at least 256 columns, chunk length a multiple of 64.  For the
// 16-bit tiers a chunk is also at most kMixedChainCols columns: the
// matrix-core products accumulate a chunk in float32 accumulators, whose
// rounding at each 32-column step is not free of bias (measured: an error
// growing linearly with the chunk length that adds up coherently in the
// first output steps), and the chunks' partial sums are added in float64.
constexpr int64_t kMixedChainCols = 4096;
void choose_chunks(p2o_plan_s* h, int64_t* n_pc, int64_t* pc_len) {
  const int64_t base = h->nf * ((h->Nd + kRowsPerWave - 1) / kRowsPerWave);
  int64_t n = std::max<int64_t>(1, (kTargetWaves + base - 1) / base);
  n = std::min<int64_t>(n, std::max<int64_t>(1, h->Nm / 256));
  if (is_mixed(h->prec))
    n = std::max<int64_t>(n, (h->Nm + kMixedChainCols - 1) / kMixedChainCols);
  int64_t len = (h->Nm + n - 1) / n;
  len = (len + 63) / 64 * 64;
  *pc_len = len;
  *n_pc = (h->Nm + len - 1) / len;
}

struct WsLayout {
  size_t a_off, b_off, c_off, total;
};

int64_t round8(int64_t n) { return (n + 7) / 8 * 8; }

// bfloat16 operand planes: F's are stored per 32-column chunk in the
// matrix-core slot order, F*'s in sensor order; both pitches are multiples
// of 32 (zero-padded), so every 32-entry chunk lies inside its plane row.
int64_t plane_pitch(const p2o_plan_s* h, p2o_op op) {
  return ((op == P2O_F ? h->Nm : h->Nd) + 31) / 32 * 32;
}
int plane_slot_order(const p2o_plan_s* h, p2o_op op) {
  return op == P2O_F ? (uses_lo(h->prec) ? 1 : 2) : 0;
}

// F : a = transformed x [nrhs][nf][Nm], b = partial spectra [nrhs][n_pc][nf][Nd]
// F*: a = transformed x [nrhs][nf][Nd], b = product      [nrhs][nf][Nm]
// mixed plans: c = a split into bfloat16 planes [nrhs][nf][4][plane_pitch]
// for the matrix-core product.
bool use_mfma(const p2o_plan_s* h, p2o_op op, int64_t nrhs) {
  if (h->mfma_min_rhs[op] <= 0 || nrhs < h->mfma_min_rhs[op]) return false;
  return h->prec == P2O_FP64 || h->prec == P2O_MIXED_BF16 || h->prec == P2O_FAST_BF16;
}

// bfloat16 matrix-core products: the forward transform writes the operand
// planes directly (no float32 spectra in between).
bool planes_path(const p2o_plan_s* h, p2o_op op, int64_t nrhs) {
  return is_mixed(h->prec) && use_mfma(h, op, nrhs);
}

WsLayout ws_layout(const p2o_plan_s* h, p2o_op op, int64_t nrhs) {
  const bool planes = planes_path(h, op, nrhs);
  const size_t vb = is_mixed(h->prec) ? 8 : 16;  // complex vector entry
  const int64_t nin = (op == P2O_F) ? h->Nm : h->Nd;
  const size_t a_bytes = planes ? 0 : (size_t)nrhs * h->nf * nin * vb;
  const size_t b_bytes = (op == P2O_F) ? (size_t)nrhs * h->n_pc * h->nf * h->Nd * 16
                                       : (size_t)nrhs * h->nf * h->Nm * vb;
  const size_t c_bytes = planes ? (size_t)nrhs * h->nf * 4 * plane_pitch(h, op) * 2 : 0;
  WsLayout w{};
  w.a_off = 0;
  w.b_off = align_up(a_bytes);
  w.c_off = w.b_off + align_up(b_bytes);
  w.total = w.c_off + align_up(c_bytes);
  return w;
}

p2o_status ensure_ws(p2o_plan_s* h, int64_t nrhs) {
  const size_t need = std::max(ws_layout(h, P2O_F, nrhs).total,
                               ws_layout(h, P2O_FADJ, nrhs).total);
  if (need <= h->ws_bytes) return P2O_OK;
  if (h->ws) {
    TRY_HIP(hipFree(h->ws));
    h->ws = nullptr;
    h->ws_bytes = 0;
  }
  TRY_HIP(hipMalloc(&h->ws, need));
  h->ws_bytes = need;
  return P2O_OK;
}

// The plan-owned temporaries of the online posterior mean grow on demand
// (the stream is drained before an older, smaller buffer is freed) and are
// kept for later calls.
p2o_status ensure_aux(p2o_plan_s* h, size_t need, hipStream_t s) {
  if (need <= h->aux_bytes) return P2O_OK;
  if (h->aux) {
    TRY_HIP(hipStreamSynchronize(s));
    TRY_HIP(hipFree(h->aux));
    h->aux = nullptr;
    h->aux_bytes = 0;
  }
  TRY_HIP(hipMalloc(&h->aux, need));
  h->aux_bytes = need;
  return P2O_OK;
}

void free_plan(p2o_plan_s* h) {
  if (!h) return;
  (void)hipFree(h->tw64);
  (void)hipFree(h->tw32);
  (void)hipFree(h->perm);
  (void)hipFree(h->fhat);
  (void)hipFree(h->scales);
  (void)hipFree(h->scratch);
  (void)hipFree(h->ws);
  (void)hipFree(h->aux);
  (void)hipFree(h->prior_w);
  for (int op = 0; op < 2; ++op) {
    for (auto& pr : h->pending[op]) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  }
  delete h;
}

p2o_status make_tables(p2o_plan_s* h) {
  const int L = h->fft.L;
  std::vector<cpx<double>> w64(L);
  std::vector<cpx<float>> w32(L);
  const long double two_pi = 6.283185307179586476925286766559005768L;
  for (int m = 0; m < L; ++m) {
    const long double a = two_pi * (long double)m / (long double)L;
    w64[m] = {(double)std::cos(a), (double)-std::sin(a)};
    w32[m] = {(float)w64[m].x, (float)w64[m].y};
  }
  const std::vector<int> perm = make_perm(h->fft);
  TRY_HIP(hipMalloc(&h->tw64, sizeof(cpx<double>) * L));
  TRY_HIP(hipMalloc(&h->tw32, sizeof(cpx<float>) * L));
  TRY_HIP(hipMalloc(&h->perm, sizeof(int) * perm.size()));
  TRY_HIP(hipMemcpy(h->tw64, w64.data(), sizeof(cpx<double>) * L, hipMemcpyHostToDevice));
  TRY_HIP(hipMemcpy(h->tw32, w32.data(), sizeof(cpx<float>) * L, hipMemcpyHostToDevice));
  TRY_HIP(hipMemcpy(h->perm, perm.data(), sizeof(int) * perm.size(), hipMemcpyHostToDevice));
  return P2O_OK;
}

p2o_status begin_impl(int64_t Nd, int64_t Nm, int64_t Nt, p2o_prec prec,
                      p2o_plan_s** out) {
  FftDesc d{};
  if (!make_fft_desc(Nt, &d)) return P2O_EUNSUPPORTED;
  // one column of the transform must fit the 64 KB LDS tile in float64;
  // the setup transform walks the sensors on the second grid axis
  if ((int64_t)d.N * 16 > 65536 || Nd > 65535) return P2O_EUNSUPPORTED;
  const int64_t nf = d.N + 1;
  int64_t bytes;
  if (!mul3(nf, Nd, Nm, &bytes) || __builtin_mul_overflow(bytes, entry_bytes(prec), &bytes))
    return P2O_ENOMEM;
  p2o_plan_s* h = new (std::nothrow) p2o_plan_s;
  if (!h) return P2O_ENOMEM;
  h->Nd = Nd;
  h->Nm = Nm;
  h->Nt = Nt;
  h->fft = d;
  h->L = d.L;
  h->N = d.N;
  h->nf = nf;
  h->prec = prec;
  h->ntiles = (Nm + kScaleTile - 1) / kScaleTile;
  choose_chunks(h, &h->n_pc, &h->pc_len);
  if (prec == P2O_MIXED_FP16) h->mfma_min_rhs[0] = h->mfma_min_rhs[1] = 0;
  hipError_t e = hipGetDevice(&h->device);
  if (e != hipSuccess) {
    free_plan(h);
    return hip_fail(e);
  }
  p2o_status st = make_tables(h);
  if (st == P2O_OK) {
    // 64 zero bytes past the last block: the matrix-core F* kernel's last
    // granule of a row may run up to 12 bytes past it (into dropped columns)
    e = hipMalloc(&h->fhat, (size_t)bytes + 64);
    if (e == hipSuccess) e = hipMemset(static_cast<char*>(h->fhat) + bytes, 0, 64);
    if (e != hipSuccess) st = hip_fail(e);
  }
  if (st == P2O_OK && is_mixed(prec)) {
    e = hipMalloc((void**)&h->scales, sizeof(float) * nf * h->ntiles);
    if (e != hipSuccess) st = hip_fail(e);
  }
  if (st != P2O_OK) {
    free_plan(h);
    return st;
  }
  *out = h;
  return P2O_OK;
}

// Transform columns p0..p1-1 of the time-domain blocks (row stride `ld`
// within one block row) into the stored frequency blocks.
p2o_status columns_impl(p2o_plan_s* h, const double* src, int64_t ld,
                        int64_t p0, int64_t p1, hipStream_t s) {
  const int64_t pc = p1 - p0;
  FftIo io{};
  io.in = src;
  io.ncols = pc;
  io.in_row = h->Nd * ld;
  io.in_batch = ld;
  io.nparts = 1;
  io.scale = 1.0;
  if (!is_mixed(h->prec)) {
    io.out = static_cast<cpx<double>*>(h->fhat) + p0;
    io.out_row = h->Nd * h->Nm;
    io.out_batch = h->Nm;
    TRY_HIP(launch_rfft_fwd_f64(h->fft, h->tw64, h->perm, io, h->Nd, s));
  } else {
    const size_t need = (size_t)h->nf * h->Nd * pc * sizeof(cpx<double>);
    if (need > h->scratch_bytes) {
      if (h->scratch) {
        TRY_HIP(hipStreamSynchronize(s));
        TRY_HIP(hipFree(h->scratch));
        h->scratch = nullptr;
        h->scratch_bytes = 0;
      }
      TRY_HIP(hipMalloc(&h->scratch, need));
      h->scratch_bytes = need;
    }
    io.out = h->scratch;
    io.out_row = h->Nd * pc;
    io.out_batch = pc;
    TRY_HIP(launch_rfft_fwd_f64(h->fft, h->tw64, h->perm, io, h->Nd, s));
    TRY_HIP(launch_quantise(static_cast<const cpx<double>*>(h->scratch), h->nf, h->Nd,
                            h->Nm, p0, pc, static_cast<uint2*>(h->fhat), h->scales,
                            fmt_of(h->prec), uses_lo(h->prec), s));
  }
  TRY_HIP(hipStreamSynchronize(s));
  h->cols_done += pc;
  return P2O_OK;
}

p2o_status end_impl(p2o_plan_s* h) {
  if (h->cols_done != h->Nm) return P2O_ESTATE;
  if (h->scratch) {
    TRY_HIP(hipFree(h->scratch));
    h->scratch = nullptr;
    h->scratch_bytes = 0;
  }
  load_tuned(h);
  h->ready = true;
  return P2O_OK;
}

bool cfg_valid(const p2o_plan_s* h, p2o_op op, int cfg) {
  if (cfg < 0 || cfg >= gemv_candidates(is_mixed(h->prec), op)) return false;
  const int v = gemv_vec_width(is_mixed(h->prec), uses_lo(h->prec), op, cfg);
  return h->Nm % v == 0;
}

// Candidate 0 of every table loads one entry per lane and is valid for
// any shape.
int default_cfg(const p2o_plan_s* h, p2o_op op) {
  (void)h;
  (void)op;
  return 0;
}

// The frequency-block product of `op` with candidate `cfg`; `a` is the
// transformed input, `b` the product (F: partial spectra), `c` scratch for
// the bfloat16 operand planes of the mixed matrix-core path.
hipError_t launch_product(const p2o_plan_s* h, p2o_op op, void* a, void* b, void* c,
                          int64_t nrhs, int cfg, hipStream_t s) {
  GemvShape g{h->nf, h->Nd, h->Nm, nrhs, (int)h->n_pc, h->pc_len};
  const bool mfma = use_mfma(h, op, nrhs);
  if (!is_mixed(h->prec)) {
    const auto* A = static_cast<const cpx<double>*>(h->fhat);
    if (mfma) {
      if (op == P2O_F)
        return launch_gemm_rows_f64(A, static_cast<const cpx<double>*>(a),
                                    static_cast<cpx<double>*>(b), g, s);
      return launch_gemm_cols_f64(A, static_cast<const cpx<double>*>(a),
                                  static_cast<cpx<double>*>(b), g, s);
    }
    if (op == P2O_F)
      return launch_gemv_rows_f64(A, static_cast<const cpx<double>*>(a),
                                  static_cast<cpx<double>*>(b), g, cfg, s);
    return launch_gemv_cols_f64(A, static_cast<const cpx<double>*>(a),
                                static_cast<cpx<double>*>(b), g, cfg, s);
  }
  const Fmt16 fmt = fmt_of(h->prec);
  const bool lo = uses_lo(h->prec);
  if (mfma) {  // operand planes written by the forward transform
    auto* planes = static_cast<uint16_t*>(c);
    if (op == P2O_F)
      return launch_gemm_rows_bf16(h->fhat, h->scales, planes, static_cast<cpx<double>*>(b),
                                   g, plane_pitch(h, op), lo, s);
    return launch_gemm_cols_bf16(h->fhat, h->scales, planes, static_cast<cpx<float>*>(b), g,
                                 plane_pitch(h, op), lo, s);
  }
  if (op == P2O_F)
    return launch_gemv_rows_mixed(h->fhat, h->scales, static_cast<const cpx<float>*>(a),
                                  static_cast<cpx<double>*>(b), g, fmt, lo, cfg, s);
  return launch_gemv_cols_mixed(h->fhat, h->scales, static_cast<const cpx<float>*>(a),
                                static_cast<cpx<float>*>(b), g, fmt, lo, cfg, s);
}

// ------------------------------------------------------------ tuning cache
// A flat JSON object {"key": index, ...}, one entry per line, in the file
// named by P2O_TUNE_CACHE.  Key: device architecture, precision, op and
// the plan shape.
std::string tune_key(const p2o_plan_s* h, p2o_op op) {
  hipDeviceProp_t prop{};
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) arch = prop.gcnArchName;
  std::ostringstream k;
  k << arch << "|prec" << (int)h->prec << "|op" << (int)op << "|" << h->Nd << "x" << h->Nm
    << "x" << h->Nt;
  return k.str();
}

std::map<std::string, int> read_cache(const char* path) {
  std::map<std::string, int> m;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    const size_t q0 = line.find('"');
    const size_t q1 = q0 == std::string::npos ? q0 : line.find('"', q0 + 1);
    const size_t c = q1 == std::string::npos ? q1 : line.find(':', q1);
    if (c == std::string::npos) continue;
    m[line.substr(q0 + 1, q1 - q0 - 1)] = std::atoi(line.c_str() + c + 1);
  }
  return m;
}

void write_cache(const char* path, const std::map<std::string, int>& m) {
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp);
    f << "{\n";
    size_t i = 0;
    for (const auto& kv : m)
      f << "  \"" << kv.first << "\": " << kv.second << (++i < m.size() ? ",\n" : "\n");
    f << "}\n";
  }
  std::rename(tmp.c_str(), path);
}

void load_tuned(p2o_plan_s* h) {
  const char* path = std::getenv("P2O_TUNE_CACHE");
  for (int op = 0; op < 2; ++op) {
    h->cfg[op] = default_cfg(h, (p2o_op)op);
    if (!path) continue;
    const auto m = read_cache(path);
    const auto it = m.find(tune_key(h, (p2o_op)op));
    if (it != m.end() && cfg_valid(h, (p2o_op)op, it->second)) h->cfg[op] = it->second;
  }
}

p2o_status timed_begin(p2o_plan_s* h, p2o_op op, hipStream_t s) {
  if (!h->timing) return P2O_OK;
  hipEvent_t a, b;
  TRY_HIP(hipEventCreate(&a));
  TRY_HIP(hipEventCreate(&b));
  h->pending[op].push_back({a, b});
  TRY_HIP(hipEventRecord(a, s));
  return P2O_OK;
}

p2o_status timed_end(p2o_plan_s* h, p2o_op op, hipStream_t s) {
  if (!h->timing) return P2O_OK;
  TRY_HIP(hipEventRecord(h->pending[op].back().second, s));
  return P2O_OK;
}

// Forward transform of x (float64, [nrhs][Nt][n_in]) into the workspace's
// input-spectrum region (float64 or float32 by plan precision).
hipError_t enqueue_forward(const p2o_plan_s* h, p2o_op op, const double* x, int64_t nrhs,
                           char* ws, hipStream_t s) {
  const WsLayout w = ws_layout(h, op, nrhs);
  const int64_t nin = (op == P2O_F) ? h->Nm : h->Nd;
  FftIo f{};
  f.in = x;
  f.out = ws + w.a_off;
  f.ncols = nin;
  f.in_row = nin;
  f.in_batch = h->Nt * nin;
  f.out_row = nin;
  f.out_batch = h->nf * nin;
  f.nparts = 1;
  f.scale = 1.0;
  if (planes_path(h, op, nrhs)) {
    f.out = nullptr;
    f.planes = reinterpret_cast<uint16_t*>(ws + w.c_off);
    f.n8 = plane_pitch(h, op);
    f.slot_order = plane_slot_order(h, op);
    f.nbins = h->nf;
    f.col_scales = (op == P2O_F) ? h->scales : nullptr;  // F's operand carries the scales
  }
  if (!is_mixed(h->prec)) return launch_rfft_fwd_f64(h->fft, h->tw64, h->perm, f, nrhs, s);
  return launch_rfft_fwd_f32(h->fft, h->tw32, h->perm, f, nrhs, s);
}

// Inverse transform of the product region into y ([nrhs][Nt][n_out]),
// summing F's partial spectra, truncating to Nt steps, times out_scale.
hipError_t enqueue_inverse(const p2o_plan_s* h, p2o_op op, double* y, int64_t nrhs,
                           double out_scale, const char* ws, hipStream_t s) {
  const WsLayout w = ws_layout(h, op, nrhs);
  const int64_t nout = (op == P2O_F) ? h->Nd : h->Nm;
  FftIo v{};
  v.in = ws + w.b_off;
  v.out = y;
  v.ncols = nout;
  v.in_row = nout;
  v.nparts = (op == P2O_F) ? (int)h->n_pc : 1;
  v.part_stride = h->nf * nout;
  v.in_batch = (int64_t)v.nparts * h->nf * nout;
  v.out_row = nout;
  v.out_batch = h->Nt * nout;
  v.scale = out_scale / (double)h->L;
  if (!is_mixed(h->prec)) return launch_rfft_inv_f64(h->fft, h->tw64, h->perm, v, nrhs, s);
  // F's partial spectra are float64 (combined in float64); F*'s product is float32
  return launch_rfft_inv_f32(h->fft, h->tw32, h->perm, v, op == P2O_F, nrhs, s);
}

// One apply on the workspace `ws` (ws_layout(h, op, nrhs).total bytes; the
// plan's own workspace unless a caller brings another), with the product
// kernel timed when the plan's timing is on and `timed`.
p2o_status apply_on(p2o_plan_s* h, p2o_op op, const double* x, double* y, int64_t nrhs,
                    char* ws, bool timed, hipStream_t s, double out_scale) {
  const WsLayout w = ws_layout(h, op, nrhs);
  TRY_HIP(enqueue_forward(h, op, x, nrhs, ws, s));
  if (timed) TRY_ST(timed_begin(h, op, s));
  TRY_HIP(launch_product(h, op, ws + w.a_off, ws + w.b_off, ws + w.c_off, nrhs, h->cfg[op], s));
  if (timed) TRY_ST(timed_end(h, op, s));
  TRY_HIP(enqueue_inverse(h, op, y, nrhs, out_scale, ws, s));
  return P2O_OK;
}

p2o_status apply_impl(p2o_plan_s* h, p2o_op op, const double* x, double* y, int64_t nrhs,
                      hipStream_t s, double out_scale = 1.0) {
  return apply_on(h, op, x, y, nrhs, static_cast<char*>(h->ws), true, s, out_scale);
}

}  // namespace

extern "C" {

p2o_status p2o_setup_begin(int64_t Nd, int64_t Nm, int64_t Nt, p2o_prec prec,
                           void* stream, p2o_handle* out) {
  (void)stream;
  if (!out) return P2O_EINVAL;
  *out = nullptr;
  if (Nd < 1 || Nm < 1 || Nt < 1 || !valid_prec(prec)) return P2O_EINVAL;
  return begin_impl(Nd, Nm, Nt, prec, out);
}

p2o_status p2o_setup_columns(p2o_handle h, const double* blocks_chunk,
                             int64_t p0, int64_t p1, void* stream) {
  if (!h || !blocks_chunk) return P2O_EINVAL;
  if (h->ready) return P2O_ESTATE;
  if (p0 < 0 || p1 <= p0 || p1 > h->Nm) return P2O_EINVAL;
  if (is_mixed(h->prec) &&
      (p0 % kScaleTile != 0 || (p1 % kScaleTile != 0 && p1 != h->Nm)))
    return P2O_EINVAL;
  return columns_impl(h, blocks_chunk, p1 - p0, p0, p1, (hipStream_t)stream);
}

p2o_status p2o_setup_end(p2o_handle h, void* stream) {
  (void)stream;
  if (!h) return P2O_EINVAL;
  if (h->ready) return P2O_ESTATE;
  return end_impl(h);
}

p2o_status p2o_setup(const double* blocks, int64_t Nd, int64_t Nm, int64_t Nt,
                     p2o_prec prec, void* stream, p2o_handle* out) {
  if (!out) return P2O_EINVAL;
  *out = nullptr;
  if (!blocks) return P2O_EINVAL;
  p2o_handle h = nullptr;
  p2o_status st = p2o_setup_begin(Nd, Nm, Nt, prec, stream, &h);
  if (st != P2O_OK) return st;
  // mixed precisions stage float64 spectra per chunk: keep that under ~1 GB
  int64_t chunk = Nm;
  if (is_mixed(prec)) {
    const int64_t per_col = h->nf * Nd * 16;
    chunk = std::max<int64_t>(1, ((int64_t)1 << 30) / per_col / kScaleTile) * kScaleTile;
  }
  for (int64_t p0 = 0; p0 < Nm && st == P2O_OK; p0 += chunk) {
    const int64_t p1 = std::min(Nm, p0 + chunk);
    st = columns_impl(h, blocks + p0, Nm, p0, p1, (hipStream_t)stream);
  }
  if (st == P2O_OK) st = end_impl(h);
  if (st != P2O_OK) {
    free_plan(h);
    return st;
  }
  *out = h;
  return P2O_OK;
}

p2o_status p2o_get_info(p2o_handle h, int64_t* Nd, int64_t* Nm, int64_t* Nt,
                        int64_t* L, int* prec) {
  if (!h) return P2O_EINVAL;
  if (Nd) *Nd = h->Nd;
  if (Nm) *Nm = h->Nm;
  if (Nt) *Nt = h->Nt;
  if (L) *L = h->L;
  if (prec) *prec = (int)h->prec;
  return P2O_OK;
}

p2o_status p2o_reserve(p2o_handle h, int64_t nrhs, void* stream) {
  if (!h || nrhs < 1) return P2O_EINVAL;
  if (h->ws) TRY_HIP(hipStreamSynchronize((hipStream_t)stream));
  return ensure_ws(h, nrhs);
}

p2o_status p2o_apply(p2o_handle h, p2o_op op, const double* x, double* y,
                     int64_t nrhs, void* stream) {
  if (!h || !x || !y || nrhs < 1 || nrhs > 65535) return P2O_EINVAL;
  if (op != P2O_F && op != P2O_FADJ) return P2O_EINVAL;
  if (!h->ready) return P2O_ESTATE;
  (void)hipGetLastError();  // launch checks below must see only our errors
  TRY_ST(ensure_ws(h, nrhs));
  hipStream_t s = (hipStream_t)stream;
  return apply_impl(h, op, x, y, nrhs, s);
}

void p2o_destroy(p2o_handle h) { free_plan(h); }

p2o_status p2o_read_bandwidth(const void* buf, int64_t bytes, double* sink, void* stream) {
  if (!buf || !sink || bytes < 16 || bytes % 16 != 0 || ((uintptr_t)buf & 15) != 0)
    return P2O_EINVAL;
  (void)hipGetLastError();
  TRY_HIP(launch_read_stream(buf, bytes, sink, (hipStream_t)stream));
  return P2O_OK;
}

const char* p2o_status_string(p2o_status s) {
  switch (s) {
    case P2O_OK: return "ok";
    case P2O_EINVAL: return "invalid argument";
    case P2O_ENOMEM: return "out of device memory or size overflow";
    case P2O_EHIP: return "HIP runtime error";
    case P2O_ENOTPD: return "matrix is not positive definite";
    case P2O_ESTATE: return "call out of order for this handle";
    case P2O_EUNSUPPORTED: return "unsupported request";
  }
  return "unknown status";
}

p2o_status p2o_last_hip_error(int* code) {
  if (!code) return P2O_EINVAL;
  *code = g_last_hip;
  return P2O_OK;
}

p2o_status p2o_set_prior(p2o_handle h, const p2o_prior_grid* prior, void* stream) {
  if (!h) return P2O_EINVAL;
  (void)hipGetLastError();
  if (!prior) {
    if (h->prior_w) {
      TRY_HIP(hipStreamSynchronize((hipStream_t)stream));
      TRY_HIP(hipFree(h->prior_w));
    }
    h->prior_w = nullptr;
    return P2O_OK;
  }
  if (prior->nx < 1 || prior->ny < 1 || prior->nx * prior->ny != h->Nm || prior->radius < 0 ||
      prior->radius > kMaxPriorRadius || !(prior->length > 0) || !(prior->delta > 0))
    return P2O_EINVAL;
  std::vector<double> w(prior->radius + 1);
  for (int a = 0; a <= prior->radius; ++a)
    w[a] = std::exp(-(double)a * a / (2.0 * prior->length * prior->length));
  double* dw = nullptr;
  TRY_HIP(hipMalloc(&dw, w.size() * sizeof(double)));
  hipError_t e = hipMemcpy(dw, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(dw);
    return hip_fail(e);
  }
  if (h->prior_w) {
    TRY_HIP(hipStreamSynchronize((hipStream_t)stream));
    TRY_HIP(hipFree(h->prior_w));
  }
  h->prior_w = dw;
  h->prior_nx = prior->nx;
  h->prior_ny = prior->ny;
  h->prior_r = prior->radius;
  h->prior_delta = prior->delta;
  return P2O_OK;
}

p2o_status p2o_set_kernel_timing(p2o_handle h, int enable) {
  if (!h) return P2O_EINVAL;
  h->timing = enable != 0;
  return P2O_OK;
}

p2o_status p2o_kernel_time(p2o_handle h, p2o_op op, double* total_ms,
                           int64_t* launches) {
  if (!h || (op != P2O_F && op != P2O_FADJ)) return P2O_EINVAL;
  for (auto& pr : h->pending[op]) {
    TRY_HIP(hipEventSynchronize(pr.second));
    float ms = 0.f;
    TRY_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
    h->kernel_ms[op] += ms;
    h->kernel_launches[op] += 1;
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  h->pending[op].clear();
  if (total_ms) *total_ms = h->kernel_ms[op];
  if (launches) *launches = h->kernel_launches[op];
  h->kernel_ms[op] = 0;
  h->kernel_launches[op] = 0;
  return P2O_OK;
}

p2o_status p2o_get_config(p2o_handle h, p2o_op op, int64_t* cfg, int64_t* n_candidates) {
  if (!h || (op != P2O_F && op != P2O_FADJ)) return P2O_EINVAL;
  if (cfg) *cfg = h->cfg[op];
  if (n_candidates) *n_candidates = gemv_candidates(is_mixed(h->prec), op);
  return P2O_OK;
}

p2o_status p2o_set_config(p2o_handle h, p2o_op op, int64_t cfg) {
  if (!h || (op != P2O_F && op != P2O_FADJ)) return P2O_EINVAL;
  if (cfg < 0 || cfg >= gemv_candidates(is_mixed(h->prec), op)) return P2O_EINVAL;
  if (!cfg_valid(h, op, (int)cfg)) return P2O_EUNSUPPORTED;
  h->cfg[op] = (int)cfg;
  return P2O_OK;
}

p2o_status p2o_set_mfma_threshold(p2o_handle h, p2o_op op, int64_t min_rhs) {
  if (!h || (op != P2O_F && op != P2O_FADJ)) return P2O_EINVAL;
  h->mfma_min_rhs[op] = min_rhs;
  return P2O_OK;
}

p2o_status p2o_autotune(p2o_handle h, p2o_op op, int reps, double* times_ms,
                        int64_t max_times, int64_t* chosen, void* stream) {
  if (!h || (op != P2O_F && op != P2O_FADJ) || reps < 1 || max_times < 0 ||
      (max_times > 0 && !times_ms))
    return P2O_EINVAL;
  if (!h->ready) return P2O_ESTATE;
  (void)hipGetLastError();
  hipStream_t s = (hipStream_t)stream;
  TRY_ST(ensure_ws(h, 1));
  const WsLayout w = ws_layout(h, op, 1);
  char* ws = static_cast<char*>(h->ws);
  TRY_HIP(hipMemsetAsync(ws + w.a_off, 0, w.b_off - w.a_off, s));
  const int n = gemv_candidates(is_mixed(h->prec), op);
  hipEvent_t e0, e1;
  TRY_HIP(hipEventCreate(&e0));
  TRY_HIP(hipEventCreate(&e1));
  int best = -1;
  float best_ms = 0.f;
  hipError_t err = hipSuccess;
  for (int c = 0; c < n && err == hipSuccess; ++c) {
    float ms = -1.f;
    if (cfg_valid(h, op, c)) {
      err = launch_product(h, op, ws + w.a_off, ws + w.b_off, ws + w.c_off, 1, c, s);  // warm-up
      if (err == hipSuccess) err = hipEventRecord(e0, s);
      for (int r = 0; r < reps && err == hipSuccess; ++r)
        err = launch_product(h, op, ws + w.a_off, ws + w.b_off, ws + w.c_off, 1, c, s);
      if (err == hipSuccess) err = hipEventRecord(e1, s);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
      ms /= reps;
      if (err == hipSuccess && (best < 0 || ms < best_ms)) {
        best = c;
        best_ms = ms;
      }
    }
    if (c < max_times) times_ms[c] = ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return hip_fail(err);
  h->cfg[op] = best;
  if (chosen) *chosen = best;
  if (const char* path = std::getenv("P2O_TUNE_CACHE")) {
    auto m = read_cache(path);
    m[tune_key(h, op)] = best;
    write_cache(path, m);
  }
  return P2O_OK;
}

}  // extern "C"

// ----------------------------------------------------------------- Phase 2/4
namespace {

// Device buffers of one inversion call, freed on every exit path.
struct DevBufs {
  std::vector<void*> ptrs;
  ~DevBufs() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  hipError_t alloc(void** out, size_t bytes) {
    const hipError_t e = hipMalloc(out, std::max<size_t>(bytes, 256));
    if (e == hipSuccess) ptrs.push_back(*out);
    return e;
  }
};

// Solves with K's Cholesky factor: the per-right-hand-side kernels for a
// few right-hand sides, the blocked matrix-core variant for many.
constexpr int64_t kSolveManyFrom = 16;
hipError_t cholesky_solve(const double* K, double* Y, double* scratch, int64_t n, int64_t nrhs,
                          hipStream_t s) {
  if (nrhs >= kSolveManyFrom) return launch_cholesky_solve_many(K, Y, n, nrhs, s);
  return launch_cholesky_solve(K, Y, scratch, n, nrhs, s);
}

bool same_time_grid(const p2o_plan_s* a, const p2o_plan_s* b) {
  return a->Nt == b->Nt && a->Nm == b->Nm && a->L == b->L;
}

// The time-domain blocks F_0 .. F_{Nt-1} of an FP64 plan, recovered from
// its frequency blocks by one inverse transform over all Nd Nm series
// (exact up to rounding: the spectra are those of the zero-padded series):
// out [Nt][Nd][Nm], i.e. the (Nt Nd) x Nm matrix whose row t Nd + s is row s
// of F_t.
hipError_t time_blocks(const p2o_plan_s* h, double* out, hipStream_t s) {
  FftIo io{};
  io.in = h->fhat;
  io.out = out;
  io.ncols = h->Nd * h->Nm;
  io.in_row = h->Nd * h->Nm;
  io.out_row = h->Nd * h->Nm;
  io.nparts = 1;
  io.scale = 1.0 / (double)h->L;
  return launch_rfft_inv_f64(h->fft, h->tw64, h->perm, io, 1, s);
}

// Bound on the temporaries of the unit-vector assembly: P2O_WORKSPACE_MB
// (MiB) when set to a positive integer, else 8 GiB.
size_t workspace_budget() {
  if (const char* v = std::getenv("P2O_WORKSPACE_MB")) {
    const long long mb = std::atoll(v);
    if (mb > 0) return (size_t)mb << 20;
  }
  return (size_t)8 << 30;
}

// Rows of hf's F applied after Gamma_prior times ha's F*: for every unit
// vector e_j of ha's data space (j = i Nd_a + s: sensor s, step i),
// row j of `out` (leading dimension ldo) receives F_hf Gamma_prior F_ha^* e_j
// ([Nt][Nd_f]).  The paper's Phase 2 matvecs on unit vectors: the
// spectrum of Gamma_prior F_ha^* e_j (truncated to Nt steps, zero padded)
// is generated directly, for all Nt steps of a sensor at once by a running
// sum over the steps (launch_unit_spectra, from ha's time-domain blocks with
// the prior's spatial factor applied), then hf's F product and inverse
// transform, whose output rows are scattered to j = i Nd_a + s.
p2o_status assemble_rows(p2o_plan_s* ha, p2o_plan_s* hf, const p2o_plan_s* hp,
                         double prior_var, double* out, int64_t ldo, hipStream_t s) {
  const int64_t Nt = hf->Nt, Nm = hf->Nm, nda = ha->Nd;
  const bool prior = hp->prior_w != nullptr;
  DevBufs bufs;
  void* a;  // ha's time-domain rows (i Nd_a + s), times C
  TRY_HIP(bufs.alloc(&a, (size_t)Nt * nda * Nm * 8));
  TRY_HIP(time_blocks(ha, static_cast<double*>(a), s));
  if (prior) {
    void *t1, *t2;
    TRY_HIP(bufs.alloc(&t1, (size_t)Nt * nda * Nm * 8));
    TRY_HIP(bufs.alloc(&t2, (size_t)Nt * nda * Nm * 8));
    TRY_HIP(launch_apply_prior(static_cast<double*>(a), static_cast<double*>(t1),
                               static_cast<double*>(t2), Nt * nda, hp->prior_nx, hp->prior_ny,
                               hp->prior_w, hp->prior_r, hp->prior_delta, s));
  }
  // unit vectors per pass: whole sensors when the temporary budget holds a
  // sensor's Nt steps, else runs of steps of one sensor
  const size_t per = (size_t)hf->nf * Nm * 16 + (size_t)hf->n_pc * hf->nf * hf->Nd * 16;
  const int64_t upp = std::max<int64_t>(1, std::min<int64_t>(65535, (int64_t)(workspace_budget() / per)));
  const int64_t ni = std::min(Nt, upp);
  const int64_t ns = ni < Nt ? 1 : std::max<int64_t>(1, std::min(nda, upp / Nt));
  void *xh, *parts;
  TRY_HIP(bufs.alloc(&xh, (size_t)ns * ni * hf->nf * Nm * 16));
  TRY_HIP(bufs.alloc(&parts, (size_t)ns * ni * hf->n_pc * hf->nf * hf->Nd * 16));
  const int64_t in_batch = hf->n_pc * hf->nf * hf->Nd;  // complex entries a unit vector
  for (int64_t s0 = 0; s0 < nda; s0 += ns) {
    const int nsb = (int)std::min(ns, nda - s0);
    for (int64_t i0 = 0; i0 < Nt; i0 += ni) {
      const int64_t nib = std::min(ni, Nt - i0);
      TRY_HIP(launch_unit_spectra(static_cast<const double*>(a), nda, Nm, hf->nf, hf->L,
                                  hf->tw64, s0, nsb, i0, nib, prior_var,
                                  static_cast<cpx<double>*>(xh), s));
      TRY_HIP(launch_product(hf, P2O_F, xh, parts, nullptr, nsb * nib, hf->cfg[P2O_F], s));
      for (int j = 0; j < nsb; ++j) {  // sensor s0 + j: step i to row i Nd_a + s0 + j
        FftIo o{};
        o.in = static_cast<const cpx<double>*>(parts) + (int64_t)j * nib * in_batch;
        o.out = out + (i0 * nda + s0 + j) * ldo;
        o.ncols = hf->Nd;
        o.in_row = hf->Nd;
        o.nparts = (int)hf->n_pc;
        o.part_stride = hf->nf * hf->Nd;
        o.in_batch = in_batch;
        o.out_row = hf->Nd;
        o.out_batch = nda * ldo;
        o.scale = 1.0 / (double)hf->L;
        TRY_HIP(launch_rfft_inv_f64(hf->fft, hf->tw64, hf->perm, o, nib, s));
      }
    }
  }
  // the scratch buffers are freed on return: finish their users first
  TRY_HIP(hipStreamSynchronize(s));
  return P2O_OK;
}

// The same rows as assemble_rows, from the Gram form of the product.  With
// the stacked time-domain blocks of ha (rows (a, j)) and of hf (rows (b, i)),
//   G = prior_var Fa C Ff^T,
// the entry of F_hf Gamma_prior F_ha^* coupling output (t, i) with unit
// vector (u, j) is the sum over l <= min(t, u) of G[(u - l, j)][(t - l, i)]
// (the block Toeplitz F_hf and F_ha share their time steps): one matrix-core
// GEMM and one pass of prefix sums along the block diagonals.  With `lower`
// (ha == hf: the product is symmetric) only the lower triangle of `out` is
// written.
p2o_status assemble_gram(const p2o_plan_s* ha, const p2o_plan_s* hf, const p2o_plan_s* hp,
                         double prior_var, double* out, int64_t ldo, bool lower,
                         hipStream_t s) {
  const int64_t na = ha->Nt * ha->Nd, nb = hf->Nt * hf->Nd, Nm = hf->Nm;
  const bool prior = hp->prior_w != nullptr;
  DevBufs bufs;
  void *fa, *ff = nullptr;
  TRY_HIP(bufs.alloc(&fa, (size_t)na * Nm * 8));
  TRY_HIP(time_blocks(ha, static_cast<double*>(fa), s));
  if (hf == ha && !prior) {
    ff = fa;
  } else {
    TRY_HIP(bufs.alloc(&ff, (size_t)nb * Nm * 8));
    if (hf == ha)
      TRY_HIP(hipMemcpyAsync(ff, fa, (size_t)nb * Nm * 8, hipMemcpyDeviceToDevice, s));
    else
      TRY_HIP(time_blocks(hf, static_cast<double*>(ff), s));
  }
  if (prior) {  // Ff <- Ff C (C symmetric): C on every row
    void *t1, *t2;
    TRY_HIP(bufs.alloc(&t1, (size_t)nb * Nm * 8));
    TRY_HIP(bufs.alloc(&t2, (size_t)nb * Nm * 8));
    TRY_HIP(launch_apply_prior(static_cast<double*>(ff), static_cast<double*>(t1),
                               static_cast<double*>(t2), nb, hp->prior_nx, hp->prior_ny,
                               hp->prior_w, hp->prior_r, hp->prior_delta, s));
  }
  TRY_HIP(launch_dgemm_nt_set(lower, na, nb, Nm, prior_var, static_cast<const double*>(fa), Nm,
                              static_cast<const double*>(ff), Nm, out, ldo, s));
  TRY_HIP(launch_block_diag_scan(out, ldo, ha->Nt, ha->Nd, hf->Nd, lower, s));
  // the scratch buffers are freed on return: finish their users first
  TRY_HIP(hipStreamSynchronize(s));
  return P2O_OK;
}

}  // namespace

extern "C" {

p2o_status p2o_hessian_assemble(p2o_handle h, double prior_var,
                                const double* noise_var, double* K,
                                void* stream) {
  if (!h || !noise_var || !K) return P2O_EINVAL;
  if (!h->ready) return P2O_ESTATE;
  if (h->prec != P2O_FP64) return P2O_EUNSUPPORTED;
  (void)hipGetLastError();
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = h->Nt * h->Nd;
  if (h->assembly == P2O_ASSEMBLE_GRAM) {
    TRY_ST(assemble_gram(h, h, h, prior_var, K, n, true, s));
    TRY_HIP(launch_add_diagonal(K, noise_var, n, s));
    TRY_HIP(launch_mirror_lower(K, n, s));
  } else {
    TRY_ST(assemble_rows(h, h, h, prior_var, K, n, s));
    TRY_HIP(launch_add_diagonal(K, noise_var, n, s));
    TRY_HIP(launch_symmetrize(K, n, s));
  }
  TRY_HIP(hipStreamSynchronize(s));
  return P2O_OK;
}

p2o_status p2o_set_assembly(p2o_handle h, p2o_assembly method) {
  if (!h || (method != P2O_ASSEMBLE_MATVEC && method != P2O_ASSEMBLE_GRAM)) return P2O_EINVAL;
  h->assembly = method;
  return P2O_OK;
}

p2o_status p2o_qoi_precompute(p2o_handle hF, p2o_handle hq, const double* Kfac,
                              double prior_var, double* Q, double* Gq, void* stream) {
  if (!hF || !hq || !Kfac || !Q || !Gq) return P2O_EINVAL;
  if (!hF->ready || !hq->ready) return P2O_ESTATE;
  if (hF->prec != P2O_FP64 || hq->prec != P2O_FP64) return P2O_EUNSUPPORTED;
  if (!same_time_grid(hF, hq)) return P2O_EINVAL;
  (void)hipGetLastError();
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = hF->Nt * hF->Nd, nq = hq->Nt * hq->Nd;
  DevBufs bufs;
  void* bt;  // rows j: F Gp Fq^* e_j (columns of B = F Gp Fq^*)
  TRY_HIP(bufs.alloc(&bt, (size_t)nq * n * 8));
  double* Bt = static_cast<double*>(bt);
  const bool gram = hF->assembly == P2O_ASSEMBLE_GRAM;
  if (gram) {
    TRY_ST(assemble_gram(hq, hF, hF, prior_var, Bt, n, false, s));
    TRY_ST(assemble_gram(hq, hq, hF, prior_var, Gq, nq, true, s));  // lower triangle
  } else {
    TRY_ST(assemble_rows(hq, hF, hF, prior_var, Bt, n, s));
    TRY_ST(assemble_rows(hq, hq, hF, prior_var, Gq, nq, s));  // Fq Gp Fq^*
  }
  // Q = Fq Gp F^* K^{-1} = (K^{-1} B)^T: row j of Q is K^{-1} (column j of B)
  TRY_HIP(hipMemcpyAsync(Q, Bt, (size_t)nq * n * 8, hipMemcpyDeviceToDevice, s));
  TRY_HIP(launch_cholesky_solve_many(Kfac, Q, n, nq, s));
  // Gq = Fq Gp Fq^* - Q B (symmetric: lower triangle, then mirrored)
  TRY_HIP(launch_dgemm_nt_lower(nq, n, -1.0, Q, n, Bt, n, Gq, nq, s));
  TRY_HIP(launch_mirror_lower(Gq, nq, s));
  TRY_HIP(hipStreamSynchronize(s));
  return P2O_OK;
}

p2o_status p2o_qoi_predict(const double* Q, int64_t nq, int64_t n, const double* d, double* q,
                           int64_t nrhs, void* stream) {
  if (!Q || !d || !q || nq < 1 || n < 1 || nrhs < 1) return P2O_EINVAL;
  (void)hipGetLastError();
  TRY_HIP(launch_qoi_gemv(Q, d, q, nq, n, nrhs, (hipStream_t)stream));
  return P2O_OK;
}

p2o_status p2o_posterior_solve(p2o_handle h, double* K, const double* d,
                               double* m_out, int64_t nrhs, double prior_var,
                               int refine_steps, int64_t* failed_pivot,
                               void* stream) {
  if (!h || !K || !d || !m_out || nrhs < 1 || nrhs > 65535 || refine_steps < 0)
    return P2O_EINVAL;
  if (!h->ready) return P2O_ESTATE;
  if (h->prec != P2O_FP64) return P2O_EUNSUPPORTED;
  (void)hipGetLastError();
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = h->Nt * h->Nd;
  const int64_t nchunks = (n + 1023) / 1024;
  DevBufs bufs;
  void *diag, *info, *x, *r, *rows, *psolve, *psymv, *pchol;
  TRY_HIP(bufs.alloc(&pchol, cholesky_scratch_bytes(n)));
  TRY_HIP(bufs.alloc(&diag, n * 8));
  TRY_HIP(bufs.alloc(&info, 8));
  TRY_HIP(bufs.alloc(&x, (size_t)nrhs * n * 8));
  TRY_HIP(bufs.alloc(&r, (size_t)nrhs * n * 8));
  TRY_HIP(bufs.alloc(&rows, (size_t)nrhs * n * 8));
  TRY_HIP(bufs.alloc(&psolve, cholesky_solve_scratch(n, nrhs)));
  TRY_HIP(bufs.alloc(&psymv, (size_t)nchunks * nrhs * n * 8));
  const int64_t minus_one = -1;
  TRY_HIP(hipMemcpyAsync(info, &minus_one, 8, hipMemcpyHostToDevice, s));
  TRY_HIP(launch_copy_diagonal(K, static_cast<double*>(diag), n, s));
  TRY_HIP(launch_cholesky(K, n, static_cast<int64_t*>(info), static_cast<double*>(pchol), s));
  int64_t piv = -1;
  TRY_HIP(hipMemcpyAsync(&piv, info, 8, hipMemcpyDeviceToHost, s));
  TRY_HIP(hipStreamSynchronize(s));
  if (piv >= 0) {
    if (failed_pivot) *failed_pivot = piv;
    return P2O_ENOTPD;
  }
  double* X = static_cast<double*>(x);
  double* Rr = static_cast<double*>(r);
  TRY_HIP(hipMemcpyAsync(X, d, (size_t)nrhs * n * 8, hipMemcpyDeviceToDevice, s));
  TRY_HIP(cholesky_solve(K, X, static_cast<double*>(psolve), n, nrhs, s));
  for (int it = 0; it < refine_steps; ++it) {
    TRY_HIP(launch_residual(K, static_cast<const double*>(diag), d, X, Rr,
                            static_cast<double*>(rows), static_cast<double*>(psymv), n, nrhs, s));
    TRY_HIP(cholesky_solve(K, Rr, static_cast<double*>(psolve), n, nrhs, s));
    TRY_HIP(launch_axpy(X, Rr, 1.0, nrhs * n, s));
  }
  TRY_ST(ensure_ws(h, nrhs));
  TRY_ST(apply_impl(h, P2O_FADJ, X, m_out, nrhs, s, prior_var));
  if (h->prior_w) {  // Gamma_prior = prior_var (I (x) C)
    void *t1, *t2;
    TRY_HIP(bufs.alloc(&t1, (size_t)nrhs * h->Nt * h->Nm * 8));
    TRY_HIP(bufs.alloc(&t2, (size_t)nrhs * h->Nt * h->Nm * 8));
    TRY_HIP(launch_apply_prior(m_out, static_cast<double*>(t1), static_cast<double*>(t2),
                               nrhs * h->Nt, h->prior_nx, h->prior_ny, h->prior_w, h->prior_r,
                               h->prior_delta, s));
  }
  TRY_HIP(hipStreamSynchronize(s));
  return P2O_OK;
}

p2o_status p2o_posterior_mean(p2o_handle h, const double* Kfac, const double* d, double* m_out,
                              int64_t nrhs, double prior_var, void* stream) {
  if (!h || !Kfac || !d || !m_out || nrhs < 1 || nrhs > 65535) return P2O_EINVAL;
  if (!h->ready) return P2O_ESTATE;
  if (h->prec != P2O_FP64) return P2O_EUNSUPPORTED;
  (void)hipGetLastError();
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = h->Nt * h->Nd;
  // plan-owned: [x: nrhs n][solve scratch][prior temporaries: 2 nrhs Nt Nm]
  const size_t x_bytes = align_up((size_t)nrhs * n * 8);
  const size_t solve_bytes = align_up(cholesky_solve_scratch(n, nrhs));
  const size_t prior_bytes = h->prior_w ? 2 * align_up((size_t)nrhs * h->Nt * h->Nm * 8) : 0;
  TRY_ST(ensure_aux(h, x_bytes + solve_bytes + prior_bytes, s));
  TRY_ST(ensure_ws(h, nrhs));
  char* aux = static_cast<char*>(h->aux);
  double* X = reinterpret_cast<double*>(aux);
  TRY_HIP(hipMemcpyAsync(X, d, (size_t)nrhs * n * 8, hipMemcpyDeviceToDevice, s));
  TRY_HIP(cholesky_solve(Kfac, X, reinterpret_cast<double*>(aux + x_bytes), n, nrhs, s));
  TRY_ST(apply_impl(h, P2O_FADJ, X, m_out, nrhs, s, prior_var));
  if (h->prior_w) {  // Gamma_prior = prior_var (I (x) C)
    double* t1 = reinterpret_cast<double*>(aux + x_bytes + solve_bytes);
    double* t2 = t1 + prior_bytes / 16;
    TRY_HIP(launch_apply_prior(m_out, t1, t2, nrhs * h->Nt, h->prior_nx, h->prior_ny,
                               h->prior_w, h->prior_r, h->prior_delta, s));
  }
  TRY_HIP(hipStreamSynchronize(s));
  return P2O_OK;
}

p2o_status p2o_posterior_invert(p2o_handle h, const double* Kfac, double* Kinv, void* stream) {
  if (!h || !Kfac || !Kinv) return P2O_EINVAL;
  if (!h->ready) return P2O_ESTATE;
  if (h->prec != P2O_FP64) return P2O_EUNSUPPORTED;
  (void)hipGetLastError();
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = h->Nt * h->Nd;
  TRY_HIP(launch_identity(Kinv, n, s));
  if (cholesky_inverse_by_square_fits(Kinv, n)) {
    // L^{-T} by the forward sweep, then K^{-1} = L^{-T} L^{-1} in place
    // (lower triangle and diagonal), mirrored: exactly symmetric
    DevBufs bufs;
    void* diag;
    TRY_HIP(bufs.alloc(&diag, (size_t)n * 8));
    TRY_HIP(launch_cholesky_inverse_by_square(Kfac, Kinv, static_cast<double*>(diag), n, s));
    TRY_HIP(launch_set_diagonal(Kinv, static_cast<const double*>(diag), n, s));
    TRY_HIP(launch_mirror_lower(Kinv, n, s));
    TRY_HIP(hipStreamSynchronize(s));  // before diag is freed
    return P2O_OK;
  }
  // row j of Kinv = K^{-1} e_j: the solves of K X = I, all n at once,
  // restricted to the upper triangle, which is then mirrored (exactly
  // symmetric)
  TRY_HIP(launch_cholesky_inverse_upper(Kfac, Kinv, n, s));
  TRY_HIP(launch_mirror_upper(Kinv, n, s));
  TRY_HIP(hipStreamSynchronize(s));
  return P2O_OK;
}

}  // extern "C"

namespace {

// Bytes of the temporaries of the online posterior mean from K^{-1}:
// [x = K^{-1} d: nrhs n][F* apply workspace][prior temporaries].
struct KinvLayout {
  size_t ws_off, prior_off, total;
};

KinvLayout kinv_layout(const p2o_plan_s* h, int64_t nrhs) {
  const int64_t n = h->Nt * h->Nd;
  KinvLayout l{};
  l.ws_off = align_up((size_t)nrhs * n * 8);
  l.prior_off = l.ws_off + align_up(ws_layout(h, P2O_FADJ, nrhs).total);
  l.total = l.prior_off + (h->prior_w ? 2 * align_up((size_t)nrhs * h->Nt * h->Nm * 8) : 0);
  return l;
}

p2o_status kinv_check(const p2o_plan_s* h, const double* Kinv, const double* d,
                      const double* m_out, int64_t nrhs) {
  if (!h || !Kinv || !d || !m_out || nrhs < 1 || nrhs > 65535) return P2O_EINVAL;
  if (!h->ready) return P2O_ESTATE;
  if (h->prec != P2O_FP64) return P2O_EUNSUPPORTED;
  return P2O_OK;
}

// m = prior_var (I (x) C) F* (Kinv d) on the temporaries at `tmp`
// (kinv_layout bytes); stream-ordered, allocates nothing.
p2o_status kinv_enqueue(p2o_plan_s* h, const double* Kinv, const double* d, double* m_out,
                        int64_t nrhs, double prior_var, char* tmp, bool timed, hipStream_t s) {
  const int64_t n = h->Nt * h->Nd;
  const KinvLayout l = kinv_layout(h, nrhs);
  double* X = reinterpret_cast<double*>(tmp);
  TRY_HIP(launch_qoi_gemv(Kinv, d, X, n, n, nrhs, s));
  TRY_ST(apply_on(h, P2O_FADJ, X, m_out, nrhs, tmp + l.ws_off, timed, s, prior_var));
  if (h->prior_w) {
    double* t1 = reinterpret_cast<double*>(tmp + l.prior_off);
    double* t2 = t1 + (l.total - l.prior_off) / 16;
    TRY_HIP(launch_apply_prior(m_out, t1, t2, nrhs * h->Nt, h->prior_nx, h->prior_ny,
                               h->prior_w, h->prior_r, h->prior_delta, s));
  }
  return P2O_OK;
}

}  // namespace

extern "C" {

p2o_status p2o_posterior_mean_kinv(p2o_handle h, const double* Kinv, const double* d,
                                   double* m_out, int64_t nrhs, double prior_var, void* stream) {
  TRY_ST(kinv_check(h, Kinv, d, m_out, nrhs));
  (void)hipGetLastError();
  hipStream_t s = (hipStream_t)stream;
  TRY_ST(ensure_aux(h, kinv_layout(h, nrhs).total, s));
  return kinv_enqueue(h, Kinv, d, m_out, nrhs, prior_var, static_cast<char*>(h->aux), true, s);
}

}  // extern "C"

// ---------------------------------------- allocation-free online variant
// Fixed device scratch of p2o_posterior_mean_kinv_noalloc: every device the
// library runs on holds its own copy of this array until the process ends.
// In host code `scratch` names a host-side stand-in, not device memory:
// only the per-device address obtained from hipGetSymbolAddress is ever
// handed to kernels or copies.
namespace {

constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mutex;
char* g_scratch_dev[kMaxScratchDevices] = {};

// The device address of `scratch` on `device`, looked up once per device
// with that device current (the caller's current device is restored).
p2o_status scratch_on_device(int device, char** out) {
  if (device < 0 || device >= kMaxScratchDevices) return P2O_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_dev[device]) {
    int current = 0;
    TRY_HIP(hipGetDevice(&current));
    if (current != device) TRY_HIP(hipSetDevice(device));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (current != device) (void)hipSetDevice(current);
    if (e != hipSuccess) return hip_fail(e);
    if (!ptr) return P2O_EHIP;
    g_scratch_dev[device] = static_cast<char*>(ptr);
  }
  *out = g_scratch_dev[device];
  return P2O_OK;
}

}  // namespace

extern "C" {

p2o_status p2o_posterior_mean_kinv_noalloc(p2o_handle h, const double* Kinv, const double* d,
                                           double* m_out, int64_t nrhs, double prior_var,
                                           void* stream) {
  TRY_ST(kinv_check(h, Kinv, d, m_out, nrhs));
  if (kinv_layout(h, nrhs).total > kNoAllocScratchBytes) return P2O_ENOMEM;
  char* base = nullptr;
  TRY_ST(scratch_on_device(h->device, &base));
  (void)hipGetLastError();
  // no part of the scratch needs to start at zero: every kernel writes what
  // a later one reads (K^{-1} d, the transformed d, the products, the prior
  // temporaries); the product kernel is not event-timed here
  return kinv_enqueue(h, Kinv, d, m_out, nrhs, prior_var, base, false, (hipStream_t)stream);
}

}  // extern "C"

// ------------------------------------------------------ batched instances
struct p2o_batch_s {
  std::vector<p2o_handle> plans;
  BatchClass cls = kClassF64;
  BatchInst* dev = nullptr;  // work table of the last p2o_batch_apply
  int cfg[2] = {-1, -1};     // persistent-kernel configuration per op (-1: tune cache or 0)
};

struct p2o_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  BatchInst* dev = nullptr;  // work table the captured launch reads
};

namespace {

BatchClass class_of(p2o_prec p) {
  switch (p) {
    case P2O_FP64: return kClassF64;
    case P2O_MIXED_FP16: return kClassMixedFp16;
    case P2O_MIXED_BF16: return kClassMixedBf16;
    case P2O_FAST_BF16: return kClassFastBf16;
  }
  return kClassF64;
}

// Tune-cache key of a batch: architecture, class, op and a digest (FNV-1a)
// of every instance's shape and right-hand-side count.
std::string batch_key(p2o_batch b, p2o_op op, const int64_t* nrhs) {
  uint64_t hsh = 1469598103934665603ull;
  auto mix = [&](int64_t v) {
    for (int i = 0; i < 8; ++i) {
      hsh ^= (uint64_t)((v >> (8 * i)) & 0xff);
      hsh *= 1099511628211ull;
    }
  };
  for (size_t i = 0; i < b->plans.size(); ++i) {
    const p2o_plan_s* h = b->plans[i];
    mix(h->Nd);
    mix(h->Nm);
    mix(h->Nt);
    mix(nrhs[i]);
    mix(h->mfma_min_rhs[op]);
  }
  hipDeviceProp_t prop{};
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, b->plans[0]->device) == hipSuccess) arch = prop.gcnArchName;
  std::ostringstream k;
  k << arch << "|batch|class" << (int)b->cls << "|op" << (int)op << "|n" << b->plans.size()
    << "|" << std::hex << hsh;
  return k.str();
}

// The configuration an apply uses: the one set or tuned on this batch, else
// a tune-cache entry for these shapes and counts, else configuration 0.
int batch_cfg(p2o_batch b, p2o_op op, const int64_t* nrhs) {
  if (b->cfg[op] >= 0) return b->cfg[op];
  if (const char* path = std::getenv("P2O_TUNE_CACHE")) {
    const auto m = read_cache(path);
    const auto it = m.find(batch_key(b, op, nrhs));
    if (it != m.end() && it->second >= 0 && it->second < batch_config_count()) return it->second;
  }
  return 0;
}

// Validate the per-instance arguments, reserve workspaces and build the
// work table (host copy) for one batched apply in configuration `cfg`.
// bfloat16 instances on the matrix-core path get their own product launch
// (the warp-specialised kernels of gemm_bf16.hip, bitwise equal to the
// persistent kernel's units and faster: their loads and products run on
// different wavefronts); they are listed in `own` and left out of the
// table.  All other instances share the one persistent launch.
p2o_status batch_prepare(p2o_batch b, p2o_op op, const double* const* x, double* const* y,
                         const int64_t* nrhs, int cfg, std::vector<BatchInst>* table,
                         int64_t* total, std::vector<int>* own) {
  if (!b || !x || !y || !nrhs || (op != P2O_F && op != P2O_FADJ)) return P2O_EINVAL;
  const size_t n = b->plans.size();
  table->clear();
  own->clear();
  int64_t units = 0;
  for (size_t i = 0; i < n; ++i) {
    p2o_plan_s* h = b->plans[i];
    if (!x[i] || !y[i] || nrhs[i] < 1 || nrhs[i] > 65535) return P2O_EINVAL;
    TRY_ST(ensure_ws(h, nrhs[i]));
    const WsLayout w = ws_layout(h, op, nrhs[i]);
    char* ws = static_cast<char*>(h->ws);
    const bool matrix = use_mfma(h, op, nrhs[i]) && h->prec != P2O_MIXED_FP16;
    if (matrix && (b->cls == kClassMixedBf16 || b->cls == kClassFastBf16)) {
      own->push_back((int)i);
      continue;
    }
    table->push_back(BatchInst{});
    BatchInst& I = table->back();
    I.fhat = h->fhat;
    I.scales = h->scales;
    I.in = ws + ((matrix && is_mixed(h->prec)) ? w.c_off : w.a_off);
    I.out = ws + w.b_off;
    I.g = GemvShape{h->nf, h->Nd, h->Nm, nrhs[i], (int)h->n_pc, h->pc_len};
    I.n8 = plane_pitch(h, op);
    I.path = matrix ? kPathMatrix : kPathVector;
    I.unit_begin = units;
    const int64_t nu = batch_units(b->cls, op, I.path, I.g, cfg);
    if (nu < 0) return P2O_EINVAL;  // a path the persistent kernel does not run
    units += nu;
  }
  *total = units;
  return P2O_OK;
}

// Enqueue one batched apply whose work table is already on the device:
// every instance's forward transform (writing the bfloat16 operand planes
// for matrix-core instances), one persistent product launch over the
// table's instances, the product launches of the instances in `own`, every
// instance's inverse transform.
p2o_status batch_enqueue(p2o_batch b, p2o_op op, const double* const* x, double* const* y,
                         const int64_t* nrhs, const std::vector<BatchInst>& table,
                         const BatchInst* dev_table, int64_t total, int cfg,
                         const std::vector<int>& own, hipStream_t s) {
  const size_t n = b->plans.size();
  for (size_t i = 0; i < n; ++i)
    TRY_HIP(enqueue_forward(b->plans[i], op, x[i], nrhs[i], static_cast<char*>(b->plans[i]->ws), s));
  if (total > 0) TRY_HIP(launch_batch_product(b->cls, op, dev_table, (int)table.size(), total, cfg, s));
  for (const int i : own) {
    p2o_plan_s* h = b->plans[i];
    const WsLayout w = ws_layout(h, op, nrhs[i]);
    char* ws = static_cast<char*>(h->ws);
    TRY_HIP(launch_product(h, op, ws + w.a_off, ws + w.b_off, ws + w.c_off, nrhs[i],
                           default_cfg(h, op), s));
  }
  for (size_t i = 0; i < n; ++i)
    TRY_HIP(enqueue_inverse(b->plans[i], op, y[i], nrhs[i], 1.0,
                            static_cast<const char*>(b->plans[i]->ws), s));
  return P2O_OK;
}

}  // namespace

extern "C" {

p2o_status p2o_batch_create(const p2o_handle* plans, int64_t n, p2o_batch* out) {
  if (!out) return P2O_EINVAL;
  *out = nullptr;
  if (!plans || n < 1 || n > (1 << 20)) return P2O_EINVAL;
  for (int64_t i = 0; i < n; ++i) {
    if (!plans[i]) return P2O_EINVAL;
    if (!plans[i]->ready) return P2O_ESTATE;
    if (plans[i]->prec != plans[0]->prec || plans[i]->device != plans[0]->device)
      return P2O_EINVAL;
    for (int64_t j = 0; j < i; ++j)
      if (plans[j] == plans[i]) return P2O_EINVAL;  // instances own their workspaces
  }
  auto* b = new (std::nothrow) p2o_batch_s;
  if (!b) return P2O_ENOMEM;
  b->plans.assign(plans, plans + n);
  b->cls = class_of(plans[0]->prec);
  const hipError_t e = hipMalloc((void**)&b->dev, sizeof(BatchInst) * n);
  if (e != hipSuccess) {
    delete b;
    return hip_fail(e);
  }
  *out = b;
  return P2O_OK;
}

p2o_status p2o_batch_apply(p2o_batch b, p2o_op op, const double* const* x, double* const* y,
                           const int64_t* nrhs, void* stream) {
  (void)hipGetLastError();
  if (!b || !nrhs || (op != P2O_F && op != P2O_FADJ)) return P2O_EINVAL;
  std::vector<BatchInst> table;
  std::vector<int> own;
  int64_t total = 0;
  const int cfg = batch_cfg(b, op, nrhs);
  TRY_ST(batch_prepare(b, op, x, y, nrhs, cfg, &table, &total, &own));
  hipStream_t s = (hipStream_t)stream;
  TRY_HIP(hipStreamSynchronize(s));  // the previous apply has finished reading the table
  if (!table.empty())
    TRY_HIP(hipMemcpy(b->dev, table.data(), sizeof(BatchInst) * table.size(), hipMemcpyHostToDevice));
  return batch_enqueue(b, op, x, y, nrhs, table, b->dev, total, cfg, own, s);
}

p2o_status p2o_batch_set_config(p2o_batch b, p2o_op op, int64_t cfg) {
  if (!b || (op != P2O_F && op != P2O_FADJ)) return P2O_EINVAL;
  if (cfg < -1 || cfg >= batch_config_count()) return P2O_EINVAL;
  b->cfg[op] = (int)cfg;
  return P2O_OK;
}

p2o_status p2o_batch_get_config(p2o_batch b, p2o_op op, int64_t* cfg, int64_t* n_candidates) {
  if (!b || (op != P2O_F && op != P2O_FADJ)) return P2O_EINVAL;
  if (cfg) *cfg = b->cfg[op];
  if (n_candidates) *n_candidates = batch_config_count();
  return P2O_OK;
}

p2o_status p2o_batch_autotune(p2o_batch b, p2o_op op, const double* const* x, double* const* y,
                              const int64_t* nrhs, int reps, double* times_ms, int64_t max_times,
                              int64_t* chosen, void* stream) {
  if (!b || !nrhs || (op != P2O_F && op != P2O_FADJ) || reps < 1 || max_times < 0 ||
      (max_times > 0 && !times_ms))
    return P2O_EINVAL;
  (void)hipGetLastError();
  hipStream_t s = (hipStream_t)stream;
  const int n = batch_config_count();
  hipEvent_t e0, e1;
  TRY_HIP(hipEventCreate(&e0));
  TRY_HIP(hipEventCreate(&e1));
  int best = -1;
  float best_ms = 0.f;
  p2o_status st = P2O_OK;
  for (int c = 0; c < n && st == P2O_OK; ++c) {
    std::vector<BatchInst> table;
    std::vector<int> own;
    int64_t total = 0;
    st = batch_prepare(b, op, x, y, nrhs, c, &table, &total, &own);
    if (st != P2O_OK) break;
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess && !table.empty())
      e = hipMemcpy(b->dev, table.data(), sizeof(BatchInst) * table.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) { st = hip_fail(e); break; }
    // one whole apply (transforms included) leaves valid inputs in the
    // workspaces, then the persistent product launch alone is timed (an
    // empty one, when every instance has its own launch, takes 0 ms)
    st = batch_enqueue(b, op, x, y, nrhs, table, b->dev, total, c, own, s);
    if (st != P2O_OK) break;
    e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && e == hipSuccess && total > 0; ++r)
      e = launch_batch_product(b->cls, op, b->dev, (int)table.size(), total, c, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) { st = hip_fail(e); break; }
    ms /= (float)reps;
    if (c < max_times) times_ms[c] = ms;
    if (best < 0 || ms < best_ms) {
      best = c;
      best_ms = ms;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != P2O_OK) return st;
  b->cfg[op] = best;
  if (chosen) *chosen = best;
  if (const char* path = std::getenv("P2O_TUNE_CACHE")) {
    auto m = read_cache(path);
    m[batch_key(b, op, nrhs)] = best;
    write_cache(path, m);
  }
  return P2O_OK;
}

p2o_status p2o_graph_capture(p2o_batch b, p2o_op op, const double* const* x, double* const* y,
                             const int64_t* nrhs, void* stream, p2o_graph* out) {
  if (!out) return P2O_EINVAL;
  *out = nullptr;
  (void)hipGetLastError();
  if (!b || !nrhs || (op != P2O_F && op != P2O_FADJ)) return P2O_EINVAL;
  std::vector<BatchInst> table;
  std::vector<int> own;
  int64_t total = 0;
  const int cfg = batch_cfg(b, op, nrhs);
  TRY_ST(batch_prepare(b, op, x, y, nrhs, cfg, &table, &total, &own));
  TRY_HIP(hipStreamSynchronize((hipStream_t)stream));
  auto* g = new (std::nothrow) p2o_graph_s;
  if (!g) return P2O_ENOMEM;
  hipError_t e = hipMalloc((void**)&g->dev, sizeof(BatchInst) * std::max<size_t>(1, table.size()));
  if (e == hipSuccess && !table.empty())
    e = hipMemcpy(g->dev, table.data(), sizeof(BatchInst) * table.size(), hipMemcpyHostToDevice);
  hipStream_t cs = nullptr;
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  p2o_status st = P2O_OK;
  if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    st = batch_enqueue(b, op, x, y, nrhs, table, g->dev, total, cfg, own, cs);
    const hipError_t e2 = hipStreamEndCapture(cs, &g->graph);
    if (st == P2O_OK && e2 != hipSuccess) e = e2;
  }
  if (e == hipSuccess && st == P2O_OK) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (cs) (void)hipStreamDestroy(cs);
  if (e != hipSuccess || st != P2O_OK) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    (void)hipFree(g->dev);
    delete g;
    return st != P2O_OK ? st : hip_fail(e);
  }
  *out = g;
  return P2O_OK;
}

p2o_status p2o_batch_capture(p2o_batch b, p2o_op op, const double* const* x, double* const* y,
                             const int64_t* nrhs, void* stream, p2o_graph* out) {
  return p2o_graph_capture(b, op, x, y, nrhs, stream, out);
}

p2o_status p2o_graph_launch(p2o_graph g, void* stream) {
  if (!g) return P2O_EINVAL;
  TRY_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
  return P2O_OK;
}

void p2o_graph_destroy(p2o_graph g) {
  if (!g) return;
  (void)hipGraphExecDestroy(g->exec);
  (void)hipGraphDestroy(g->graph);
  (void)hipFree(g->dev);
  delete g;
}

void p2o_batch_destroy(p2o_batch b) {
  if (!b) return;
  (void)hipFree(b->dev);
  delete b;
}

}  // extern "C"
