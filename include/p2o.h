/*
 * p2o.h - C ABI of the MI355X (gfx950) library for the shift-invariant
 * parameter-to-observable map of "Real-time Bayesian inference at extreme
 * scale: a digital twin for tsunami early warning".
 *
 * The map (section "FFT-based Hessian matvecs", eq. ShiftInvariance) is the
 * block lower-triangular Toeplitz matrix F with Nt x Nt blocks of size
 * Nd x Nm; block (i, j) is F_{i-j} for j <= i.  Only the first block column
 * F_0 .. F_{Nt-1} is stored, and F is applied through a block-circulant
 * embedding of length L diagonalised by the DFT: d = F m becomes one Nd x Nm
 * complex block product per frequency.  F* is the Euclidean transpose F^T.
 * On top of F and F* the library forms the data-space Hessian
 * K = Gamma_noise + F Gamma_prior F* and the posterior mean
 * m = Gamma_prior F* K^{-1} d (section "Real-time Bayesian inference and
 * prediction framework", Phases 2 and 4, zero prior mean).
 *
 * Conventions shared by every entry point
 *   - Blocks:  [Nt][Nd][Nm] row-major float64, blocks[k] = F_k = the paper's
 *              F_{k+1,1}.
 *   - Vectors: a parameter vector is [nrhs][Nt][Nm], a data vector
 *              [nrhs][Nt][Nd]; row-major float64; time step outermost
 *              within one right-hand side.
 *   - Pointers to arrays are DEVICE pointers unless stated otherwise.  The
 *     caller owns every buffer it passes; the library owns the frequency
 *     blocks, the scales and its workspaces, and frees them in p2o_destroy.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Every call is
 *     ordered on it and returns without waiting for the device, except the
 *     setup calls, p2o_reserve, p2o_autotune, p2o_hessian_assemble,
 *     p2o_posterior_solve and p2o_qoi_precompute, which may allocate or
 *     synchronise the stream.
 *   - Errors are reported only through the return code; nothing is thrown
 *     across the ABI.  On any code other than P2O_OK the outputs are
 *     unspecified and the handle remains usable.  P2O_EHIP carries the HIP
 *     error code, readable with p2o_last_hip_error (per calling thread).
 *   - A handle is not thread-safe: serialise calls on one handle.
 *   - L is the smallest even integer >= 2*Nt whose prime factors are all in
 *     {2, 3, 5, 7} (L = 2*Nt whenever 2*Nt is such a number, e.g. Nt = 32,
 *     200, 420); L >= 2*Nt - 1 is what makes the circulant embedding exact.
 *     The library stores nf = L/2 + 1 frequency blocks.
 */
#ifndef P2O_H
#define P2O_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct p2o_plan_s* p2o_handle;

typedef enum {
  P2O_OK = 0,
  P2O_EINVAL = 1,        /* bad argument: null pointer, size < 1, bad enum  */
  P2O_ENOMEM = 2,        /* device allocation failed or size overflows      */
  P2O_EHIP = 3,          /* a HIP runtime call failed                        */
  P2O_ENOTPD = 4,        /* Cholesky met a non-positive pivot                */
  P2O_ESTATE = 5,        /* call out of order (e.g. apply before setup_end)  */
  P2O_EUNSUPPORTED = 6   /* valid request this build does not provide        */
} p2o_status;

typedef enum {
  P2O_F = 0,     /* y = F x : x parameter vector, y data vector       */
  P2O_FADJ = 1   /* y = F* x: x data vector,      y parameter vector  */
} p2o_op;

/* Precision tiers.  The mixed tiers store every real component v of a
 * frequency-block entry as 16-bit terms with one power-of-two float32 scale
 * s = 2^e per (frequency k, 256 consecutive columns) sub-block, over all
 * sensors:
 *   e     from the sub-block's largest component magnitude M, M in
 *         [2^(E-1), 2^E): e = E for bfloat16 (so |v/s| < 1), e = E - 15 for
 *         binary16 (|v/s| < 2^15); clamped to [-120, 120]; E = 0 for an
 *         all-zero sub-block;
 *   hi    = r16(v / s),  lo = r16((v / s - hi) / c),  value = s (hi + c lo),
 *         c = 1 (bfloat16) or 2^-11 (binary16), r16 rounding to nearest
 *         even first to float32, then to the 16-bit format;
 * so the stored value differs from v by about 2^-16 |v| (bfloat16) or
 * 2^-22 |v| (binary16).  Transforms run in float32 and block products
 * accumulate in float32; F's column-chunk partial sums are combined in
 * float64, F*'s products (a sum over sensors) are float32 throughout.  8
 * bytes per complex block entry (4 for the hi-only tier). */
typedef enum {
  /* Frequency blocks stored as complex float64, transforms and block
   * products in float64 (16 bytes per complex block entry). */
  P2O_FP64 = 0,
  /* bfloat16 hi + lo terms (the default mixed tier). */
  P2O_MIXED = 1,
  /* bfloat16 hi term only: half the block bytes, error ~1e-3 (stated, not
   * within 1e-5). */
  P2O_FAST = 2,
  /* binary16 hi + lo terms (error ~1e-7; vector units only). */
  P2O_MIXED_FP16 = 3,
  /* Names that spell out the 16-bit format of the two bfloat16 tiers. */
  P2O_MIXED_BF16 = P2O_MIXED,
  P2O_FAST_BF16 = P2O_FAST
} p2o_prec;

/* ---------------------------------------------------------------- setup */

/* One-shot setup from all blocks at once.
 *   blocks  device [Nt][Nd][Nm] float64 (first block column, see above).
 *           Not retained: the caller may free it once `stream` has drained.
 *   Nd, Nm, Nt >= 1;  prec one of p2o_prec.
 *   out     host pointer receiving the new handle (set to NULL on error).
 * Allocates the frequency blocks (nf*Nd*Nm complex entries of the chosen
 * precision) and synchronises `stream` before returning. */
p2o_status p2o_setup(const double* blocks, int64_t Nd, int64_t Nm, int64_t Nt,
                     p2o_prec prec, void* stream, p2o_handle* out);

/* Chunked setup, so the time-domain blocks never need to co-reside with the
 * frequency blocks: begin, then setup_columns for column ranges that cover
 * [0, Nm) exactly once (any order), then setup_end.
 *   blocks_chunk  device [Nt][Nd][p1-p0] float64, columns p0..p1-1 of every
 *                 block; 0 <= p0 < p1 <= Nm.  For the mixed precisions p0
 *                 must be a multiple of 256 and p1 a multiple of 256 or Nm.
 * setup_columns synchronises `stream` before returning. */
p2o_status p2o_setup_begin(int64_t Nd, int64_t Nm, int64_t Nt, p2o_prec prec,
                           void* stream, p2o_handle* out);
p2o_status p2o_setup_columns(p2o_handle h, const double* blocks_chunk,
                             int64_t p0, int64_t p1, void* stream);
p2o_status p2o_setup_end(p2o_handle h, void* stream);

/* Query the shape and precision of a plan (host out-pointers may be NULL). */
p2o_status p2o_get_info(p2o_handle h, int64_t* Nd, int64_t* Nm, int64_t* Nt,
                        int64_t* L, int* prec);

/* Pre-allocate the apply workspace for up to `nrhs` right-hand sides, so
 * that later p2o_apply calls with nrhs <= this do not allocate. */
p2o_status p2o_reserve(p2o_handle h, int64_t nrhs, void* stream);

/* ---------------------------------------------------------------- apply */

/* y = F x (op = P2O_F) or y = F* x (op = P2O_FADJ) for nrhs >= 1
 * right-hand sides, through the frequency blocks (exact up to rounding).
 *   P2O_F   : x [nrhs][Nt][Nm], y [nrhs][Nt][Nd]
 *   P2O_FADJ: x [nrhs][Nt][Nd], y [nrhs][Nt][Nm]
 * Input and output are float64 whatever the plan precision; x and y must
 * not overlap.  May allocate workspace on first use of a larger nrhs. */
p2o_status p2o_apply(p2o_handle h, p2o_op op, const double* x, double* y,
                     int64_t nrhs, void* stream);

/* --------------------------------------------------------------- tuning */

/* The frequency-block product kernel of each op has a small table of
 * candidate configurations (rows per wavefront for F, column groups per
 * wavefront for F*, load vector width).  Candidate 0 that is valid for the
 * plan's shape is the default; a candidate whose vector width does not
 * divide Nm is not valid.
 *
 * p2o_autotune times every valid candidate for `op` on one right-hand
 * side (`reps` timed launches each, after one warm-up) on the plan's own
 * frequency blocks, and keeps the fastest for later p2o_apply calls.
 *   times_ms  host array (may be NULL when max_times = 0); entry c receives
 *             candidate c's mean time in ms, or -1 if it is not valid.
 *   chosen    host pointer (may be NULL) receiving the chosen index.
 * If the environment variable P2O_TUNE_CACHE names a file, the choice is
 * stored there (a flat JSON object keyed by architecture, precision, op and
 * shape) and p2o_setup / p2o_setup_end apply stored choices to new plans.
 * Synchronises `stream`; allocates the single-RHS workspace if needed. */
p2o_status p2o_autotune(p2o_handle h, p2o_op op, int reps, double* times_ms,
                        int64_t max_times, int64_t* chosen, void* stream);

/* Current candidate index for `op` and the table size (host pointers, may
 * be NULL). */
p2o_status p2o_get_config(p2o_handle h, p2o_op op, int64_t* cfg,
                          int64_t* n_candidates);

/* Force candidate `cfg` for `op`: P2O_EINVAL if out of range,
 * P2O_EUNSUPPORTED if not valid for this plan's shape. */
p2o_status p2o_set_config(p2o_handle h, p2o_op op, int64_t cfg);

/* Switch the frequency-block product of `op` from the vector-unit kernels
 * above to matrix-core (MFMA) kernels once a call has at least `min_rhs`
 * right-hand sides (default 8); min_rhs <= 0 keeps the vector-unit kernels
 * for every nrhs.  P2O_FP64 plans use float64 MFMA; P2O_MIXED_BF16 and
 * P2O_FAST_BF16 plans use bfloat16 MFMA with the vector split into hi + lo
 * bfloat16 terms and float32 accumulation (same error class as their
 * vector-unit kernels); P2O_MIXED_FP16 plans always use the vector units. */
p2o_status p2o_set_mfma_threshold(p2o_handle h, p2o_op op, int64_t min_rhs);

/* ---------------------------------------------------- batched instances */

/* A batch groups independent, set-up plans of uneven shape (all of one
 * precision, on one device, each plan at most once: instances use their
 * own workspaces) so that one call applies all of them.  Per instance the
 * block product takes the vector-unit path or the matrix-core path by its
 * right-hand-side count (p2o_set_mfma_threshold of that plan).  The
 * products of the vector-path instances (and of FP64 instances on the
 * float64 matrix cores) run in ONE persistent kernel launch that walks
 * their work units; each bfloat16 instance on the matrix-core path gets
 * its own launch of the single-plan product kernel (bitwise equal
 * results); each instance's transforms are launched around them.
 * The plans must outlive the batch.  NULL-safe destroy. */
typedef struct p2o_batch_s* p2o_batch;
typedef struct p2o_graph_s* p2o_graph;

p2o_status p2o_batch_create(const p2o_handle* plans, int64_t n, p2o_batch* out);

/* y[i] = F x[i] or F* x[i] for every instance i < n.
 *   x, y   HOST arrays of n device pointers, laid out as for p2o_apply;
 *   nrhs   HOST array of n right-hand-side counts (1..65535).
 * Synchronises `stream` first (the work table is reused between calls),
 * may allocate instance workspaces; then enqueues without waiting. */
p2o_status p2o_batch_apply(p2o_batch b, p2o_op op, const double* const* x,
                           double* const* y, const int64_t* nrhs, void* stream);

/* The persistent kernel has a small table of configurations (its tiles):
 * vector-unit rows per wavefront for F (4, 2, 8) and column groups per
 * wavefront for F* (2, 1, 4) for candidates 0..2.  All give the same
 * results bit for bit (each output's sums run in the same order).  A batch
 * whose instances all have their own launches has an empty persistent
 * launch: every candidate then times at ~0 ms.
 * p2o_batch_autotune times every candidate's product launch for `op` on
 * these inputs (one whole apply first, then `reps` timed launches), keeps
 * the fastest for this batch and, when P2O_TUNE_CACHE names a file, stores
 * it there under a key of the architecture, precision class, op and a
 * digest of every instance's (Nd, Nm, Nt, nrhs, matrix-core threshold);
 * applies and captures of a batch with no configuration set look that key
 * up, else use candidate 0.  Arguments as p2o_batch_apply, plus
 *   times_ms  host array (may be NULL when max_times = 0) receiving each
 *             candidate's mean product time in ms;
 *   chosen    host pointer (may be NULL) receiving the chosen index.
 * Synchronises `stream`; overwrites y. */
p2o_status p2o_batch_autotune(p2o_batch b, p2o_op op, const double* const* x,
                              double* const* y, const int64_t* nrhs, int reps,
                              double* times_ms, int64_t max_times, int64_t* chosen,
                              void* stream);
/* Force candidate cfg (0 .. n-1) for `op`, or -1 to return to the tune
 * cache / default; P2O_EINVAL out of range.  Host-side only. */
p2o_status p2o_batch_set_config(p2o_batch b, p2o_op op, int64_t cfg);
/* The configuration set for `op` (-1 if none) and the number of candidates
 * (host pointers, may be NULL). */
p2o_status p2o_batch_get_config(p2o_batch b, p2o_op op, int64_t* cfg, int64_t* n_candidates);

/* Capture one batched apply on fixed buffers into a HIP graph (workspaces
 * are reserved before capture; the graph holds no allocation or memset).
 * p2o_graph_launch replays it on `stream`; replays read x and write y at
 * the captured addresses.  p2o_batch_capture is the same call under its
 * earlier name. */
p2o_status p2o_graph_capture(p2o_batch b, p2o_op op, const double* const* x,
                             double* const* y, const int64_t* nrhs, void* stream,
                             p2o_graph* out);
p2o_status p2o_batch_capture(p2o_batch b, p2o_op op, const double* const* x,
                             double* const* y, const int64_t* nrhs, void* stream,
                             p2o_graph* out);
p2o_status p2o_graph_launch(p2o_graph g, void* stream);
void p2o_graph_destroy(p2o_graph g);
void p2o_batch_destroy(p2o_batch b);

/* ------------------------------------------------------ inversion (FP64) */

/* K = Gamma_noise + F Gamma_prior F* (Phase 2), Gamma_prior =
 * prior_var * (I (x) C) (C = I unless p2o_set_prior selected a spatial
 * covariance), Gamma_noise = diag(noise_var), formed as the paper does
 * (one F Gamma_prior F* product per unit vector of data space, in batches)
 * or in Gram form, as p2o_set_assembly selects.
 *   noise_var  device [Nt*Nd] float64 (> 0 expected, not checked)
 *   K          device [(Nt*Nd)^2] float64 row-major, caller-allocated;
 *              entry (i*Nd + s, j*Nd + r) couples sensor s at step i with
 *              sensor r at step j.  K is symmetrised: (K + K^T)/2 by the
 *              unit-vector method, the lower triangle mirrored by the Gram
 *              form.
 * Requires a P2O_FP64 plan (else P2O_EUNSUPPORTED).  Allocates a temporary
 * workspace and synchronises `stream`.  The unit-vector method keeps the
 * time-domain blocks ((Nt Nd) Nm doubles, three times that with a spatial
 * prior) plus per-pass buffers bounded by the environment variable
 * P2O_WORKSPACE_MB (MiB; default 8 GiB; at least one unit vector's
 * spectra); see p2o_assembly for the Gram form. */
p2o_status p2o_hessian_assemble(p2o_handle h, double prior_var,
                                const double* noise_var, double* K,
                                void* stream);

/* How p2o_hessian_assemble and p2o_qoi_precompute (there: the p2o plan's
 * setting) form their products F Gamma_prior F* (and Fq Gamma_prior F*,
 * Fq Gamma_prior Fq*); both give the same matrix up to rounding.
 *   P2O_ASSEMBLE_MATVEC (default): the paper's Phase 2, one FFT-based
 *     F Gamma_prior F* product per unit vector of data space, in batches
 *     (about 8 nf Nd^2 Nm Nt flops for K).
 *   P2O_ASSEMBLE_GRAM: the time-domain blocks F_0 .. F_{Nt-1} are recovered
 *     from the frequency blocks by one inverse transform and stacked into
 *     the (Nt Nd) x Nm matrix A (row t*Nd + s = row s of F_t); then
 *     G = prior_var A C A^T (one float64 matrix-core GEMM, lower triangle,
 *     about (Nt Nd)^2 Nm flops) and, because F is block lower triangular
 *     Toeplitz, block (t, u) of F Gamma_prior F* is the sum over
 *     l <= min(t, u) of block (t - l, u - l) of G: prefix sums along the
 *     block diagonals.  Needs (Nt Nd) Nm doubles of temporary memory (three
 *     times that again with a spatial prior). */
typedef enum {
  P2O_ASSEMBLE_MATVEC = 0,
  P2O_ASSEMBLE_GRAM = 1
} p2o_assembly;

/* Selects the assembly method of the plan's later inversion calls.
 * P2O_EINVAL on a null handle or an unknown method.  Host-side only. */
p2o_status p2o_set_assembly(p2o_handle h, p2o_assembly method);

/* Posterior mean m = Gamma_prior F* K^{-1} d (Phase 4, zero prior mean;
 * Gamma_prior as for p2o_hessian_assemble).
 *   K      device [(Nt*Nd)^2] float64; on return its lower triangle holds
 *          the Cholesky factor L (K = L L^T) and its strict upper triangle
 *          is unchanged.
 *   d      device [nrhs][Nt][Nd];  m_out device [nrhs][Nt][Nm].
 *   refine_steps  >= 0 rounds of iterative refinement x += K^{-1}(d - K x),
 *          with the residual formed in float64 from the untouched upper
 *          triangle and a saved copy of the diagonal.
 *   failed_pivot  HOST pointer (may be NULL); on P2O_ENOTPD receives the
 *          0-based index of the first non-positive pivot.
 * Requires a P2O_FP64 plan.  Synchronises `stream`. */
p2o_status p2o_posterior_solve(p2o_handle h, double* K, const double* d,
                               double* m_out, int64_t nrhs, double prior_var,
                               int refine_steps, int64_t* failed_pivot,
                               void* stream);

/* Phase 4 online inference with K already factored (offline, by
 * p2o_posterior_solve): m = Gamma_prior F* K^{-1} d from the Cholesky factor
 * alone (two triangular sweeps and one F* apply; no refinement, which
 * would need K itself).
 *   Kfac   device [(Nt*Nd)^2]: K after p2o_posterior_solve (the factor in
 *          its lower triangle; the upper triangle is not read).
 *   d      device [nrhs][Nt][Nd];  m_out device [nrhs][Nt][Nm].
 * Requires a P2O_FP64 plan (else P2O_EUNSUPPORTED); P2O_EINVAL on null
 * pointers or nrhs outside 1 .. 65535.  Its temporaries (n*nrhs doubles,
 * the inverted 64 x 64 diagonal blocks of the factor, which every call
 * forms again, and the F* apply workspace) are plan-owned and grow on
 * demand.  Synchronises `stream`. */
p2o_status p2o_posterior_mean(p2o_handle h, const double* Kfac, const double* d, double* m_out,
                              int64_t nrhs, double prior_var, void* stream);

/* Offline, once per factorisation (the paper's Phases 2-3 end with K
 * factored; this goes one step further): K^{-1} itself, so that the online
 * posterior mean is one pass over a matrix instead of two sequential
 * triangular sweeps (section "Real-time Bayesian inference and prediction
 * framework": Phase 4 must run in real time).
 *   Kfac  device [(Nt*Nd)^2]: K after p2o_posterior_solve (the factor in its
 *         lower triangle; the upper triangle is not read).
 *   Kinv  device [(Nt*Nd)^2] float64 row-major, caller-allocated, must not
 *         overlap Kfac; receives K^{-1}, exactly symmetric.  Where Kinv is
 *         16-byte aligned, n = Nt*Nd even and n >= 512: L^{-T} by a forward
 *         sweep over the identity, then K^{-1} = L^{-T} L^{-1} as one
 *         symmetric matrix-core product in place (about 2 n^3 / 3 flops;
 *         n doubles of temporary device memory).  Otherwise the solves of
 *         K X = I restricted to the upper triangle (about n^3 flops).  The
 *         triangle computed is mirrored onto the other.
 * An explicit inverse applied to d has an error of the order of
 * cond(K) u ||K^{-1}|| ||d||, against cond(K) u ||K^{-1} d|| for the
 * triangular sweeps: the same for a well-conditioned K, possibly larger
 * for a badly conditioned one.
 * Requires a P2O_FP64 plan (else P2O_EUNSUPPORTED); P2O_EINVAL on null
 * pointers.  Synchronises `stream`. */
p2o_status p2o_posterior_invert(p2o_handle h, const double* Kfac, double* Kinv, void* stream);

/* Phase 4 online inference from K^{-1} (p2o_posterior_invert):
 * m = Gamma_prior F* (K^{-1} d): one pass over K^{-1} (an HBM-bound
 * matrix-vector product, 8 n^2 bytes) and one F* apply.
 *   Kinv  device [(Nt*Nd)^2] (all of it is read).
 *   d     device [nrhs][Nt][Nd];  m_out device [nrhs][Nt][Nm].
 * Requires a P2O_FP64 plan (else P2O_EUNSUPPORTED); P2O_EINVAL on null
 * pointers or nrhs outside 1 .. 65535.  Stream-ordered: does not
 * synchronise.  Temporaries (n*nrhs doubles plus the F* apply workspace,
 * and 2*nrhs*Nt*Nm doubles with a spatial prior) are plan-owned: the first
 * call with a larger nrhs allocates them (draining `stream` first if an
 * older buffer is replaced), later calls allocate nothing. */
p2o_status p2o_posterior_mean_kinv(p2o_handle h, const double* Kinv, const double* d,
                                   double* m_out, int64_t nrhs, double prior_var, void* stream);

/* p2o_posterior_mean_kinv for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same computation on the same kernels (results equal to
 * p2o_posterior_mean_kinv's bit for bit), with every temporary in one
 * fixed 64 MiB device array that each GPU the library runs on holds until
 * the process ends.  Calls no hipMalloc, hipFree or other allocating
 * routine; the first call on a device looks up that array's address
 * (hipGetSymbolAddress) and keeps it.  The temporaries need
 *   8 n nrhs + (16 nf Nd + 16 nf Nm) nrhs bytes (n = Nt*Nd, nf = L/2 + 1,
 *   each part rounded up to 256 bytes), plus 2 * 8 nrhs Nt Nm with a
 *   spatial prior;
 * beyond 64 MiB the call returns P2O_ENOMEM and does nothing (at Nd = 100,
 * Nm = 5000, Nt = 200: up to 3 right-hand sides without a spatial prior).
 * All calls on one GPU share that GPU's array, which keeps the last call's
 * contents: calls that overlap on one GPU (other streams, other threads,
 * other plans) race and must be serialised by the caller.  Arguments,
 * errors and stream ordering as p2o_posterior_mean_kinv. */
p2o_status p2o_posterior_mean_kinv_noalloc(p2o_handle h, const double* Kinv, const double* d,
                                           double* m_out, int64_t nrhs, double prior_var,
                                           void* stream);

/* --------------------------------------------- spatial prior covariance
 * The inversion calls below take Gamma_prior = prior_var * (I_Nt (x) C):
 * the same spatial covariance C on every time step (time-invariant, which
 * keeps G* = Gamma_prior F* block Toeplitz, section "Real-time Bayesian
 * inference and prediction framework", Phase 2).  By default C = I.
 * p2o_set_prior selects a synthetic smooth SPD stand-in for the paper's
 * Matern-type prior (whose elliptic solves need a mesh): with the Nm
 * parameters on an nx x ny grid (p = ix*ny + iy),
 *   C x = delta x + B (B x),
 *   (B x)[ix, iy] = sum_{|a|,|b| <= radius} w_a w_b x[ix + a, iy + b],
 *   w_a = exp(-a^2 / (2 length^2)), zero outside the grid,
 * so B is symmetric and C symmetric positive definite. */
typedef struct {
  int64_t nx, ny;  /* grid, nx * ny == Nm */
  int radius;      /* window half-width, 0 .. 32 */
  double length;   /* Gaussian length scale in grid points, > 0 */
  double delta;    /* nugget, > 0 */
} p2o_prior_grid;

/* Sets the plan's spatial prior (copied; prior may be freed on return), or
 * restores C = I when prior is NULL.  P2O_EINVAL on a grid that does not
 * match Nm or parameters out of range (the plan keeps its previous prior).
 * Used by p2o_hessian_assemble, p2o_posterior_solve and
 * p2o_qoi_precompute (there the p2o plan's prior governs).  May
 * synchronise `stream` (replacing an earlier prior). */
p2o_status p2o_set_prior(p2o_handle h, const p2o_prior_grid* prior, void* stream);

/* ---------------------------------------------- QoI prediction (FP64)
 * The parameter-to-QoI (p2q) map Fq is another shift-invariant block
 * Toeplitz operator, Nq forecast locations instead of Nd sensors (section
 * "Real-time Bayesian inference and prediction framework"): set it up as an
 * ordinary plan with Nd = Nq; p2o_apply(P2O_F) on it gives q = Fq m. */

/* Phase 3 precomputations of the QoI posterior (zero prior mean,
 * Gamma_prior = prior_var * (I (x) C) with hF's spatial prior C):
 *   Q  = Fq Gamma_post F* Gamma_noise^{-1} = Fq Gamma_prior F* K^{-1}
 *        (the data-to-QoI map; the two forms agree by Sherman-Morrison-
 *        Woodbury), so that Q d = Fq m_map;
 *   Gq = Fq Gamma_post Fq* = Fq Gamma_prior Fq* - Q (F Gamma_prior Fq*)
 *        (the QoI posterior covariance), symmetrised.
 * Formed from the N_t Nq unit vectors of QoI space with the F / F* machinery
 * of p2o_hessian_assemble (or in Gram form, as hF's p2o_set_assembly
 * selects) and one blocked solve with K's factor for all of them at once.
 *   hF    the p2o plan (Nd, Nm, Nt), hq the p2q plan (Nq, Nm, Nt); both
 *         P2O_FP64 and ready, with the same Nm and Nt (else P2O_EINVAL).
 *   Kfac  device [(Nt*Nd)^2]: K after p2o_posterior_solve (its Cholesky
 *         factor in the lower triangle; the upper triangle is not read).
 *   Q     device [(Nt*Nq)][(Nt*Nd)] row-major, caller-allocated; row
 *         t*Nq + q, column i*Nd + s.
 *   Gq    device [(Nt*Nq)^2] row-major, caller-allocated.
 * Allocates temporaries (the (Nt*Nq) x (Nt*Nd) matrix F Gamma_prior Fq*,
 * plus up to ~8 GB of transform workspace) and synchronises `stream`. */
p2o_status p2o_qoi_precompute(p2o_handle hF, p2o_handle hq, const double* Kfac,
                              double prior_var, double* Q, double* Gq, void* stream);

/* Phase 4 QoI prediction from data: q[r] = Q d[r] for r < nrhs.
 *   Q  device [nq][n] row-major (from p2o_qoi_precompute: nq = Nt*Nq,
 *      n = Nt*Nd); d device [nrhs][n]; q device [nrhs][nq].
 * Stream-ordered, allocates nothing; P2O_EINVAL on null pointers or sizes
 * below 1. */
p2o_status p2o_qoi_predict(const double* Q, int64_t nq, int64_t n, const double* d, double* q,
                           int64_t nrhs, void* stream);

/* ------------------------------------------------------------ housekeeping */

/* Frees the frequency blocks, scales and workspaces; NULL-safe. */
void p2o_destroy(p2o_handle h);

/* Static description of a status code. */
const char* p2o_status_string(p2o_status s);

/* The HIP error behind the last P2O_EHIP returned on this thread. */
p2o_status p2o_last_hip_error(int* code);

/* Measurement aid: reads `bytes` of device memory at `buf` once with the
 * non-temporal 16-byte loads the block-product kernels stream their
 * frequency blocks with, and nothing else, so that the caller can time the
 * device's streaming-read ceiling (section "Peak performance" quotes the
 * paper's kernels as a fraction of memory bandwidth).
 *   buf    device, 16-byte aligned;  bytes a positive multiple of 16.
 *   sink   device [1] double; written only in the (practically impossible)
 *          case that the folded data equal a fixed pattern.
 * Stream-ordered, allocates nothing; P2O_EINVAL on bad arguments. */
p2o_status p2o_read_bandwidth(const void* buf, int64_t bytes, double* sink, void* stream);

/* Kernel timing: when enabled, p2o_apply brackets each frequency-block
 * product kernel with HIP events on `stream`.  p2o_kernel_time reads back
 * the summed milliseconds and launch count since the last reset for
 * op = P2O_F or P2O_FADJ (synchronises on the last event). */
p2o_status p2o_set_kernel_timing(p2o_handle h, int enable);
p2o_status p2o_kernel_time(p2o_handle h, p2o_op op, double* total_ms,
                           int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* P2O_H */
