/*
 * sorsvd.h - C ABI of the MI355X (gfx950) Subspace-Orbit Randomized SVD library.
 *
 * Method: Kaloorazi & de Lamare, "Subspace-Orbit Randomized Decomposition for
 * Low-rank Matrix Approximation", Sec. III, Alg. 3 (basic SOR-SVD) and Alg. 4
 * (SOR-SVD with power method), eqs. (T1), (AT1), (M), the rank-k truncated SVD
 * of M and the lift A_hat = (Q1 U~_k) S~_k (Q2 V~_k)^T.
 *
 * Conventions for every entry point
 *   - Matrices are ROW-MAJOR with a leading dimension in elements (lda >= cols).
 *   - Every matrix pointer is a DEVICE pointer (HIP global memory) unless the
 *     comment says "host". The library never allocates device memory: the
 *     caller passes a workspace of at least the size the matching
 *     *_workspace_bytes() call returns. Results depend only on the arguments.
 *     Process-wide state, all opt-in: the pass-timing events of
 *     sorsvd_pass_timing (created and freed by that call, per process), batch
 *     plans with their side streams and graphs (sorsvd_batch_create / _graph,
 *     freed by the matching destroy calls), and the 64 MiB device array that sorsvd_noalloc uses as
 *     its workspace (per device, until the process ends). The batch autotuner's
 *     cache file is read and written only when SORSVD_TUNE_CACHE names one.
 *   - `stream` is a hipStream_t (NULL = the default stream). All work is
 *     enqueued on it asynchronously; results are valid once the stream has
 *     completed. Argument errors are detected synchronously, before anything is
 *     enqueued, and reported by the return value.
 *   - Return value: SORSVD_OK or a negative sorsvd_status. Conditions found on
 *     the device (non-finite input, Jacobi sweep cap reached) are recorded in
 *     the sorsvd_info record at the start of the workspace; read it with
 *     sorsvd_read_info() after the stream has run.
 *   - Calls that share a workspace must not overlap in time.
 */
#ifndef SORSVD_H
#define SORSVD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum sorsvd_status {
  SORSVD_OK = 0,
  SORSVD_EINVAL = -1,        /* bad shape, leading dimension, null pointer or dtype */
  SORSVD_EWORKSPACE = -2,    /* workspace smaller than *_workspace_bytes() */
  SORSVD_EHIP = -3,          /* a HIP launch or runtime call failed */
  SORSVD_ENOCONV = -4,       /* (info flag) Jacobi reached its sweep cap */
  SORSVD_ENONFINITE = -5,    /* (info flag) A holds Inf or NaN */
  SORSVD_ETOL = -6,          /* sorsvd_auto: the tolerance was not met, fallback included */
  SORSVD_EUNSUPPORTED = -7   /* valid request outside what the library implements */
} sorsvd_status;

/* Element types. A's type sets the arithmetic of the passes over A:
 *   F64  -> FP64 MFMA, FP64 accumulation;
 *   F32  -> FP32 MFMA, FP32 accumulation (partials summed in FP64);
 *   BF16 -> BF16 MFMA, FP32 accumulation; the skinny operands are rounded to
 *           BF16 (with opts.refine the projection pass splits Q2 into a BF16
 *           high and low part).
 *   F16  -> IEEE binary16 A (raw 16-bit words), FP16 MFMA, FP32 accumulation;
 *           as BF16, with 11 instead of 8 significant bits in A and in the
 *           skinny operands. FP16's range (normal 2^-14 .. 65504) is covered
 *           by power-of-two column scaling: opts.col_exp gives e_j with
 *           A = A_stored diag(2^-e_j) (sorsvd_pack_f16 chooses them), and the
 *           library undoes the scaling exactly on the skinny operands and the
 *           FP64 outputs. Skinny operands are stored multiplied by 2^12 (and
 *           by 2^(min e - e_j) on row j of an A X operand) to stay clear of
 *           FP16 subnormals; the output is scaled back exactly.
 * QR, the core SVD and the lift always run in FP64. */
typedef enum sorsvd_dtype {
  SORSVD_F64 = 0,
  SORSVD_F32 = 1,
  SORSVD_BF16 = 2,
  SORSVD_DIAG = 3,
  SORSVD_F16 = 4
} sorsvd_dtype;
/* SORSVD_DIAG: A = diag(sigma), m = n, given by its diagonal: A points to n FP64
 * values on the device (lda is not used). Every pass is diag(sigma) X in FP64;
 * everything else is the FP64 path. The Gaussian Omega is rotation-invariant,
 * so a SOR-SVD of diag(sigma) is distributed exactly as one of U diag(sigma) V^T
 * with Haar U, V: this form labels the training spectra of the (k, q)
 * predictor at O(n l) per pass. No explicit residual (opts.residual) for it. */

/* Optional settings; pass NULL for the defaults (all fields 0). */
typedef struct sorsvd_opts {
  int64_t l;          /* sketch width l, k <= l <= min(m, n); 0 means l = k */
  int32_t max_sweeps; /* Jacobi sweep cap of the core SVD; 0 means 40 */
  int32_t refine;     /* BF16 / FP16 A only: 1 = projection pass with Q2 split hi+lo (with
                         pass_efficient: the last orbit product with Q1 split hi+lo) */
  int32_t residual;   /* 1 = also compute ||A - U S V^T||_F explicitly (one more pass over A,
                         FP32 MFMA for FP32 / BF16 / FP16 A, FP64 for FP64 A, FP64 accumulation) */
  int32_t split;      /* split of the contraction in the passes; 0 = automatic */
  int32_t tile;       /* BF16 / FP16 passes: 64*tile rows (columns) of A per workgroup, tile in {1,2,4};
                         0 = automatic */
  int32_t pass_efficient; /* 1 = the pass-efficient core matrix (Sec. III, eq. M_approx): 2q + 2
                             passes instead of 2q + 3. With orthonormalisation after every
                             product, Q2 spans A^T Q1, so Q1^T A = R2^T Q2^T and M_approx equals
                             M = Q1^T A Q2 in exact arithmetic; it is formed as T2^T Q2 from the
                             last orbit product T2 = A^T Q1 kept before its QR (FP64, no
                             pseudo-inverse, no pass over A). BF16 / FP16 A with refine = 1:
                             the last orbit product takes Q1 split into 16-bit hi + lo parts
                             (2 LP columns in one pass over A, the halves added in FP64), so
                             T2 carries Q1 as the refinement projection would carry Q2;
                             without refine it takes Q1 in 16 bits (M then holds Q1's 16-bit
                             rounding). The error identity stays valid. */
  const int32_t* col_exp; /* FP16 A only (else SORSVD_EUNSUPPORTED): DEVICE array of n column
                             exponents, A = A_stored diag(2^-e_j); NULL = no scaling. The
                             result (U, S, V, ||A||_F, errors) is that of A, not of A_stored.
                             |e_j| <= 256 keeps every FP64 intermediate in range; larger
                             values set flags bit 3 and the run goes on with them. */
  int32_t literal;    /* 1 = Alg. 4 as printed: T2 <- Omega, q + 1 times {T1 = A T2; T2 = A^T T1}
                         with no orthonormalisation between the products, then Q1 = qr(T1),
                         Q2 = qr(T2) and M = Q1^T A Q2. The products' condition number grows
                         as (sigma_1 / sigma_l)^(2q+2), so this mode suits well-conditioned
                         inputs only (the default orthonormalises after every product, same
                         spans in exact arithmetic by Lemma 1). Not with pass_efficient, not
                         for the DIAG type (SORSVD_EUNSUPPORTED). */
  int32_t out_f32;    /* 1 = U and V are written as FP32 (the U and V pointers are float*,
                         ldu / ldv in elements); S and everything before the output stay FP64 */
} sorsvd_opts;

/* Result record, kept by the library in the first 256 bytes of the workspace. */
typedef struct sorsvd_info {
  double a_fro;            /* ||A||_F, accumulated in FP64 during the first pass */
  double err_fro;          /* sqrt(||A||_F^2 - sum_j s_j^2) / ||A||_F (Th. 2 split) */
  double err_fro_explicit; /* ||A - U S V^T||_F / ||A||_F if opts.residual, else -1 */
  int32_t sweeps;          /* Jacobi sweeps taken by the core SVD */
  int32_t flags;           /* bit 0: sweep cap reached; bit 1: non-finite entry in A;
                              bit 2: a Cholesky-QR pivot stayed <= 0 after the shift, so its
                              column was dropped from Q (sketch columns dependent to
                              rounding: a sketch condition number near 1/u);
                              bit 3: a column exponent outside +-256 (opts.col_exp) */
  double a_noise_rel;      /* opts.residual with BF16 / FP16 A: sqrt(sum ulp(a_ij)^2 / 12) / ||A||_F,
                              the expected relative size of the rounding of A to 16 bits; the error
                              against A before rounding is about
                              sqrt(err_fro_explicit^2 - a_noise_rel^2) plus twice the
                              share of the noise the rank-k fit absorbs (see
                              sorsvd_auto). 0 otherwise */
} sorsvd_info;

/* Workspace size in bytes for sorsvd() with the same arguments. Returns 0 for
 * invalid arguments. */
size_t sorsvd_workspace_bytes(int64_t m, int64_t n, int64_t k, int32_t q,
                              int32_t a_type, const sorsvd_opts* opts);

/*
 * sorsvd - rank-k SOR-SVD of A (Alg. 3 for q = 0, Alg. 4 for q > 0).
 *
 *   A    m x n, type a_type, leading dimension lda >= n. Read only.
 *   k    target rank, 1 <= k <= min(m, n).  q >= 0 power steps.
 *   seed Philox key word of Omega: Omega[i][j] is N(0,1) draw number i + j*n of
 *        key (seed, 0) (see sorsvd_philox_normal).
 *   U    m x k FP64 (FP32 with opts.out_f32), ldu >= k.   S  k FP64 (descending).
 *   V    n x k FP64 (FP32 with opts.out_f32), ldv >= k.
 *
 * Steps (Sec. III): T1 = A Omega; Q1 = qr(T1); Q2 = qr(A^T Q1); q times
 * {Q1 = qr(A Q2); Q2 = qr(A^T Q1)}; M = Q1^T A Q2; M = U~ S~ V~^T (FP64 one-sided
 * Jacobi); U = Q1 U~_k, V = Q2 V~_k. Orthonormalising after every product
 * spans exactly what Alg. 4's unorthonormalised products span (Lemma 1).
 * Sign convention: the largest-|.| entry of each U column is positive (lowest
 * row on ties); V's column is flipped with it.
 */
int sorsvd(const void* A, int64_t lda, int32_t a_type, int64_t m, int64_t n,
           int64_t k, int32_t q, uint64_t seed,
           void* U, int64_t ldu, double* S, void* V, int64_t ldv,
           void* workspace, size_t ws_bytes, void* stream, const sorsvd_opts* opts);

/* Copy the sorsvd_info record out of `workspace` into host memory `out`,
 * after waiting for `stream`. */
int sorsvd_read_info(const void* workspace, sorsvd_info* out, void* stream);

/*
 * sorsvd_noalloc - sorsvd() that allocates nothing, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). Arguments as sorsvd(); the workspace is a
 * fixed array of SORSVD_NOALLOC_BYTES in device memory that the library holds
 * on every device it runs on until the process ends (its address is taken on
 * a device's first call). A problem whose workspace (sorsvd_workspace_bytes)
 * exceeds it returns SORSVD_EWORKSPACE before anything is enqueued. Every
 * call on a device shares that device's array: calls that overlap on one
 * device (other streams, other threads) race, and must be serialised by the
 * caller. info (host, nullable): when given, the stream is synchronised and
 * the result record copied there (leave it null under graph capture).
 */
#define SORSVD_NOALLOC_BYTES ((size_t)64 << 20)
int sorsvd_noalloc(const void* A, int64_t lda, int32_t a_type, int64_t m, int64_t n,
                   int64_t k, int32_t q, uint64_t seed,
                   void* U, int64_t ldu, double* S, void* V, int64_t ldv,
                   void* stream, const sorsvd_opts* opts, sorsvd_info* info);

/*
 * sorsvd_pack_f16 - FP16 storage of an FP32 / FP64 matrix with power-of-two
 * column scaling (the input form of SORSVD_F16 with opts.col_exp). Not part
 * of the method: it extends the reduced-precision storage of A to FP16's
 * range.
 *
 *   A        m x n, a_type SORSVD_F32 or SORSVD_F64 (else SORSVD_EUNSUPPORTED),
 *            leading dimension lda >= n. Read only.
 *   out      m x n FP16 (raw binary16 words), leading dimension ldo >= n:
 *            out_ij = fp16(A_ij 2^e_j), rounded once to nearest-even.
 *   col_exp  n int32: e_j = 14 - floor(log2 max_i |A_ij|), clamped to
 *            [-256, 256]; 0 for a column without a finite nonzero entry. Every
 *            column's largest entry lands in [2^14, 2^15].
 * Non-finite entries are ignored when choosing e_j and stored as Inf / NaN.
 * Two kernels on `stream`; no workspace. SORSVD_EINVAL for bad shapes or
 * leading dimensions, or null pointers with m, n > 0.
 */
int sorsvd_pack_f16(const void* A, int64_t lda, int32_t a_type, int64_t m, int64_t n, uint16_t* out,
                    int64_t ldo, int32_t* col_exp, void* stream);

/*
 * sorsvd_philox_normal - the Gaussian draw of Alg. 3 / Alg. 4 step 1.
 * out (device, FP64) is rows x cols COLUMN-major with leading dimension rows:
 * element (i, j) is draw e = i + j*rows of key (seed, stream_id): Philox4x64-10
 * block with counter (e / 4, 0, word2, 0), Box-Muller pair of that block, member
 * e % 4. Bitwise equal to the CPU reference of the same definition.
 */
int sorsvd_philox_normal(uint64_t seed, uint64_t stream_id, uint64_t word2,
                         int64_t rows, int64_t cols, double* out, void* stream);

/*
 * Single steps of the path, for callers that compose their own pipeline and
 * for per-step checks. Skinny operands are FP64 row-major with leading
 * dimension l; they are rounded to A's compute type inside the pass (FP16:
 * after the 2^12 lift, without column exponents; BF16 and FP16 projections
 * split Q2 into high and low parts).
 *
 * sorsvd_step_sketch: T (m x l) = A X, X n x l           (eq. T1; Alg. 4 T1 update)
 * sorsvd_step_orbit:  T (n x l) = A^T Y, Y m x l         (eq. AT1; Alg. 4 T2 update)
 * sorsvd_step_qr:     T (rows x l) = Q R, Q rows x l orthonormal, R l x l upper
 *                     triangular with positive diagonal (QR step of Alg. 3/4).
 *                     Q may alias T. Requires l <= rows.
 * sorsvd_step_project: M (l x l) = Q1^T A Q2              (eq. M)
 * sorsvd_step_core_svd: M (l x l) = U~ diag(s) V~^T, descending; writes the
 *                     first k columns of U~ and V~ (l x k each) and s (k).
 * Each needs the workspace size returned by sorsvd_step_workspace_bytes(m, n, l, a_type).
 */
size_t sorsvd_step_workspace_bytes(int64_t m, int64_t n, int64_t l, int32_t a_type);
int sorsvd_step_sketch(const void* A, int64_t lda, int32_t a_type, int64_t m, int64_t n,
                       const double* X, int64_t l, double* T,
                       void* workspace, size_t ws_bytes, void* stream);
int sorsvd_step_orbit(const void* A, int64_t lda, int32_t a_type, int64_t m, int64_t n,
                      const double* Y, int64_t l, double* T,
                      void* workspace, size_t ws_bytes, void* stream);
int sorsvd_step_qr(const double* T, int64_t rows, int64_t l, double* Q, double* R,
                   void* workspace, size_t ws_bytes, void* stream);
int sorsvd_step_project(const void* A, int64_t lda, int32_t a_type, int64_t m, int64_t n,
                        const double* Q1, const double* Q2, int64_t l, double* M,
                        void* workspace, size_t ws_bytes, void* stream);
int sorsvd_step_core_svd(const double* M, int64_t l, int64_t k, double* Ut, double* s,
                         double* Vt, int32_t max_sweeps,
                         void* workspace, size_t ws_bytes, void* stream);

/*
 * Profiling aid (not part of the method). sorsvd_pass_timing(1, capacity)
 * creates 2*capacity HIP events; from then on every launch of the pass kernel
 * over A (the sketch, orbit and projection products) is bracketed by a pair of
 * events recorded on the call's stream, until `capacity` launches have been
 * recorded. sorsvd_pass_timing_read() waits for the recorded events and
 * returns the summed kernel time in ms, the number of launches, and the
 * algorithmic bytes of A (m n element-size per launch) and flops (2 m n l per
 * launch) they covered, then starts a new count. sorsvd_pass_timing(0, 0)
 * destroys the events. Process-wide; not for concurrent use from several threads.
 */
int sorsvd_pass_timing(int32_t enable, int32_t capacity);
int sorsvd_pass_timing_read(double* total_ms, int64_t* launches, double* bytes, double* flops);

/*
 * Batched SOR-SVD: many independent problems of uneven sizes (each one is
 * Alg. 3 for q = 0, Alg. 4 for q > 0, exactly as sorsvd() computes it), run
 * together so that every step of the method is one launch over the whole batch.
 *
 * One problem. A (m x n, row-major, lda >= n, batch dtype) is read only; U
 * (m x k, ldu >= k), S (k) and V (n x k, ldv >= k) are FP64 outputs with the
 * same meaning, sign convention and Omega draw (key (seed, 0)) as sorsvd().
 * l = sketch width (0 means k; k <= l <= min(m, n), l rounded up to a multiple
 * of 16 must be <= 128). q >= 0 power steps, per problem.
 */
typedef struct sorsvd_problem {
  const void* A;
  int64_t lda, m, n;
  int32_t k, l, q, reserved;
  uint64_t seed;
  double* U;
  int64_t ldu;
  double* S;
  double* V;
  int64_t ldv;
} sorsvd_problem;

/* Host-side plan of a batch (opaque; created and freed by the library). */
typedef struct sorsvd_batch sorsvd_batch;

/*
 * sorsvd_batch_create - validate `count` problems (1..65535) and build the
 * plan: per-step work lists ordered largest item first, the workspace layout
 * and the default launch configuration (or the one stored for this batch
 * shape in the tuning cache file named by the environment variable
 * SORSVD_TUNE_CACHE). a_type: SORSVD_F32, SORSVD_F64 or SORSVD_DIAG (BF16 ->
 * SORSVD_EUNSUPPORTED). opts: NULL, or only max_sweeps set (other fields
 * non-zero -> SORSVD_EUNSUPPORTED). On success *out holds the plan and
 * *ws_bytes the device workspace it needs. The problem array is copied; the
 * device buffers it points to must stay valid while the plan is used.
 */
int sorsvd_batch_create(int32_t count, const sorsvd_problem* problems, int32_t a_type,
                        const sorsvd_opts* opts, sorsvd_batch** out, size_t* ws_bytes);

/* Bind the plan to a device workspace (256-byte aligned, >= *ws_bytes) and
 * copy the problem table and work lists into it; waits for `stream`. Must be
 * called once before run, autotune or graph; again after a new workspace. */
int sorsvd_batch_upload(sorsvd_batch* b, void* workspace, size_t ws_bytes, void* stream);

/* Enqueue the whole batch on `stream`: Omega, 2q + 3 passes over each A with
 * their Cholesky QRs, projection, core SVDs, lifts, sign convention and the
 * result records. Problems with smaller q sit out the later power steps.
 * The launches of one step that serve problems of different sketch widths
 * run on side streams of the plan, forked from `stream` and joined back to it
 * before the next step (the plan creates them at its first run, on the
 * device current then, and frees them with the plan); the work is complete
 * when `stream` is. */
int sorsvd_batch_run(const sorsvd_batch* b, void* workspace, void* stream);

/* Launch configuration of the three pass kinds (sketch, orbit, projection):
 * config[2i] = tile height in units of 64 rows (1 or 2), config[2i + 1] =
 * persistent workgroups. Results are bitwise the same for every configuration. */
int sorsvd_batch_get_config(const sorsvd_batch* b, int32_t* config /* host, 6 */);
int sorsvd_batch_set_config(sorsvd_batch* b, const int32_t* config /* host, 6 */);

/* Time each pass kind over tile heights {1, 2} x grids {256 .. 4096} with HIP
 * events on `stream` (synchronous), keep the fastest, append it to the tuning
 * cache file if SORSVD_TUNE_CACHE is set, write it to config_out (host, 6
 * entries, may be NULL), and leave the results of a complete run behind. */
int sorsvd_batch_autotune(sorsvd_batch* b, void* workspace, void* stream, int32_t* config_out);

/* Copy the `count` result records (same fields as sorsvd_info) into host
 * memory `out`, after waiting for `stream`. */
int sorsvd_batch_read_info(const sorsvd_batch* b, sorsvd_info* out, void* stream);

/* Capture the launch sequence of sorsvd_batch_run (no memsets, no allocations)
 * in a HIP graph on a library-created stream and instantiate it: *graph_exec
 * receives a hipGraphExec_t. Replays with sorsvd_graph_launch recompute the
 * batch from the current contents of the A buffers; free with
 * sorsvd_graph_destroy. The plan's configuration at capture time is frozen
 * into the graph. Pass timing (sorsvd_pass_timing) does not see graph replays. */
int sorsvd_batch_graph(const sorsvd_batch* b, void* workspace, void** graph_exec);
int sorsvd_graph_launch(void* graph_exec, void* stream);
int sorsvd_graph_destroy(void* graph_exec);

/* Number of problems of a plan (0 for NULL). */
int32_t sorsvd_batch_count(const sorsvd_batch* b);

/* Free a plan and its side streams (NULL is allowed). Does not touch device
 * memory. */
void sorsvd_batch_destroy(sorsvd_batch* b);

/*
 * Learned choice of (k, q) for a target tolerance (extension of the method:
 * the error check of the method is the judge, fixed (k, q) the fallback).
 *
 * sorsvd_probe_features: the probe sketch Y0 = A Omega[:, :l], l = min(128, m, n),
 *   Omega of key (seed, 0) as in sorsvd(); s_j = singular values of Y0 (Cholesky
 *   QR of Y0, then the core SVD of R); features (device, 128 FP32):
 *   f_j = clamp(log10(s_j / s_1) / 8, -1, 0) for j < l, -1 beyond.
 *   Workspace: sorsvd_probe_workspace_bytes(m, n, a_type). FP16 A:
 *   SORSVD_EUNSUPPORTED here and in sorsvd_auto (workspace sizes 0).
 *
 * The network: 128 -> 64 (tanh) -> 64 (tanh) -> 4, FP32, parameters one flat
 * device vector of sorsvd_mlp_param_count() = 12676 values: W1 (64 x 128,
 * row-major), b1 (64), W2 (64 x 64), b2, W3 (4 x 64), b3 (4). Output y_q
 * predicts log2 of the smallest k (= l) whose SOR-SVD with q power steps meets
 * the tolerance, q = 0..3.
 *   sorsvd_mlp_forward:  Y (batch x 4) from X (batch x 128), row-major.
 *   sorsvd_mlp_backward: forward, then grad (12676) of the loss
 *       mean over batch x 4 of (y - T)^2, and the loss itself (device, 1 float).
 *   sorsvd_mlp_adam: one Adam step (step >= 1) on params with moments m, v.
 *   sorsvd_mlp_train_step: backward + Adam (beta1 0.9, beta2 0.999, eps 1e-8).
 *   work: device scratch of sorsvd_mlp_work_floats(batch) floats (activations;
 *   backward and train_step keep them there between their kernels).
 *
 * sorsvd_auto: probe -> network -> (k, q) -> SOR-SVD -> judge -> fallback.
 *   For each q the network's width is taken with 25% head-room (60% for BF16
 *   A), rounded up to a multiple of 8 and capped at min(1024, m, n); a q whose
 *   raw prediction exceeds that cap is dropped. Among the rest the (k, q) of
 *   the least modelled run time wins: P passes (P = 2q + 3, 2q + 2 for BF16 A,
 *   whose runs take the refinement split and the pass-efficient core matrix,
 *   as with opts.refine = opts.pass_efficient = 1), each the larger of its
 *   bytes at 5 TB/s and its flops at the MFMA rate reached, plus the FP64
 *   Cholesky QRs and ~1e-11 k^3 s of core SVD. Judge: the error identity
 *   (FP32/FP64), or for BF16 the explicit residual corrected for the rounding
 *   of A to BF16: sqrt(err_fro_explicit^2 - (1 - 2 rho) a_noise_rel^2) with
 *   rho = min(1, 2.5 k (m^-1/2 + n^-1/2)^2), an allowance for the share of
 *   the rounding noise a rank-k fit absorbs (2.5 times the i.i.d. share;
 *   measured shares near the tolerance stay below 1.9 times it), so that the
 *   judge errs on the safe side. BF16 runs take q >= 1 (with q = 0 the BF16
 *   rounding of the skinny operand leaves a subspace error near 1e-3). If the
 *   judge rejects, or no predicted width fits, the fixed ladder (256, 2),
 *   (512, 2), (1024, 2) (widths capped at min(m, n)) runs until the judge
 *   accepts. params = NULL skips the network (the ladder only).
 *   With the network, the first run starts from the probe: Omega is nested in
 *   its width and Cholesky QR keeps column prefixes, so the leading k columns
 *   of the probe's Q are Q1 of the run's first sketch (one pass and one QR
 *   fewer) when k <= 128.
 *   U, V need ldu, ldv >= min(1024, m, n) (the first k_used columns are the
 *   result), S as many entries. Synchronous: waits for `stream`. Returns
 *   SORSVD_OK, or SORSVD_ETOL with the fallback's result left in U, S, V.
 *   Workspace: sorsvd_auto_workspace_bytes(m, n, a_type).
 */
typedef struct sorsvd_auto_info {
  int32_t k_used, q_used;  /* the (k, q) of the returned result */
  int32_t used_fallback;   /* 1 if the result is the fallback's */
  int32_t runs;            /* SOR-SVDs run (1 or 2) */
  double err;              /* the judge's error of the returned result */
  double k_pred[4];        /* network widths 2^y_q before head-room (0 without params) */
  int32_t flags;           /* sorsvd_info.flags of the returned result */
  int32_t reserved;
  double err_stored;       /* explicit error against the stored A before the
                              16-bit rounding-noise correction (the judge's
                              input for BF16 A; equal to err otherwise) */
} sorsvd_auto_info;

size_t sorsvd_probe_workspace_bytes(int64_t m, int64_t n, int32_t a_type);
int sorsvd_probe_features(const void* A, int64_t lda, int32_t a_type, int64_t m, int64_t n, uint64_t seed,
                          float* features, void* workspace, size_t ws_bytes, void* stream);
int32_t sorsvd_mlp_param_count(void);
size_t sorsvd_mlp_work_floats(int32_t batch);
int sorsvd_mlp_forward(const float* params, const float* X, int32_t batch, float* Y, float* work, void* stream);
int sorsvd_mlp_backward(const float* params, const float* X, const float* T, int32_t batch, float* grad,
                        float* loss, float* work, void* stream);
int sorsvd_mlp_adam(float* params, const float* grad, float* m, float* v, int64_t step, float lr, float beta1,
                    float beta2, float eps, void* stream);
int sorsvd_mlp_train_step(float* params, float* m, float* v, const float* X, const float* T, int32_t batch,
                          int64_t step, float lr, float* grad, float* loss, float* work, void* stream);
size_t sorsvd_auto_workspace_bytes(int64_t m, int64_t n, int32_t a_type);
int sorsvd_auto(const void* A, int64_t lda, int32_t a_type, int64_t m, int64_t n, uint64_t seed, double tol,
                const float* params, double* U, int64_t ldu, double* S, double* V, int64_t ldv,
                void* workspace, size_t ws_bytes, void* stream, sorsvd_auto_info* out);

/*
 * sorsvd_predict_kq - the (k, q) that sorsvd_auto would run first, without
 * running it: the probe sketch (one pass over A), its features and the
 * network (params as for sorsvd_auto), then the q of the least modelled time
 * among the predicted widths (with head-room) that fit min(1024, m, n).
 * The network was trained for tol = 1e-3 (tol must be > 0; it does not
 * rescale the prediction). k_pred (host, nullable): the 4 raw predicted
 * widths 2^y_q, q = 0..3. Returns SORSVD_OK, or SORSVD_ETOL with the first
 * rung of the fixed ladder (256, 2) when no predicted width fits.
 * Workspace: sorsvd_auto_workspace_bytes(m, n, a_type). Synchronises the
 * stream (the prediction is read back).
 */
int sorsvd_predict_kq(const void* A, int64_t lda, int32_t a_type, int64_t m, int64_t n, uint64_t seed,
                      const float* params, double tol, int64_t* k_out, int32_t* q_out, double* k_pred,
                      void* workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Theorem bounds for one draw of Omega (Sec. IV: Th. 4 and Th. 5,
 * deterministic in Omega; Th. 6 and Th. 7, expectations over Omega), for a
 * matrix whose right singular vectors are known (a synthetic A =
 * U diag(sigma) V^T, or V from a reference SVD). With r = l - p, V1 the first
 * r right singular vectors, Omega1 = V1^T Omega and Omega2 = V2^T Omega (the
 * partition of Sec. IV-A); Omega is the FP64 draw that sorsvd() makes with
 * the same seed (for FP32 / 16-bit A the run uses that draw rounded).
 *
 *   V1     device, n x r row-major (ldv >= r): the first r right singular
 *          vectors of A.
 *   sigma  host, nsig >= max(r, k) + 1 singular values of A, descending (all
 *          min(m, n) of them for the Frobenius-norm floor of Th. 1).
 *   k, q   the rank and power steps of the run; 2 <= p + k <= l <= n.
 *   th4    host, nullable: k lower bounds on sigma_j(A_hat) (Th. 4).
 *   th6    host, nullable: k lower bounds on E sigma_j(A_hat) (Th. 6; NaN
 *          unless p >= 2).
 *   out    host: ||Omega2||_2, ||Omega1^+||_2 and the error upper bounds of
 *          Th. 5 and Th. 7 (NaN unless p >= 2) in the Frobenius and 2-norm.
 *          Th. 5 takes tau = (sigma_k / sigma_{l-p+1}) beta with the power
 *          method (the printed tau is not dimensionless).
 * ||Omega2||_2 comes from Omega^T Omega - Omega1^T Omega1 (V orthogonal), so
 * V2 is never needed; ||Omega1^+||_2 = 1 / sigma_min(Omega1). Workspace:
 * sorsvd_bounds_workspace_bytes(n, l, p). Synchronises the stream. Returns
 * SORSVD_EINVAL for bad sizes or a sigma that is not descending and
 * nonnegative with sigma_k > 0.
 */
typedef struct sorsvd_bounds_info {
  double omega2_norm;      /* ||Omega2||_2 */
  double omega1_pinv_norm; /* ||Omega1^+||_2 */
  double th5_fro, th5_2;   /* Th. 5 upper bounds on ||A - A_hat|| */
  double th7_fro, th7_2;   /* Th. 7 upper bounds on E ||A - A_hat|| */
} sorsvd_bounds_info;

size_t sorsvd_bounds_workspace_bytes(int64_t n, int64_t l, int64_t p);
int sorsvd_bounds(const double* V1, int64_t ldv, int64_t n, int64_t l, int64_t p, int64_t k, int32_t q,
                  uint64_t seed, const double* sigma, int64_t nsig, double* th4, double* th6,
                  sorsvd_bounds_info* out, void* workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Robust PCA by the ALM-SOR-SVD iteration (Sec. V, "Robust Principal
 * Component Analysis", Table III): split X = L + S (L low-rank, S sparse) by
 * the inexact augmented-Lagrange-multiplier method with a SOR-SVD of width l
 * and q power steps in place of the SVD of every iteration:
 *   (U, z, V) = SOR-SVD(X - S + Y / mu),  L = U shrink_{1/mu}(z) V^T,
 *   S = shrink_{lambda/mu}(X - L + Y / mu),  Y += mu (X - L - S),
 *   mu = min(1.5 mu, mu_bar),
 * with shrink_e(x) = sgn(x) max(|x| - e, 0), lambda = 1 / sqrt(max(m, n)),
 * Y_0 = X / max(||X||_2, ||X||_max / lambda), mu_0 = 1.25 / ||X||_2,
 * mu_bar = 1e7 mu_0, S_0 = 0 (the inexact ALM's initial values, which the
 * paper adopts; the table's max in the mu update is read as the capped min).
 * ||X||_2 is estimated by a SOR-SVD of X of width min(32, m, n) with eight
 * power steps. Iteration i draws Omega with seed + i. It stops when
 * ||X - L - S||_F < tol ||X||_F or after max_iter iterations.
 *   X: m x n FP64 row-major device array (ldx >= n), read only.
 *   L, S: m x n FP64 row-major device outputs (ld >= n); S also holds the
 *     iterate during the run.
 *   l: 1 <= l <= min(m, n, 128) (the paper's experiments use l = 2 rank(L));
 *   q >= 0; tol > 0; max_iter >= 1.
 *   workspace: sorsvd_rpca_workspace_bytes(m, n, l, q) bytes, 256-byte
 *   aligned; the library synchronises `stream` once per iteration to read the
 *   residual.
 * Returns SORSVD_OK (tolerance met), SORSVD_ETOL (max_iter reached; L and S
 * hold the last iterate), or an error status; *out is filled in both of the
 * first two cases.
 * ------------------------------------------------------------------------ */
typedef struct sorsvd_rpca_info {
  int32_t iters;   /* iterations taken */
  int32_t rank;    /* singular values kept by the last thresholding */
  int64_t nnz_s;   /* nonzero entries of S */
  double xi;       /* ||X - L - S||_F / ||X||_F after the last iteration */
  double lambda;   /* 1 / sqrt(max(m, n)) */
  double norm2;    /* the estimate of ||X||_2 used for mu_0 and Y_0 */
} sorsvd_rpca_info;

size_t sorsvd_rpca_workspace_bytes(int64_t m, int64_t n, int64_t l, int32_t q);
int sorsvd_rpca(const double* X, int64_t ldx, int64_t m, int64_t n, int64_t l, int32_t q, uint64_t seed,
                double tol, int32_t max_iter, double* L, double* S, int64_t ld, void* workspace, size_t ws_bytes,
                void* stream, sorsvd_rpca_info* out);

/* Human-readable text of a status code (static storage). */
const char* sorsvd_status_string(int status);

/* Library version string (static storage). */
const char* sorsvd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SORSVD_H */
