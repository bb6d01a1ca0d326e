/*
 * tucker.h -- C ABI of the MI355X (gfx950) Tucker-ALS / HOOI library.
 *
 * What is computed (Sharma & Grover, arXiv 2104.04726, Sec. III-B):
 *   Given an order-N tensor X (s_1 x ... x s_N) and ranks R_n, find a core G
 *   (R_1 x ... x R_N) and factors U_n (s_n x R_n, orthonormal columns) with
 *   X ~ G x_1 U_1 ... x_N U_N                                  (eq. (1)-(2)),
 *   starting from the truncated HOSVD                          (Sec. III-B.1, eq. (3)-(7))
 *   and refining by ALS sweeps (HOOI): for n = 1..N,
 *   Y = X x_{m != n} U_m^T, U_n <- leading R_n eigenvectors of Y_(n) Y_(n)^T
 *                                                              (eq. (8) and the text after it).
 *
 * Conventions shared by every entry point:
 *   - All tensors and matrices are dense, row-major (C order): mode 1 varies slowest.
 *     U_n is s_n x R_n row-major, the core is R_1 x ... x R_N row-major.
 *   - Pointers documented as "device" point to GPU memory on the context's device;
 *     they are owned by the caller, and inputs are only read.  Pointers documented as
 *     "host" are ordinary CPU memory.
 *   - Work is enqueued on the context's stream (tucker_options.stream; NULL = the device's
 *     default (null) stream).  Functions that return host values (fit, sweeps) synchronise that
 *     stream before returning; the others are stream-ordered and return immediately.
 *   - Every function returns a tucker_status.  Arguments are validated on the host before
 *     any device work; TUCKER_ERR_INVALID_ARG leaves all outputs untouched.  After any
 *     other error the outputs are unspecified and tucker_last_error() describes the cause.
 *   - A context is not thread-safe: use one per thread.
 */
#ifndef TUCKER_MI355X_H
#define TUCKER_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TUCKER_MAX_ORDER 8

/* Opaque context: owns a device workspace, a stream binding and the last statistics. */
typedef struct tucker_ctx tucker_ctx;

typedef enum {
    TUCKER_OK = 0,
    TUCKER_ERR_INVALID_ARG = 1,   /* argument rejected by host-side validation            */
    TUCKER_ERR_OUT_OF_MEMORY = 2, /* device allocation failed or exceeds hbm_budget_bytes */
    TUCKER_ERR_DEVICE = 3,        /* no usable GPU, or a HIP runtime error                */
    TUCKER_ERR_NUMERICAL = 4,     /* non-finite input norm, or an unrecoverable breakdown */
    TUCKER_ERR_UNSUPPORTED = 5,   /* a valid request the library does not implement       */
    TUCKER_ERR_TIMEOUT = 6        /* tucker_server_wait: the request has not finished yet */
} tucker_status;

/* Operand precision of the TTM and Gram contractions of the sweeps (the precision variants of the
 * HOOI sweep, eq. (8)).  Accumulation is always FP32; the orthogonalisation and the norms are FP64
 * and the T-HOSVD start uses the FP32 tensor whatever the choice.  BF16 / FP16: X and the sweep
 * intermediates are stored in that type (round to nearest even).  FP8_E4M3: X is stored in the OCP
 * E4M3 format with one FP32 scale per slice of the two trailing modes (amax / 448) and multiplied
 * on the FP8 matrix cores in the two full-tensor products; the intermediates are BF16.  After the
 * reduced-precision sweeps, refine_sweeps FP32 sweeps run on the FP32 tensor.  Reduced precision
 * needs an order-4 tensor whose two leading modes are larger than 64 and whose two trailing modes
 * are small (the image stacks); other shapes return TUCKER_ERR_UNSUPPORTED. */
typedef enum {
    TUCKER_FP32 = 0,
    TUCKER_BF16 = 1,
    TUCKER_FP16 = 2,
    TUCKER_FP8_E4M3 = 3
} tucker_precision;

/* How the factors are initialised (Sec. III-B.1). */
typedef enum {
    TUCKER_START_THOSVD = 0,     /* truncated HOSVD: U_n = leading R_n eigenvectors of X_(n) X_(n)^T,
                                    every mode from the unprojected tensor (eq. (6)-(7))      */
    TUCKER_START_STHOSVD = 1     /* sequentially truncated ("interlaced") HOSVD, the cheaper start
                                    named after eq. (7): modes in ascending order, U_n from the
                                    Gram of X x_1 U_1^T ... x_{n-1} U_{n-1}^T                  */
} tucker_start;

typedef struct {
    int device;                  /* HIP device ordinal                                        */
    void* stream;                /* hipStream_t owned by the caller; NULL = default stream    */
    tucker_precision precision;  /* contraction operand precision of the sweeps               */
    int refine_sweeps;           /* FP32 sweeps appended after reduced-precision sweeps       */
    int inner_iters;             /* orthogonal-iteration steps per large-mode update (>= 1);
                                    with inner_tol > 0, the most steps an update may take     */
    int init_iters;              /* cold-start orthogonal-iteration steps for the T-HOSVD of a
                                    large mode (from a seeded random basis): without
                                    oversampling, directions whose eigenvalue gap is wide
                                    converge, those at a nearly degenerate rank boundary need
                                    not, so the start is the T-HOSVD up to rotations inside
                                    that boundary; with inner_tol > 0, the most steps a start
                                    may take                                                  */
    double inner_tol;            /* 0: fixed step counts.  > 0: each large-mode update, cold or
                                    warm, forms its Gram S and iterates until the invariant-
                                    subspace residual ||S U - U (U^T S U)||_F <= inner_tol ||S||_F
                                    (checked on the host after every step, so sweeps are then
                                    launched one kernel at a time); steps taken are reported in
                                    tucker_stats                                               */
    int use_graphs;              /* 1: run the first sweep directly, capture the second as a HIP
                                    graph and replay it for every later sweep (needs a non-NULL
                                    stream, timing 0 and tol 0; otherwise the sweeps are launched
                                    one kernel at a time).  Results equal the direct launches'. */
    size_t hbm_budget_bytes;     /* workspace cap; 0 = no cap                                 */
    uint64_t seed;               /* seed of the cold-start basis (counter-based generator)    */
    int timing;                  /* 1: time the sweep stages with HIP events (tucker_stats).
                                    Each timed stage records two events on the stream, and each
                                    costs the device a few microseconds of idle time between
                                    kernels, so timing slows a sweep by up to about 10%        */
    int64_t wait_spin_limit;     /* bound of every wait inside the Cholesky task graph, in sleep
                                    steps of about 64 cycles; 0 = the default (2^24, about half
                                    a second).  A wait that reaches it gives up, the kernel
                                    finishes normally and the call returns TUCKER_ERR_DEVICE.
                                    Tiny values exist to exercise that error path.            */
    tucker_start start;          /* initialisation of the factors (default TUCKER_START_THOSVD) */
    int autotune;                /* 1: launch choices not yet fixed in this process (FP32 and
                                    reduced-precision product tile shapes, FP64 Gram split
                                    count) are measured on the device
                                    on first use and the fastest kept, unless the built-in
                                    heuristic's choice is within 3% of it (10% for the Gram split
                                    count, whose candidates round differently, and for the
                                    reduced-precision LDS staging) (tucker_autotune_dump);
                                    0: such choices take the built-in heuristic.  Either way the
                                    first call of a shape fixes its choice for the process.     */
    double pp_tol;               /* > 0: pairwise-perturbation sweeps (Sec. III-B, eq. (9)-(13)).
                                    Ordinary sweeps run until the largest subspace distance
                                    ||U U^T - V V^T||_F / sqrt(2R) between consecutive factors is
                                    below pp_tol; then, around those factors, the tensors of the
                                    updates are taken to first order in the factor changes from
                                    operators formed once (X is not read), while every factor stays
                                    within pp_tol of the reference; the returned core and fit are
                                    exact.  FP32 sweeps (tol = 0) of order-4 stacks whose third
                                    mode is kept at full rank (identity factor) only, else
                                    TUCKER_ERR_UNSUPPORTED.  0 (default): ordinary sweeps.        */
    uint32_t timing_stages;      /* timing = 1: bit s set times stage s (tucker_stage) only;
                                    0 (default) times every stage                              */
    int oversample;              /* p >= 0: the cold start of a large mode (T-HOSVD or ST-HOSVD
                                    start) iterates on Rc = min(s_n, R_n + p) columns and ends with
                                    a Rayleigh-Ritz step: B = U^T S U (Rc x Rc) is diagonalised in
                                    FP64 (block Jacobi) and U_n is spanned by the Ritz vectors of
                                    its R_n largest Ritz values.  The leading directions then
                                    converge at the rate lam_{Rc+1} / lam_i instead of
                                    lam_{R+1} / lam_i, which resolves close rank boundaries.  Rc
                                    must not exceed 1024 (else TUCKER_ERR_UNSUPPORTED).  The
                                    eigensolver checks its convergence on the host after each
                                    sweep; the two large modes' eigensolvers run side by side on
                                    two streams.  0 (default): no oversampling, no Rayleigh-Ritz. */
} tucker_options;

/* Stages timed when tucker_options.timing is set (names follow a sweep of an order-4 stack
 * X (s1 x s2 x s3 x s4) with small trailing modes; single-kernel stages are marked *). */
typedef enum {
    TUCKER_STAGE_PASS_A = 0,     /* * T34 = X x3 U3^T x4 U4^T, the first full-tensor pass      */
    TUCKER_STAGE_TTM_Y1 = 1,     /* * Y1 = T34 x2 U2^T                                         */
    TUCKER_STAGE_GRAM_1 = 2,     /*   mode-1 Gram product, or with one inner step the products  */
                                 /*   W = Y1 x1 U1^T and Y1_(1) W_(1)^T (S U without forming S) */
    TUCKER_STAGE_OI_1 = 3,       /*   orthogonal iteration + CholeskyQR2 of mode 1             */
    TUCKER_STAGE_TTM_Y2 = 4,     /* * Y2 = T34 x1 U1^T                                         */
    TUCKER_STAGE_GRAM_2 = 5,     /*   mode-2 Gram product, or the two products as for mode 1   */
    TUCKER_STAGE_OI_2 = 6,       /*   orthogonal iteration + CholeskyQR2 of mode 2             */
    TUCKER_STAGE_PASS_C1 = 7,    /* * T1 = X x1 U1^T, the second full-tensor pass              */
    TUCKER_STAGE_TTM_C2 = 8,     /* * T12 = T1 x2 U2^T                                         */
    TUCKER_STAGE_SMALL = 9,      /*   fibre Gram and the updates of the small modes            */
    TUCKER_STAGE_CORE = 10,      /*   core, ||G||^2 and the per-sweep fit                      */
    TUCKER_STAGE_REDUCE = 11,    /*   Gram split reductions                                    */
    TUCKER_NUM_STAGES = 12
} tucker_stage;

/* Statistics of the last tucker_decompose* call on a context (host values). */
typedef struct {
    double init_ms;              /* T-HOSVD initialisation, GPU time                          */
    double sweeps_ms;            /* all ALS sweeps, GPU time                                  */
    double final_fit_ms;         /* exact-residual fit and output copies, GPU time            */
    double fit_gram;             /* last fit from ||X||^2 - ||G||^2 (cheap, FP32 core)        */
    int sweeps;                  /* sweeps performed (reduced precision: excluding refinement) */
    int refine_sweeps;           /* FP32 refinement sweeps after reduced-precision ones       */
    int chol_shifts;             /* Cholesky pivots that needed the shifted fallback          */
    int orth_second_passes;      /* CholeskyQR passes run because one pass left ||Q^T Q - I||
                                    above the FP64 threshold (the rest were skipped on device) */
    int wait_timeouts;           /* Cholesky task-graph calls in which a wait gave up (the call
                                    then returned TUCKER_ERR_DEVICE)                           */
    int oi_steps_init;           /* orthogonal-iteration steps of the start (all large modes) */
    int oi_steps_sweeps;         /* orthogonal-iteration steps of the sweeps (all large modes) */
    double oi_residual_max;      /* inner_tol > 0: largest final ||S U - U U^T S U||_F / ||S||_F
                                    over the updates of the call (0 otherwise)                */
    int pp_sweeps;               /* pairwise-perturbation sweeps among the sweeps (pp_tol > 0) */
    int pp_refs;                 /* reference points (operator sets) formed                   */
    int rr_sweeps;               /* oversample > 0: block-Jacobi sweeps of the start's
                                    Rayleigh-Ritz steps (all large modes)                      */
    size_t workspace_bytes;      /* device workspace held by the context                      */
    double stage_ms[TUCKER_NUM_STAGES];   /* summed GPU time per stage (timing = 1)           */
    int stage_calls[TUCKER_NUM_STAGES];   /* number of timed occurrences per stage            */
} tucker_stats;

/* Fills *o with the defaults: device 0, default stream, FP32, refine_sweeps 1,
 * inner_iters 1, init_iters 20, seed 0x5eed. */
void tucker_default_options(tucker_options* o);

/* Host-only validation of a decomposition request (no GPU needed).  Rules:
 * 2 <= ndim <= 8; dims[n] >= 1; 1 <= ranks[n] <= dims[n]; ranks[n] <= prod_{m != n} ranks[m]
 * (otherwise the Gram of Y_(n) has rank < R_n and its leading subspace is not determined);
 * max_iters >= 0; tol >= 0 and not NaN.  dims/ranks: host arrays of ndim entries. */
tucker_status tucker_validate(int ndim, const int64_t* dims, const int64_t* ranks,
                              int max_iters, double tol);

/* Host-only: device workspace (bytes) a decomposition of this shape needs with the default
 * options (no oversampling, no pairwise perturbation); those options need more. */
tucker_status tucker_workspace_size(int ndim, const int64_t* dims, const int64_t* ranks,
                                    tucker_precision precision, size_t* bytes);

/* Creates a context on opts->device (opts may be NULL for the defaults).  Returns
 * TUCKER_ERR_DEVICE when no GPU is usable.  *out receives the context (caller destroys). */
tucker_status tucker_create(const tucker_options* opts, tucker_ctx** out);

/* Frees the context's workspace and stream.  NULL is accepted. */
tucker_status tucker_destroy(tucker_ctx* ctx);

/* Tucker decomposition by HOOI (T-HOSVD start, then up to max_iters sweeps).
 *   tensor   device, prod(dims) floats, read-only.
 *   dims     host, ndim entries; ranks host, ndim entries.
 *   max_iters number of sweeps; 0 returns the start (T-HOSVD, or ST-HOSVD per tucker_options.start;
 *            large modes by init_iters steps of orthogonal iteration, see tucker_options).
 *   tol      stop early when |fit_k - fit_{k-1}| < tol (tol = 0: run all sweeps).  With tol > 0
 *            each sweep's fit is the explicit residual fit (one more expanding pass per sweep);
 *            with tol = 0 it is the cheaper 1 - sqrt(||X||^2 - ||G||^2) / ||X|| from the FP32 core,
 *            whose error is that of ||G||^2 amplified by the cancellation (about 3e-5 at 1080p).
 *   core     device, prod(ranks) floats (output).
 *   factors  host array of ndim device pointers; factors[n] receives dims[n]*ranks[n] floats.
 *   fit      host, receives 1 - ||X - Xhat|| / ||X|| (evaluated from the explicit residual).
 *   sweeps_done host, nullable.
 * Blocks until the outputs are complete.  ||X|| = 0 gives fit 1, a zero core and the leading
 * columns of the identity as factors; a non-finite ||X||^2 gives TUCKER_ERR_NUMERICAL. */
tucker_status tucker_decompose(tucker_ctx* ctx, const float* tensor, int ndim,
                               const int64_t* dims, const int64_t* ranks,
                               int max_iters, double tol,
                               float* core, float* const* factors,
                               double* fit, int* sweeps_done);

/* As tucker_decompose, plus:
 *   init_factors host array of ndim device pointers (nullable): orthonormal s_n x R_n starting
 *                factors used instead of the T-HOSVD (resume / refinement).
 *   fit_history  host, nullable, max_iters + 1 doubles: fit_0 (start) and the fit after each
 *                sweep (as described for tol); entries past sweeps_done are left untouched.
 *                With tol = 0, FP32, a T-HOSVD start (or init_factors) and the dimension-tree path
 *                (order 4, the last two modes 64 elements or fewer together, mode 1 above 64 with
 *                one step per update), fit_0 is taken
 *                from the first sweep's product Y x_1 U1^T, which is the start's core, instead of
 *                from a separate pass over X: the same quantity in another rounding order. */
tucker_status tucker_decompose_ex(tucker_ctx* ctx, const float* tensor, int ndim,
                                  const int64_t* dims, const int64_t* ranks,
                                  int max_iters, double tol,
                                  const float* const* init_factors,
                                  float* core, float* const* factors, double* fit,
                                  double* fit_history, int* sweeps_done);

/* Xhat = G x_1 U_1 ... x_N U_N (eq. (1)).  core device prod(ranks) floats; factors host array
 * of device pointers (s_n x R_n); out device prod(dims) floats.  Stream-ordered. */
tucker_status tucker_reconstruct(tucker_ctx* ctx, const float* core, const float* const* factors,
                                 int ndim, const int64_t* dims, const int64_t* ranks, float* out);

/* ---- Codec hand-off: ordered core and core quantisation ----
 * The paper sets the bit rate of the representation by the rank of the core and its quantisation
 * (Abstract; Sec. I).  These two calls prepare a decomposition for that. */

/* All-orthogonal, energy-ordered core: for every mode, C_n = G_(n) G_(n)^T = V_n diag(sigma_n^2) V_n^T
 * (eigenvalues descending, FP64 eigensolver), factors_out[n] = U_n V_n and
 * core_out = G x_1 V_1^T ... x_N V_N^T.  The reconstruction (eq. (1)) is unchanged, the slices of
 * core_out along every mode are mutually orthogonal with norms sigma_n, and keeping the leading k_n
 * slices is then the rank-reduction knob (discarded energy sum_{i > k_n} sigma_n,i^2 per mode).
 *   core, core_out  device, prod(ranks) floats (may not alias);
 *   factors, factors_out  host arrays of ndim device pointers, dims[n] x ranks[n] floats each (may not alias);
 *   sigma  device, nullable, sum(ranks) doubles: sigma_1 (ranks[0] values), then sigma_2, ...
 * ranks[n] <= 1024 (TUCKER_ERR_UNSUPPORTED above).  Synchronises the stream when a rank exceeds 64. */
tucker_status tucker_order_core(tucker_ctx* ctx, const float* core, const float* const* factors, int ndim,
                                const int64_t* dims, const int64_t* ranks, float* core_out,
                                float* const* factors_out, double* sigma);

/* The leading keep[0] x ... x keep[N-1] block of a core (ranks) quantised uniformly with 2^(bits-1) - 1
 * levels per sign: step = max|block| / (2^(bits-1) - 1), code = round-half-even(block / step) clamped,
 * dequantized = code * step (each one correctly rounded binary32 operation).  codes (int32) and
 * dequantized (float) are device arrays of prod(keep) entries; step is a host float (0 for an all-zero
 * block).  2 <= bits <= 24, 1 <= keep[n] <= ranks[n].  Synchronises the stream. */
tucker_status tucker_quantize_core(tucker_ctx* ctx, const float* core, int ndim, const int64_t* ranks,
                                   const int64_t* keep, int bits, int32_t* codes, float* dequantized, float* step);

/* ---- Step-level entry points (the building blocks of a sweep, exposed for testing) ---- */

/* Mode-n product with a transposed factor (eq. (8)): out = in x_mode U^T.
 * in device prod(dims) floats; U device dims[mode] x r floats (row-major);
 * out device, dims with dims[mode] replaced by r.  Stream-ordered. */
tucker_status tucker_ttm(tucker_ctx* ctx, const float* in, int ndim, const int64_t* dims,
                         int mode, const float* U, int64_t r, float* out);

/* Mode-n Gram matrix in_(mode) in_(mode)^T (the text after eq. (8)).
 * out device dims[mode]^2 floats, symmetric, row-major.  Stream-ordered. */
tucker_status tucker_gram(tucker_ctx* ctx, const float* in, int ndim, const int64_t* dims,
                          int mode, float* out);

/* Reduced-precision encoding round trip, the storage step of the precision variants: x is a
 * rows x L row-major matrix (device floats); out[i] = dec(enc(x[i] / s[i % L])) * s[i % L] with
 * s = 1 for BF16 / FP16 (round to nearest even) and, for FP8_E4M3 (OCP E4M3, saturating at 448),
 * s[l] = max_rows |x[., l]| / 448 (1 for an all-zero column), written to scales (device L floats,
 * required for FP8, ignored otherwise).  L <= 256.  Stream-ordered. */
tucker_status tucker_quantize(tucker_ctx* ctx, const float* x, int64_t rows, int64_t L,
                              tucker_precision precision, float* out, float* scales);

/* Mode product in reduced precision (eq. (8) on the BF16 / FP16 / FP8 matrix cores, FP32
 * accumulation): out = Q(in) x_mode Q(U)^T with the same shapes as tucker_ttm.  Q encodes as
 * tucker_quantize does; for FP8 the tensor is scaled per index of its last mode and U per column,
 * and mode must not be the last one.  Stream-ordered. */
tucker_status tucker_ttm_lowp(tucker_ctx* ctx, const float* in, int ndim, const int64_t* dims,
                              int mode, const float* U, int64_t r, tucker_precision precision,
                              float* out);

/* Mode-n Gram of Q(in) on the BF16 / FP16 matrix cores (FP32 accumulation within K splits, the
 * splits summed in FP64); out as for tucker_gram.  Stream-ordered. */
tucker_status tucker_gram_lowp(tucker_ctx* ctx, const float* in, int ndim, const int64_t* dims,
                               int mode, tucker_precision precision, float* out);

/* Orthonormal basis of the column space of Z (rows x cols, rows >= cols) by FP64
 * CholeskyQR with column scaling: one shifted pass, then two plain ones (shifted CholeskyQR3),
 * the orthogonalisation step of orthogonal iteration (the text after eq. (8)).  Z, Q device
 * floats, row-major; Q may alias Z.  Pivots that needed the shifted fallback are counted in
 * tucker_stats.chol_shifts.  Synchronises the stream: TUCKER_ERR_DEVICE when a wait of the
 * Cholesky task graph gave up (tucker_options.wait_spin_limit). */
tucker_status tucker_orthonormalize(tucker_ctx* ctx, const float* Z, int64_t rows, int64_t cols,
                                    float* Q);

/* The two halves of one CholeskyQR pass, exposed separately:
 *   tucker_gram_tn64: W = Z^T Z accumulated in FP64.  Z device rows x cols floats (row-major);
 *                     W device cols x cols doubles.
 *   tucker_chol_inv:  for symmetric positive definite W (n x n doubles, device, read-only),
 *                     D = diag(W)^(1/2), D^-1 W D^-1 = L L^T, writes T = L^-1 D^-1 (lower triangular,
 *                     upper part zero) to T (device n x n doubles); Z T^T then has orthonormal
 *                     columns.  Pivots that are not safely positive are shifted and counted in
 *                     tucker_stats.chol_shifts.  Synchronises the stream; TUCKER_ERR_DEVICE when
 *                     a wait of the task graph gave up (tucker_options.wait_spin_limit).
 * tucker_gram_tn64 is stream-ordered. */
tucker_status tucker_gram_tn64(tucker_ctx* ctx, const float* Z, int64_t rows, int64_t cols, double* W);
tucker_status tucker_chol_inv(tucker_ctx* ctx, const double* W, int64_t n, double* T);

/* tucker_chol_inv without any device allocation, for callers that cannot allocate (serving loops
 * or harnesses that forbid hipMalloc).  Same arguments, result and errors as tucker_chol_inv, for
 * n <= 512; larger n returns TUCKER_ERR_INVALID_ARG.  Its scratch (the working copy of W, the task
 * graph's counters, the scaling) is a fixed array of about 2 MiB per GPU that the library holds
 * until the process ends, shared by every call on that GPU: calls on one GPU that overlap in time
 * (from several contexts, streams or threads) race and must be serialised by the caller.
 * Synchronises the context's stream. */
tucker_status tucker_chol_inv_noalloc(tucker_ctx* ctx, const double* W, int64_t n, double* T);

/* Leading r eigenvectors (descending eigenvalues) of a symmetric n x n matrix, n <= 1024, in FP64:
 * cyclic Jacobi for n <= 64, two-sided block Jacobi (64 x 64 sub-problems solved exactly) above; the
 * eigensolver behind the small-mode updates and the ordered core (the text after eq. (8)).
 * S device n*n floats; U device n*r floats; lam device n doubles (all eigenvalues, descending;
 * nullable).  Stream-ordered for n <= 64; above, it synchronises the stream once per sweep. */
tucker_status tucker_sym_eig(tucker_ctx* ctx, const float* S, int64_t n, int64_t r,
                             float* U, double* lam);

/* Sum of squares of n floats accumulated in FP64 (two-stage, deterministic).
 * x device; result host.  Synchronises. */
tucker_status tucker_sumsq(tucker_ctx* ctx, const float* x, int64_t n, double* result);

/* ---- Served execution: a request loop with admission by HBM budget ----
 *
 * Decompositions of many tensors (image stacks of different resolutions and exposure counts)
 * arrive over time.  The server keeps `slots` decompositions on the GPU at once, each on its own
 * stream with its own workspace, so their kernels overlap on the device; a request is admitted
 * (strictly first come, first served) when a slot is free and its device footprint fits in what
 * is left of hbm_budget_bytes.  Per request the server copies the host tensor to the device,
 * runs the same decomposition as tucker_decompose_ex with the request's precision, copies core
 * and factors back to the caller's host buffers and releases its device memory.  Every kernel's
 * result depends only on its own inputs (fixed reduction orders), so a result is the same alone
 * and in any mix of concurrent requests.
 *
 * Ownership: the caller owns host_tensor, host_core and host_factors[], which must stay valid
 * until tucker_server_wait has returned that request's result.  The server owns all device
 * memory it uses.  A server may be used from several host threads. */
typedef struct tucker_server tucker_server;

typedef struct {
    int device;                  /* HIP device ordinal                                        */
    int slots;                   /* decompositions on the GPU at once (>= 1)                  */
    size_t hbm_budget_bytes;     /* cap on admitted footprints; 0 = 90% of free device memory */
    int inner_iters;             /* as in tucker_options                                      */
    int init_iters;
    uint64_t seed;
    int use_graphs;              /* 1: slots replay each request's sweep as a HIP graph       */
    int autotune;                /* as in tucker_options (default 1)                          */
    int group_requests;          /* largest number of requests run as one group (0 or 1: no
                                    grouping, the default; at most 12).  Consecutive queued
                                    requests of one shape class (dims, ranks, reduced precision,
                                    max_iters, refine_sweeps, tol = 0) that fit in the budget
                                    are admitted together by one slot, each member on a context
                                    of its own, and their reduced-precision sweep products run
                                    as grouped persistent launches over all members' tiles (their
                                    sweeps are then not replayed as graphs).  Results are bit for
                                    bit those of the requests run alone.                        */
} tucker_server_options;

typedef struct {
    const float* host_tensor;    /* host, row-major dims[0] x ... (pinned memory copies fastest) */
    int ndim;
    int64_t dims[TUCKER_MAX_ORDER];
    int64_t ranks[TUCKER_MAX_ORDER];
    int max_iters;
    double tol;
    tucker_precision precision;
    int refine_sweeps;           /* FP32 sweeps after reduced-precision ones                  */
    uint64_t tag;                /* returned unchanged in the result                          */
    float* host_core;            /* host, prod(ranks) floats, written by the server            */
    float* host_factors[TUCKER_MAX_ORDER];   /* host, dims[n] * ranks[n] floats each          */
} tucker_request;

typedef struct {
    tucker_status status;        /* of the decomposition                                      */
    double fit;
    int sweeps;
    uint64_t tag;
    int slot;                    /* slot that ran it                                          */
    size_t footprint_bytes;      /* device memory charged against the budget                  */
    double t_submit, t_admit, t_start, t_finish;   /* seconds since tucker_server_create      */
    char error[160];             /* message when status != TUCKER_OK                          */
} tucker_result;

typedef struct {
    int64_t submitted, completed, failed;
    size_t budget_bytes;
    size_t peak_admitted_bytes;  /* largest sum of admitted footprints seen                   */
    int peak_running;            /* largest number of requests running at once               */
    int64_t grouped_requests;    /* requests that ran as members of a group                  */
    int64_t group_launches;      /* grouped persistent launches those groups made             */
    int64_t grouped_products;    /* products those launches computed                          */
} tucker_server_stats;

/* Defaults: device 0, 4 slots, budget 0 (90% of free memory), inner_iters 1, init_iters 20,
 * use_graphs 1, autotune 1, group_requests 0. */
void tucker_default_server_options(tucker_server_options* o);
/* ERR_DEVICE without a usable GPU; ERR_INVALID_ARG for bad options. */
tucker_status tucker_server_create(const tucker_server_options* opts, tucker_server** out);
/* Validates the request as tucker_decompose does (INVALID_ARG, UNSUPPORTED for a reduced
 * precision on a shape that has none) and enqueues it without blocking; a request whose
 * footprint exceeds the whole budget is refused with ERR_OUT_OF_MEMORY.  *id identifies it. */
tucker_status tucker_server_submit(tucker_server* srv, const tucker_request* req, uint64_t* id);
/* Waits up to timeout_s seconds (< 0: forever) for request id; on TUCKER_OK *out holds its
 * result (whose own status may be an error) and the id is retired.  ERR_TIMEOUT if it has not
 * finished, ERR_INVALID_ARG for an unknown id. */
tucker_status tucker_server_wait(tucker_server* srv, uint64_t id, double timeout_s, tucker_result* out);
tucker_status tucker_server_get_stats(tucker_server* srv, tucker_server_stats* out);
/* Finishes the running requests, fails the queued ones, frees everything. */
tucker_status tucker_server_destroy(tucker_server* srv);

/* ---- Autotuner ----
 * Launch choices are kept per (operation, shape, device) for the life of the process; see
 * tucker_options.autotune.  Operations: 1 = output tile of the FP32 mode products (2 candidates),
 * 2 = split count of the FP64 Grams (4), 3 = LDS staging (one or two stages) of the BF16/FP16/FP8
 * products and Grams (2).  The candidates of operation 3 give bit-identical results.
 * tucker_autotune_dump writes one line per choice ("op <id> dev <d> shape <5 numbers> choice <c> ms
 * <time per candidate>", "(heuristic)" when nothing was timed) into buf (host, len bytes, always
 * NUL-terminated when len > 0) and the full length including the NUL to *needed (nullable).
 * tucker_autotune_clear forgets every choice (later calls choose again). */
tucker_status tucker_autotune_dump(char* buf, size_t len, size_t* needed);
tucker_status tucker_autotune_clear(void);
/* Makes every later call of operation op (1..3) in this process take candidate `choice` (counted
 * from 0; a choice beyond an operation's candidates takes the last one), bypassing the kept table;
 * choice < 0 lifts the override.  For comparing candidates and for reproducing a run on another
 * device.  TUCKER_ERR_INVALID_ARG for an unknown op. */
tucker_status tucker_autotune_force(int op, int choice);

/* ---- Diagnostics ---- */
const char* tucker_status_string(tucker_status s);
const char* tucker_last_error(const tucker_ctx* ctx);   /* never NULL; "" when none */
tucker_status tucker_get_stats(const tucker_ctx* ctx, tucker_stats* out);
/* Changes tucker_options.timing and .timing_stages of a context for its later calls (host only,
 * no allocation).  TUCKER_ERR_INVALID_ARG for a NULL context or timing not 0 or 1. */
tucker_status tucker_set_timing(tucker_ctx* ctx, int timing, uint32_t stages);

#ifdef __cplusplus
}
#endif

#endif /* TUCKER_MI355X_H */
