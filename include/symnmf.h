/*
 * symnmf.h -- C ABI of the MI355X (gfx950) randomized symmetric NMF library.
 *
 * Method: Hayashi, Aksoy, Ballard, Park, "Randomized Algorithms for Symmetric
 * Nonnegative Matrix Factorization" (arXiv 2402.08134).  The library solves
 * the regularised surrogate (Section 2.1.1, eq. surrogate_symnmf_obj)
 *
 *     min_{W, H >= 0}  ||X - W H^T||_F^2 + alpha ||W - H||_F^2
 *
 * by alternating updates of W (from H) then H (from W), on
 *   - the full X (dense GEMM or CSR SpMM products),
 *   - a low-rank approximate input X ~ U Lambda U^T (Algorithm LAI-SymNMF),
 *   - leverage-score sampled problems (Algorithm LvS-SymNMF, hybrid sampling
 *     of Section 4.2),
 * with the HALS rule (eq. symhals_update2) or exact NLS by block principal
 * pivoting (Section 2.1.1 / Appendix "Update() function").
 *
 * Conventions (all entry points):
 *   - Every call returns a status code (SYMNMF_OK = 0 on success); no C++
 *     exception crosses the ABI.  On failure, symnmf_last_error(ctx) holds a
 *     message (for symnmf_create failures use symnmf_last_error(NULL)).
 *   - Pointers named "device" are HIP device pointers on the current device;
 *     "host" pointers are ordinary CPU memory.  Matrices are row-major.
 *   - Work is ordered on the hip stream given to symnmf_create.  Calls that
 *     return host values (create, residual, stats, history, iterate's
 *     iteration count, sample count) synchronise that stream.
 *   - A context is used by one host thread at a time.  Results are
 *     deterministic (bitwise) for fixed inputs, options and seed.
 *   - Sizes: 1 <= k <= 64; LAI rank k <= l <= 96 and l <= n.
 */
#ifndef SYMNMF_API_H_
#define SYMNMF_API_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SYMNMF_OK 0
#define SYMNMF_E_INVALID 1     /* bad argument (null pointer, size, dtype) */
#define SYMNMF_E_UNSUPPORTED 2 /* valid but not supported combination     */
#define SYMNMF_E_NOMEM 3       /* device allocation failed                */
#define SYMNMF_E_DEVICE 4      /* a HIP runtime call failed               */
#define SYMNMF_E_NUMERIC 5     /* numerical breakdown (e.g. Cholesky)     */
#define SYMNMF_E_STATE 6       /* call not valid in the context's state   */

/* matrix kinds and element types */
#define SYMNMF_DENSE 0
#define SYMNMF_CSR 1
#define SYMNMF_F64 0
#define SYMNMF_F32 1
#define SYMNMF_BF16 2

/* update rules.  HALS and BPP solve the NLS subproblems of the regularised
 * alternating scheme (eq. ANLS4symNMF, Section 2.1.1):
 *   HALS:  one sweep of the regularised HALS rule (eq. symhals_update2)
 *   BPP:   the exact per-row NLS solution by block principal pivoting
 * PGNCG works on the SymNMF objective ||X - H H^T||_F itself (Section 2.1.3;
 * Algorithm LAI-PGNCG-SymNMF in LAI mode; alpha is not used):
 *   PGNCG: H <- max(H - Z, 0), Z from options.cg_iters conjugate-gradient
 *          steps on the Gauss-Newton normal equations J^T J z = J^T r from
 *          z = 0 (standard CG; it stops early when <P, J^T J P> is not
 *          positive).  One product with X per iteration; W is kept equal
 *          to H.  Residual log entry t: ||X - H_t H_t^T|| / ||X|| of the
 *          factor iteration t starts from (the stop rule sees it before the
 *          step).  Not available with sampling (s > 0). */
#define SYMNMF_RULE_HALS 0
#define SYMNMF_RULE_BPP 1
#define SYMNMF_RULE_PGNCG 2

/* stopping modes */
#define SYMNMF_STOP_NONE 0   /* run exactly the requested iterations         */
#define SYMNMF_STOP_STALL 1  /* normalised residual fails to drop by more than
                                stop_tol for stop_patience iterations
                                (Section 5.1: 1e-4, four iterations)       */
#define SYMNMF_STOP_TARGET 2 /* normalised residual <= target              */
#define SYMNMF_STOP_STALL_OR_TARGET 3 /* whichever of the two comes first  */

/* residual modes for symnmf_residual */
#define SYMNMF_RESID_FAST 0  /* trace identity from the latest products
                                (Appendix "Fast residual evaluation")      */
#define SYMNMF_RESID_EXACT 1 /* FP64-accumulated pass against X            */
#define SYMNMF_RESID_LAI 2   /* against U Lambda U^T (Appendix, LAI residual) */

/* which factor */
#define SYMNMF_W 0
#define SYMNMF_H 1

/* context modes (symnmf_stats.mode) */
#define SYMNMF_MODE_PLAIN 0
#define SYMNMF_MODE_LAI 1
#define SYMNMF_MODE_LVS 2

/* phases of symnmf_stats.phase_ms (options.timing = 1):
 *   PRODUCT: the X-product kernel of each half-iteration (dense GEMM or CSR
 *            SpMM; one launch each), and the residual products of LvS
 *   UPDATE:  the fused NLS update kernel of each HALS / BPP half-iteration
 *            (one launch; BPP: the right-hand-side pass, the pivoting kernel
 *            and the write-back pass), and the PGNCG passes
 *   SAMPLE:  LvS leverage scores, sampler and sampled operands
 *   LAI:     the whole randomized range finder and Apx-EVD (symnmf_lai)
 *   WARM:    the learned warm start (symnmf_warmstart)
 *   REDUCE:  the fixed-order reduction of the update's block partials (Gram
 *            matrices, Lambda U^T F) after each HALS / BPP half-iteration */
#define SYMNMF_PHASE_PRODUCT 0
#define SYMNMF_PHASE_UPDATE 1
#define SYMNMF_PHASE_SAMPLE 2
#define SYMNMF_PHASE_LAI 3
#define SYMNMF_PHASE_WARM 4   /* symnmf_warmstart: features, network, scale fit */
#define SYMNMF_PHASE_REDUCE 5
#define SYMNMF_NUM_PHASES 6

/* stats flags */
#define SYMNMF_FLAG_LEV_SHIFT 1    /* chol(H^T H) needed a diagonal shift   */
#define SYMNMF_FLAG_CHOLQR_SHIFT 2 /* CholeskyQR2 needed a diagonal shift   */
#define SYMNMF_FLAG_BPP_CAP 4      /* a BPP row hit the pivoting cap (5 kp + 10
                                      exchanges); its last iterate, clamped at
                                      zero, was kept                         */

/* The data matrix X (symmetric, n x n).  All pointers are device pointers,
 * BORROWED: the caller keeps them alive and unchanged until symnmf_destroy.
 *   DENSE: values = n x n row-major with leading dimension ld >= n; dtype
 *          F64, F32 or BF16.
 *   CSR:   row_ptr int32[n+1], col_idx int32[nnz] (sorted within each row),
 *          values[nnz] of dtype F32 or F64.  Both triangles are stored. */
typedef struct symnmf_matrix {
  int32_t kind;
  int32_t dtype;
  int64_t n;
  int64_t ld;
  int64_t nnz;
  const void* values;
  const int32_t* row_ptr;
  const int32_t* col_idx;
} symnmf_matrix;

/* Options; fill with symnmf_default_options() and then override fields.
 * Defaults are the paper's settings (Section 5). */
typedef struct symnmf_options {
  int32_t struct_size;    /* sizeof(symnmf_options)                         */
  int32_t rule;           /* SYMNMF_RULE_HALS (default), _BPP or _PGNCG     */
  int32_t compute_dtype;  /* dense products: F64 (needs F64 X), F32, BF16;
                             CSR products: the dtype of X, or BF16 with FP32
                             values -- the iteration products then gather a
                             BF16 copy of the factor rows (FP32 values, FP64
                             sums; HALS and BPP rules only);
                             default: the dtype of X                         */
  int32_t stop_mode;      /* default SYMNMF_STOP_NONE                       */
  double stop_tol;        /* default 1e-4                                   */
  int32_t stop_patience;  /* default 4                                      */
  int32_t check_every;    /* iterations between host polls of the stop flag
                             (default 8); iterations after a stop are skipped
                             on the device                                  */
  double target;          /* residual target for SYMNMF_STOP_TARGET         */
  double tau;             /* hybrid threshold; < 0 means 1/s (Section 5.2)  */
  int32_t resid_every;    /* LvS: evaluate the residual every this many
                             iterations (needs a full product); default 1   */
  int32_t max_history;    /* capacity of the per-iteration residual log
                             (default 4096)                                 */
  int32_t timing;         /* 1: bracket the kernels of each phase with HIP
                             events on the stream and accumulate their
                             durations into symnmf_stats.phase_ms (default 0;
                             adds two event records per timed launch)       */
  int32_t graphs;         /* 1 (default): once the operands of an iteration
                             are in place, plain and LAI iterations are
                             replayed from HIP graphs captured on the
                             stream (blocks of check_every iterations, or 8
                             without a stop rule); 0: every kernel is
                             launched directly.  Not used with timing = 1
                             or in LvS mode.  Same results either way.     */
  int32_t cg_iters;       /* PGNCG: CG steps per iteration, 1..64 (default
                             5; the paper does not state its value)        */
  int32_t reserved[3];
} symnmf_options;

typedef struct symnmf_stats {
  int32_t struct_size;
  int32_t mode;           /* SYMNMF_MODE_*                                  */
  int32_t iterations;     /* completed iterations (all iterate calls)       */
  int32_t stopped;        /* 1 once the stop rule fired                     */
  int32_t k;
  int32_t l;              /* LAI rank (0 if none)                           */
  int64_t n;
  double alpha;           /* regulariser used                               */
  double zeta;            /* mean of all n^2 entries of X                   */
  double normsq;          /* ||X||_F^2                                      */
  double maxval;          /* max(X)                                         */
  double last_residual;   /* last normalised residual from the log          */
  int64_t s_D;            /* LvS: deterministic rows in the last sample     */
  int64_t sample_rows;    /* LvS: distinct rows in the last sample          */
  double theta_over_k;    /* LvS: deterministic leverage mass / k           */
  int32_t flags;          /* SYMNMF_FLAG_* */
  int32_t reserved[7];
  double warm_beta;       /* scale of the last symnmf_warmstart (0: the
                             random start was kept, or none ran)           */
  double phase_ms[SYMNMF_NUM_PHASES];     /* with options.timing: summed
                             device time of the timed launches per phase    */
  int64_t phase_calls[SYMNMF_NUM_PHASES]; /* timed launches per phase       */
  int64_t graph_launches; /* iteration graphs replayed (options.graphs)     */
} symnmf_stats;

typedef struct symnmf_ctx symnmf_ctx;

/* Fill *opt with the defaults listed above.  Host pointer. */
int symnmf_default_options(symnmf_options* opt);

/* Create a solver context (Section 2.1.1; initialisation of Section 5).
 *   out:   host pointer receiving the new context (owned by the caller, freed
 *          with symnmf_destroy).
 *   X:     host pointer to the matrix descriptor (device data, borrowed).
 *   k:     rank, 1..64.
 *   alpha: regulariser; alpha <= 0 selects alpha = max(X) (Section 5.1).
 *   s:     number of leverage-score samples per half-iteration; 0 = no
 *          sampling, s > 0 selects LvS mode (CSR X only, else E_UNSUPPORTED).
 *   seed:  Philox-4x32-10 key for the random initial H, the sketch and the
 *          sample draws.
 *   opt:   host pointer or NULL for defaults.
 *   hip_stream: the hipStream_t to order all work on (NULL = null stream).
 * Runs one pass over X for ||X||_F^2, mean, max and row sums, then sets
 * H0 = U[0,1) * 2 sqrt(zeta / k) and W0 = H0.  Synchronises the stream.
 * Errors: E_INVALID (null pointers, n < 1, k out of range, bad dtype),
 * E_UNSUPPORTED, E_NOMEM, E_DEVICE. */
int symnmf_create(symnmf_ctx** out, const symnmf_matrix* X, int32_t k, double alpha, int64_t s,
                  uint64_t seed, const symnmf_options* opt, void* hip_stream);

/* Build the low-rank approximate input X ~ U Lambda U^T with Algorithm
 * Apx-EVD (randomized range finder, Algorithm RRF, with 2q+1 products by X,
 * each followed by CholeskyQR in FP64, CholeskyQR2 after the last one;
 * T = Q^T X Q; Jacobi EVD of T;
 * U = Q Q_T) and switch the context to LAI mode (Algorithm LAI-SymNMF).
 * Dense or CSR X (the algorithms need only products with X: CSR products
 * run through the sparse kernel), no sampling.  l: k <= l <= min(n, 96).
 * q >= 0.  Errors: E_INVALID, E_UNSUPPORTED (s > 0), E_NUMERIC (CholeskyQR2
 * breakdown even with the shift), E_STATE. */
int symnmf_lai(symnmf_ctx* ctx, int32_t l, int32_t q);

/* Algorithm Ada-RRF (appendix "Adaptive Randomized Range Finder") followed
 * by Apx-EVD, as symnmf_lai but with the number of power iterations chosen
 * on the fly: Q = qr(X Omega); then up to q_max rounds of B^T = X Q, the
 * normalised QB residual sqrt((||X||^2 - ||B||_F^2) / ||X||^2) (the trace
 * identity of that appendix), Q = qr(B^T), stop when the residual fell by
 * less than tol since the previous round (the paper uses 1e-3; the first
 * round is compared with +infinity), otherwise Y = X Q, Q = qr(Y).
 * *rounds (may be NULL): completed rounds (each one two products with X);
 * *qb_residual (may be NULL): the last residual checked.  Synchronises once
 * per round.  E_INVALID for q_max outside 1..64 or tol < 0; otherwise as
 * symnmf_lai. */
int symnmf_lai_adaptive(symnmf_ctx* ctx, int32_t l, int32_t q_max, double tol, int32_t* rounds,
                        double* qb_residual);

/* Iterative refinement (Section 3.3, "Iterative Refinement"): switch a
 * context in LAI mode back to the full X for the following iterations, keeping
 * the current factors.  The stop rule becomes (stop_mode, target) with the
 * context's tolerance and patience, and its state is reset (the first refined
 * residual starts a fresh stall count).  Errors: E_STATE (not in LAI mode),
 * E_INVALID (stop_mode). */
int symnmf_refine(symnmf_ctx* ctx, int32_t stop_mode, double target);

/* Run up to `iters` iterations (each: W from H, then H from W) in the
 * context's mode.  With a stop mode set, iterations after the rule fires are
 * skipped on the device.  *done (host pointer, may be NULL) receives the
 * iterations completed by this call.  Synchronises the stream. */
int symnmf_iterate(symnmf_ctx* ctx, int32_t iters, int32_t* done);

/* Normalised residuals of the current factors (Appendix "Stopping
 * criteria").  out (host, 2 doubles) = { ||X - W H^T|| / ||X||,
 * ||X - H H^T|| / ||X|| }, norms against the matrix the mode names
 * (SYMNMF_RESID_LAI: U Lambda U^T, normalised by ||Lambda||).
 * SYMNMF_RESID_FAST uses the trace identity and the Gram matrices of the
 * current factors (one full product for each entry).
 * Synchronises the stream.  Errors: E_INVALID (mode), E_STATE (LAI residual
 * without symnmf_lai). */
int symnmf_residual(symnmf_ctx* ctx, int32_t mode, double out[2]);

/* Copy a factor (which = SYMNMF_W or SYMNMF_H) from / to caller-owned device
 * memory holding n x k row-major values of `dtype` (F64 or F32).
 * set_factor also refreshes the Gram matrix of that factor.  Stream-ordered. */
int symnmf_set_factor(symnmf_ctx* ctx, int32_t which, const void* src, int32_t dtype);
int symnmf_get_factor(symnmf_ctx* ctx, int32_t which, void* dst, int32_t dtype);

/* Export the LAI factors: U (device, n x l FP64 row-major) and lambda
 * (device, l FP64, descending).  Either may be NULL.  Errors: E_STATE. */
int symnmf_get_lai(symnmf_ctx* ctx, void* U, void* lambda);

/* Parity hook: the Gaussian sketch Omega of Algorithm RRF (Section 2.2.1)
 * that symnmf_lai and symnmf_lai_adaptive draw for rank l, into caller-owned
 * device memory (n x l FP64, row-major).  Entry (i, j) is Gaussian number
 * i l + j of the Philox-4x32-10 stream (key = seed, sub-stream 0, tag 2):
 * block e gives two 64-bit words v0, v1, and the value is
 * sqrt(-2 ln x) cos(2 pi b 2^-53) with x = 1 - (v0 >> 11) 2^-53 and
 * b = v1 >> 11 (Box-Muller).  The logarithm (atanh series after reduction to
 * [sqrt(1/2), sqrt(2)), ln 2 split in two) and the cosine (quarter-turn
 * reduction done exactly on b, Taylor series of sin and cos) are the
 * library's own, each step one correctly rounded FP64 operation in a fixed
 * order with nothing fused, so the values are fixed bit for bit.
 * 1 <= l <= n.  Stream-ordered.  Errors: E_INVALID. */
int symnmf_get_sketch(symnmf_ctx* ctx, int32_t l, void* Omega);

/* Y = X * B with the context's product kernel (dense GEMM in the compute
 * dtype, or CSR SpMM).  B: device, n x c (c <= 96) of the factor dtype
 * (F64 when the compute dtype is F64, else F32); Y: device, n x c of the same
 * dtype.  Stream-ordered. */
int symnmf_apply_x(symnmf_ctx* ctx, const void* B, int32_t c, void* Y);

/* One half-iteration in the context's mode: side 0 updates W from H, side 1
 * updates H from W (W then H is the order of Algorithms LAI-SymNMF and
 * LvS-SymNMF).  half_iter selects the Philox sub-stream of the LvS draws.
 * Stream-ordered. */
int symnmf_half_step(symnmf_ctx* ctx, int32_t side, int32_t half_iter);

/* Leverage scores (eq. lev_score_def) of the current factor `which`, via
 * chol(F^T F) and a triangular solve (Algorithm LvS-SymNMF):
 * lev[i] = ||F[i,:] R^{-1}||^2.  lev: device, n doubles.  Stream-ordered. */
int symnmf_leverage(symnmf_ctx* ctx, int32_t which, void* lev);

/* Hybrid leverage-score sample (Section 4.2, eq. SH) from given scores.
 *   lev:     device, n doubles (leverage scores of a rank-k factor).
 *   half_iter: Philox sub-stream of the draws.
 *   rows:    device, int32[cap]: sampled rows, ascending.
 *   weights: device, double[cap]: the row's diagonal entry of S^T S
 *            (1 for deterministic rows, c / (s_R p~_i) for a row drawn c times).
 *   cap:     capacity, >= s.   count: host, receives the number of rows.
 * Rows with lev_i / k >= tau are deterministic; s_R = s - s_D draws with
 * replacement from p~_i = w_i / W_R, w_i = floor(lev_i 2^40).  Uses the
 * context's k, s, tau and seed.  Synchronises the stream. */
int symnmf_sample(symnmf_ctx* ctx, const void* lev, int32_t half_iter, void* rows, void* weights,
                  int64_t cap, int64_t* count);

/* Per-iteration normalised residual log (fast mode): host array out[cap],
 * *count receives the number of entries (<= cap).  Synchronises. */
int symnmf_history(symnmf_ctx* ctx, double* out, int32_t cap, int32_t* count);

/* Statistics and counters (host struct; set out->struct_size).  Synchronises. */
int symnmf_get_stats(symnmf_ctx* ctx, symnmf_stats* out);

/* Last error message of the context (or of the last failed create when ctx is
 * NULL).  The string is owned by the library and valid until the next call
 * on the same context. */
const char* symnmf_last_error(const symnmf_ctx* ctx);

/* Free everything the context owns (never touches X).  NULL is a no-op.
 * Device blocks go back to the library's cache of device memory (per device
 * and size, up to 16 GiB), from which later contexts and networks of the
 * same sizes are served without hipMalloc. */
void symnmf_destroy(symnmf_ctx* ctx);

/* Return every cached device block to the HIP runtime (hipFree).  Call only
 * when no context or network is being used by another thread. */
int symnmf_trim_cache(void);

/* ---- learned warm start ----------------------------------------------------
 * Not part of the paper's method: the paper starts from a random H (Section 5,
 * experimental setup) and mentions SVD-based starts as the alternative.  This
 * start builds on the LAI basis of Section 3.  For every entry (i, j), j < k,
 * of H, six features are taken from the embedding (c_j = sqrt(n) U[:, j],
 * s_j the sign whose part of c_j has the larger norm, a_ij = s_j c_ij, r_i the
 * norm of row i of c_0..c_{k-1}, m_i = max_j a_ij, d the row sums of X):
 *   f_ij = [a_ij, r_i, m_i, a_ij - m_i, lam_j / lam_0, log(max(d_i/mean d, 1e-6))]
 * A network shared by all columns, 6 -> 64 -> 64 -> 64 -> 1 with ReLU and a
 * softplus output, maps f_ij to Ht[i, j] >= 0; the start is H0 = W0 = beta Ht
 * with beta^2 = tr(Ht^T X Ht) / ||Ht^T Ht||_F^2 (the least-squares multiple).
 * Parameters: W1 (6 x 64) b1 (64) W2 (64 x 64) b2 W3 (64 x 64) b3 W4 (64 x 1)
 * b4 (1), each W row-major (in x out), FP32, contiguous in that order. */
#define SYMNMF_MLP_FEATURES 6
#define SYMNMF_MLP_HIDDEN 64

typedef struct symnmf_mlp symnmf_mlp;

/* New network of the given hidden width (only SYMNMF_MLP_HIDDEN), weights
 * W = (2u - 1) sqrt(6 / fan_in) with u the Philox uniforms of stream
 * (seed, sub = layer index 0..3, tag 6) in row-major order, biases 0.  Its
 * kernels run on hip_stream (NULL: the default stream).  Synchronises. */
int symnmf_mlp_create(symnmf_mlp** out, int32_t hidden, uint64_t seed, void* hip_stream);
int symnmf_mlp_num_params(const symnmf_mlp* net, int64_t* count);
/* Copy all parameters from / to caller-owned DEVICE memory (FP32, layout
 * above).  set_params also clears the Adam state. */
int symnmf_mlp_set_params(symnmf_mlp* net, const float* params);
int symnmf_mlp_get_params(symnmf_mlp* net, float* params);
/* Y[e] = network(F[e]) for rows x 6 feature rows (device FP32, row-major);
 * rows == 0 is a no-op. */
int symnmf_mlp_forward(symnmf_mlp* net, const float* F, int64_t rows, float* Y);
/* Gradient of L = 1/(2 rows) sum_e (Y[e] - T[e])^2 with respect to every
 * parameter, into grad (device FP32, parameter layout).  *loss (host, may be
 * NULL; when given, the call synchronises) receives L. */
int symnmf_mlp_gradient(symnmf_mlp* net, const float* F, const float* T, int64_t rows, float* grad, double* loss);
/* One Adam step (b1 0.9, b2 0.999, eps 1e-8, bias-corrected, step count kept
 * by the network) on the gradient of L for this batch; *loss as above (the
 * loss before the step). */
int symnmf_mlp_train_step(symnmf_mlp* net, const float* F, const float* T, int64_t rows, double lr, double* loss);
/* Write the parameters to a file (host path; the library's own format, read
 * by symnmf_mlp_load): 8 bytes "SYMNMLP1", int32 hidden width, int32 feature
 * count (6), int64 parameter count, then the FP32 parameters in the layout
 * above, all little-endian.  The Adam state is not written.  Waits for the
 * network's stream.  Errors: E_INVALID (null path, cannot write), E_DEVICE. */
int symnmf_mlp_save(symnmf_mlp* net, const char* path);
/* New network (as symnmf_mlp_create, on hip_stream) with the parameters of a
 * file written by symnmf_mlp_save; fresh Adam state.  Errors: E_INVALID
 * (cannot read, wrong magic, widths, count or length; message via
 * symnmf_mlp_last_error(NULL)), E_NOMEM, E_DEVICE. */
int symnmf_mlp_load(symnmf_mlp** out, const char* path, void* hip_stream);
const char* symnmf_mlp_last_error(const symnmf_mlp* net);
void symnmf_mlp_destroy(symnmf_mlp* net);

/* The (n k) x 6 feature rows f_ij (row-major over (i, j), FP32) of the
 * context's LAI basis into caller-owned device memory.  Needs symnmf_lai
 * (E_STATE otherwise). */
int symnmf_warm_features(symnmf_ctx* ctx, float* F);
/* Replace W and H by the learned start beta Ht.  Needs symnmf_lai (E_STATE
 * otherwise); the context stays in its mode (LAI: iterate on U Lambda U^T, or
 * symnmf_refine to continue on X).  When the fit is not positive, or lam_0 <= 0,
 * the random start is kept and beta = 0.  *beta_out (host, may be NULL;
 * when given, the call synchronises).  The network's stream must have
 * finished updating its parameters.  Allocates temporaries of (n k)(6 + 1)
 * floats plus n k factor elements for the duration of the call. */
int symnmf_warmstart(symnmf_ctx* ctx, const symnmf_mlp* net, double* beta_out);

/* symnmf_warmstart for callers that cannot allocate device memory: code
 * running under HIP graph capture, tight serving loops, and hosts that forbid
 * hipMalloc.  Same arguments, result and errors as symnmf_warmstart (bitwise
 * the same H, W and beta), but the temporaries (features, network output and
 * the converted start: (28 + factor element size) n k bytes, each piece
 * rounded up to 256 bytes) live in a static device array of 64 MiB per GPU,
 * held from library load until the process ends; the call makes no hipMalloc,
 * hipFree or other allocating call.  Limit: that sum <= 64 MiB, e.g.
 * n k <= 2,097,152 with FP32 factors (n = 32768 at k = 64) and <= 1,864,128
 * with FP64 factors; larger n k gives E_INVALID before any work is enqueued.
 * Every call on one GPU uses the same array, and each call overwrites it
 * completely before reading it (nothing is assumed to start at zero): calls
 * that overlap on one GPU (other threads, other streams, or a second call
 * enqueued before the first one's stream work has run) race and must be
 * serialised by the caller. */
int symnmf_warmstart_noalloc(symnmf_ctx* ctx, const symnmf_mlp* net, double* beta_out);

#ifdef __cplusplus
}
#endif

#endif /* SYMNMF_API_H_ */
