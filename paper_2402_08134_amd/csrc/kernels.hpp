// Host-side launchers of the gfx950 kernels (internal to libsymnmf).
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>

#include "common.hpp"
#include <hip/hip_ext.h>
#include "../../include/symnmf.h"

// A bump allocator over one device buffer owned by the context.  Every
// launcher that needs temporaries takes them from here; launches happen on
// one in-order stream, so a later launcher may reuse the space as soon as the
// previous launcher's kernels have been enqueued.  Requests beyond the
// capacity return nullptr and the launcher fails before launching anything.
struct Workspace {
  char* base = nullptr;
  size_t cap = 0;
  size_t off = 0;
  void reset() { off = 0; }
  void* raw(size_t bytes) {
    const size_t a = (off + 255) & ~(size_t)255;
    if (base == nullptr || a + bytes > cap) return nullptr;
    off = a + bytes;
    return base + a;
  }
  double* dbl(size_t n) { return (double*)raw(n * sizeof(double)); }
  // doubles still available after alignment of the next request
  size_t avail_doubles() const {
    const size_t a = (off + 255) & ~(size_t)255;
    return base == nullptr || a >= cap ? 0 : (cap - a) / sizeof(double);
  }
  int* i32(size_t n) { return (int*)raw(n * sizeof(int)); }
  uint64_t* u64(size_t n) { return (uint64_t*)raw(n * sizeof(uint64_t)); }
};

inline size_t dtype_size(int dt) { return dt == SYMNMF_F64 ? 8 : (dt == SYMNMF_F32 ? 4 : 2); }

// ---- dense X ---------------------------------------------------------------
int dense_scalars(const void* X, int dtype, int64_t ld, int n, Workspace& ws, double* d_rowsum, double* d_out3,
                  hipStream_t s);

struct GemmPlan {
  int cp = 16;       // output columns padded to a multiple of 16
  int rt = 1;        // 16-row MFMA tiles per wave
  int kchunk = 64;   // K range per split
  int splits = 1;    // number of K splits (partial outputs)
  int64_t ldt = 0;   // row length of the transposed B panel
  bool cols = false;    // FP32: the row-contiguous product (kchunk = rows per split)
  int ct = 1;           // cols: 64-column blocks per wave
};
GemmPlan gemm_plan(int n, int c, int compute_dtype);
// Bytes of the transposed-B scratch for products with up to cmax columns.
size_t gemm_bt_bytes(int n, int cmax);
// Y = X B.  X dtype F64 / F32 / BF16; B F64 or F32 (F64 only with F64 X);
// Bt: scratch of gemm_bt_bytes; P: partials buffer of splits * n * cp
// elements of the accumulator type (double for F64 X, float otherwise); Y of
// ydtype with leading dim ldy.
int dense_gemm(const void* X, int xdtype, int64_t ldx, const void* B, int bdtype, int64_t ldb, int n, int c,
               const GemmPlan& p, void* Bt, void* P, void* Y, int ydtype, int64_t ldy, const DevState* st,
               hipStream_t s);
// P = X Bt^T from an already transposed, zero-padded B panel (cp rows of
// ldt elements: FP64 for F64 X, FP32 for F32 X, BF16 for BF16 X); the split-K
// partials stay in P for the consumer to reduce.
int dense_gemm_bt(const void* X, int xdtype, int64_t ldx, const void* Bt, int n, int c, const GemmPlan& p, void* P,
                  const DevState* st, hipStream_t s);
// Bt (cp x ldt, element type of the compute dtype) = F^T zero padded.
int factor_transpose(const void* F, int fdtype, int n, int k, void* Bt, int cdtype, const GemmPlan& p,
                     const DevState* st, hipStream_t s);
int convert_f32_bf16(const float* src, int64_t lds, void* dst, int64_t ldd, int n, hipStream_t s);
// d_sum = sum_ij (X_ij - w_i . h_j)^2, k <= 64.
int dense_resid_exact(const void* X, int xdtype, int64_t ldx, int n, int k, const void* W, const void* H, int fdtype,
                      Workspace& ws, double* d_sum, hipStream_t s);

// ---- CSR X -----------------------------------------------------------------
int csr_scalars(const int* rp, const void* val, int vdtype, int n, int64_t nnz, Workspace& ws, double* d_rowsum,
                double* d_out3, hipStream_t s);
// Y = X B (B n x c of bdtype, Y n x c of ydtype, c <= 128).
int csr_spmm(const int* rp, const int* ci, const void* val, int vdtype, int n, const void* B, int bdtype, int c,
             void* Y, int ydtype, const DevState* st, hipStream_t s, int64_t ldy = 0);
// out[i] = BF16(F[i]) (round to nearest even) for count FP32 values.
int to_bf16(const float* F, int64_t count, void* out, hipStream_t s);
// d_sum = sum over stored (i, j) of X_ij (w_i . h_j).
int csr_resid_cross(const int* rp, const int* ci, const void* val, int vdtype, int n, int k, const void* W,
                    const void* H, int fdtype, Workspace& ws, double* d_sum, hipStream_t s);

// ---- factor-side kernels ----------------------------------------------------
// out[0] = sum of part[0..nb) in a fixed order.
void sum_partials(const double* part, int nb, double* out, hipStream_t s);
int init_uniform_factor(void* F, int fdtype, int n, int k, double scale, uint64_t seed, hipStream_t s);
int gen_gaussian(double* out, int64_t count, uint64_t seed, uint32_t sub, uint32_t tag, hipStream_t s);
int copy_convert(const void* src, int sdtype, void* dst, int ddtype, int64_t count, hipStream_t s);

// G (ca x cb, FP64, ld cb) = A^T diag(w) B over rows (all rows, or the rows
// listed in `rows` with count *d_count when rows != nullptr; w == nullptr
// means unit weights).  If Ghat != nullptr it also receives G + alpha I
// padded to kp x kp with the identity.  ca, cb <= 128.
int gram(const void* A, int adtype, int64_t lda, int ca, const void* B, int bdtype, int64_t ldb, int cb, int n,
         const int* rows, const double* w, const int* d_count, int max_rows, Workspace& ws, double* G,
         double* Ghat, int kp, double alpha, const DevState* st, hipStream_t s, double* Ginv = nullptr);
// part[b] partial sums of sum_e A[e] B[e] over count elements; returns nb.
int dot_partials(const void* A, const void* B, int dtype, int64_t count, Workspace& ws, double** part,
                 const DevState* st, hipStream_t s);

// out[0] = sum_i A[i] B[i] (one workgroup, fixed order).
void frob_dot(const double* A, const double* B, int count, double* out, hipStream_t s);

// Fused end-of-iteration step: residual r = sqrt(max(normsq - 2 dot +
// <Ga, Gb>, 0) / normsq), log, stop rule.  dot_part == nullptr only counts
// the iteration (no residual evaluated).
struct StopRule {
  int mode;
  double tol;
  int patience;
  double target;
  int max_hist;
};
void finish_iteration(const double* dot_part, int nb, const double* Ga, const double* Gb, int k,
                      const double* d_normsq, DevState* st, double* hist, StopRule rule, hipStream_t s);

// Fused half-step update (right-hand side, HALS sweep, factor write-back,
// block partials of the next Gram / U^T F / residual dot).
struct UpdateArgs {
  int n = 0, k = 0, l = 0, splits = 1, cp = 0;
  int64_t ldt = 0;
  const void* P = nullptr;           // YMODE 0: partials [splits][n][cp]
  const int* seg_ptr = nullptr;      // YMODE 1: sampled slab, segment j = the stored
  const int* seg_src = nullptr;      // X[j][r] w_r of row j with r in the sample,
  const double* seg_val = nullptr;   // in column order
  const void* U = nullptr;           // YMODE 2: U (n x l, the factor type) and M = Lambda U^T F (l x k)
  const double* M = nullptr;
  const void* Src = nullptr;         // the fixed factor (alpha term, YMODE 1 rows)
  void* Dst = nullptr;               // the factor being updated (in place)
  void* Dt = nullptr;                // optional copy of Dst: transposed (cp x ldt) or,
  int dt_rows = 0;                   // when dt_rows, row-major (n x ldt)
  const double* Ghat = nullptr;      // G + alpha I padded to kp x kp
  double alpha = 0.0;
  double* part = nullptr;            // [nb][pstride]: F^T F (k*k) then U^T F (l*k, YMODE 2)
  int pstride = 0;
  double* dpart = nullptr;           // [nb] or nullptr
  // rule: 0 HALS sweep; 1 only write the regularised right-hand side
  // y + alpha src of every row to Yhat (n x kp FP64) and stop; 2 take the
  // new rows from Yhat (an exact NLS solution) instead of the sweep
  int rule = 0;
  double* Yhat = nullptr;
  // when set, the update kernel is launched with hipExtLaunchKernel and these
  // events take its start and end times (phase timing)
  hipEvent_t ev_start = nullptr, ev_stop = nullptr;
};
// Read-only small operands of the update, passed as separate restrict-
// qualified kernel arguments so the compiler reads them with scalar loads.
struct UpdateRO {
  const double* Ghat = nullptr;  // kp x kp
  const double* Ginv = nullptr;  // kp reciprocals of diag(Ghat)
  const double* M = nullptr;     // YMODE 2
};
// Blocks of the fused update for n rows, padded width kp and padded LAI
// width lp (0 without LAI); update_blocks_max(n) bounds it over every mode.
int update_blocks(int n, int kp, int lp, int fdtype);
int update_blocks_max(int n);
bool update_lpr8(int n, int kp, int lp, int tf_bytes);
// pdtype: element type of P (F32 or F64); tdtype: element type of Dt.
int fused_update(const UpdateArgs& a, const UpdateRO& ro, int kp, int ymode, int fdtype, int pdtype, int tdtype,
                 int nb, const DevState* st, hipStream_t s);
// Reduce nb partial rows of E doubles (E = k*k, or k*k + l*k when M is
// wanted).
int update_reduce(const double* part, int nb, int E, int k, int l, int kp, double alpha, const double* lam,
                  double* G, double* Ghat, double* Ginv, double* M, const DevState* st, hipStream_t s);
int pad_identity(double* Ghat, double* Ginv, int k, int kp, hipStream_t s);
// M (l x kp, zero padded) = diag(lam) Z, Z l x k.
int scale_rows(const double* Z, const double* lam, int l, int k, int kp, double* M, hipStream_t s);

// ---- projected Gauss-Newton with conjugate gradients ------------------------
// Operands of the row passes (k_pgncg.hip).  R, Pd, Z: n x kp FP64 CG
// vectors (gradient residual, direction, accumulated step), zero padded.
struct CgArgs {
  int n = 0, k = 0, l = 0, splits = 1, cp = 0;
  int64_t ldt = 0;
  const void* P = nullptr;        // init, YMODE 0: product partials [splits][n][cp]
  const double* U = nullptr;      // init YMODE 2 / final in LAI mode: U (n x l)
  const double* Mlai = nullptr;   // init YMODE 2: Lambda U^T H (l x kp)
  void* H = nullptr;              // the factor (read; replaced by the final pass)
  void* W = nullptr;              // receives a copy of the new H (final pass)
  void* Dt = nullptr;             // optional transposed panel of the new H (cp x ldt)
  double* R = nullptr;
  double* Pd = nullptr;
  double* Z = nullptr;
  double* part = nullptr;         // block partials
  int pstride = 0;                // doubles per partial row (final pass)
  double* dpart = nullptr;        // init: <h, y> per block
  int first = 0;                  // step / final: the first CG step (no P_prev, Z)
};
int cg_blocks(int n);
size_t cg_partial_doubles(int k);
// pass 0: init (R = -2 (Y - H G), partials of the first step's scalars and
// R^T H, residual dot); 1: one CG step; 2: last step and projected update.
// pdtype: element type of a.P; tdtype: element type of a.Dt; G: k x k Gram
// of H; cg: scalars and M (see cg_reduce).  Exactly nb blocks.
int cg_pass(int pass, const CgArgs& a, int kp, int ymode, int fdtype, int pdtype, int tdtype, const double* G,
            const double* cg, int nb, const DevState* st, hipStream_t s);
// Reduce nb partial rows of init/step passes into cg = [e, beta, step, done,
// 4 spare, M (k x k)]; l1: scratch of ceil(nb / 32) * cg_partial_doubles(k).
int cg_reduce(const double* part, int nb, int k, double* l1, double* cg, bool init, const DevState* st,
              hipStream_t s);

// Exact NLS per row by block principal pivoting.  Yhat (n x kp FP64): the
// regularised right-hand side on entry, the solution on exit.  Dst (n x k,
// fdtype) is the current factor, whose support starts the pivoting.  Ghat:
// kp x kp FP64, identity in the padding.  Sets flag_bit in *d_flags for a row
// that hit the pivoting cap (its clamped last iterate is kept).
int bpp_update(int n, int k, int kp, double* Yhat, const void* Dst, int fdtype, const double* Ghat, int* d_flags,
               int flag_bit, const DevState* st, hipStream_t s);

// out (n x c, odtype, ld ldo) = A (n x l, adtype, lda) * diag(scale) * M
// (l x c FP64 row-major; scale may be nullptr).
int rowmat(const void* A, int adtype, int64_t lda, int n, int l, const double* M, const double* scale, int c,
           void* out, int odtype, int64_t ldo, const DevState* st, hipStream_t s);

// One-workgroup dense kernels on small FP64 matrices.
// R upper with R^T R = G + shift I (shift 0 first, then growing shifts if a
// pivot is not positive); Rinv = R^{-1}; flag bit set when a shift was used;
// sets *d_fail when even the last shift failed.
int chol_inverse(const double* G, int k, double* R, double* Rinv, int* d_flags, int flag_bit, int* d_fail,
                 hipStream_t s);
// Symmetric EVD of the l x l matrix (T + T^T)/2 by parallel cyclic Jacobi;
// eigenvalues descending in lam, eigenvectors as columns of V (l x l).
int jacobi_evd(const double* T, int l, double* V, double* lam, hipStream_t s);
// Flip the sign of each column of U (n x l FP64) so that its entry of largest
// magnitude is positive (first such row on ties).
int column_sign_fix(double* U, int n, int l, Workspace& ws, hipStream_t s);

// Scans.
int exclusive_scan_i32(const int* in, int* out, int n, Workspace& ws, hipStream_t s);  // out has n+1 entries
// inclusive scan of in, with its totals over 1024-item blocks given (bsum)
int inclusive_scan_u64_from_sums(const uint64_t* in, uint64_t* out, int n, const uint64_t* bsum, hipStream_t s);
// the totals of (det[i] || counts[i] > 0) over 1024-row blocks (bsum: ceil(n / 1024) ints)
int selected_block_sums(const int* det, const int* counts, int n, int* bsum, hipStream_t s);

// ---- leverage-score sampling -----------------------------------------------
int leverage_scores(const void* F, int fdtype, int n, int k, const double* Rinv, double* lev, const DevState* st,
                    hipStream_t s);

struct SampleBuffers {
  uint64_t* w = nullptr;       // n quantised weights
  uint64_t* prefix = nullptr;  // n inclusive prefix sums
  int* counts = nullptr;       // n draw counts (kept zero between calls)
  int* flags = nullptr;        // n+1 selection flags / positions
  int* info = nullptr;         // [0] s_D, [1] s_R, [2] rows kept (<= cap), [3] rows selected
  double* theta = nullptr;     // deterministic leverage mass
};
// rows/weights: capacity >= s; the number of rows lands in info[2].
// wmask (n doubles, may be nullptr): each row's weight, 0 off the sample.
int hybrid_sample(const double* lev, int n, int k, int64_t s_total, double tau, uint64_t seed, uint32_t half_iter,
                  SampleBuffers& sb, int* rows, double* weights, int64_t cap, Workspace& ws, const DevState* st,
                  hipStream_t s, double* wmask = nullptr);

// Sampled slab of X S^T S: segment j lists (r, X[r][j] w_r) for the stored
// entries of the sampled rows r that have column j (w: the sample's weight
// of every row, 0 off it), in column order; X is symmetric, so these are the
// entries of row j whose column is in the sample.  seg_cnt (n ints) must be
// zero on entry and is zero again on exit; seg_ptr has n + 1 entries.
int sampled_slab(const int* rp, const int* ci, const void* val, int vdtype, int n, const int* rows,
                 const int* d_count, int max_rows, const double* wmask, int* seg_cnt,
                 int* seg_ptr, int* seg_src, double* seg_val, int64_t seg_cap, Workspace& ws, const DevState* st,
                 hipStream_t s);

// ---- learned warm start ------------------------------------------------------
constexpr int MLP_D_IN = 6;     // features per entry of H
constexpr int MLP_HIDDEN = 64;  // width of the three hidden layers
// Number of parameters (W1 b1 W2 b2 W3 b3 W4 b4, each W in x out row-major),
// or -1 for an unsupported width.
int mlp_param_count(int hidden);
// Philox initialisation (tag MLP, sub = layer): W = (2u - 1) sqrt(6 / in), b = 0.
int mlp_init(float* p, uint64_t seed, hipStream_t s);
// Y[e] = softplus(network(F[e])) for rows x 6 features.
int mlp_forward(const float* p, const float* F, int64_t rows, float* Y, hipStream_t s);
// Doubles of scratch mlp_gradient needs for `rows` entries.
size_t mlp_train_scratch_doubles(int64_t rows);
// Gradient of 1/(2 rows) sum (y - t)^2 into grad (parameter layout); the loss
// sum (not halved, not divided) lands in *d_losssum.  h1..h3: rows x HIDDEN;
// dza, dzb: rows x HIDDEN.
int mlp_gradient(const float* p, const float* F, const float* T, int64_t rows, float* h1, float* h2, float* h3,
                 float* dza, float* dzb, float* grad, double* scratch, double* d_losssum, hipStream_t s);
// One Adam step (b1 0.9, b2 0.999, eps 1e-8) with step count t >= 1.
int mlp_adam(float* p, const float* g, float* m, float* v, int np, double lr, int64_t t, hipStream_t s);
// Entry features ((n k) x 6 FP32) from the LAI basis U (n x l FP64), lam, the
// row sums and their total; info: 2k + 2 doubles (signs, eigenvalue ratios,
// mean row sum, a flag set when lam_0 <= 0).
int warm_features(const double* U, int n, int l, int k, const double* lam, const double* rowsum,
                  const double* d_total, float* F, double* info, Workspace& ws, hipStream_t s);
// H = W = beta Ht (fdtype) with beta = sqrt(*num / *den) when both are
// positive and *flag == 0; beta or 0 to *beta_out.
int warm_apply(const float* Ht, int64_t count, const double* num, const double* den, const double* flag, void* H,
               void* W, int fdtype, double* beta_out, hipStream_t s);
