// Factor-side kernels: random fills, Gram matrices, the fused end-of-iteration
// residual / stop step, the regularised HALS sweep, row-times-small-matrix
// products, and one-workgroup FP64 Cholesky / Jacobi EVD on k x k and l x l
// matrices.  All reductions use fixed orders so results are bitwise
// reproducible.
#include "kernels.hpp"

namespace {

__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ part, int nb, double* __restrict__ out) {
  __shared__ double sc[8];
  double v = 0.0;
  int i = threadIdx.x;
  for (; i + 7 * 256 < nb; i += 8 * 256) {  // 8 loads in flight, added in order
    double u[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) u[q] = part[i + q * 256];
#pragma unroll
    for (int q = 0; q < 8; ++q) v += u[q];
  }
  for (; i < nb; i += 256) v += part[i];
  const double t = block_sum(v, sc);
  if (threadIdx.x == 0) out[0] = t;
}

template <typename TF>
__global__ __launch_bounds__(256) void k_init_uniform(TF* __restrict__ F, int64_t count, double scale, uint64_t seed) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= count) return;
  F[e] = (TF)(u53(philox_value(seed, (uint64_t)e, 0, TAG_H0)) * scale);
}

template <typename TS, typename TD>
__global__ __launch_bounds__(256) void k_convert(const TS* __restrict__ src, TD* __restrict__ dst, int64_t count) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < count) dst[e] = (TD)src[e];
}

// ---------------------------------------------------------------------------
// Gram: part[b] = sum over this block's rows of w_r a_r^T b_r (FP64).
// 16 x 16 threads; thread (ty, tx) owns entries (ty + 16 i, tx + 16 j).
// ---------------------------------------------------------------------------
template <typename TA, typename TB, int T>
__global__ __launch_bounds__(256) void k_gram(const TA* __restrict__ A, int64_t lda, int ca, const TB* __restrict__ B,
                                              int64_t ldb, int cb, int n, const int* __restrict__ rows,
                                              const double* __restrict__ w, const int* __restrict__ d_count,
                                              int rows_per_block, double* __restrict__ part,
                                              const DevState* __restrict__ st) {
  if (stopped(st)) return;
  constexpr int RB = 16;
  constexpr int CM = 16 * T;
  __shared__ double As[RB][CM + 1];
  __shared__ double Bs[RB][CM + 1];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int nrows = rows ? *d_count : n;
  // selected rows: the device-side count (about half the capacity the grid
  // is sized for) spread over all the blocks, 16-row chunks (n = 2^20,
  // s = 8192: two chunks a block instead of five in 96 of 256 blocks)
  const int rpb = rows ? 16 * ((nrows + 16 * (int)gridDim.x - 1) / (16 * (int)gridDim.x)) : rows_per_block;
  const int r0 = blockIdx.x * rpb;
  const int r1 = min(nrows, r0 + rpb);
  double acc[T][T];
#pragma unroll
  for (int i = 0; i < T; ++i)
#pragma unroll
    for (int j = 0; j < T; ++j) acc[i][j] = 0.0;
  // Each thread stages EPT entries of the 16-row chunk; the next chunk's
  // values are loaded into registers while the current one is multiplied.
  constexpr int EPT = (RB * CM + 255) / 256;
  double na[EPT], nbv[EPT];
  auto fetch = [&](int rb) {
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = tid + 256 * u;
      const int rr = e / CM, q = e - rr * CM;
      const int r = rb + rr;
      double a = 0.0, b = 0.0;
      if (e < RB * CM && r < r1) {
        const int src = rows ? rows[r] : r;
        if (q < ca) a = (double)A[(int64_t)src * lda + q] * (w ? w[r] : 1.0);
        if (q < cb) b = (double)B[(int64_t)src * ldb + q];
      }
      na[u] = a;
      nbv[u] = b;
    }
  };
  if (r0 < r1) fetch(r0);
  for (int rb = r0; rb < r1; rb += RB) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = tid + 256 * u;
      if (e < RB * CM) {
        const int rr = e / CM, q = e - rr * CM;
        As[rr][q] = na[u];
        Bs[rr][q] = nbv[u];
      }
    }
    __syncthreads();
    if (rb + RB < r1) fetch(rb + RB);
#pragma unroll 4
    for (int rr = 0; rr < RB; ++rr) {
      double bv[T];
#pragma unroll
      for (int j = 0; j < T; ++j) bv[j] = Bs[rr][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < T; ++i) {
        const double a = As[rr][ty + 16 * i];
#pragma unroll
        for (int j = 0; j < T; ++j) acc[i][j] = fma(a, bv[j], acc[i][j]);
      }
    }
  }
  double* out = part + (int64_t)blockIdx.x * ca * cb;
#pragma unroll
  for (int i = 0; i < T; ++i)
#pragma unroll
    for (int j = 0; j < T; ++j) {
      const int p = ty + 16 * i, q = tx + 16 * j;
      if (p < ca && q < cb) out[p * cb + q] = acc[i][j];
    }
}

// Fixed-order sum of the nb block partials (ca x cb each) and the epilogue
// (G, Ghat = G + alpha I padded to kp x kp, 1/diag).  A block takes 16
// entries; its 16 slices of threads each sum a contiguous run of partials
// (16 loads in flight), and the slice sums are added in slice order (one
// thread summing all 256 partials 8 loads at a time took 13.5 us at
// n = 16384, l = 48).
constexpr int GR_SLICES = 16, GR_COLS = 16;

__global__ __launch_bounds__(GR_SLICES * GR_COLS) void k_gram_reduce(
    const double* __restrict__ part, int nb, int ca, int cb, double* __restrict__ G, double* __restrict__ Ghat,
    int kp, double alpha, double* __restrict__ Ginv, const DevState* __restrict__ st) {
  if (stopped(st)) return;
  __shared__ double ps[GR_SLICES][GR_COLS + 1];
  const int c = threadIdx.x % GR_COLS, sl = threadIdx.x / GR_COLS;
  const int e = blockIdx.x * GR_COLS + c;
  const int E = ca * cb;
  const int per = (nb + GR_SLICES - 1) / GR_SLICES;
  const int b0 = sl * per;
  const int cnt = max(0, min(per, nb - b0));
  double acc = 0.0;
  if (e < E) {
    const double* p = part + (int64_t)b0 * E + e;
    int b = 0;
    for (; b + 16 <= cnt; b += 16) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = p[(int64_t)(b + u) * E];
#pragma unroll
      for (int u = 0; u < 16; ++u) acc += v[u];
    }
    for (; b < cnt; ++b) acc += p[(int64_t)b * E];
  }
  ps[sl][c] = acc;
  __syncthreads();
  if (sl != 0) return;
  if (e < E) {
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < GR_SLICES; ++j) t += ps[j][c];
    if (G) G[e] = t;
    if (Ghat) {
      const int p = e / cb, q = e - p * cb;
      Ghat[p * kp + q] = t + (p == q ? alpha : 0.0);
      if (Ginv && p == q) Ginv[p] = 1.0 / (t + alpha);
    }
  }
  if (Ghat && e < kp * kp) {
    const int p = e / kp, q = e - p * kp;
    if (p >= ca || q >= cb) Ghat[e] = (p == q) ? 1.0 : 0.0;
  }
}

__global__ __launch_bounds__(256) void k_frob(const double* __restrict__ A, const double* __restrict__ B, int count,
                                              double* __restrict__ out) {
  __shared__ double sc[8];
  double v = 0.0;
  for (int i = threadIdx.x; i < count; i += 256) v = fma(A[i], B[i], v);
  const double t = block_sum(v, sc);
  if (threadIdx.x == 0) out[0] = t;
}

template <typename T>
__global__ __launch_bounds__(256) void k_dot(const T* __restrict__ A, const T* __restrict__ B, int64_t count,
                                             double* __restrict__ part, const DevState* __restrict__ st) {
  if (stopped(st)) return;
  __shared__ double sc[8];
  double v = 0.0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += stride)
    v = fma((double)A[e], (double)B[e], v);
  const double t = block_sum(v, sc);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_finish_iteration(const double* __restrict__ dot_part, int nb,
                                                          const double* __restrict__ Ga,
                                                          const double* __restrict__ Gb, int k,
                                                          const double* __restrict__ d_normsq, DevState* st,
                                                          double* __restrict__ hist, StopRule rule) {
  if (st->done) return;
  if (dot_part == nullptr) {  // iteration without a residual evaluation
    if (threadIdx.x == 0) st->iter += 1;
    return;
  }
  __shared__ double sc[8];
  double d = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) d += dot_part[i];
  const double dot = block_sum(d, sc);
  double g = 0.0;
  for (int i = threadIdx.x; i < k * k; i += 256) g = fma(Ga[i], Gb[i], g);
  const double gg = block_sum(g, sc);
  if (threadIdx.x == 0) {
    const double nx = *d_normsq;
    const double r2 = nx - 2.0 * dot + gg;
    const double r = sqrt(fmax(r2, 0.0) / nx);
    const int t = st->iter;
    if (t < rule.max_hist) hist[t] = r;
    if (t > 0) st->stall = (st->prev - r <= rule.tol) ? st->stall + 1 : 0;
    st->prev = r;
    st->last = r;
    st->iter = t + 1;
    const bool stall = (rule.mode == SYMNMF_STOP_STALL || rule.mode == SYMNMF_STOP_STALL_OR_TARGET) &&
                       st->stall >= rule.patience;
    const bool hit = (rule.mode == SYMNMF_STOP_TARGET || rule.mode == SYMNMF_STOP_STALL_OR_TARGET) &&
                     r <= rule.target;
    if (stall || hit) st->done = 1;
  }
}

template <typename TA, typename TO>
__global__ __launch_bounds__(256) void k_rowmat(const TA* __restrict__ A, int64_t lda, int n, int l,
                                                const double* __restrict__ M, const double* __restrict__ scale, int c,
                                                TO* __restrict__ out, int64_t ldo, const DevState* __restrict__ st) {
  if (stopped(st)) return;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)n * c) return;
  const int j = (int)(e / c), q = (int)(e - (int64_t)j * c);
  const TA* a = A + (int64_t)j * lda;
  double acc = 0.0;
  // loads of 8 terms issued together, summed in order
  int p = 0;
  for (; p + 8 <= l; p += 8) {
    double av[8], mv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      av[u] = (double)a[p + u] * (scale ? scale[p + u] : 1.0);
      mv[u] = M[(p + u) * c + q];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = fma(av[u], mv[u], acc);
  }
  for (; p < l; ++p) acc = fma((double)a[p] * (scale ? scale[p] : 1.0), M[p * c + q], acc);
  out[(int64_t)j * ldo + q] = (TO)acc;
}

// out = A diag(scale) M on the FP64 matrix cores, for l, c <= 96: each wave
// takes 16 rows and all CT = c / 16 (rounded up) output tiles; the block
// stages diag(scale) M in LDS (rows padded to a multiple of 4 and columns to
// CT 16 with zeros), lane (li, lg) feeds A[r0 + li][4 s + lg] and
// M[4 s + lg][16 t + li] to v_mfma_f64_16x16x4f64 and holds output rows
// lg + 4 v of column li of each tile.  A row's entries are read 4 at a time
// by the 4 lane groups (one 16- or 32-byte run per row and step).
template <typename TA, typename TO, int CT>
__global__ __launch_bounds__(256) void k_rowmat_mfma(const TA* __restrict__ A, int64_t lda, int n, int l,
                                                     const double* __restrict__ M, const double* __restrict__ scale,
                                                     int c, TO* __restrict__ out, int64_t ldo,
                                                     const DevState* __restrict__ st) {
  if (stopped(st)) return;
  constexpr int CP = 16 * CT;
  __shared__ double Ms[96 * CP];
  const int l4 = 4 * ((l + 3) / 4);
  for (int e = threadIdx.x; e < l4 * CP; e += 256) {
    const int p = e / CP, q = e - p * CP;
    const bool in = p < l && q < c;
    const double v = M[in ? p * c + q : 0];   // clamped index, masked value
    const double sv = scale ? scale[in ? p : 0] : 1.0;
    Ms[e] = in ? v * sv : 0.0;
  }
  __syncthreads();
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  const int r0 = (blockIdx.x * 4 + wid) * 16;
  if (r0 >= n) return;   // after the only barrier
  const int ra = r0 + li < n ? r0 + li : n - 1;   // clamped row, its values unused beyond n
  const TA* arow = A + (int64_t)ra * lda;
  doublex4 acc[CT];
#pragma unroll
  for (int t = 0; t < CT; ++t) acc[t] = doublex4{0.0, 0.0, 0.0, 0.0};
  for (int s4 = 0; s4 < l4; s4 += 4) {
    const int p = s4 + lg;
    const double av = p < l ? (double)arow[p < l ? p : 0] : 0.0;
#pragma unroll
    for (int t = 0; t < CT; ++t)
      acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Ms[p * CP + 16 * t + li], acc[t], 0, 0, 0);
  }
#pragma unroll
  for (int t = 0; t < CT; ++t) {
    const int q = 16 * t + li;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = r0 + lg + 4 * v;
      if (r < n && q < c) out[(int64_t)r * ldo + q] = (TO)acc[t][v];
    }
  }
}

template <typename TA, typename TO>
int rowmat_mfma(const TA* A, int64_t lda, int n, int l, const double* M, const double* scale, int c, TO* out,
                int64_t ldo, const DevState* st, hipStream_t s) {
  const int nb = ceil_div(n, 64);
  switch ((c + 15) / 16) {
    case 1: k_rowmat_mfma<TA, TO, 1><<<nb, 256, 0, s>>>(A, lda, n, l, M, scale, c, out, ldo, st); return 0;
    case 2: k_rowmat_mfma<TA, TO, 2><<<nb, 256, 0, s>>>(A, lda, n, l, M, scale, c, out, ldo, st); return 0;
    case 3: k_rowmat_mfma<TA, TO, 3><<<nb, 256, 0, s>>>(A, lda, n, l, M, scale, c, out, ldo, st); return 0;
    case 4: k_rowmat_mfma<TA, TO, 4><<<nb, 256, 0, s>>>(A, lda, n, l, M, scale, c, out, ldo, st); return 0;
    case 5: k_rowmat_mfma<TA, TO, 5><<<nb, 256, 0, s>>>(A, lda, n, l, M, scale, c, out, ldo, st); return 0;
    case 6: k_rowmat_mfma<TA, TO, 6><<<nb, 256, 0, s>>>(A, lda, n, l, M, scale, c, out, ldo, st); return 0;
    default: return -1;
  }
}

// ---------------------------------------------------------------------------
// One-workgroup Cholesky (upper R, R^T R = G + shift I) and R^{-1}.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_chol_inverse(const double* __restrict__ G, int k, double* __restrict__ R,
                                                      double* __restrict__ Rinv, int* d_flags, int flag_bit,
                                                      int* d_fail) {
  extern __shared__ double A[];  // k x (k + 1) factor, then k x (k + 1) inverse
  double* Xi = A + k * (k + 1);
  __shared__ int bad;
  __shared__ double shift;
  const int lda = k + 1;
  const int tid = threadIdx.x;
  double trace = 0.0;
  for (int i = 0; i < k; ++i) trace += G[i * k + i];
  for (int attempt = 0; attempt < 6; ++attempt) {
    if (tid == 0) {
      bad = 0;
      shift = attempt == 0 ? 0.0 : 1e-12 * pow(100.0, (double)(attempt - 1)) * fmax(trace, 1e-300) / k;
    }
    __syncthreads();
    for (int e = tid; e < k * k; e += 256) {
      const int p = e / k, q = e - p * k;
      A[p * lda + q] = G[e] + (p == q ? shift : 0.0);
    }
    __syncthreads();
    for (int j = 0; j < k; ++j) {
      if (tid == 0) {
        const double d = A[j * lda + j];
        if (!(d > 0.0) || !isfinite(d)) bad = 1;
        A[j * lda + j] = bad ? 1.0 : sqrt(d);
      }
      __syncthreads();
      if (bad) break;
      const double djj = A[j * lda + j];
      for (int q = j + 1 + tid; q < k; q += 256) A[j * lda + q] /= djj;
      __syncthreads();
      const int m = k - j - 1;
      for (int e = tid; e < m * m; e += 256) {
        const int p = j + 1 + e / m, q = j + 1 + e % m;
        if (q >= p) A[p * lda + q] -= A[j * lda + p] * A[j * lda + q];
      }
      __syncthreads();
    }
    if (!bad) break;
    __syncthreads();
  }
  if (bad) {
    if (tid == 0) *d_fail = 1;
    return;
  }
  if (tid == 0 && shift > 0.0 && d_flags) atomicOr(d_flags, flag_bit);
  for (int e = tid; e < k * k; e += 256) {
    const int p = e / k, q = e - p * k;
    R[e] = (q >= p) ? A[p * lda + q] : 0.0;
  }
  // Rinv column c: solve R x = e_c by back substitution (x_i = 0 for i > c),
  // the column kept in LDS.
  for (int c = tid; c < k; c += 256) {
    for (int i = k - 1; i >= 0; --i) {
      double v = 0.0;
      if (i <= c) {
        // four independent partial sums shorten the dependent chain
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int p = i + 1;
        for (; p + 3 <= c; p += 4) {
          s0 = fma(A[i * lda + p], Xi[p * lda + c], s0);
          s1 = fma(A[i * lda + p + 1], Xi[(p + 1) * lda + c], s1);
          s2 = fma(A[i * lda + p + 2], Xi[(p + 2) * lda + c], s2);
          s3 = fma(A[i * lda + p + 3], Xi[(p + 3) * lda + c], s3);
        }
        for (; p <= c; ++p) s0 = fma(A[i * lda + p], Xi[p * lda + c], s0);
        v = ((i == c) ? 1.0 : 0.0) - ((s0 + s1) + (s2 + s3));
        v /= A[i * lda + i];
      }
      Xi[i * lda + c] = v;
    }
  }
  __syncthreads();
  for (int e = tid; e < k * k; e += 256) {
    const int p = e / k, q = e - p * k;
    Rinv[e] = Xi[p * lda + q];
  }
}

// v of lane `lane` (a constant), in every lane
__device__ __forceinline__ double lane_value(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// ---------------------------------------------------------------------------
// Blocked Cholesky G + shift I = L L^T and L^{-1} (k <= 64) in one workgroup
// of four waves, on 16 x 16 tiles (KT a side; rows and columns beyond k are
// the identity).  For each tile column J: wave 0 factors the diagonal tile
// in registers (lane r holds row r; pivots and rows broadcast with
// v_readlane) and inverts it by forward substitution; then the tiles below
// it become L_IJ = A_IJ L_JJ^{-T} and the trailing tiles A_II' -= L_IJ
// L_I'J^T, on the FP64 matrix cores, a tile a wave.  The inverse's
// off-diagonal tiles follow by diagonals, X_IJ = -X_II (sum_P L_IP X_PJ):
// register v of the inner sum's accumulator holds K index lg + 4 v, which
// is the outer product's B operand of step v, so the sum never leaves the
// registers.  Retries with the same growing shifts as k_chol_inverse.  At
// k = 64: 22 us, against 68 us for a single wave holding a row per lane
// (64 dependent steps with a square root and a division each) and 47 us
// for this kernel with its 16-step loop not unrolled (a conditional exit
// in it: the tile's rows then need dynamic register indexing).
// ---------------------------------------------------------------------------
// 1 / a for a positive normal a: v_rcp_f64 refined by two Newton steps
__device__ __forceinline__ double recip_nr(double a) {
  double y = __builtin_amdgcn_rcp(a);
  double e = fma(-a, y, 1.0);
  y = fma(y, e, y);
  e = fma(-a, y, 1.0);
  return fma(y, e, y);
}

template <int KT>
__global__ __launch_bounds__(256) void k_chol_blk(const double* __restrict__ G, int k, double* __restrict__ R,
                                                  double* __restrict__ Rinv, int* d_flags, int flag_bit,
                                                  int* d_fail) {
  constexpr int KM = 16 * KT, LD = KM + 1;
  extern __shared__ double chol_lds[];
  double* A = chol_lds;       // KM x LD: the matrix, then L in its lower triangle
  double* X = A + KM * LD;    // KM x LD: L^{-1} in its lower triangle
  __shared__ int bad;
  const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63, li = lane & 15, lg = lane >> 4;
  double shift = 0.0, grow = 0.0;
  for (int attempt = 0; attempt < 6; ++attempt) {
    if (attempt == 1) {   // the trace, only when a shift is needed
      double tr = 0.0;
      for (int i = lane; i < k; i += 64) tr += G[i * k + i];
      tr = wave_sum(tr);
      grow = 1e-12 * fmax(tr, 1e-300) / k;
    }
    if (attempt > 0) {
      shift = grow;  // 1e-12, 1e-10, ... times tr(G) / k
      grow *= 100.0;
    }
    // all of a thread's loads in flight at once (clamped index, masked value)
#pragma unroll
    for (int i = 0; i < KM * KM / 256; ++i) {
      const int e = tid + 256 * i, p = e / KM, q = e - p * KM;
      const bool in = p < k && q < k;
      const double g = G[in ? p * k + q : 0];
      A[p * LD + q] = in ? g + (p == q ? shift : 0.0) : (p == q ? 1.0 : 0.0);
    }
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int J = 0; J < KT; ++J) {
      if (wid == 0) {
        // symmetric elimination: step j takes row j (lane j) off the rows
        // below with the factor A[r][j] / pivot, so only a reciprocal
        // (v_rcp_f64 and two Newton steps) is on the chain of dependent
        // steps; the columns are scaled by 1 / sqrt(pivot) at the end
        const int r = li;
        double* at = A + (16 * J + r) * LD + 16 * J;
        double d[16], pv[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) d[c] = at[c];
        bool fail = false;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          // no early exit: a break would keep the loop from being
          // unrolled, and d[j] would need dynamic register indexing
          const double piv = lane_value(d[j], j);   // the same in every lane
          fail = fail || !(piv > 0.0) || !isfinite(piv);
          pv[j] = piv;
          const double cj = !fail && r > j ? d[j] * recip_nr(piv) : 0.0;
#pragma unroll
          for (int c = j + 1; c < 16; ++c) d[c] = fma(-cj, lane_value(d[c], j), d[c]);
        }
        if (fail) {
          if (lane == 0) bad = 1;
        } else {
          // lane r: 1 / L[r][r]; L[r][j] = d[j] / sqrt(pivot j) for r >= j
          double mp = 1.0;
#pragma unroll
          for (int j = 0; j < 16; ++j) mp = r == j ? pv[j] : mp;
          const double rs = 1.0 / sqrt(mp);
          double rsv[16];
#pragma unroll
          for (int j = 0; j < 16; ++j) {
            rsv[j] = lane_value(rs, j);
            d[j] = r >= j ? d[j] * rsv[j] : 0.0;
          }
          if (lane < 16) {
#pragma unroll
            for (int c = 0; c < 16; ++c) at[c] = d[c];
          }
          wave_sync();
          // X = L^{-1} by forward substitution, lane c column c (rows above
          // c come out zero)
          double x[16];
          const double* lt = A + 16 * J * LD + 16 * J;
#pragma unroll
          for (int rr = 0; rr < 16; ++rr) {
            double s0 = rr == li ? 1.0 : 0.0, s1 = 0.0;
#pragma unroll
            for (int q = 0; q < rr; ++q) {
              if (q & 1)
                s1 = fma(-lt[rr * LD + q], x[q], s1);
              else
                s0 = fma(-lt[rr * LD + q], x[q], s0);
            }
            x[rr] = (s0 + s1) * rsv[rr];
          }
          if (lane < 16) {
#pragma unroll
            for (int rr = 0; rr < 16; ++rr) X[(16 * J + rr) * LD + 16 * J + li] = x[rr];
          }
        }
      }
      __syncthreads();
      if (bad) break;
      // the tiles below the diagonal one: L_IJ = A_IJ X_JJ^T
      if (wid < KT - 1 - J) {
        const int I = J + 1 + wid;
        doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 4; ++s)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[(16 * I + li) * LD + 16 * J + 4 * s + lg],
                                                     X[(16 * J + li) * LD + 16 * J + 4 * s + lg], acc, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) A[(16 * I + lg + 4 * v) * LD + 16 * J + li] = acc[v];
      }
      __syncthreads();
      // the trailing tiles (I, I2), J < I2 <= I: A_II2 -= L_IJ L_I2J^T
      const int m = KT - 1 - J;
      for (int t = wid; t < m * (m + 1) / 2; t += 4) {
        int t2 = t, I = J + 1;
        while (t2 >= I - J) {
          t2 -= I - J;
          ++I;
        }
        const int I2 = J + 1 + t2;
        doublex4 acc;
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] = A[(16 * I + lg + 4 * v) * LD + 16 * I2 + li];
#pragma unroll
        for (int s = 0; s < 4; ++s)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-A[(16 * I + li) * LD + 16 * J + 4 * s + lg],
                                                     A[(16 * I2 + li) * LD + 16 * J + 4 * s + lg], acc, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) A[(16 * I + lg + 4 * v) * LD + 16 * I2 + li] = acc[v];
      }
      __syncthreads();
    }
    if (!bad) break;
    __syncthreads();   // every wave has read the flag before the next attempt resets it
  }
  if (bad) {
    if (tid == 0) *d_fail = 1;
    return;
  }
  if (tid == 0 && shift > 0.0 && d_flags) atomicOr(d_flags, flag_bit);
  // the inverse's off-diagonal tiles, diagonal dd by diagonal
  for (int dd = 1; dd < KT; ++dd) {
    if (wid < KT - dd) {
      const int I = dd + wid, J = I - dd;
      doublex4 T = {0.0, 0.0, 0.0, 0.0};
      for (int P = J; P < I; ++P) {
#pragma unroll
        for (int s = 0; s < 4; ++s)
          T = __builtin_amdgcn_mfma_f64_16x16x4f64(A[(16 * I + li) * LD + 16 * P + 4 * s + lg],
                                                   X[(16 * P + 4 * s + lg) * LD + 16 * J + li], T, 0, 0, 0);
      }
      doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < 4; ++s)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-X[(16 * I + li) * LD + 16 * I + 4 * s + lg], T[s], acc, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) X[(16 * I + lg + 4 * v) * LD + 16 * J + li] = acc[v];
    }
    __syncthreads();
  }
  // R = L^T, R^{-1} = (L^{-1})^T
  for (int e = tid; e < k * k; e += 256) {
    const int p = e / k, q = e - p * k;
    R[e] = q >= p ? A[q * LD + p] : 0.0;
    Rinv[e] = q >= p ? X[q * LD + p] : 0.0;
  }
}

// Threads of the Jacobi workgroup: one pass over the (m/2)^2 2 x 2 blocks and
// the m^2/2 eigenvector pairs of a step (measured at l = 48: the whole
// symnmf_lai 3.07 ms with 256 threads, 2.92 ms with 1024).  A variant with A
// in two copies, where every task computes its two rotations itself and a
// step takes one barrier instead of two, measured slower (l = 48: 539 against
// 322 us): the rotations' square roots and divisions, repeated by all sixteen
// waves, cost the one CU more FP64 issue time than the barrier.
constexpr int JACOBI_NT = 1024;

// ---------------------------------------------------------------------------
// Parallel cyclic Jacobi (round-robin pairing) on A = (T + T^T) / 2 in LDS;
// V accumulated in LDS next to A, then columns sorted by descending
// eigenvalue into V.
// ---------------------------------------------------------------------------
// Pair `t` of round-robin step `step` over m (even) indices: index 0 fixed,
// 1..m-1 rotated by the step; returned with p < q.
__device__ __forceinline__ void jacobi_pair(int t, int step, int m, int& p, int& q) {
  // both sums are below 2 (m - 1): one conditional subtraction each, no
  // integer division
  int x = t - 1 + step, y = m - 2 - t + step;
  x -= x >= m - 1 ? m - 1 : 0;
  y -= y >= m - 1 ? m - 1 : 0;
  const int a = t == 0 ? 0 : 1 + x, b = 1 + y;
  p = a < b ? a : b;
  q = a < b ? b : a;
}

__global__ __launch_bounds__(JACOBI_NT) void k_jacobi(const double* __restrict__ T, int l, double* __restrict__ V,
                                                double* __restrict__ lam) {
  // A: m x (m + 1) (m = l rounded up to even; the extra row and column are
  // zero, so rotations that pair with them are the identity), then the
  // eigenvectors V (m x (m + 1)).
  extern __shared__ double A[];
  const int m = l + (l & 1);
  const int lda = m + 1;
  double* Vw = A + m * lda;
  __shared__ double2 rot[48];  // (c, s) of each pair of the step
  __shared__ double red[JACOBI_NT / 64];
  __shared__ int order[96];
  __shared__ int conv;
  const int tid = threadIdx.x;
  const int half = m / 2;
  for (int e = tid; e < m * m; e += JACOBI_NT) {
    const int p = e / m, q = e - p * m;
    A[p * lda + q] = (p < l && q < l) ? 0.5 * (T[p * l + q] + T[q * l + p]) : 0.0;
    Vw[p * lda + q] = (p == q) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, dg = 0.0;
    for (int e = tid; e < m * m; e += JACOBI_NT) {
      const int p = e / m, q = e - p * m;
      const double a = A[p * lda + q];
      if (p == q) dg += a * a; else off += a * a;
    }
    const double toff = block_sum(off, red);
    __syncthreads();
    const double tdg = block_sum(dg, red);
    if (tid == 0) conv = (toff <= 1e-30 * (toff + tdg)) ? 1 : 0;
    __syncthreads();
    if (conv) break;
    for (int step = 0; step < m - 1; ++step) {
      // round-robin (circle) pairing: index 0 fixed, 1..m-1 rotate by `step`
      if (tid < half) {
        int p, q;
        jacobi_pair(tid, step, m, p, q);
        double c = 1.0, s = 0.0;
        const double apq = A[p * lda + q];
        if (fabs(apq) > 1e-300) {
          const double theta = (A[q * lda + q] - A[p * lda + p]) / (2.0 * apq);
          const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
        }
        rot[tid] = make_double2(c, s);
      }
      __syncthreads();
      // one task per (pair a, pair b): the 2 x 2 block of A on the rows of
      // pair a and the columns of pair b (its columns rotated by pair b, then
      // its rows by pair a), and rows 2a, 2a + 1 of V on the columns of pair
      // b.  Pair indices are recomputed, so every read of a task is issued at
      // once; the tasks touch disjoint entries.
      for (int e = tid; e < half * half; e += JACOBI_NT) {
        const int a = e / half, b = e - a * half;
        int pa, qa, pb, qb;
        jacobi_pair(a, step, m, pa, qa);
        jacobi_pair(b, step, m, pb, qb);
        const double2 ra = rot[a], rb = rot[b];
        const double x00 = A[pa * lda + pb], x01 = A[pa * lda + qb];
        const double x10 = A[qa * lda + pb], x11 = A[qa * lda + qb];
        const int r0 = 2 * a;
        const double v0p = Vw[r0 * lda + pb], v0q = Vw[r0 * lda + qb];
        const double v1p = Vw[(r0 + 1) * lda + pb], v1q = Vw[(r0 + 1) * lda + qb];
        const double ca = ra.x, sa = ra.y, cb = rb.x, sb = rb.y;
        const double y00 = cb * x00 - sb * x01, y01 = sb * x00 + cb * x01;
        const double y10 = cb * x10 - sb * x11, y11 = sb * x10 + cb * x11;
        A[pa * lda + pb] = ca * y00 - sa * y10;
        A[qa * lda + pb] = sa * y00 + ca * y10;
        A[pa * lda + qb] = ca * y01 - sa * y11;
        A[qa * lda + qb] = sa * y01 + ca * y11;
        Vw[r0 * lda + pb] = cb * v0p - sb * v0q;
        Vw[r0 * lda + qb] = sb * v0p + cb * v0q;
        Vw[(r0 + 1) * lda + pb] = cb * v1p - sb * v1q;
        Vw[(r0 + 1) * lda + qb] = sb * v1p + cb * v1q;
      }
      __syncthreads();
    }
  }
  // rank of each eigenvalue in descending order (ties by index)
  for (int i = tid; i < l; i += JACOBI_NT) {
    const double v = A[i * lda + i];
    int rank = 0;
    for (int j = 0; j < l; ++j) {
      const double u = A[j * lda + j];
      rank += (u > v || (u == v && j < i)) ? 1 : 0;
    }
    order[rank] = i;
  }
  __syncthreads();
  for (int i = tid; i < l; i += JACOBI_NT) lam[i] = A[order[i] * lda + order[i]];
  for (int e = tid; e < l * l; e += JACOBI_NT) {
    const int r = e / l, j = e - r * l;
    V[e] = Vw[r * lda + order[j]];
  }
}

__global__ __launch_bounds__(256) void k_col_argmax(const double* __restrict__ U, int n, int l, double* __restrict__ sgn) {
  __shared__ double bv[256];
  __shared__ int bi[256];
  const int j = blockIdx.x;
  double best = -1.0;
  int bidx = 0x7fffffff;
  int i = threadIdx.x;
  for (; i + 7 * 256 < n; i += 8 * 256) {   // 8 loads in flight, compared in row order
    double a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = fabs(U[(int64_t)(i + 256 * u) * l + j]);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (a[u] > best) {
        best = a[u];
        bidx = i + 256 * u;
      }
    }
  }
  for (; i < n; i += 256) {
    const double a = fabs(U[(int64_t)i * l + j]);
    if (a > best) {
      best = a;
      bidx = i;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = bidx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const double a = bv[threadIdx.x + o];
      const int ai = bi[threadIdx.x + o];
      if (a > bv[threadIdx.x] || (a == bv[threadIdx.x] && ai < bi[threadIdx.x])) {
        bv[threadIdx.x] = a;
        bi[threadIdx.x] = ai;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) sgn[j] = (U[(int64_t)bi[0] * l + j] < 0.0) ? -1.0 : 1.0;
}

__global__ __launch_bounds__(256) void k_col_scale(double* __restrict__ U, int n, int l, const double* __restrict__ sgn) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)n * l) return;
  U[e] *= sgn[e % l];
}

// ---------------------------------------------------------------------------
// Scans: 1024 items per block (4 per thread); the block totals, then each
// block's pass adding the totals of the blocks before it.
// ---------------------------------------------------------------------------

// The scans' input: an array, or the sampler's selection flag of each row
// (deterministic, or drawn at least once) formed on the fly.
template <typename T>
struct ScanArray {
  const T* p;
  __device__ T operator()(int i) const { return p[i]; }
};
struct ScanSelected {
  const int* det;
  const int* counts;
  __device__ int operator()(int i) const { return (det[i] || counts[i] > 0) ? 1 : 0; }
};

template <typename T, typename L>
__global__ __launch_bounds__(256) void k_scan_blocks(L in, int n, T* __restrict__ bsum) {
  __shared__ T ws[4];
  const int base = blockIdx.x * 1024 + threadIdx.x * 4;
  T s = 0;
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (base + u < n) s += in(base + u);
  T tot;
  block_exclusive_scan<T>(s, ws, tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Each block's offset is the sum of the block totals before it, read by the
// block itself (integers: exact in any order; at most a few thousand totals,
// cache-resident), so the scan takes two launches, not three.
template <typename T, bool INCLUSIVE, typename L>
__global__ __launch_bounds__(256) void k_scan_apply(L in, int n, const T* __restrict__ bsum, T* __restrict__ out,
                                                    T* __restrict__ grand) {
  __shared__ T ws[4];
  T pre = 0;
  for (int b = threadIdx.x; b < (int)blockIdx.x; b += 256) pre += bsum[b];
  T off;
  block_exclusive_scan<T>(pre, ws, off);
  const int base = blockIdx.x * 1024 + threadIdx.x * 4;
  T v[4];
  T s = 0;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    v[u] = (base + u < n) ? in(base + u) : (T)0;
    s += v[u];
  }
  T tot;
  T run = block_exclusive_scan<T>(s, ws, tot) + off;
  if (grand && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *grand = off + tot;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    if (INCLUSIVE) run += v[u];
    if (base + u < n) out[base + u] = run;
    if (!INCLUSIVE) run += v[u];
  }
}

template <typename TA, typename TB, int T>
void gram_launch(const void* A, int64_t lda, int ca, const void* B, int64_t ldb, int cb, int n, const int* rows,
                 const double* w, const int* d_count, int nb, int rpb, double* part, const DevState* st,
                 hipStream_t s) {
  k_gram<TA, TB, T><<<nb, 256, 0, s>>>((const TA*)A, lda, ca, (const TB*)B, ldb, cb, n, rows, w, d_count, rpb, part,
                                       st);
}

template <typename TA, typename TB>
void gram_t(int t, const void* A, int64_t lda, int ca, const void* B, int64_t ldb, int cb, int n, const int* rows,
            const double* w, const int* d_count, int nb, int rpb, double* part, const DevState* st, hipStream_t s) {
  switch (t) {
    case 1: gram_launch<TA, TB, 1>(A, lda, ca, B, ldb, cb, n, rows, w, d_count, nb, rpb, part, st, s); break;
    case 2: gram_launch<TA, TB, 2>(A, lda, ca, B, ldb, cb, n, rows, w, d_count, nb, rpb, part, st, s); break;
    case 3: gram_launch<TA, TB, 3>(A, lda, ca, B, ldb, cb, n, rows, w, d_count, nb, rpb, part, st, s); break;
    case 4: gram_launch<TA, TB, 4>(A, lda, ca, B, ldb, cb, n, rows, w, d_count, nb, rpb, part, st, s); break;
    case 5: gram_launch<TA, TB, 5>(A, lda, ca, B, ldb, cb, n, rows, w, d_count, nb, rpb, part, st, s); break;
    default: gram_launch<TA, TB, 6>(A, lda, ca, B, ldb, cb, n, rows, w, d_count, nb, rpb, part, st, s); break;
  }
}

}  // namespace

// ===========================================================================
// Launchers
// ===========================================================================

void sum_partials(const double* part, int nb, double* out, hipStream_t s) {
  k_sum_partials<<<1, 256, 0, s>>>(part, nb, out);
}

int init_uniform_factor(void* F, int fdtype, int n, int k, double scale, uint64_t seed, hipStream_t s) {
  const int64_t cnt = (int64_t)n * k;
  if (fdtype == SYMNMF_F64)
    k_init_uniform<double><<<ceil_div(cnt, 256), 256, 0, s>>>((double*)F, cnt, scale, seed);
  else
    k_init_uniform<float><<<ceil_div(cnt, 256), 256, 0, s>>>((float*)F, cnt, scale, seed);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int copy_convert(const void* src, int sdtype, void* dst, int ddtype, int64_t count, hipStream_t s) {
  const int nb = ceil_div(count, 256);
  if (sdtype == SYMNMF_F64 && ddtype == SYMNMF_F64)
    k_convert<double, double><<<nb, 256, 0, s>>>((const double*)src, (double*)dst, count);
  else if (sdtype == SYMNMF_F64 && ddtype == SYMNMF_F32)
    k_convert<double, float><<<nb, 256, 0, s>>>((const double*)src, (float*)dst, count);
  else if (sdtype == SYMNMF_F32 && ddtype == SYMNMF_F64)
    k_convert<float, double><<<nb, 256, 0, s>>>((const float*)src, (double*)dst, count);
  else if (sdtype == SYMNMF_F32 && ddtype == SYMNMF_F32)
    k_convert<float, float><<<nb, 256, 0, s>>>((const float*)src, (float*)dst, count);
  else
    return -1;
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int gram(const void* A, int adtype, int64_t lda, int ca, const void* B, int bdtype, int64_t ldb, int cb, int n,
         const int* rows, const double* w, const int* d_count, int max_rows, Workspace& ws, double* G, double* Ghat,
         int kp, double alpha, const DevState* st, hipStream_t s, double* Ginv) {
  if (ca > 96 || cb > 96 || ca < 1 || cb < 1) return -1;
  const int t = ceil_div(std::max(ca, cb), 16);
  const int nrows = rows ? max_rows : n;
  // 64 rows per block (256 blocks at n = 16384; more rows per block chain
  // more load latencies); past 2^16 rows up to 1024 blocks, so that each SIMD
  // has several waves whose chunk loads overlap (the partials must fit the
  // workspace)
  int nbmax = nrows > (1 << 16) ? 1024 : 256;
  // at most half of the free workspace: callers take several Gram matrices
  // one after another without releasing it
  nbmax = (int)std::min<size_t>((size_t)nbmax, std::max<size_t>(1, ws.avail_doubles() / (2 * (size_t)ca * cb)));
  const int nb = std::max(1, std::min(nbmax, ceil_div(std::max(nrows, 1), 64)));
  const int rpb = 16 * ceil_div(ceil_div(std::max(nrows, 1), nb), 16);
  double* part = ws.dbl((size_t)nb * ca * cb);
  if (!part) return -1;
  if (adtype == SYMNMF_F64 && bdtype == SYMNMF_F64)
    gram_t<double, double>(t, A, lda, ca, B, ldb, cb, n, rows, w, d_count, nb, rpb, part, st, s);
  else if (adtype == SYMNMF_F32 && bdtype == SYMNMF_F32)
    gram_t<float, float>(t, A, lda, ca, B, ldb, cb, n, rows, w, d_count, nb, rpb, part, st, s);
  else if (adtype == SYMNMF_F64 && bdtype == SYMNMF_F32)
    gram_t<double, float>(t, A, lda, ca, B, ldb, cb, n, rows, w, d_count, nb, rpb, part, st, s);
  else if (adtype == SYMNMF_F32 && bdtype == SYMNMF_F64)
    gram_t<float, double>(t, A, lda, ca, B, ldb, cb, n, rows, w, d_count, nb, rpb, part, st, s);
  else
    return -1;
  const int tot = std::max(ca * cb, Ghat ? kp * kp : 0);
  k_gram_reduce<<<ceil_div(tot, GR_COLS), GR_SLICES * GR_COLS, 0, s>>>(part, nb, ca, cb, G, Ghat, kp, alpha, Ginv, st);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int dot_partials(const void* A, const void* B, int dtype, int64_t count, Workspace& ws, double** part,
                 const DevState* st, hipStream_t s) {
  const int nb = std::max(1, std::min(512, ceil_div(count, 256 * 16)));
  *part = ws.dbl(nb);
  if (!*part) return -1;
  if (dtype == SYMNMF_F64)
    k_dot<double><<<nb, 256, 0, s>>>((const double*)A, (const double*)B, count, *part, st);
  else
    k_dot<float><<<nb, 256, 0, s>>>((const float*)A, (const float*)B, count, *part, st);
  return hipGetLastError() == hipSuccess ? nb : -1;
}

void frob_dot(const double* A, const double* B, int count, double* out, hipStream_t s) {
  k_frob<<<1, 256, 0, s>>>(A, B, count, out);
}

void finish_iteration(const double* dot_part, int nb, const double* Ga, const double* Gb, int k,
                      const double* d_normsq, DevState* st, double* hist, StopRule rule, hipStream_t s) {
  k_finish_iteration<<<1, 256, 0, s>>>(dot_part, nb, Ga, Gb, k, d_normsq, st, hist, rule);
}

int rowmat(const void* A, int adtype, int64_t lda, int n, int l, const double* M, const double* scale, int c,
           void* out, int odtype, int64_t ldo, const DevState* st, hipStream_t s) {
  if (l >= 1 && l <= 96 && c >= 1 && c <= 96) {
    int rc;
    if (adtype == SYMNMF_F64 && odtype == SYMNMF_F64)
      rc = rowmat_mfma<double, double>((const double*)A, lda, n, l, M, scale, c, (double*)out, ldo, st, s);
    else if (adtype == SYMNMF_F64 && odtype == SYMNMF_F32)
      rc = rowmat_mfma<double, float>((const double*)A, lda, n, l, M, scale, c, (float*)out, ldo, st, s);
    else if (adtype == SYMNMF_F32 && odtype == SYMNMF_F64)
      rc = rowmat_mfma<float, double>((const float*)A, lda, n, l, M, scale, c, (double*)out, ldo, st, s);
    else if (adtype == SYMNMF_F32 && odtype == SYMNMF_F32)
      rc = rowmat_mfma<float, float>((const float*)A, lda, n, l, M, scale, c, (float*)out, ldo, st, s);
    else
      return -1;
    if (rc) return rc;
    return hipGetLastError() == hipSuccess ? 0 : -1;
  }
  const int nb = ceil_div((int64_t)n * c, 256);
  if (adtype == SYMNMF_F64 && odtype == SYMNMF_F64)
    k_rowmat<double, double><<<nb, 256, 0, s>>>((const double*)A, lda, n, l, M, scale, c, (double*)out, ldo, st);
  else if (adtype == SYMNMF_F64 && odtype == SYMNMF_F32)
    k_rowmat<double, float><<<nb, 256, 0, s>>>((const double*)A, lda, n, l, M, scale, c, (float*)out, ldo, st);
  else if (adtype == SYMNMF_F32 && odtype == SYMNMF_F64)
    k_rowmat<float, double><<<nb, 256, 0, s>>>((const float*)A, lda, n, l, M, scale, c, (double*)out, ldo, st);
  else if (adtype == SYMNMF_F32 && odtype == SYMNMF_F32)
    k_rowmat<float, float><<<nb, 256, 0, s>>>((const float*)A, lda, n, l, M, scale, c, (float*)out, ldo, st);
  else
    return -1;
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int chol_inverse(const double* G, int k, double* R, double* Rinv, int* d_flags, int flag_bit, int* d_fail,
                 hipStream_t s) {
  if (k >= 1 && k <= 64) {
    const int kt = ceil_div(k, 16);
    const size_t lds = 2 * sizeof(double) * (16 * kt) * (16 * kt + 1);
    switch (kt) {
      case 1: k_chol_blk<1><<<1, 256, lds, s>>>(G, k, R, Rinv, d_flags, flag_bit, d_fail); break;
      case 2: k_chol_blk<2><<<1, 256, lds, s>>>(G, k, R, Rinv, d_flags, flag_bit, d_fail); break;
      case 3: k_chol_blk<3><<<1, 256, lds, s>>>(G, k, R, Rinv, d_flags, flag_bit, d_fail); break;
      default:
        if (hipFuncSetAttribute((const void*)k_chol_blk<4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
            hipSuccess)
          return -1;
        k_chol_blk<4><<<1, 256, lds, s>>>(G, k, R, Rinv, d_flags, flag_bit, d_fail);
        break;
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
  }
  const size_t lds = 2 * (size_t)k * (k + 1) * sizeof(double);
  if (k > 96) return -1;
  if (lds > 65536) {
    if (hipFuncSetAttribute((const void*)k_chol_inverse, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
        hipSuccess)
      return -1;
  }
  k_chol_inverse<<<1, 256, lds, s>>>(G, k, R, Rinv, d_flags, flag_bit, d_fail);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int jacobi_evd(const double* T, int l, double* V, double* lam, hipStream_t s) {
  if (l > 96) return -1;
  const int m = l + (l & 1);
  const size_t lds = 2 * (size_t)m * (m + 1) * sizeof(double);
  if (lds > 65536) {
    if (hipFuncSetAttribute((const void*)k_jacobi, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
      return -1;
  }
  k_jacobi<<<1, JACOBI_NT, lds, s>>>(T, l, V, lam);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int column_sign_fix(double* U, int n, int l, Workspace& ws, hipStream_t s) {
  double* sgn = ws.dbl(l);
  if (!sgn) return -1;
  k_col_argmax<<<l, 256, 0, s>>>(U, n, l, sgn);
  k_col_scale<<<ceil_div((int64_t)n * l, 256), 256, 0, s>>>(U, n, l, sgn);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int exclusive_scan_i32(const int* in, int* out, int n, Workspace& ws, hipStream_t s) {
  const int nb = std::max(1, ceil_div(n, 1024));
  int* bsum = ws.i32(nb);
  if (!bsum) return -1;
  k_scan_blocks<int><<<nb, 256, 0, s>>>(ScanArray<int>{in}, n, bsum);
  k_scan_apply<int, false><<<nb, 256, 0, s>>>(ScanArray<int>{in}, n, bsum, out, out + n);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int selected_block_sums(const int* det, const int* counts, int n, int* bsum, hipStream_t s) {
  const int nb = std::max(1, ceil_div(n, 1024));
  k_scan_blocks<int><<<nb, 256, 0, s>>>(ScanSelected{det, counts}, n, bsum);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int inclusive_scan_u64_from_sums(const uint64_t* in, uint64_t* out, int n, const uint64_t* bsum, hipStream_t s) {
  const int nb = std::max(1, ceil_div(n, 1024));
  k_scan_apply<uint64_t, true><<<nb, 256, 0, s>>>(ScanArray<uint64_t>{in}, n, bsum, out, (uint64_t*)nullptr);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

