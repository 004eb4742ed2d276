// Dense-X kernels: one-time scalars pass, the product Y = X B on MFMA
// (FP64, FP32 and BF16 inputs), split-K reduction, FP32 -> BF16 conversion and
// the exact residual pass.
//
// The product X B (B = H, W, the sketch Omega or the basis Q) is the main
// cost of every iteration (Section 2.1.2: X H is reused by a whole HALS
// sweep; Section 3.1 complexity).  X is streamed exactly once per product, so
// the kernel is laid out for HBM streaming: each wave owns 16*RT rows of X
// and reads them with 16-byte loads straight into MFMA A-operands; the B
// panel of the current K tile is staged once per workgroup in LDS and shared
// by its four waves.
#include "kernels.hpp"

namespace {

// ---------------------------------------------------------------------------
// Scalars pass: per column j (= row j, X symmetric) the sum, the sum of
// squares and the max over a chunk of rows; then a fixed-order combine.
// ---------------------------------------------------------------------------
template <typename TX>
__global__ __launch_bounds__(256) void k_dense_colstats(const TX* __restrict__ X, int64_t ld, int n, int rows_per_chunk,
                                                        double* __restrict__ psum, double* __restrict__ psq,
                                                        double* __restrict__ pmax) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int c = blockIdx.y;
  if (j >= n) return;
  const int r0 = c * rows_per_chunk;
  const int r1 = min(n, r0 + rows_per_chunk);
  double s = 0.0, q = 0.0, m = -INFINITY;
  for (int r = r0; r < r1; ++r) {
    const double v = to_f64(X[(int64_t)r * ld + j]);
    s += v;
    q += v * v;
    m = fmax(m, v);
  }
  psum[(int64_t)c * n + j] = s;
  psq[(int64_t)c * n + j] = q;
  pmax[(int64_t)c * n + j] = m;
}

__global__ __launch_bounds__(256) void k_colstats_combine(int n, int chunks, const double* __restrict__ psum,
                                                          const double* __restrict__ psq,
                                                          const double* __restrict__ pmax,
                                                          double* __restrict__ rowsum, double* __restrict__ bpart) {
  __shared__ double sc[8];
  const int j = blockIdx.x * 256 + threadIdx.x;
  double s = 0.0, q = 0.0, m = -INFINITY;
  if (j < n) {
    for (int c = 0; c < chunks; ++c) {
      s += psum[(int64_t)c * n + j];
      q += psq[(int64_t)c * n + j];
      m = fmax(m, pmax[(int64_t)c * n + j]);
    }
    rowsum[j] = s;
  }
  const double ts = block_sum(j < n ? s : 0.0, sc);
  const double tq = block_sum(j < n ? q : 0.0, sc);
  // max: fixed tree via LDS
  __shared__ double smax[256];
  smax[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    bpart[3 * blockIdx.x + 0] = ts;
    bpart[3 * blockIdx.x + 1] = tq;
    bpart[3 * blockIdx.x + 2] = smax[0];
  }
}

__global__ void k_scalars_final(int nb, const double* __restrict__ bpart, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0, q = 0.0, m = -INFINITY;
  for (int b = 0; b < nb; ++b) {
    s += bpart[3 * b];
    q += bpart[3 * b + 1];
    m = fmax(m, bpart[3 * b + 2]);
  }
  out[0] = q;  // ||X||_F^2
  out[1] = s;  // sum of all entries
  out[2] = m;  // max entry
}

// ---------------------------------------------------------------------------
// MFMA product P[split] = X[:, krange] B[krange, :], FP32 or FP64 operands.
// v_mfma_{f32,f64}_16x16x4: lane l supplies A[l%16][l/16] and B[l/16][l%16];
// accumulator element v of lane l is D[4*(l/16)+v][l%16].  A lane reads four
// consecutive columns of its X row (k0+4g..k0+4g+3, g = l/16) and issues one
// MFMA per column, pairing it with the matching row of the staged B tile,
// which covers the 16 columns k0..k0+15 per sub-step.
// ---------------------------------------------------------------------------
template <typename T> struct Mfma;
template <> struct Mfma<float> {
  using acc_t = floatx4;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<double> {
  using acc_t = doublex4;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = floatx4; };
template <> struct Vec4<double> { using type = doublex4; };

constexpr int GEMM_KT = 64;

template <typename TX, typename TB, int NT, int RT>
__global__ __launch_bounds__(256) void k_gemm_mfma(const TX* __restrict__ X, int64_t ldx, const TB* __restrict__ B,
                                                   int64_t ldb, int n, int c, int kchunk, TX* __restrict__ P, int cp,
                                                   const DevState* __restrict__ st) {
  if (stopped(st)) return;
  using M = Mfma<TX>;
  using acc_t = typename M::acc_t;
  constexpr int CP = 16 * NT;
  constexpr int LDB = CP + 4;
  __shared__ TX Bs[GEMM_KT * LDB];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int row_base = blockIdx.x * (64 * RT) + wave * (16 * RT);
  const int kb = blockIdx.y * kchunk;
  const int ke = min(n, kb + kchunk);

  acc_t acc[RT][NT];
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[r][t] = acc_t{0, 0, 0, 0};

  const TX* xrow[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int rr = min(row_base + 16 * r + li, n - 1);
    xrow[r] = X + (int64_t)rr * ldx;
  }
  const bool vec_ok = ((ldx & 3) == 0) && ((((uintptr_t)X) & (4 * sizeof(TX) - 1)) == 0);

  for (int k0 = kb; k0 < ke; k0 += GEMM_KT) {
    // Issue the X loads for this tile first so they overlap the B staging.
    TX xv[RT][4][4];
    if (vec_ok && k0 + GEMM_KT <= ke) {
#pragma unroll
      for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int ss = 0; ss < 4; ++ss) {
          typename Vec4<TX>::type v =
              __builtin_nontemporal_load((const typename Vec4<TX>::type*)(xrow[r] + k0 + 16 * ss + 4 * lg));
          xv[r][ss][0] = v.x;
          xv[r][ss][1] = v.y;
          xv[r][ss][2] = v.z;
          xv[r][ss][3] = v.w;
        }
    } else {
#pragma unroll
      for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int ss = 0; ss < 4; ++ss)
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int col = k0 + 16 * ss + 4 * lg + t;
            xv[r][ss][t] = (col < ke) ? xrow[r][col] : (TX)0;
          }
    }
    __syncthreads();
    for (int e = tid; e < GEMM_KT * CP; e += 256) {
      const int kk = e / CP, cc = e - kk * CP;
      const int kg = k0 + kk;
      TX v = (TX)0;
      if (kg < ke && cc < c) v = (TX)B[(int64_t)kg * ldb + cc];
      Bs[kk * LDB + cc] = v;
    }
    __syncthreads();
#pragma unroll
    for (int ss = 0; ss < 4; ++ss)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const TX* brow = Bs + (16 * ss + 4 * lg + t) * LDB + li;
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) {
          const TX b = brow[16 * ct];
#pragma unroll
          for (int r = 0; r < RT; ++r) acc[r][ct] = M::mma(xv[r][ss][t], b, acc[r][ct]);
        }
      }
  }
  TX* out = P + (int64_t)blockIdx.y * n * cp;
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = row_base + 16 * r + 4 * lg + v;
      if (row < n) {
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) {
          const int col = 16 * ct + li;
          if (col < cp) out[(int64_t)row * cp + col] = acc[r][ct][v];
        }
      }
    }
}

// ---------------------------------------------------------------------------
// BF16 MFMA product (FP32 accumulate): v_mfma_f32_16x16x32_bf16.  Lane l
// supplies 8 consecutive K values of A row l%16 and of B column l%16, group
// g = l/16 covering K offsets 8g..8g+7 of the 32-wide step; accumulator layout
// as above.  B is rounded to BF16 (nearest even) while staged, transposed, in
// LDS so a lane reads its 8 values with one 16-byte load.
// ---------------------------------------------------------------------------
constexpr int BF_KT = 128;

template <typename TB, int NT, int RT>
__global__ __launch_bounds__(256) void k_gemm_bf16(const __bf16* __restrict__ X, int64_t ldx,
                                                   const TB* __restrict__ B, int64_t ldb, int n, int c, int kchunk,
                                                   float* __restrict__ P, int cp, const DevState* __restrict__ st) {
  if (stopped(st)) return;
  constexpr int CP = 16 * NT;
  constexpr int LDK = BF_KT + 8;  // bf16 elements per staged B column
  __shared__ __bf16 Bs[CP * LDK];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int row_base = blockIdx.x * (64 * RT) + wave * (16 * RT);
  const int kb = blockIdx.y * kchunk;
  const int ke = min(n, kb + kchunk);

  floatx4 acc[RT][NT];
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[r][t] = floatx4{0, 0, 0, 0};

  const __bf16* xrow[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int rr = min(row_base + 16 * r + li, n - 1);
    xrow[r] = X + (int64_t)rr * ldx;
  }
  const bool vec_ok = ((ldx & 7) == 0) && ((((uintptr_t)X) & 15) == 0);

  for (int k0 = kb; k0 < ke; k0 += BF_KT) {
    bf16x8 xv[RT][4];
    if (vec_ok && k0 + BF_KT <= ke) {
#pragma unroll
      for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int ss = 0; ss < 4; ++ss)
          xv[r][ss] = __builtin_nontemporal_load((const bf16x8*)(xrow[r] + k0 + 32 * ss + 8 * lg));
    } else {
#pragma unroll
      for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int ss = 0; ss < 4; ++ss)
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const int col = k0 + 32 * ss + 8 * lg + t;
            xv[r][ss][t] = (col < ke) ? xrow[r][col] : (__bf16)0.0f;
          }
    }
    __syncthreads();
    for (int e = tid; e < BF_KT * CP; e += 256) {
      const int kk = e / CP, cc = e - kk * CP;
      const int kg = k0 + kk;
      float v = 0.0f;
      if (kg < ke && cc < c) v = (float)B[(int64_t)kg * ldb + cc];
      Bs[cc * LDK + kk] = (__bf16)v;
    }
    __syncthreads();
#pragma unroll
    for (int ss = 0; ss < 4; ++ss)
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) {
        const bf16x8 b = *(const bf16x8*)(Bs + (16 * ct + li) * LDK + 32 * ss + 8 * lg);
#pragma unroll
        for (int r = 0; r < RT; ++r)
          acc[r][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xv[r][ss], b, acc[r][ct], 0, 0, 0);
      }
  }
  float* out = P + (int64_t)blockIdx.y * n * cp;
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = row_base + 16 * r + 4 * lg + v;
      if (row < n) {
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) {
          const int col = 16 * ct + li;
          if (col < cp) out[(int64_t)row * cp + col] = acc[r][ct][v];
        }
      }
    }
}

// Y[r][j] = sum_s P[s][r][j], j < c, fixed order over s.
template <typename TP, typename TY>
__global__ __launch_bounds__(256) void k_splitk_reduce(const TP* __restrict__ P, int splits, int n, int c, int cp,
                                                       TY* __restrict__ Y, int64_t ldy,
                                                       const DevState* __restrict__ st) {
  if (stopped(st)) return;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)n * c) return;
  const int r = (int)(e / c), j = (int)(e - (int64_t)r * c);
  double acc = 0.0;
  for (int s = 0; s < splits; ++s) acc += (double)P[((int64_t)s * n + r) * cp + j];
  Y[(int64_t)r * ldy + j] = (TY)acc;
}

__global__ __launch_bounds__(256) void k_f32_to_bf16(const float* __restrict__ src, int64_t lds, __bf16* __restrict__ dst,
                                                     int64_t ldd, int n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t tot = (int64_t)n * n;
  if (e >= tot) return;
  const int64_t r = e / n, c = e - r * n;
  dst[r * ldd + c] = (__bf16)src[r * lds + c];
}

// ---------------------------------------------------------------------------
// Exact residual pass: sum over all (i, j) of (X_ij - w_i . h_j)^2 in FP64.
// A 64 x 64 tile per workgroup; the factor rows of the tile are staged in LDS
// as FP64.
// ---------------------------------------------------------------------------
template <typename TX, typename TF>
__global__ __launch_bounds__(256) void k_resid_exact_dense(const TX* __restrict__ X, int64_t ldx, int n, int k,
                                                           const TF* __restrict__ W, const TF* __restrict__ H,
                                                           double* __restrict__ part) {
  __shared__ double Ws[64 * 65];
  __shared__ double Hs[64 * 65];
  __shared__ double sc[8];
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int tid = threadIdx.x;
  double acc = 0.0;
  // k <= 64 (checked by the caller): one stage holds every factor column.
  for (int e = tid; e < 64 * 64; e += 256) {
    const int r = e >> 6, q = e & 63;
    Ws[r * 65 + q] = (i0 + r < n && q < k) ? (double)W[(int64_t)(i0 + r) * k + q] : 0.0;
    Hs[r * 65 + q] = (j0 + r < n && q < k) ? (double)H[(int64_t)(j0 + r) * k + q] : 0.0;
  }
  __syncthreads();
  const int tj = tid & 63, ti = tid >> 6;
  const int j = j0 + tj;
  for (int ii = ti; ii < 64; ii += 4) {
    const int i = i0 + ii;
    if (i < n && j < n) {
      double d = 0.0;
      for (int q = 0; q < k; ++q) d = fma(Ws[ii * 65 + q], Hs[tj * 65 + q], d);
      const double e = to_f64(X[(int64_t)i * ldx + j]) - d;
      acc = fma(e, e, acc);
    }
  }
  const double t = block_sum(acc, sc);
  if (tid == 0) part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = t;
}

}  // namespace

// ===========================================================================
// Launchers
// ===========================================================================

int dense_scalars(const void* X, int dtype, int64_t ld, int n, Workspace& ws, double* d_rowsum, double* d_out3,
                  hipStream_t s) {
  const int chunks = std::max(1, std::min(64, ceil_div(n, 256)));
  const int rpc = ceil_div(n, chunks);
  double* psum = ws.dbl((size_t)3 * chunks * n + 3 * (size_t)ceil_div(n, 256));
  double* psq = psum + (size_t)chunks * n;
  double* pmax = psq + (size_t)chunks * n;
  double* bpart = pmax + (size_t)chunks * n;
  if (!psum) return -1;
  dim3 g(ceil_div(n, 256), chunks);
  if (dtype == SYMNMF_F64)
    k_dense_colstats<double><<<g, 256, 0, s>>>((const double*)X, ld, n, rpc, psum, psq, pmax);
  else if (dtype == SYMNMF_F32)
    k_dense_colstats<float><<<g, 256, 0, s>>>((const float*)X, ld, n, rpc, psum, psq, pmax);
  else
    k_dense_colstats<__bf16><<<g, 256, 0, s>>>((const __bf16*)X, ld, n, rpc, psum, psq, pmax);
  const int nb = ceil_div(n, 256);
  k_colstats_combine<<<nb, 256, 0, s>>>(n, chunks, psum, psq, pmax, d_rowsum, bpart);
  k_scalars_final<<<1, 64, 0, s>>>(nb, bpart, d_out3);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

namespace {
template <typename TX, typename TB, int NT>
void launch_mfma_nt(const TX* X, int64_t ldx, const TB* B, int64_t ldb, int n, int c, int kchunk, int splits, TX* P,
                    int cp, const DevState* st, hipStream_t s) {
  constexpr int RT = 2;
  dim3 g(ceil_div(n, 64 * RT), splits);
  k_gemm_mfma<TX, TB, NT, RT><<<g, 256, 0, s>>>(X, ldx, B, ldb, n, c, kchunk, P, cp, st);
}
template <typename TB, int NT>
void launch_bf16_nt(const __bf16* X, int64_t ldx, const TB* B, int64_t ldb, int n, int c, int kchunk, int splits,
                    float* P, int cp, const DevState* st, hipStream_t s) {
  constexpr int RT = 2;
  dim3 g(ceil_div(n, 64 * RT), splits);
  k_gemm_bf16<TB, NT, RT><<<g, 256, 0, s>>>(X, ldx, B, ldb, n, c, kchunk, P, cp, st);
}

template <typename TX, typename TB>
void dispatch_mfma(int nt, const TX* X, int64_t ldx, const TB* B, int64_t ldb, int n, int c, int kchunk, int splits,
                   TX* P, int cp, const DevState* st, hipStream_t s) {
  switch (nt) {
    case 1: launch_mfma_nt<TX, TB, 1>(X, ldx, B, ldb, n, c, kchunk, splits, P, cp, st, s); break;
    case 2: launch_mfma_nt<TX, TB, 2>(X, ldx, B, ldb, n, c, kchunk, splits, P, cp, st, s); break;
    case 3: launch_mfma_nt<TX, TB, 3>(X, ldx, B, ldb, n, c, kchunk, splits, P, cp, st, s); break;
    case 4: launch_mfma_nt<TX, TB, 4>(X, ldx, B, ldb, n, c, kchunk, splits, P, cp, st, s); break;
    case 5: launch_mfma_nt<TX, TB, 5>(X, ldx, B, ldb, n, c, kchunk, splits, P, cp, st, s); break;
    default: launch_mfma_nt<TX, TB, 6>(X, ldx, B, ldb, n, c, kchunk, splits, P, cp, st, s); break;
  }
}
template <typename TB>
void dispatch_bf16(int nt, const __bf16* X, int64_t ldx, const TB* B, int64_t ldb, int n, int c, int kchunk,
                   int splits, float* P, int cp, const DevState* st, hipStream_t s) {
  switch (nt) {
    case 1: launch_bf16_nt<TB, 1>(X, ldx, B, ldb, n, c, kchunk, splits, P, cp, st, s); break;
    case 2: launch_bf16_nt<TB, 2>(X, ldx, B, ldb, n, c, kchunk, splits, P, cp, st, s); break;
    case 3: launch_bf16_nt<TB, 3>(X, ldx, B, ldb, n, c, kchunk, splits, P, cp, st, s); break;
    case 4: launch_bf16_nt<TB, 4>(X, ldx, B, ldb, n, c, kchunk, splits, P, cp, st, s); break;
    case 5: launch_bf16_nt<TB, 5>(X, ldx, B, ldb, n, c, kchunk, splits, P, cp, st, s); break;
    default: launch_bf16_nt<TB, 6>(X, ldx, B, ldb, n, c, kchunk, splits, P, cp, st, s); break;
  }
}
}  // namespace

GemmPlan gemm_plan(int n, int c, int compute_dtype) {
  GemmPlan p;
  p.cp = 16 * ceil_div(c, 16);
  const int kt = compute_dtype == SYMNMF_BF16 ? BF_KT : GEMM_KT;
  const int row_blocks = ceil_div(n, 128);
  int splits = std::max(1, ceil_div(1024, row_blocks));
  const int max_splits = std::max(1, ceil_div(n, kt));
  splits = std::min(splits, max_splits);
  p.kchunk = kt * ceil_div(ceil_div(n, splits), kt);
  p.splits = ceil_div(n, p.kchunk);
  return p;
}

int dense_gemm(const void* X, int xdtype, int64_t ldx, const void* B, int bdtype, int64_t ldb, int n, int c,
               const GemmPlan& p, void* P, void* Y, int ydtype, int64_t ldy, const DevState* st, hipStream_t s) {
  const int nt = p.cp / 16;
  if (nt < 1 || nt > 6) return -1;
  if (xdtype == SYMNMF_F64) {
    if (bdtype != SYMNMF_F64) return -1;
    dispatch_mfma<double, double>(nt, (const double*)X, ldx, (const double*)B, ldb, n, c, p.kchunk, p.splits,
                                  (double*)P, p.cp, st, s);
    const int64_t tot = (int64_t)n * c;
    if (ydtype == SYMNMF_F64)
      k_splitk_reduce<double, double><<<ceil_div(tot, 256), 256, 0, s>>>((const double*)P, p.splits, n, c, p.cp,
                                                                          (double*)Y, ldy, st);
    else
      return -1;
  } else {
    if (xdtype == SYMNMF_F32) {
      if (bdtype == SYMNMF_F32)
        dispatch_mfma<float, float>(nt, (const float*)X, ldx, (const float*)B, ldb, n, c, p.kchunk, p.splits,
                                    (float*)P, p.cp, st, s);
      else
        dispatch_mfma<float, double>(nt, (const float*)X, ldx, (const double*)B, ldb, n, c, p.kchunk, p.splits,
                                     (float*)P, p.cp, st, s);
    } else {
      if (bdtype == SYMNMF_F32)
        dispatch_bf16<float>(nt, (const __bf16*)X, ldx, (const float*)B, ldb, n, c, p.kchunk, p.splits, (float*)P,
                             p.cp, st, s);
      else
        dispatch_bf16<double>(nt, (const __bf16*)X, ldx, (const double*)B, ldb, n, c, p.kchunk, p.splits,
                              (float*)P, p.cp, st, s);
    }
    const int64_t tot = (int64_t)n * c;
    if (ydtype == SYMNMF_F32)
      k_splitk_reduce<float, float><<<ceil_div(tot, 256), 256, 0, s>>>((const float*)P, p.splits, n, c, p.cp,
                                                                        (float*)Y, ldy, st);
    else
      k_splitk_reduce<float, double><<<ceil_div(tot, 256), 256, 0, s>>>((const float*)P, p.splits, n, c, p.cp,
                                                                         (double*)Y, ldy, st);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int convert_f32_bf16(const float* src, int64_t lds, void* dst, int64_t ldd, int n, hipStream_t s) {
  const int64_t tot = (int64_t)n * n;
  k_f32_to_bf16<<<(unsigned)ceil_div(tot, 256), 256, 0, s>>>(src, lds, (__bf16*)dst, ldd, n);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int dense_resid_exact(const void* X, int xdtype, int64_t ldx, int n, int k, const void* W, const void* H, int fdtype,
                      Workspace& ws, double* d_sum, hipStream_t s) {
  dim3 g(ceil_div(n, 64), ceil_div(n, 64));
  const int nb = g.x * g.y;
  double* part = ws.dbl(nb);
  if (!part) return -1;
#define RX(TX, TF) \
  k_resid_exact_dense<TX, TF><<<g, 256, 0, s>>>((const TX*)X, ldx, n, k, (const TF*)W, (const TF*)H, part)
  if (fdtype == SYMNMF_F64) {
    if (xdtype == SYMNMF_F64) RX(double, double);
    else if (xdtype == SYMNMF_F32) RX(float, double);
    else RX(__bf16, double);
  } else {
    if (xdtype == SYMNMF_F64) RX(double, float);
    else if (xdtype == SYMNMF_F32) RX(float, float);
    else RX(__bf16, float);
  }
#undef RX
  sum_partials(part, nb, d_sum, s);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
