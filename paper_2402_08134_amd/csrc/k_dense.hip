// Dense-X kernels: one-time scalars pass, the product Y = X B on MFMA
// (FP64, FP32 and BF16 inputs), split-K reduction, FP32 -> BF16 conversion
// and the exact residual pass.
//
// The product X B (B = H, W, the sketch Omega or the basis Q) is the main
// cost of every iteration (Section 2.1.2: X H is reused by a whole HALS
// sweep; Section 3.1 complexity).  X is streamed exactly once per product,
// LDS-free, from HBM into registers.  FP32 and BF16 read X along its rows
// (k_gemm_cols*: Y^T = B^T X, X symmetric); FP64 keeps the row-owner layout
// (k_gemm_mfma).  The B operand is a transposed, zero-padded panel Bt.
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
  int r = r0;
  for (; r + 8 <= r1; r += 8) {  // 8 loads in flight, summed in row order
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = to_f64(X[(int64_t)(r + u) * ld + j]);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      s += v[u];
      q += v[u] * v[u];
      m = fmax(m, v[u]);
    }
  }
  for (; r < r1; ++r) {
    const double v = to_f64(X[(int64_t)r * ld + j]);
    s += v;
    q += v * v;
    m = fmax(m, v);
  }
  psum[(int64_t)c * n + j] = s;
  psq[(int64_t)c * n + j] = q;
  pmax[(int64_t)c * n + j] = m;
}

// The same for FP32 X with 16-byte loads: thread owns columns 4 t .. 4 t + 3
// (same per-column order of the sums as above).
__global__ __launch_bounds__(256) void k_dense_colstats_f4(const float* __restrict__ X, int64_t ld, int n,
                                                           int rows_per_chunk, double* __restrict__ psum,
                                                           double* __restrict__ psq, double* __restrict__ pmax) {
  const int j = 4 * (blockIdx.x * 256 + threadIdx.x);
  const int c = blockIdx.y;
  if (j >= n) return;
  const int r0 = c * rows_per_chunk;
  const int r1 = min(n, r0 + rows_per_chunk);
  double s[4] = {0, 0, 0, 0}, q[4] = {0, 0, 0, 0}, m[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
  auto add = [&](const floatx4& v) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const double d = (double)v[t];
      s[t] += d;
      q[t] += d * d;
      m[t] = fmax(m[t], d);
    }
  };
  int r = r0;
  for (; r + 8 <= r1; r += 8) {
    floatx4 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = __builtin_nontemporal_load((const floatx4*)(X + (int64_t)(r + u) * ld + j));
#pragma unroll
    for (int u = 0; u < 8; ++u) add(v[u]);
  }
  for (; r < r1; ++r) add(*(const floatx4*)(X + (int64_t)r * ld + j));
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    psum[(int64_t)c * n + j + t] = s[t];
    psq[(int64_t)c * n + j + t] = q[t];
    pmax[(int64_t)c * n + j + t] = m[t];
  }
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
// Row-owner MFMA product P[split] = X[:, krange] B[krange, :] (FP64).
//
// The B operand is first written transposed and zero padded, Bt[q][j] =
// B[j][q] (q < cp, j < npad), so a lane fetches its B values for four
// consecutive K with one 16-byte load, exactly like its X values.  No LDS and
// no barrier: each wave owns 16*RT rows of X, streams its K range tile by
// tile and prefetches the next X tile into registers while the MFMAs of the
// current one run (B tiles are small and come from L1/L2, issued before the
// X prefetch so waiting on them does not wait on the prefetch).
//
// v_mfma_{f32,f64}_16x16x4: lane l supplies A[l%16][l/16] and B[l/16][l%16];
// the accumulator layout is given by Mfma<T>::out_row.  A lane holds four
// consecutive K values (4g..4g+3 of a 16-wide sub-step, g = l/16) and issues
// one MFMA per value.
// ---------------------------------------------------------------------------
// Accumulator rows differ between the two instructions (measured on gfx950):
// f32: element v of lane l is row 4*(l/16) + v; f64: row (l/16) + 4*v.  The
// column is l%16 for both.
template <typename T> struct Mfma;
template <> struct Mfma<float> {
  using acc_t = floatx4;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int lg, int v) { return 4 * lg + v; }
};
template <> struct Mfma<double> {
  using acc_t = doublex4;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int lg, int v) { return lg + 4 * v; }
};

template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = floatx4; };
template <> struct Vec4<double> { using type = doublex4; };

constexpr int GEMM_KT = 64;   // K per tile, FP32 / FP64 (4 sub-steps of 16)
constexpr int BT_PAD = 128;   // Bt row length is n rounded up to this

template <typename TB, typename TO>
__global__ __launch_bounds__(256) void k_transpose_pad(const TB* __restrict__ B, int64_t ldb, int n, int c,
                                                       TO* __restrict__ Bt, int64_t ldt, int cp,
                                                       const DevState* __restrict__ st) {
  if (stopped(st)) return;
  __shared__ double tile[32][33];
  const int j0 = blockIdx.x * 32, q0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int j = j0 + r, q = q0 + tx;
    tile[r][tx] = (j < n && q < c) ? (double)B[(int64_t)j * ldb + q] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int q = q0 + r, j = j0 + tx;
    if (q < cp && j < ldt) Bt[(int64_t)q * ldt + j] = (TO)tile[tx][r];
  }
}

template <typename TX, int NT, int RT, bool VEC>
__global__ __launch_bounds__(256) void k_gemm_mfma(const TX* __restrict__ X, int64_t ldx, const TX* __restrict__ Bt,
                                                   int64_t ldt, int n, int kchunk, TX* __restrict__ P, int cp,
                                                   const DevState* __restrict__ st) {
  if (stopped(st)) return;
  using M = Mfma<TX>;
  using acc_t = typename M::acc_t;
  using V4 = typename Vec4<TX>::type;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int row_base = (blockIdx.x * 4 + wave) * (16 * RT);
  if (row_base >= n) return;
  const int kb = blockIdx.y * kchunk;
  const int ke = min(n, kb + kchunk);

  acc_t acc[RT][NT];
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[r][t] = acc_t{0, 0, 0, 0};

  const TX* xrow[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) xrow[r] = X + (int64_t)min(row_base + 16 * r + li, n - 1) * ldx + 4 * lg;
  const TX* brow[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) brow[t] = Bt + (int64_t)(16 * t + li) * ldt + 4 * lg;

  const int nfull = VEC ? (ke - kb) / GEMM_KT : 0;
  // Software pipeline with two register buffers used in turn (no copies, so
  // the compiler cannot merge them): the X and B operands of the next tile
  // are loaded while the MFMAs of the current one run.  Everything consumed
  // by a compute step was issued before the loads it overlaps, so the
  // in-order load counter never makes it wait for the prefetch.
  V4 x0[RT][4], b0[NT][4], x1[RT][4], b1[NT][4];
  auto load = [&](V4 (&xv)[RT][4], V4 (&bv)[NT][4], int k0) {
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int ss = 0; ss < 4; ++ss) xv[r][ss] = __builtin_nontemporal_load((const V4*)(xrow[r] + k0 + 16 * ss));
#pragma unroll
    for (int ct = 0; ct < NT; ++ct)
#pragma unroll
      for (int ss = 0; ss < 4; ++ss) bv[ct][ss] = *(const V4*)(brow[ct] + k0 + 16 * ss);
  };
  auto compute = [&](const V4 (&xv)[RT][4], const V4 (&bv)[NT][4]) {
#pragma unroll
    for (int ss = 0; ss < 4; ++ss)
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int ct = 0; ct < NT; ++ct)
#pragma unroll
          for (int r = 0; r < RT; ++r) acc[r][ct] = M::mma(xv[r][ss][u], bv[ct][ss][u], acc[r][ct]);
  };
  int t = 0;
  if (nfull > 0) load(x0, b0, kb);
  for (; t + 2 < nfull; t += 2) {
    load(x1, b1, kb + (t + 1) * GEMM_KT);
    compute(x0, b0);
    load(x0, b0, kb + (t + 2) * GEMM_KT);
    compute(x1, b1);
  }
  if (t + 1 < nfull) {
    load(x1, b1, kb + (t + 1) * GEMM_KT);
    compute(x0, b0);
    compute(x1, b1);
  } else if (t < nfull) {
    compute(x0, b0);
  }
  // Remaining K (partial last tile, or every tile when X is not aligned for
  // vector loads): guarded scalar loads of X; Bt is zero padded.
  for (int k0 = kb + nfull * GEMM_KT; k0 < ke; k0 += GEMM_KT) {
#pragma unroll
    for (int ss = 0; ss < 4; ++ss) {
      TX xs[RT][4];
      TX bs[NT][4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int col = k0 + 16 * ss + 4 * lg + u;
#pragma unroll
        for (int r = 0; r < RT; ++r) xs[r][u] = (col < ke) ? xrow[r][col - 4 * lg] : (TX)0;
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) bs[ct][u] = brow[ct][k0 + 16 * ss + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int ct = 0; ct < NT; ++ct)
#pragma unroll
          for (int r = 0; r < RT; ++r) acc[r][ct] = M::mma(xs[r][u], bs[ct][u], acc[r][ct]);
    }
  }
  TX* out = P + (int64_t)blockIdx.y * n * cp;
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = row_base + 16 * r + M::out_row(lg, v);
      if (row < n) {
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) out[(int64_t)row * cp + 16 * ct + li] = acc[r][ct][v];
      }
    }
}

// ---------------------------------------------------------------------------
// FP32 product read along rows of X: Y^T = B^T X, which is (X B)^T because X
// is symmetric.  Each wave owns 64 * CT output rows j (a strip of X's
// columns) and a range of X's rows i (split-K).  One K step takes 4 rows;
// lane (ln, lq) = (lane % 16, lane / 16) holds X[i0 + 4 lq + s][j0 + 4 ln ..
// + 3] for the steps s = 0..3 of a 16-row tile, so a wave's load instruction
// covers 4 rows x 256 contiguous bytes (measured on MI355X: a pure read in
// this pattern streams at about 6.7 TB/s, against 6.0 TB/s for 16 rows x 64
// bytes).  v_mfma_f32_16x16x4f32 with A = the B panel (Bt[c][i], lane ->
// (c = 16 t + ln, K = lq), one float4 of Bt per lane holds the tile's 4
// steps) and B = X (lane -> (K = lq, column ln)); element u of the X float4
// feeds the MFMA of the columns j0 + 4 ln + u.  Output lane (ln, lq), v ->
// c = 16 t + 4 lq + v: one float4 store of 4 consecutive c per (t, u).
// DS tiles are in flight (register ring, no LDS).  The partials land in
// P[split][j][c] like those of k_gemm_mfma.
template <int NT, int CT, bool VEC>
__global__ __launch_bounds__(256) void k_gemm_cols(const float* __restrict__ X, int64_t ldx,
                                                   const float* __restrict__ Bt, int64_t ldt, int n, int rchunk,
                                                   float* __restrict__ P, int cp, const DevState* __restrict__ st) {
  if (stopped(st)) return;
  constexpr int DS = 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ln = lane & 15, lq = lane >> 4;
  const int j0 = (blockIdx.x * 4 + wave) * (64 * CT);
  if (j0 >= n) return;
  const int ib = blockIdx.y * rchunk;
  const int ie = min(n, ib + rchunk);
  const int ntile = (ie - ib + 15) / 16;
  const bool full = VEC && (j0 + 64 * CT <= n);

  floatx4 acc[NT][CT][4];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[t][ct][u] = floatx4{0, 0, 0, 0};
  const float* bp[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) bp[t] = Bt + (int64_t)(16 * t + ln) * ldt + 4 * lq;

  floatx4 xv[DS][CT][4], bv[DS][NT];
  // Tile rows beyond n (last split only) read row n - 1 of X; the padded Bt
  // is zero there, so they add nothing.
  auto load = [&](floatx4 (&xd)[CT][4], floatx4 (&bd)[NT], int tile) {
    const int i0 = ib + 16 * tile;
#pragma unroll
    for (int t = 0; t < NT; ++t) bd[t] = *(const floatx4*)(bp[t] + i0);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const float* xr = X + (int64_t)min(i0 + 4 * lq + s, n - 1) * ldx + j0 + 4 * ln;
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        if (full) {
          xd[ct][s] = __builtin_nontemporal_load((const floatx4*)(xr + 64 * ct));
        } else {
#pragma unroll
          for (int u = 0; u < 4; ++u) xd[ct][s][u] = (j0 + 64 * ct + 4 * ln + u < n) ? xr[64 * ct + u] : 0.0f;
        }
      }
    }
  };
  auto compute = [&](const floatx4 (&xd)[CT][4], const floatx4 (&bd)[NT]) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int u = 0; u < 4; ++u)
            acc[t][ct][u] = __builtin_amdgcn_mfma_f32_16x16x4f32(bd[t][s], xd[ct][s][u], acc[t][ct][u], 0, 0, 0);
  };
#pragma unroll
  for (int d = 0; d < DS - 1; ++d)
    if (d < ntile) load(xv[d], bv[d], d);
  for (int tile = 0; tile < ntile; tile += DS) {
#pragma unroll
    for (int d = 0; d < DS; ++d) {
      const int pre = tile + d + DS - 1;  // tile prefetched into slot (d + DS - 1) % DS
      if (pre < ntile) load(xv[(d + DS - 1) % DS], bv[(d + DS - 1) % DS], pre);
      if (tile + d < ntile) compute(xv[d], bv[d]);
    }
  }
  float* out = P + (int64_t)blockIdx.y * n * cp;
#pragma unroll
  for (int ct = 0; ct < CT; ++ct)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = j0 + 64 * ct + 4 * ln + u;
      if (j < n) {
#pragma unroll
        for (int t = 0; t < NT; ++t) *(floatx4*)(out + (int64_t)j * cp + 16 * t + 4 * lq) = acc[t][ct][u];
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

// One block per row (grid-stride over rows: a launch covers at most 65535
// rows, since a dispatch counts its work-items in 32 bits per dimension).
__global__ __launch_bounds__(256) void k_f32_to_bf16(const float* __restrict__ src, int64_t lds, __bf16* __restrict__ dst,
                                                     int64_t ldd, int n) {
  for (int64_t r = blockIdx.x; r < n; r += gridDim.x) {
    const float* sr = src + r * lds;
    __bf16* dr = dst + r * ldd;
    for (int c = threadIdx.x; c < n; c += 256) dr[c] = (__bf16)sr[c];
  }
}

// BF16 product read along rows of X, the same scheme as k_gemm_cols with
// v_mfma_f32_16x16x32_bf16 (B operand lane (ln, lq) -> K 8 lq .. 8 lq + 7 of
// column ln).  One K step takes 32 rows: lane (ln, lq) loads 8 BF16 of each
// of the rows i0 + 8 lq + e (e = 0..7) at columns j0 + 8 ln .. + 7 (a wave's
// load instruction covers 4 rows x 256 contiguous bytes), transposes that
// 8 x 8 block in registers (v_perm_b32, 4 per 16 loaded bytes), and feeds
// column u of it to the MFMA of the columns j0 + 8 ln + u.  A = the BF16
// B panel: one 16-byte load of Bt[16 t + ln][i0 + 8 lq ..] per K step.  A
// wave owns 128 output rows j; output lane (ln, lq), v -> c = 16 t + 4 lq + v.
__device__ __forceinline__ void transpose8_bf16(const uint32_t (&in)[8][4], uint32_t (&out)[8][4]) {
  // out[u] dword d = {in[2d] element u, in[2d + 1] element u} (low, high half)
#pragma unroll
  for (int u = 0; u < 8; ++u)
#pragma unroll
    for (int d = 0; d < 4; ++d)
      out[u][d] = __builtin_amdgcn_perm(in[2 * d + 1][u >> 1], in[2 * d][u >> 1], (u & 1) ? 0x07060302u : 0x05040100u);
}

template <int NT, bool VEC>
__global__ __launch_bounds__(256) void k_gemm_cols_bf16(const __bf16* __restrict__ X, int64_t ldx,
                                                        const __bf16* __restrict__ Bt, int64_t ldt, int n, int rchunk,
                                                        float* __restrict__ P, int cp,
                                                        const DevState* __restrict__ st) {
  if (stopped(st)) return;
  constexpr int DS = 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ln = lane & 15, lq = lane >> 4;
  const int j0 = (blockIdx.x * 4 + wave) * 128;
  if (j0 >= n) return;
  const int ib = blockIdx.y * rchunk;
  const int ie = min(n, ib + rchunk);
  const int nstep = (ie - ib + 31) / 32;
  const bool full = VEC && (j0 + 128 <= n);
  const unsigned short* Xs = reinterpret_cast<const unsigned short*>(X);

  floatx4 acc[NT][8];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[t][u] = floatx4{0, 0, 0, 0};
  const __bf16* bp[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) bp[t] = Bt + (int64_t)(16 * t + ln) * ldt + 8 * lq;

  uint32_t xv[DS][8][4];
  bf16x8 bv[DS][NT];
  // Rows beyond n (last split only) read row n - 1; the padded Bt is zero there.
  auto load = [&](uint32_t (&xd)[8][4], bf16x8 (&bd)[NT], int step) {
    const int i0 = ib + 32 * step;
#pragma unroll
    for (int t = 0; t < NT; ++t) bd[t] = *(const bf16x8*)(bp[t] + i0);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t ro = (int64_t)min(i0 + 8 * lq + e, n - 1) * ldx + j0 + 8 * ln;
      if (full) {
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
        const u32x4 v = __builtin_nontemporal_load((const u32x4*)(X + ro));
        xd[e][0] = v[0];
        xd[e][1] = v[1];
        xd[e][2] = v[2];
        xd[e][3] = v[3];
      } else {
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          const int c0 = j0 + 8 * ln + 2 * d;
          const uint32_t lo = (c0 < n) ? (uint32_t)Xs[ro + 2 * d] : 0u;
          const uint32_t hi = (c0 + 1 < n) ? (uint32_t)Xs[ro + 2 * d + 1] : 0u;
          xd[e][d] = lo | (hi << 16);
        }
      }
    }
  };
  auto compute = [&](const uint32_t (&xd)[8][4], const bf16x8 (&bd)[NT]) {
    uint32_t tr[8][4];
    transpose8_bf16(xd, tr);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      bf16x8 xb;
      __builtin_memcpy(&xb, tr[u], 16);
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bd[t], xb, acc[t][u], 0, 0, 0);
    }
  };
#pragma unroll
  for (int d = 0; d < DS - 1; ++d)
    if (d < nstep) load(xv[d], bv[d], d);
  for (int step = 0; step < nstep; step += DS) {
#pragma unroll
    for (int d = 0; d < DS; ++d) {
      const int pre = step + d + DS - 1;
      if (pre < nstep) load(xv[(d + DS - 1) % DS], bv[(d + DS - 1) % DS], pre);
      if (step + d < nstep) compute(xv[d], bv[d]);
    }
  }
  float* out = P + (int64_t)blockIdx.y * n * cp;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int j = j0 + 8 * ln + u;
    if (j < n) {
#pragma unroll
      for (int t = 0; t < NT; ++t) *(floatx4*)(out + (int64_t)j * cp + 16 * t + 4 * lq) = acc[t][u];
    }
  }
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
  else if (dtype == SYMNMF_F32 && n % 4 == 0 && ld % 4 == 0 && (uintptr_t)X % 16 == 0)
    k_dense_colstats_f4<<<dim3(ceil_div(n, 1024), chunks), 256, 0, s>>>((const float*)X, ld, n, rpc, psum, psq, pmax);
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
template <typename TX, int NT, int RT>
void launch_mfma(const TX* X, int64_t ldx, bool vec, const TX* Bt, int64_t ldt, int n, const GemmPlan& p, TX* P,
                 const DevState* st, hipStream_t s) {
  dim3 g(ceil_div(ceil_div(n, 16 * RT), 4), p.splits);
  if (vec)
    k_gemm_mfma<TX, NT, RT, true><<<g, 256, 0, s>>>(X, ldx, Bt, ldt, n, p.kchunk, P, p.cp, st);
  else
    k_gemm_mfma<TX, NT, RT, false><<<g, 256, 0, s>>>(X, ldx, Bt, ldt, n, p.kchunk, P, p.cp, st);
}
// FP64 rows per wave (16 * RT) by operand width: more rows amortise the B
// loads, fewer keep the registers of wide B panels in budget.
int pick_rt_f64(int nt) { return nt <= 2 ? 2 : 1; }

template <typename TX>
int dispatch_mfma(int nt, int rt, const TX* X, int64_t ldx, bool vec, const TX* Bt, int64_t ldt, int n,
                  const GemmPlan& p, TX* P, const DevState* st, hipStream_t s) {
#define CASE(NT_, RT_) \
  if (nt == NT_ && rt == RT_) { launch_mfma<TX, NT_, RT_>(X, ldx, vec, Bt, ldt, n, p, P, st, s); return 0; }
  CASE(1, 2) CASE(2, 2) CASE(3, 1) CASE(4, 1) CASE(5, 1) CASE(6, 1)
#undef CASE
  return -1;
}
template <int NT, int CT>
void launch_cols(const float* X, int64_t ldx, bool vec, const float* Bt, int64_t ldt, int n, const GemmPlan& p, float* P,
                 const DevState* st, hipStream_t s) {
  dim3 g(ceil_div(n, 4 * 64 * CT), p.splits);
  if (vec)
    k_gemm_cols<NT, CT, true><<<g, 256, 0, s>>>(X, ldx, Bt, ldt, n, p.kchunk, P, p.cp, st);
  else
    k_gemm_cols<NT, CT, false><<<g, 256, 0, s>>>(X, ldx, Bt, ldt, n, p.kchunk, P, p.cp, st);
}

int dispatch_cols(int nt, int ct, const float* X, int64_t ldx, bool vec, const float* Bt, int64_t ldt, int n,
                  const GemmPlan& p, float* P, const DevState* st, hipStream_t s) {
#define CASE(NT_, CT_) \
  if (nt == NT_ && ct == CT_) { launch_cols<NT_, CT_>(X, ldx, vec, Bt, ldt, n, p, P, st, s); return 0; }
  CASE(1, 2) CASE(2, 2) CASE(3, 2) CASE(4, 2) CASE(5, 1) CASE(6, 1)
#undef CASE
  return -1;
}

template <int NT>
void launch_cols_bf16(const __bf16* X, int64_t ldx, bool vec, const __bf16* Bt, int64_t ldt, int n,
                      const GemmPlan& p, float* P, const DevState* st, hipStream_t s) {
  dim3 g(ceil_div(n, 4 * 128), p.splits);
  if (vec)
    k_gemm_cols_bf16<NT, true><<<g, 256, 0, s>>>(X, ldx, Bt, ldt, n, p.kchunk, P, p.cp, st);
  else
    k_gemm_cols_bf16<NT, false><<<g, 256, 0, s>>>(X, ldx, Bt, ldt, n, p.kchunk, P, p.cp, st);
}

int dispatch_cols_bf16(int nt, const __bf16* X, int64_t ldx, bool vec, const __bf16* Bt, int64_t ldt, int n,
                       const GemmPlan& p, float* P, const DevState* st, hipStream_t s) {
  switch (nt) {
    case 1: launch_cols_bf16<1>(X, ldx, vec, Bt, ldt, n, p, P, st, s); return 0;
    case 2: launch_cols_bf16<2>(X, ldx, vec, Bt, ldt, n, p, P, st, s); return 0;
    case 3: launch_cols_bf16<3>(X, ldx, vec, Bt, ldt, n, p, P, st, s); return 0;
    case 4: launch_cols_bf16<4>(X, ldx, vec, Bt, ldt, n, p, P, st, s); return 0;
    case 5: launch_cols_bf16<5>(X, ldx, vec, Bt, ldt, n, p, P, st, s); return 0;
    case 6: launch_cols_bf16<6>(X, ldx, vec, Bt, ldt, n, p, P, st, s); return 0;
    default: return -1;
  }
}

}  // namespace

GemmPlan gemm_plan(int n, int c, int compute_dtype) {
  GemmPlan p;
  p.cp = 16 * ceil_div(c, 16);
  p.ldt = (int64_t)BT_PAD * ceil_div(n, BT_PAD);
  if (compute_dtype == SYMNMF_F32) {
    // row-contiguous product: strips of 64 * ct columns, about one wave per
    // SIMD in total, splits of at least 256 rows (multiples of the 16-row K
    // step)
    p.cols = true;
    // two 64-column blocks per wave up to 64 output columns for FP32 MFMA
    // (measured at n = 16384: X Q at l = 48 317 -> 290 us, k = 64 361 ->
    // 338 us; at n = 65536, k = 64 5.14 -> 4.48 ms)
    p.ct = p.cp <= 64 ? 2 : 1;
    const int step = 16;
    const int strips = ceil_div(n, 64 * p.ct);
    // about 1024 waves (2048 or 512 measured slower at n = 16384)
    int splits = std::max(1, ceil_div(1024, strips));
    splits = std::min(splits, std::max(1, n / 256));
    p.kchunk = step * ceil_div(ceil_div(n, splits), step);
    p.splits = ceil_div(n, p.kchunk);
    return p;
  }
  if (compute_dtype == SYMNMF_BF16) {
    // the same for BF16: strips of 128 columns, splits in multiples of 32 rows
    p.cols = true;
    const int strips = ceil_div(n, 128);
    int splits = std::max(1, ceil_div(1024, strips));
    splits = std::min(splits, std::max(1, n / 256));
    p.kchunk = 32 * ceil_div(ceil_div(n, splits), 32);
    p.splits = ceil_div(n, p.kchunk);
    return p;
  }
  // FP64: the row-owner kernel, about two waves per SIMD (256 CUs x 4 SIMDs)
  p.rt = pick_rt_f64(p.cp / 16);
  const int kt = GEMM_KT;
  const int waves = ceil_div(n, 16 * p.rt);
  int splits = std::max(1, ceil_div(2048, waves));
  splits = std::min(splits, std::max(1, ceil_div(n, 4 * kt)));
  p.kchunk = kt * ceil_div(ceil_div(n, splits), kt);
  p.splits = ceil_div(n, p.kchunk);
  return p;
}

size_t gemm_bt_bytes(int n, int cmax) { return (size_t)16 * ceil_div(cmax, 16) * BT_PAD * ceil_div(n, BT_PAD) * 8; }

int dense_gemm_bt(const void* X, int xdtype, int64_t ldx, const void* Bt, int n, int c, const GemmPlan& p, void* P,
                  const DevState* st, hipStream_t s) {
  const int nt = p.cp / 16;
  if (nt < 1 || nt > 6 || p.cp < c) return -1;
  int rc;
  if (xdtype == SYMNMF_F64) {
    const bool vec = (ldx % 4 == 0) && ((uintptr_t)X % 32 == 0);
    rc = dispatch_mfma<double>(nt, p.rt, (const double*)X, ldx, vec, (const double*)Bt, p.ldt, n, p, (double*)P, st, s);
  } else if (xdtype == SYMNMF_F32) {
    const bool vec = (ldx % 4 == 0) && ((uintptr_t)X % 16 == 0);
    rc = dispatch_cols(nt, p.ct, (const float*)X, ldx, vec, (const float*)Bt, p.ldt, n, p, (float*)P, st, s);
  } else {
    const bool vec = (ldx % 8 == 0) && ((uintptr_t)X % 16 == 0);
    rc = dispatch_cols_bf16(nt, (const __bf16*)X, ldx, vec, (const __bf16*)Bt, p.ldt, n, p, (float*)P, st, s);
  }
  if (rc) return rc;
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int factor_transpose(const void* F, int fdtype, int n, int k, void* Bt, int cdtype, const GemmPlan& p,
                     const DevState* st, hipStream_t s) {
  dim3 tg(ceil_div(p.ldt, 32), ceil_div(p.cp, 32));
  if (fdtype == SYMNMF_F64 && cdtype == SYMNMF_F64)
    k_transpose_pad<double, double><<<tg, 256, 0, s>>>((const double*)F, k, n, k, (double*)Bt, p.ldt, p.cp, st);
  else if (fdtype == SYMNMF_F32 && cdtype == SYMNMF_F32)
    k_transpose_pad<float, float><<<tg, 256, 0, s>>>((const float*)F, k, n, k, (float*)Bt, p.ldt, p.cp, st);
  else if (fdtype == SYMNMF_F32 && cdtype == SYMNMF_BF16)
    k_transpose_pad<float, __bf16><<<tg, 256, 0, s>>>((const float*)F, k, n, k, (__bf16*)Bt, p.ldt, p.cp, st);
  else
    return -1;
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int dense_gemm(const void* X, int xdtype, int64_t ldx, const void* B, int bdtype, int64_t ldb, int n, int c,
               const GemmPlan& p, void* Bt, void* P, void* Y, int ydtype, int64_t ldy, const DevState* st,
               hipStream_t s) {
  const int nt = p.cp / 16;
  if (nt < 1 || nt > 6) return -1;
  dim3 tg(ceil_div(p.ldt, 32), ceil_div(p.cp, 32));
  const int64_t tot = (int64_t)n * c;
  if (xdtype == SYMNMF_F64) {
    if (bdtype != SYMNMF_F64 || ydtype != SYMNMF_F64) return -1;
    k_transpose_pad<double, double><<<tg, 256, 0, s>>>((const double*)B, ldb, n, c, (double*)Bt, p.ldt, p.cp, st);
    const bool vec = (ldx % 4 == 0) && ((uintptr_t)X % 32 == 0);
    if (dispatch_mfma<double>(nt, p.rt, (const double*)X, ldx, vec, (const double*)Bt, p.ldt, n, p, (double*)P, st, s))
      return -1;
    k_splitk_reduce<double, double><<<ceil_div(tot, 256), 256, 0, s>>>((const double*)P, p.splits, n, c, p.cp,
                                                                        (double*)Y, ldy, st);
  } else if (xdtype == SYMNMF_F32) {
    if (bdtype == SYMNMF_F32)
      k_transpose_pad<float, float><<<tg, 256, 0, s>>>((const float*)B, ldb, n, c, (float*)Bt, p.ldt, p.cp, st);
    else
      k_transpose_pad<double, float><<<tg, 256, 0, s>>>((const double*)B, ldb, n, c, (float*)Bt, p.ldt, p.cp, st);
    const bool vec = (ldx % 4 == 0) && ((uintptr_t)X % 16 == 0);
    if (dispatch_cols(nt, p.ct, (const float*)X, ldx, vec, (const float*)Bt, p.ldt, n, p, (float*)P, st, s))
      return -1;
  } else {
    if (bdtype == SYMNMF_F32)
      k_transpose_pad<float, __bf16><<<tg, 256, 0, s>>>((const float*)B, ldb, n, c, (__bf16*)Bt, p.ldt, p.cp, st);
    else
      k_transpose_pad<double, __bf16><<<tg, 256, 0, s>>>((const double*)B, ldb, n, c, (__bf16*)Bt, p.ldt, p.cp, st);
    const bool vec = (ldx % 8 == 0) && ((uintptr_t)X % 16 == 0);
    if (dispatch_cols_bf16(nt, (const __bf16*)X, ldx, vec, (const __bf16*)Bt, p.ldt, n, p, (float*)P, st, s))
      return -1;
  }
  if (xdtype != SYMNMF_F64) {
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
  k_f32_to_bf16<<<std::max(1, std::min(n, 65535)), 256, 0, s>>>(src, lds, (__bf16*)dst, ldd, n);
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
