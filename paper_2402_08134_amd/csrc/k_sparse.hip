// CSR-X kernels: scalars pass, SpMM Y = X B and the cross term of the exact
// residual.  The sparse product is the "MM" cost of the sparse experiments
// (Section 5.2); a wavefront owns one row, its lanes own the output columns
// (so every B-row gather is one contiguous 64..512-byte read) and, for narrow
// B, several lane groups walk different nonzeros of the row and are combined
// by a fixed shuffle tree.
#include "kernels.hpp"

namespace {

// Scalars pass over CSR values: 16 lanes per row (each group reads its row's
// values in coalesced 16-element runs and sums them with shuffles inside the
// group), the 16 groups of a block walk a contiguous range of rows; per block
// one partial (sum, sum of squares, max) in a fixed order.
template <typename TV>
__global__ __launch_bounds__(256) void k_csr_rowstats(const int* __restrict__ rp, const TV* __restrict__ val, int n,
                                                      int rows_per_block, double* __restrict__ rowsum,
                                                      double* __restrict__ bpart) {
  __shared__ double red[3][16];
  const int g = threadIdx.x >> 4, li = threadIdx.x & 15;
  const int r0 = blockIdx.x * rows_per_block;
  const int r1 = min(n, r0 + rows_per_block);
  double s = 0.0, q = 0.0, m = -INFINITY;
  for (int i = r0 + g; i < r1; i += 16) {
    double rs = 0.0, rq = 0.0, rm = -INFINITY;
    const int e1 = rp[i + 1];
    for (int e = rp[i] + li; e < e1; e += 16) {
      const double v = (double)val[e];
      rs += v;
      rq += v * v;
      rm = fmax(rm, v);
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) {
      rs += __shfl_xor(rs, o, 16);
      rq += __shfl_xor(rq, o, 16);
      rm = fmax(rm, __shfl_xor(rm, o, 16));
    }
    if (li == 0) rowsum[i] = rs;
    s += rs;
    q += rq;
    m = fmax(m, rm);
  }
  if (li == 0) {
    red[0][g] = s;
    red[1][g] = q;
    red[2][g] = m;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int t = threadIdx.x;
    double v = t == 2 ? -INFINITY : 0.0;
    for (int j = 0; j < 16; ++j) v = t == 2 ? fmax(v, red[2][j]) : v + red[t][j];
    bpart[3 * blockIdx.x + t] = v;
  }
}

// The block partials in a fixed order: thread t sums partials t, t + 256, ...
// in turn, then a fixed tree over the threads.
__global__ __launch_bounds__(256) void k_csr_scalars_final(int nb, const double* __restrict__ bpart,
                                                           double* __restrict__ out) {
  __shared__ double sc[8];
  __shared__ double smax[256];
  double s = 0.0, q = 0.0, m = -INFINITY;
  int b = threadIdx.x;
  for (; b + 7 * 256 < nb; b += 8 * 256) {   // 8 partials' loads in flight, added in order
    double u[8][3];
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
      for (int c = 0; c < 3; ++c) u[j][c] = bpart[3 * (b + 256 * j) + c];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      s += u[j][0];
      q += u[j][1];
      m = fmax(m, u[j][2]);
    }
  }
  for (; b < nb; b += 256) {
    s += bpart[3 * b];
    q += bpart[3 * b + 1];
    m = fmax(m, bpart[3 * b + 2]);
  }
  const double ts = block_sum(s, sc);
  const double tq = block_sum(q, sc);
  smax[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = tq;
    out[1] = ts;
    out[2] = smax[0];
  }
}

// Wave per row.  CW lanes per group cover the columns (CPL columns per lane,
// lane li owns columns li, li + CW, ...); 64 / CW groups take every G-th
// nonzero.  FP64 accumulation.
template <typename TV, typename TB, typename TY, int CW, int CPL>
__global__ __launch_bounds__(256) void k_csr_spmm(const int* __restrict__ rp, const int* __restrict__ ci,
                                                  const TV* __restrict__ val, int n, const TB* __restrict__ B, int c,
                                                  TY* __restrict__ Y, int64_t ldy, const DevState* __restrict__ st) {
  if (stopped(st)) return;
  constexpr int G = 64 / CW;
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const int g = lane / CW, li = lane - g * CW;
  double acc[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) acc[q] = 0.0;
  const int e0 = rp[row], e1 = rp[row + 1];
  int e = e0 + g;
  // gathers in flight per group: 8 when a whole wave takes each nonzero
  // (measured at n = 2^20, c = 64: 1457 -> 1296 us), 4 otherwise
  constexpr int UN = G == 1 ? 8 : 4;
  for (; e + (UN - 1) * G < e1; e += UN * G) {
    int j[UN];
    double v[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      j[u] = ci[e + u * G];
      v[u] = (double)val[e + u * G];
    }
    // column index clamped and masked instead of a branch per load (a branch
    // around each load serialises them)
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const TB* brow = B + (int64_t)j[u] * c;
#pragma unroll
      for (int q = 0; q < CPL; ++q) {
        const int col = li + q * CW;
        const double b = (double)brow[col < c ? col : c - 1];
        acc[q] = fma(v[u], col < c ? b : 0.0, acc[q]);
      }
    }
  }
  for (; e < e1; e += G) {
    const int j = ci[e];
    const double v = (double)val[e];
    const TB* brow = B + (int64_t)j * c;
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const int col = li + q * CW;
      const double b = (double)brow[col < c ? col : c - 1];
      acc[q] = fma(v, col < c ? b : 0.0, acc[q]);
    }
  }
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
#pragma unroll
    for (int o = CW; o < 64; o <<= 1) acc[q] += __shfl_xor(acc[q], o, 64);
  }
  if (g == 0) {
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const int col = li + q * CW;
      if (col < c) Y[(int64_t)row * ldy + col] = (TY)acc[q];
    }
  }
}

__global__ __launch_bounds__(256) void k_to_bf16(const float* __restrict__ F, int64_t count, __bf16* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < count) out[i] = (__bf16)F[i];
}

// The same product with 16-byte row pieces: VEC adjacent columns per lane
// (4 FP32 or 8 BF16), CW = ceil(c / VEC) lanes per group, so one load
// instruction of the wave gathers 64 / CW factor rows and each group keeps UN
// of them in flight.  Needs c % VEC == 0 and 16-byte aligned rows of B.
template <typename TB>
struct Piece;
template <>
struct Piece<float> {
  static constexpr int VEC = 4;
  __device__ static void load(const float* p, double (&x)[4]) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    x[0] = v.x;
    x[1] = v.y;
    x[2] = v.z;
    x[3] = v.w;
  }
};
template <>
struct Piece<__bf16> {
  static constexpr int VEC = 8;
  __device__ static void load(const __bf16* p, double (&x)[8]) {
    const uint4 v = *reinterpret_cast<const uint4*>(p);
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      x[2 * u] = (double)__uint_as_float(w[u] << 16);
      x[2 * u + 1] = (double)__uint_as_float(w[u] & 0xffff0000u);
    }
  }
};

template <typename TV, typename TB, typename TY, int CW, int UN>
__global__ __launch_bounds__(256) void k_csr_spmm_vec(const int* __restrict__ rp, const int* __restrict__ ci,
                                                      const TV* __restrict__ val, int n, const TB* __restrict__ B,
                                                      int c, TY* __restrict__ Y, int64_t ldy,
                                                      const DevState* __restrict__ st) {
  if (stopped(st)) return;
  constexpr int VEC = Piece<TB>::VEC, G = 64 / CW;
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const int g = lane / CW, li = lane - g * CW;
  const int col0 = li * VEC;
  const bool live = col0 < c;
  const int off = live ? col0 : c - VEC;  // clamped piece, masked below
  double acc[VEC];
#pragma unroll
  for (int u = 0; u < VEC; ++u) acc[u] = 0.0;
  const int e0 = rp[row], e1 = rp[row + 1];
  int e = e0 + g;
  for (; e + (UN - 1) * G < e1; e += UN * G) {
    int j[UN];
    double v[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      j[u] = ci[e + u * G];
      v[u] = live ? (double)val[e + u * G] : 0.0;
    }
    double x[UN][VEC];
#pragma unroll
    for (int u = 0; u < UN; ++u) Piece<TB>::load(B + (int64_t)j[u] * c + off, x[u]);
#pragma unroll
    for (int u = 0; u < UN; ++u)
#pragma unroll
      for (int q = 0; q < VEC; ++q) acc[q] = fma(v[u], x[u][q], acc[q]);
  }
  for (; e < e1; e += G) {
    const int j = ci[e];
    const double v = live ? (double)val[e] : 0.0;
    double x[VEC];
    Piece<TB>::load(B + (int64_t)j * c + off, x);
#pragma unroll
    for (int q = 0; q < VEC; ++q) acc[q] = fma(v, x[q], acc[q]);
  }
#pragma unroll
  for (int q = 0; q < VEC; ++q) {
#pragma unroll
    for (int o = CW; o < 64; o <<= 1) acc[q] += __shfl_xor(acc[q], o, 64);
  }
  if (g == 0 && live) {
#pragma unroll
    for (int q = 0; q < VEC; ++q) Y[(int64_t)row * ldy + col0 + q] = (TY)acc[q];
  }
}

// sum over stored (i, j) of X_ij (w_i . h_j); wave per row, lane per column.
template <typename TV, typename TF>
__global__ __launch_bounds__(256) void k_csr_cross(const int* __restrict__ rp, const int* __restrict__ ci,
                                                   const TV* __restrict__ val, int n, int k, const TF* __restrict__ W,
                                                   const TF* __restrict__ H, double* __restrict__ part) {
  __shared__ double sc[8];
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  double acc = 0.0;
  if (row < n && lane < k) {
    const double wi = (double)W[(int64_t)row * k + lane];
    for (int e = rp[row]; e < rp[row + 1]; ++e) acc = fma((double)val[e] * wi, (double)H[(int64_t)ci[e] * k + lane], acc);
  }
  const double t = block_sum(acc, sc);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

template <typename TV, typename TB, typename TY>
void spmm_dispatch(const int* rp, const int* ci, const TV* val, int n, const TB* B, int c, TY* Y, int64_t ldy,
                   const DevState* st, hipStream_t s) {
  const int nb = ceil_div(n, 4);
  if constexpr (!std::is_same<TB, double>::value) {
    constexpr int VEC = Piece<TB>::VEC;
    if (c % VEC == 0 && (reinterpret_cast<uintptr_t>(B) & 15) == 0 && c <= 16 * VEC) {
      const int cw = ceil_div(c, VEC);
      if (cw <= 4)
        k_csr_spmm_vec<TV, TB, TY, 4, 2><<<nb, 256, 0, s>>>(rp, ci, val, n, B, c, Y, ldy, st);
      else if (cw <= 8)
        k_csr_spmm_vec<TV, TB, TY, 8, 2><<<nb, 256, 0, s>>>(rp, ci, val, n, B, c, Y, ldy, st);
      else
        k_csr_spmm_vec<TV, TB, TY, 16, 4><<<nb, 256, 0, s>>>(rp, ci, val, n, B, c, Y, ldy, st);
      return;
    }
  }
  if (c <= 16)
    k_csr_spmm<TV, TB, TY, 16, 1><<<nb, 256, 0, s>>>(rp, ci, val, n, B, c, Y, ldy, st);
  else if (c <= 32)
    k_csr_spmm<TV, TB, TY, 32, 1><<<nb, 256, 0, s>>>(rp, ci, val, n, B, c, Y, ldy, st);
  else if (c <= 64)
    k_csr_spmm<TV, TB, TY, 64, 1><<<nb, 256, 0, s>>>(rp, ci, val, n, B, c, Y, ldy, st);
  else
    k_csr_spmm<TV, TB, TY, 64, 2><<<nb, 256, 0, s>>>(rp, ci, val, n, B, c, Y, ldy, st);
}

}  // namespace

int csr_scalars(const int* rp, const void* val, int vdtype, int n, int64_t nnz, Workspace& ws, double* d_rowsum,
                double* d_out3, hipStream_t s) {
  (void)nnz;
  // at least 16 rows (one per lane group) a block and up to 16384 blocks:
  // a lane group walks its rows one after another, each a chain of
  // dependent reads, so short walks and many waves (n = 2^20: 64 rows a
  // block, four a group; with 1024 rows a block the pass took 137 us)
  const int rows_per_block = std::max(16, ceil_div(n, 16384));
  const int nb = ceil_div(n, rows_per_block);
  double* bpart = ws.dbl(3 * (size_t)nb);
  if (!bpart) return -1;
  if (vdtype == SYMNMF_F64)
    k_csr_rowstats<double><<<nb, 256, 0, s>>>(rp, (const double*)val, n, rows_per_block, d_rowsum, bpart);
  else
    k_csr_rowstats<float><<<nb, 256, 0, s>>>(rp, (const float*)val, n, rows_per_block, d_rowsum, bpart);
  k_csr_scalars_final<<<1, 256, 0, s>>>(nb, bpart, d_out3);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int csr_spmm(const int* rp, const int* ci, const void* val, int vdtype, int n, const void* B, int bdtype, int c,
             void* Y, int ydtype, const DevState* st, hipStream_t s, int64_t ldy) {
  if (c > 128) return -1;
  if (ldy <= 0) ldy = c;
  if (vdtype == SYMNMF_F64) {
    if (bdtype != SYMNMF_F64 || ydtype != SYMNMF_F64) return -1;
    spmm_dispatch<double, double, double>(rp, ci, (const double*)val, n, (const double*)B, c, (double*)Y, ldy, st, s);
  } else {
    if (bdtype == SYMNMF_F32 && ydtype == SYMNMF_F32)
      spmm_dispatch<float, float, float>(rp, ci, (const float*)val, n, (const float*)B, c, (float*)Y, ldy, st, s);
    else if (bdtype == SYMNMF_BF16 && ydtype == SYMNMF_F32)
      spmm_dispatch<float, __bf16, float>(rp, ci, (const float*)val, n, (const __bf16*)B, c, (float*)Y, ldy, st, s);
    else if (bdtype == SYMNMF_F64 && ydtype == SYMNMF_F64)
      spmm_dispatch<float, double, double>(rp, ci, (const float*)val, n, (const double*)B, c, (double*)Y, ldy, st, s);
    else if (bdtype == SYMNMF_F64 && ydtype == SYMNMF_F32)
      spmm_dispatch<float, double, float>(rp, ci, (const float*)val, n, (const double*)B, c, (float*)Y, ldy, st, s);
    else
      return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int to_bf16(const float* F, int64_t count, void* out, hipStream_t s) {
  if (count <= 0) return 0;
  k_to_bf16<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(F, count, (__bf16*)out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int csr_resid_cross(const int* rp, const int* ci, const void* val, int vdtype, int n, int k, const void* W,
                    const void* H, int fdtype, Workspace& ws, double* d_sum, hipStream_t s) {
  if (k > 64) return -1;
  const int nb = ceil_div(n, 4);
  double* part = ws.dbl(nb);
  if (!part) return -1;
  if (vdtype == SYMNMF_F64 && fdtype == SYMNMF_F64)
    k_csr_cross<double, double><<<nb, 256, 0, s>>>(rp, ci, (const double*)val, n, k, (const double*)W,
                                                   (const double*)H, part);
  else if (vdtype == SYMNMF_F32 && fdtype == SYMNMF_F32)
    k_csr_cross<float, float><<<nb, 256, 0, s>>>(rp, ci, (const float*)val, n, k, (const float*)W,
                                                 (const float*)H, part);
  else if (vdtype == SYMNMF_F32 && fdtype == SYMNMF_F64)
    k_csr_cross<float, double><<<nb, 256, 0, s>>>(rp, ci, (const float*)val, n, k, (const double*)W,
                                                  (const double*)H, part);
  else
    return -1;
  sum_partials(part, nb, d_sum, s);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
