// Leverage-score sampling (Algorithm LvS-SymNMF, hybrid scheme of
// Section 4.2).
//
// Leverage scores lev_i = ||F[i,:] R^{-1}||^2 with R = chol(F^T F): one row per
// thread, R^{-1} read with wave-uniform (scalar) loads.
//
// Hybrid sampler, all on the device and in integer arithmetic where it decides
// which rows are drawn:
//   1. rows with lev_i / k >= tau are deterministic (weight 1); the others get
//      the integer weight w_i = floor(lev_i * 2^40);
//   2. inclusive prefix sums of w (uint64) give W_R = sum w;
//   3. draw j < s_R = s - s_D takes r = mulhi64(v_j, W_R) (v_j: Philox value j
//      of stream (seed, half-iteration, SAMPLE)) and the smallest row whose
//      prefix exceeds r; draws are counted per row with integer atomics;
//   4. selected rows are compacted in ascending order with their weight
//      (1, or c W_R / (s_R w_i) for a row drawn c times: c draws of
//      1 / (s_R p~_i) with p~_i = w_i / W_R).
//
// Sampled product X S^T S F: X is symmetric, so the sampled columns are the
// sampled CSR rows.  They are scattered into a transposed slab (segment i
// holds the (r, X_ri w_r) of all sampled rows r with X_ri != 0), sorted by r
// inside each segment so the HALS sweep sums them in a fixed order.
#include "kernels.hpp"

namespace {

// Thread per row; R^{-1} (upper triangular) staged once per 256-row block
// in LDS and read as broadcasts.
template <int KP, typename TF>
__global__ __launch_bounds__(256) void k_leverage(const TF* __restrict__ F, int n, int k,
                                                  const double* __restrict__ Rinv, double* __restrict__ lev,
                                                  const DevState* __restrict__ st) {
  if (stopped(st)) return;
  __shared__ double Rs[KP * KP];
  for (int e = threadIdx.x; e < KP * KP; e += 256) {
    const int p = e / KP, i = e - p * KP;
    Rs[e] = (p < k && i < k) ? Rinv[p * k + i] : 0.0;
  }
  __syncthreads();
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  double h[KP];
#pragma unroll
  for (int i = 0; i < KP; ++i) {
    const double x = (double)F[(int64_t)j * k + (i < k ? i : k - 1)];
    h[i] = i < k ? x : 0.0;
  }
  double acc = 0.0;
#pragma unroll
  for (int i = 0; i < KP; ++i) {
    if (i < k) {
      double q = 0.0;
#pragma unroll
      for (int p = 0; p <= i; ++p) q = fma(h[p], Rs[p * KP + i], q);
      acc = fma(q, q, acc);
    }
  }
  lev[j] = acc;
}

__global__ void k_sample_reset(int* info, double* theta) {
  if (threadIdx.x == 0) {
    info[0] = 0;
    info[1] = 0;
    info[2] = 0;
    info[3] = 0;
    theta[0] = 0.0;
  }
}

__global__ __launch_bounds__(256) void k_quantize(const double* __restrict__ lev, int n, int k, double tau,
                                                  uint64_t* __restrict__ w, int* __restrict__ det,
                                                  int* __restrict__ info, double* __restrict__ tpart,
                                                  const DevState* __restrict__ st) {
  if (stopped(st)) return;
  __shared__ double sc[8];
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  const int i = blockIdx.x * 256 + threadIdx.x;
  double th = 0.0;
  if (i < n) {
    const double l = lev[i];
    const bool d = (l / (double)k) >= tau;
    det[i] = d ? 1 : 0;
    w[i] = d ? 0ull : (uint64_t)(l * 1099511627776.0);  // floor(l * 2^40), l >= 0
    if (d) {
      th = l;
      atomicAdd(&cnt, 1);
    }
  }
  const double t = block_sum(th, sc);
  __syncthreads();
  if (threadIdx.x == 0) {
    tpart[blockIdx.x] = t;
    if (cnt) atomicAdd(&info[0], cnt);
  }
}

__global__ __launch_bounds__(256) void k_draw(const uint64_t* __restrict__ prefix, int n, int64_t s_total,
                                              uint64_t seed, uint32_t half_iter, int* __restrict__ counts,
                                              int* __restrict__ info, const DevState* __restrict__ st) {
  if (stopped(st)) return;
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t s_R = s_total - (int64_t)info[0];
  if (j == 0) info[1] = (int)(s_R > 0 ? s_R : 0);
  if (j >= s_R) return;
  const uint64_t WR = prefix[n - 1];
  if (WR == 0) return;
  const uint64_t v = philox_value(seed, (uint64_t)j, half_iter, TAG_SAMPLE);
  const uint64_t r = __umul64hi(v, WR);
  int lo = 0, hi = n - 1;  // smallest i with prefix[i] > r (exists: prefix[n-1] = WR > r)
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] > r) hi = mid; else lo = mid + 1;
  }
  atomicAdd(&counts[lo], 1);
}

__global__ __launch_bounds__(256) void k_select(const int* __restrict__ det, const int* __restrict__ counts, int n,
                                                int* __restrict__ sel, const DevState* __restrict__ st) {
  if (stopped(st)) return;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) sel[i] = (det[i] || counts[i] > 0) ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_emit(const int* __restrict__ det, int* __restrict__ counts,
                                              const uint64_t* __restrict__ w, const uint64_t* __restrict__ prefix,
                                              const int* __restrict__ sel, const int* __restrict__ pos, int n,
                                              int* __restrict__ rows, double* __restrict__ weights, int64_t cap,
                                              int* __restrict__ info, const DevState* __restrict__ st) {
  if (stopped(st)) return;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i == 0) {
    info[2] = (int)min((int64_t)pos[n], cap);
    info[3] = pos[n];
  }
  if (i >= n) return;
  if (sel[i] && pos[i] < cap) {
    const int p = pos[i];
    rows[p] = i;
    if (det[i]) {
      weights[p] = 1.0;
    } else {
      const double WR = (double)prefix[n - 1];
      const double sR = (double)info[1];
      weights[p] = ((double)counts[i] * WR) / (sR * (double)w[i]);
    }
  }
  counts[i] = 0;
}

// One wave per sampled row; lanes walk the row's nonzeros.
__global__ __launch_bounds__(256) void k_slab_count(const int* __restrict__ rp, const int* __restrict__ ci,
                                                    const int* __restrict__ rows, const int* __restrict__ d_count,
                                                    int* __restrict__ cnt, const DevState* __restrict__ st) {
  if (stopped(st)) return;
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= *d_count) return;
  const int r = rows[t];
  for (int e = rp[r] + (threadIdx.x & 63); e < rp[r + 1]; e += 64) atomicAdd(&cnt[ci[e]], 1);
}

template <typename TV>
__global__ __launch_bounds__(256) void k_slab_fill(const int* __restrict__ rp, const int* __restrict__ ci,
                                                   const TV* __restrict__ val, const int* __restrict__ rows,
                                                   const double* __restrict__ weights, const int* __restrict__ d_count,
                                                   int* __restrict__ cnt, const int* __restrict__ seg_ptr,
                                                   int* __restrict__ seg_src, double* __restrict__ seg_val,
                                                   int64_t seg_cap, const DevState* __restrict__ st) {
  if (stopped(st)) return;
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= *d_count) return;
  const int r = rows[t];
  const double wr = weights[t];
  for (int e = rp[r] + (threadIdx.x & 63); e < rp[r + 1]; e += 64) {
    const int i = ci[e];
    const int p = seg_ptr[i] + atomicSub(&cnt[i], 1) - 1;
    if (p < seg_cap) {
      seg_src[p] = r;
      seg_val[p] = (double)val[e] * wr;
    }
  }
}

__global__ __launch_bounds__(256) void k_slab_sort(const int* __restrict__ seg_ptr, int n, int* __restrict__ seg_src,
                                                   double* __restrict__ seg_val, int64_t seg_cap,
                                                   const DevState* __restrict__ st) {
  if (stopped(st)) return;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int e0 = (int)min((int64_t)seg_ptr[i], seg_cap), e1 = (int)min((int64_t)seg_ptr[i + 1], seg_cap);
  for (int a = e0 + 1; a < e1; ++a) {
    const int ks = seg_src[a];
    const double kv = seg_val[a];
    int b = a - 1;
    while (b >= e0 && seg_src[b] > ks) {
      seg_src[b + 1] = seg_src[b];
      seg_val[b + 1] = seg_val[b];
      --b;
    }
    seg_src[b + 1] = ks;
    seg_val[b + 1] = kv;
  }
}

template <int KP, typename TF>
void lev_launch(const void* F, int n, int k, const double* Rinv, double* lev, const DevState* st, hipStream_t s) {
  k_leverage<KP, TF><<<ceil_div(n, 256), 256, 0, s>>>((const TF*)F, n, k, Rinv, lev, st);
}

}  // namespace

int leverage_scores(const void* F, int fdtype, int n, int k, const double* Rinv, double* lev, const DevState* st,
                    hipStream_t s) {
  const int kp = k <= 16 ? 16 : (k <= 32 ? 32 : 64);
  if (k > 64) return -1;
  if (fdtype == SYMNMF_F64) {
    if (kp == 16) lev_launch<16, double>(F, n, k, Rinv, lev, st, s);
    else if (kp == 32) lev_launch<32, double>(F, n, k, Rinv, lev, st, s);
    else lev_launch<64, double>(F, n, k, Rinv, lev, st, s);
  } else {
    if (kp == 16) lev_launch<16, float>(F, n, k, Rinv, lev, st, s);
    else if (kp == 32) lev_launch<32, float>(F, n, k, Rinv, lev, st, s);
    else lev_launch<64, float>(F, n, k, Rinv, lev, st, s);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int hybrid_sample(const double* lev, int n, int k, int64_t s_total, double tau, uint64_t seed, uint32_t half_iter,
                  SampleBuffers& sb, int* rows, double* weights, int64_t cap, Workspace& ws, const DevState* st,
                  hipStream_t s) {
  const int nb = ceil_div(n, 256);
  double* tpart = ws.dbl(nb);
  int* sel = ws.i32(n);
  int* pos = ws.i32((size_t)n + 1);
  if (!tpart || !sel || !pos) return -1;
  k_sample_reset<<<1, 64, 0, s>>>(sb.info, sb.theta);
  k_quantize<<<nb, 256, 0, s>>>(lev, n, k, tau, sb.w, sb.flags, sb.info, tpart, st);
  sum_partials(tpart, nb, sb.theta, s);
  if (inclusive_scan_u64(sb.w, sb.prefix, n, ws, s)) return -1;
  if (s_total > 0) k_draw<<<ceil_div(s_total, 256), 256, 0, s>>>(sb.prefix, n, s_total, seed, half_iter, sb.counts, sb.info, st);
  k_select<<<nb, 256, 0, s>>>(sb.flags, sb.counts, n, sel, st);
  if (exclusive_scan_i32(sel, pos, n, ws, s)) return -1;
  k_emit<<<nb, 256, 0, s>>>(sb.flags, sb.counts, sb.w, sb.prefix, sel, pos, n, rows, weights, cap, sb.info, st);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int sampled_slab(const int* rp, const int* ci, const void* val, int vdtype, int n, const int* rows,
                 const double* weights, const int* d_count, int max_rows, int* seg_cnt, int* seg_ptr, int* seg_src,
                 double* seg_val, int64_t seg_cap, Workspace& ws, const DevState* st, hipStream_t s) {
  const int nbw = std::max(1, ceil_div(max_rows, 4));
  k_slab_count<<<nbw, 256, 0, s>>>(rp, ci, rows, d_count, seg_cnt, st);
  if (exclusive_scan_i32(seg_cnt, seg_ptr, n, ws, s)) return -1;
  if (vdtype == SYMNMF_F64)
    k_slab_fill<double><<<nbw, 256, 0, s>>>(rp, ci, (const double*)val, rows, weights, d_count, seg_cnt, seg_ptr,
                                            seg_src, seg_val, seg_cap, st);
  else
    k_slab_fill<float><<<nbw, 256, 0, s>>>(rp, ci, (const float*)val, rows, weights, d_count, seg_cnt, seg_ptr,
                                           seg_src, seg_val, seg_cap, st);
  k_slab_sort<<<ceil_div(n, 256), 256, 0, s>>>(seg_ptr, n, seg_src, seg_val, seg_cap, st);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
