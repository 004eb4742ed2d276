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
// Sampled product X S^T S F: row j of it is the sum over the stored X[j][r]
// with r in the sample of X[j][r] w_r F[r, :].  The emit step writes w_r for
// every row (0 off the sample).  The slab of these entries is built without
// sorting: the sampled rows' entries are counted per column (X symmetric: the
// rows j that have any), the counts scanned, and then only those rows j walk
// their own CSR row against the weights and write the sampled entries in
// column order, each at its rank among the row's sampled entries.
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

// FP32 factors on the FP64 matrix cores: Z = F R^{-1} for 16 rows at a time
// with v_mfma_f64_16x16x4f64, lev = row sums of Z o Z.  R^{-1} is upper
// triangular, so the output tile of columns 16 J .. 16 J + 15 needs only the
// K steps p < 16 (J + 1): 4 (J + 1) steps of 4.  Each wave keeps those B
// operands (R^{-1}[4 s + lg][16 J + li] in lane (li, lg), zero below the
// diagonal) in registers for all its row groups.  A group's 16 rows are
// read with coalesced loads into the wave's LDS slab (row stride KP + 1
// floats), from which lane (li, lg) takes A[li][lg] = F[r0 + li][4 s + lg].
// The four accumulator registers of lane (li, lg) hold rows lg + 4 v of
// column li; squares are summed over the tiles and then over the 16 lanes
// of a DPP row.
// At KP = 64 the kernel is held to 168 registers, three waves per SIMD
// instead of two (137 VGPRs + 32 AGPRs otherwise): n = 2^20, leverage with
// its Cholesky 216 -> 210 us.
template <int KP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KP == 64 ? 3 : 1))) void k_leverage_mfma(const float* __restrict__ F, int n, int k,
                                                       const double* __restrict__ Rinv, double* __restrict__ lev,
                                                       int iters, const DevState* __restrict__ st) {
  if (stopped(st)) return;
  constexpr int KT = KP / 16, NB = 2 * KT * (KT + 1), LW = KP + 1;
  __shared__ float slab[4][16 * LW];
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  float* hs = slab[wid];
  double breg[NB];
  {
    int b = 0;
#pragma unroll
    for (int J = 0; J < KT; ++J)
#pragma unroll
      for (int s4 = 0; s4 < 4 * (J + 1); ++s4, ++b) {
        const int p = 4 * s4 + lg, i = 16 * J + li;
        const bool in = p <= i && i < k;
        const double v = Rinv[in ? p * k + i : 0];   // clamped index, masked value
        breg[b] = in ? v : 0.0;
      }
  }
  const int groups = (n + 15) / 16;
  for (int it = 0; it < iters; ++it) {
    const int grp = (it * gridDim.x + blockIdx.x) * 4 + wid;
    const int r0 = 16 * grp;
    // the group's rows (16 k floats, contiguous) into the slab
    const int rows = grp < groups ? min(16, n - r0) : 0;
    if (k == KP) {
      // 16 KP floats as float4 pieces: piece e is row e / (KP / 4)
      constexpr int P4 = KP / 4;
      const float4* src = reinterpret_cast<const float4*>(F);
#pragma unroll
      for (int e = lane; e < 16 * P4; e += 64) {
        const int r = e / P4, c = 4 * (e - r * P4);
        const float4 v = src[r < rows ? (int64_t)r0 * P4 + e : 0];   // clamped index, masked value
        float* d = hs + r * LW + c;
        d[0] = r < rows ? v.x : 0.0f;
        d[1] = r < rows ? v.y : 0.0f;
        d[2] = r < rows ? v.z : 0.0f;
        d[3] = r < rows ? v.w : 0.0f;
      }
    } else {
      for (int e = lane; e < 16 * k; e += 64) {
        const int r = e / k, c = e - r * k;
        const float v = F[r < rows ? (int64_t)r0 * k + e : 0];   // clamped index, masked value
        hs[r * LW + c] = r < rows ? v : 0.0f;
      }
    }
    __syncthreads();
    double a[4 * KT];
#pragma unroll
    for (int s4 = 0; s4 < 4 * KT; ++s4) {
      const int p = 4 * s4 + lg;
      a[s4] = p < k ? (double)hs[li * LW + p] : 0.0;
    }
    // K step outermost, so the tiles' matrix-core chains interleave
    doublex4 acc[KT];
#pragma unroll
    for (int J = 0; J < KT; ++J) acc[J] = doublex4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s4 = 0; s4 < 4 * KT; ++s4) {
#pragma unroll
      for (int J = s4 / 4; J < KT; ++J) {
        // B operand of tile J, step s4: index 2 J (J + 1) + s4 in breg
        acc[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s4], breg[2 * J * (J + 1) + s4], acc[J], 0, 0, 0);
      }
    }
    double t[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int J = 0; J < KT; ++J)
#pragma unroll
      for (int v = 0; v < 4; ++v) t[v] = fma(acc[J][v], acc[J][v], t[v]);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double tot = row16_sum(t[v]);
      const int r = lg + 4 * v;
      if (li == 0 && r < rows) lev[r0 + r] = tot;
    }
    __syncthreads();
  }
}

// The block partials of the deterministic rows' leverage mass (summed in the
// order of a fixed-order partial sum: 8 loads in flight per thread) and their
// count; info[1] is cleared for a sample without draws.
__global__ __launch_bounds__(256) void k_sample_totals(const double* __restrict__ tpart,
                                                       const int* __restrict__ cpart, int nb,
                                                       double* __restrict__ theta, int* __restrict__ info) {
  __shared__ double sc[8];
  double v = 0.0;
  int c = 0;
  int i = threadIdx.x;
  for (; i + 7 * 256 < nb; i += 8 * 256) {
    double u[8];
    int cu[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      u[q] = tpart[i + q * 256];
      cu[q] = cpart[i + q * 256];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      v += u[q];
      c += cu[q];
    }
  }
  for (; i < nb; i += 256) {
    v += tpart[i];
    c += cpart[i];
  }
  const double t = block_sum(v, sc);
  const double ct = block_sum((double)c, sc);   // an integer count, exact in FP64
  if (threadIdx.x == 0) {
    theta[0] = t;
    info[0] = (int)ct;
    info[1] = 0;
  }
}

// 1024 rows a block, four a thread in the order of the device scans, so the
// block's sum of the quantised weights is the prefix scan's block total
// (wsum) and that scan takes one launch.
__global__ __launch_bounds__(256) void k_quantize(const double* __restrict__ lev, int n, int k, double tau,
                                                  uint64_t* __restrict__ w, int* __restrict__ det,
                                                  double* __restrict__ tpart, int* __restrict__ cpart,
                                                  uint64_t* __restrict__ wsum, const DevState* __restrict__ st) {
  if (stopped(st)) return;
  __shared__ double sc[8];
  __shared__ unsigned long long su[4];
  const int base = blockIdx.x * 1024 + threadIdx.x * 4;
  double th = 0.0;
  int cnt = 0;
  unsigned long long ws = 0;
  double lv[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) lv[u] = lev[min(base + u, n - 1)];   // the four loads in flight together
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = base + u;
    if (i < n) {
      const double l = lv[u];
      const bool d = (l / (double)k) >= tau;
      const uint64_t q = d ? 0ull : (uint64_t)(l * 1099511627776.0);  // floor(l * 2^40), l >= 0
      det[i] = d ? 1 : 0;
      w[i] = q;
      ws += q;
      if (d) {
        th += l;
        ++cnt;
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) ws += __shfl_xor(ws, o);
  if ((threadIdx.x & 63) == 0) su[threadIdx.x >> 6] = ws;
  const double t = block_sum(th, sc);
  const double c = block_sum((double)cnt, sc);   // an integer count, exact in FP64
  if (threadIdx.x == 0) {
    tpart[blockIdx.x] = t;
    cpart[blockIdx.x] = (int)c;
    wsum[blockIdx.x] = (uint64_t)(su[0] + su[1] + su[2] + su[3]);
  }
}

constexpr int DRAW_COARSE = 4096;   // pieces of 1024 rows the draw's LDS table covers (32 KB)

__global__ __launch_bounds__(256) void k_draw(const uint64_t* __restrict__ prefix, int n, int64_t s_total,
                                              uint64_t seed, uint32_t half_iter, int* __restrict__ counts,
                                              int* __restrict__ info, const DevState* __restrict__ st) {
  if (stopped(st)) return;
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t s_R = s_total - (int64_t)info[0];
  if (j == 0) info[1] = (int)(s_R > 0 ? s_R : 0);
  // the prefix at the end of every 1024 rows, in LDS, narrows each search to
  // one 1024-row piece (half of the dependent reads from memory)
  __shared__ uint64_t coarse[DRAW_COARSE];
  const int nbk = (n + 1023) / 1024;
  const bool two_level = nbk <= DRAW_COARSE;
  if (two_level) {
    for (int b = threadIdx.x; b < nbk; b += 256) coarse[b] = prefix[min(1024 * b + 1023, n - 1)];
    __syncthreads();
  }
  if (j >= s_R) return;
  const uint64_t WR = prefix[n - 1];
  if (WR == 0) return;
  const uint64_t v = philox_value(seed, (uint64_t)j, half_iter, TAG_SAMPLE);
  const uint64_t r = __umul64hi(v, WR);
  // smallest i with prefix[i] > r (exists: prefix[n-1] = WR > r)
  int lo = 0, hi = n - 1;
  if (two_level) {
    int bl = 0, bh = nbk - 1;   // smallest piece whose last prefix exceeds r
    while (bl < bh) {
      const int mid = (bl + bh) >> 1;
      if (coarse[mid] > r) bh = mid; else bl = mid + 1;
    }
    lo = 1024 * bl;
    hi = min(1024 * bl + 1023, n - 1);
  }
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] > r) hi = mid; else lo = mid + 1;
  }
  atomicAdd(&counts[lo], 1);
}

// The sample's rows in order: the selected rows (deterministic, or drawn at
// least once) get their places from an exclusive scan over 1024-row blocks
// (each block adds the totals of the blocks before it, given in bsum), and
// each takes its row index and weight at its place; every row's weight (0
// off the sample) goes to wmask and the draw counts are cleared.
__global__ __launch_bounds__(256) void k_select_emit(const int* __restrict__ det, int* __restrict__ counts,
                                                     const uint64_t* __restrict__ w,
                                                     const uint64_t* __restrict__ prefix,
                                                     const int* __restrict__ bsum, int n, int* __restrict__ rows,
                                                     double* __restrict__ weights, int64_t cap,
                                                     int* __restrict__ info, double* __restrict__ wmask,
                                                     const DevState* __restrict__ st) {
  if (stopped(st)) return;
  __shared__ int wsi[4];
  int pre = 0;
  for (int b = threadIdx.x; b < (int)blockIdx.x; b += 256) pre += bsum[b];
  int off;
  block_exclusive_scan<int>(pre, wsi, off);
  const int base = blockIdx.x * 1024 + threadIdx.x * 4;
  int dt[4], cu[4], sel[4], s = 0;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = base + u;
    dt[u] = i < n ? det[i] : 0;
    cu[u] = i < n ? counts[i] : 0;
    sel[u] = (dt[u] || cu[u] > 0) ? 1 : 0;
    s += sel[u];
  }
  int tot;
  int run = block_exclusive_scan<int>(s, wsi, tot) + off;
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
    info[2] = (int)min((int64_t)(off + tot), cap);
    info[3] = off + tot;
  }
  const double WR = (double)prefix[n - 1];
  const double sR = (double)info[1];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = base + u;
    if (i < n) {
      double wt = 0.0;
      if (sel[u] && run < cap) {
        rows[run] = i;
        wt = dt[u] ? 1.0 : ((double)cu[u] * WR) / (sR * (double)w[i]);
        weights[run] = wt;
      }
      if (wmask) wmask[i] = wt;
      counts[i] = 0;
    }
    run += sel[u];
  }
}

// One wave per sampled row; lanes walk the row's nonzeros.  X symmetric:
// the row's column i gets one entry in segment i.
__global__ __launch_bounds__(256) void k_slab_count(const int* __restrict__ rp, const int* __restrict__ ci,
                                                    const int* __restrict__ rows, const int* __restrict__ d_count,
                                                    int* __restrict__ cnt, const DevState* __restrict__ st) {
  if (stopped(st)) return;
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= *d_count) return;
  const int r = rows[t];
  for (int e = rp[r] + (threadIdx.x & 63); e < rp[r + 1]; e += 64) atomicAdd(&cnt[ci[e]], 1);
}

// The sampled slab by scatter: a wave per sampled row r puts each stored
// entry X[r][i] (times r's weight) into row i's segment (X is symmetric),
// at a slot taken by counting cnt[i] down (which leaves cnt cleared); the
// slots within a segment depend on the order of the atomics, so
// k_slab_order then puts every segment in column order.
template <typename TV>
__global__ __launch_bounds__(256) void k_slab_scatter(const int* __restrict__ rp, const int* __restrict__ ci,
                                                      const TV* __restrict__ val, const int* __restrict__ rows,
                                                      const int* __restrict__ d_count, const double* __restrict__ wmask,
                                                      int* __restrict__ cnt, const int* __restrict__ seg_ptr,
                                                      int* __restrict__ seg_src, double* __restrict__ seg_val,
                                                      int64_t seg_cap, const DevState* __restrict__ st) {
  if (stopped(st)) return;
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= *d_count) return;
  const int r = rows[t];
  const double w = wmask[r];
  for (int e = rp[r] + (threadIdx.x & 63); e < rp[r + 1]; e += 64) {
    const int i = ci[e];
    const int64_t p = (int64_t)seg_ptr[i] + atomicSub(&cnt[i], 1) - 1;
    if (p < seg_cap) {
      seg_src[p] = r;
      seg_val[p] = (double)val[e] * w;
    }
  }
}

// Column order within every segment of two or more entries (a few per cent
// of the rows; a few have tens).  A wave reads the bounds of 64 consecutive
// rows, takes those rows four at a time, 16 lanes each: up to 64 entries
// are read into registers (four per lane), each entry's rank is counted
// against all the row's keys (broadcast by lane shuffles within the 16-lane
// row), and every entry is written to its rank: keys are distinct, so the
// ranks are a permutation.  A longer segment (a row adjacent to many
// sampled rows: hubs of a skewed graph) is written again in order from the
// row's own stored entries, 16 at a time, each tested against the sample's
// weights (a ballot gives each hit its place): time in the row's length, not
// in the square of the segment's.
template <typename TV>
__global__ __launch_bounds__(256) void k_slab_order(const int* __restrict__ rp, const int* __restrict__ ci,
                                                    const TV* __restrict__ val, const double* __restrict__ wmask,
                                                    const int* __restrict__ seg_ptr, int n, int64_t seg_cap,
                                                    int* __restrict__ seg_src, double* __restrict__ seg_val,
                                                    const DevState* __restrict__ st) {
  if (stopped(st)) return;
  const int lane = threadIdx.x & 63, g = lane >> 4, li = lane & 15;
  const int j0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 64;
  if (j0 >= n) return;   // the same for the whole wave
  const int jl = j0 + lane;
  const int sb = jl < n ? seg_ptr[jl] : 0;
  const int se = jl < n ? (int)min((int64_t)seg_ptr[jl + 1], seg_cap) : 0;
  uint64_t act = __ballot(se - sb >= 2);
  while (act) {   // the same for the whole wave
    uint64_t m = act;
    for (int t = 0; t < g; ++t) m &= m - 1;
    const bool have = m != 0;
    const int src = have ? __ffsll((unsigned long long)m) - 1 : 0;
    const int b = __shfl(sb, src);
    const int c = have ? __shfl(se, src) - b : 0;
    const int row = __shfl(jl, src);   // every lane takes part in the shuffles
    if (c <= 64) {
      int key[4];
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = li + 16 * u;
        key[u] = q < c ? seg_src[b + q] : 0x7fffffff;
        v[u] = q < c ? seg_val[b + q] : 0.0;
      }
      int rank[4] = {0, 0, 0, 0};
      // c is the same in the 16 lanes of a row, so every lane a shuffle
      // reads from is active
      for (int q = 0; q < c; ++q) {
        const int kq = __shfl(key[q >> 4], (lane & 48) + (q & 15));
#pragma unroll
        for (int u = 0; u < 4; ++u) rank[u] += kq < key[u] ? 1 : 0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (li + 16 * u < c) {
          seg_src[b + rank[u]] = key[u];
          seg_val[b + rank[u]] = v[u];
        }
      }
    } else {
      const int e0 = rp[row], e1 = rp[row + 1];
      const int sh = lane & 48;
      int base = b;
      for (int e = e0 + li; e - li < e1; e += 16) {   // the same trips for the row's 16 lanes
        const bool ok = e < e1;
        const int r = ci[ok ? e : e0];
        const double w = wmask[r];
        const bool hit = ok && w != 0.0;
        const uint64_t mb = (__ballot(hit) >> sh) & 0xFFFFull;
        if (hit) {
          const int p = base + __popcll(mb & ((1ull << li) - 1ull));
          if (p < seg_cap) {
            seg_src[p] = r;
            seg_val[p] = (double)val[e] * w;
          }
        }
        base += __popcll(mb);
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) act &= act - 1;
  }
}

// a 32-bit word of lanes 32..63 of x <-> lanes 0..31 of y (halves), or of the
// odd 16-lane rows of x <-> the even rows of y
__device__ __forceinline__ void swap_f32(float& x, float& y, bool halves) {
  const unsigned ux = __float_as_uint(x), uy = __float_as_uint(y);
  const auto r = halves ? __builtin_amdgcn_permlane32_swap(ux, uy, false, false)
                        : __builtin_amdgcn_permlane16_swap(ux, uy, false, false);
  x = __uint_as_float(r[0]);
  y = __uint_as_float(r[1]);
}

// The same products with k = KP and a 16-byte aligned factor, without LDS:
// lane (li, lg) reads float4 pieces lg, lg + 4, ... of row li of its group
// (4 KT pieces, the next group's in flight during this group's products);
// a 4 x 4 transpose across the lane groups by permlane swaps (per li: piece
// 4 p + r of lane group r, element t -> lane group t, element r) leaves
// lane (li, lg) the row's columns 4 s + lg, the A operand of K step s.
// Each wave walks its own groups, so no workgroup barrier.  At n = 2^20,
// k = 64: 101 us against 141 us with the LDS staging and its barriers (the
// FP64 matrix cores at 66% of their peak over the 40 products of a group;
// split accumulator chains or two waves per SIMD changed nothing).
template <int KP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KP == 64 ? 3 : 1))) void k_leverage_rows(
    const float* __restrict__ F, int n, const double* __restrict__ Rinv, double* __restrict__ lev,
    const DevState* __restrict__ st) {
  if (stopped(st)) return;
  constexpr int KT = KP / 16, NB = 2 * KT * (KT + 1);
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  double breg[NB];
  {
    int b = 0;
#pragma unroll
    for (int J = 0; J < KT; ++J)
#pragma unroll
      for (int s4 = 0; s4 < 4 * (J + 1); ++s4, ++b) {
        const int p = 4 * s4 + lg, i = 16 * J + li;
        const double v = Rinv[p <= i ? p * KP + i : 0];   // clamped index, masked value
        breg[b] = p <= i ? v : 0.0;
      }
  }
  const int groups = (n + 15) / 16, gstride = 4 * gridDim.x;
  float4 x[KT];
  auto load = [&](int g) {
    const float4* src = reinterpret_cast<const float4*>(F + (int64_t)min(16 * g + li, n - 1) * KP);
#pragma unroll
    for (int q = 0; q < KT; ++q) x[q] = src[lg + 4 * q];
  };
  int grp = 4 * blockIdx.x + wid;
  if (grp < groups) load(grp);
  for (; grp < groups; grp += gstride) {
    double a[4 * KT];
#pragma unroll
    for (int q = 0; q < KT; ++q) {
      float e[4] = {x[q].x, x[q].y, x[q].z, x[q].w};
      swap_f32(e[0], e[2], true);
      swap_f32(e[1], e[3], true);
      swap_f32(e[0], e[1], false);
      swap_f32(e[2], e[3], false);
#pragma unroll
      for (int t = 0; t < 4; ++t) a[4 * q + t] = (double)e[t];
    }
    if (grp + gstride < groups) load(grp + gstride);
    doublex4 acc[KT];
#pragma unroll
    for (int J = 0; J < KT; ++J) acc[J] = doublex4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s4 = 0; s4 < 4 * KT; ++s4) {
#pragma unroll
      for (int J = s4 / 4; J < KT; ++J)
        acc[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s4], breg[2 * J * (J + 1) + s4], acc[J], 0, 0, 0);
    }
    double t[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int J = 0; J < KT; ++J)
#pragma unroll
      for (int v = 0; v < 4; ++v) t[v] = fma(acc[J][v], acc[J][v], t[v]);
    const int r0 = 16 * grp, rows = min(16, n - r0);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double tot = row16_sum(t[v]);
      const int r = lg + 4 * v;
      if (li == 0 && r < rows) lev[r0 + r] = tot;
    }
  }
}

template <int KP, typename TF>
void lev_launch(const void* F, int n, int k, const double* Rinv, double* lev, const DevState* st, hipStream_t s) {
  if constexpr (std::is_same<TF, float>::value) {
    // four 16-row groups per block and step; about four blocks per CU
    // (float4 row pieces need a 16-byte aligned factor)
    if ((reinterpret_cast<uintptr_t>(F) & 15) != 0) {
      k_leverage<KP, TF><<<ceil_div(n, 256), 256, 0, s>>>((const TF*)F, n, k, Rinv, lev, st);
      return;
    }
    const int groups = ceil_div(n, 16);
    const int nb = std::max(1, std::min(1024, ceil_div(groups, 4)));
    if (k == KP) {
      // at KP = 64 three waves per SIMD: 768 blocks fill the chip once
      // (n = 2^20: 101 against 104 us with 1024)
      const int nbr = KP == 64 ? std::max(1, std::min(768, ceil_div(groups, 4))) : nb;
      k_leverage_rows<KP><<<nbr, 256, 0, s>>>((const float*)F, n, Rinv, lev, st);
      return;
    }
    const int iters = ceil_div(groups, 4 * nb);
    k_leverage_mfma<KP><<<nb, 256, 0, s>>>((const float*)F, n, k, Rinv, lev, iters, st);
    return;
  }
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
                  hipStream_t s, double* wmask) {
  const int nq = ceil_div(n, 1024);
  double* tpart = ws.dbl(nq);
  int* cpart = ws.i32(nq);
  uint64_t* wsum = ws.u64(nq);
  int* bsel = ws.i32(nq);
  if (!tpart || !cpart || !wsum || !bsel) return -1;
  k_quantize<<<nq, 256, 0, s>>>(lev, n, k, tau, sb.w, sb.flags, tpart, cpart, wsum, st);
  k_sample_totals<<<1, 256, 0, s>>>(tpart, cpart, nq, sb.theta, sb.info);
  if (inclusive_scan_u64_from_sums(sb.w, sb.prefix, n, wsum, s)) return -1;
  if (s_total > 0) k_draw<<<ceil_div(s_total, 256), 256, 0, s>>>(sb.prefix, n, s_total, seed, half_iter, sb.counts, sb.info, st);
  if (selected_block_sums(sb.flags, sb.counts, n, bsel, s)) return -1;
  k_select_emit<<<nq, 256, 0, s>>>(sb.flags, sb.counts, sb.w, sb.prefix, bsel, n, rows, weights, cap, sb.info, wmask,
                                   st);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int sampled_slab(const int* rp, const int* ci, const void* val, int vdtype, int n, const int* rows,
                 const int* d_count, int max_rows, const double* wmask, int* seg_cnt,
                 int* seg_ptr, int* seg_src, double* seg_val, int64_t seg_cap, Workspace& ws, const DevState* st,
                 hipStream_t s) {
  if (!wmask) return -1;
  const int nbw = std::max(1, ceil_div(max_rows, 4));
  k_slab_count<<<nbw, 256, 0, s>>>(rp, ci, rows, d_count, seg_cnt, st);
  if (exclusive_scan_i32(seg_cnt, seg_ptr, n, ws, s)) return -1;
  if (vdtype == SYMNMF_F64)
    k_slab_scatter<double><<<nbw, 256, 0, s>>>(rp, ci, (const double*)val, rows, d_count, wmask, seg_cnt, seg_ptr,
                                               seg_src, seg_val, seg_cap, st);
  else
    k_slab_scatter<float><<<nbw, 256, 0, s>>>(rp, ci, (const float*)val, rows, d_count, wmask, seg_cnt, seg_ptr,
                                              seg_src, seg_val, seg_cap, st);
  if (vdtype == SYMNMF_F64)
    k_slab_order<double><<<ceil_div(n, 256), 256, 0, s>>>(rp, ci, (const double*)val, wmask, seg_ptr, n, seg_cap,
                                                          seg_src, seg_val, st);
  else
    k_slab_order<float><<<ceil_div(n, 256), 256, 0, s>>>(rp, ci, (const float*)val, wmask, seg_ptr, n, seg_cap,
                                                         seg_src, seg_val, st);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
