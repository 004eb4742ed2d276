// Fused half-step update: one kernel forms the right-hand side of every row,
// applies the regularised HALS sweep, writes the new factor (and, for the
// dense product, its padded transpose for the next GEMM) and accumulates the
// block partials of the next step's small products -- the Gram matrix of the
// new factor, for the LAI path U^T F, and the residual dot product -- so a
// half-iteration needs the product, this kernel and one small reduction.
//
// Right-hand side of row j (Update(G, Y) of the Appendix with the
// regularised pair; Y stored as X F, row-major):
//   YMODE 0  y_j = sum_s P[s][j]          split-K partials of X F (or X F)
//   YMODE 1  y_j = sum_e v_e F[src_e]     transposed sampled slab (LvS)
//   YMODE 2  y_j = U[j,:] M,  M = Lambda U^T F   (LAI)
// and the HALS target is y_j + alpha F[j].
#include "kernels.hpp"

namespace {

template <int KP, int LP, typename TF, typename TP, typename TT, int YMODE, int NTH>
__global__ __launch_bounds__(NTH) void k_update(UpdateArgs a, const double* __restrict__ Gh,
                                                const double* __restrict__ Ginv, const double* __restrict__ M,
                                                const TF* __restrict__ Src, const DevState* __restrict__ st) {
  if (stopped(st)) return;
  constexpr int TY = NTH / 16;
  constexpr int GI = KP / TY;
  constexpr int GJ = KP / 16;
  constexpr int ZI = LP > 0 ? LP / TY : 1;
  constexpr int LW = KP + 1;
  constexpr int LU = LP + 1;
  // LDS: Ghat (KP x KP) and M (l x KP) as FP64, then the chunk's new rows and
  // (LAI) U rows.  Ghat and M are read with wave-uniform addresses
  // (broadcast); holding them in scalar registers instead would spill.
  extern __shared__ __align__(16) unsigned char smem[];
  double* gs = reinterpret_cast<double*>(smem);
  double* ms = gs + KP * KP;
  TF* wl = reinterpret_cast<TF*>(ms + (LP > 0 ? LP * KP : 0));  // NTH x LW
  TF* us = wl + NTH * LW;                                        // NTH x LU
  __shared__ double sc[8];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int n = a.n, k = a.k, l = a.l;
  TF* __restrict__ Dst = (TF*)a.Dst;
  const double alpha = a.alpha;
  for (int e = tid; e < KP * KP; e += NTH) gs[e] = Gh[e];
  if (LP > 0)
    for (int e = tid; e < l * KP; e += NTH) ms[e] = M[e];
  __syncthreads();

  double gacc[GI][GJ];
  double zacc[ZI][GJ];
#pragma unroll
  for (int i = 0; i < GI; ++i)
#pragma unroll
    for (int j = 0; j < GJ; ++j) gacc[i][j] = 0.0;
#pragma unroll
  for (int i = 0; i < ZI; ++i)
#pragma unroll
    for (int j = 0; j < GJ; ++j) zacc[i][j] = 0.0;
  double dot = 0.0;

  for (int base = blockIdx.x * NTH; base < n; base += gridDim.x * NTH) {
    const int row = base + tid;
    if (LP > 0) {
      // stage the chunk's U rows (coalesced)
      for (int e = tid; e < NTH * l; e += NTH) {
        const int r = e / l, p = e - r * l;
        us[r * LU + p] = (base + r < n) ? (TF)a.U[(int64_t)(base + r) * l + p] : (TF)0;
      }
      __syncthreads();
    }
    if (row < n) {
      const int64_t rb = (int64_t)row * k;
      double y[KP];
#pragma unroll
      for (int i = 0; i < KP; ++i) y[i] = 0.0;
      // Loads are never guarded by a branch (a branch per element makes the
      // compiler wait for each load in turn): padded buffers are read in
      // full, factor rows with a clamped column index and a zero mask.
      if (YMODE == 0) {
        const TP* pr = (const TP*)a.P + (int64_t)row * a.cp;  // cp == KP, zero padded
        const int64_t sstride = (int64_t)n * a.cp;
        for (int sp = 0; sp < a.splits; ++sp) {
#pragma unroll
          for (int i = 0; i < KP; ++i) y[i] += (double)pr[sp * sstride + i];
        }
      } else if (YMODE == 1) {
        const int e1 = a.seg_ptr[row + 1];
        for (int e = a.seg_ptr[row]; e < e1; ++e) {
          const double v = a.seg_val[e];
          const TF* sr = Src + (int64_t)a.seg_src[e] * k;
#pragma unroll
          for (int i = 0; i < KP; ++i) {
            const double x = (double)sr[i < k ? i : k - 1];
            y[i] = fma(v, i < k ? x : 0.0, y[i]);
          }
        }
      } else {
        const TF* u = us + tid * LU;
        for (int p = 0; p < l; ++p) {
          const double up = (double)u[p];
          const double* m = ms + p * KP;  // l x KP, zero padded
#pragma unroll
          for (int i = 0; i < KP; ++i) y[i] = fma(up, m[i], y[i]);
        }
      }
      // HALS target y + alpha src, and the current row
      double w[KP];
      double sv[KP];
#pragma unroll
      for (int i = 0; i < KP; ++i) {
        const int ic = i < k ? i : k - 1;
        const double xs = (double)Src[rb + ic];
        const double xd = (double)Dst[rb + ic];
        sv[i] = i < k ? xs : 0.0;
        w[i] = i < k ? xd : 0.0;
        y[i] = fma(alpha, sv[i], y[i]);
      }
      // Regularised HALS sweep over the KP columns in order.  Padded columns
      // have Ghat = identity, zero target and zero start, so they stay zero.
#pragma unroll
      for (int i = 0; i < KP; ++i) {
        const double* g = gs + i * KP;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
        for (int q = 0; q < KP; q += 4) {
          s0 = fma(w[q], g[q], s0);
          s1 = fma(w[q + 1], g[q + 1], s1);
          s2 = fma(w[q + 2], g[q + 2], s2);
          s3 = fma(w[q + 3], g[q + 3], s3);
        }
        const double sum = (s0 + s1) + (s2 + s3);
        w[i] = fmax(0.0, fma(y[i] - sum, Ginv[i], w[i]));
      }
#pragma unroll
      for (int i = 0; i < KP; ++i) {
        const TF wt = (TF)w[i];
        // product part of the target: y - alpha src (zero on padded columns)
        dot = fma((double)wt, fma(-alpha, sv[i], y[i]), dot);
        wl[tid * LW + i] = wt;
      }
#pragma unroll
      for (int i = 0; i < KP; ++i) {
        if (i < k) {
          Dst[rb + i] = wl[tid * LW + i];
          if (a.Dt) ((TT*)a.Dt)[(int64_t)i * a.ldt + row] = (TT)wl[tid * LW + i];
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < KP; ++i) wl[tid * LW + i] = (TF)0;
    }
    __syncthreads();
    // block partial of F^T F over this chunk
#pragma unroll 4
    for (int r = 0; r < NTH; ++r) {
      double bv[GJ];
#pragma unroll
      for (int j = 0; j < GJ; ++j) bv[j] = (double)wl[r * LW + tx + 16 * j];
#pragma unroll
      for (int i = 0; i < GI; ++i) {
        const double av = (double)wl[r * LW + ty + TY * i];
#pragma unroll
        for (int j = 0; j < GJ; ++j) gacc[i][j] = fma(av, bv[j], gacc[i][j]);
      }
    }
    // block partial of U^T F (LAI: the next half-step's M)
    if (LP > 0) {
#pragma unroll 4
      for (int r = 0; r < NTH; ++r) {
        double bv[GJ];
#pragma unroll
        for (int j = 0; j < GJ; ++j) bv[j] = (double)wl[r * LW + tx + 16 * j];
#pragma unroll
        for (int i = 0; i < ZI; ++i) {
          const double uv = (double)us[r * LU + ty + TY * i];
#pragma unroll
          for (int j = 0; j < GJ; ++j) zacc[i][j] = fma(uv, bv[j], zacc[i][j]);
        }
      }
    }
    __syncthreads();
  }
  double* gp = a.gpart + (int64_t)blockIdx.x * k * k;
#pragma unroll
  for (int i = 0; i < GI; ++i)
#pragma unroll
    for (int j = 0; j < GJ; ++j) {
      const int p = ty + TY * i, q = tx + 16 * j;
      if (p < k && q < k) gp[p * k + q] = gacc[i][j];
    }
  if (LP > 0) {
    double* zp = a.zpart + (int64_t)blockIdx.x * l * k;
#pragma unroll
    for (int i = 0; i < ZI; ++i)
#pragma unroll
      for (int j = 0; j < GJ; ++j) {
        const int p = ty + TY * i, q = tx + 16 * j;
        if (p < l && q < k) zp[p * k + q] = zacc[i][j];
      }
  }
  if (a.dpart) {
    const double t = block_sum(dot, sc);
    if (tid == 0) a.dpart[blockIdx.x] = t;
  }
}

// Fixed-order reduction of the block partials: G (k x k), Ghat = G + alpha I
// (k x k part of the kp x kp padded matrix; the padding is set once), the
// reciprocals of its diagonal, and, when zpart is given, M = diag(lam) Z with
// Z (l x k) the reduced U^T F.
__device__ __forceinline__ double sum_strided(const double* __restrict__ p, int nb, int64_t stride) {
  double acc = 0.0;
  int b = 0;
  for (; b + 8 <= nb; b += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = p[(int64_t)(b + u) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u];
  }
  for (; b < nb; ++b) acc += p[(int64_t)b * stride];
  return acc;
}

__global__ __launch_bounds__(256) void k_update_reduce(const double* __restrict__ gpart,
                                                       const double* __restrict__ zpart, int nb, int k, int l, int kp,
                                                       double alpha, const double* __restrict__ lam,
                                                       double* __restrict__ G, double* __restrict__ Ghat,
                                                       double* __restrict__ Ginv, double* __restrict__ M,
                                                       const DevState* __restrict__ st) {
  if (stopped(st)) return;
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int kk = k * k;
  if (e < kk) {
    const double acc = sum_strided(gpart + e, nb, kk);
    const int p = e / k, q = e - p * k;
    if (G) G[e] = acc;
    if (Ghat) Ghat[p * kp + q] = acc + (p == q ? alpha : 0.0);
    if (Ginv && p == q) Ginv[p] = 1.0 / (acc + alpha);
  } else if (zpart && e < kk + l * k) {
    const int f = e - kk;
    const int p = f / k, q = f - p * k;
    M[p * kp + q] = lam[p] * sum_strided(zpart + f, nb, (int64_t)l * k);  // l x kp, padding stays 0
  }
}

__global__ __launch_bounds__(256) void k_scale_rows(const double* __restrict__ Z, const double* __restrict__ lam,
                                                    int l, int k, int kp, double* __restrict__ M) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= l * kp) return;
  const int p = e / kp, q = e - p * kp;
  M[e] = q < k ? lam[p] * Z[p * k + q] : 0.0;
}

__global__ __launch_bounds__(256) void k_pad_identity(double* __restrict__ Ghat, double* __restrict__ Ginv, int k,
                                                      int kp) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= kp * kp) return;
  const int p = e / kp, q = e - p * kp;
  if (p >= k || q >= k) Ghat[e] = (p == q) ? 1.0 : 0.0;
  if (Ginv && e < kp && e >= k) Ginv[e] = 1.0;
}

template <int KP, int LP, typename TF>
constexpr size_t update_lds(int nth) {
  return 8 * (size_t)KP * (KP + LP) + sizeof(TF) * (size_t)nth * ((KP + 1) + (LP > 0 ? LP + 1 : 0));
}

template <int KP, int LP, typename TF, typename TP, typename TT, int YMODE>
int launch_update(const UpdateArgs& a, const UpdateRO& ro, int nb, const DevState* st, hipStream_t s) {
  // 128 threads (rows) per block for FP32 factors unless the LDS footprint
  // would exceed the 160 KB of a CU; 64 for FP64 factors.
  constexpr int NTH = (sizeof(TF) == 8 || update_lds<KP, LP, TF>(128) > 160 * 1024) ? 64 : 128;
  const size_t lds = update_lds<KP, LP, TF>(NTH);
  auto kern = k_update<KP, LP, TF, TP, TT, YMODE, NTH>;
  if (lds > 65536 &&
      hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return -1;
  // exactly nb blocks (the reduction reads nb partials); rows beyond
  // nb * NTH are covered by the grid-stride loop
  kern<<<nb, NTH, lds, s>>>(a, ro.Ghat, ro.Ginv, ro.M, (const TF*)a.Src, st);
  return 0;
}

template <int KP, typename TF, typename TP, typename TT>
int dispatch_lp(const UpdateArgs& a, const UpdateRO& ro, int ymode, int nb, const DevState* st, hipStream_t s) {
  if (ymode == 0) return launch_update<KP, 0, TF, TP, TT, 0>(a, ro, nb, st, s);
  if (ymode == 1) return launch_update<KP, 0, TF, TP, TT, 1>(a, ro, nb, st, s);
  const int lp = 16 * ceil_div(a.l, 16);
  switch (lp) {
    case 16: return launch_update<KP, 16, TF, TP, TT, 2>(a, ro, nb, st, s);
    case 32: return launch_update<KP, 32, TF, TP, TT, 2>(a, ro, nb, st, s);
    case 48: return launch_update<KP, 48, TF, TP, TT, 2>(a, ro, nb, st, s);
    case 64: return launch_update<KP, 64, TF, TP, TT, 2>(a, ro, nb, st, s);
    case 80: return launch_update<KP, 80, TF, TP, TT, 2>(a, ro, nb, st, s);
    case 96: return launch_update<KP, 96, TF, TP, TT, 2>(a, ro, nb, st, s);
    default: return -1;
  }
}

template <typename TF, typename TP, typename TT>
int dispatch_kp(const UpdateArgs& a, const UpdateRO& ro, int kp, int ymode, int nb, const DevState* st,
                hipStream_t s) {
  switch (kp) {
    case 16: return dispatch_lp<16, TF, TP, TT>(a, ro, ymode, nb, st, s);
    case 32: return dispatch_lp<32, TF, TP, TT>(a, ro, ymode, nb, st, s);
    case 48: return dispatch_lp<48, TF, TP, TT>(a, ro, ymode, nb, st, s);
    case 64: return dispatch_lp<64, TF, TP, TT>(a, ro, ymode, nb, st, s);
    default: return -1;
  }
}

}  // namespace

int update_blocks(int n, int fdtype) {
  const int nth = fdtype == SYMNMF_F64 ? 64 : 128;
  return std::max(1, std::min(1024, ceil_div(n, nth)));
}

int fused_update(const UpdateArgs& a, const UpdateRO& ro, int kp, int ymode, int fdtype, int pdtype, int tdtype,
                 int nb, const DevState* st, hipStream_t s) {
  int rc;
  if (fdtype == SYMNMF_F64) {
    if (pdtype != SYMNMF_F64) return -1;
    rc = dispatch_kp<double, double, double>(a, ro, kp, ymode, nb, st, s);
  } else if (pdtype == SYMNMF_F32) {
    if (tdtype == SYMNMF_BF16) rc = dispatch_kp<float, float, __bf16>(a, ro, kp, ymode, nb, st, s);
    else rc = dispatch_kp<float, float, float>(a, ro, kp, ymode, nb, st, s);
  } else {
    return -1;
  }
  if (rc) return rc;
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int update_reduce(const double* gpart, const double* zpart, int nb, int k, int l, int kp, double alpha,
                  const double* lam, double* G, double* Ghat, double* Ginv, double* M, const DevState* st,
                  hipStream_t s) {
  const int E = k * k + (zpart ? l * k : 0);
  k_update_reduce<<<ceil_div(E, 256), 256, 0, s>>>(gpart, zpart, nb, k, l, kp, alpha, lam, G, Ghat, Ginv, M, st);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int scale_rows(const double* Z, const double* lam, int l, int k, int kp, double* M, hipStream_t s) {
  k_scale_rows<<<ceil_div(l * kp, 256), 256, 0, s>>>(Z, lam, l, k, kp, M);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int pad_identity(double* Ghat, double* Ginv, int k, int kp, hipStream_t s) {
  k_pad_identity<<<ceil_div(kp * kp, 256), 256, 0, s>>>(Ghat, Ginv, k, kp);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
