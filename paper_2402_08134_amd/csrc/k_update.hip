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
//   YMODE 1  y_j = sum_e v_e F[src_e]     sampled slab (LvS): the stored
//            X[j][r] w_r of row j with r in the sample, in column order
//   YMODE 2  y_j = U[j,:] M,  M = Lambda U^T F   (LAI)
// and the HALS target is y_j + alpha F[j].
#include "kernels.hpp"

#include <type_traits>

namespace {

// Rows per block chunk: 32 rows x 16 lanes = 512 threads (measured on
// MI355X at n = 16384: a LAI iteration 68 us with 16-row, 256-thread blocks,
// 62 us with 32, 67 us with 64; the same 512 blocks in each case).
constexpr int UPD_RPB = 32;

// Column held in slot c by lane g of a row: with 16 lanes per row the
// columns interleave (g + 16 c); with LPR = 2, 4 or 8 lanes each lane holds
// runs of 4 adjacent columns (4 LPR (c / 4) + 4 g + c mod 4), so the lanes of
// a row read 4 LPR adjacent values per step.
template <int LPR>
__device__ __forceinline__ constexpr int col_of(int g, int c) {
  return LPR == 16 ? g + 16 * c : 4 * LPR * (c >> 2) + 4 * g + (c & 3);
}
// Slot and owning lane of column i.
template <int LPR>
__device__ __forceinline__ constexpr int slot_of(int i) {
  return LPR == 16 ? i >> 4 : 4 * (i / (4 * LPR)) + (i & 3);
}
template <int LPR>
__device__ __forceinline__ constexpr int owner_of(int i) {
  return LPR == 16 ? i & 15 : (i >> 2) % LPR;
}
// Sum over the LPR lanes of a row (contiguous lanes of a DPP row): pairs,
// quads, halves (row_half_mirror), full row (row_mirror) as needed.
template <int LPR>
__device__ __forceinline__ double lanes_sum(double v) {
  v += dpp_double<0xB1>(v);
  if (LPR >= 4) v += dpp_double<0x4E>(v);
  if (LPR >= 8) v += dpp_double<0x141>(v);
  if (LPR >= 16) v += dpp_double<0x140>(v);
  return v;
}

// Waves per SIMD the register allocation must leave room for: the long-factor
// update without a LAI term (KP = 64) otherwise takes more than 128 VGPRs and
// runs one 512-thread block per CU.
template <int KP, int LP, int LPR>
constexpr int upd_waves() { return KP == 64 && LP == 0 ? (LPR >= 8 ? 4 : 2) : 1; }

// LPR lanes per row (16, or 8 for long factors with KP a multiple of 32:
// three DPP steps per column sum instead of four and half as many lanes per
// row), 512 threads per block.  Lane g of a row owns the KP / LPR columns
// col_of(g, c).  The HALS sweep over column i sums w_q Ghat[i][q] over the
// row's lanes and the lane owning column i applies the update.
template <int KP, int LP, typename TF, typename TP, typename TT, int YMODE, int LPR>
__global__ __launch_bounds__(16 * UPD_RPB) __attribute__((amdgpu_waves_per_eu(upd_waves<KP, LP, LPR>())))
void k_update(UpdateArgs a, const double* __restrict__ Gh,
                                                const double* __restrict__ Ginv, const double* __restrict__ M,
                                                const TF* __restrict__ Src, const DevState* __restrict__ st) {
  if (stopped(st)) return;
  constexpr int NTH = 16 * UPD_RPB, RPB = NTH / LPR;
  constexpr int CPL = KP / LPR;   // HALS columns per lane
  constexpr int TCPL = KP / 16;   // entries per thread of the 16 x 16 partial tile
  constexpr int ZI = LP > 0 ? LP / 16 : 1;
  constexpr int LW = KP + 1;
  constexpr int LU = LP + 1;
  extern __shared__ __align__(16) unsigned char smem[];
  double* gs = reinterpret_cast<double*>(smem);          // KP x KP
  double* gi = gs + KP * KP;                              // KP
  double* ms = gi + KP;                                   // l x KP (LAI)
  TF* wl = reinterpret_cast<TF*>(ms + (LP > 0 ? LP * KP : 0));  // RPB x LW
  TF* us = wl + RPB * LW;                                         // RPB x LU (LAI)
  // LAI right-hand sides of the chunk (RPB x LW doubles, 8-byte aligned)
  double* ys = reinterpret_cast<double*>(
      (reinterpret_cast<uintptr_t>(us + (LP > 0 ? RPB * LU : 0)) + 7) & ~(uintptr_t)7);
  __shared__ double sc[8];
  const int tid = threadIdx.x;
  const int g = tid % LPR, rs = tid / LPR;     // lane in row, row slot
  // Gram / U^T F tile: two 16 x 16 tiles of threads, each over half of the
  // chunk's rows, added together at the end
  const int th = tid >> 8, tx = tid & 15, ty = (tid & 255) >> 4;
  const int n = a.n, k = a.k, l = a.l;
  TF* __restrict__ Dst = (TF*)a.Dst;
  const double alpha = a.alpha;
  // LAI with KP <= 32: this thread's share of a chunk's U rows, held in
  // registers; the first chunk's loads are issued with the staging loads
  // below and each next chunk's while the current one is processed.  Clamped
  // index, masked value: every load stays inside U.  The factor rows of the
  // HALS target are likewise loaded before the right-hand side (EARLY).  At
  // KP = 64 with a LAI term the extra live registers made the kernel slower
  // (127 -> 155 us at n = 65536, l = 80), so there the loads stay where they
  // are used.
  constexpr bool UREG = LP > 0 && KP <= 32;
  constexpr bool EARLY = LP == 0 || KP <= 32;
  constexpr int UPT = UREG ? (RPB * LP + NTH - 1) / NTH : 1;
  const TF* __restrict__ Ut = (const TF*)a.U;  // U in the factor type
  TF ureg[UPT];
  auto load_u = [&](int b) {
#pragma unroll
    for (int t = 0; t < UPT; ++t) {
      const int e = tid + t * NTH, r = e / l, p = e - r * l;
      const bool ok = e < RPB * l && b + r < n;
      const TF v = Ut[ok ? (int64_t)(b + r) * l + p : 0];
      ureg[t] = ok ? v : (TF)0;
    }
  };
  // this row's old factor and the source of the alpha term (EARLY): with U
  // in registers the first chunk's are issued here, before the staging
  // loads, so their latency overlaps the staging and U M
  TF xs_r[CPL], xd_r[CPL];
  auto load_rows = [&](int b) {
    const int64_t rb = (int64_t)min(b + rs, n - 1) * k;
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const int q = col_of<LPR>(g, c);
      const int qc = q < k ? q : k - 1;
      xs_r[c] = Src[rb + qc];
      xd_r[c] = Dst[rb + qc];
    }
  };
  if (UREG) load_rows(blockIdx.x * RPB);
  if (UREG && l > 0) load_u(blockIdx.x * RPB);
  for (int e = tid; e < KP * KP; e += NTH) gs[e] = Gh[e];
  for (int e = tid; e < KP; e += NTH) gi[e] = Ginv[e];
  if (LP > 0)
    for (int e = tid; e < l * KP; e += NTH) ms[e] = M[e];
  __syncthreads();

  // Without a LAI term at KP = 64 the Gram partial runs on the FP64 matrix
  // cores: wave w accumulates the 16 x 16 tiles (w / 2, 2 (w % 2)) and
  // (w / 2, 2 (w % 2) + 1) of F^T F, four chunk rows per instruction.
  constexpr bool GMF = LP == 0 && KP == 64;
  // With a LAI term both partials run there: with KT = KP / 16 tiles per
  // row, tile t (t < NGT = KT^2) is F^T F tile (t / KT, t % KT) and tile
  // NGT + z is U^T F tile (z / KT, z % KT); wave w takes tiles w, w + 8, ...
  // Only at KP = 32: at KP = 64 (five tiles per wave) the LAI iteration at
  // n = 65536, l = 80 measured 289 -> 335 us, so there the VALU tile stays.
  constexpr bool GMZ = LP > 0 && KP == 32;
  // With a LAI term at KP = 32 the right-hand sides U[j,:] M of the chunk are
  // one (RPB x LP) x (LP x KP) product on the FP64 matrix cores: wave w takes
  // the 16 x 16 output tiles w, w + 8, ... (row tile t / KT, column tile
  // t % KT), LP / 4 steps each, and leaves them in LDS for the sweep.
  constexpr bool UMF = GMZ && YMODE == 2;
  constexpr int UMT = (RPB / 16) * (KP / 16);
  constexpr int KT = KP / 16, NGT = KT * KT, NTT = NGT + (LP / 16) * KT;
  constexpr int TPW = GMZ ? (NTT + 7) / 8 : 2;
  doublex4 gm[TPW > 2 ? TPW : 2];
#pragma unroll
  for (int h = 0; h < (TPW > 2 ? TPW : 2); ++h) gm[h] = doublex4{0.0, 0.0, 0.0, 0.0};
  double gacc[TCPL][TCPL];
  double zacc[ZI][TCPL];
#pragma unroll
  for (int i = 0; i < TCPL; ++i)
#pragma unroll
    for (int j = 0; j < TCPL; ++j) gacc[i][j] = 0.0;
#pragma unroll
  for (int i = 0; i < ZI; ++i)
#pragma unroll
    for (int j = 0; j < TCPL; ++j) zacc[i][j] = 0.0;
  double dot = 0.0;

  for (int base = blockIdx.x * RPB; base < n; base += gridDim.x * RPB) {
    const int row = base + rs;
    if (LP > 0) {
      if (UREG) {
#pragma unroll
        for (int t = 0; t < UPT; ++t) {
          const int e = tid + t * NTH;
          if (e < RPB * l) {
            const int r = e / l, p = e - r * l;
            us[r * LU + p] = ureg[t];
          }
        }
      } else {
        for (int e = tid; e < RPB * l; e += NTH) {
          const int r = e / l, p = e - r * l;
          us[r * LU + p] = (base + r < n) ? Ut[(int64_t)(base + r) * l + p] : (TF)0;
        }
      }
      __syncthreads();
      if (UREG && l > 0 && base + gridDim.x * RPB < n) load_u(base + gridDim.x * RPB);
      if (UMF) {
        const int wid = tid >> 6, li = tid & 15, lg = (tid & 63) >> 4;
        for (int t = wid; t < UMT; t += NTH / 64) {   // the same for the whole wave
          const int r0 = 16 * (t / KT), c0 = 16 * (t % KT);
          doublex4 acc = doublex4{0.0, 0.0, 0.0, 0.0};
          for (int s4 = 0; s4 < l; s4 += 4) {
            // A[i][p] = U[r0 + i][s4 + p], B[p][j] = M[s4 + p][c0 + j]; lane
            // (li, lg) supplies A[li][lg] and B[lg][li]; p beyond l reads
            // the zero padding of M
            const int pa = s4 + lg < LP ? s4 + lg : LP - 1;
            const double av = s4 + lg < l ? (double)us[(r0 + li) * LU + pa] : 0.0;
            const double bv = s4 + lg < l ? ms[(s4 + lg) * KP + c0 + li] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
          }
          // accumulator element v of lane (li, lg): row lg + 4 v, column li
#pragma unroll
          for (int v = 0; v < 4; ++v) ys[(r0 + lg + 4 * v) * LW + c0 + li] = acc[v];
        }
        __syncthreads();
      }
    }
    if (row < n) {
      const int64_t rb = (int64_t)row * k;
      double y[CPL], w[CPL];
      // otherwise issued here, before the right-hand side, so their latency
      // overlaps it
      if (EARLY && !(UREG && base == blockIdx.x * RPB)) load_rows(base);
#pragma unroll
      for (int c = 0; c < CPL; ++c) y[c] = 0.0;
      // Loads are never guarded by a branch (a branch per element makes the
      // compiler wait for each load in turn): padded buffers are read in
      // full, factor rows with a clamped column index and a zero mask.
      if (YMODE == 0) {
        const TP* pr = (const TP*)a.P + (int64_t)row * a.cp;  // cp == KP, zero padded
        const int64_t sstride = (int64_t)n * a.cp;
        for (int sp = 0; sp < a.splits; ++sp) {
#pragma unroll
          for (int c = 0; c < CPL; ++c) y[c] += (double)pr[sp * sstride + col_of<LPR>(g, c)];
        }
      } else if (YMODE == 1) {
        const int e1 = a.seg_ptr[row + 1];
        for (int e = a.seg_ptr[row]; e < e1; ++e) {
          const double v = a.seg_val[e];
          const TF* sr = Src + (int64_t)a.seg_src[e] * k;
#pragma unroll
          for (int c = 0; c < CPL; ++c) {
            const int q = col_of<LPR>(g, c);
            const double x = (double)sr[q < k ? q : k - 1];
            y[c] = fma(v, q < k ? x : 0.0, y[c]);
          }
        }
      } else if (UMF) {
#pragma unroll
        for (int c = 0; c < CPL; ++c) y[c] = ys[rs * LW + col_of<LPR>(g, c)];
      } else {
        const TF* u = us + rs * LU;
        for (int p = 0; p < l; ++p) {
          const double up = (double)u[p];
#pragma unroll
          for (int c = 0; c < CPL; ++c) y[c] = fma(up, ms[p * KP + col_of<LPR>(g, c)], y[c]);
        }
      }
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        const int q = col_of<LPR>(g, c);
        const int qc = q < k ? q : k - 1;
        const double xs = EARLY ? (double)xs_r[c] : (double)Src[rb + qc];
        const double xd = EARLY ? (double)xd_r[c] : (double)Dst[rb + qc];
        w[c] = q < k ? xd : 0.0;
        y[c] = fma(alpha, q < k ? xs : 0.0, y[c]);   // HALS target y + alpha src
      }
      if (a.rule == 1) {
#pragma unroll
        for (int c = 0; c < CPL; ++c) a.Yhat[(int64_t)row * KP + col_of<LPR>(g, c)] = y[c];
      } else if (a.rule == 2) {
#pragma unroll
        for (int c = 0; c < CPL; ++c) w[c] = a.Yhat[(int64_t)row * KP + col_of<LPR>(g, c)];
      } else {
        // Regularised HALS sweep over the KP columns in order.  Padded columns
        // have Ghat = identity, zero target and zero start, so they stay zero.
#pragma unroll
        for (int i = 0; i < KP; ++i) {
          // slot changed by column i - 1 goes last: the other terms of the
          // dot product do not wait for that column's result
          const int cp = i == 0 ? -1 : slot_of<LPR>(i - 1);
          double part = 0.0;
#pragma unroll
          for (int c = 0; c < CPL; ++c)
            if (c != cp) part = fma(w[c], gs[i * KP + col_of<LPR>(g, c)], part);
          if (cp >= 0) part = fma(w[cp], gs[i * KP + col_of<LPR>(g, cp)], part);
          part = lanes_sum<LPR>(part);
          // slot and owning lane of column i
          const int ci = slot_of<LPR>(i);
          const int own = owner_of<LPR>(i);
          const double cand = fmax(0.0, fma(y[ci] - part, gi[i], w[ci]));
          w[ci] = (g == own) ? cand : w[ci];
        }
      }
      if (a.rule != 1) {
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
          const int q = col_of<LPR>(g, c);
          const TF wt = (TF)w[c];
          if (a.dpart) {  // product part of the target (src reloaded: fewer live registers)
            const double xs = q < k ? (double)Src[rb + (q < k ? q : k - 1)] : 0.0;
            dot = fma((double)wt, fma(-alpha, xs, y[c]), dot);
          }
          wl[rs * LW + q] = wt;
          if (q < k) {
            Dst[rb + q] = wt;
            if (a.Dt) {
              if (a.dt_rows) ((TT*)a.Dt)[(int64_t)row * a.ldt + q] = (TT)wt;
              else ((TT*)a.Dt)[(int64_t)q * a.ldt + row] = (TT)wt;
            }
          }
        }
      }
    } else {
#pragma unroll
      for (int c = 0; c < CPL; ++c) wl[rs * LW + col_of<LPR>(g, c)] = (TF)0;
    }
    __syncthreads();
    // block partials of F^T F and (LAI) U^T F over this chunk (none when
    // only the right-hand side is written)
    if (GMZ && a.rule != 1) {
      const int wid = tid >> 6, li = tid & 15, lg = (tid & 63) >> 4;
#pragma unroll
      for (int h = 0; h < TPW; ++h) {
        const int t = wid + 8 * h;
        if (t < NTT) {   // the same for the whole wave
          const bool zt = t >= NGT;
          const int tt = zt ? t - NGT : t;
          const int ca = 16 * (tt / KT) + li, cb = 16 * (tt % KT) + li;
#pragma unroll 4
          for (int s4 = 0; s4 < RPB / 4; ++s4) {
            const int r = 4 * s4 + lg;
            const double av = zt ? (double)us[r * LU + ca] : (double)wl[r * LW + ca];
            gm[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, (double)wl[r * LW + cb], gm[h], 0, 0, 0);
          }
        }
      }
    } else if (GMF && a.rule != 1) {
      // lane l supplies A[l % 16][l / 16] = F[r0 + l / 16][16 (w / 2) + l % 16]
      // and B[l / 16][l % 16] = F[r0 + l / 16][16 tb + l % 16]
      const int wid = tid >> 6, li = tid & 15, lg = (tid & 63) >> 4;
      const int ca = 16 * (wid >> 1) + li, cb = 32 * (wid & 1) + li;
#pragma unroll 4
      for (int s4 = 0; s4 < RPB / 4; ++s4) {
        const TF* wr = wl + (4 * s4 + lg) * LW;
        const double av = (double)wr[ca];
        gm[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, (double)wr[cb], gm[0], 0, 0, 0);
        gm[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, (double)wr[cb + 16], gm[1], 0, 0, 0);
      }
    } else if (a.rule != 1) {
#pragma unroll 4
      for (int rr = 0; rr < RPB / 2; ++rr) {
        const int r = th * (RPB / 2) + rr;
        double bv[TCPL];
#pragma unroll
        for (int j = 0; j < TCPL; ++j) bv[j] = (double)wl[r * LW + tx + 16 * j];
#pragma unroll
        for (int i = 0; i < TCPL; ++i) {
          const double av = (double)wl[r * LW + ty + 16 * i];
#pragma unroll
          for (int j = 0; j < TCPL; ++j) gacc[i][j] = fma(av, bv[j], gacc[i][j]);
        }
        if (LP > 0) {
#pragma unroll
          for (int i = 0; i < ZI; ++i) {
            const double uv = (double)us[r * LU + ty + 16 * i];
#pragma unroll
            for (int j = 0; j < TCPL; ++j) zacc[i][j] = fma(uv, bv[j], zacc[i][j]);
          }
        }
      }
    }
    __syncthreads();
  }
  if (a.rule == 1) return;
  // the second tile's sums onto the first's, through the staging area (free
  // now: it holds at least KP (KP + LP) doubles, the size of both tiles)
  if (!GMF && !GMZ) {
    double* cmb = reinterpret_cast<double*>(smem);
    const int t8 = tid & 255;
    if (th == 1) {
#pragma unroll
      for (int i = 0; i < TCPL; ++i)
#pragma unroll
        for (int j = 0; j < TCPL; ++j) cmb[(i * TCPL + j) * 256 + t8] = gacc[i][j];
      if (LP > 0) {
#pragma unroll
        for (int i = 0; i < ZI; ++i)
#pragma unroll
          for (int j = 0; j < TCPL; ++j) cmb[(TCPL * TCPL + i * TCPL + j) * 256 + t8] = zacc[i][j];
      }
    }
    __syncthreads();
    if (th == 0) {
#pragma unroll
      for (int i = 0; i < TCPL; ++i)
#pragma unroll
        for (int j = 0; j < TCPL; ++j) gacc[i][j] += cmb[(i * TCPL + j) * 256 + t8];
      if (LP > 0) {
#pragma unroll
        for (int i = 0; i < ZI; ++i)
#pragma unroll
          for (int j = 0; j < TCPL; ++j) zacc[i][j] += cmb[(TCPL * TCPL + i * TCPL + j) * 256 + t8];
      }
    }
  }
  // unified partial row of this block: [F^T F (k x k) | U^T F (l x k)]
  double* gp = a.part + (int64_t)blockIdx.x * a.pstride;
  if (GMF) {
    // accumulator element v of lane l: row l / 16 + 4 v, column l % 16
    const int wid = tid >> 6, li = tid & 15, lg = (tid & 63) >> 4;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int p = 16 * (wid >> 1) + lg + 4 * v, q = 32 * (wid & 1) + 16 * h + li;
        if (p < k && q < k) gp[p * k + q] = gm[h][v];
      }
  } else if (GMZ) {
    const int wid = tid >> 6, li = tid & 15, lg = (tid & 63) >> 4;
#pragma unroll
    for (int h = 0; h < TPW; ++h) {
      const int t = wid + 8 * h;
      if (t < NTT) {
        const bool zt = t >= NGT;
        const int tt = zt ? t - NGT : t;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int p = 16 * (tt / KT) + lg + 4 * v, q = 16 * (tt % KT) + li;
          if (!zt && p < k && q < k) gp[p * k + q] = gm[h][v];
          if (zt && p < l && q < k) gp[k * k + p * k + q] = gm[h][v];
        }
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < TCPL; ++i)
#pragma unroll
      for (int j = 0; j < TCPL; ++j) {
        const int p = ty + 16 * i, q = tx + 16 * j;
        if (tid < 256 && p < k && q < k) gp[p * k + q] = gacc[i][j];
      }
  }
  if (LP > 0 && !GMZ && tid < 256) {
    double* zp = gp + k * k;
#pragma unroll
    for (int i = 0; i < ZI; ++i)
#pragma unroll
      for (int j = 0; j < TCPL; ++j) {
        const int p = ty + 16 * i, q = tx + 16 * j;
        if (p < l && q < k) zp[p * k + q] = zacc[i][j];
      }
  }
  if (a.dpart) {
    const double t = block_sum(dot, sc);
    if (tid == 0) a.dpart[blockIdx.x] = t;
  }
}
// Fixed-order reduction of the block partials (unified rows of E = k*k
// [+ l*k] doubles) in one kernel: G (k x k), Ghat = G + alpha I (k x k part of
// the kp x kp padded matrix; the padding is set once), the reciprocals of its
// diagonal, and, for the LAI path, M = diag(lam) Z (l x kp, zero padded) with
// Z the reduced U^T F.  A block takes 16 entries; its 16 slices of threads
// each sum a contiguous run of partial rows (16 loads in flight), the slice
// sums are added in slice order and the epilogue is applied per entry.  One
// launch instead of a level over groups of 32 rows plus a final level: a LAI
// iteration at n = 16384, k = 32, l = 48 measured 61.9 -> 56.8 us.
constexpr int RED_SLICES = 16, RED_COLS = 16;

__device__ __forceinline__ double sum_rows16(const double* __restrict__ p, int cnt, int64_t stride) {
  double acc = 0.0;
  int b = 0;
  for (; b + 16 <= cnt; b += 16) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = p[(int64_t)(b + u) * stride];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc += v[u];
  }
  for (; b < cnt; ++b) acc += p[(int64_t)b * stride];
  return acc;
}

__global__ __launch_bounds__(RED_SLICES * RED_COLS) void k_update_reduce(
    const double* __restrict__ part, int nb, int E, int k, int l, int kp, double alpha,
    const double* __restrict__ lam, double* __restrict__ G, double* __restrict__ Ghat, double* __restrict__ Ginv,
    double* __restrict__ M, const DevState* __restrict__ st) {
  if (stopped(st)) return;
  __shared__ double ps[RED_SLICES][RED_COLS + 1];
  const int c = threadIdx.x % RED_COLS, sl = threadIdx.x / RED_COLS;
  const int e = blockIdx.x * RED_COLS + c;
  const int per = (nb + RED_SLICES - 1) / RED_SLICES;
  const int b0 = sl * per;
  const int cnt = max(0, min(per, nb - b0));
  ps[sl][c] = e < E ? sum_rows16(part + (int64_t)b0 * E + e, cnt, E) : 0.0;
  __syncthreads();
  if (sl != 0 || e >= E) return;
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < RED_SLICES; ++j) acc += ps[j][c];
  const int kk = k * k;
  if (e < kk) {
    const int p = e / k, q = e - p * k;
    if (G) G[e] = acc;
    if (Ghat) Ghat[p * kp + q] = acc + (p == q ? alpha : 0.0);
    if (Ginv && p == q) Ginv[p] = 1.0 / (acc + alpha);
  } else {
    const int f = e - kk;
    const int p = f / k, q = f - p * k;
    M[p * kp + q] = lam[p] * acc;  // l x kp, padding stays 0
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

// ---------------------------------------------------------------------------
// Blocked HALS sweep for long factors: padded width 64, FP32 factors, no LAI
// term, the HALS rule.  The sweep over the columns (Update of the Appendix)
// is reassociated per block B of 16 columns: the terms of the 48 columns
// outside B, W[:, not B] Ghat[not B, B] with the current values (new before
// B, old after it), are one product on the FP64 matrix cores per 16-row tile,
// and only the 16 x 16 part inside B stays serial.  A lane owns a whole row,
// so that serial part needs no cross-lane sums: 16 FMAs per column instead of
// 64 plus a lane reduction.
//
// A wave owns 64 rows and keeps them in an LDS slab (FP32, the values the
// matrix-core operands read; the row's block values are FP64 in registers
// during the block's sweep).  The product's 16 x 16 tiles come out with a row
// spread over four lanes 16 apart; a 4 x 4 transpose across the wave's four
// 16-lane rows (two lane-half swaps and two row-pair swaps per 32-bit word)
// leaves each lane its own row.  The block's four slabs form a 256-row chunk
// whose Gram partial F^T F the waves share: the 10 tiles on and above the
// diagonal, each mirrored when written.
//
// The earlier blocks' new values enter the later blocks' products as the
// FP32 values the factor stores; at n = 65536, k = 64 the blocked and the
// unblocked sweep agree to 2e-8 (relative).  At n = 2^20, k = 64 (sparse
// graph) the update takes 472 us against 700 us unblocked (LvS 477 against
// 725); about 6700 FP64 FMAs per row, on the FP64 units the matrix and the
// vector instructions share on this chip, put its floor near 180 us.
constexpr int BK_LW = 68;     // slab row stride in floats (16-byte rows, 272 B)
constexpr int BK_ROWS = 256;  // rows per block chunk (4 waves x 64)
constexpr int BK_XR = 13;     // sampled-slab rows whose extra entries a chunk holds in LDS

__device__ __forceinline__ void swap_words(double& x, double& y, bool halves) {
  const unsigned long long ux = (unsigned long long)__double_as_longlong(x);
  const unsigned long long uy = (unsigned long long)__double_as_longlong(y);
  const unsigned xl = (unsigned)ux, xh = (unsigned)(ux >> 32), yl = (unsigned)uy, yh = (unsigned)(uy >> 32);
  unsigned nxl, nyl, nxh, nyh;
  if (halves) {   // lanes 32..63 of x <-> lanes 0..31 of y
    const auto l = __builtin_amdgcn_permlane32_swap(xl, yl, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(xh, yh, false, false);
    nxl = l[0]; nyl = l[1]; nxh = h[0]; nyh = h[1];
  } else {        // odd 16-lane rows of x <-> even 16-lane rows of y
    const auto l = __builtin_amdgcn_permlane16_swap(xl, yl, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(xh, yh, false, false);
    nxl = l[0]; nyl = l[1]; nxh = h[0]; nyh = h[1];
  }
  x = __longlong_as_double((long long)(((unsigned long long)nxh << 32) | nxl));
  y = __longlong_as_double((long long)(((unsigned long long)nyh << 32) | nyl));
}

// e[t] in lane (li, r) holds entry (r, t) of a 4 x 4 matrix per li; after the
// call e[t] in lane (li, r) holds entry (t, r).
__device__ __forceinline__ void transpose4(double (&e)[4]) {
  swap_words(e[0], e[2], true);
  swap_words(e[1], e[3], true);
  swap_words(e[0], e[1], false);
  swap_words(e[2], e[3], false);
}

template <typename TT, int YMODE, bool DOT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void k_update_blk(UpdateArgs a, const double* __restrict__ Gh, const double* __restrict__ Ginv,
                  const float* __restrict__ Src, const DevState* __restrict__ st) {
  if (stopped(st)) return;
  extern __shared__ __align__(16) unsigned char smem[];
  float* slab = reinterpret_cast<float*>(smem);  // BK_ROWS x BK_LW
  // the four diagonal 16 x 16 blocks of Ghat and 1 / diag(Ghat), read by
  // every lane alike (wave-uniform values kept out of scalar registers)
  double* gd = reinterpret_cast<double*>(smem + sizeof(float) * BK_ROWS * BK_LW);
  double* gv = gd + 4 * 256;
  __shared__ double sc[8];
  __shared__ double hx[BK_XR - 8][64];   // held extras' sums beyond the slab's padding (sampled slab)
  __shared__ int wx[4];                   // rows with held extras per wave (sampled slab)
  const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63, li = lane & 15, lg = lane >> 4;
  float* sw = slab + wid * 64 * BK_LW;
  const int n = a.n, k = a.k, k4 = a.k >> 2;   // k a multiple of 4
  const double alpha = a.alpha;
  float* __restrict__ Dst = (float*)a.Dst;
  // padding columns k..63 of the slab stay zero (the sweep writes back zeros there)
  for (int e = tid; e < BK_ROWS * 64; e += 256) {
    const int r = e >> 6, q = e & 63;
    if (q >= k) slab[r * BK_LW + q] = 0.f;
  }
  for (int e = tid; e < 4 * 256; e += 256) {
    const int b = e >> 8, i = (e >> 4) & 15, q = e & 15;
    gd[e] = Gh[(16 * b + i) * 64 + 16 * b + q];
  }
  if (tid < 64) gv[tid] = Ginv[tid];
  __syncthreads();
  // Gram tiles of this wave: tau = wid, wid + 4, wid + 8 of the 10 tiles
  // (I, J), I <= J, numbered row by row
  doublex4 gt[3];
#pragma unroll
  for (int h = 0; h < 3; ++h) gt[h] = doublex4{0.0, 0.0, 0.0, 0.0};
  double dot = 0.0;

  // The row's loads of the next block (the next chunk's first after the last
  // block) are issued during the current block, after its other global
  // loads, so that waiting for those does not wait for these: the
  // alpha-term source, and the product part (YMODE 0 with one partial) or
  // the gathered row of the row's first sampled entry (YMODE 1, within a
  // chunk: the entry is known from the chunk's start).  With more than one
  // partial every block loads its own at its start.
  const bool pre = YMODE == 1 || a.splits == 1;
  float4 pp[4], ps[4];
  auto load_p = [&](int rowq, int bq) {   // product partial 0 of row rowq, or gathered row rowq
    const float* pr = YMODE == 0 ? (const float*)a.P + (int64_t)rowq * a.cp + 16 * bq
                                 : Src + (int64_t)rowq * k;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int q = 16 * bq + 4 * m;
      pp[m] = *reinterpret_cast<const float4*>(YMODE == 0 ? pr + 4 * m : pr + (q < k ? q : k - 4));
    }
  };
  auto load_s = [&](int rowq, int bq) {   // alpha-term source
    const float* sr = Src + (int64_t)rowq * k;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int q = 16 * bq + 4 * m;
      ps[m] = *reinterpret_cast<const float4*>(sr + (q < k ? q : k - 4));
    }
  };
  if (pre && blockIdx.x * BK_ROWS < n) {
    const int r = min(blockIdx.x * BK_ROWS + 64 * wid + lane, n - 1);
    if (YMODE == 0) load_p(r, 0);
    load_s(r, 0);
  }

  for (int base = blockIdx.x * BK_ROWS; base < n; base += gridDim.x * BK_ROWS) {
    const int r0 = base + 64 * wid;
    const int row = r0 + lane;
    const bool live = row < n;
    const int rowc = live ? row : n - 1;
    const int nbase = base + gridDim.x * BK_ROWS;   // the next chunk, if any
    // YMODE 1: the row's segment of the sampled slab, and its first entry.
    // Rows with more entries (a few per cent, but in most waves, and a few
    // rows with tens of entries once the scores concentrate) have the sum
    // of their later entries ("extras") formed once per chunk: the chunk's
    // first BK_XR such rows, numbered in row order, each by a 16-lane group
    // of the wave that owns it (4 columns per lane, FP64, the entries in
    // segment order), kept in LDS as 64 doubles -- slot p < 8 in the slab's
    // unused columns 64..67 of rows 32 p .. 32 p + 31, the rest in hx -- and
    // each block the owning lane adds its block's 16 values.  Read per
    // block, the extras were chains of dependent global reads, and the block
    // with the most of them set the kernel's time (n = 2^20, k = 64: 596 us;
    // 477 us held).
    int e0 = 0, e1 = 0, s0 = rowc;
    double v0 = 0.0;
    int xq = BK_XR;   // the row's slot (< BK_XR when its extras are held)
    if (YMODE == 1) {
      e0 = live ? a.seg_ptr[row] : 0;
      e1 = live ? a.seg_ptr[row + 1] : 0;
      if (e0 < e1) {
        v0 = a.seg_val[e0];
        s0 = a.seg_src[e0];
      }
      const bool xr = e1 - e0 > 1;
      const uint64_t bm = __ballot(xr);
      const int inc = __popcll(bm & ((2ull << lane) - 1ull));   // inclusive rank among the wave's such rows
      if (lane == 0) wx[wid] = __popcll(bm);
      __syncthreads();
      int before = 0;   // such rows of the lower waves
#pragma unroll
      for (int u = 0; u < 3; ++u) before += u < wid ? wx[u] : 0;
      if (xr && before + inc - 1 < BK_XR) xq = before + inc - 1;
      // group lg sums wave-local such row t = 4 r + lg, the row of the first
      // lane whose inclusive rank exceeds t
      const int nh = min(__popcll(bm), BK_XR - before);
      for (int r = 0; 4 * r < nh; ++r) {
        int own = 0;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int o = __popcll(__ballot(inc <= 4 * r + g));
          own = lg == g ? o : own;
        }
        const int t = 4 * r + lg;
        const int f0 = __shfl(e0, own & 63) + 1, f1 = __shfl(e1, own & 63);
        if (t < nh) {
          const int q = 4 * li, qc = q < k ? q : k - 4;
          double z[4] = {0.0, 0.0, 0.0, 0.0};
          for (int e = f0; e < f1; e += 4) {   // four entries' loads in flight at once
            double vu[4];
            float4 xu[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int eu = min(e + u, f1 - 1);
              vu[u] = e + u < f1 ? a.seg_val[eu] : 0.0;
              xu[u] = *reinterpret_cast<const float4*>(Src + (int64_t)a.seg_src[eu] * k + qc);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              z[0] = fma(vu[u], (double)xu[u].x, z[0]);
              z[1] = fma(vu[u], (double)xu[u].y, z[1]);
              z[2] = fma(vu[u], (double)xu[u].z, z[2]);
              z[3] = fma(vu[u], (double)xu[u].w, z[3]);
            }
          }
          if (q >= k) z[0] = z[1] = z[2] = z[3] = 0.0;
          const int p = before + t;
          double* d0 = p < 8 ? reinterpret_cast<double*>(slab + (32 * p + 2 * li) * BK_LW + 64) : &hx[p - 8][4 * li];
          double* d1 = p < 8 ? reinterpret_cast<double*>(slab + (32 * p + 2 * li + 1) * BK_LW + 64) : &hx[p - 8][4 * li + 2];
          *reinterpret_cast<double2*>(d0) = make_double2(z[0], z[1]);
          *reinterpret_cast<double2*>(d1) = make_double2(z[2], z[3]);
        }
      }
    }
    // old factor rows of the wave -> slab; the 64 rows are contiguous (64 k
    // floats), read as float4 with a clamped index and a zero mask
    {
      const float4* s4 = reinterpret_cast<const float4*>(Dst + (int64_t)min(r0, n - 1) * k);
      const int tot = 64 * k4, lim = (n - r0) * k4;
      for (int e = lane; e < tot; e += 64) {
        const int rr = e / k4, c4 = e - rr * k4;
        const float4 v = s4[e < lim ? e : 0];
        *reinterpret_cast<float4*>(sw + rr * BK_LW + 4 * c4) = e < lim ? v : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
    if (YMODE == 1)
      __syncthreads();   // the held extras are read across the waves
    else
      wave_sync();
    // the block loop stays rolled: unrolled, the compiler hoists the LDS reads
    // of all four blocks and spills
#pragma unroll 1
    for (int b = 0; b < 4; ++b) {
      // this row's right-hand side (with the alpha term) on the block's 16
      // columns
      double y[16], w[16];
      if (!pre) {
        load_p(rowc, b);
        load_s(rowc, b);
      } else if (YMODE == 1 && b == 0) {
        load_p(s0, 0);
      }
      // the product part (summed over the partials in FP64; kept raw for the
      // residual's dot with one partial) and the alpha-term source
      float4 pc[4];
      if (YMODE == 0) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          pc[m] = pp[m];
          y[4 * m] = (double)pp[m].x;
          y[4 * m + 1] = (double)pp[m].y;
          y[4 * m + 2] = (double)pp[m].z;
          y[4 * m + 3] = (double)pp[m].w;
        }
        const float* pr = (const float*)a.P + (int64_t)rowc * a.cp + 16 * b;
        const int64_t sstride = (int64_t)n * a.cp;
        for (int sp = 1; sp < a.splits; ++sp) {
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const float4 v = *reinterpret_cast<const float4*>(pr + sp * sstride + 4 * m);
            y[4 * m] += (double)v.x;
            y[4 * m + 1] += (double)v.y;
            y[4 * m + 2] += (double)v.z;
            y[4 * m + 3] += (double)v.w;
          }
        }
      } else {
        // the first entry's row (prefetched) and the alpha term, then the
        // rest of the segment (the alpha source taken first frees its
        // registers before the segment's loads)
        const double v = e0 < e1 ? v0 : 0.0;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const bool ok = 16 * b + 4 * m < k;
          const bool oks = live && ok;
          y[4 * m] = live ? fma(alpha, oks ? (double)ps[m].x : 0.0, v * (ok ? (double)pp[m].x : 0.0)) : 0.0;
          y[4 * m + 1] = live ? fma(alpha, oks ? (double)ps[m].y : 0.0, v * (ok ? (double)pp[m].y : 0.0)) : 0.0;
          y[4 * m + 2] = live ? fma(alpha, oks ? (double)ps[m].z : 0.0, v * (ok ? (double)pp[m].z : 0.0)) : 0.0;
          y[4 * m + 3] = live ? fma(alpha, oks ? (double)ps[m].w : 0.0, v * (ok ? (double)pp[m].w : 0.0)) : 0.0;
        }
        // the row's held extras: columns 16 b + 4 m .. + 3 of slot p sit in
        // padding rows 32 p + 8 b + 2 m and + 1, or in hx[p - 8]
        if (xq < BK_XR) {
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const int c = 4 * (4 * b + m);
            const double* d0 = xq < 8 ? reinterpret_cast<const double*>(slab + (32 * xq + 8 * b + 2 * m) * BK_LW + 64)
                                      : &hx[xq - 8][c];
            const double* d1 = xq < 8 ? reinterpret_cast<const double*>(slab + (32 * xq + 8 * b + 2 * m + 1) * BK_LW + 64)
                                      : &hx[xq - 8][c + 2];
            const double2 z0 = *reinterpret_cast<const double2*>(d0), z1 = *reinterpret_cast<const double2*>(d1);
            y[4 * m] += z0.x;
            y[4 * m + 1] += z0.y;
            y[4 * m + 2] += z1.x;
            y[4 * m + 3] += z1.y;
          }
        }
        // the extras of rows beyond the held ones
        const int nheld = xq < BK_XR ? e1 - e0 : 1;
        for (int e = e0 + nheld; e < e1; ++e) {
          const double v = a.seg_val[e];
          const float* sr = Src + (int64_t)a.seg_src[e] * k;
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const int q = 16 * b + 4 * m;
            const float4 x = *reinterpret_cast<const float4*>(sr + (q < k ? q : k - 4));
            const bool ok = q < k;
            y[4 * m] = fma(v, ok ? (double)x.x : 0.0, y[4 * m]);
            y[4 * m + 1] = fma(v, ok ? (double)x.y : 0.0, y[4 * m + 1]);
            y[4 * m + 2] = fma(v, ok ? (double)x.z : 0.0, y[4 * m + 2]);
            y[4 * m + 3] = fma(v, ok ? (double)x.w : 0.0, y[4 * m + 3]);
          }
        }
      }
#pragma unroll
      for (int m = 0; m < 4 && YMODE == 0; ++m) {
        const bool ok = live && 16 * b + 4 * m < k;
        const float4 x = ok ? ps[m] : make_float4(0.f, 0.f, 0.f, 0.f);
        y[4 * m] = live ? fma(alpha, (double)x.x, y[4 * m]) : 0.0;
        y[4 * m + 1] = live ? fma(alpha, (double)x.y, y[4 * m + 1]) : 0.0;
        y[4 * m + 2] = live ? fma(alpha, (double)x.z, y[4 * m + 2]) : 0.0;
        y[4 * m + 3] = live ? fma(alpha, (double)x.w, y[4 * m + 3]) : 0.0;
      }

      // W[:, not B] Ghat[not B, B] for the wave's four 16-row tiles, as its
      // transpose: A[m][p] = Ghat[4 s + p][16 b + m] (lane (li, lg) supplies
      // A[li][lg]), B[p][r] = W[16 t + r][4 s + p] (lane supplies B[lg][li]),
      // over the 12 K steps s outside the block (s = j, or j + 4 from the
      // block on); lane (li, lg) ends with rows 16 t + li, columns
      // 16 b + lg + 4 v
      double ga[12];
#pragma unroll
      for (int j = 0; j < 12; ++j) {
        const int s = j < 4 * b ? j : j + 4;
        ga[j] = Gh[(4 * s + lg) * 64 + 16 * b + li];
      }
      // the next block's loads go out now and stay in flight through this
      // block's products and sweep
      if (pre) {
        if (b < 3) {
          load_p(YMODE == 0 ? rowc : s0, b + 1);
          load_s(rowc, b + 1);
        } else if (nbase < n) {
          const int r = min(nbase + 64 * wid + lane, n - 1);
          if (YMODE == 0) load_p(r, 0);
          load_s(r, 0);
        }
      }
      doublex4 acc[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        acc[t] = doublex4{0.0, 0.0, 0.0, 0.0};
        const float* wr = sw + (16 * t + li) * BK_LW + lg;
#pragma unroll
        for (int j = 0; j < 12; ++j) {
          const int s = j < 4 * b ? j : j + 4;
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ga[j], (double)wr[4 * s], acc[t], 0, 0, 0);
        }
      }
      // lane (li, g) collects row 16 g + li, column 16 b + t + 4 v from
      // e[t] of round v, and takes it off the right-hand side at once
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double e[4] = {acc[0][v], acc[1][v], acc[2][v], acc[3][v]};
        transpose4(e);
#pragma unroll
        for (int t = 0; t < 4; ++t) y[t + 4 * v] -= e[t];
      }
      // this row's old values on the block (read after the products: fewer
      // live registers there)
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const float4 wo = *reinterpret_cast<const float4*>(sw + lane * BK_LW + 16 * b + 4 * m);
        w[4 * m] = wo.x;
        w[4 * m + 1] = wo.y;
        w[4 * m + 2] = wo.z;
        w[4 * m + 3] = wo.w;
      }
      // the serial part: columns 16 b .. 16 b + 15 in order, the sum over the
      // block's columns in four chains with the term of the column changed
      // last added last; row i of the block of Ghat is read at column i, its
      // first half one column ahead (the barrier, which takes column i's
      // result, keeps later reads from being hoisted: all 256 values held in
      // registers at once spill, a whole row ahead spills too; half a row
      // ahead: n = 2^20, k = 64 update 470 -> 462 us)
      const double* gb = gd + 256 * b;
      double gn[8];   // the first 8 entries of the next column's row
#pragma unroll
      for (int q = 0; q < 8; ++q) gn[q] = gb[q];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        double gc[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) gc[q] = q < 8 ? gn[q] : gb[16 * i + q];
        if (i + 1 < 16) {
#pragma unroll
          for (int q = 0; q < 8; ++q) gn[q] = gb[16 * (i + 1) + q];
        }
        double sc4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          if (q == i - 1) continue;
          sc4[q & 3] = fma(w[q], gc[q], sc4[q & 3]);
        }
        double part = (sc4[0] + sc4[1]) + (sc4[2] + sc4[3]);
        if (i > 0) part = fma(w[i - 1], gc[i - 1], part);
        w[i] = fmax(0.0, fma(y[i] - part, gv[16 * b + i], w[i]));
        asm volatile("" : "+v"(w[i]) : : "memory");   // column i done before the next reads
      }
      // new values back to the slab; the residual's product part
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        float4 o;
        o.x = (float)w[4 * m];
        o.y = (float)w[4 * m + 1];
        o.z = (float)w[4 * m + 2];
        o.w = (float)w[4 * m + 3];
        *reinterpret_cast<float4*>(sw + lane * BK_LW + 16 * b + 4 * m) = o;
      }
      if (DOT && YMODE == 0) {
        // <new factor, product part> over the block (rows past n: zero); the
        // partials past the first are read again (no prefetch is in flight
        // with more than one)
        const float* pr = (const float*)a.P + (int64_t)rowc * a.cp + 16 * b;
        const int64_t sstride = (int64_t)n * a.cp;
        const double f = live ? 1.0 : 0.0;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          double q0 = (double)pc[m].x, q1 = (double)pc[m].y, q2 = (double)pc[m].z, q3 = (double)pc[m].w;
          for (int sp = 1; sp < a.splits; ++sp) {
            const float4 v = *reinterpret_cast<const float4*>(pr + sp * sstride + 4 * m);
            q0 += (double)v.x;
            q1 += (double)v.y;
            q2 += (double)v.z;
            q3 += (double)v.w;
          }
          dot = fma((double)(float)w[4 * m] * f, q0, dot);
          dot = fma((double)(float)w[4 * m + 1] * f, q1, dot);
          dot = fma((double)(float)w[4 * m + 2] * f, q2, dot);
          dot = fma((double)(float)w[4 * m + 3] * f, q3, dot);
        }
      }
      wave_sync();
    }
    // the new rows: factor (row-major, float4), then the copy for the next product
    {
      float4* d4 = reinterpret_cast<float4*>(Dst + (int64_t)min(r0, n - 1) * k);
      const int tot = 64 * k4, lim = (n - r0) * k4;
      for (int e = lane; e < tot && e < lim; e += 64) {
        const int rr = e / k4, c4 = e - rr * k4;
        d4[e] = *reinterpret_cast<const float4*>(sw + rr * BK_LW + 4 * c4);
      }
    }
    if (a.Dt) {
      TT* dt = (TT*)a.Dt;
      if (a.dt_rows) {
        for (int e = lane; e < 64 * k; e += 64) {
          const int rr = e / k, q = e - rr * k;
          if (r0 + rr < n) dt[(int64_t)(r0 + rr) * a.ldt + q] = (TT)sw[rr * BK_LW + q];
        }
      } else if (live) {
        for (int q = 0; q < k; ++q) dt[(int64_t)q * a.ldt + row] = (TT)sw[lane * BK_LW + q];
      }
    }
    __syncthreads();
    // Gram partial of the chunk's 256 rows: lane supplies A[li][lg] =
    // F[4 s + lg][16 I + li] and B[lg][li] = F[4 s + lg][16 J + li]
#pragma unroll
    for (int h = 0; h < 3; ++h) {
      const int tau = wid + 4 * h;
      if (tau < 10) {   // wave-uniform
        const int I = tau < 4 ? 0 : tau < 7 ? 1 : tau < 9 ? 2 : 3;
        const int J = I + tau - (I == 0 ? 0 : I == 1 ? 4 : I == 2 ? 7 : 9);
        const float* ca = slab + 16 * I + li;
        const float* cb = slab + 16 * J + li;
#pragma unroll 8
        for (int s = 0; s < BK_ROWS / 4; ++s) {
          const int r = (4 * s + lg) * BK_LW;
          gt[h] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)ca[r], (double)cb[r], gt[h], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // this block's partial row: F^T F (k x k), each upper tile and its mirror
  double* gp = a.part + (int64_t)blockIdx.x * a.pstride;
#pragma unroll
  for (int h = 0; h < 3; ++h) {
    const int tau = wid + 4 * h;
    if (tau < 10) {
      const int I = tau < 4 ? 0 : tau < 7 ? 1 : tau < 9 ? 2 : 3;
      const int J = I + tau - (I == 0 ? 0 : I == 1 ? 4 : I == 2 ? 7 : 9);
      // accumulator element v: row 16 I + lg + 4 v, column 16 J + li
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int p = 16 * I + lg + 4 * v, q = 16 * J + li;
        if (p < k && q < k) {
          gp[p * k + q] = gt[h][v];
          if (I != J) gp[q * k + p] = gt[h][v];
        }
      }
    }
  }
  if (DOT) {
    const double t = block_sum(dot, sc);
    if (tid == 0) a.dpart[blockIdx.x] = t;
  }
}

// Whether the blocked sweep takes a HALS half-step: padded width 64, FP32
// factors and products, no LAI term, k a multiple of 4 (float4 rows), and a
// long factor (n >= 32768).  BPP's passes keep the unblocked kernel (the same
// block count, so the reduction reads the same partial rows).
bool use_blocked(const UpdateArgs& a, int kp, int lp) {
  return kp == 64 && lp == 0 && a.rule == 0 && (a.k & 3) == 0 && a.n >= 32768;
}

template <typename TT, int YMODE>
int launch_update_blk(const UpdateArgs& a, const UpdateRO& ro, int nb, const DevState* st, hipStream_t s) {
  const size_t lds = sizeof(float) * BK_ROWS * BK_LW + sizeof(double) * (4 * 256 + 64);
  // the residual's dot product (YMODE 0 only) is its own instantiation: the
  // kept product part costs registers
  auto kern = YMODE == 0 && a.dpart ? k_update_blk<TT, YMODE, true> : k_update_blk<TT, YMODE, false>;
  if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return -1;
  if (a.ev_start)
    hipExtLaunchKernelGGL(kern, dim3(nb), dim3(256), (uint32_t)lds, s, a.ev_start, a.ev_stop, 0u, a, ro.Ghat, ro.Ginv,
                          (const float*)a.Src, st);
  else
    kern<<<nb, 256, lds, s>>>(a, ro.Ghat, ro.Ginv, (const float*)a.Src, st);
  return 0;
}

template <int KP, int LP, typename TF, typename TP, typename TT, int YMODE, int LPR>
int launch_update_lpr(const UpdateArgs& a, const UpdateRO& ro, int nb, const DevState* st, hipStream_t s) {
  constexpr int RPB = 16 * UPD_RPB / LPR;
  const size_t lds = 8 * (size_t)KP * (KP + 1 + LP) + sizeof(TF) * RPB * ((KP + 1) + (LP > 0 ? LP + 1 : 0)) +
                     (LP > 0 && KP == 32 && YMODE == 2 ? 8 * (size_t)RPB * (KP + 1) + 8 : 0);
  auto kern = k_update<KP, LP, TF, TP, TT, YMODE, LPR>;
  if (lds > 65536 &&
      hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return -1;
  // exactly nb blocks (the reduction reads nb partials); rows beyond
  // RPB * nb are covered by the grid-stride loop
  if (a.ev_start)
    hipExtLaunchKernelGGL(kern, dim3(nb), dim3(16 * UPD_RPB), (uint32_t)lds, s, a.ev_start, a.ev_stop, 0u, a, ro.Ghat,
                          ro.Ginv, ro.M, (const TF*)a.Src, st);
  else
    kern<<<nb, 16 * UPD_RPB, lds, s>>>(a, ro.Ghat, ro.Ginv, ro.M, (const TF*)a.Src, st);
  return 0;
}

// 8 lanes per row where update_lpr8 allows it, else 16.  Fewer lanes per row
// for the long factor without a LAI term (KP = 64, n = 2^20, FP32) passed the
// parity tests and measured slower: 4 lanes (232 VGPRs, two waves per SIMD)
// plain iteration 3.80 -> 4.02 ms, 2 lanes (256 VGPRs and spills) 22.9 ms.
template <int KP, int LP, typename TF, typename TP, typename TT, int YMODE>
int launch_update(const UpdateArgs& a, const UpdateRO& ro, int nb, const DevState* st, hipStream_t s) {
  if constexpr (KP == 64 && LP == 0 && YMODE < 2 && std::is_same_v<TF, float> && std::is_same_v<TP, float>) {
    if (use_blocked(a, KP, LP)) return launch_update_blk<TT, YMODE>(a, ro, nb, st, s);
  }
  if constexpr (KP % 32 == 0) {
    if (update_lpr8(a.n, KP, LP, sizeof(TF))) return launch_update_lpr<KP, LP, TF, TP, TT, YMODE, 8>(a, ro, nb, st, s);
  }
  return launch_update_lpr<KP, LP, TF, TP, TT, YMODE, 16>(a, ro, nb, st, s);
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

// 8 lanes per row (64-row chunks) where the padded width is a multiple of
// 32 and the staging fits in LDS: for the LAI right-hand side at any n (LAI
// iteration at n = 16384, k = 32, l = 48: 56.6 -> 49.9 us, with 256 blocks of
// 64 rows), for the product or the sampled slab once every one of the 512
// blocks has a full chunk (the block count is then 512 with either layout).
bool update_lpr8(int n, int kp, int lp, int tf_bytes) {
  if (kp % 32 != 0) return false;
  const size_t lds = 8 * (size_t)kp * (kp + 1 + lp) + (size_t)tf_bytes * 64 * ((kp + 1) + (lp > 0 ? lp + 1 : 0));
  if (lds > (size_t)160 * 1024) return false;
  return lp > 0 || n >= 512 * 64;
}

// One block per chunk, at most 512 (grid-stride beyond 512 chunks): with
// 16 lanes per row, measured at n = 16384 against 128, 256, 768 and 1024, it
// is the fastest update plus partial-sum reduction.  lp: padded l (LAI), else 0.
int update_blocks(int n, int kp, int lp, int fdtype) {
  const int rpb = update_lpr8(n, kp, lp, fdtype == SYMNMF_F64 ? 8 : 4) ? 2 * UPD_RPB : UPD_RPB;
  return std::max(1, std::min(512, ceil_div(n, rpb)));
}

int update_blocks_max(int n) { return std::max(1, std::min(512, ceil_div(n, UPD_RPB))); }

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

int update_reduce(const double* part, int nb, int E, int k, int l, int kp, double alpha, const double* lam,
                  double* G, double* Ghat, double* Ginv, double* M, const DevState* st, hipStream_t s) {
  k_update_reduce<<<ceil_div(E, RED_COLS), RED_SLICES * RED_COLS, 0, s>>>(part, nb, E, k, l, kp, alpha, lam, G, Ghat,
                                                                          Ginv, M, st);
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
