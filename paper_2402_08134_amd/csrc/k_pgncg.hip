// Projected Gauss-Newton with conjugate gradients (Section 2.1.3; Algorithm
// LAI-PGNCG-SymNMF in the appendix on LAI-SymNMF).  One iteration solves the
// normal equations J^T J z = J^T r of the Gauss-Newton least-squares problem
// by a few CG steps from z = 0 and sets H <- max(H - Z, 0).  With
// G = H^T H and Y = X H (or U (Lambda (U^T H)) in LAI mode):
//   J^T r       = -2 (Y - H G)
//   J^T J vec P = 2 (P G + H (P^T H))
//
// Every CG step is ONE pass over the rows plus one small reduction.  The
// step length needs <P, J^T J P> = 2 (<P^T P, G> + tr(M M)) with M = P^T H,
// and the next direction P' = R' + beta P needs only
//   <P'^T P', G> = r'Gr' + 2 beta r'Gp + beta^2 pGp   (sums over rows)
//   M' = R'^T H + beta M,
// so the pass that forms R' also accumulates ||R'||^2, the three quadratic
// forms and the k x k matrix R'^T H, and the next pass applies the direction
// update on the fly.  The CG vectors R, P, Z are FP64, n x KP (zero padded).
//
// Thread layout (all passes): 512 threads = 32 row groups of 16 lanes; a
// group owns 2 consecutive rows of a 64-row chunk and lane g of it the
// columns q = g + 16 c (measured at n = 16384, k = 32: with 256 threads and
// 4 rows per lane a CG step took 16 us).  Row products with a k x k matrix (P G, H M, R' G)
// read the group's rows from LDS (one broadcast per row and i) and the
// matrix from LDS; the k x k block partials use the 16 x 16 thread tile of
// the fused update.
#include "kernels.hpp"

namespace {

constexpr int CG_RPL = 2;                        // rows per lane
constexpr int CG_NT = 512;                       // threads of a row pass
constexpr int CG_RPB = (CG_NT / 16) * CG_RPL;    // rows per chunk (64)
constexpr int CG_E0 = 4;             // scalars ahead of the k x k block in a partial row

template <int KP> constexpr int cg_lw() { return KP + 2; }

// KP x KP copy of a k x k row-major matrix, zero padded.
template <int KP>
__device__ __forceinline__ void stage_square(double* S, const double* __restrict__ A, int k) {
  for (int e = threadIdx.x; e < KP * KP; e += CG_NT) {
    const int p = e / KP, q = e - p * KP;
    S[e] = (p < k && q < k) ? A[p * k + q] : 0.0;
  }
}

// out[j][c] = sum_i T[row j of the group][i] * B[i][g + 16 c]
template <int KP>
__device__ __forceinline__ void rows_times(const double* T, const double* B, int rg, int g,
                                           double (&out)[CG_RPL][KP / 16]) {
  constexpr int CPL = KP / 16, LW = cg_lw<KP>();
  const double* t0 = T + CG_RPL * rg * LW;
#pragma unroll
  for (int j = 0; j < CG_RPL; ++j)
#pragma unroll
    for (int c = 0; c < CPL; ++c) out[j][c] = 0.0;
#pragma unroll 4
  for (int i = 0; i < KP; ++i) {
    double b[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) b[c] = B[i * KP + g + 16 * c];
#pragma unroll
    for (int j = 0; j < CG_RPL; ++j) {
      const double tv = t0[j * LW + i];
#pragma unroll
      for (int c = 0; c < CPL; ++c) out[j][c] = fma(tv, b[c], out[j][c]);
    }
  }
}

// gacc[i][j] += sum over the chunk's rows r of A[r][ty + 16 i] * B[r][tx + 16 j]
template <int KP>
__device__ __forceinline__ void tile_gram(const double* A, const double* B, int tx, int ty,
                                          double (&gacc)[KP / 16][KP / 16]) {
  constexpr int CPL = KP / 16, LW = cg_lw<KP>();
#pragma unroll 4
  for (int r = 0; r < CG_RPB; ++r) {
    double bv[CPL];
#pragma unroll
    for (int j = 0; j < CPL; ++j) bv[j] = B[r * LW + tx + 16 * j];
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
      const double av = A[r * LW + ty + 16 * i];
#pragma unroll
      for (int j = 0; j < CPL; ++j) gacc[i][j] = fma(av, bv[j], gacc[i][j]);
    }
  }
}

// Block sums of N values at once (fixed order: wave trees, then the waves
// in order); the totals land in v of thread 0.  sc: (waves) * N doubles.
template <int N>
__device__ __forceinline__ void block_sums(double (&v)[N], double* sc) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += __shfl_xor(v[i], o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < N; ++i) sc[w * N + i] = v[i];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double t = sc[i];
      for (int q = 1; q < nw; ++q) t += sc[q * N + i];
      v[i] = t;
    }
}

// Partial row of this block: [e, a1, a2, a3, K (k x k)]; dpart (when given)
// receives the block's residual dot.
template <int KP>
__device__ __forceinline__ void write_cg_partials(double* __restrict__ part, int k, double e, double a1, double a2,
                                                  double a3, const double (&gacc)[KP / 16][KP / 16], double* sc,
                                                  double dot = 0.0, double* __restrict__ dpart = nullptr) {
  constexpr int CPL = KP / 16;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double* gp = part + (int64_t)blockIdx.x * (CG_E0 + k * k);
  double v[5] = {e, a1, a2, a3, dot};
  block_sums<5>(v, sc);
  if (threadIdx.x == 0) {
    gp[0] = v[0];
    gp[1] = v[1];
    gp[2] = v[2];
    gp[3] = v[3];
    if (dpart) dpart[blockIdx.x] = v[4];
  }
  if (threadIdx.x < 256)
#pragma unroll
    for (int i = 0; i < CPL; ++i)
#pragma unroll
      for (int j = 0; j < CPL; ++j) {
        const int p = ty + 16 * i, q = tx + 16 * j;
        if (p < k && q < k) gp[CG_E0 + p * k + q] = gacc[i][j];
      }
}

// First pass of an iteration: R = -2 (Y - H G) (the gradient J^T r), the
// start of CG (P = R), and the residual dot <H, Y>.  Right-hand side as in
// the fused update: YMODE 0 split-K partials of X H (or the CSR product),
// YMODE 2 U[j,:] M with M = Lambda U^T H.
template <int KP, typename TF, typename TP, int YMODE>
__global__ __launch_bounds__(CG_NT) void k_cg_init(CgArgs a, const double* __restrict__ G, const TF* __restrict__ H,
                                                 const DevState* __restrict__ st) {
  if (stopped(st)) return;
  constexpr int CPL = KP / 16, LW = cg_lw<KP>();
  extern __shared__ __align__(16) unsigned char smem[];
  double* Gs = reinterpret_cast<double*>(smem);  // KP x KP
  double* T1 = Gs + KP * KP;                     // chunk rows of R
  double* T2 = T1 + CG_RPB * LW;                 // chunk rows of H
  double* Ml = T2 + CG_RPB * LW;                 // YMODE 2: Lambda U^T H (l x KP)
  __shared__ double sc[40];
  const int tid = threadIdx.x, g = tid & 15, rg = tid >> 4;
  const int tx = tid & 15, ty = tid >> 4;
  const int n = a.n, k = a.k;
  stage_square<KP>(Gs, G, k);
  if (YMODE == 2)
    for (int e = tid; e < a.l * KP; e += CG_NT) Ml[e] = a.Mlai[e];
  __syncthreads();
  double gacc[CPL][CPL];
#pragma unroll
  for (int i = 0; i < CPL; ++i)
#pragma unroll
    for (int j = 0; j < CPL; ++j) gacc[i][j] = 0.0;
  double e = 0.0, a1 = 0.0, dot = 0.0;
  for (int base = blockIdx.x * CG_RPB; base < n; base += gridDim.x * CG_RPB) {
    double y[CG_RPL][CPL];
#pragma unroll
    for (int j = 0; j < CG_RPL; ++j)
#pragma unroll
      for (int c = 0; c < CPL; ++c) y[j][c] = 0.0;
    if (YMODE == 2) {
      // y = U[row, :] M for the group's 4 rows: 8 terms of U per row loaded
      // together, M from LDS
      const double* u[CG_RPL];
#pragma unroll
      for (int j = 0; j < CG_RPL; ++j) u[j] = a.U + (int64_t)min(base + CG_RPL * rg + j, n - 1) * a.l;
      for (int p0 = 0; p0 < a.l; p0 += 8) {
        double uv[CG_RPL][8];
#pragma unroll
        for (int j = 0; j < CG_RPL; ++j)
#pragma unroll
          for (int w = 0; w < 8; ++w) uv[j][w] = p0 + w < a.l ? u[j][p0 + w] : 0.0;
#pragma unroll
        for (int w = 0; w < 8; ++w) {
          const int p = min(p0 + w, a.l - 1);
#pragma unroll
          for (int c = 0; c < CPL; ++c) {
            const double mv = Ml[p * KP + g + 16 * c];
#pragma unroll
            for (int j = 0; j < CG_RPL; ++j) y[j][c] = fma(uv[j][w], mv, y[j][c]);
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < CG_RPL; ++j) {
      const int row = base + CG_RPL * rg + j;
      const int rr = min(row, n - 1);
      const bool ok = row < n;
      if (YMODE == 0) {
        const TP* pr = (const TP*)a.P + (int64_t)rr * a.cp + g;
        const int64_t sstride = (int64_t)n * a.cp;
        for (int sp = 0; sp < a.splits; ++sp) {
#pragma unroll
          for (int c = 0; c < CPL; ++c) y[j][c] += (double)pr[sp * sstride + 16 * c];
        }
      }
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        const int q = g + 16 * c;
        const bool m = ok && q < k;
        const double hv = (double)H[(int64_t)rr * k + (q < k ? q : k - 1)];
        const double h = m ? hv : 0.0;
        y[j][c] = m ? y[j][c] : 0.0;
        T2[(CG_RPL * rg + j) * LW + q] = h;
        dot = fma(h, y[j][c], dot);
      }
    }
    __syncthreads();
    double t[CG_RPL][CPL];
    rows_times<KP>(T2, Gs, rg, g, t);  // H G
#pragma unroll
    for (int j = 0; j < CG_RPL; ++j) {
      const int row = base + CG_RPL * rg + j;
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        const int q = g + 16 * c;
        const double r = -2.0 * (y[j][c] - t[j][c]);  // zero on padded rows and columns
        y[j][c] = r;
        e = fma(r, r, e);
        T1[(CG_RPL * rg + j) * LW + q] = r;
        if (row < n) a.R[(int64_t)row * KP + q] = r;
      }
    }
    __syncthreads();
    rows_times<KP>(T1, Gs, rg, g, t);  // R G
#pragma unroll
    for (int j = 0; j < CG_RPL; ++j)
#pragma unroll
      for (int c = 0; c < CPL; ++c) a1 = fma(y[j][c], t[j][c], a1);
    if (tid < 256) tile_gram<KP>(T1, T2, tx, ty, gacc);  // R^T H
    __syncthreads();
  }
  write_cg_partials<KP>(a.part, k, e, a1, 0.0, 0.0, gacc, sc, dot, a.dpart);
}

// One CG step.  cg: [0] e = ||R||^2, [1] beta, [2] step length, [3] done,
// then M = P^T H (k x k) at offset 8, for the direction P = R + beta P_prev
// of this step (P_prev and Z are not read on the first step).
template <int KP, typename TF>
__global__ __launch_bounds__(CG_NT) void k_cg_step(CgArgs a, const double* __restrict__ G,
                                                 const double* __restrict__ cg, const TF* __restrict__ H,
                                                 const DevState* __restrict__ st) {
  if (stopped(st)) return;
  constexpr int CPL = KP / 16, LW = cg_lw<KP>();
  extern __shared__ __align__(16) unsigned char smem[];
  double* Gs = reinterpret_cast<double*>(smem);  // KP x KP
  double* Ms = Gs + KP * KP;                     // KP x KP
  double* T1 = Ms + KP * KP;                     // chunk rows of P, then of R'
  double* T2 = T1 + CG_RPB * LW;                 // chunk rows of H
  __shared__ double sc[40];
  const int tid = threadIdx.x, g = tid & 15, rg = tid >> 4;
  const int tx = tid & 15, ty = tid >> 4;
  const int n = a.n, k = a.k;
  const bool first = a.first != 0;
  stage_square<KP>(Gs, G, k);
  stage_square<KP>(Ms, cg + 8, k);
  const double beta = cg[1], step = cg[2];
  __syncthreads();
  double gacc[CPL][CPL];
#pragma unroll
  for (int i = 0; i < CPL; ++i)
#pragma unroll
    for (int j = 0; j < CPL; ++j) gacc[i][j] = 0.0;
  double e = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  for (int base = blockIdx.x * CG_RPB; base < n; base += gridDim.x * CG_RPB) {
    double r[CG_RPL][CPL], p[CG_RPL][CPL], zo[CG_RPL][CPL];
#pragma unroll
    for (int j = 0; j < CG_RPL; ++j) {
      const int row = base + CG_RPL * rg + j;
      const int rr = min(row, n - 1);
      const bool ok = row < n;
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        const int q = g + 16 * c;
        const int64_t idx = (int64_t)rr * KP + q;
        const double rv = ok ? a.R[idx] : 0.0;
        const double pv = first ? 0.0 : (ok ? a.Pd[idx] : 0.0);
        zo[j][c] = first ? 0.0 : a.Z[idx];  // loaded early; used after the products
        const double hv = (double)H[(int64_t)rr * k + (q < k ? q : k - 1)];
        r[j][c] = rv;
        p[j][c] = fma(beta, pv, rv);
        T1[(CG_RPL * rg + j) * LW + q] = p[j][c];
        T2[(CG_RPL * rg + j) * LW + q] = (ok && q < k) ? hv : 0.0;
        if (ok) a.Pd[idx] = p[j][c];
      }
    }
    __syncthreads();
    double u[CG_RPL][CPL], v[CG_RPL][CPL];
    rows_times<KP>(T1, Gs, rg, g, u);  // P G
    rows_times<KP>(T2, Ms, rg, g, v);  // H M
#pragma unroll
    for (int j = 0; j < CG_RPL; ++j) {
      const int row = base + CG_RPL * rg + j;
      const bool ok = row < n;
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        const int q = g + 16 * c;
        const int64_t idx = (int64_t)(ok ? row : n - 1) * KP + q;
        const double z = fma(step, p[j][c], zo[j][c]);
        const double y = 2.0 * (u[j][c] + v[j][c]);
        const double rn = fma(-step, y, r[j][c]);
        a2 = fma(rn, u[j][c], a2);
        a3 = fma(p[j][c], u[j][c], a3);
        e = fma(rn, rn, e);
        r[j][c] = rn;
        if (ok) {
          a.Z[idx] = z;
          a.R[idx] = rn;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < CG_RPL; ++j)
#pragma unroll
      for (int c = 0; c < CPL; ++c) T1[(CG_RPL * rg + j) * LW + g + 16 * c] = r[j][c];
    __syncthreads();
    rows_times<KP>(T1, Gs, rg, g, u);  // R' G
#pragma unroll
    for (int j = 0; j < CG_RPL; ++j)
#pragma unroll
      for (int c = 0; c < CPL; ++c) a1 = fma(r[j][c], u[j][c], a1);
    if (tid < 256) tile_gram<KP>(T1, T2, tx, ty, gacc);  // R'^T H
    __syncthreads();
  }
  write_cg_partials<KP>(a.part, k, e, a1, a2, a3, gacc, sc);
}

// Last CG step and the projected update: Z += step * (R + beta P_prev),
// H <- max(H - Z, 0) written to H, to W and (dense product) to the padded
// transposed panel, with the block partials of the new Gram H^T H and, in
// LAI mode, of U^T H (the layout the update reduction expects).
template <int KP, int LP, typename TF, typename TT>
__global__ __launch_bounds__(CG_NT) void k_cg_final(CgArgs a, const double* __restrict__ cg,
                                                  const DevState* __restrict__ st) {
  if (stopped(st)) return;
  constexpr int CPL = KP / 16, LW = cg_lw<KP>();
  constexpr int ZI = LP > 0 ? LP / 16 : 1;
  constexpr int LU = LP + 1;
  extern __shared__ __align__(16) unsigned char smem[];
  double* T1 = reinterpret_cast<double*>(smem);  // chunk rows of the new H
  double* Us = T1 + CG_RPB * LW;                 // LAI: chunk rows of U (CG_RPB x LU)
  const int tid = threadIdx.x, g = tid & 15, rg = tid >> 4;
  const int tx = tid & 15, ty = tid >> 4;
  const int n = a.n, k = a.k, l = a.l;
  const bool first = a.first != 0;
  TF* __restrict__ H = (TF*)a.H;
  TF* __restrict__ W = (TF*)a.W;
  const double beta = cg[1], step = cg[2];
  double gacc[CPL][CPL];
  double zacc[ZI][CPL];
#pragma unroll
  for (int i = 0; i < CPL; ++i)
#pragma unroll
    for (int j = 0; j < CPL; ++j) gacc[i][j] = 0.0;
#pragma unroll
  for (int i = 0; i < ZI; ++i)
#pragma unroll
    for (int j = 0; j < CPL; ++j) zacc[i][j] = 0.0;
  for (int base = blockIdx.x * CG_RPB; base < n; base += gridDim.x * CG_RPB) {
#pragma unroll
    for (int j = 0; j < CG_RPL; ++j) {
      const int row = base + CG_RPL * rg + j;
      const int rr = min(row, n - 1);
      const bool ok = row < n;
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        const int q = g + 16 * c;
        const int64_t idx = (int64_t)rr * KP + q;
        const double rv = a.R[idx];
        const double pv = first ? 0.0 : a.Pd[idx];
        const double zv = first ? 0.0 : a.Z[idx];
        const double z = fma(step, fma(beta, pv, rv), zv);
        const int64_t hi = (int64_t)rr * k + (q < k ? q : k - 1);
        const TF hn = (TF)fmax((double)H[hi] - z, 0.0);
        const bool m = ok && q < k;
        T1[(CG_RPL * rg + j) * LW + q] = m ? (double)hn : 0.0;
        if (m) {
          H[hi] = hn;
          W[hi] = hn;
          if (a.Dt) ((TT*)a.Dt)[(int64_t)q * a.ldt + row] = (TT)hn;
        }
      }
    }
    if (LP > 0)
      for (int e = tid; e < CG_RPB * LP; e += CG_NT) {
        const int r = e / LP, p = e - r * LP;
        Us[r * LU + p] = (base + r < n && p < l) ? a.U[(int64_t)(base + r) * l + p] : 0.0;
      }
    __syncthreads();
    if (tid < 256) tile_gram<KP>(T1, T1, tx, ty, gacc);
    if (LP > 0 && tid < 256) {
#pragma unroll 4
      for (int r = 0; r < CG_RPB; ++r) {
        double bv[CPL];
#pragma unroll
        for (int j = 0; j < CPL; ++j) bv[j] = T1[r * LW + tx + 16 * j];
#pragma unroll
        for (int i = 0; i < ZI; ++i) {
          const double uv = Us[r * LU + ty + 16 * i];
#pragma unroll
          for (int j = 0; j < CPL; ++j) zacc[i][j] = fma(uv, bv[j], zacc[i][j]);
        }
      }
    }
    __syncthreads();
  }
  if (tid >= 256) return;
  double* gp = a.part + (int64_t)blockIdx.x * a.pstride;
#pragma unroll
  for (int i = 0; i < CPL; ++i)
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
      const int p = ty + 16 * i, q = tx + 16 * j;
      if (p < k && q < k) gp[p * k + q] = gacc[i][j];
    }
  if (LP > 0) {
    double* zp = gp + k * k;
#pragma unroll
    for (int i = 0; i < ZI; ++i)
#pragma unroll
      for (int j = 0; j < CPL; ++j) {
        const int p = ty + 16 * i, q = tx + 16 * j;
        if (p < l && q < k) zp[p * k + q] = zacc[i][j];
      }
  }
}

// ---- reduction of the CG partials -----------------------------------------

constexpr int CG_GROUP = 32;

// Sum of nb values at stride `stride`, in order; loads issued 8 at a time.
__device__ __forceinline__ double sum_rows(const double* __restrict__ p, int nb, int64_t stride) {
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

__global__ __launch_bounds__(256) void k_cg_sum_groups(const double* __restrict__ part, int nb, int E,
                                                       double* __restrict__ out, const DevState* __restrict__ st) {
  if (stopped(st)) return;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= E) return;
  const int b0 = blockIdx.y * CG_GROUP;
  out[(int64_t)blockIdx.y * E + e] = sum_rows(part + (int64_t)b0 * E + e, min(CG_GROUP, nb - b0), E);
}

// Totals of the partial rows, then the CG scalars of the next pass:
//   beta = e_new / e (0 on the first pass of an iteration or once done),
//   M' = K + beta M, <P', J^T J P'> = 2 (a1 + 2 beta a2 + beta^2 a3 + tr(M' M')),
//   step = e_new / <P', J^T J P'>; CG is done (step 0 from then on) when that
// product is not positive.
__global__ __launch_bounds__(256) void k_cg_scalars(const double* __restrict__ part, int cnt, int k,
                                                    double* __restrict__ cg, int init,
                                                    const DevState* __restrict__ st) {
  if (stopped(st)) return;
  // tot: the CG_E0 scalars, then K (later M') with row stride k + 1 so that
  // the transposed reads of tr(M' M') do not collide in LDS banks
  extern __shared__ __align__(16) unsigned char smem[];
  double* tot = reinterpret_cast<double*>(smem);
  double* Ml = tot + CG_E0;
  __shared__ double sc[40];
  const int E = CG_E0 + k * k, kk = k * k, tid = threadIdx.x;
  for (int e = tid; e < E; e += 256) {
    const double v = sum_rows(part + e, cnt, E);
    if (e < CG_E0) {
      tot[e] = v;
    } else {
      const int f = e - CG_E0, p = f / k, q = f - p * k;
      Ml[p * (k + 1) + q] = v;
    }
  }
  const double e_old = cg[0];
  const bool done_old = !init && cg[3] != 0.0;
  __syncthreads();
  const double e_new = tot[0];
  const double beta = (init || done_old || !(e_old > 0.0)) ? 0.0 : e_new / e_old;
  if (!init)
    for (int e = tid; e < kk; e += 256) {
      const int p = e / k, q = e - p * k;
      Ml[p * (k + 1) + q] = fma(beta, cg[8 + e], Ml[p * (k + 1) + q]);
    }
  __syncthreads();
  double tv[1] = {0.0};
  for (int e = tid; e < kk; e += 256) {
    const int p = e / k, q = e - p * k;
    const double m = Ml[p * (k + 1) + q];
    tv[0] = fma(m, Ml[q * (k + 1) + p], tv[0]);
    cg[8 + e] = m;
  }
  block_sums<1>(tv, sc);
  const double tm = tv[0];
  if (tid == 0) {
    const double pgp = fma(beta * beta, tot[3], fma(2.0 * beta, tot[2], tot[1]));
    const double pap = 2.0 * (pgp + tm);
    const bool done = done_old || !(pap > 0.0);
    cg[0] = e_new;
    cg[1] = done ? 0.0 : beta;
    cg[2] = done ? 0.0 : e_new / pap;
    cg[3] = done ? 1.0 : 0.0;
  }
}

int set_lds(const void* kern, size_t lds) {
  if (lds <= 65536) return 0;
  return hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess ? 0 : -1;
}

template <int KP, typename TF, typename TP>
int launch_init(const CgArgs& a, int ymode, const double* G, int nb, const DevState* st, hipStream_t s) {
  const size_t lds = 8 * ((size_t)KP * KP + 2 * CG_RPB * cg_lw<KP>() + (ymode == 2 ? (size_t)a.l * KP : 0));
  if (ymode == 0) {
    auto kern = k_cg_init<KP, TF, TP, 0>;
    if (set_lds((const void*)kern, lds)) return -1;
    kern<<<nb, CG_NT, lds, s>>>(a, G, (const TF*)a.H, st);
  } else {
    auto kern = k_cg_init<KP, TF, TP, 2>;
    if (set_lds((const void*)kern, lds)) return -1;
    kern<<<nb, CG_NT, lds, s>>>(a, G, (const TF*)a.H, st);
  }
  return 0;
}

template <int KP, typename TF>
int launch_step(const CgArgs& a, const double* G, const double* cg, int nb, const DevState* st, hipStream_t s) {
  const size_t lds = 8 * (2 * (size_t)KP * KP + 2 * CG_RPB * cg_lw<KP>());
  auto kern = k_cg_step<KP, TF>;
  if (set_lds((const void*)kern, lds)) return -1;
  kern<<<nb, CG_NT, lds, s>>>(a, G, cg, (const TF*)a.H, st);
  return 0;
}

template <int KP, int LP, typename TF, typename TT>
int launch_final(const CgArgs& a, const double* cg, int nb, const DevState* st, hipStream_t s) {
  const size_t lds = 8 * (size_t)CG_RPB * (cg_lw<KP>() + (LP > 0 ? LP + 1 : 0));
  auto kern = k_cg_final<KP, LP, TF, TT>;
  if (set_lds((const void*)kern, lds)) return -1;
  kern<<<nb, CG_NT, lds, s>>>(a, cg, st);
  return 0;
}

template <int KP, typename TF, typename TT>
int final_lp(const CgArgs& a, const double* cg, int nb, const DevState* st, hipStream_t s) {
  if (a.l == 0) return launch_final<KP, 0, TF, TT>(a, cg, nb, st, s);
  switch (16 * ceil_div(a.l, 16)) {
    case 16: return launch_final<KP, 16, TF, TT>(a, cg, nb, st, s);
    case 32: return launch_final<KP, 32, TF, TT>(a, cg, nb, st, s);
    case 48: return launch_final<KP, 48, TF, TT>(a, cg, nb, st, s);
    case 64: return launch_final<KP, 64, TF, TT>(a, cg, nb, st, s);
    case 80: return launch_final<KP, 80, TF, TT>(a, cg, nb, st, s);
    case 96: return launch_final<KP, 96, TF, TT>(a, cg, nb, st, s);
    default: return -1;
  }
}

template <int KP>
int dispatch_pass(int pass, const CgArgs& a, int ymode, int fdtype, int pdtype, int tdtype, const double* G,
                  const double* cg, int nb, const DevState* st, hipStream_t s) {
  if (fdtype == SYMNMF_F64) {
    if (pass == 0) return pdtype == SYMNMF_F64 ? launch_init<KP, double, double>(a, ymode, G, nb, st, s) : -1;
    if (pass == 1) return launch_step<KP, double>(a, G, cg, nb, st, s);
    return tdtype == SYMNMF_F64 ? final_lp<KP, double, double>(a, cg, nb, st, s) : -1;
  }
  if (fdtype != SYMNMF_F32) return -1;
  if (pass == 0)
    return pdtype == SYMNMF_F32 ? launch_init<KP, float, float>(a, ymode, G, nb, st, s) : -1;
  if (pass == 1) return launch_step<KP, float>(a, G, cg, nb, st, s);
  if (tdtype == SYMNMF_BF16) return final_lp<KP, float, __bf16>(a, cg, nb, st, s);
  if (tdtype == SYMNMF_F32) return final_lp<KP, float, float>(a, cg, nb, st, s);
  return -1;
}

}  // namespace

int cg_blocks(int n) { return std::max(1, std::min(256, ceil_div(n, CG_RPB))); }

int cg_pass(int pass, const CgArgs& a, int kp, int ymode, int fdtype, int pdtype, int tdtype, const double* G,
            const double* cg, int nb, const DevState* st, hipStream_t s) {
  if (nb < 1 || a.k < 1 || a.k > kp || (ymode != 0 && ymode != 2)) return -1;
  int rc;
  switch (kp) {
    case 16: rc = dispatch_pass<16>(pass, a, ymode, fdtype, pdtype, tdtype, G, cg, nb, st, s); break;
    case 32: rc = dispatch_pass<32>(pass, a, ymode, fdtype, pdtype, tdtype, G, cg, nb, st, s); break;
    case 48: rc = dispatch_pass<48>(pass, a, ymode, fdtype, pdtype, tdtype, G, cg, nb, st, s); break;
    case 64: rc = dispatch_pass<64>(pass, a, ymode, fdtype, pdtype, tdtype, G, cg, nb, st, s); break;
    default: return -1;
  }
  if (rc) return rc;
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

size_t cg_partial_doubles(int k) { return (size_t)CG_E0 + (size_t)k * k; }

int cg_reduce(const double* part, int nb, int k, double* l1, double* cg, bool init, const DevState* st,
              hipStream_t s) {
  const int E = (int)cg_partial_doubles(k);
  const double* src = part;
  int cnt = nb;
  if (nb > CG_GROUP) {
    const int groups = ceil_div(nb, CG_GROUP);
    dim3 g1(ceil_div(E, 256), groups);
    k_cg_sum_groups<<<g1, 256, 0, s>>>(part, nb, E, l1, st);
    src = l1;
    cnt = groups;
  }
  const size_t lds = 8 * ((size_t)CG_E0 + (size_t)k * (k + 1));
  if (lds > 65536 &&
      hipFuncSetAttribute((const void*)k_cg_scalars, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
          hipSuccess)
    return -1;
  k_cg_scalars<<<1, 256, lds, s>>>(src, cnt, k, cg, init ? 1 : 0, st);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
