// Exact per-row NLS by block principal pivoting, the paper's BPP update rule
// (Section 2.1, the ANLS subproblems of eq. ANLS4symNMF solved exactly; the
// method is Kim and Park's block principal pivoting, which the paper cites).
//
// Row j solves  min_{x >= 0} 1/2 x^T Ghat x - x^T yhat_j  with Ghat = G + alpha I
// (symmetric positive definite for alpha > 0) and yhat_j the regularised
// right-hand side.  Complementarity: with the passive set F, x_F solves
// Ghat_FF x_F = yhat_F, x is zero off F, and the dual y = Ghat x - yhat is zero
// on F.  A pivoting step exchanges the infeasible variables (x_i < 0 on F,
// y_i < 0 off F) between the two sets: all of them while their number keeps
// falling, then up to three more full exchanges, then only the largest index
// (the backup rule that makes the method terminate).
//
// GPU mapping: one wavefront per row, lane i owns variable i and keeps row i
// of the working matrix in registers; the passive set is a wave-uniform
// 64-bit mask.  The reduced system is solved as the full KP x KP system with
// the rows and columns outside F replaced by the identity (zero right-hand
// side there), by Gauss-Jordan elimination without pivoting (every principal
// submatrix of an SPD matrix is SPD, so all pivots are positive).  The
// trailing block left by elimination stays symmetric, so pivot row J beyond
// column J equals column J, which lane c holds in its register J: each pivot
// step writes one value per lane to a per-wave LDS slot and reads the pivot
// row back as broadcasts.  LDS operations of one wavefront complete in
// order, so the slot needs no barrier, only a compiler scheduling fence.
#include "kernels.hpp"

namespace {

template <int J, int KP>
struct Eliminate {
  template <int C>
  __device__ __forceinline__ static void update_cols(double (&A)[KP], double f, const double* col) {
    if constexpr (C < KP) {
      A[C] = fma(-f, col[C], A[C]);
      update_cols<C + 1>(A, f, col);
    }
  }
  // Pivot J: subtract f_i = A_i[J] / A_J[J] times row J from every other row.
  __device__ __forceinline__ static void run(double (&A)[KP], double& b, double& d, int lane, double* col,
                                            double* bsl) {
    if constexpr (J < KP) {
      col[lane] = A[J];
      bsl[lane] = b;
      __builtin_amdgcn_wave_barrier();
      const double pj = col[J];
      const double bj = bsl[J];
      const double f = (lane == J) ? 0.0 : A[J] / pj;
      update_cols<J + 1>(A, f, col);
      b = fma(-f, bj, b);
      d = (lane == J) ? pj : d;
      __builtin_amdgcn_wave_barrier();
      Eliminate<J + 1, KP>::run(A, b, d, lane, col, bsl);
    }
  }
};

template <int KP, typename TF>
__global__ __launch_bounds__(256) void k_bpp(int n, int k, double* __restrict__ Yhat, const TF* __restrict__ Dst,
                                             const double* __restrict__ Ghat, int* __restrict__ d_flags,
                                             int flag_bit, const DevState* __restrict__ st) {
  if (stopped(st)) return;
  constexpr int LDG = KP + 1;  // padded LDS row: lanes reading different rows hit different banks
  __shared__ double gs[KP * LDG];
  __shared__ double slot[4][2][64];
  for (int e = threadIdx.x; e < KP * KP; e += 256) {
    const int p = e / KP, q = e - p * KP;
    gs[p * LDG + q] = Ghat[e];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  double* col = slot[wv][0];
  double* bsl = slot[wv][1];
  const int li = lane < KP ? lane : KP - 1;
  const double* gr = gs + li * LDG;  // row li of Ghat
  const bool act = lane < k;
  const int kc = lane < k ? lane : k - 1;
  const int cap = 5 * KP + 10;
  for (int row = blockIdx.x * 4 + wv; row < n; row += gridDim.x * 4) {
    const double yh = act ? Yhat[(int64_t)row * KP + li] : 0.0;
    const double x0 = (double)Dst[(int64_t)row * k + kc];
    uint64_t F = __ballot(act && x0 > 0.0);
    int best = k + 1, backup = 3;
    double x = 0.0;
    for (int it = 0;; ++it) {
      const bool inF = (F >> lane) & 1ull;
      double A[KP];
#pragma unroll
      for (int c = 0; c < KP; ++c) {
        const double gv = gr[c];  // read unconditionally: a guarded read becomes a branch
        const bool keep = inF && ((F >> c) & 1ull);
        A[c] = keep ? gv : (c == lane ? 1.0 : 0.0);
      }
      double b = inF ? yh : 0.0, d = 1.0;
      Eliminate<0, KP>::run(A, b, d, lane, col, bsl);
      x = b / d;
      // dual y = Ghat x - yhat
      col[lane] = x;
      __builtin_amdgcn_wave_barrier();
      double y = -yh;
#pragma unroll
      for (int c = 0; c < KP; ++c) y = fma(gr[c], col[c], y);
      __builtin_amdgcn_wave_barrier();
      const bool bad = act && (inF ? (x < 0.0) : (y < 0.0));
      const uint64_t V = __ballot(bad);
      if (V == 0) break;
      if (it >= cap) {
        if (lane == 0) atomicOr(d_flags, flag_bit);
        break;
      }
      const int nv = __popcll(V);
      if (nv < best) {
        best = nv;
        backup = 3;
        F ^= V;
      } else if (backup > 0) {
        --backup;
        F ^= V;
      } else {
        F ^= 1ull << (63 - __clzll(V));
      }
    }
    if (lane < KP) Yhat[(int64_t)row * KP + lane] = act ? fmax(x, 0.0) : 0.0;
  }
}

template <int KP>
int launch(int n, int k, double* Yhat, const void* Dst, int fdtype, const double* Ghat, int* d_flags, int flag_bit,
           const DevState* st, hipStream_t s) {
  const int nb = std::max(1, std::min(4096, ceil_div(n, 4)));
  if (fdtype == SYMNMF_F64)
    k_bpp<KP, double><<<nb, 256, 0, s>>>(n, k, Yhat, (const double*)Dst, Ghat, d_flags, flag_bit, st);
  else
    k_bpp<KP, float><<<nb, 256, 0, s>>>(n, k, Yhat, (const float*)Dst, Ghat, d_flags, flag_bit, st);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

int bpp_update(int n, int k, int kp, double* Yhat, const void* Dst, int fdtype, const double* Ghat, int* d_flags,
               int flag_bit, const DevState* st, hipStream_t s) {
  if (k < 1 || k > kp) return -1;
  switch (kp) {
    case 16: return launch<16>(n, k, Yhat, Dst, fdtype, Ghat, d_flags, flag_bit, st, s);
    case 32: return launch<32>(n, k, Yhat, Dst, fdtype, Ghat, d_flags, flag_bit, st, s);
    case 48: return launch<48>(n, k, Yhat, Dst, fdtype, Ghat, d_flags, flag_bit, st, s);
    case 64: return launch<64>(n, k, Yhat, Dst, fdtype, Ghat, d_flags, flag_bit, st, s);
    default: return -1;
  }
}
