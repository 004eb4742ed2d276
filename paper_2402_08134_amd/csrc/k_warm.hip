// Learned warm start: entry features from the LAI basis, and the small
// column-shared network (inference, and training: forward, backward, weight
// gradients, Adam).  Not part of the paper's method, which starts from a
// random H (Section 5); the start built here feeds the same iterations.
//
// Features of entry (i, j), j < k (c_j = sqrt(n) U[:, j], s_j the sign whose
// part of c_j has the larger norm, a_ij = s_j c_ij, r_i the norm of row i of
// (c_0..c_{k-1}), m_i = max_j a_ij, d the row sums of X):
//   [a_ij, r_i, m_i, a_ij - m_i, lam_j / lam_0, log(max(d_i / mean d, 1e-6))]
// Network 6 -> H -> H -> H -> 1 (ReLU, softplus output), one thread per
// entry with every weight in LDS (8833 floats at H = 64): the weights are
// read as wave-wide broadcasts, so the layers run on the FP32 vector units at
// one LDS read per four FMAs.  Weight gradients are block partial sums in
// FP64 over fixed entry ranges, reduced in a fixed order.
#include "kernels.hpp"

namespace {

constexpr int WS_TILE = 32;  // entries staged per step of the weight-gradient kernel

__device__ __forceinline__ float softplus_f(float z) { return fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))); }
__device__ __forceinline__ float sigmoid_f(float z) { return 1.f / (1.f + expf(-z)); }

// ---- features --------------------------------------------------------------

// Per block and column j < k: sums of squares of the positive and of the
// negative parts of U[:, j] over the block's rows.  Thread t: column t % 64,
// row phase t / 64.
__global__ __launch_bounds__(256) void k_ws_colparts(const double* __restrict__ U, int n, int l, int k,
                                                     double* __restrict__ part) {
  __shared__ double sp[4][64], sn[4][64];
  const int j = threadIdx.x & 63, r = threadIdx.x >> 6;
  double p = 0.0, q = 0.0;
  if (j < k) {
    const int step = gridDim.x * 4;
    int i = blockIdx.x * 4 + r;
    for (; i + 7 * step < n; i += 8 * step) {   // 8 loads in flight, added in row order
      double u[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) u[t] = U[(int64_t)(i + t * step) * l + j];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        p += u[t] > 0.0 ? u[t] * u[t] : 0.0;
        q += u[t] < 0.0 ? u[t] * u[t] : 0.0;
      }
    }
    for (; i < n; i += step) {
      const double u = U[(int64_t)i * l + j];
      p += u > 0.0 ? u * u : 0.0;
      q += u < 0.0 ? u * u : 0.0;
    }
  }
  sp[r][j] = p;
  sn[r][j] = q;
  __syncthreads();
  if (r == 0 && j < k) {
    part[(int64_t)blockIdx.x * 2 * k + j] = ((sp[0][j] + sp[1][j]) + sp[2][j]) + sp[3][j];
    part[(int64_t)blockIdx.x * 2 * k + k + j] = ((sn[0][j] + sn[1][j]) + sn[2][j]) + sn[3][j];
  }
}

// info[0..k) = s_j, info[k..2k) = lam_j / lam_0, info[2k] = mean row sum,
// info[2k+1] = 1 when lam_0 <= 0 (no usable spectrum).  One block: thread t
// sums the partials b = t/64, t/64 + 4, ... of column t % 64; the four
// phases are combined in a fixed order.
__global__ __launch_bounds__(256) void k_ws_info(const double* __restrict__ part, int nb, int k,
                                                 const double* __restrict__ lam, const double* __restrict__ total,
                                                 int n, double* __restrict__ info) {
  __shared__ double sp[4][64], sn[4][64];
  const int j = threadIdx.x & 63, r = threadIdx.x >> 6;
  double p = 0.0, q = 0.0;
  if (j < k) {
    for (int b = r; b < nb; b += 4) {
      p += part[(int64_t)b * 2 * k + j];
      q += part[(int64_t)b * 2 * k + k + j];
    }
  }
  sp[r][j] = p;
  sn[r][j] = q;
  __syncthreads();
  if (r == 0 && j < k) {
    const double P = ((sp[0][j] + sp[1][j]) + sp[2][j]) + sp[3][j];
    const double Q = ((sn[0][j] + sn[1][j]) + sn[2][j]) + sn[3][j];
    info[j] = P >= Q ? 1.0 : -1.0;
    info[k + j] = lam[j] / lam[0];
  }
  if (threadIdx.x == 0) {
    info[2 * k] = *total / n;
    info[2 * k + 1] = lam[0] > 0.0 ? 0.0 : 1.0;
  }
}

// 16 lanes per row (columns li, li + 16, ... of the k <= 64), so the row's
// reads and its 6 k feature writes are spread over the lanes; the row's norm
// and max are combined across the 16 lanes in a fixed order.
__global__ __launch_bounds__(256) void k_ws_features(const double* __restrict__ U, int n, int l, int k,
                                                     const double* __restrict__ info,
                                                     const double* __restrict__ rowsum, float* __restrict__ F) {
  const int i = blockIdx.x * 16 + (threadIdx.x >> 4), li = threadIdx.x & 15;
  const bool live = i < n;   // the whole 16-lane group alike
  const double sn = sqrt((double)n);
  const double* u = U + (int64_t)(live ? i : 0) * l;
  double c[4];
  double r2 = 0.0, m = -INFINITY;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int j = li + 16 * t;
    c[t] = live && j < k ? sn * u[j] : 0.0;
    r2 += c[t] * c[t];
    if (j < k) m = fmax(m, info[j] * c[t]);
  }
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) {
    r2 += __shfl_xor(r2, o, 16);
    m = fmax(m, __shfl_xor(m, o, 16));
  }
  if (!live) return;
  const double r = sqrt(r2);
  const double ld = log(fmax(rowsum[i] / info[2 * k], 1e-6));
  float* f = F + (int64_t)i * k * 6;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int j = li + 16 * t;
    if (j < k) {
      const double a = info[j] * c[t];
      f[6 * j + 0] = (float)a;
      f[6 * j + 1] = (float)r;
      f[6 * j + 2] = (float)m;
      f[6 * j + 3] = (float)(a - m);
      f[6 * j + 4] = (float)info[k + j];
      f[6 * j + 5] = (float)ld;
    }
  }
}

// ---- network -----------------------------------------------------------------

template <int D, int H>
struct Layout {
  static constexpr int W1 = 0, B1 = D * H, W2 = B1 + H, B2 = W2 + H * H, W3 = B2 + H, B3 = W3 + H * H,
                       W4 = B3 + H, B4 = W4 + H, NP = B4 + 1;
};

// out[o] = relu(bias[o] + sum_i in[i] W[i][o]) for an IN-vector held in registers.
template <int IN, int H>
__device__ __forceinline__ void dense_relu(const float* __restrict__ in, const float* __restrict__ W,
                                           const float* __restrict__ bias, float* __restrict__ out) {
#pragma unroll
  for (int o = 0; o < H; ++o) out[o] = bias[o];
#pragma unroll
  for (int i = 0; i < IN; ++i) {
    const float x = in[i];
#pragma unroll
    for (int o = 0; o < H; ++o) out[o] = fmaf(x, W[i * H + o], out[o]);
  }
#pragma unroll
  for (int o = 0; o < H; ++o) out[o] = fmaxf(out[o], 0.f);
}

// Inference (TRAIN = false): Y[e] = softplus(z_e).  Training (TRAIN = true):
// store h1, h2, h3 (rows x H), dz[e] = (y - t) sigmoid(z) / N, and the block
// partial of sum (y - t)^2.
template <int D, int H, bool TRAIN>
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ P, const float* __restrict__ F,
                                                     const float* __restrict__ T, int64_t rows, float inv_n,
                                                     float* __restrict__ Y, float* __restrict__ h1,
                                                     float* __restrict__ h2, float* __restrict__ h3,
                                                     float* __restrict__ dz, double* __restrict__ loss_part) {
  using Lay = Layout<D, H>;
  // The weights are the same for every lane: they are read straight from
  // the (read-only) parameter array at wave-uniform addresses, which the
  // compiler turns into scalar loads feeding the FMAs as SGPR operands.
  __shared__ double sc[8];
  double lacc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < rows; e += (int64_t)gridDim.x * 256) {
    // An empty asm that claims to change a (scalar, zero) offset of the
    // weights keeps the compiler from hoisting all 8833 weight loads out of
    // the loop (they would not fit in scalar registers); it emits no
    // instruction.
    int woff = 0;
    asm volatile("" : "+s"(woff));
    const float* __restrict__ w = P + woff;
    float x[D], a[H], b[H];
#pragma unroll
    for (int i = 0; i < D; ++i) x[i] = F[e * D + i];
    dense_relu<D, H>(x, w + Lay::W1, w + Lay::B1, a);
    if (TRAIN) {
#pragma unroll
      for (int o = 0; o < H; ++o) h1[e * H + o] = a[o];
    }
    dense_relu<H, H>(a, w + Lay::W2, w + Lay::B2, b);
    if (TRAIN) {
#pragma unroll
      for (int o = 0; o < H; ++o) h2[e * H + o] = b[o];
    }
    dense_relu<H, H>(b, w + Lay::W3, w + Lay::B3, a);
    float z = w[Lay::B4];
#pragma unroll
    for (int i = 0; i < H; ++i) z = fmaf(a[i], w[Lay::W4 + i], z);
    const float y = softplus_f(z);
    if (TRAIN) {
#pragma unroll
      for (int o = 0; o < H; ++o) h3[e * H + o] = a[o];
      const float diff = y - T[e];
      dz[e] = diff * sigmoid_f(z) * inv_n;
      lacc += (double)diff * (double)diff;
    } else {
      Y[e] = y;
    }
  }
  if (TRAIN) {
    const double t = block_sum(lacc, sc);
    if (threadIdx.x == 0) loss_part[blockIdx.x] = t;
  }
}

// Inference of the 6-64-64-64-1 network on the FP32 matrix cores
// (v_mfma_f32_16x16x4f32), 16 entries a wave per pass.  Every layer is taken
// as outputs x entries, D = W^T X^T: lane (e, g) = (lane % 16, lane / 16)
// ends with register v of output tile T holding output 16 T + 4 g + v of
// entry e, which is, as it stands, the next layer's B operand of K step
// (T, v) for the K index 16 T + 4 g + v; the A operands are the weights
// W[i][16 T_out + e] for that index, staged in LDS once per block in lane
// order.  The biases start the accumulators; the last layer is a dot
// product of each lane's 16 outputs, summed over the four lane groups.
// Sums are taken in another order than the one-entry-per-thread forward
// (FP32 rounding differences only).
template <int D, int H>
__global__ __launch_bounds__(256) void k_mlp_infer(const float* __restrict__ P, const float* __restrict__ F,
                                                   int64_t rows, float* __restrict__ Y) {
  static_assert(D <= 8 && H == 64, "two K steps for the inputs, four 16-wide output tiles");
  using Lay = Layout<D, H>;
  __shared__ float w1s[4 * 2 * 64];    // [T_out][s][lane]
  __shared__ float w2s[4 * 16 * 64];   // [T_out][T][v][lane]
  __shared__ float w3s[4 * 16 * 64];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, ln = lane & 15, g = lane >> 4;
  for (int x = tid; x < 4 * 2 * 64; x += 256) {
    const int L = x & 63, s = (x >> 6) & 1, to = x >> 7;
    const int i = 4 * s + (L >> 4), o = 16 * to + (L & 15);
    w1s[x] = i < D ? P[Lay::W1 + i * H + o] : 0.f;
  }
  for (int x = tid; x < 4 * 16 * 64; x += 256) {
    const int L = x & 63, st = (x >> 6) & 15, to = x >> 10;
    const int i = 16 * (st >> 2) + 4 * (L >> 4) + (st & 3), o = 16 * to + (L & 15);
    w2s[x] = P[Lay::W2 + i * H + o];
    w3s[x] = P[Lay::W3 + i * H + o];
  }
  // this lane's biases and last-layer weights (outputs 16 T + 4 g + v)
  float b1[4][4], b2[4][4], b3[4][4], w4[4][4];
#pragma unroll
  for (int T = 0; T < 4; ++T)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int o = 16 * T + 4 * g + v;
      b1[T][v] = P[Lay::B1 + o];
      b2[T][v] = P[Lay::B2 + o];
      b3[T][v] = P[Lay::B3 + o];
      w4[T][v] = P[Lay::W4 + o];
    }
  const float b4 = P[Lay::B4];
  __syncthreads();
  const int64_t groups = (rows + 15) / 16;
  for (int64_t grp = (int64_t)blockIdx.x * 4 + wid; grp < groups; grp += (int64_t)gridDim.x * 4) {
    const int64_t e = 16 * grp + ln;
    const bool valid = e < rows;
    float xb[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int i = 4 * s + g;
      xb[s] = valid && i < D ? F[e * D + i] : 0.f;
    }
    floatx4 a[4], c[4];
#pragma unroll
    for (int T = 0; T < 4; ++T) {
      c[T] = floatx4{b1[T][0], b1[T][1], b1[T][2], b1[T][3]};
#pragma unroll
      for (int s = 0; s < 2; ++s)
        c[T] = __builtin_amdgcn_mfma_f32_16x16x4f32(w1s[(T * 2 + s) * 64 + lane], xb[s], c[T], 0, 0, 0);
    }
#pragma unroll
    for (int T = 0; T < 4; ++T)
#pragma unroll
      for (int v = 0; v < 4; ++v) a[T][v] = fmaxf(c[T][v], 0.f);
#pragma unroll
    for (int layer = 0; layer < 2; ++layer) {
      const float* ws = layer == 0 ? w2s : w3s;
#pragma unroll
      for (int T = 0; T < 4; ++T)
        c[T] = layer == 0 ? floatx4{b2[T][0], b2[T][1], b2[T][2], b2[T][3]}
                          : floatx4{b3[T][0], b3[T][1], b3[T][2], b3[T][3]};
#pragma unroll
      for (int Tk = 0; Tk < 4; ++Tk)
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
          for (int T = 0; T < 4; ++T)
            c[T] = __builtin_amdgcn_mfma_f32_16x16x4f32(ws[((T * 4 + Tk) * 4 + v) * 64 + lane], a[Tk][v], c[T], 0, 0, 0);
#pragma unroll
      for (int T = 0; T < 4; ++T)
#pragma unroll
        for (int v = 0; v < 4; ++v) a[T][v] = fmaxf(c[T][v], 0.f);
    }
    float z = 0.f;
#pragma unroll
    for (int T = 0; T < 4; ++T)
#pragma unroll
      for (int v = 0; v < 4; ++v) z = fmaf(a[T][v], w4[T][v], z);
    z += __shfl_xor(z, 16);
    z += __shfl_xor(z, 32);
    if (g == 0 && valid) Y[e] = softplus_f(z + b4);
  }
}

// dz_in[e][i] = (sum_o dz_out[e][o] W[i][o]) * (h_in[e][i] > 0), W (IN x OUT)
// at offset woff of the parameters.
template <int IN, int OUT>
__global__ __launch_bounds__(256) void k_mlp_backprop(const float* __restrict__ P, int woff,
                                                      const float* __restrict__ dz_out,
                                                      const float* __restrict__ h_in, int64_t rows,
                                                      float* __restrict__ dz_in) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < rows; e += (int64_t)gridDim.x * 256) {
    // wave-uniform weight reads (scalar loads), kept inside the loop as in
    // the forward kernel
    int zero = 0;
    asm volatile("" : "+s"(zero));
    const float* __restrict__ w = P + woff + zero;
    float d[OUT];
#pragma unroll
    for (int o = 0; o < OUT; ++o) d[o] = dz_out[e * OUT + o];
#pragma unroll
    for (int i = 0; i < IN; ++i) {
      float acc = 0.f;
#pragma unroll
      for (int o = 0; o < OUT; ++o) acc = fmaf(d[o], w[i * OUT + o], acc);
      dz_in[e * IN + i] = h_in[e * IN + i] > 0.f ? acc : 0.f;
    }
  }
}

// Block partial of [h_in^T dz (IN x OUT) | sum dz (OUT)] over entries
// [b * chunk, (b + 1) * chunk), FP64.
template <int IN, int OUT>
__global__ __launch_bounds__(256) void k_mlp_wgrad(const float* __restrict__ h_in, const float* __restrict__ dz,
                                                   int64_t rows, int64_t chunk, double* __restrict__ part) {
  constexpr int E = IN * OUT + OUT;
  constexpr int PER = (E + 255) / 256;
  static_assert(256 % OUT == 0, "output width must divide the block");
  __shared__ float hs[WS_TILE][IN];
  __shared__ float ds[WS_TILE][OUT];
  double acc[PER];
#pragma unroll
  for (int s = 0; s < PER; ++s) acc[s] = 0.0;
  // 256 is a multiple of OUT, so this thread's output column o is the same
  // for every one of its PER outputs; only the input row differs.
  const int o = threadIdx.x % OUT;
  const int64_t e0 = (int64_t)blockIdx.x * chunk;
  const int64_t e1 = e0 + chunk < rows ? e0 + chunk : rows;
  for (int64_t t0 = e0; t0 < e1; t0 += WS_TILE) {
    const int cnt = (int)(e1 - t0 < WS_TILE ? e1 - t0 : WS_TILE);
    __syncthreads();
    for (int q = threadIdx.x; q < WS_TILE * IN; q += 256) {
      const int r = q / IN, i = q - r * IN;
      hs[r][i] = r < cnt ? h_in[(t0 + r) * IN + i] : 0.f;
    }
    for (int q = threadIdx.x; q < WS_TILE * OUT; q += 256) {
      const int r = q / OUT, c = q - r * OUT;
      ds[r][c] = r < cnt ? dz[(t0 + r) * OUT + c] : 0.f;
    }
    __syncthreads();
    for (int r = 0; r < WS_TILE; ++r) {
      const double d = (double)ds[r][o];
#pragma unroll
      for (int s = 0; s < PER; ++s) {
        const int q = threadIdx.x + 256 * s;
        if (q < IN * OUT) acc[s] = fma((double)hs[r][q / OUT], d, acc[s]);
        else if (q < E) acc[s] += d;
      }
    }
  }
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int q = threadIdx.x + 256 * s;
    if (q < E) part[(int64_t)blockIdx.x * E + q] = acc[s];
  }
}

// grad[off + q] = sum over nb block partials of part[b][q] (fixed order).
__global__ __launch_bounds__(256) void k_mlp_reduce(const double* __restrict__ part, int nb, int E,
                                                    float* __restrict__ grad, int off) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= E) return;
  double acc = 0.0;
  for (int b = 0; b < nb; ++b) acc += part[(int64_t)b * E + q];
  grad[off + q] = (float)acc;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, int np, double lr,
                                              double b1, double b2, double eps, double c1, double c2) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= np) return;
  const double gq = g[q];
  const double mq = b1 * (double)m[q] + (1.0 - b1) * gq;
  const double vq = b2 * (double)v[q] + (1.0 - b2) * gq * gq;
  m[q] = (float)mq;
  v[q] = (float)vq;
  p[q] = (float)((double)p[q] - lr * (mq / c1) / (sqrt(vq / c2) + eps));
}

__global__ __launch_bounds__(256) void k_mlp_init(float* __restrict__ p, int fan_in, int fan_out, int off,
                                                  uint64_t seed, uint32_t sub) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= fan_in * fan_out) return;
  const double u = u53(philox_value(seed, (uint64_t)q, sub, TAG_MLP));
  p[off + q] = (float)((2.0 * u - 1.0) * sqrt(6.0 / fan_in));
}

// H = W = beta Ht with beta^2 = num / den, when num > 0, den > 0 and the
// spectrum was usable; otherwise the factors are left as they are.  beta (or
// 0) is written to *beta_out.
template <typename TF>
__global__ __launch_bounds__(256) void k_warm_apply(const float* __restrict__ Ht, int64_t count,
                                                    const double* __restrict__ num, const double* __restrict__ den,
                                                    const double* __restrict__ flag, TF* __restrict__ H,
                                                    TF* __restrict__ W, double* __restrict__ beta_out) {
  const double a = *num, b = *den;
  const bool ok = a > 0.0 && b > 0.0 && *flag == 0.0;
  const double beta = ok ? sqrt(a / b) : 0.0;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e == 0) *beta_out = beta;
  if (!ok || e >= count) return;
  const TF v = (TF)(beta * (double)Ht[e]);
  H[e] = v;
  W[e] = v;
}

int nblocks(int64_t rows) { return (int)std::max<int64_t>(1, std::min<int64_t>(2048, (rows + 255) / 256)); }

}  // namespace

int mlp_param_count(int hidden) {
  if (hidden != MLP_HIDDEN) return -1;
  return Layout<MLP_D_IN, MLP_HIDDEN>::NP;
}

int mlp_init(float* p, uint64_t seed, hipStream_t s) {
  using Lay = Layout<MLP_D_IN, MLP_HIDDEN>;
  constexpr int D = MLP_D_IN, H = MLP_HIDDEN;
  if (hipMemsetAsync(p, 0, sizeof(float) * Lay::NP, s) != hipSuccess) return -1;
  const int fin[4] = {D, H, H, H}, fout[4] = {H, H, H, 1}, off[4] = {Lay::W1, Lay::W2, Lay::W3, Lay::W4};
  for (int L = 0; L < 4; ++L)
    k_mlp_init<<<ceil_div(fin[L] * fout[L], 256), 256, 0, s>>>(p, fin[L], fout[L], off[L], seed, (uint32_t)L);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int mlp_forward(const float* p, const float* F, int64_t rows, float* Y, hipStream_t s) {
  if (rows <= 0) return 0;
  // two blocks per CU, each staging the weights in LDS once
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(512, (rows + 63) / 64));
  k_mlp_infer<MLP_D_IN, MLP_HIDDEN><<<nb, 256, 0, s>>>(p, F, rows, Y);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

size_t mlp_train_scratch_doubles(int64_t rows) {
  const int nb = nblocks(rows);
  constexpr int H = MLP_HIDDEN;
  return (size_t)nb + (size_t)nb * (H * H + H);  // loss partials, largest gradient partials
}

int mlp_gradient(const float* p, const float* F, const float* T, int64_t rows, float* h1, float* h2, float* h3,
                 float* dza, float* dzb, float* grad, double* scratch, double* d_losssum, hipStream_t s) {
  using Lay = Layout<MLP_D_IN, MLP_HIDDEN>;
  constexpr int D = MLP_D_IN, H = MLP_HIDDEN;
  if (rows <= 0) return -1;
  const int nb = nblocks(rows);
  double* loss_part = scratch;
  double* part = scratch + nb;
  k_mlp_forward<D, H, true><<<nb, 256, 0, s>>>(p, F, T, rows, (float)(1.0 / (double)rows), nullptr, h1, h2, h3, dza,
                                              loss_part);
  sum_partials(loss_part, nb, d_losssum, s);
  const int64_t chunk = (rows + nb - 1) / nb;
  // layer 4: dz4 (rows x 1) in dza; h3
  k_mlp_wgrad<H, 1><<<nb, 256, 0, s>>>(h3, dza, rows, chunk, part);
  k_mlp_reduce<<<ceil_div(H + 1, 256), 256, 0, s>>>(part, nb, H + 1, grad, Lay::W4);
  k_mlp_backprop<H, 1><<<nb, 256, 0, s>>>(p, Lay::W4, dza, h3, rows, dzb);  // dz3
  // layer 3
  k_mlp_wgrad<H, H><<<nb, 256, 0, s>>>(h2, dzb, rows, chunk, part);
  k_mlp_reduce<<<ceil_div(H * H + H, 256), 256, 0, s>>>(part, nb, H * H + H, grad, Lay::W3);
  k_mlp_backprop<H, H><<<nb, 256, 0, s>>>(p, Lay::W3, dzb, h2, rows, dza);  // dz2
  // layer 2
  k_mlp_wgrad<H, H><<<nb, 256, 0, s>>>(h1, dza, rows, chunk, part);
  k_mlp_reduce<<<ceil_div(H * H + H, 256), 256, 0, s>>>(part, nb, H * H + H, grad, Lay::W2);
  k_mlp_backprop<H, H><<<nb, 256, 0, s>>>(p, Lay::W2, dza, h1, rows, dzb);  // dz1
  // layer 1
  k_mlp_wgrad<D, H><<<nb, 256, 0, s>>>(F, dzb, rows, chunk, part);
  k_mlp_reduce<<<ceil_div(D * H + H, 256), 256, 0, s>>>(part, nb, D * H + H, grad, Lay::W1);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int mlp_adam(float* p, const float* g, float* m, float* v, int np, double lr, int64_t t, hipStream_t s) {
  const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
  const double c1 = 1.0 - std::pow(b1, (double)t), c2 = 1.0 - std::pow(b2, (double)t);
  k_adam<<<ceil_div(np, 256), 256, 0, s>>>(p, g, m, v, np, lr, b1, b2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int warm_features(const double* U, int n, int l, int k, const double* lam, const double* rowsum,
                  const double* d_total, float* F, double* info, Workspace& ws, hipStream_t s) {
  if (k < 1 || k > 64 || k > l) return -1;
  const int nb = std::max(1, std::min(64, ceil_div(n, 64)));
  double* part = ws.dbl((size_t)nb * 2 * k);
  if (!part) return -1;
  k_ws_colparts<<<nb, 256, 0, s>>>(U, n, l, k, part);
  k_ws_info<<<1, 256, 0, s>>>(part, nb, k, lam, d_total, n, info);
  k_ws_features<<<ceil_div(n, 16), 256, 0, s>>>(U, n, l, k, info, rowsum, F);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int warm_apply(const float* Ht, int64_t count, const double* num, const double* den, const double* flag, void* H,
               void* W, int fdtype, double* beta_out, hipStream_t s) {
  const int nb = (int)std::max<int64_t>(1, (count + 255) / 256);
  if (fdtype == SYMNMF_F64)
    k_warm_apply<double><<<nb, 256, 0, s>>>(Ht, count, num, den, flag, (double*)H, (double*)W, beta_out);
  else
    k_warm_apply<float><<<nb, 256, 0, s>>>(Ht, count, num, den, flag, (float*)H, (float*)W, beta_out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
