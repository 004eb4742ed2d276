// Shared device/host helpers of the gfx950 SymNMF library.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx8 __attribute__((ext_vector_type(8)));

#define SYM_HD __host__ __device__

// Device-side stop state shared by the iteration kernels: once `done` is
// set, every later kernel of the iteration loop returns at entry.
struct DevState {
  int done;
  int iter;       // completed iterations
  int stall;      // consecutive iterations without a sufficient drop
  int flags;      // numeric fallback flags
  double prev;    // previous normalised residual
  double last;    // latest normalised residual
};

__device__ __forceinline__ bool stopped(const DevState* st) { return st != nullptr && st->done != 0; }

// ---------------------------------------------------------------------------
// Philox-4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11).
// Stream layout: key = (seed lo, seed hi); counter = (block lo, block hi, sub,
// tag); a block's words (w0, w1, w2, w3) give 64-bit values w0|w1<<32 and
// w2|w3<<32; value e of a stream lives in block e/2.
// ---------------------------------------------------------------------------
enum : uint32_t { TAG_H0 = 1, TAG_OMEGA = 2, TAG_SAMPLE = 3, TAG_MLP = 6 };

__device__ __forceinline__ void philox_block(uint64_t seed, uint64_t block, uint32_t sub, uint32_t tag,
                                             uint64_t& v0, uint64_t& v1) {
  uint32_t x0 = (uint32_t)block, x1 = (uint32_t)(block >> 32), x2 = sub, x3 = tag;
  uint32_t key0 = (uint32_t)seed, key1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t m0 = (uint64_t)0xD2511F53u * x0;
    const uint64_t m1 = (uint64_t)0xCD9E8D57u * x2;
    const uint32_t y0 = (uint32_t)(m1 >> 32) ^ x1 ^ key0;
    const uint32_t y2 = (uint32_t)(m0 >> 32) ^ x3 ^ key1;
    x1 = (uint32_t)m1;
    x3 = (uint32_t)m0;
    x0 = y0;
    x2 = y2;
    key0 += 0x9E3779B9u;
    key1 += 0xBB67AE85u;
  }
  v0 = (uint64_t)x0 | ((uint64_t)x1 << 32);
  v1 = (uint64_t)x2 | ((uint64_t)x3 << 32);
}

__device__ __forceinline__ uint64_t philox_value(uint64_t seed, uint64_t e, uint32_t sub, uint32_t tag) {
  uint64_t a, b;
  philox_block(seed, e >> 1, sub, tag, a, b);
  return (e & 1) ? b : a;
}

__device__ __forceinline__ double u53(uint64_t v) { return (double)(v >> 11) * 0x1.0p-53; }

// ---------------------------------------------------------------------------
// Conversions.
// ---------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ double to_f64(T v) { return (double)v; }
template <> __device__ __forceinline__ double to_f64<__bf16>(__bf16 v) { return (double)(float)v; }
template <typename T> __device__ __forceinline__ float to_f32(T v) { return (float)v; }
template <> __device__ __forceinline__ float to_f32<__bf16>(__bf16 v) { return (float)v; }

template <typename T> __device__ __forceinline__ T from_f64(double v) { return (T)v; }

// ---------------------------------------------------------------------------
// Wave-level helpers (wave64).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum of a double over the 16 lanes of a DPP row, every lane receiving the
// total: quad_perm [1,0,3,2] and [2,3,0,1] (pairs, quads), then
// row_half_mirror and row_mirror (halves, full row).  DPP moves are plain
// VALU operations, unlike the LDS permutes behind __shfl_xor.
template <int CTRL>
__device__ __forceinline__ double dpp_double(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_double<0xB1>(v);   // quad_perm(1,0,3,2)
  v += dpp_double<0x4E>(v);   // quad_perm(2,3,0,1)
  v += dpp_double<0x141>(v);  // row_half_mirror
  v += dpp_double<0x140>(v);  // row_mirror
  return v;
}

// Exclusive prefix of v over a 256-thread block (4 waves; wsum: 4 entries of
// LDS); total receives the block's sum in every thread.
template <typename T>
__device__ inline T block_exclusive_scan(T v, T* wsum, T& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  T off = 0;
  for (int i = 0; i < w; ++i) off += wsum[i];
  total = 0;
  for (int i = 0; i < 4; ++i) total += wsum[i];
  __syncthreads();
  return off + x - v;
}

// LDS written by some lanes of a wave and read by others: order the two at
// wavefront scope
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Block-wide FP64 sum with a fixed reduction tree (deterministic).
// `scratch` holds >= blockDim.x/64 doubles.  Result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* scratch) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) scratch[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) t += scratch[i];
  }
  return t;
}

static inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }
