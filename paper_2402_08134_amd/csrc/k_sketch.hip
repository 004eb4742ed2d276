// The Gaussian sketch Omega of Algorithm RRF (Section 2.2.1), drawn from the
// Philox-4x32-10 stream (key = seed, counter = (element, sub, tag)) by the
// Box-Muller transform with this library's own logarithm and cosine, so the
// values are fixed bit for bit by the definition below rather than by a math
// library.
//
// Every floating-point step is one correctly rounded IEEE-754 FP64 operation
// (+, -, *, / and sqrt), in the order written; this file is compiled with
// floating-point contraction off, so no multiply-add is fused.
//
//   uniforms   a = v0 >> 11, b = v1 >> 11 (53-bit integers of the block's two
//              64-bit words); x = (2^53 - a) 2^-53 in (0, 1]
//   log x      x = m 2^e with m in [sqrt(1/2), sqrt(2)) (frexp, doubled when
//              below sqrt(1/2)); s = (m - 1) / (m + 1), z = s s;
//              ln m = 2 s (1 + z/3 + z^2/5 + ... + z^11/23) by Horner from
//              the innermost term (the atanh series: ln m = 2 atanh s, and
//              |s| <= 0.1716 leaves a remainder below 2^-62 relative);
//              ln x = e LN2_HI + (e LN2_LO + ln m), where LN2_HI is ln 2 cut
//              to 32 fraction bits (so e LN2_HI is exact) and LN2_LO the
//              double nearest ln 2 - LN2_HI (Cody and Waite's split constant)
//   cos(2 pi b 2^-53)
//              quarter turns: q = (b + 2^50) >> 51, f = (b - q 2^51) 2^-51 in
//              [-1/2, 1/2] (both exact); theta = f (pi/2) (pi/2 the double
//              nearest), t = theta theta;
//              sin theta = theta + (theta t) S(t), S = sum_{j=1..8}
//              (-1)^j t^(j-1) / (2j+1)!,  cos theta = 1 + t C(t),
//              C = sum_{j=1..9} (-1)^j t^(j-1) / (2j)!, both by Horner from
//              the innermost coefficient; each coefficient is the double
//              nearest +-1/n! (n! <= 18! is exact in FP64; the dropped Taylor
//              terms are below 2^-62 relative for |theta| <= pi/4);
//              q mod 4 = 0, 1, 2, 3 gives cos theta, -sin theta, -cos theta,
//              sin theta
//   Gaussian   sqrt(-2 ln x) * cos(2 pi b 2^-53)
#include "kernels.hpp"

namespace {

constexpr double kLn2Hi = 0x1.62e42fee00000p-1;
constexpr double kLn2Lo = 0x1.a39ef35793c76p-33;
constexpr double kSqrtHalf = 0x1.6a09e667f3bcdp-1;
constexpr double kHalfPi = 0x1.921fb54442d18p+0;

__device__ __forceinline__ double fact(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= (double)i;  // exact up to 18!
  return f;
}

__device__ double sketch_log(uint64_t a) {
  const double x = (double)((1ull << 53) - a) * 0x1.0p-53;  // exact, in (0, 1]
  int e = 0;
  double m = frexp(x, &e);  // m in [1/2, 1)
  if (m < kSqrtHalf) {
    m = m * 2.0;
    e -= 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double z = s * s;
  double p = 1.0 / 23.0;
#pragma unroll
  for (int j = 10; j >= 0; --j) p = 1.0 / (double)(2 * j + 1) + z * p;
  const double lnm = (s + s) * p;
  const double de = (double)e;
  return de * kLn2Hi + (de * kLn2Lo + lnm);
}

__device__ double sketch_cos_turn(uint64_t b) {
  const uint64_t q = (b + (1ull << 50)) >> 51;
  const int64_t fi = (int64_t)b - (int64_t)(q << 51);
  const double theta = ((double)fi * 0x1.0p-51) * kHalfPi;
  const double t = theta * theta;
  double S = 1.0 / fact(17);
#pragma unroll
  for (int j = 7; j >= 1; --j) S = ((j & 1) ? -1.0 : 1.0) / fact(2 * j + 1) + t * S;
  double C = -1.0 / fact(18);  // (-1)^9 / 18!
#pragma unroll
  for (int j = 8; j >= 1; --j) C = ((j & 1) ? -1.0 : 1.0) / fact(2 * j) + t * C;
  const double sn = theta + (theta * t) * S;
  const double cs = 1.0 + t * C;
  switch (q & 3) {
    case 0: return cs;
    case 1: return -sn;
    case 2: return -cs;
    default: return sn;
  }
}

__global__ __launch_bounds__(256) void k_gaussian(double* __restrict__ out, int64_t count, uint64_t seed, uint32_t sub,
                                                  uint32_t tag) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= count) return;
  uint64_t v0, v1;
  philox_block(seed, (uint64_t)e, sub, tag, v0, v1);
  const double r2 = -2.0 * sketch_log(v0 >> 11);
  out[e] = sqrt(r2) * sketch_cos_turn(v1 >> 11);
}

}  // namespace

int gen_gaussian(double* out, int64_t count, uint64_t seed, uint32_t sub, uint32_t tag, hipStream_t s) {
  if (count <= 0) return 0;
  k_gaussian<<<ceil_div(count, 256), 256, 0, s>>>(out, count, seed, sub, tag);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
