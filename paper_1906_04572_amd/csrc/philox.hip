// Gaussian test matrix Omega (Sec. 3.1: n x l, i.i.d. standard normal).
//
// Stream definition (implemented here independently of any CPU code):
//   counter (i, j, tag = 0, sub), key (seed, 0) -> Philox4x64-10 (Salmon et
//   al., SC'11) -> words w0, w1 -> u1 = ((w0 >> 11) + 1) 2^-53 in (0, 1],
//   u2 = (w1 >> 11) 2^-53 in [0, 1) -> z = sqrt(-2 ln u1) cos(2 pi u2)
//   (Box-Muller), where ln and cos are the truncated series
//     ln u  = e LN2_HI + (e LN2_LO + 2 s P(s^2)),  u = f 2^e, f in [1/sqrt2, sqrt2],
//             s = (f - 1)/(f + 1),  P = sum_{k<=11} s^(2k)/(2k+1)
//     cos 2 pi u2 by the exact quadrant split v = 4 u2, q = floor v, f = v - q
//             (f -> 1 - f above 1/2), x = (pi/2) g, and the degree-18 Taylor
//             sums of cos x and sin x / x in x^2,
//   all evaluated with separately rounded IEEE double operations (no fused
//   multiply-add: this file is compiled with contraction off), so every
//   implementation of the definition yields identical bits.
#include "internal.hpp"

#pragma clang fp contract(off)

namespace corutv {
namespace {

constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kM1 = 0xCA5A826395121157ull;
constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kW1 = 0xBB67AE8584CAA73Bull;

// 1/(2k+1), correctly rounded.
__constant__ double kLn[12] = {1.0, 0.3333333333333333, 0.2, 0.14285714285714285,
                               0.1111111111111111, 0.09090909090909091, 0.07692307692307693,
                               0.06666666666666667, 0.058823529411764705, 0.05263157894736842,
                               0.047619047619047616, 0.043478260869565216};
// (-1)^k/(2k)! and (-1)^k/(2k+1)!, correctly rounded.
__constant__ double kCos[10] = {1.0, -0.5, 0.041666666666666664, -0.001388888888888889,
                                2.48015873015873e-05, -2.755731922398589e-07, 2.08767569878681e-09,
                                -1.1470745597729725e-11, 4.779477332387385e-14,
                                -1.5619206968586225e-16};
__constant__ double kSin[10] = {1.0, -0.16666666666666666, 0.008333333333333333,
                                -0.0001984126984126984, 2.7557319223985893e-06,
                                -2.505210838544172e-08, 1.6059043836821613e-10,
                                -7.647163731819816e-13, 2.8114572543455206e-15,
                                -8.22063524662433e-18};
constexpr double kLn2Hi = 0x1.62e42fee00000p-1;   // ln 2 to 32 significant bits
constexpr double kLn2Lo = 0x1.a39ef35793c76p-33;  // ln 2 - kLn2Hi
constexpr double kHalfPi = 0x1.921fb54442d18p+0;
constexpr double kSqrt2 = 0x1.6a09e667f3bcdp+0;

__device__ __forceinline__ void philox10(uint64_t c[4], uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += kW0;
      k1 += kW1;
    }
    const uint64_t lo0 = kM0 * c[0], hi0 = __umul64hi(kM0, c[0]);
    const uint64_t lo1 = kM1 * c[2], hi1 = __umul64hi(kM1, c[2]);
    const uint64_t n0 = hi1 ^ c[1] ^ k0;
    const uint64_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__device__ __forceinline__ double series_ln(double u) {
  const uint64_t b = (uint64_t)__double_as_longlong(u);
  int e = (int)((b >> 52) & 0x7FF) - 1023;
  double f = __longlong_as_double((long long)((b & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull));
  if (f > kSqrt2) {
    f = f * 0.5;
    e += 1;
  }
  const double s = (f - 1.0) / (f + 1.0);
  const double s2 = s * s;
  double p = kLn[11];
#pragma unroll
  for (int k = 10; k >= 0; --k) p = p * s2 + kLn[k];
  const double lnf = 2.0 * (s * p);
  const double ef = (double)e;
  return ef * kLn2Hi + (ef * kLn2Lo + lnf);
}

__device__ __forceinline__ double series_cos_2pi(double u2) {
  const double v = 4.0 * u2;
  const double quad = floor(v);
  const double f = v - quad;
  const bool hi = f > 0.5;
  const double g = hi ? (1.0 - f) : f;
  const double x = kHalfPi * g;
  const double x2 = x * x;
  double pc = kCos[9], ps = kSin[9];
#pragma unroll
  for (int k = 8; k >= 0; --k) {
    pc = pc * x2 + kCos[k];
    ps = ps * x2 + kSin[k];
  }
  const double c = pc, s = x * ps;
  const double cf = hi ? s : c;
  const double sf = hi ? c : s;
  const int q = (int)quad;
  return q == 0 ? cf : (q == 1 ? -sf : (q == 2 ? -cf : sf));
}

__device__ __forceinline__ double gauss(uint64_t i, uint64_t j, uint64_t tag, uint64_t sub,
                                        uint64_t seed) {
  uint64_t c[4] = {i, j, tag, sub};
  philox10(c, seed, 0ull);
  const double u1 = (double)((c[0] >> 11) + 1ull) * 0x1p-53;
  const double u2 = (double)(c[1] >> 11) * 0x1p-53;
  const double r = sqrt(-2.0 * series_ln(u1));
  return r * series_cos_2pi(u2);
}

// One thread per entry; columns ell..ellp-1 are written as zeros.
__global__ void omega_kernel(int64_t n, int ell, int ellp, uint64_t seed, uint32_t sub,
                             double* __restrict__ out64, float* __restrict__ out32, int64_t ld) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = n * (int64_t)ellp;
  if (idx >= total) return;
  const int64_t i = idx % n;
  const int j = (int)(idx / n);
  double z = 0.0;
  if (j < ell) z = gauss((uint64_t)i, (uint64_t)j, 0ull, (uint64_t)sub, seed);
  if (out64) out64[(int64_t)j * ld + i] = z;
  if (out32) out32[(int64_t)j * ld + i] = (float)z;
}

}  // namespace

hipError_t launch_omega(int64_t n, int ell, int ellp, uint64_t seed, uint32_t sub, double* out64,
                        float* out32, int64_t ld, hipStream_t st) {
  const int64_t total = n * (int64_t)ellp;
  if (total == 0) return hipSuccess;
  const int threads = 256;
  const int64_t blocks = (total + threads - 1) / threads;
  omega_kernel<<<dim3((unsigned)blocks), dim3(threads), 0, st>>>(n, ell, ellp, seed, sub, out64,
                                                                 out32, ld);
  return hipGetLastError();
}

}  // namespace corutv
