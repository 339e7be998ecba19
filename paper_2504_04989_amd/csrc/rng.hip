// The Gaussian test tensor Omega of Alg. 2 (its first step draws randn with
// n2 rows, Sec. 3), generated from a 64-bit seed by a counter-based
// generator so that the host (tsvd_omega) and the device (the seed-taking
// entry points, into the caller's workspace) produce the same numbers bit for
// bit, with no state and no allocation.
//
// Element e of the C-contiguous n2 x b x n3 tensor:
//   pair p = e / 2;  (w0, w1, w2, w3) = Philox4x32-10(counter = (p_lo, p_hi, 0, 0),
//                                                     key = (seed_lo, seed_hi))
//   u1 = (2 x1 + 1) 2^-53, x1 = (w0 >> 6) 2^26 + (w1 >> 6)   (52-bit integer)
//   u2 = (2 x2 + 1) 2^-53, x2 = (w2 >> 6) 2^26 + (w3 >> 6)
//   r = sqrt(-2 ln u1), theta = 2 pi u2  (Box-Muller)
//   Omega[e] = r cos(theta) for even e, r sin(theta) for odd e.
// Philox4x32-10 is the generator of Salmon, Moraes, Dror and Shaw,
// "Parallel random numbers: as easy as 1, 2, 3" (SC'11): ten rounds of two
// 32 x 32 -> 64-bit multiplications by 0xD2511F53 and 0xCD9E8D57, the key
// bumped by the Weyl constants 0x9E3779B9 and 0xBB67AE85 between rounds.
//
// The logarithm, sine, cosine and square root are evaluated here with a fixed
// sequence of IEEE-754 double additions, multiplications and divisions
// (no fused multiply-add: contraction is switched off), so that every
// platform that rounds those operations correctly gets the same bits:
//   ln u      = e ln 2 + 2 atanh(s), u = 2^e m, m in (sqrt(1/2), sqrt(2)],
//               s = (m - 1) / (m + 1), atanh by its Taylor series to s^21;
//   sin, cos  of theta = (pi / 2)(j + f), j = floor(4 u2): Taylor series of
//               sin and cos of (pi / 2) f to degree 25 / 24, rotated by j;
//   sqrt x    = five Newton steps y <- (y + x / y) / 2 from an exponent-halving
//               initial guess.
// Values are accurate to a few units in the last place of FP64; FP32 outputs
// are the FP64 values rounded once.
#include <string.h>

#include "../../include/tsvd_rbk.h"
#include "common.h"
#include "kernels.h"

namespace tsvd {

__host__ __device__ inline void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                              uint32_t k1, uint32_t out[4]) {
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

__host__ __device__ inline uint64_t dbits(double x) {
  uint64_t u;
  memcpy(&u, &x, 8);
  return u;
}
__host__ __device__ inline double bitsd(uint64_t u) {
  double x;
  memcpy(&x, &u, 8);
  return x;
}

// uniform in (0, 1) from two 32-bit words: (2 x + 1) 2^-53, x a 52-bit integer
__host__ __device__ inline double rng_unit(uint32_t hi, uint32_t lo) {
  const uint64_t x = ((uint64_t)(hi >> 6) << 26) | (uint64_t)(lo >> 6);
  return (double)(2 * x + 1) * 0x1p-53;
}

// natural logarithm of u in (0, 1) (normal numbers only)
__host__ __device__ inline double rng_log(double u) {
#pragma clang fp contract(off)
  const uint64_t b = dbits(u);
  int e = (int)((b >> 52) & 0x7ff) - 1023;
  double m = bitsd((b & 0x000fffffffffffffull) | 0x3ff0000000000000ull);  // [1, 2)
  if (m > 0x1.6a09e667f3bcdp+0) {
    m = m * 0.5;
    e = e + 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double s2 = s * s;
  double p = 1.0 / 21.0;
  p = p * s2 + 1.0 / 19.0;
  p = p * s2 + 1.0 / 17.0;
  p = p * s2 + 1.0 / 15.0;
  p = p * s2 + 1.0 / 13.0;
  p = p * s2 + 1.0 / 11.0;
  p = p * s2 + 1.0 / 9.0;
  p = p * s2 + 1.0 / 7.0;
  p = p * s2 + 1.0 / 5.0;
  p = p * s2 + 1.0 / 3.0;
  p = p * s2 + 1.0;
  const double lm = 2.0 * s * p;
  return (double)e * 0x1.62e42fefa39efp-1 + lm;
}

__host__ __device__ inline double rng_sqrt(double x) {
#pragma clang fp contract(off)
  if (!(x > 0.0)) return 0.0;
  double y = bitsd((dbits(x) >> 1) + 0x1ff8000000000000ull);
  for (int i = 0; i < 5; ++i) y = 0.5 * (y + x / y);
  return y;
}

// (cos(2 pi u), sin(2 pi u)) for u in (0, 1)
__host__ __device__ inline void rng_sincos2pi(double u, double* c, double* s) {
#pragma clang fp contract(off)
  const double v = u * 4.0;
  const int j = (int)v;
  const double x = (v - (double)j) * 0x1.921fb54442d18p+0;  // [0, pi/2)
  const double x2 = x * x;
  double ps = 1.0 / 15511210043330985984000000.0;  // 1/25!
  ps = ps * x2 - 1.0 / 25852016738884976640000.0;  // -1/23!
  ps = ps * x2 + 1.0 / 51090942171709440000.0;     // 1/21!
  ps = ps * x2 - 1.0 / 121645100408832000.0;       // -1/19!
  ps = ps * x2 + 1.0 / 355687428096000.0;          // 1/17!
  ps = ps * x2 - 1.0 / 1307674368000.0;            // -1/15!
  ps = ps * x2 + 1.0 / 6227020800.0;               // 1/13!
  ps = ps * x2 - 1.0 / 39916800.0;                 // -1/11!
  ps = ps * x2 + 1.0 / 362880.0;                   // 1/9!
  ps = ps * x2 - 1.0 / 5040.0;                     // -1/7!
  ps = ps * x2 + 1.0 / 120.0;                      // 1/5!
  ps = ps * x2 - 1.0 / 6.0;                        // -1/3!
  double pc = 1.0 / 620448401733239439360000.0;      // 1/24!
  pc = pc * x2 - 1.0 / 1124000727777607680000.0;    // -1/22!
  pc = pc * x2 + 1.0 / 2432902008176640000.0;       // 1/20!
  pc = pc * x2 - 1.0 / 6402373705728000.0;          // -1/18!
  pc = pc * x2 + 1.0 / 20922789888000.0;            // 1/16!
  pc = pc * x2 - 1.0 / 87178291200.0;               // -1/14!
  pc = pc * x2 + 1.0 / 479001600.0;                 // 1/12!
  pc = pc * x2 - 1.0 / 3628800.0;                   // -1/10!
  pc = pc * x2 + 1.0 / 40320.0;                     // 1/8!
  pc = pc * x2 - 1.0 / 720.0;                       // -1/6!
  pc = pc * x2 + 1.0 / 24.0;                        // 1/4!
  pc = pc * x2 - 0.5;                               // -1/2!
  const double sn = x + x * x2 * ps;
  const double cs = 1.0 + x2 * pc;
  switch (j & 3) {
    case 0: *c = cs; *s = sn; break;
    case 1: *c = -sn; *s = cs; break;
    case 2: *c = -cs; *s = -sn; break;
    default: *c = sn; *s = -cs; break;
  }
}

// Omega[e] for element e (see the file comment)
__host__ __device__ inline void rng_normal_pair(uint64_t p, uint64_t seed, double* z0, double* z1) {
#pragma clang fp contract(off)
  uint32_t w[4];
  philox4x32_10((uint32_t)p, (uint32_t)(p >> 32), 0u, 0u, (uint32_t)seed, (uint32_t)(seed >> 32), w);
  const double u1 = rng_unit(w[0], w[1]);
  const double u2 = rng_unit(w[2], w[3]);
  const double r = rng_sqrt(-2.0 * rng_log(u1));
  double c, s;
  rng_sincos2pi(u2, &c, &s);
  *z0 = r * c;
  *z1 = r * s;
}

template <typename T>
__global__ __launch_bounds__(256) void omega_kernel(T* __restrict__ out, int64_t n, uint64_t seed) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (2 * p >= n) return;
  double z0, z1;
  rng_normal_pair((uint64_t)p, seed, &z0, &z1);
  out[2 * p] = (T)z0;
  if (2 * p + 1 < n) out[2 * p + 1] = (T)z1;
}

hipError_t omega_fill(void* out, int64_t n, uint64_t seed, DType t, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t pairs = (n + 1) / 2;
  const dim3 grid((unsigned)((pairs + 255) / 256));
  if (t == DT_F64)
    hipLaunchKernelGGL(omega_kernel<double>, grid, dim3(256), 0, s, static_cast<double*>(out), n, seed);
  else
    hipLaunchKernelGGL(omega_kernel<float>, grid, dim3(256), 0, s, static_cast<float*>(out), n, seed);
  return hipGetLastError();
}

void omega_host(double* out, int64_t n, uint64_t seed) {
  for (int64_t p = 0; 2 * p < n; ++p) {
    double z0, z1;
    rng_normal_pair((uint64_t)p, seed, &z0, &z1);
    out[2 * p] = z0;
    if (2 * p + 1 < n) out[2 * p + 1] = z1;
  }
}

}  // namespace tsvd
