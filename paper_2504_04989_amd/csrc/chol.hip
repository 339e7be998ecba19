// Per-slice shifted Cholesky factorisation of a b x b Hermitian Gram matrix
// and the inverse of its factor, for CholeskyQR orthonormalisation of a
// Krylov block (the per-slice economy QR of Alg. TQR, used on each block of
// the Krylov basis of Alg. 2).
//
// Input: nsum FP64 partial Gram matrices (split-K products W^H W), summed in
// a fixed order (deterministic).  Output: Rinv = R^{-1}, R upper triangular
// with G + s I = R^H R, stored b x b row-major with zeros below the diagonal.
// The shift s = shift_coef * trace(G) is used on the first pass of shifted
// CholeskyQR (Fukaya et al., 2020), which keeps the factorisation defined for
// rank-deficient or ill-conditioned blocks.
//
// One 256-thread workgroup per slice; the lower triangle lives in LDS in
// packed row order when it fits (see chol_uses_lds) or in global scratch.
#include "common.h"
#include "kernels.h"

namespace tsvd {

__device__ __forceinline__ int64_t tri(int i, int c) { return (int64_t)i * (i + 1) / 2 + c; }

__global__ __launch_bounds__(256) void chol_inv_kernel(const cx<double>* __restrict__ Gpart, int nsum, int64_t part_stride,
                                                       cx<double>* __restrict__ Rinv, cx<double>* gscratch, int b,
                                                       double shift_coef, int* info) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[4];
  __shared__ cx<double> colj[1024];
  __shared__ double s_piv;
  __shared__ int s_bad;
  const int f = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t ntri = (int64_t)b * (b + 1) / 2;
  cx<double>* L = gscratch ? gscratch + (int64_t)f * ntri : reinterpret_cast<cx<double>*>(smem);
  const cx<double>* G = Gpart + (int64_t)f * b * b;

  // Sum the partials (lower triangle, Hermitian average) and the trace.
  double tr = 0;
  for (int64_t t = tid; t < (int64_t)b * b; t += 256) {
    const int i = (int)(t / b), c = (int)(t % b);
    if (c > i) continue;
    double re = 0, im = 0, re2 = 0, im2 = 0;
    for (int s = 0; s < nsum; ++s) {
      const cx<double> g = G[s * part_stride + (int64_t)i * b + c];
      const cx<double> h = G[s * part_stride + (int64_t)c * b + i];
      re += g.re;
      im += g.im;
      re2 += h.re;
      im2 += h.im;
    }
    cx<double> v{0.5 * (re + re2), 0.5 * (im - im2)};
    if (i == c) {
      v.im = 0;
      tr += v.re;
    }
    L[tri(i, c)] = v;
  }
  tr = block_sum<256>(tr, red);
  const double shift = shift_coef * tr;
  if (tid == 0) s_bad = 0;
  __syncthreads();

  // Right-looking Cholesky, lower: G + shift I = L L^H.
  for (int j = 0; j < b; ++j) {
    if (tid == 0) {
      const double d = L[tri(j, j)].re + shift;
      double piv;
      if (d > 0 && isfinite(d)) {
        piv = sqrt(d);
      } else {
        piv = 1.0;  // breakdown: keep the factor invertible, report it
        s_bad = 1;
      }
      s_piv = piv;
      L[tri(j, j)] = cx<double>{piv, 0};
    }
    __syncthreads();
    const double inv = 1.0 / s_piv;
    for (int i = j + 1 + tid; i < b; i += 256) {
      cx<double> v = L[tri(i, j)];
      v.re *= inv;
      v.im *= inv;
      L[tri(i, j)] = v;
      colj[i] = v;
    }
    __syncthreads();
    // trailing update L[i][c] -= L[i][j] conj(L[c][j]), j < c <= i
    const int n = b - j - 1;
    const int64_t cnt = (int64_t)n * (n + 1) / 2;
    for (int64_t t = tid; t < cnt; t += 256) {
      // t -> (ii, cc) with 0 <= cc <= ii < n
      int ii = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
      while ((int64_t)ii * (ii + 1) / 2 > t) --ii;
      while ((int64_t)(ii + 1) * (ii + 2) / 2 <= t) ++ii;
      const int cc = (int)(t - (int64_t)ii * (ii + 1) / 2);
      const int i = j + 1 + ii, c = j + 1 + cc;
      const cx<double> a = colj[i], bb = colj[c];
      cx<double> v = L[tri(i, c)];
      v.re -= a.re * bb.re + a.im * bb.im;
      v.im -= a.im * bb.re - a.re * bb.im;
      L[tri(i, c)] = v;
    }
    __syncthreads();
  }
  if (tid == 0 && s_bad) atomicAdd(&info[INFO_CHOL_BREAKDOWN], 1);

  // In-place inverse of the lower factor: X = L^{-1} by forward elimination of
  // [L | I], one row of X per step, the remaining right-hand sides updated in
  // parallel.
  for (int j = 0; j < b; ++j) {
    for (int i = j + 1 + tid; i < b; i += 256) colj[i] = L[tri(i, j)];
    if (tid == 0) s_piv = L[tri(j, j)].re;
    __syncthreads();
    const double inv = 1.0 / s_piv;
    for (int c = tid; c <= j; c += 256) {
      cx<double> v = (c == j) ? cx<double>{1.0, 0.0} : L[tri(j, c)];
      v.re *= inv;
      v.im *= inv;
      L[tri(j, c)] = v;
    }
    __syncthreads();
    const int64_t cnt = (int64_t)(b - j - 1) * (j + 1);
    for (int64_t t = tid; t < cnt; t += 256) {
      const int i = j + 1 + (int)(t / (j + 1));
      const int c = (int)(t % (j + 1));
      const cx<double> lij = colj[i];
      const cx<double> x = L[tri(j, c)];
      cx<double> v = (c == j) ? cx<double>{0.0, 0.0} : L[tri(i, c)];
      v.re -= lij.re * x.re - lij.im * x.im;
      v.im -= lij.re * x.im + lij.im * x.re;
      L[tri(i, c)] = v;
    }
    __syncthreads();
  }
  // R^{-1} = (L^{-1})^H, upper triangular, row-major b x b.
  cx<double>* out = Rinv + (int64_t)f * b * b;
  for (int64_t t = tid; t < (int64_t)b * b; t += 256) {
    const int r = (int)(t / b), c = (int)(t % b);
    cx<double> v{0, 0};
    if (c >= r) {
      const cx<double> x = L[tri(c, r)];
      v = cx<double>{x.re, -x.im};
    }
    out[t] = v;
  }
}

hipError_t chol_inv_ex(const double* Gpart, int nsum, int64_t part_stride, double* Rinv, void* gscratch, int b,
                       int batch, double shift_coef, int* info, hipStream_t s) {
  if (batch <= 0 || b <= 0) return hipSuccess;
  if (b > 1024) return hipErrorInvalidValue;
  const size_t tri_bytes = (size_t)b * (b + 1) / 2 * sizeof(cx<double>);
  const bool use_lds = chol_uses_lds(b);
  const size_t sm = use_lds ? tri_bytes : 0;
  if (use_lds) {
    static bool attr_set = false;
    if (!attr_set) {
      (void)hipFuncSetAttribute((const void*)chol_inv_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 140 * 1024);
      attr_set = true;
    }
  }
  hipLaunchKernelGGL(chol_inv_kernel, dim3(batch), dim3(256), sm, s, (const cx<double>*)Gpart, nsum, part_stride,
                     (cx<double>*)Rinv, use_lds ? nullptr : (cx<double>*)gscratch, b, shift_coef, info);
  return hipGetLastError();
}

}  // namespace tsvd
