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
// One 256-thread workgroup per slice, threads arranged 16 x 16 over (row,
// column) of the trailing triangle; the lower triangle lives in LDS in packed
// row order when it fits (see chol_uses_lds) or in global scratch.
#include "common.h"
#include "kernels.h"

#ifdef TSVD_PHASE_PROF
__device__ unsigned long long g_phase[16];
#define PHASE_T0() unsigned long long ph_t = clock64()
#define PHASE(i)                                            \
  do {                                                      \
    if (blockIdx.x == 0 && threadIdx.x == 0) {              \
      const unsigned long long now = clock64();             \
      atomicAdd(&g_phase[i], now - ph_t);                   \
      ph_t = now;                                           \
    }                                                       \
  } while (0)
#else
#define PHASE_T0()
#define PHASE(i)
#endif

namespace tsvd {

__device__ __forceinline__ int tri(int i, int c) { return i * (i + 1) / 2 + c; }

// mode 0: Gpart holds partial Gram matrices, factor G + shift I = R^H R.
// mode 1: Gpart holds partials of an upper triangular R (its strict lower part
//         is ignored); only the inverse is formed.
template <bool LDS>
__global__ __launch_bounds__(256) void chol_inv_kernel(const cx<double>* __restrict__ Gpart, int nsum,
                                                       int64_t part_stride, cx<double>* __restrict__ Rinv,
                                                       cx<double>* gscratch, int b, double shift_coef, int* info,
                                                       int mode) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ cx<double> colj[1024];
  __shared__ double red[4];
  const int f = blockIdx.x;
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int64_t ntri = (int64_t)b * (b + 1) / 2;
  cx<double>* L = LDS ? reinterpret_cast<cx<double>*>(smem) : gscratch + (int64_t)f * ntri;
  const cx<double>* G = Gpart + (int64_t)f * b * b;
  PHASE_T0();

  if (mode == 1) {
    // L = R^H from the (summed) upper triangle of R
    for (int s = 0; s < nsum; ++s) {
      const cx<double>* Gs = G + s * part_stride;
      for (int i = ty; i < b; i += 16) {
        for (int c = tx; c <= i; c += 16) {
          const cx<double> r = Gs[(int64_t)c * b + i];
          cx<double> v{r.re, -r.im};
          if (s > 0) {
            const cx<double> o = L[tri(i, c)];
            v.re += o.re;
            v.im += o.im;
          }
          L[tri(i, c)] = v;
        }
      }
    }
    __syncthreads();
  } else {
  // Sum the partials into the lower triangle (partial index outermost so the
    // loads of one thread are independent), then the Hermitian average.
    for (int s = 0; s < nsum; ++s) {
      const cx<double>* Gs = G + s * part_stride;
      for (int i = ty; i < b; i += 16) {
#pragma unroll 4
        for (int c = tx; c <= i; c += 16) {
          const cx<double> g = Gs[(int64_t)i * b + c];
          const cx<double> h = Gs[(int64_t)c * b + i];
          cx<double> v{0.5 * (g.re + h.re), 0.5 * (g.im - h.im)};
          if (s > 0) {
            const cx<double> o = L[tri(i, c)];
            v.re += o.re;
            v.im += o.im;
          }
          L[tri(i, c)] = v;
        }
      }
    }
    __syncthreads();
    double tr = 0;
    for (int i = tid; i < b; i += 256) tr += L[tri(i, i)].re;
    tr = block_sum<256>(tr, red);
    const double shift = shift_coef * tr;
    PHASE(0);

    // Right-looking Cholesky, lower: G + shift I = L L^H.
    int bad = 0;
    for (int j = 0; j < b; ++j) {
      const double dj = L[tri(j, j)].re + shift;
      double piv = 1.0;
      if (dj > 0 && isfinite(dj))
        piv = sqrt(dj);
      else
        bad = 1;  // breakdown: keep the factor invertible, report it
      const double inv = 1.0 / piv;
      for (int i = j + 1 + tid; i < b; i += 256) {
        cx<double> v = L[tri(i, j)];
        v.re *= inv;
        v.im *= inv;
        colj[i] = v;
      }
      __syncthreads();
      if (tid == 0) L[tri(j, j)] = cx<double>{piv, 0};
      // L[i][c] -= L[i][j] conj(L[c][j]) for j < c <= i; column j takes its scaled values
      for (int i = j + 1 + ty; i < b; i += 16) {
        const cx<double> a = colj[i];
        if (tx == 0) L[tri(i, j)] = a;
        for (int c = j + 1 + tx; c <= i; c += 16) {
          const cx<double> bb = colj[c];
          cx<double> v = L[tri(i, c)];
          v.re -= a.re * bb.re + a.im * bb.im;
          v.im -= a.im * bb.re - a.re * bb.im;
          L[tri(i, c)] = v;
        }
      }
      __syncthreads();
    }
    if (tid == 0 && bad) atomicAdd(&info[INFO_CHOL_BREAKDOWN], 1);
    PHASE(1);
  }

  // In-place inverse of the lower factor, X = L^{-1}: forward elimination of
  // [L | I], one row of X per step; the later right-hand sides are updated
  // with the new row.
  for (int j = 0; j < b; ++j) {
    for (int i = j + 1 + tid; i < b; i += 256) colj[i] = L[tri(i, j)];
    const cx<double> djj = L[tri(j, j)];
    const double den = djj.re * djj.re + djj.im * djj.im;
    const cx<double> inv{djj.re / den, -djj.im / den};
    __syncthreads();
    for (int c = tid; c <= j; c += 256) {
      const cx<double> x = (c == j) ? cx<double>{1.0, 0.0} : L[tri(j, c)];
      L[tri(j, c)] = cx<double>{x.re * inv.re - x.im * inv.im, x.re * inv.im + x.im * inv.re};
    }
    __syncthreads();
    for (int i = j + 1 + ty; i < b; i += 16) {
      const cx<double> lij = colj[i];
      for (int c = tx; c <= j; c += 16) {
        const cx<double> x = L[tri(j, c)];
        cx<double> v = (c == j) ? cx<double>{0.0, 0.0} : L[tri(i, c)];
        v.re -= lij.re * x.re - lij.im * x.im;
        v.im -= lij.re * x.im + lij.im * x.re;
        L[tri(i, c)] = v;
      }
    }
    __syncthreads();
  }
  PHASE(2);
  // R^{-1} = (L^{-1})^H, upper triangular, row-major b x b.
  cx<double>* out = Rinv + (int64_t)f * b * b;
  for (int r = ty; r < b; r += 16) {
    for (int c = tx; c < b; c += 16) {
      cx<double> v{0, 0};
      if (c >= r) {
        const cx<double> x = L[tri(c, r)];
        v = cx<double>{x.re, -x.im};
      }
      out[(int64_t)r * b + c] = v;
    }
  }
  PHASE(3);
}

hipError_t chol_inv_ex(const double* Gpart, int nsum, int64_t part_stride, double* Rinv, void* gscratch, int b,
                       int batch, double shift_coef, int* info, hipStream_t s, int mode) {
  if (batch <= 0 || b <= 0) return hipSuccess;
  if (b > 1024) return hipErrorInvalidValue;
  const size_t tri_bytes = (size_t)b * (b + 1) / 2 * sizeof(cx<double>);
  const bool use_lds = chol_uses_lds(b);
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)chol_inv_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              140 * 1024);
    (void)hipGetLastError();
    attr_set = true;
  }
  if (use_lds)
    hipLaunchKernelGGL(chol_inv_kernel<true>, dim3(batch), dim3(256), tri_bytes, s, (const cx<double>*)Gpart, nsum,
                       part_stride, (cx<double>*)Rinv, nullptr, b, shift_coef, info, mode);
  else
    hipLaunchKernelGGL(chol_inv_kernel<false>, dim3(batch), dim3(256), 0, s, (const cx<double>*)Gpart, nsum,
                       part_stride, (cx<double>*)Rinv, (cx<double>*)gscratch, b, shift_coef, info, mode);
  return hipGetLastError();
}

}  // namespace tsvd
