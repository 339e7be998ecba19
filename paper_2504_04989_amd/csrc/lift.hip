// Small element-wise kernels around the lift of Alg. 2 (U_f = Q_f W_k,
// V_f = C_f^H W_k diag(1/sigma)) and the phase convention of the outputs.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace tsvd {

__global__ void zero_info_kernel(int* info) {
  if (threadIdx.x < INFO_COUNT) info[threadIdx.x] = 0;
}
hipError_t zero_info(int* info, hipStream_t s) {
  hipLaunchKernelGGL(zero_info_kernel, dim3(1), dim3(64), 0, s, info);
  return hipGetLastError();
}

// Wout[f][r][c] = W[f][r][c] * g(lambda[f][c]); g = sqrt (mode 0), 1/sqrt (mode 1,
// zero for lambda <= 0), 1 (mode 2).  Output FP64.
__global__ void scale_cols_kernel(const cx<double>* W, const double* lambda, cx<double>* out, int m, int k,
                                  int64_t total, int mode) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int c = (int)(t % k);
  const int64_t f = t / ((int64_t)m * k);
  const double l = lambda[f * k + c];
  double g = 1.0;
  if (mode == 0) g = l > 0 ? sqrt(l) : 0.0;
  if (mode == 1) g = l > 0 ? 1.0 / sqrt(l) : 0.0;
  const cx<double> w = W[t];
  out[t] = cx<double>{w.re * g, w.im * g};
}
hipError_t scale_cols(const double* W, const double* lambda, void* Wout, int m, int k, int batch, int scale_mode,
                      DType t, hipStream_t s) {
  (void)t;
  const int64_t total = (int64_t)batch * m * k;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(scale_cols_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, (const cx<double>*)W,
                     lambda, (cx<double>*)Wout, m, k, total, scale_mode);
  return hipGetLastError();
}

// Ws[f][r][c] = W[f][r][c] / lambda[f][c] where lambda[f][c] > thr * lambda[f][0]
// and lambda[f][c] > 0, else 0: the eigenvectors of a Gram X^H X (or X X^H)
// weighted by sigma^-2 over the singular values kept by a relative cut-off
// sigma_c > sqrt(thr) sigma_0.
__global__ void pinv_weights_kernel(const cx<double>* W, const double* lambda, cx<double>* out, int m, int k,
                                    int64_t total, double thr) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int c = (int)(t % k);
  const int64_t f = t / ((int64_t)m * k);
  const double l = lambda[f * k + c], l0 = lambda[f * k];
  const double g = (l > 0.0 && l > thr * l0) ? 1.0 / l : 0.0;
  const cx<double> w = W[t];
  out[t] = cx<double>{w.re * g, w.im * g};
}
hipError_t pinv_weights(const double* W, const double* lambda, void* Ws, int m, int k, int batch, double thr,
                        hipStream_t s) {
  const int64_t total = (int64_t)batch * m * k;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(pinv_weights_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     (const cx<double>*)W, lambda, (cx<double>*)Ws, m, k, total, thr);
  return hipGetLastError();
}

// W_k rounded to complex FP32, and W_k diag(1 / sigma) likewise (sigma =
// sqrt(lambda), 0 where lambda <= 0): the thin operands of the lift products
// U_f = Q_f W_k and V_f = T_f W_k Sigma^{-1} on the FP32 path.
__global__ void lift_operands_kernel(const cx<double>* __restrict__ W, const double* __restrict__ lambda,
                                     cx<float>* __restrict__ Wf, cx<float>* __restrict__ Wsf, int m, int k,
                                     int64_t total) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int c = (int)(t % k);
  const int64_t f = t / ((int64_t)m * k);
  const double l = lambda[f * k + c];
  const double g = l > 0 ? 1.0 / sqrt(l) : 0.0;
  const cx<double> w = W[t];
  Wf[t] = cx<float>{(float)w.re, (float)w.im};
  Wsf[t] = cx<float>{(float)(w.re * g), (float)(w.im * g)};
}
hipError_t lift_operands_f32(const double* W, const double* lambda, void* Wf, void* Wsf, int m, int k, int batch,
                             hipStream_t s) {
  const int64_t total = (int64_t)batch * m * k;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(lift_operands_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     (const cx<double>*)W, lambda, (cx<float>*)Wf, (cx<float>*)Wsf, m, k, total);
  return hipGetLastError();
}

// Uout[f][i][c] = Uin[f][i][c] * sigma[f][c]
template <typename T>
__global__ void scale_by_kernel(const cx<T>* U, const double* sigma, cx<T>* out, int64_t n1, int k, int64_t total) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int c = (int)(t % k);
  const int64_t f = t / (n1 * k);
  const T g = (T)sigma[f * k + c];
  const cx<T> u = U[t];
  out[t] = cx<T>{u.re * g, u.im * g};
}
hipError_t scale_cols_by(const void* Uin, const double* sigma, void* Uout, int64_t n1, int k, int batch, DType t,
                         hipStream_t s) {
  const int64_t total = (int64_t)batch * n1 * k;
  if (total == 0) return hipSuccess;
  const dim3 g((unsigned)((total + 255) / 256));
  if (t == DT_F64)
    hipLaunchKernelGGL(scale_by_kernel<double>, g, dim3(256), 0, s, (const cx<double>*)Uin, sigma, (cx<double>*)Uout,
                       n1, k, total);
  else
    hipLaunchKernelGGL(scale_by_kernel<float>, g, dim3(256), 0, s, (const cx<float>*)Uin, sigma, (cx<float>*)Uout, n1,
                       k, total);
  return hipGetLastError();
}

// sigma = sqrt(max(lambda, 0)) in FP64, and as complex (sigma, 0) in the
// working precision for the inverse transform of the singular tubes.
template <typename T>
__global__ void sigma_kernel(const double* lambda, double* sigma, cx<T>* scx, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double l = lambda[t];
  const double sg = l > 0 ? sqrt(l) : 0.0;
  sigma[t] = sg;
  scx[t] = cx<T>{(T)sg, (T)0};
}
hipError_t sigma_from_lambda(const double* lambda, double* sigma, void* scx, int64_t n, DType t, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const dim3 g((unsigned)((n + 255) / 256));
  if (t == DT_F64)
    hipLaunchKernelGGL(sigma_kernel<double>, g, dim3(256), 0, s, lambda, sigma, (cx<double>*)scx, n);
  else
    hipLaunchKernelGGL(sigma_kernel<float>, g, dim3(256), 0, s, lambda, sigma, (cx<float>*)scx, n);
  return hipGetLastError();
}

// FP64 lift of the right factor: P = T_f W_k (F x n2 x k) on entry; per
// column, sigma_j = ||P(:, j)||_2 (sum of squares in row order), then
// V(:, j) = P(:, j) / sigma_j in place (left zero when sigma_j = 0), and sigma
// as FP64 and as complex (sigma, 0).  ||T_f w_j|| = ||C_f^H w_j|| is sigma_j
// to a relative accuracy of about u sigma_1 / sigma_j, where sqrt(lambda_j)
// carries the Gram's absolute error m u lambda_1 / (2 lambda_j).
__global__ void colnorm_sigma_kernel(cx<double>* __restrict__ P, int64_t n2, int k, int64_t total,
                                     double* __restrict__ sigma, cx<double>* __restrict__ scx) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int c = (int)(t % k);
  const int64_t f = t / k;
  cx<double>* col = P + f * n2 * k + c;
  double ss = 0.0;
  for (int64_t i = 0; i < n2; ++i) {
    const cx<double> v = col[i * k];
    ss += v.re * v.re + v.im * v.im;
  }
  const double sg = sqrt(ss);
  if (sg > 0) {
    const double inv = 1.0 / sg;
    for (int64_t i = 0; i < n2; ++i) {
      cx<double> v = col[i * k];
      col[i * k] = cx<double>{v.re * inv, v.im * inv};
    }
  }
  sigma[t] = sg;
  scx[t] = cx<double>{sg, 0.0};
}
hipError_t colnorm_sigma(void* P, int64_t n2, int k, int batch, double* sigma, void* scx, hipStream_t s) {
  const int64_t total = (int64_t)batch * k;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(colnorm_sigma_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, (cx<double>*)P,
                     n2, k, total, sigma, (cx<double>*)scx);
  return hipGetLastError();
}

// R_f (r x n, dtype T, row-major) = upper-trapezoidal part of the sum of
// nsum FP64 partial products (partial s of slice f at part + s * part_stride
// + f * r * n complex doubles); entries below the diagonal are written as 0.
template <typename T>
__global__ void triu_store_kernel(const cx<double>* __restrict__ part, int nsum, int64_t part_stride, int r, int n,
                                  int batch, cx<T>* __restrict__ R) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)r * n;
  if (t >= per * batch) return;
  const int64_t e = t % per;
  const int i = (int)(e / n), j = (int)(e % n);
  cx<double> v{0.0, 0.0};
  if (j >= i) {
    for (int s = 0; s < nsum; ++s) {
      const cx<double> w = part[s * part_stride + t];
      v.re += w.re;
      v.im += w.im;
    }
  }
  R[t] = cx<T>{(T)v.re, (T)v.im};
}
hipError_t triu_store(const double* part, int nsum, int64_t part_stride, int r, int n, int batch, void* R, DType t,
                      hipStream_t s) {
  const int64_t tot = (int64_t)r * n * batch;
  if (tot == 0) return hipSuccess;
  const dim3 g((unsigned)((tot + 255) / 256));
  if (t == DT_F64)
    hipLaunchKernelGGL(triu_store_kernel<double>, g, dim3(256), 0, s, (const cx<double>*)part, nsum, part_stride, r,
                       n, batch, (cx<double>*)R);
  else
    hipLaunchKernelGGL(triu_store_kernel<float>, g, dim3(256), 0, s, (const cx<double>*)part, nsum, part_stride, r,
                       n, batch, (cx<float>*)R);
  return hipGetLastError();
}

// C = mask ? M : X elementwise (X == nullptr: 0), the data step of the
// completion iteration; four elements per thread.
template <typename T>
__global__ void masked_merge_kernel(const T* __restrict__ M, const unsigned char* __restrict__ mask,
                                    const T* __restrict__ X, T* __restrict__ C, int64_t n) {
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t i = i0 + u;
    if (i < n) C[i] = mask[i] ? M[i] : (X ? X[i] : (T)0);
  }
}
hipError_t masked_merge(const void* M, const unsigned char* mask, const void* X, void* C, int64_t n, DType t,
                        hipStream_t s) {
  if (n == 0) return hipSuccess;
  const dim3 g((unsigned)((n + 1023) / 1024));
  if (t == DT_F64)
    hipLaunchKernelGGL(masked_merge_kernel<double>, g, dim3(256), 0, s, (const double*)M, mask, (const double*)X,
                       (double*)C, n);
  else
    hipLaunchKernelGGL(masked_merge_kernel<float>, g, dim3(256), 0, s, (const float*)M, mask, (const float*)X,
                       (float*)C, n);
  return hipGetLastError();
}

// Adjoint through the rank-k truncation: the eigenvector coupling across the
// cut.  One thread per entry (x, y) of slice f.
__global__ void gap_weights_kernel(const cx<double>* __restrict__ M, const double* __restrict__ lam, int m, int k,
                                   int64_t total, double rel_tol, cx<double>* __restrict__ S, int* __restrict__ info) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int64_t per = (int64_t)m * m;
  const int64_t f = t / per;
  const int x = (int)((t - f * per) / m), y = (int)((t - f * per) % m);
  cx<double> out{0.0, 0.0};
  if ((x < k) != (y < k)) {
    const double* l = lam + f * m;
    const int a = x < y ? x : y, c = x < y ? y : x;  // a in the top k, c outside it
    const double gap = l[a] - l[c];
    if (gap > rel_tol * l[0]) {
      const cx<double> mxy = M[t], myx = M[f * per + (int64_t)y * m + x];
      out = cx<double>{(mxy.re + myx.re) / gap, (mxy.im - myx.im) / gap};
    } else if (x < y) {
      atomicAdd(&info[INFO_TIE], 1);
    }
  }
  S[t] = out;
}
hipError_t gap_weights(const void* M, const double* lambda, int m, int k, int batch, double rel_tol, void* S,
                       int* info, hipStream_t s) {
  const int64_t total = (int64_t)batch * m * m;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(gap_weights_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     (const cx<double>*)M, lambda, m, k, total, rel_tol, (cx<double>*)S, info);
  return hipGetLastError();
}

// Second pass of the FP64 small SVD.  tail_split: per slice, the number J of
// leading eigenpairs of the first pass that are kept: the largest J < k with
// lambda_{J-1} >= tau lambda_0 and lambda_{J-1} / lambda_J >= min_ratio (no
// such J: J = k, the first pass is kept whole); W1m = W1 with the columns
// from J on cleared.
__global__ void tail_split_kernel(const double* __restrict__ lam1, const cx<double>* __restrict__ W1,
                                  cx<double>* __restrict__ W1m, int m, int k, double tau, double min_ratio,
                                  int* __restrict__ J) {
  __shared__ int js;
  const int f = blockIdx.x;
  if (threadIdx.x == 0) {
    const double* l = lam1 + (int64_t)f * k;
    int best = 0;
    for (int j = 1; j < k; ++j) {
      const double a = l[j - 1], bj = l[j];
      if (a >= tau * l[0] && (bj <= 0.0 || a >= min_ratio * bj)) best = j;
    }
    if (best == 0) best = k;
    js = best;
    J[f] = best;
  }
  __syncthreads();
  const int jf = js;
  const int64_t per = (int64_t)m * k;
  for (int64_t e = threadIdx.x; e < per; e += blockDim.x) {
    const int c = (int)(e % k);
    W1m[(int64_t)f * per + e] = c < jf ? W1[(int64_t)f * per + e] : cx<double>{0.0, 0.0};
  }
}
hipError_t tail_split(const double* lam1, const void* W1, void* W1m, int m, int k, int batch, double tau,
                      double min_ratio, int* J, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(tail_split_kernel, dim3(batch), dim3(256), 0, s, lam1, (const cx<double>*)W1, (cx<double>*)W1m,
                     m, k, tau, min_ratio, J);
  return hipGetLastError();
}

// merge: column c of the result takes the first pass's eigenpair c when
// c < J, else the second pass's eigenpair c - J.
__global__ void tail_merge_kernel(const double* __restrict__ lam1, const cx<double>* __restrict__ W1,
                                  const double* __restrict__ lam2, const cx<double>* __restrict__ W2,
                                  const int* __restrict__ J, int m, int k, int batch, double* __restrict__ lam,
                                  cx<double>* __restrict__ W) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)m * k;
  if (t >= per * batch) return;
  const int f = (int)(t / per);
  const int64_t e = t % per;
  const int r = (int)(e / k), c = (int)(e % k);
  const int jf = J[f];
  const int64_t base = (int64_t)f * per + (int64_t)r * k;
  W[t] = c < jf ? W1[base + c] : W2[base + (c - jf)];
  if (r == 0) lam[(int64_t)f * k + c] = c < jf ? lam1[(int64_t)f * k + c] : lam2[(int64_t)f * k + (c - jf)];
}
hipError_t tail_merge(const double* lam1, const void* W1, const double* lam2, const void* W2, const int* J, int m,
                      int k, int batch, double* lam, void* W, hipStream_t s) {
  const int64_t tot = (int64_t)m * k * batch;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(tail_merge_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, lam1,
                     (const cx<double>*)W1, lam2, (const cx<double>*)W2, J, m, k, batch, lam, (cx<double>*)W);
  return hipGetLastError();
}

// Phase convention: for every slice f and column j, find the entry of U_f(:, j)
// of largest modulus (lowest row index on ties) and multiply U_f(:, j) and
// V_f(:, j) by the conjugate of its phase, so that entry becomes real positive.
// Three coalesced passes (rows of U_f are contiguous over j):
//  1. partial column maxima of |U_f(i, j)|^2 over chunks of rows;
//  2. per (f, j): the chunk results combined in chunk order, and the phase;
//  3. U_f and V_f scaled elementwise.
constexpr int CANON_MAXCH = 64;  // row chunks per slice

static int canon_chunk_rows(int64_t n1) {
  const int64_t cr = (n1 + CANON_MAXCH - 1) / CANON_MAXCH;
  return (int)std::max<int64_t>(64, cr);
}

size_t canon_scratch_bytes(int64_t n1, int k, int batch) {
  const int64_t nch = (n1 + canon_chunk_rows(n1) - 1) / canon_chunk_rows(n1);
  // partial maxima (as double) and row indices, then one complex double phase per column
  return (size_t)batch * k * (size_t)(nch * (8 + 4) + 16) + 256;
}

template <typename T>
__global__ __launch_bounds__(256) void canon_colmax_kernel(const cx<T>* __restrict__ U, int64_t n1, int k, int cr,
                                                           double* __restrict__ pv, int* __restrict__ pi) {
  const int ch = blockIdx.x, nch = gridDim.x;
  const int64_t f = blockIdx.y;
  const cx<T>* u = U + f * n1 * k;
  const int64_t r0 = (int64_t)ch * cr, r1 = min(n1, r0 + cr);
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    T best = -1;
    int bi = 0x7fffffff;
    for (int64_t i = r0; i < r1; ++i) {
      const cx<T> a = u[i * k + j];
      const T m2 = a.re * a.re + a.im * a.im;
      if (m2 > best) {
        best = m2;
        bi = (int)i;
      }
    }
    pv[(f * nch + ch) * k + j] = (double)best;
    pi[(f * nch + ch) * k + j] = bi;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void canon_pick_kernel(const cx<T>* __restrict__ U, int64_t n1, int k, int nch,
                                                         const double* __restrict__ pv, const int* __restrict__ pi,
                                                         cx<double>* __restrict__ ph) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t f = blockIdx.y;
  if (j >= k) return;
  double best = -1;
  int bi = 0x7fffffff;
  for (int ch = 0; ch < nch; ++ch) {  // chunks in row order: a tie keeps the lower row
    const double v = pv[(f * nch + ch) * k + j];
    if (v > best) {
      best = v;
      bi = pi[(f * nch + ch) * k + j];
    }
  }
  T c = 1, s = 0;
  if (best > 0) {
    const cx<T> a = U[f * n1 * k + (int64_t)bi * k + j];
    const T r = sqrt(a.re * a.re + a.im * a.im);
    c = a.re / r;
    s = -a.im / r;  // conj(phase)
  }
  ph[f * k + j] = cx<double>{(double)c, (double)s};
}

template <typename T>
__global__ __launch_bounds__(256) void canon_scale_kernel(cx<T>* __restrict__ X, int64_t rows, int k, int batch,
                                                          const cx<double>* __restrict__ ph) {
  const int64_t per = rows * k, total = per * batch;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t f = e / per;
    const int j = (int)(e % k);
    const cx<double> p = ph[f * k + j];
    const T c = (T)p.re, s = (T)p.im;
    const cx<T> a = X[e];
    X[e] = cx<T>{a.re * c - a.im * s, a.re * s + a.im * c};
  }
}

template <typename T>
static hipError_t canon_t(cx<T>* U, int64_t n1, cx<T>* V, int64_t n2, int k, int batch, void* scratch,
                          hipStream_t s) {
  const int cr = canon_chunk_rows(n1);
  const int nch = (int)((n1 + cr - 1) / cr);
  unsigned char* w = static_cast<unsigned char*>(scratch);
  double* pv = reinterpret_cast<double*>(w);
  int* pi = reinterpret_cast<int*>(w + (size_t)batch * nch * k * 8);
  cx<double>* ph = reinterpret_cast<cx<double>*>(w + (((size_t)batch * nch * k * 12 + 255) & ~(size_t)255));
  hipLaunchKernelGGL(canon_colmax_kernel<T>, dim3(nch, batch), dim3(256), 0, s, U, n1, k, cr, pv, pi);
  hipLaunchKernelGGL(canon_pick_kernel<T>, dim3((k + 255) / 256, batch), dim3(256), 0, s, U, n1, k, nch, pv, pi, ph);
  const int64_t nu = n1 * k * batch, nv = n2 * k * batch;
  hipLaunchKernelGGL(canon_scale_kernel<T>, dim3((unsigned)std::min<int64_t>((nu + 255) / 256, 8192)), dim3(256), 0,
                     s, U, n1, k, batch, ph);
  hipLaunchKernelGGL(canon_scale_kernel<T>, dim3((unsigned)std::min<int64_t>((nv + 255) / 256, 8192)), dim3(256), 0,
                     s, V, n2, k, batch, ph);
  return hipGetLastError();
}

hipError_t canon_phase(void* U, int64_t n1, void* V, int64_t n2, int k, int batch, DType t, void* scratch,
                       hipStream_t s) {
  if (batch == 0 || k == 0) return hipSuccess;
  if (t == DT_F64) return canon_t<double>((cx<double>*)U, n1, (cx<double>*)V, n2, k, batch, scratch, s);
  return canon_t<float>((cx<float>*)U, n1, (cx<float>*)V, n2, k, batch, scratch, s);
}

}  // namespace tsvd
