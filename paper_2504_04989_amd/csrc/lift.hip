// Small element-wise kernels around the lift of Alg. 2 (U_f = Q_f W_k,
// V_f = C_f^H W_k diag(1/sigma)) and the phase convention of the outputs.
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

// Phase convention: for every slice f and column j, find the entry of U_f(:, j)
// of largest modulus (lowest row index on ties) and multiply U_f(:, j) and
// V_f(:, j) by the conjugate of its phase, so that entry becomes real positive.
// One workgroup per (f, j).
template <typename T>
__global__ __launch_bounds__(256) void canon_kernel(cx<T>* U, int64_t n1, cx<T>* V, int64_t n2, int k) {
  __shared__ T sv[4];
  __shared__ int si[4];
  __shared__ T s_c, s_s;
  const int j = blockIdx.x;
  const int64_t f = blockIdx.y;
  cx<T>* u = U + f * n1 * k + j;
  cx<T>* v = V + f * n2 * k + j;
  T best = -1;
  int bi = 0x7fffffff;
  for (int64_t i = threadIdx.x; i < n1; i += 256) {
    const cx<T> a = u[i * k];
    const T m2 = a.re * a.re + a.im * a.im;
    if (m2 > best) {
      best = m2;
      bi = (int)i;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const T ob = __shfl_xor(best, off, 64);
    const int oi = __shfl_xor(bi, off, 64);
    if (ob > best || (ob == best && oi < bi)) {
      best = ob;
      bi = oi;
    }
  }
  if ((threadIdx.x & 63) == 0) {
    sv[threadIdx.x >> 6] = best;
    si[threadIdx.x >> 6] = bi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    T b = sv[0];
    int i0 = si[0];
    for (int w = 1; w < 4; ++w)
      if (sv[w] > b || (sv[w] == b && si[w] < i0)) {
        b = sv[w];
        i0 = si[w];
      }
    T c = 1, s = 0;
    if (b > 0) {
      const cx<T> a = u[(int64_t)i0 * k];
      const T r = sqrt(a.re * a.re + a.im * a.im);
      c = a.re / r;
      s = -a.im / r;  // conj(phase)
    }
    s_c = c;
    s_s = s;
  }
  __syncthreads();
  const T c = s_c, s = s_s;
  for (int64_t i = threadIdx.x; i < n1; i += 256) {
    const cx<T> a = u[i * k];
    u[i * k] = cx<T>{a.re * c - a.im * s, a.re * s + a.im * c};
  }
  for (int64_t i = threadIdx.x; i < n2; i += 256) {
    const cx<T> a = v[i * k];
    v[i * k] = cx<T>{a.re * c - a.im * s, a.re * s + a.im * c};
  }
}
hipError_t canon_phase(void* U, int64_t n1, void* V, int64_t n2, int k, int batch, DType t, hipStream_t s) {
  if (batch == 0 || k == 0) return hipSuccess;
  const dim3 g(k, batch);
  if (t == DT_F64)
    hipLaunchKernelGGL(canon_kernel<double>, g, dim3(256), 0, s, (cx<double>*)U, n1, (cx<double>*)V, n2, k);
  else
    hipLaunchKernelGGL(canon_kernel<float>, g, dim3(256), 0, s, (cx<float>*)U, n1, (cx<float>*)V, n2, k);
  return hipGetLastError();
}

}  // namespace tsvd
