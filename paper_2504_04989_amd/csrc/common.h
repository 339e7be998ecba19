// Shared device/host definitions for the gfx950 T-SVD kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tsvd {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// Interleaved complex value, 8 B (float) or 16 B (double) aligned so a
// complex element moves with one vector load/store.
template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};

// 16x16x4 MFMA: D(16x16) += A(16x4) B(4x16).  Lane l supplies A[l%16][l/16]
// and B[l/16][l%16].  Accumulator r of lane l holds D[row(l/16, r)][l%16]:
// row = 4*(l/16) + r for f32 and (l/16) + 4*r for f64 (measured on gfx950).
template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  typedef f32x4 acc_t;
  static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int q4, int r) { return 4 * q4 + r; }
};
template <>
struct Mfma<double> {
  typedef f64x4 acc_t;
  static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int q4, int r) { return q4 + 4 * r; }
};

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-wide sum for blockDim.x == NT (multiple of 64); `red` holds NT/64
// entries of shared memory.  All threads receive the result.
template <int NT, typename T>
__device__ __forceinline__ T block_sum(T v, T* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  T s = 0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) s += red[i];
  return s;
}

// Diagnostic counters kept at the start of the workspace.
enum { INFO_CHOL_SHIFTED = 0, INFO_CHOL_BREAKDOWN = 1, INFO_EIG_NOCONV = 2, INFO_NONFINITE = 3, INFO_TIE = 4,
       INFO_COUNT = 8 };

}  // namespace tsvd
