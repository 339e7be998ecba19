// Batched complex GEMM on gfx950 MFMA (16x16x4 f32 / f64).
//
// Complex products use four real MFMA streams per output tile
// (re += ar br - ai bi, im += ar bi + ai br); operands are staged through LDS
// in planar re / im arrays whose layout follows the global layout so that
// both the coalesced global loads and the MFMA fragment reads stay
// bank-conflict-light.  One 256-thread workgroup (4 waves) owns a BM x BN
// output tile; each wave owns a (BM/WM) x (BN/WN) sub-tile of 16x16 MFMA
// tiles.  The K loop double-buffers through registers: the next K tile is
// fetched from HBM while the current one is multiplied out of LDS.
#include "common.h"
#include "kernels.h"

namespace tsvd {

template <typename S, typename T>
__device__ __forceinline__ void ld_cx(const void* base, int64_t idx, T& re, T& im) {
  const cx<S> v = reinterpret_cast<const cx<S>*>(base)[idx];
  re = static_cast<T>(v.re);
  im = static_cast<T>(v.im);
}

template <typename TAs, typename TBs, typename TCs, typename T, bool AC, bool BC, int BM, int BN, int BK, int WM,
          int WN>
__global__ __launch_bounds__(256) void zgemm_kernel(const GemmDesc d) {
  constexpr int NT = 256;
  static_assert(WM * WN == 4, "4 waves");
  constexpr int TM = BM / WM / 16;
  constexpr int TN = BN / WN / 16;
  static_assert(TM >= 1 && TN >= 1, "tile");
  constexpr int SA = AC ? (BM + 16) : (BK + 1);  // AC: [k][m], else [m][k]
  constexpr int SB = BC ? (BK + 1) : (BN + 16);  // BC: [n][k], else [k][n]
  constexpr int A_ELEMS = AC ? BK * SA : BM * SA;
  constexpr int B_ELEMS = BC ? BN * SB : BK * SB;
  constexpr int EA = BM * BK / NT;
  constexpr int EB = BK * BN / NT;
  static_assert(EA * NT == BM * BK && EB * NT == BK * BN, "load split");
  typedef typename Mfma<T>::acc_t acc_t;

  __shared__ T sAr[A_ELEMS], sAi[A_ELEMS], sBr[B_ELEMS], sBi[B_ELEMS];

  const int tid = threadIdx.x;
  const int f = blockIdx.z % d.batch;
  const int split = blockIdx.z / d.batch;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const int M = d.M, N = d.N;
  int kbeg = 0, kend = d.K;
  if (d.nsplit > 1) {
    kbeg = split * d.kchunk;
    kend = min(d.K, kbeg + d.kchunk);
  }
  const cx<TAs>* Ab = reinterpret_cast<const cx<TAs>*>(d.A) + (int64_t)f * d.strideA;
  const cx<TBs>* Bb = reinterpret_cast<const cx<TBs>*>(d.B) + (int64_t)f * d.strideB;

  T ra_r[EA], ra_i[EA], rb_r[EB], rb_i[EB];

  auto gload = [&](int kt) {
#pragma unroll
    for (int i = 0; i < EA; ++i) {
      const int e = tid + i * NT;
      const int m = AC ? (e % BM) : (e / BK);
      const int k = AC ? (e / BM) : (e % BK);
      const int gm = m0 + m, gk = kt + k;
      T re = 0, im = 0;
      if (gm < M && gk < kend) {
        const int64_t idx = AC ? ((int64_t)gk * d.lda + gm) : ((int64_t)gm * d.lda + gk);
        ld_cx<TAs, T>(Ab, idx, re, im);
        if (AC) im = -im;
      }
      ra_r[i] = re;
      ra_i[i] = im;
    }
#pragma unroll
    for (int i = 0; i < EB; ++i) {
      const int e = tid + i * NT;
      const int n = BC ? (e / BK) : (e % BN);
      const int k = BC ? (e % BK) : (e / BN);
      const int gn = n0 + n, gk = kt + k;
      T re = 0, im = 0;
      if (gn < N && gk < kend) {
        const int64_t idx = BC ? ((int64_t)gn * d.ldb + gk) : ((int64_t)gk * d.ldb + gn);
        for (int j = 0; j < d.b_nsum; ++j) {
          T r2, i2;
          ld_cx<TBs, T>(Bb + j * d.b_sum_stride, idx, r2, i2);
          re += r2;
          im += i2;
        }
        if (BC) im = -im;
      }
      rb_r[i] = re;
      rb_i[i] = im;
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int i = 0; i < EA; ++i) {
      const int e = tid + i * NT;
      const int m = AC ? (e % BM) : (e / BK);
      const int k = AC ? (e / BM) : (e % BK);
      const int s = AC ? (k * SA + m) : (m * SA + k);
      sAr[s] = ra_r[i];
      sAi[s] = ra_i[i];
    }
#pragma unroll
    for (int i = 0; i < EB; ++i) {
      const int e = tid + i * NT;
      const int n = BC ? (e / BK) : (e % BN);
      const int k = BC ? (e % BK) : (e / BN);
      const int s = BC ? (n * SB + k) : (k * SB + n);
      sBr[s] = rb_r[i];
      sBi[s] = rb_i[i];
    }
  };

  const int lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave % WM) * (BM / WM), wn0 = (wave / WM) * (BN / WN);
  const int r16 = lane & 15, q4 = lane >> 4;

  acc_t acc_r[TM][TN], acc_i[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      acc_r[a][b] = acc_t{0, 0, 0, 0};
      acc_i[a][b] = acc_t{0, 0, 0, 0};
    }

  if (kbeg < kend) gload(kbeg);
  for (int kt = kbeg; kt < kend; kt += BK) {
    __syncthreads();
    sstore();
    __syncthreads();
    if (kt + BK < kend) gload(kt + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kq = kk + q4;
      T ar[TM], ai[TM], nai[TM], br[TN], bi[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) {
        const int m = wm0 + a * 16 + r16;
        const int s = AC ? (kq * SA + m) : (m * SA + kq);
        ar[a] = sAr[s];
        ai[a] = sAi[s];
        nai[a] = -ai[a];
      }
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        const int n = wn0 + b * 16 + r16;
        const int s = BC ? (n * SB + kq) : (kq * SB + n);
        br[b] = sBr[s];
        bi[b] = sBi[s];
      }
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc_r[a][b] = Mfma<T>::run(ar[a], br[b], acc_r[a][b]);
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc_i[a][b] = Mfma<T>::run(ar[a], bi[b], acc_i[a][b]);
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc_r[a][b] = Mfma<T>::run(nai[a], bi[b], acc_r[a][b]);
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc_i[a][b] = Mfma<T>::run(ai[a], br[b], acc_i[a][b]);
    }
  }

  // epilogue
  cx<TCs>* Cb = reinterpret_cast<cx<TCs>*>(d.C) + (int64_t)f * d.strideC;
  if (d.nsplit > 1) Cb += (int64_t)split * d.c_split_stride;
  const T alpha = static_cast<T>(d.alpha);
  const T beta = static_cast<T>(d.beta);
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm0 + a * 16 + Mfma<T>::row(q4, r);
        const int gn = n0 + wn0 + b * 16 + r16;
        if (gm < M && gn < N) {
          const int64_t idx = (int64_t)gm * d.ldc + gn;
          T vr = alpha * acc_r[a][b][r];
          T vi = alpha * acc_i[a][b][r];
          if (d.nsplit <= 1 && d.beta != 0.0) {
            const cx<TCs> o = Cb[idx];
            vr += beta * static_cast<T>(o.re);
            vi += beta * static_cast<T>(o.im);
          }
          cx<TCs> out;
          out.re = static_cast<TCs>(vr);
          out.im = static_cast<TCs>(vi);
          Cb[idx] = out;
        }
      }
}

template <typename TAs, typename TBs, typename TCs, typename T, bool AC, bool BC>
static hipError_t launch(const GemmDesc& d, hipStream_t s) {
  constexpr int BM = 64, BN = 64, BK = 16;
  dim3 grid((d.M + BM - 1) / BM, (d.N + BN - 1) / BN, d.batch * (d.nsplit > 1 ? d.nsplit : 1));
  if (grid.x == 0 || grid.y == 0 || grid.z == 0) return hipSuccess;
  hipLaunchKernelGGL((zgemm_kernel<TAs, TBs, TCs, T, AC, BC, BM, BN, BK, 2, 2>), grid, dim3(256), 0, s, d);
  return hipGetLastError();
}

template <typename TAs, typename TBs, typename TCs, typename T>
static hipError_t launch_conj(const GemmDesc& d, hipStream_t s) {
  if (!d.a_conj && !d.b_conj) return launch<TAs, TBs, TCs, T, false, false>(d, s);
  if (d.a_conj && !d.b_conj) return launch<TAs, TBs, TCs, T, true, false>(d, s);
  if (!d.a_conj && d.b_conj) return launch<TAs, TBs, TCs, T, false, true>(d, s);
  return hipErrorInvalidValue;
}

hipError_t zgemm(const GemmDesc& d, hipStream_t s) {
  if (d.M <= 0 || d.N <= 0 || d.batch <= 0) return hipSuccess;
  if (d.nsplit > 1 && d.beta != 0.0) return hipErrorInvalidValue;
  const DType a = d.ta, b = d.tb, c = d.tc, t = d.compute;
  if (a == DT_F32 && b == DT_F32 && c == DT_F32 && t == DT_F32) return launch_conj<float, float, float, float>(d, s);
  if (a == DT_F64 && b == DT_F64 && c == DT_F64 && t == DT_F64) return launch_conj<double, double, double, double>(d, s);
  if (a == DT_F32 && b == DT_F32 && c == DT_F64 && t == DT_F64) return launch_conj<float, float, double, double>(d, s);
  if (a == DT_F32 && b == DT_F64 && c == DT_F32 && t == DT_F64) return launch_conj<float, double, float, double>(d, s);
  if (a == DT_F32 && b == DT_F64 && c == DT_F32 && t == DT_F32) return launch_conj<float, double, float, float>(d, s);
  if (a == DT_F64 && b == DT_F32 && c == DT_F32 && t == DT_F64) return launch_conj<double, float, float, double>(d, s);
  return hipErrorInvalidValue;
}

}  // namespace tsvd
