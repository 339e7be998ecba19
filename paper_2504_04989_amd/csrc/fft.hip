// Mode-3 DFT of a real third-order tensor and its inverse (Sec. 2: DFT along
// the tubes; Alg. TP: only the first n3/2 + 1 Fourier slices are formed, the
// others follow by conjugate symmetry).
//
// Layout: the real tensor is tube-contiguous (ntubes x n3); the spectrum is
// slice-major (F x ntubes, interleaved complex), which is the per-slice
// row-major matrix layout the GEMMs consume.
//
// Arithmetic is FP64 for both storage types (FP32 data is widened on load and
// rounded once on store).  One workgroup owns 2*NP consecutive tubes.  The tubes are read from HBM
// with fully coalesced loads, two real tubes are packed into one complex
// sequence z = x_a + i x_b in LDS, a self-sorting (Stockham) mixed-radix FFT
// with radices 2, 3, 4, 5, 7, 11, 13 runs out of LDS, and the two real
// spectra are separated with X_a[f] = (Z[f] + conj Z[-f]) / 2,
// X_b[f] = (Z[f] - conj Z[-f]) / (2i) while writing the slice-major output
// (coalesced across tubes).  The inverse packs two Hermitian half spectra
// the same way.  Lengths with a prime factor above 13 use a direct DFT.
#include "common.h"
#include "kernels.h"

namespace tsvd {

struct FftPlan {
  int N;
  int nf;
  int fac[24];
  int direct;  // 1: no supported factorisation, use the direct DFT
};

static FftPlan make_plan(int N) {
  FftPlan p{};
  p.N = N;
  int n = N;
  const int radices[] = {4, 2, 3, 5, 7, 11, 13};
  for (int r : radices)
    while (n % r == 0 && p.nf < 24) {
      p.fac[p.nf++] = r;
      n /= r;
    }
  p.direct = (n != 1);
  return p;
}

template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return cx<T>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cx<T> cconj(cx<T> a) {
  return cx<T>{a.re, -a.im};
}

// exp(-2 pi i t / N) for t = 0..N-1, computed in FP64 (exact at the quarter points).
template <typename T>
__device__ void make_twiddles(cx<T>* tw, int N) {
  for (int t = threadIdx.x; t < N; t += blockDim.x) {
    double s, c;
    sincospi(-2.0 * (double)t / (double)N, &s, &c);
    tw[t] = cx<T>{(T)c, (T)s};
  }
}

// One Stockham pass with radix R: Ns = product of the radices already done.
// Butterfly j of a length-N sequence reads in[j + r N/R], multiplies by the
// twiddle w^(r k N/(Ns R)) (k = j mod Ns), takes a length-R DFT and writes
// out[(j / Ns) Ns R + k + r Ns].
template <typename T, bool INV, int R>
__device__ void stockham_pass(const cx<T>* in, cx<T>* out, const cx<T>* tw, int N, int Ns, int NP) {
  const int nb = N / R;
  const int tws = N / (Ns * R);
  const int SP = N + 1;  // padded sequence stride (LDS banks)
  for (int idx = threadIdx.x; idx < NP * nb; idx += blockDim.x) {
    const int p = idx / nb;
    const int j = idx - p * nb;
    const int k = j % Ns;
    const cx<T>* a = in + p * SP;
    cx<T>* o = out + p * SP;
    cx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      cx<T> x = a[j + r * nb];
      if (r > 0) {
        cx<T> w = tw[(r * k * tws) % N];
        if (INV) w = cconj(w);
        x = cmul(x, w);
      }
      v[r] = x;
    }
    cx<T> V[R];
    if (R == 2) {
      V[0] = cx<T>{v[0].re + v[1].re, v[0].im + v[1].im};
      V[1] = cx<T>{v[0].re - v[1].re, v[0].im - v[1].im};
    } else if (R == 4) {
      const cx<T> t0{v[0].re + v[2].re, v[0].im + v[2].im};
      const cx<T> t1{v[0].re - v[2].re, v[0].im - v[2].im};
      const cx<T> t2{v[1].re + v[3].re, v[1].im + v[3].im};
      const cx<T> d{v[1].re - v[3].re, v[1].im - v[3].im};
      // forward: t3 = -i d ; inverse: t3 = +i d
      const cx<T> t3 = INV ? cx<T>{-d.im, d.re} : cx<T>{d.im, -d.re};
      V[0] = cx<T>{t0.re + t2.re, t0.im + t2.im};
      V[2] = cx<T>{t0.re - t2.re, t0.im - t2.im};
      V[1] = cx<T>{t1.re + t3.re, t1.im + t3.im};
      V[3] = cx<T>{t1.re - t3.re, t1.im - t3.im};
    } else {
      const int st = N / R;
#pragma unroll
      for (int s = 0; s < R; ++s) {
        cx<T> acc = v[0];
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cx<T> w = tw[((r * s) % R) * st];
          if (INV) w = cconj(w);
          const cx<T> y = cmul(v[r], w);
          acc.re += y.re;
          acc.im += y.im;
        }
        V[s] = acc;
      }
    }
    const int base = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) o[base + r * Ns] = V[r];
  }
}

template <typename T, bool INV>
__device__ cx<T>* run_passes(cx<T>* b0, cx<T>* b1, const cx<T>* tw, const FftPlan& plan, int NP) {
  cx<T>* in = b0;
  cx<T>* out = b1;
  int Ns = 1;
  for (int s = 0; s < plan.nf; ++s) {
    const int R = plan.fac[s];
    switch (R) {
      case 2: stockham_pass<T, INV, 2>(in, out, tw, plan.N, Ns, NP); break;
      case 3: stockham_pass<T, INV, 3>(in, out, tw, plan.N, Ns, NP); break;
      case 4: stockham_pass<T, INV, 4>(in, out, tw, plan.N, Ns, NP); break;
      case 5: stockham_pass<T, INV, 5>(in, out, tw, plan.N, Ns, NP); break;
      case 7: stockham_pass<T, INV, 7>(in, out, tw, plan.N, Ns, NP); break;
      case 11: stockham_pass<T, INV, 11>(in, out, tw, plan.N, Ns, NP); break;
      default: stockham_pass<T, INV, 13>(in, out, tw, plan.N, Ns, NP); break;
    }
    __syncthreads();
    cx<T>* t = in;
    in = out;
    out = t;
    Ns *= R;
  }
  return in;
}

// T: storage type of the tensor and its spectrum; C: arithmetic type (FP64
// for FP32 storage, so that every output is the correctly rounded value of a
// DFT whose error is far below the FP32 rounding of the result).
template <typename T, typename C>
__global__ __launch_bounds__(256) void fft_r2c_kernel(const T* __restrict__ X, cx<T>* __restrict__ Xb, int64_t ntubes,
                                                      FftPlan plan, int NP) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int N = plan.N;
  cx<C>* tw = reinterpret_cast<cx<C>*>(smem);
  cx<C>* b0 = tw + N;
  const int SP = N + 1;
  cx<C>* b1 = b0 + NP * SP;
  make_twiddles(tw, N);
  const int64_t t0 = (int64_t)blockIdx.x * 2 * NP;
  const int ntw = (int)min((int64_t)2 * NP, ntubes - t0);
  const T* src = X + t0 * N;
  const int total = ntw * N;
  for (int g = threadIdx.x; g < 2 * NP * N; g += blockDim.x) {
    const int tube = g / N, t = g - tube * N;
    const C v = (g < total) ? (C)src[g] : (C)0;
    C* dst = reinterpret_cast<C*>(&b0[(tube >> 1) * SP + t]);
    dst[tube & 1] = v;
  }
  __syncthreads();
  const cx<C>* Z = run_passes<C, false>(b0, b1, tw, plan, NP);
  const int F = N / 2 + 1;
  for (int idx = threadIdx.x; idx < F * 2 * NP; idx += blockDim.x) {
    const int f = idx / (2 * NP), tube = idx - f * 2 * NP;
    if (tube >= ntw) continue;
    const int p = tube >> 1;
    const cx<C> zf = Z[p * SP + f];
    const cx<C> zm = Z[p * SP + (f == 0 ? 0 : N - f)];
    cx<T> o;
    if (!(tube & 1)) {
      o.re = (T)((zf.re + zm.re) * (C)0.5);
      o.im = (T)((zf.im - zm.im) * (C)0.5);
    } else {
      o.re = (T)((zf.im + zm.im) * (C)0.5);
      o.im = (T)((zm.re - zf.re) * (C)0.5);
    }
    Xb[(int64_t)f * ntubes + t0 + tube] = o;
  }
}

template <typename T, typename C>
__global__ __launch_bounds__(256) void fft_c2r_kernel(const cx<T>* __restrict__ Xb, int64_t slice_stride,
                                                      T* __restrict__ X, int64_t ntubes, FftPlan plan, int NP) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int N = plan.N;
  cx<C>* tw = reinterpret_cast<cx<C>*>(smem);
  cx<C>* b0 = tw + N;
  const int SP = N + 1;
  cx<C>* b1 = b0 + NP * SP;
  make_twiddles(tw, N);
  const int64_t t0 = (int64_t)blockIdx.x * 2 * NP;
  const int ntw = (int)min((int64_t)2 * NP, ntubes - t0);
  const int F = N / 2 + 1;
  for (int idx = threadIdx.x; idx < F * NP; idx += blockDim.x) {
    const int f = idx / NP, p = idx - f * NP;
    const int ta = 2 * p, tb = 2 * p + 1;
    cx<C> a{0, 0}, b{0, 0};
    if (ta < ntw) {
      const cx<T> v = Xb[(int64_t)f * slice_stride + t0 + ta];
      a = cx<C>{(C)v.re, (C)v.im};
    }
    if (tb < ntw) {
      const cx<T> v = Xb[(int64_t)f * slice_stride + t0 + tb];
      b = cx<C>{(C)v.re, (C)v.im};
    }
    if (f == 0 || 2 * f == N) {
      a.im = 0;
      b.im = 0;
    }
    b0[p * SP + f] = cx<C>{a.re - b.im, a.im + b.re};
    if (f > 0 && 2 * f != N) b0[p * SP + (N - f)] = cx<C>{a.re + b.im, b.re - a.im};
  }
  __syncthreads();
  const cx<C>* Z = run_passes<C, true>(b0, b1, tw, plan, NP);
  const C invN = (C)1 / (C)N;
  const int total = ntw * N;
  T* dst = X + t0 * N;
  for (int g = threadIdx.x; g < total; g += blockDim.x) {
    const int tube = g / N, t = g - tube * N;
    const cx<C> z = Z[(tube >> 1) * SP + t];
    dst[g] = (T)(((tube & 1) ? z.im : z.re) * invN);
  }
}

// Direct DFT for lengths with a prime factor above 13: one thread per output.
template <typename T>
__global__ void dft_r2c_direct(const T* X, cx<T>* Xb, int64_t ntubes, int N) {
  const int F = N / 2 + 1;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ntubes * F) return;
  const int f = (int)(idx / ntubes);
  const int64_t tube = idx - (int64_t)f * ntubes;
  const T* x = X + tube * N;
  double re = 0, im = 0;
  for (int t = 0; t < N; ++t) {
    double s, c;
    sincospi(-2.0 * (double)(((int64_t)f * t) % N) / N, &s, &c);
    re += (double)x[t] * c;
    im += (double)x[t] * s;
  }
  if (f == 0 || 2 * f == N) im = 0;
  Xb[(int64_t)f * ntubes + tube] = cx<T>{(T)re, (T)im};
}

template <typename T>
__global__ void dft_c2r_direct(const cx<T>* Xb, int64_t slice_stride, T* X, int64_t ntubes, int N) {
  const int F = N / 2 + 1;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ntubes * N) return;
  const int64_t tube = idx / N;
  const int t = (int)(idx - tube * N);
  double acc = 0;
  for (int f = 0; f < F; ++f) {
    const cx<T> z = Xb[(int64_t)f * slice_stride + tube];
    double s, c;
    sincospi(2.0 * (double)(((int64_t)f * t) % N) / N, &s, &c);
    const double term = (double)z.re * c - (double)z.im * s;
    acc += (f == 0 || 2 * f == N) ? (double)z.re * c : 2.0 * term;
  }
  X[idx] = (T)(acc / N);
}

template <typename C>
static int pick_np(int N) {
  const int budget = 64 * 1024 / (int)sizeof(cx<C>);
  int np = (budget - N) / (2 * (N + 1));
  if (np > 64) np = 64;
  return np;
}

template <typename T>
static hipError_t r2c_t(const void* X, void* Xb, int64_t ntubes, int n3, hipStream_t s) {
  if (ntubes <= 0) return hipSuccess;
  FftPlan plan = make_plan(n3);
  const int NP = pick_np<double>(n3);
  if (plan.direct || NP < 1) {
    const int64_t total = ntubes * (n3 / 2 + 1);
    hipLaunchKernelGGL(dft_r2c_direct<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, (const T*)X,
                       (cx<T>*)Xb, ntubes, n3);
    return hipGetLastError();
  }
  const int64_t nblk = (ntubes + 2 * NP - 1) / (2 * NP);
  const size_t sm = (size_t)(n3 + 2 * NP * (n3 + 1)) * sizeof(cx<double>);
  hipLaunchKernelGGL((fft_r2c_kernel<T, double>), dim3((unsigned)nblk), dim3(256), sm, s, (const T*)X, (cx<T>*)Xb,
                     ntubes, plan, NP);
  return hipGetLastError();
}

template <typename T>
static hipError_t c2r_t(const void* Xb, int64_t stride, void* X, int64_t ntubes, int n3, hipStream_t s) {
  if (ntubes <= 0) return hipSuccess;
  FftPlan plan = make_plan(n3);
  const int NP = pick_np<double>(n3);
  if (plan.direct || NP < 1) {
    const int64_t total = ntubes * n3;
    hipLaunchKernelGGL(dft_c2r_direct<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       (const cx<T>*)Xb, stride, (T*)X, ntubes, n3);
    return hipGetLastError();
  }
  const int64_t nblk = (ntubes + 2 * NP - 1) / (2 * NP);
  const size_t sm = (size_t)(n3 + 2 * NP * (n3 + 1)) * sizeof(cx<double>);
  hipLaunchKernelGGL((fft_c2r_kernel<T, double>), dim3((unsigned)nblk), dim3(256), sm, s, (const cx<T>*)Xb, stride,
                     (T*)X, ntubes, plan, NP);
  return hipGetLastError();
}

bool fft_pow2_supported(int n3);
hipError_t fft_r2c_pow2(const void* X, void* Xb, int64_t ntubes, int n3, DType t, hipStream_t s);
hipError_t fft_c2r_pow2(const void* Xb, int64_t stride, void* X, int64_t ntubes, int n3, DType t, hipStream_t s);

bool fft_reg_supported(int n3, DType t);
hipError_t fft_r2c_reg(const void* X, void* Xb, int64_t ntubes, int n3, hipStream_t s);
hipError_t fft_c2r_reg(const void* Xb, int64_t stride, void* X, int64_t ntubes, int n3, hipStream_t s);

hipError_t fft_r2c(const void* X, void* Xb, int64_t ntubes, int n3, DType t, hipStream_t s) {
  if (fft_reg_supported(n3, t)) return fft_r2c_reg(X, Xb, ntubes, n3, s);
  if (fft_pow2_supported(n3)) return fft_r2c_pow2(X, Xb, ntubes, n3, t, s);
  return t == DT_F64 ? r2c_t<double>(X, Xb, ntubes, n3, s) : r2c_t<float>(X, Xb, ntubes, n3, s);
}

hipError_t fft_c2r(const void* Xb, int64_t slice_stride, void* X, int64_t ntubes, int n3, DType t, hipStream_t s) {
  if (fft_reg_supported(n3, t)) return fft_c2r_reg(Xb, slice_stride, X, ntubes, n3, s);
  if (fft_pow2_supported(n3)) return fft_c2r_pow2(Xb, slice_stride, X, ntubes, n3, t, s);
  return t == DT_F64 ? c2r_t<double>(Xb, slice_stride, X, ntubes, n3, s)
                     : c2r_t<float>(Xb, slice_stride, X, ntubes, n3, s);
}

}  // namespace tsvd

// ---------------------------------------------------------------------------
// Power-of-two lengths 8 <= N <= 256: compile-time length and radices (4,
// then a final 2 when log2 N is odd), FP64 arithmetic, sequences of a
// workgroup at a padded LDS stride of N + 1 complex elements (the untangle
// step reads element f of every sequence at once), float4 / double2 tube loads.
// ---------------------------------------------------------------------------
namespace tsvd {
namespace {

template <int N>
struct P2 {
  static constexpr int SP = N + 1;
  // tube pairs per workgroup: N twiddles + 2 buffers of NP sequences in ~40 KB
  static constexpr int NP0 = (40 * 1024 / 16 - N) / (2 * SP);
  static constexpr int NP = NP0 > 64 ? 64 : NP0;
};

// One Stockham pass of radix R on NPs sequences (stride SP) with Ns = product
// of the radices done so far; twiddles tw[t] = exp(-2 pi i t / N).
template <int N, int R, int Ns, bool INV>
__device__ __forceinline__ void p2_pass(const cx<double>* in, cx<double>* out, const cx<double>* tw, int NPs) {
  constexpr int nb = N / R;
  constexpr int tws = N / (Ns * R);
  constexpr int SP = P2<N>::SP;
  for (int idx = threadIdx.x; idx < NPs * nb; idx += blockDim.x) {
    const int p = idx / nb;  // compile-time divisor
    const int j = idx - p * nb;
    const int k = j % Ns;
    const cx<double>* a = in + p * SP;
    cx<double>* o = out + p * SP;
    cx<double> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      cx<double> x = a[j + r * nb];
      if (r > 0 && Ns > 1) {
        cx<double> w = tw[(r * k * tws) % N];
        if (INV) w.im = -w.im;
        x = cx<double>{x.re * w.re - x.im * w.im, x.re * w.im + x.im * w.re};
      }
      v[r] = x;
    }
    cx<double> V[R];
    if (R == 2) {
      V[0] = cx<double>{v[0].re + v[1].re, v[0].im + v[1].im};
      V[1] = cx<double>{v[0].re - v[1].re, v[0].im - v[1].im};
    } else {
      const cx<double> t0{v[0].re + v[2].re, v[0].im + v[2].im};
      const cx<double> t1{v[0].re - v[2].re, v[0].im - v[2].im};
      const cx<double> t2{v[1].re + v[3].re, v[1].im + v[3].im};
      const cx<double> d{v[1].re - v[3].re, v[1].im - v[3].im};
      const cx<double> t3 = INV ? cx<double>{-d.im, d.re} : cx<double>{d.im, -d.re};
      V[0] = cx<double>{t0.re + t2.re, t0.im + t2.im};
      V[2] = cx<double>{t0.re - t2.re, t0.im - t2.im};
      V[1] = cx<double>{t1.re + t3.re, t1.im + t3.im};
      V[3] = cx<double>{t1.re - t3.re, t1.im - t3.im};
    }
    const int base = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) o[base + r * Ns] = V[r];
  }
}

template <int N, int Ns, bool INV>
__device__ __forceinline__ cx<double>* p2_passes(cx<double>* in, cx<double>* out, const cx<double>* tw, int NPs) {
  if constexpr (Ns >= N) {
    return in;
  } else if constexpr (N / Ns >= 4) {
    p2_pass<N, 4, Ns, INV>(in, out, tw, NPs);
    __syncthreads();
    return p2_passes<N, Ns * 4, INV>(out, in, tw, NPs);
  } else {
    p2_pass<N, 2, Ns, INV>(in, out, tw, NPs);
    __syncthreads();
    return p2_passes<N, Ns * 2, INV>(out, in, tw, NPs);
  }
}

template <typename T, int N>
__global__ __launch_bounds__(256) void fft_r2c_p2_kernel(const T* __restrict__ X, cx<T>* __restrict__ Xb,
                                                         int64_t ntubes) {
  constexpr int NP = P2<N>::NP;
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int SP = P2<N>::SP;
  constexpr int F = N / 2 + 1;
  cx<double>* tw = reinterpret_cast<cx<double>*>(smem);
  cx<double>* b0 = tw + N;
  cx<double>* b1 = b0 + NP * SP;
  for (int t = threadIdx.x; t < N; t += blockDim.x) {
    double s, c;
    sincospi(-2.0 * (double)t / (double)N, &s, &c);
    tw[t] = cx<double>{c, s};
  }
  const int64_t t0 = (int64_t)blockIdx.x * 2 * NP;
  const int ntw = (int)min((int64_t)2 * NP, ntubes - t0);
  const T* src = X + t0 * N;
  // tubes are contiguous: 4 (FP32) or 2 (FP64) consecutive samples per
  // access; all of a thread's loads are issued before any is used
  constexpr int VW = sizeof(T) == 4 ? 4 : 2;
  constexpr int NVEC = 2 * NP * N / VW;
  constexpr int PERT = (NVEC + 255) / 256;
  const int lim = ntw * N;
  double v[PERT][VW];
#pragma unroll
  for (int it = 0; it < PERT; ++it) {
    const int e0 = (threadIdx.x + 256 * it) * VW;
    if (e0 < lim) {
      if constexpr (VW == 4) {
        const float4 x = *reinterpret_cast<const float4*>(src + e0);
        v[it][0] = x.x; v[it][1] = x.y; v[it][2] = x.z; v[it][3] = x.w;
      } else {
        const double2 x = *reinterpret_cast<const double2*>(src + e0);
        v[it][0] = x.x; v[it][1] = x.y;
      }
    } else {
#pragma unroll
      for (int i = 0; i < VW; ++i) v[it][i] = 0.0;
    }
  }
#pragma unroll
  for (int it = 0; it < PERT; ++it) {
    const int g = threadIdx.x + 256 * it;
    if (g < NVEC) {
      const int e0 = g * VW;
      const int tube = e0 / N, t = e0 - tube * N;  // compile-time divisor
      double* dst = reinterpret_cast<double*>(&b0[(tube >> 1) * SP + t]) + (tube & 1);
#pragma unroll
      for (int i = 0; i < VW; ++i) dst[2 * i] = v[it][i];
    }
  }
  __syncthreads();
  const cx<double>* Z = p2_passes<N, 1, false>(b0, b1, tw, NP);
  for (int idx = threadIdx.x; idx < F * 2 * NP; idx += blockDim.x) {
    const int f = idx / (2 * NP), tube = idx - f * 2 * NP;
    if (tube >= ntw) continue;
    const int p = tube >> 1;
    const cx<double> zf = Z[p * SP + f];
    const cx<double> zm = Z[p * SP + (f == 0 ? 0 : N - f)];
    cx<T> o;
    if (!(tube & 1)) {
      o.re = (T)(0.5 * (zf.re + zm.re));
      o.im = (T)(0.5 * (zf.im - zm.im));
    } else {
      o.re = (T)(0.5 * (zf.im + zm.im));
      o.im = (T)(0.5 * (zm.re - zf.re));
    }
    Xb[(int64_t)f * ntubes + t0 + tube] = o;
  }
}

template <typename T, int N>
__global__ __launch_bounds__(256) void fft_c2r_p2_kernel(const cx<T>* __restrict__ Xb, int64_t slice_stride,
                                                         T* __restrict__ X, int64_t ntubes) {
  constexpr int NP = P2<N>::NP;
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int SP = P2<N>::SP;
  constexpr int F = N / 2 + 1;
  cx<double>* tw = reinterpret_cast<cx<double>*>(smem);
  cx<double>* b0 = tw + N;
  cx<double>* b1 = b0 + NP * SP;
  for (int t = threadIdx.x; t < N; t += blockDim.x) {
    double s, c;
    sincospi(-2.0 * (double)t / (double)N, &s, &c);
    tw[t] = cx<double>{c, s};
  }
  const int64_t t0 = (int64_t)blockIdx.x * 2 * NP;
  const int ntw = (int)min((int64_t)2 * NP, ntubes - t0);
  for (int idx = threadIdx.x; idx < F * NP; idx += blockDim.x) {
    const int f = idx / NP, p = idx - f * NP;
    const int ta = 2 * p, tb = 2 * p + 1;
    cx<double> a{0, 0}, b{0, 0};
    if (ta < ntw) {
      const cx<T> v = Xb[(int64_t)f * slice_stride + t0 + ta];
      a = cx<double>{(double)v.re, (double)v.im};
    }
    if (tb < ntw) {
      const cx<T> v = Xb[(int64_t)f * slice_stride + t0 + tb];
      b = cx<double>{(double)v.re, (double)v.im};
    }
    if (f == 0 || 2 * f == N) {
      a.im = 0;
      b.im = 0;
    }
    b0[p * SP + f] = cx<double>{a.re - b.im, a.im + b.re};
    if (f > 0 && 2 * f != N) b0[p * SP + (N - f)] = cx<double>{a.re + b.im, b.re - a.im};
  }
  __syncthreads();
  const cx<double>* Z = p2_passes<N, 1, true>(b0, b1, tw, NP);
  constexpr double invN = 1.0 / N;
  const int total = ntw * N;
  T* dst = X + t0 * N;
  for (int g = threadIdx.x; g < total; g += blockDim.x) {
    const int tube = g / N, t = g - tube * N;
    const cx<double> z = Z[(tube >> 1) * SP + t];
    dst[g] = (T)(((tube & 1) ? z.im : z.re) * invN);
  }
}


template <typename T, int N>
hipError_t p2_r2c(const void* X, void* Xb, int64_t ntubes, hipStream_t s) {
  constexpr int NP = P2<N>::NP;
  const int64_t nblk = (ntubes + 2 * NP - 1) / (2 * NP);
  const size_t sm = (size_t)(N + 2 * NP * P2<N>::SP) * sizeof(cx<double>);
  hipLaunchKernelGGL((fft_r2c_p2_kernel<T, N>), dim3((unsigned)nblk), dim3(256), sm, s, (const T*)X, (cx<T>*)Xb,
                     ntubes);
  return hipGetLastError();
}

template <typename T, int N>
hipError_t p2_c2r(const void* Xb, int64_t stride, void* X, int64_t ntubes, hipStream_t s) {
  constexpr int NP = P2<N>::NP;
  const int64_t nblk = (ntubes + 2 * NP - 1) / (2 * NP);
  const size_t sm = (size_t)(N + 2 * NP * P2<N>::SP) * sizeof(cx<double>);
  hipLaunchKernelGGL((fft_c2r_p2_kernel<T, N>), dim3((unsigned)nblk), dim3(256), sm, s, (const cx<T>*)Xb, stride,
                     (T*)X, ntubes);
  return hipGetLastError();
}

template <typename T>
hipError_t p2_r2c_dispatch(const void* X, void* Xb, int64_t ntubes, int n3, hipStream_t s) {
  switch (n3) {
    case 8: return p2_r2c<T, 8>(X, Xb, ntubes, s);
    case 16: return p2_r2c<T, 16>(X, Xb, ntubes, s);
    case 32: return p2_r2c<T, 32>(X, Xb, ntubes, s);
    case 64: return p2_r2c<T, 64>(X, Xb, ntubes, s);
    case 128: return p2_r2c<T, 128>(X, Xb, ntubes, s);
    case 256: return p2_r2c<T, 256>(X, Xb, ntubes, s);
    default: return hipErrorNotSupported;
  }
}
template <typename T>
hipError_t p2_c2r_dispatch(const void* Xb, int64_t stride, void* X, int64_t ntubes, int n3, hipStream_t s) {
  switch (n3) {
    case 8: return p2_c2r<T, 8>(Xb, stride, X, ntubes, s);
    case 16: return p2_c2r<T, 16>(Xb, stride, X, ntubes, s);
    case 32: return p2_c2r<T, 32>(Xb, stride, X, ntubes, s);
    case 64: return p2_c2r<T, 64>(Xb, stride, X, ntubes, s);
    case 128: return p2_c2r<T, 128>(Xb, stride, X, ntubes, s);
    case 256: return p2_c2r<T, 256>(Xb, stride, X, ntubes, s);
    default: return hipErrorNotSupported;
  }
}

}  // namespace

bool fft_pow2_supported(int n3) { return n3 >= 8 && n3 <= 256 && (n3 & (n3 - 1)) == 0; }

hipError_t fft_r2c_pow2(const void* X, void* Xb, int64_t ntubes, int n3, DType t, hipStream_t s) {
  if (ntubes <= 0) return hipSuccess;
  return t == DT_F64 ? p2_r2c_dispatch<double>(X, Xb, ntubes, n3, s) : p2_r2c_dispatch<float>(X, Xb, ntubes, n3, s);
}
hipError_t fft_c2r_pow2(const void* Xb, int64_t stride, void* X, int64_t ntubes, int n3, DType t, hipStream_t s) {
  if (ntubes <= 0) return hipSuccess;
  return t == DT_F64 ? p2_c2r_dispatch<double>(Xb, stride, X, ntubes, n3, s)
                     : p2_c2r_dispatch<float>(Xb, stride, X, ntubes, n3, s);
}

}  // namespace tsvd

// ---------------------------------------------------------------------------
// FP32 tubes of length N in {8, 16, 32, 64}: one thread per tube, the whole
// transform in registers.  A workgroup moves 256 consecutive tubes between HBM
// and LDS with coalesced 16-byte accesses (FP32, padded row stride N + 4, so
// that the 16-byte per-thread row accesses are bank-conflict free); each thread
// then widens its own tube to FP64, packs it into the N/2-point complex sequence
// z[n] = x[2n] + i x[2n+1], runs an unrolled radix-2 decimation-in-frequency FFT
// with compile-time twiddles, separates the spectrum of the real tube
// X[f] = E[f] + w^f O[f] (E, O the spectra of the even and odd samples,
// w = exp(-2 pi i / N)) and writes X[0..N/2] slice-major, coalesced across the
// threads.  The inverse runs the same steps backwards.  LDS is touched once per
// sample in each direction, which keeps the kernel on the HBM roofline.
// ---------------------------------------------------------------------------
namespace tsvd {
namespace {

// cos and sin of 2 pi k / n at compile time: the angle is reduced to the first
// octant by exact integer arithmetic and the Taylor series is summed in FP64.
constexpr double ct_sin_poly(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int i = 1; i < 14; ++i) {
    term = -term * x2 / (double)((2 * i) * (2 * i + 1));
    sum += term;
  }
  return sum;
}
constexpr double ct_cos_poly(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int i = 1; i < 14; ++i) {
    term = -term * x2 / (double)((2 * i - 1) * (2 * i));
    sum += term;
  }
  return sum;
}
struct CtCS {
  double c, s;
};
constexpr CtCS ct_turn(int k, int n) {
  k %= n;
  if (k < 0) k += n;
  const int q = (4 * k) / n;      // quadrant
  const int rn = 4 * k - q * n;   // remainder, in units of (pi / 2) / n
  double cq = 1.0, sq = 0.0;
  if (rn != 0) {
    constexpr double half_pi = 1.57079632679489661923;
    if (2 * rn <= n) {
      const double phi = half_pi * (double)rn / (double)n;
      cq = ct_cos_poly(phi);
      sq = ct_sin_poly(phi);
    } else {
      const double psi = half_pi * (double)(n - rn) / (double)n;
      cq = ct_sin_poly(psi);
      sq = ct_cos_poly(psi);
    }
  }
  switch (q) {
    case 0: return CtCS{cq, sq};
    case 1: return CtCS{-sq, cq};
    case 2: return CtCS{-cq, -sq};
    default: return CtCS{sq, -cq};
  }
}

// cos / sin of 2 pi k / N for k < N, evaluated by the compiler
template <int N>
struct CtTab {
  double c[N], s[N];
  constexpr CtTab() : c(), s() {
    for (int k = 0; k < N; ++k) {
      const CtCS w = ct_turn(k, N);
      c[k] = w.c;
      s[k] = w.s;
    }
  }
};

constexpr int ct_bitrev(int v, int bits) {
  int r = 0;
  for (int i = 0; i < bits; ++i) r |= ((v >> i) & 1) << (bits - 1 - i);
  return r;
}
constexpr int ct_log2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// In-place M-point complex DFT (sign -1, or +1 when INV, unnormalised) of
// (re, im); the result is left in bit-reversed order.
template <int M, bool INV>
__device__ __forceinline__ void reg_dif(double (&re)[M], double (&im)[M]) {
  constexpr CtTab<M> tw{};
#pragma unroll
  for (int len = M; len >= 2; len >>= 1) {
    const int half = len >> 1;
#pragma unroll
    for (int i0 = 0; i0 < M; i0 += len) {
#pragma unroll
      for (int j = 0; j < half; ++j) {
        const int a = i0 + j, b = a + half;
        const double ur = re[a], ui = im[a], vr = re[b], vi = im[b];
        re[a] = ur + vr;
        im[a] = ui + vi;
        const double dr = ur - vr, di = ui - vi;
        const int e = j * (M / len);  // twiddle exp(-+2 pi i e / M)
        if (e == 0) {
          re[b] = dr;
          im[b] = di;
        } else if (4 * e == M) {  // -i (forward) or +i (inverse)
          re[b] = INV ? -di : di;
          im[b] = INV ? dr : -dr;
        } else {
          const double wr = tw.c[e], wi = INV ? tw.s[e] : -tw.s[e];
          re[b] = fma(dr, wr, -di * wi);
          im[b] = fma(dr, wi, di * wr);
        }
      }
    }
  }
}

#ifndef TSVD_FFT_REG_TUBES
#define TSVD_FFT_REG_TUBES 256
#endif
constexpr int REG_TUBES = TSVD_FFT_REG_TUBES;  // tubes (threads) per workgroup
#ifndef TSVD_FFT_NT
#define TSVD_FFT_NT 3
#endif
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
// streaming accesses: every sample and every spectrum entry is touched once
__device__ __forceinline__ float4 ld_stream4(const float4* p) {
#if TSVD_FFT_NT & 1
  const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
#else
  return *p;
#endif
}
__device__ __forceinline__ float2 ld_stream2(const float2* p) {
#if TSVD_FFT_NT & 1
  const f32x2 v = __builtin_nontemporal_load(reinterpret_cast<const f32x2*>(p));
  return make_float2(v.x, v.y);
#else
  return *p;
#endif
}
__device__ __forceinline__ void st_stream2(float2* p, float a, float b) {
#if TSVD_FFT_NT & 2
  f32x2 v;
  v.x = a;
  v.y = b;
  __builtin_nontemporal_store(v, reinterpret_cast<f32x2*>(p));
#else
  *p = make_float2(a, b);
#endif
}
__device__ __forceinline__ void st_stream4(float4* p, float4 x) {
#if TSVD_FFT_NT & 2
  f32x4 v;
  v.x = x.x;
  v.y = x.y;
  v.z = x.z;
  v.w = x.w;
  __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(p));
#else
  *p = x;
#endif
}

// One complex FP32 value z as the pair (hi, lo) of complex bf16 values with
// hi = bf16(z) and lo = bf16(z - hi) (round to nearest even), packed as
// (re_hi | im_hi << 16, re_lo | im_lo << 16): the operand form of the
// three-product BF16 Krylov products, 8 bytes like the FP32 value.
__device__ __forceinline__ void st_split2(float2* p, float a, float b) {
  const __bf16 ha = (__bf16)a, hb = (__bf16)b;
  const __bf16 la = (__bf16)(a - (float)ha), lb = (__bf16)(b - (float)hb);
  const uint32_t h = (uint32_t)__builtin_bit_cast(unsigned short, ha) |
                     ((uint32_t)__builtin_bit_cast(unsigned short, hb) << 16);
  const uint32_t l = (uint32_t)__builtin_bit_cast(unsigned short, la) |
                     ((uint32_t)__builtin_bit_cast(unsigned short, lb) << 16);
  st_stream2(p, __uint_as_float(h), __uint_as_float(l));
}

// SPLIT: the half spectrum is written as (hi, lo) bf16 pairs (st_split2)
// instead of complex FP32.
template <int N, bool SPLIT>
__global__ __launch_bounds__(REG_TUBES) void fft_r2c_reg_kernel(const float* __restrict__ X,
                                                                 float2* __restrict__ Xb, int64_t ntubes) {
  constexpr int M = N / 2, LB = ct_log2(M), SPF = N + 4;
  constexpr int NV = REG_TUBES * N / 4;  // float4 per workgroup
  __shared__ __align__(16) float buf[REG_TUBES * SPF];
  const int tid = threadIdx.x;
  const int64_t t0 = (int64_t)blockIdx.x * REG_TUBES;
  const int ntw = (int)min((int64_t)REG_TUBES, ntubes - t0);
  const int lim = ntw * (N / 4);
  const float4* src = reinterpret_cast<const float4*>(X + t0 * N);
  float4 v[NV / REG_TUBES];
#pragma unroll
  for (int it = 0; it < NV / REG_TUBES; ++it) {
    const int g = tid + REG_TUBES * it;
    v[it] = g < lim ? ld_stream4(src + g) : make_float4(0.f, 0.f, 0.f, 0.f);
  }
#pragma unroll
  for (int it = 0; it < NV / REG_TUBES; ++it) {
    const int g = tid + REG_TUBES * it;
    const int tube = g / (N / 4), c = g - tube * (N / 4);
    *reinterpret_cast<float4*>(&buf[tube * SPF + 4 * c]) = v[it];
  }
  __syncthreads();
  double re[M], im[M];
#pragma unroll
  for (int c = 0; c < N / 4; ++c) {
    const float4 x = *reinterpret_cast<const float4*>(&buf[tid * SPF + 4 * c]);
    re[2 * c] = x.x;
    im[2 * c] = x.y;
    re[2 * c + 1] = x.z;
    im[2 * c + 1] = x.w;
  }
  reg_dif<M, false>(re, im);
  if (tid >= ntw) return;
  constexpr CtTab<N> tw{};
  float2* out = Xb + t0 + tid;
  // Z[k] sits at register bitrev(k); Z[M] = Z[0]
#pragma unroll
  for (int f = 0; f <= M / 2; ++f) {
    const int g = M - f;  // partner frequency
    const int pf = ct_bitrev(f % M, LB), pg = ct_bitrev(g % M, LB);
    const double zfr = re[pf], zfi = im[pf], zgr = re[pg], zgi = im[pg];
    // X[f] = E + w^f O with E = (Z[f] + conj Z[g]) / 2, O = -i (Z[f] - conj Z[g]) / 2
    // X[g] = conj(E) - w^f conj(O)  (E[g] = conj E[f], O[g] = conj O[f], w^g = -conj w^f)
    const double er = 0.5 * (zfr + zgr), ei = 0.5 * (zfi - zgi);
    const double orr = 0.5 * (zfi + zgi), oi = -0.5 * (zfr - zgr);
    const double wr = tw.c[f], wi = -tw.s[f];
    const double tr = fma(wr, orr, -wi * oi), ti = fma(wr, oi, wi * orr);
    if (SPLIT) {
      st_split2(out + (int64_t)f * ntubes, (float)(er + tr), (float)(ei + ti));
      if (g != f) st_split2(out + (int64_t)g * ntubes, (float)(er - tr), (float)(ti - ei));
    } else {
      st_stream2(out + (int64_t)f * ntubes, (float)(er + tr), (float)(ei + ti));
      if (g != f) st_stream2(out + (int64_t)g * ntubes, (float)(er - tr), (float)(ti - ei));
    }
  }
}

template <int N>
__global__ __launch_bounds__(REG_TUBES) void fft_c2r_reg_kernel(const float2* __restrict__ Xb, int64_t slice_stride,
                                                                 float* __restrict__ X, int64_t ntubes) {
  constexpr int M = N / 2, LB = ct_log2(M), SPF = N + 4;
  constexpr int NV = REG_TUBES * N / 4;
  __shared__ __align__(16) float buf[REG_TUBES * SPF];
  const int tid = threadIdx.x;
  const int64_t t0 = (int64_t)blockIdx.x * REG_TUBES;
  const int ntw = (int)min((int64_t)REG_TUBES, ntubes - t0);
  double re[M], im[M];
  {
    constexpr CtTab<N> tw{};
    const int tt = tid < ntw ? tid : 0;  // threads past the end read tube 0 and store nothing
    const float2* in = Xb + t0 + tt;
    float2 x[M + 1];
#pragma unroll
    for (int f = 0; f <= M; ++f) x[f] = ld_stream2(in + (int64_t)f * slice_stride);
    x[0].y = 0.f;
    x[M].y = 0.f;
    // Z'[f] = (X[f] + conj X[M-f]) + i w^{-f} (X[f] - conj X[M-f]), f < M
#pragma unroll
    for (int f = 0; f < M; ++f) {
      const double ar = x[f].x, ai = x[f].y, br = x[M - f].x, bi = -(double)x[M - f].y;
      const double sr = ar + br, si = ai + bi, dr = ar - br, di = ai - bi;
      const double wr = tw.c[f], wi = tw.s[f];  // w^{-f}
      const double orr = fma(dr, wr, -di * wi), oi = fma(dr, wi, di * wr);
      re[f] = sr - oi;
      im[f] = si + orr;
    }
  }
  // unnormalised inverse DFT; z[n] = x[2n] + i x[2n+1] (times N) lands at register bitrev(n)
  reg_dif<M, true>(re, im);
  constexpr double invN = 1.0 / N;
#pragma unroll
  for (int c = 0; c < N / 4; ++c) {
    const int p0 = ct_bitrev(2 * c, LB), p1 = ct_bitrev(2 * c + 1, LB);
    float4 o;
    o.x = (float)(re[p0] * invN);
    o.y = (float)(im[p0] * invN);
    o.z = (float)(re[p1] * invN);
    o.w = (float)(im[p1] * invN);
    *reinterpret_cast<float4*>(&buf[tid * SPF + 4 * c]) = o;
  }
  __syncthreads();
  const int lim = ntw * (N / 4);
  float4* dst = reinterpret_cast<float4*>(X + t0 * N);
#pragma unroll
  for (int it = 0; it < NV / REG_TUBES; ++it) {
    const int g = tid + REG_TUBES * it;
    const int tube = g / (N / 4), c = g - tube * (N / 4);
    if (g < lim) st_stream4(dst + g, *reinterpret_cast<const float4*>(&buf[tube * SPF + 4 * c]));
  }
}

template <int N, bool SPLIT = false>
hipError_t reg_r2c(const void* X, void* Xb, int64_t ntubes, hipStream_t s) {
  const int64_t nblk = (ntubes + REG_TUBES - 1) / REG_TUBES;
  hipLaunchKernelGGL((fft_r2c_reg_kernel<N, SPLIT>), dim3((unsigned)nblk), dim3(REG_TUBES), 0, s, (const float*)X,
                     (float2*)Xb, ntubes);
  return hipGetLastError();
}
template <int N>
hipError_t reg_c2r(const void* Xb, int64_t stride, void* X, int64_t ntubes, hipStream_t s) {
  const int64_t nblk = (ntubes + REG_TUBES - 1) / REG_TUBES;
  hipLaunchKernelGGL((fft_c2r_reg_kernel<N>), dim3((unsigned)nblk), dim3(REG_TUBES), 0, s, (const float2*)Xb,
                     stride, (float*)X, ntubes);
  return hipGetLastError();
}

}  // namespace

bool fft_reg_supported(int n3, DType t) { return t == DT_F32 && (n3 == 8 || n3 == 16 || n3 == 32 || n3 == 64); }

hipError_t fft_r2c_reg(const void* X, void* Xb, int64_t ntubes, int n3, hipStream_t s) {
  if (ntubes <= 0) return hipSuccess;
  switch (n3) {
    case 8: return reg_r2c<8>(X, Xb, ntubes, s);
    case 16: return reg_r2c<16>(X, Xb, ntubes, s);
    case 32: return reg_r2c<32>(X, Xb, ntubes, s);
    case 64: return reg_r2c<64>(X, Xb, ntubes, s);
    default: return hipErrorNotSupported;
  }
}
hipError_t fft_r2c_split(const void* X, void* Xb, int64_t ntubes, int n3, hipStream_t s) {
  if (ntubes <= 0) return hipSuccess;
  switch (n3) {
    case 8: return reg_r2c<8, true>(X, Xb, ntubes, s);
    case 16: return reg_r2c<16, true>(X, Xb, ntubes, s);
    case 32: return reg_r2c<32, true>(X, Xb, ntubes, s);
    case 64: return reg_r2c<64, true>(X, Xb, ntubes, s);
    default: return hipErrorNotSupported;
  }
}
hipError_t fft_c2r_reg(const void* Xb, int64_t stride, void* X, int64_t ntubes, int n3, hipStream_t s) {
  if (ntubes <= 0) return hipSuccess;
  switch (n3) {
    case 8: return reg_c2r<8>(Xb, stride, X, ntubes, s);
    case 16: return reg_c2r<16>(Xb, stride, X, ntubes, s);
    case 32: return reg_c2r<32>(Xb, stride, X, ntubes, s);
    case 64: return reg_c2r<64>(Xb, stride, X, ntubes, s);
    default: return hipErrorNotSupported;
  }
}

}  // namespace tsvd
