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
  for (int idx = threadIdx.x; idx < NP * nb; idx += blockDim.x) {
    const int p = idx / nb;
    const int j = idx - p * nb;
    const int k = j % Ns;
    const cx<T>* a = in + p * N;
    cx<T>* o = out + p * N;
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
  cx<C>* b1 = b0 + NP * N;
  make_twiddles(tw, N);
  const int64_t t0 = (int64_t)blockIdx.x * 2 * NP;
  const int ntw = (int)min((int64_t)2 * NP, ntubes - t0);
  const T* src = X + t0 * N;
  const int total = ntw * N;
  for (int g = threadIdx.x; g < 2 * NP * N; g += blockDim.x) {
    const int tube = g / N, t = g - tube * N;
    const C v = (g < total) ? (C)src[g] : (C)0;
    C* dst = reinterpret_cast<C*>(&b0[(tube >> 1) * N + t]);
    dst[tube & 1] = v;
  }
  __syncthreads();
  const cx<C>* Z = run_passes<C, false>(b0, b1, tw, plan, NP);
  const int F = N / 2 + 1;
  for (int idx = threadIdx.x; idx < F * 2 * NP; idx += blockDim.x) {
    const int f = idx / (2 * NP), tube = idx - f * 2 * NP;
    if (tube >= ntw) continue;
    const int p = tube >> 1;
    const cx<C> zf = Z[p * N + f];
    const cx<C> zm = Z[p * N + (f == 0 ? 0 : N - f)];
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
  cx<C>* b1 = b0 + NP * N;
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
    b0[p * N + f] = cx<C>{a.re - b.im, a.im + b.re};
    if (f > 0 && 2 * f != N) b0[p * N + (N - f)] = cx<C>{a.re + b.im, b.re - a.im};
  }
  __syncthreads();
  const cx<C>* Z = run_passes<C, true>(b0, b1, tw, plan, NP);
  const C invN = (C)1 / (C)N;
  const int total = ntw * N;
  T* dst = X + t0 * N;
  for (int g = threadIdx.x; g < total; g += blockDim.x) {
    const int tube = g / N, t = g - tube * N;
    const cx<C> z = Z[(tube >> 1) * N + t];
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
  int np = (budget - N) / (2 * N);
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
  const size_t sm = (size_t)(n3 + 2 * NP * n3) * sizeof(cx<double>);
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
  const size_t sm = (size_t)(n3 + 2 * NP * n3) * sizeof(cx<double>);
  hipLaunchKernelGGL((fft_c2r_kernel<T, double>), dim3((unsigned)nblk), dim3(256), sm, s, (const cx<T>*)Xb, stride,
                     (T*)X, ntubes, plan, NP);
  return hipGetLastError();
}

hipError_t fft_r2c(const void* X, void* Xb, int64_t ntubes, int n3, DType t, hipStream_t s) {
  return t == DT_F64 ? r2c_t<double>(X, Xb, ntubes, n3, s) : r2c_t<float>(X, Xb, ntubes, n3, s);
}

hipError_t fft_c2r(const void* Xb, int64_t slice_stride, void* X, int64_t ntubes, int n3, DType t, hipStream_t s) {
  return t == DT_F64 ? c2r_t<double>(Xb, slice_stride, X, ntubes, n3, s)
                     : c2r_t<float>(Xb, slice_stride, X, ntubes, n3, s);
}

}  // namespace tsvd
