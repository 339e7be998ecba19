// Krylov products of Alg. 2 with BF16 arithmetic on gfx950 MFMA
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation): C_f = op(A_f) X_f for the
// large FP32 slice A_f (n1 x n2, interleaved complex) and a thin block X_f.
//
// Complex products by four real products on planar data,
//   A^H Y:  Cr = Yr.Ar + Yi.Ai,  Ci = Yi.Ar - Yr.Ai
// (A.B meaning the sum over the contraction index); A X is the conjugate of
// the same pattern applied to Y = conj(X) (A X = conj(conj(A) conj(X))), so
// the packed thin block holds conj(X) and the imaginary part of the result
// changes sign on the way out.  Each real product is in
// BF16 (one product of the rounded operands) or BF16x3 (operands split
// x = hi + lo, hi = bf16(x), lo = bf16(x - hi); hi.hi + hi.lo + lo.hi).
//
// A prepass packs the thin block once per call into bf16 planes (re / im,
// hi / lo) laid out exactly as the kernel's LDS tiles: per 32-wide K step and
// thin chunk of NC columns, each plane is NC rows of 32 bf16 (64 B) whose
// four 16-byte chunks are XOR-swizzled by row ((row >> 2) & 3) so that the
// MFMA fragment reads are free of bank conflicts.  The main kernel then
// copies that image into LDS with plain 16-byte loads and stores (one step
// ahead, double buffered), and streams A_f from HBM straight into the MFMA
// registers: each wave owns 32 columns of the result and every element of
// A_f is read once.  Within a 32-wide step, bf16 element 2 j + t of lane group
// q4 (j = 0..3, t = 0..1) holds k = 8 j + 2 q4 + t, so that the four lane
// groups of a row read 64 contiguous bytes of A_f per load instruction.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace tsvd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int BK = 32;  // complex K per step (one bf16 MFMA)

// Occupancy target (waves per SIMD) and depth of the A_f prefetch (register
// sets: 2 = one step ahead, 3 = two steps ahead).
#ifndef TSVD_KBF_MINWAVES
#define TSVD_KBF_MINWAVES 2
#endif
#ifndef TSVD_KBF_RING
#define TSVD_KBF_RING 2
#endif

struct BArgs {
  const float* A;  // big operand (floats), slice f at A + f * strideA
  int64_t lda, strideA;
  const uint4* P;  // packed thin operand
  int64_t pslice;  // uint4 per (slice, chunk)
  float* C;
  int64_t ldc, strideC;  // floats
  float* part;           // split-K partials [split][f][M][N] complex
  int M, K, N, batch;
  int nsplit, kchunk;    // kchunk: multiple of BK
  int nbig, nthin, total, per;
};

template <int MODE>
struct BPlanes {
  static constexpr int N = MODE == KM_BF16X3 ? 4 : 2;  // rh, ih (, rl, il)
};

__device__ __forceinline__ int swz(int row, int q) { return row * 4 + (q ^ ((row >> 2) & 3)); }

// ---- prepass: X (K x N complex FP32) -> packed planes ----
template <int MODE, bool CONJ>
__global__ void kpack_kernel(const float* __restrict__ X, int64_t ldx, int64_t strideX, uint4* __restrict__ P,
                             int K, int N, int NC, int nthin, int ksteps, int batch) {
  constexpr int NPL = BPlanes<MODE>::N;
  const int64_t total = (int64_t)batch * nthin * ksteps * NC * 4;  // one thread per (row, 16-byte chunk)
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = e;
    const int q = (int)(r % 4);
    r /= 4;
    const int row = (int)(r % NC);
    r /= NC;
    const int s = (int)(r % ksteps);
    r /= ksteps;
    const int c = (int)(r % nthin);
    const int f = (int)(r / nthin);
    const int n = c * NC + row;
    const float* Xf = X + (int64_t)f * strideX;
    uint32_t w[NPL][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      uint32_t hr = 0, hi = 0, lr = 0, li = 0;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int k = s * BK + 8 * j + 2 * q + h;  // element 2 j + h of lane group q
        float xr = 0.f, xi = 0.f;
        if (k < K && n < N) {
          const float2 v = *reinterpret_cast<const float2*>(Xf + (int64_t)k * ldx + 2 * n);
          xr = v.x;
          xi = CONJ ? -v.y : v.y;
        }
        const __bf16 br = (__bf16)xr, bi = (__bf16)xi;
        hr |= (uint32_t)__builtin_bit_cast(unsigned short, br) << (16 * h);
        hi |= (uint32_t)__builtin_bit_cast(unsigned short, bi) << (16 * h);
        if (MODE == KM_BF16X3) {
          const __bf16 sr = (__bf16)(xr - (float)br), si = (__bf16)(xi - (float)bi);
          lr |= (uint32_t)__builtin_bit_cast(unsigned short, sr) << (16 * h);
          li |= (uint32_t)__builtin_bit_cast(unsigned short, si) << (16 * h);
        }
      }
      w[0][j] = hr;
      w[1][j] = hi;
      if (MODE == KM_BF16X3) {
        w[2][j] = lr;
        w[3][j] = li;
      }
    }
    uint4* blk = P + ((int64_t)(f * nthin + c) * ksteps + s) * (NPL * NC * 4);
#pragma unroll
    for (int p = 0; p < NPL; ++p) blk[p * NC * 4 + swz(row, q)] = make_uint4(w[p][0], w[p][1], w[p][2], w[p][3]);
  }
}

__device__ __forceinline__ bf16x8 neg8(bf16x8 x) {
  uint4 u = __builtin_bit_cast(uint4, x);
  u.x ^= 0x80008000u;
  u.y ^= 0x80008000u;
  u.z ^= 0x80008000u;
  u.w ^= 0x80008000u;
  return __builtin_bit_cast(bf16x8, u);
}

#define MF(a, b, c) __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0)

template <int MODE, bool HN, int TTN, bool AVEC, int TB>
__global__ __launch_bounds__(256, TSVD_KBF_MINWAVES) void kgemm_bf_kernel(const BArgs a) {
  constexpr int NPL = BPlanes<MODE>::N;
  constexpr int NC = TTN * 16;
  constexpr int BLK = NPL * NC * 4;  // uint4 per step image
  constexpr int PER = BLK / 256;     // uint4 copied per thread per step
  static_assert(PER * 256 == BLK, "image split");
  extern __shared__ __align__(16) uint4 sl[];

  const int id = blockIdx.x;
  const int t = (id & 7) * a.per + (id >> 3);
  if (t >= a.total) return;
  int r = t;
  const int bt = r % a.nbig;
  r /= a.nbig;
  const int tc = r % a.nthin;
  r /= a.nthin;
  const int sp = r % a.nsplit;
  const int f = r / a.nsplit;
  const int kb = sp * a.kchunk;
  const int ke = min(a.K, kb + a.kchunk);
  const int nfull = ke > kb ? (ke - kb) / BK : 0;  // full steps; a ragged last one follows
  const bool tail = ke > kb + nfull * BK;
  const int n0 = tc * NC;
  const int nc = min(NC, a.N - n0);
  const int tt = (nc + 15) / 16;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int q4 = lane >> 4, r16 = lane & 15;
  int col[TB], colc[TB];
  bool colok[TB];
#pragma unroll
  for (int u = 0; u < TB; ++u) {
    col[u] = bt * (64 * TB) + wave * (16 * TB) + 16 * u + r16;
    colok[u] = col[u] < a.M;
    colc[u] = colok[u] ? col[u] : a.M - 1;
  }
  const float* Af = a.A + (int64_t)f * a.strideA;
  const uint4* Pimg = a.P + (int64_t)(f * a.nthin + tc) * a.pslice + (int64_t)(kb / BK) * BLK;

  // A_f: 8 complex along K per lane and 16-column tile.  Full steps lie inside
  // [kb, ke) and load unconditionally; the ragged last step clamps each index
  // to K - 1 (those products meet zero rows of the thin image).
  // element m = 2 j + t of lane group q4 is k = k0 + 8 j + 2 q4 + t
  auto load_big = [&](int s, float (&v)[TB][16]) {
    const int k0 = kb + s * BK + 2 * q4;
#pragma unroll
    for (int u = 0; u < TB; ++u) {
      if (!HN) {
        const float* p = Af + (int64_t)colc[u] * a.lda + 2 * k0;
        if (AVEC) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float4 x = *reinterpret_cast<const float4*>(p + 16 * j);
            v[u][4 * j] = x.x; v[u][4 * j + 1] = x.y; v[u][4 * j + 2] = x.z; v[u][4 * j + 3] = x.w;
          }
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int t = 0; t < 2; ++t) {
              const float2 x = *reinterpret_cast<const float2*>(p + 16 * j + 2 * t);
              v[u][4 * j + 2 * t] = x.x;
              v[u][4 * j + 2 * t + 1] = x.y;
            }
        }
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            const float2 x =
                *reinterpret_cast<const float2*>(Af + (int64_t)(k0 + 8 * j + t) * a.lda + 2 * colc[u]);
            v[u][4 * j + 2 * t] = x.x;
            v[u][4 * j + 2 * t + 1] = x.y;
          }
      }
    }
  };
  auto load_big_tail = [&](int s, float (&v)[TB][16]) {
    const int k0 = kb + s * BK + 2 * q4;
#pragma unroll
    for (int u = 0; u < TB; ++u) {
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const int k = min(k0 + 8 * j + t, a.K - 1);
          const float* p = HN ? Af + (int64_t)k * a.lda + 2 * colc[u] : Af + (int64_t)colc[u] * a.lda + 2 * k;
          const float2 x = *reinterpret_cast<const float2*>(p);
          v[u][4 * j + 2 * t] = x.x;
          v[u][4 * j + 2 * t + 1] = x.y;
        }
    }
  };
  auto load_img = [&](int s, uint4 (&x)[PER]) {
    const uint4* src = Pimg + (int64_t)s * BLK;
#pragma unroll
    for (int j = 0; j < PER; ++j) x[j] = src[tid + 256 * j];
  };
  auto store_img = [&](uint4* dst, const uint4 (&x)[PER]) {
#pragma unroll
    for (int j = 0; j < PER; ++j) dst[tid + 256 * j] = x[j];
  };

  f32x4 cr[TTN][TB], ci[TTN][TB];
#pragma unroll
  for (int i = 0; i < TTN; ++i)
#pragma unroll
    for (int u = 0; u < TB; ++u) {
      cr[i][u] = f32x4{0.f, 0.f, 0.f, 0.f};
      ci[i][u] = f32x4{0.f, 0.f, 0.f, 0.f};
    }

  // Cr += Yr.Ar + Yi.Ai, Ci += Yi.Ar - Yr.Ai; the negative term negates the
  // thin fragment (sign bits), which is shared by the TB column tiles.
  auto compute = [&](const uint4* buf, const float (&v)[TB][16]) {
    bf16x8 arh[TB], aih[TB], arl[TB], ail[TB];
#pragma unroll
    for (int u = 0; u < TB; ++u) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const __bf16 hr = (__bf16)v[u][2 * j], hi = (__bf16)v[u][2 * j + 1];
        arh[u][j] = hr;
        aih[u][j] = hi;
        if (MODE == KM_BF16X3) {
          arl[u][j] = (__bf16)(v[u][2 * j] - (float)hr);
          ail[u][j] = (__bf16)(v[u][2 * j + 1] - (float)hi);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < TTN; ++i) {
      if (i < tt) {
        const int row = 16 * i + r16;
        const int o = swz(row, q4);
        const bf16x8 xrh = __builtin_bit_cast(bf16x8, buf[o]);
        const bf16x8 xih = __builtin_bit_cast(bf16x8, buf[NC * 4 + o]);
        const bf16x8 nrh = neg8(xrh);
        if (MODE == KM_BF16X3) {
          const bf16x8 xrl = __builtin_bit_cast(bf16x8, buf[2 * NC * 4 + o]);
          const bf16x8 xil = __builtin_bit_cast(bf16x8, buf[3 * NC * 4 + o]);
          const bf16x8 nrl = neg8(xrl);
#pragma unroll
          for (int u = 0; u < TB; ++u) {
            // small terms first
            cr[i][u] = MF(xrl, arh[u], cr[i][u]);
            cr[i][u] = MF(xrh, arl[u], cr[i][u]);
            cr[i][u] = MF(xil, aih[u], cr[i][u]);
            cr[i][u] = MF(xih, ail[u], cr[i][u]);
            ci[i][u] = MF(xil, arh[u], ci[i][u]);
            ci[i][u] = MF(xih, arl[u], ci[i][u]);
            ci[i][u] = MF(nrl, aih[u], ci[i][u]);
            ci[i][u] = MF(nrh, ail[u], ci[i][u]);
          }
        }
#pragma unroll
        for (int u = 0; u < TB; ++u) {
          cr[i][u] = MF(xrh, arh[u], cr[i][u]);
          cr[i][u] = MF(xih, aih[u], cr[i][u]);
          ci[i][u] = MF(xih, arh[u], ci[i][u]);
          ci[i][u] = MF(nrh, aih[u], ci[i][u]);
        }
      }
    }
  };

  // ---- pipeline over the full steps: thin image one step ahead (registers
  // -> the other LDS buffer), A_f one or two steps ahead in a ring of register
  // sets; every load is issued unconditionally (indices past the last full
  // step are clamped), the image first because loads complete in issue order ----
  uint4 img[PER];
  if constexpr (TSVD_KBF_RING == 3) {
    float va[TB][16], vb[TB][16], vc[TB][16];
    if (nfull > 0) {
      load_big(0, va);
      load_big(nfull > 1 ? 1 : 0, vb);
      load_img(0, img);
      store_img(sl, img);
    }
    __syncthreads();
    auto step = [&](int s, const float (&cur)[TB][16], float (&pre)[TB][16]) {
      const int sn = s + 1 < nfull ? s + 1 : nfull - 1;
      const int s2 = s + 2 < nfull ? s + 2 : nfull - 1;
      load_img(sn, img);
      load_big(s2, pre);
      if (s < nfull) {
        compute(sl + (s & 1) * BLK, cur);
        if (s + 1 < nfull) store_img(sl + ((s + 1) & 1) * BLK, img);
        __syncthreads();
      }
    };
    for (int s = 0; s < nfull; s += 3) {
      step(s, va, vc);
      step(s + 1, vb, va);
      step(s + 2, vc, vb);
    }
    if (tail) {
      load_img(nfull, img);
      store_img(sl + (nfull & 1) * BLK, img);
      load_big_tail(nfull, va);
      __syncthreads();
      compute(sl + (nfull & 1) * BLK, va);
    }
  } else {
    float va[TB][16], vb[TB][16];
    if (nfull > 0) {
      load_big(0, va);
      load_img(0, img);
      store_img(sl, img);
    }
    __syncthreads();
    auto step = [&](int s, const float (&cur)[TB][16], float (&nxt)[TB][16]) {
      const int sn = s + 1 < nfull ? s + 1 : nfull - 1;
      load_img(sn, img);
      load_big(sn, nxt);
      if (s < nfull) {
        compute(sl + (s & 1) * BLK, cur);
        if (s + 1 < nfull) store_img(sl + ((s + 1) & 1) * BLK, img);
        __syncthreads();
      }
    };
    for (int s = 0; s < nfull; s += 2) {
      step(s, va, vb);
      step(s + 1, vb, va);
    }
    if (tail) {
      load_img(nfull, img);
      store_img(sl + (nfull & 1) * BLK, img);
      load_big_tail(nfull, va);
      __syncthreads();
      compute(sl + (nfull & 1) * BLK, va);
    }
  }

  // ---- epilogue: acc[i][u][r] = C[col_u][n0 + 16 i + 4 q4 + r] ----
  float* out;
  int64_t ldo;
  if (a.nsplit > 1) {
    out = a.part + 2 * ((int64_t)sp * a.batch + f) * a.M * a.N;
    ldo = 2 * (int64_t)a.N;
  } else {
    out = a.C + (int64_t)f * a.strideC;
    ldo = a.ldc;
  }
#pragma unroll
  for (int u = 0; u < TB; ++u) {
    if (!colok[u]) continue;
#pragma unroll
    for (int i = 0; i < TTN; ++i) {
      if (i < tt) {
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int n = n0 + 16 * i + 4 * q4 + rr;
          if (n < a.N)
            *reinterpret_cast<float2*>(out + (int64_t)col[u] * ldo + 2 * n) =
                make_float2(cr[i][u][rr], HN ? ci[i][u][rr] : -ci[i][u][rr]);
        }
      }
    }
  }
}

#undef MF

__global__ void kbf_reduce_kernel(const float2* __restrict__ part, int nsplit, int batch, int M, int N,
                                  float2* __restrict__ C, int64_t ldc, int64_t strideC) {
  const int64_t per = (int64_t)M * N;
  const int64_t total = per * batch;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t f = e / per, rem = e % per;
    const int row = (int)(rem / N), n = (int)(rem % N);
    float2 s = part[e];
    for (int j = 1; j < nsplit; ++j) {
      const float2 v = part[(int64_t)j * total + e];
      s.x += v.x;
      s.y += v.y;
    }
    C[f * strideC + (int64_t)row * ldc + n] = s;
  }
}

int bf_thin_tiles(int mode, int N) {
  const int nn = std::min(N, 128);
  int tt = (nn + 15) / 16;
  if (mode == KM_BF16 && (tt & 1)) ++tt;  // the image of a step is split evenly over 256 threads
  return tt;
}

constexpr int BTB = 2;  // 16-column tiles of the result per wave

template <int MODE, bool HN, int TTN, bool AVEC>
hipError_t bf_launch_t(const BArgs& a, hipStream_t s) {
  const size_t lds = (size_t)2 * BPlanes<MODE>::N * TTN * 16 * 64;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)kgemm_bf_kernel<MODE, HN, TTN, AVEC, BTB>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipGetLastError();
    attr = true;
  }
  hipLaunchKernelGGL((kgemm_bf_kernel<MODE, HN, TTN, AVEC, BTB>), dim3(8 * a.per), dim3(256), lds, s, a);
  return hipGetLastError();
}

template <int MODE, bool HN, bool AVEC>
hipError_t bf_launch_tt(const BArgs& a, int TTN, hipStream_t s) {
  switch (TTN) {
    case 2: return bf_launch_t<MODE, HN, 2, AVEC>(a, s);
    case 4: return bf_launch_t<MODE, HN, 4, AVEC>(a, s);
    case 6: return bf_launch_t<MODE, HN, 6, AVEC>(a, s);
    case 8: return bf_launch_t<MODE, HN, 8, AVEC>(a, s);
    default: return hipErrorInvalidValue;
  }
}

template <int MODE>
hipError_t bf_launch(const BArgs& a, bool herm, bool avec, int TTN, hipStream_t s) {
  if (herm) return bf_launch_tt<MODE, true, false>(a, TTN, s);
  return avec ? bf_launch_tt<MODE, false, true>(a, TTN, s) : bf_launch_tt<MODE, false, false>(a, TTN, s);
}

}  // namespace

size_t kgemm_bf16_pack_bytes(int mode, int K, int N, int batch) {
  const int TTN = bf_thin_tiles(mode, N);
  const int NC = TTN * 16;
  const int nthin = (N + NC - 1) / NC;
  const int ksteps = (K + BK - 1) / BK;
  const int npl = mode == KM_BF16X3 ? 4 : 2;
  return (size_t)batch * nthin * ksteps * npl * NC * 64;
}

int kgemm_bf16_split(int M, int K, int N, int batch) {
  const int TTN = bf_thin_tiles(KM_BF16, N);
  const int64_t nthin = (N + TTN * 16 - 1) / (TTN * 16);
  const int64_t tiles = (int64_t)((M + 64 * BTB - 1) / (64 * BTB)) * nthin * batch;
  int ns = 1;
  while (tiles * ns < 1024 && ns < 8 && K / (2 * ns) >= 512) ns *= 2;
  return ns;
}

hipError_t kgemm_bf16(const KGemmDesc& d, void* pack, hipStream_t s) {
  const int M = d.herm ? d.cols : d.rows;
  const int K = d.herm ? d.rows : d.cols;
  if (d.sub) return hipErrorInvalidValue;  // the update form is the FP32 kernel's only
  if (M <= 0 || d.N <= 0 || d.batch <= 0) return hipSuccess;
  // BF16x3 runs on the real-embedded kernel (kgemm), which measured faster
  // for three products per term at these register budgets.
  if (!pack || d.mode != KM_BF16) return hipErrorInvalidValue;
  const int TTN = bf_thin_tiles(d.mode, d.N);
  const int NC = TTN * 16;
  const int nthin = (d.N + NC - 1) / NC;
  const int ksteps = (K + BK - 1) / BK;
  const int npl = d.mode == KM_BF16X3 ? 4 : 2;
  // 1. pack the thin block
  {
    const int64_t n = (int64_t)d.batch * nthin * ksteps * NC * 4;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 65536);
    const float* Xp = (const float*)d.X;
    uint4* Pp = (uint4*)pack;
    if (d.herm)
      hipLaunchKernelGGL((kpack_kernel<KM_BF16, false>), dim3(blocks), dim3(256), 0, s, Xp, 2 * d.ldx, 2 * d.strideX,
                         Pp, K, d.N, NC, nthin, ksteps, d.batch);
    else
      hipLaunchKernelGGL((kpack_kernel<KM_BF16, true>), dim3(blocks), dim3(256), 0, s, Xp, 2 * d.ldx, 2 * d.strideX,
                         Pp, K, d.N, NC, nthin, ksteps, d.batch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  // 2. the products
  BArgs a{};
  a.A = static_cast<const float*>(d.A);
  a.lda = 2 * d.lda;
  a.strideA = 2 * d.strideA;
  a.P = static_cast<const uint4*>(pack);
  a.pslice = (int64_t)ksteps * npl * NC * 4;
  a.C = static_cast<float*>(d.C);
  a.ldc = 2 * d.ldc;
  a.strideC = 2 * d.strideC;
  a.part = static_cast<float*>(d.part);
  a.M = M;
  a.K = K;
  a.N = d.N;
  a.batch = d.batch;
  a.nsplit = d.nsplit > 1 ? d.nsplit : 1;
  if (a.nsplit > 1 && !d.part) return hipErrorInvalidValue;
  int kc = (K + a.nsplit - 1) / a.nsplit;
  kc = (kc + BK - 1) / BK * BK;
  a.kchunk = kc;
  a.nthin = nthin;
  a.nbig = (M + 64 * BTB - 1) / (64 * BTB);
  const int64_t total = (int64_t)a.nbig * a.nthin * a.nsplit * d.batch;
  if (total >= (int64_t)1 << 30) return hipErrorInvalidValue;
  a.total = (int)total;
  a.per = (a.total + 7) / 8;
  const bool avec = (d.lda & 1) == 0 && (d.strideA & 1) == 0 && ((uintptr_t)d.A & 15) == 0;
  hipError_t e = bf_launch<KM_BF16>(a, d.herm, avec, TTN, s);
  if (e != hipSuccess || a.nsplit <= 1) return e;
  const int64_t n = (int64_t)M * d.N * d.batch;
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(kbf_reduce_kernel, dim3(blocks), dim3(256), 0, s, (const float2*)d.part, a.nsplit, d.batch, M,
                     d.N, (float2*)d.C, d.ldc, d.strideC);
  return hipGetLastError();
}

}  // namespace tsvd
