// Krylov products of Alg. 2 on gfx950 MFMA: C_f = op(A_f) X_f for every
// Fourier slice f, with A_f the large n1 x n2 slice of the transformed data
// (FP32 interleaved complex) and X_f a thin block of N columns.
//
// Complex arithmetic as real MFMA over the interleaved storage.  Along K the
// operands are read as (re, im) pairs, and each part of a complex result is
// one real dot product over 2K terms:
//   C = A X   :  Re C[m][n] = sum_k <(ar, ai), (xr, -xi)>,  Im C[m][n] = sum_k <(ai, -ar), (xr, -xi)>
//   C = A^H Y :  Re C[j][n] = sum_i <(ar, ai), (yr, yi)>,   Im C[j][n] = sum_i <(-ai, ar), (yr, yi)>
// with a = A[m][k] (A[i][j]), x = X[k][n], y = Y[i][n].  The thin operand,
// conjugated for A X, is the MFMA A operand: one row per complex column,
// staged through LDS.  The big operand A_f is the MFMA B operand in two forms
// (as loaded for the real parts; each pair swapped and one sign flipped for
// the imaginary parts) and goes from HBM straight into the registers of one
// wave, which uses it for all N columns: every element of A_f is read from
// HBM once per product.  The output tile of a wave is (N complex columns) x
// (16 TB big-dimension rows), written as contiguous (re, im) pairs.
//
// Precision modes: FP32 (v_mfma_f32_16x16x4_f32), BF16 (one bf16 product,
// v_mfma_f32_16x16x32_bf16) and BF16x3 (x = hi + lo with hi = bf16(x),
// lo = bf16(x - hi); hi*hi + hi*lo + lo*hi), all with FP32 accumulation.
//
// K step: 16 complex (32 real).  Lane (q4 = lane / 16, r = lane % 16) owns
// real k' = 8 q4 .. 8 q4 + 7 of each step, i.e. complex k = 4 q4 .. 4 q4 + 3:
// one bf16 MFMA covers the step; in FP32, MFMA block b (0..7) takes k' = 8 q4 + b.
//
// Work decomposition: tiles (slice, K split, thin chunk, big tile) are
// numbered with the big tile fastest, and workgroup ids are mapped so that
// consecutive tiles land on the same XCD (ids are dispatched round-robin over
// the 8 XCDs): the thin block of a slice stays in that XCD's L2.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace tsvd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int KSTEP = 16;  // complex K per step
constexpr int NWAVE = 4;

struct KArgs {
  const float* A;  // big operand (floats), slice f at A + f * strideA
  int64_t lda, strideA;  // in floats
  const float* X;  // thin operand (floats)
  int64_t ldx, strideX;  // in floats
  float* C;        // output (floats)
  int64_t ldc, strideC;  // in floats
  float* part;     // split-K partials: [split][f][M][N] complex
  int M, K, N, batch;
  int nsplit, kchunk;
  int nbig, nthin, total, per;
  int avec;  // big-operand rows are 16-byte aligned (vector loads allowed)
  // Tail split (nsplit == 1): tiles [0, nfull) run whole, nfull / 8 per XCD;
  // the rem tiles after them are split rsplit ways along K (chunks of
  // rkchunk) and write their partials to part, one 128 x NCH block per
  // (tile, split).  rsplit == 0: no tail split.
  int nfull, nrem, rsplit, rkchunk;
  int sub;  // C -= result (whole-K tiles written straight to C only)
};

__device__ __forceinline__ uint32_t bf16_bits(float x) {
  __bf16 h = (__bf16)x;
  return (uint32_t)__builtin_bit_cast(unsigned short, h);
}

template <int MODE>
struct Lds {
  static constexpr int WORDS = MODE == KM_F32 ? 2 * KSTEP : KSTEP;  // 32-bit words per row
  static constexpr int STRIDE = WORDS + 4;
  static constexpr int PLANES = (MODE == KM_BF16X3 || MODE == KM_BF16X3_SPLIT) ? 2 : 1;
};

// Pack of two bf16 bit patterns: lo in bits 0..15, hi in 16..31.
__device__ __forceinline__ uint32_t swap16(uint32_t x) { return (x >> 16) | (x << 16); }

template <int MODE, bool HN, int TT, int TB, bool AVEC, bool FULL>
__global__ __launch_bounds__(256, 2) void kgemm_kernel(const KArgs a) {
  typedef Lds<MODE> L;
  // three-product BF16; PRE: the big operand arrives as (hi, lo) bf16 pairs
  constexpr bool X3 = MODE == KM_BF16X3 || MODE == KM_BF16X3_SPLIT;
  constexpr bool PRE = MODE == KM_BF16X3_SPLIT;
  constexpr int NCH = TT * 8;                 // complex thin columns per tile
  constexpr int TC = NCH / 16;                // MFMA tiles of 16 complex columns
  constexpr int PLANE = NCH * L::STRIDE;      // one LDS row per complex column
  constexpr int BUF = PLANE * L::PLANES;
  constexpr int TEL = KSTEP * NCH / 256;      // thin elements per thread per step
  static_assert(TEL * 256 == KSTEP * NCH && TC * 16 == NCH && TEL == TC && KSTEP == 4 * NWAVE, "thin split");
  extern __shared__ __align__(16) uint32_t lds[];

  // ---- tile of this workgroup (XCD-aware order) ----
  const int id = blockIdx.x;
  int bt, tc, sp, f, kb, ke, rt = -1;
  if (a.rsplit == 0) {
    const int t = (id & 7) * a.per + (id >> 3);
    if (t >= a.total) return;
    int r = t;
    bt = r % a.nbig;
    r /= a.nbig;
    tc = r % a.nthin;
    r /= a.nthin;
    sp = r % a.nsplit;
    f = r / a.nsplit;
    kb = sp * a.kchunk;
    ke = min(a.K, kb + a.kchunk);
  } else {
    // each XCD first runs nfull / 8 whole tiles, then its share of the split
    // remainder (so that every XCD gets the same work)
    const int x = id & 7, l = id >> 3, fper = a.nfull / 8;
    int u;
    if (l < fper) {
      u = x * fper + l;
      sp = 0;
      kb = 0;
      ke = a.K;
    } else {
      const int w = (l - fper) * 8 + x;
      if (w >= a.nrem * a.rsplit) return;
      rt = w / a.rsplit;
      sp = w - rt * a.rsplit;
      u = a.nfull + rt;
      kb = sp * a.rkchunk;
      ke = min(a.K, kb + a.rkchunk);
    }
    bt = u % a.nbig;
    u /= a.nbig;
    tc = u % a.nthin;
    f = u / a.nthin;
  }
  const int n0 = tc * NCH;
  const int nc = min(NCH, a.N - n0);
  const int tt = FULL ? TC : (nc + 15) / 16;  // active thin tiles (all of them when FULL)

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int q4 = lane >> 4, r16 = lane & 15;
  const float* Af = a.A + (int64_t)f * a.strideA;
  const float* Xf = a.X + (int64_t)f * a.strideX;
  int col[TB], colc[TB];
  bool colok[TB];
#pragma unroll
  for (int u = 0; u < TB; ++u) {
    col[u] = bt * (NWAVE * 16 * TB) + wave * 16 * TB + u * 16 + r16;
    colok[u] = col[u] < a.M;
    colc[u] = colok[u] ? col[u] : a.M - 1;  // clamped: loads stay in bounds, results unused
  }

  // Thin element e of this thread: K index 4 wave + q4 of the step, complex
  // column 16 e + r16.  A wave's global loads read 16 consecutive columns of
  // 4 rows, and its LDS stores (row = column, word = K index) fall in 64
  // distinct banks: the rows of a 16-lane group start 20 (36) words apart,
  // i.e. at distinct multiples of 4 modulo 64.
  const int tk = 4 * wave + q4;
  // ---- full K steps: every load is issued unconditionally (clamped
  // addresses; a clamped row or column feeds only results that are never
  // stored) so that the compiler's wait counts can leave the prefetches of
  // later steps in flight ----
  auto load_big_full = [&](int k0, float (&v)[TB][8]) {
#pragma unroll
    for (int u = 0; u < TB; ++u) {
      if (!HN) {
        const float* p = Af + (int64_t)colc[u] * a.lda + 2 * (k0 + 4 * q4);
        if (AVEC) {
          const float4 x0 = *reinterpret_cast<const float4*>(p);
          const float4 x1 = *reinterpret_cast<const float4*>(p + 4);
          v[u][0] = x0.x; v[u][1] = x0.y; v[u][2] = x0.z; v[u][3] = x0.w;
          v[u][4] = x1.x; v[u][5] = x1.y; v[u][6] = x1.z; v[u][7] = x1.w;
        } else {
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const float2 x = *reinterpret_cast<const float2*>(p + 2 * c);
            v[u][2 * c] = x.x;
            v[u][2 * c + 1] = x.y;
          }
        }
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const float2 x = *reinterpret_cast<const float2*>(Af + (int64_t)(k0 + 4 * q4 + c) * a.lda + 2 * colc[u]);
          v[u][2 * c] = x.x;
          v[u][2 * c + 1] = x.y;
        }
      }
    }
  };
  auto load_thin_full = [&](int k0, float2 (&x)[TEL]) {
#pragma unroll
    for (int e = 0; e < TEL; ++e) {
      // a column past nc reads column n0 instead: it feeds only its own
      // result column, which is never stored, so it need not be zeroed (a
      // select here would let the compiler turn the load into a branch that
      // waits for it)
      const int nn = 16 * e + r16;
      x[e] = *reinterpret_cast<const float2*>(Xf + (int64_t)(k0 + tk) * a.ldx + 2 * (n0 + (nn < nc ? nn : 0)));
    }
  };

  // ---- big operand: 8 reals (4 complex along K) per lane and tile ----
  auto load_big = [&](int k0, float (&v)[TB][8]) {
    const bool full = k0 + KSTEP <= ke;
#pragma unroll
    for (int u = 0; u < TB; ++u) {
      if (!HN) {
        const float* p = Af + (int64_t)col[u] * a.lda + 2 * (k0 + 4 * q4);
        if (colok[u] && full && AVEC) {
          const float4 x0 = *reinterpret_cast<const float4*>(p);
          const float4 x1 = *reinterpret_cast<const float4*>(p + 4);
          v[u][0] = x0.x; v[u][1] = x0.y; v[u][2] = x0.z; v[u][3] = x0.w;
          v[u][4] = x1.x; v[u][5] = x1.y; v[u][6] = x1.z; v[u][7] = x1.w;
        } else {
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            float2 x = make_float2(0.f, 0.f);
            if (colok[u] && k0 + 4 * q4 + c < ke) x = *reinterpret_cast<const float2*>(p + 2 * c);
            v[u][2 * c] = x.x;
            v[u][2 * c + 1] = x.y;
          }
        }
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int i = k0 + 4 * q4 + c;
          float2 x = make_float2(0.f, 0.f);
          if (colok[u] && (full || i < ke))
            x = *reinterpret_cast<const float2*>(Af + (int64_t)i * a.lda + 2 * col[u]);
          v[u][2 * c] = x.x;
          v[u][2 * c + 1] = x.y;
        }
      }
    }
  };

  // ---- thin operand: KSTEP x NCH complex per step, k fastest in a thread group ----
  auto load_thin = [&](int k0, float2 (&x)[TEL]) {
#pragma unroll
    for (int e = 0; e < TEL; ++e) {
      const int nn = 16 * e + r16;
      float2 v = make_float2(0.f, 0.f);
      if (k0 + tk < ke && nn < nc) v = *reinterpret_cast<const float2*>(Xf + (int64_t)(k0 + tk) * a.ldx + 2 * (n0 + nn));
      x[e] = v;
    }
  };
  // the thin operand in LDS: row nn holds column nn of X (conjugated for
  // A X) as (re, im) pairs, FP32 or bf16 (hi and lo planes for BF16x3)
  auto store_thin = [&](uint32_t* buf, const float2 (&x)[TEL]) {
    constexpr uint32_t CJ = HN ? 0u : 0x80000000u;  // sign of the imaginary half
#pragma unroll
    for (int e = 0; e < TEL; ++e) {
      uint32_t* row = buf + (16 * e + r16) * L::STRIDE;
      const float xr = x[e].x, xi = x[e].y;
      if (MODE == KM_F32) {
        *reinterpret_cast<float2*>(row + 2 * tk) = make_float2(xr, HN ? xi : -xi);
      } else {
        // each value is rounded once; conjugation flips the bf16 sign bit
        const __bf16 hr = (__bf16)xr, hi = (__bf16)xi;
        row[tk] = ((uint32_t)__builtin_bit_cast(unsigned short, hr) |
                   ((uint32_t)__builtin_bit_cast(unsigned short, hi) << 16)) ^ CJ;
        if (X3) row[PLANE + tk] = (bf16_bits(xr - (float)hr) | (bf16_bits(xi - (float)hi) << 16)) ^ CJ;
      }
    }
  };

  f32x4 accr[TC][TB], acci[TC][TB];  // real and imaginary parts
#pragma unroll
  for (int i = 0; i < TC; ++i)
#pragma unroll
    for (int u = 0; u < TB; ++u) {
      accr[i][u] = f32x4{0.f, 0.f, 0.f, 0.f};
      acci[i][u] = f32x4{0.f, 0.f, 0.f, 0.f};
    }

  auto compute = [&](const uint32_t* buf, const float (&v)[TB][8]) {
    if (MODE == KM_F32) {
      // B operand of the imaginary parts: (ai, -ar) for A X, (-ai, ar) for A^H Y
      float sv[TB][8];
#pragma unroll
      for (int u = 0; u < TB; ++u)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          sv[u][2 * c] = HN ? -v[u][2 * c + 1] : v[u][2 * c + 1];
          sv[u][2 * c + 1] = HN ? v[u][2 * c] : -v[u][2 * c];
        }
#pragma unroll
      for (int i = 0; i < TC; ++i) {
        if (i < tt) {
          const float* rowp = reinterpret_cast<const float*>(buf + (16 * i + r16) * L::STRIDE + 8 * q4);
          const float4 w0 = *reinterpret_cast<const float4*>(rowp);
          const float4 w1 = *reinterpret_cast<const float4*>(rowp + 4);
          const float w[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
#pragma unroll
          for (int b = 0; b < 8; ++b)
#pragma unroll
            for (int u = 0; u < TB; ++u) {
              accr[i][u] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[b], v[u][b], accr[i][u], 0, 0, 0);
              acci[i][u] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[b], sv[u][b], acci[i][u], 0, 0, 0);
            }
        }
      }
    } else {
      // words (re | im << 16) of the lane's four complex values; the
      // imaginary parts' operand swaps the halves and flips one sign
      constexpr uint32_t SF = HN ? 0x00008000u : 0x80000000u;
      bf16x8 bh[TB], bl[TB], sh[TB], sl[TB];
#pragma unroll
      for (int u = 0; u < TB; ++u) {
        uint32_t wh[4], wl[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if (PRE) {
            // complex c of the lane's four: word 2c = hi pair, word 2c + 1 = lo pair
            wh[c] = __float_as_uint(v[u][2 * c]);
            wl[c] = __float_as_uint(v[u][2 * c + 1]);
          } else {
            const __bf16 hr = (__bf16)v[u][2 * c], hi = (__bf16)v[u][2 * c + 1];
            wh[c] = (uint32_t)__builtin_bit_cast(unsigned short, hr) |
                    ((uint32_t)__builtin_bit_cast(unsigned short, hi) << 16);
            wl[c] = X3 ? (bf16_bits(v[u][2 * c] - (float)hr) | (bf16_bits(v[u][2 * c + 1] - (float)hi) << 16)) : 0u;
          }
        }
        bh[u] = __builtin_bit_cast(bf16x8, make_uint4(wh[0], wh[1], wh[2], wh[3]));
        sh[u] = __builtin_bit_cast(bf16x8, make_uint4(swap16(wh[0]) ^ SF, swap16(wh[1]) ^ SF, swap16(wh[2]) ^ SF,
                                                      swap16(wh[3]) ^ SF));
        if (X3) {
          bl[u] = __builtin_bit_cast(bf16x8, make_uint4(wl[0], wl[1], wl[2], wl[3]));
          sl[u] = __builtin_bit_cast(bf16x8, make_uint4(swap16(wl[0]) ^ SF, swap16(wl[1]) ^ SF, swap16(wl[2]) ^ SF,
                                                        swap16(wl[3]) ^ SF));
        }
      }
#pragma unroll
      for (int i = 0; i < TC; ++i) {
        if (i < tt) {
          const uint32_t* rowp = buf + (16 * i + r16) * L::STRIDE + 4 * q4;
          const bf16x8 th = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(rowp));
          if (X3) {
            const bf16x8 tl = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(rowp + PLANE));
#pragma unroll
            for (int u = 0; u < TB; ++u) {
              accr[i][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(tl, bh[u], accr[i][u], 0, 0, 0);
              accr[i][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(th, bl[u], accr[i][u], 0, 0, 0);
              accr[i][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(th, bh[u], accr[i][u], 0, 0, 0);
              acci[i][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(tl, sh[u], acci[i][u], 0, 0, 0);
              acci[i][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(th, sl[u], acci[i][u], 0, 0, 0);
              acci[i][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(th, sh[u], acci[i][u], 0, 0, 0);
            }
          } else {
#pragma unroll
            for (int u = 0; u < TB; ++u) {
              accr[i][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(th, bh[u], accr[i][u], 0, 0, 0);
              acci[i][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(th, sh[u], acci[i][u], 0, 0, 0);
            }
          }
        }
      }
    }
  };

  // ---- main loop over the full K steps: LDS double buffer for the thin
  // operand, A_f fetched two steps ahead into a ring of three register sets
  // (unrolled by three so that every set keeps a fixed role).  Loads complete
  // in issue order, so the thin block needed at the end of a step is requested
  // before the A_f prefetch; prefetch indices past the last full step are
  // clamped (the data is not used). ----
  const int nfull = (ke - kb) / KSTEP;
  const bool tail = kb + nfull * KSTEP < ke;
  float bq0[TB][8], bq1[TB][8], bq2[TB][8];
  float2 tx[TEL];
  if (nfull > 0) {
    load_big_full(kb, bq0);
    load_big_full(kb + (nfull > 1 ? KSTEP : 0), bq1);
    load_thin_full(kb, tx);
    store_thin(lds, tx);
  }
  __syncthreads();
  // Step s of the ring (steps past the last full one only load and store
  // clamped data).  The LDS store and the barrier are unconditional, so that
  // the thin loads have a use outside the guarded MFMA phase and stay ahead of
  // the A_f prefetch (sunk into that phase they would follow it, and the wait
  // before the store would also wait for the prefetch).  A store past the
  // last full step rewrites, with the same thread's words, a buffer that no
  // later full step reads, after the barrier of the step that last read it.
  auto step = [&](int s, const float (&cur)[TB][8], float (&pre)[TB][8]) {
    const int sn = s + 1 < nfull ? s + 1 : nfull - 1;
    const int sp2 = s + 2 < nfull ? s + 2 : nfull - 1;
    load_thin_full(kb + sn * KSTEP, tx);
    load_big_full(kb + sp2 * KSTEP, pre);
    if (s < nfull) {
      // the MFMA phase at raised wave priority: the other workgroup's waves on
      // the SIMD, between their loads and LDS stores, issue around it
      __builtin_amdgcn_s_setprio(1);
      compute(lds + (s & 1) * BUF, cur);
      __builtin_amdgcn_s_setprio(0);
    }
    store_thin(lds + ((s + 1) & 1) * BUF, tx);
    __syncthreads();
  };
  for (int s = 0; s < nfull; s += 3) {
    step(s, bq0, bq2);
    step(s + 1, bq1, bq0);
    step(s + 2, bq2, bq1);
  }
  if (tail) {  // ragged last step, guarded loads
    const int k0 = kb + nfull * KSTEP;
    load_thin(k0, tx);
    store_thin(lds + (nfull & 1) * BUF, tx);
    load_big(k0, bq0);
    __syncthreads();
    compute(lds + (nfull & 1) * BUF, bq0);
  }

  // ---- epilogue: accr / acci[i][u][r] = parts of C[col][n0 + 16 i + 4 q4 + r] ----
  float* out;
  int64_t ldo;
  if (rt >= 0) {
    // tail split: the (tile, split) block of 128 big rows x NCH columns,
    // indexed from the tile's first row and column
    constexpr int BROWS = NWAVE * 16 * TB;
    out = a.part + 2 * (((int64_t)rt * a.rsplit + sp) * BROWS * NCH) - 2 * ((int64_t)bt * BROWS * NCH + n0);
    ldo = 2 * NCH;
  } else if (a.nsplit > 1) {
    out = a.part + 2 * ((int64_t)sp * a.batch + f) * a.M * a.N;
    ldo = 2 * (int64_t)a.N;
  } else {
    out = a.C + (int64_t)f * a.strideC;
    ldo = a.ldc;
  }
#pragma unroll
  for (int i = 0; i < TC; ++i) {
    if (i < tt) {
      const int n = n0 + 16 * i + 4 * q4;
#pragma unroll
      for (int u = 0; u < TB; ++u) {
        if (!colok[u]) continue;
        float* p = out + (int64_t)col[u] * ldo + 2 * n;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (n + r >= a.N) continue;
          float2* o = reinterpret_cast<float2*>(p + 2 * r);
          if (a.sub) {
            const float2 c0 = *o;
            *o = make_float2(c0.x - accr[i][u][r], c0.y - acci[i][u][r]);
          } else {
            *o = make_float2(accr[i][u][r], acci[i][u][r]);
          }
        }
      }
    }
  }
}

// (hi, lo) bf16 pairs, the big-operand form of KM_BF16X3_SPLIT:
// Xs[f][k][n] = pairs of X[f][k][n] (complex FP32, row stride ldx, slice
// stride strideX, in floats), dense K x N per slice.
__global__ void kgemm_split_thin_kernel(const float* __restrict__ X, int64_t ldx, int64_t strideX, int K, int N,
                                        int batch, uint2* __restrict__ Xs) {
  const int64_t per = (int64_t)K * N, total = per * batch;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t f = e / per, rem = e - f * per;
    const int k = (int)(rem / N), n = (int)(rem - (int64_t)k * N);
    const float2 x = *reinterpret_cast<const float2*>(X + f * strideX + (int64_t)k * ldx + 2 * n);
    const __bf16 hr = (__bf16)x.x, hi = (__bf16)x.y;
    const __bf16 lr = (__bf16)(x.x - (float)hr), li = (__bf16)(x.y - (float)hi);
    uint2 o;
    o.x = (uint32_t)__builtin_bit_cast(unsigned short, hr) | ((uint32_t)__builtin_bit_cast(unsigned short, hi) << 16);
    o.y = (uint32_t)__builtin_bit_cast(unsigned short, lr) | ((uint32_t)__builtin_bit_cast(unsigned short, li) << 16);
    Xs[e] = o;
  }
}

// C[f][row][n] = sum_s part[s][f][row][n] (fixed order), complex FP32.
__global__ void kgemm_reduce_kernel(const float2* __restrict__ part, int nsplit, int batch, int M, int N,
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

// C of the split remainder tiles: sum of the rsplit partial blocks of each
// (fixed order), written where the tile lies in C.
__global__ void kgemm_tail_reduce_kernel(const float2* __restrict__ part, int nfull, int nrem, int rsplit, int nbig,
                                         int nthin, int brows, int nch, int M, int N, float2* __restrict__ C,
                                         int64_t ldc, int64_t strideC) {
  const int64_t per = (int64_t)brows * nch;
  const int64_t total = per * nrem;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int rt = (int)(e / per);
    const int rem = (int)(e - (int64_t)rt * per);
    const int rl = rem / nch, nl = rem - (rem / nch) * nch;
    int u = nfull + rt;
    const int bt = u % nbig;
    u /= nbig;
    const int tc = u % nthin, f = u / nthin;
    const int row = bt * brows + rl, n = tc * nch + nl;
    if (row >= M || n >= N) continue;
    const float2* p = part + (int64_t)rt * rsplit * per + rem;
    float2 sum = p[0];
    for (int j = 1; j < rsplit; ++j) {
      const float2 v = p[(int64_t)j * per];
      sum.x += v.x;
      sum.y += v.y;
    }
    C[f * strideC + (int64_t)row * ldc + n] = sum;
  }
}

template <int MODE, bool HN, int TT, bool AVEC, bool FULL>
hipError_t launch_ttaf(const KArgs& a, hipStream_t s) {
  constexpr int TB = 2;
  const size_t lds = (size_t)2 * TT * 8 * Lds<MODE>::STRIDE * Lds<MODE>::PLANES * 4;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)kgemm_kernel<MODE, HN, TT, TB, AVEC, FULL>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipGetLastError();
    attr = true;
  }
  hipLaunchKernelGGL((kgemm_kernel<MODE, HN, TT, TB, AVEC, FULL>), dim3(8 * a.per), dim3(256), lds, s, a);
  return hipGetLastError();
}

// FULL: every thin chunk, the last one included, fills all TT tiles, so the
// per-tile guards are compile-time and the tile loop is straight-line code.
template <int MODE, bool HN, int TT, bool AVEC>
hipError_t launch_tta(const KArgs& a, hipStream_t s) {
  constexpr int NCH = TT * 8;
  const int nlast = a.N - (a.nthin - 1) * NCH;
  if ((nlast + 15) / 16 == TT / 2) return launch_ttaf<MODE, HN, TT, AVEC, true>(a, s);
  return launch_ttaf<MODE, HN, TT, AVEC, false>(a, s);
}

template <int MODE, bool HN, int TT>
hipError_t launch_tt(const KArgs& a, hipStream_t s) {
  // vector loads only matter for A X (rows of A_f along K)
  if (!HN && a.avec) return launch_tta<MODE, HN, TT, true>(a, s);
  return launch_tta<MODE, HN, TT, false>(a, s);
}

template <int MODE, bool HN>
hipError_t launch_mode(const KArgs& a, int TT, hipStream_t s) {
  switch (TT) {
    case 4: return launch_tt<MODE, HN, 4>(a, s);
    case 8: return launch_tt<MODE, HN, 8>(a, s);
    case 14: return launch_tt<MODE, HN, 14>(a, s);
    default: return launch_tt<MODE, HN, 16>(a, s);
  }
}

}  // namespace

int kgemm_thin_tiles(int N) {
  const int nn = N < 128 ? N : 128;
  if (nn <= 32) return 4;
  if (nn <= 64) return 8;
  if (nn <= 112) return 14;
  return 16;
}

namespace {

// Concurrent workgroup slots of the product kernel: two per CU.
int kgemm_slots() {
  static int slots = 0;
  if (!slots) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                 hipSuccess || cus <= 0)
      cus = 256;
    slots = 2 * cus;
  }
  return slots;
}

// Tail split of an unsplit product: with T tiles over S slots, the last
// T mod S tiles would run as a nearly empty extra round; they are split
// along K instead so that the round takes a fraction of a tile's time.
struct TailPlan {
  int nfull, nrem, rsplit, rkchunk;
  size_t bytes;
};
TailPlan kgemm_tail_plan(int M, int K, int N, int batch) {
  TailPlan t{0, 0, 0, 0, 0};
  const int TT = kgemm_thin_tiles(N);
  const int64_t nthin = (N + 8 * TT - 1) / (8 * TT);
  const int64_t nbig = (M + NWAVE * 16 * 2 - 1) / (NWAVE * 16 * 2);
  const int64_t tiles = nthin * nbig * batch;
  const int64_t S = kgemm_slots();
  const int64_t nfull = tiles / S * S / 8 * 8;
  const int64_t nrem = tiles - nfull;
  if (nfull == 0 || nrem == 0) return t;
  int rs = (int)std::min<int64_t>(16, S / nrem);
  rs = std::min(rs, K / (8 * KSTEP));  // at least 8 K steps per split
  if (rs < 2) return t;
  int kc = (K + rs - 1) / rs;
  kc = (kc + KSTEP - 1) / KSTEP * KSTEP;
  t.nfull = (int)nfull;
  t.nrem = (int)nrem;
  t.rsplit = (K + kc - 1) / kc;
  t.rkchunk = kc;
  t.bytes = (size_t)nrem * t.rsplit * (NWAVE * 16 * 2) * (8 * TT) * 8;
  return t;
}

}  // namespace

hipError_t split_bf16x3(const void* in, void* out, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(kgemm_split_thin_kernel, dim3(blocks), dim3(256), 0, s, static_cast<const float*>(in), (int64_t)2,
                     2 * n, (int)n, 1, 1, static_cast<uint2*>(out));
  return hipGetLastError();
}

size_t kgemm_part_bytes(int M, int K, int N, int batch, int nsplit) {
  if (nsplit > 1) return (size_t)nsplit * batch * M * N * 8;
  return kgemm_tail_plan(M, K, N, batch).bytes;
}

int kgemm_split(int M, int K, int N, int batch, int* kchunk) {
  const int TT = kgemm_thin_tiles(N);
  const int64_t nthin = (N + 8 * TT - 1) / (8 * TT);
  const int64_t nbig = (M + NWAVE * 16 * 2 - 1) / (NWAVE * 16 * 2);
  const int64_t tiles = nthin * nbig * batch;
  int ns = 1;
  while (tiles * ns < 512 && ns < 8 && (int64_t)K / (2 * ns) >= 256) ns *= 2;
  int kc = (K + ns - 1) / ns;
  kc = (kc + KSTEP - 1) / KSTEP * KSTEP;
  ns = (K + kc - 1) / kc;
  if (ns < 1) ns = 1;
  *kchunk = kc < KSTEP ? KSTEP : kc;
  return ns;
}

int kgemm_split_balanced(int M, int K, int N, int batch) {
  static int slots = 0;
  if (!slots) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                 hipSuccess || cus <= 0)
      cus = 256;
    slots = 2 * cus;  // two workgroups per CU (launch bounds)
  }
  const int TT = kgemm_thin_tiles(N);
  const int64_t tiles = (int64_t)((N + 8 * TT - 1) / (8 * TT)) * ((M + NWAVE * 16 * 2 - 1) / (NWAVE * 16 * 2)) * batch;
  int best = 1;
  double best_cost = 1e300;
  for (int ns = 1; ns <= 16; ++ns) {
    int kc = (K + ns - 1) / ns;
    kc = (kc + KSTEP - 1) / KSTEP * KSTEP;
    if ((K + kc - 1) / kc != ns) continue;  // the chunking gives fewer splits
    const int64_t rounds = (tiles * ns + slots - 1) / slots;
    const double cost = (double)rounds * (kc / KSTEP + 6);
    if (cost < best_cost) {
      best_cost = cost;
      best = ns;
    }
  }
  return best;
}

hipError_t kgemm(const KGemmDesc& d, hipStream_t s) {
  const int M = d.herm ? d.cols : d.rows;
  const int K = d.herm ? d.rows : d.cols;
  if (M <= 0 || d.N <= 0 || d.batch <= 0) return hipSuccess;
  KArgs a;
  a.A = static_cast<const float*>(d.A);
  a.lda = 2 * d.lda;
  a.strideA = 2 * d.strideA;
  a.X = static_cast<const float*>(d.X);
  a.ldx = 2 * d.ldx;
  a.strideX = 2 * d.strideX;
  a.C = static_cast<float*>(d.C);
  a.ldc = 2 * d.ldc;
  a.strideC = 2 * d.strideC;
  a.part = static_cast<float*>(d.part);
  a.M = M;
  a.K = K;
  a.N = d.N;
  a.batch = d.batch;
  int kchunk = K;
  a.nsplit = d.nsplit > 1 ? d.nsplit : 1;
  if (a.nsplit > 1) {
    if (!d.part) return hipErrorInvalidValue;
    kchunk = (K + a.nsplit - 1) / a.nsplit;
    kchunk = (kchunk + KSTEP - 1) / KSTEP * KSTEP;
  }
  a.kchunk = kchunk;
  const int TT = kgemm_thin_tiles(d.N);
  a.nthin = (d.N + 8 * TT - 1) / (8 * TT);
  a.nbig = (M + NWAVE * 16 * 2 - 1) / (NWAVE * 16 * 2);
  const int64_t total = (int64_t)a.nbig * a.nthin * a.nsplit * d.batch;
  if (total >= (int64_t)1 << 30) return hipErrorInvalidValue;
  a.total = (int)total;
  a.per = (a.total + 7) / 8;
  a.avec = ((d.lda & 1) == 0 && (d.strideA & 1) == 0 && ((uintptr_t)d.A & 15) == 0) ? 1 : 0;
  a.nfull = a.nrem = a.rsplit = a.rkchunk = 0;
  a.sub = d.sub ? 1 : 0;
  if (a.sub && a.nsplit > 1) return hipErrorInvalidValue;
  TailPlan tp{0, 0, 0, 0, 0};
  if (a.nsplit == 1 && d.part && !a.sub) {
    tp = kgemm_tail_plan(M, K, d.N, d.batch);
    if (tp.rsplit > 1 && d.part_bytes >= tp.bytes) {
      a.nfull = tp.nfull;
      a.nrem = tp.nrem;
      a.rsplit = tp.rsplit;
      a.rkchunk = tp.rkchunk;
      a.per = tp.nfull / 8 + (tp.nrem * tp.rsplit + 7) / 8;
    } else {
      tp.rsplit = 0;
    }
  }
  hipError_t e;
  switch (d.mode) {
    case KM_F32: e = d.herm ? launch_mode<KM_F32, true>(a, TT, s) : launch_mode<KM_F32, false>(a, TT, s); break;
    case KM_BF16: e = d.herm ? launch_mode<KM_BF16, true>(a, TT, s) : launch_mode<KM_BF16, false>(a, TT, s); break;
    case KM_BF16X3:
      e = d.herm ? launch_mode<KM_BF16X3, true>(a, TT, s) : launch_mode<KM_BF16X3, false>(a, TT, s);
      break;
    case KM_BF16X3_SPLIT:
      e = d.herm ? launch_mode<KM_BF16X3_SPLIT, true>(a, TT, s) : launch_mode<KM_BF16X3_SPLIT, false>(a, TT, s);
      break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  if (a.rsplit > 1) {
    const int TT = kgemm_thin_tiles(d.N);
    const int64_t n = (int64_t)a.nrem * (NWAVE * 16 * 2) * (8 * TT);
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(kgemm_tail_reduce_kernel, dim3(blocks), dim3(256), 0, s, (const float2*)d.part, a.nfull, a.nrem,
                       a.rsplit, a.nbig, a.nthin, NWAVE * 16 * 2, 8 * TT, M, d.N, (float2*)d.C, d.ldc, d.strideC);
    return hipGetLastError();
  }
  if (a.nsplit <= 1) return e;
  const int64_t n = (int64_t)M * d.N * d.batch;
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(kgemm_reduce_kernel, dim3(blocks), dim3(256), 0, s, (const float2*)d.part, a.nsplit, d.batch, M,
                     d.N, (float2*)d.C, d.ldc, d.strideC);
  return hipGetLastError();
}

}  // namespace tsvd
