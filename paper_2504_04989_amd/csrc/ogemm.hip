// FP64-arithmetic products of the orthonormalisation and the small SVD on
// FP32-stored blocks (gfx950 v_mfma_f64_16x16x4_f64):
//   TN:  P_s[f] = X_f^H Y_f over the rows of chunk s      (block Grams,
//        projections against earlier blocks, G_f = C_f C_f^H = T_f^H T_f)
//   NN:  C_f = alpha X_f B_f + beta C_f with B_f FP64      (W R^{-1}, W - Q C)
// FP32 operands are widened to FP64 exactly, so every product is exact and
// sums are accumulated in FP64: the Gram matrices and projection
// coefficients carry FP64 accuracy of the stored blocks.
//
// Same structure as the Krylov-product kernel: complex arithmetic as a real
// GEMM over interleaved storage, the tall operand X (n rows, read once)
// streams from HBM into the MFMA registers of one wave, the small operand is
// expanded into real form in LDS (double buffered) and shared by the 4 waves:
//   TN: P[j][2n+t] = sum_{i,s} X_int[i][2j+s] Ye[2n+t][2i+s],
//       Ye[2n] = (yr, yi), Ye[2n+1] = (yi, -yr)        (y = Y[i][n])
//   NN: C[m][2n+t] = sum_{k,s} X_int[m][2k+s] Be[2n+t][2k+s],
//       Be[2n] = (br, -bi), Be[2n+1] = (bi, br)        (b = B[k][n])
// K step: 8 complex (16 real); lane (q4, r16) owns real k' = 4 q4 .. 4 q4 + 3
// of each step, MFMA block b takes k' = 4 q4 + b.  Accumulator r of lane
// (q4, r16) holds real output row 16 i + q4 + 4 r, i.e. the real (q4 even)
// or imaginary (q4 odd) part of complex column n = 8 i + q4 / 2 + 2 r.
#include <algorithm>
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace tsvd {

namespace {

constexpr int OKSTEP = 8;
constexpr int OSTRIDE = 2 * OKSTEP + 2;  // doubles per LDS row (16 + pad)

struct OArgs {
  const float* X;  // tall FP32 operand (floats)
  int64_t lx, strideX;
  const void* B;   // small operand: FP32 (TN) or FP64 (NN), in its own element type
  int64_t ldb, strideB, bsum_stride;
  int nsum;
  void* C;         // TN: FP64 partials [split][f][M][N]; NN: FP32 output
  int64_t ldc, strideC;
  double alpha, beta;
  int M, K, N, batch;
  int nsplit, kchunk;
  int nbig, nthin, total, per;
  int xvec;
  int upper;  // TN: skip tiles strictly below the diagonal of a square product
  int triu;   // NN: B is upper triangular (zeros below the diagonal, stored)
};

template <bool TN, int TT, bool XVEC>
__global__ __launch_bounds__(256, 2) void ogemm_kernel(const OArgs a) {
  constexpr int ROWS = TT * 16;
  constexpr int BUF = ROWS * OSTRIDE;
  constexpr int NCH = TT * 8;
  constexpr int TEL = OKSTEP * NCH / 256;
  static_assert(TEL * 256 == OKSTEP * NCH, "thin split");
  extern __shared__ __align__(16) double olds[];

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
  const int n0 = tc * NCH;
  const int nc = min(NCH, a.N - n0);
  const int tt = (2 * nc + 15) / 16;
  if (TN && a.upper && bt * 64 > n0 + NCH - 1) return;  // every entry of this tile has row > column

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int q4 = lane >> 4, r16 = lane & 15;
  const float* Xf = a.X + (int64_t)f * a.strideX;
  const int col = bt * 64 + wave * 16 + r16;
  const bool colok = col < a.M;
  const int colc = colok ? col : a.M - 1;  // clamped: loads stay in bounds, results unused

  auto load_big = [&](int k0, float (&v)[4]) {
    const bool full = k0 + OKSTEP <= ke;
    if (!TN) {
      const float* p = Xf + (int64_t)col * a.lx + 2 * (k0 + 2 * q4);
      if (colok && full && XVEC) {
        const float4 x = *reinterpret_cast<const float4*>(p);
        v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
      } else {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          float2 x = make_float2(0.f, 0.f);
          if (colok && k0 + 2 * q4 + c < ke) x = *reinterpret_cast<const float2*>(p + 2 * c);
          v[2 * c] = x.x;
          v[2 * c + 1] = x.y;
        }
      }
    } else {
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int i = k0 + 2 * q4 + c;
        float2 x = make_float2(0.f, 0.f);
        if (colok && (full || i < ke)) x = *reinterpret_cast<const float2*>(Xf + (int64_t)i * a.lx + 2 * col);
        v[2 * c] = x.x;
        v[2 * c + 1] = x.y;
      }
    }
  };

  // full K steps: loads issued unconditionally (clamped addresses, zero by
  // select) so that wait counts can leave the next step's loads in flight
  auto load_big_full = [&](int k0, float (&v)[4]) {
    if (!TN) {
      const float* p = Xf + (int64_t)colc * a.lx + 2 * (k0 + 2 * q4);
      if (XVEC) {
        const float4 x = *reinterpret_cast<const float4*>(p);
        v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
      } else {
        const float2 x0 = *reinterpret_cast<const float2*>(p);
        const float2 x1 = *reinterpret_cast<const float2*>(p + 2);
        v[0] = x0.x; v[1] = x0.y; v[2] = x1.x; v[3] = x1.y;
      }
    } else {
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const float2 x = *reinterpret_cast<const float2*>(Xf + (int64_t)(k0 + 2 * q4 + c) * a.lx + 2 * colc);
        v[2 * c] = x.x;
        v[2 * c + 1] = x.y;
      }
    }
  };
  // the thin block is held as loaded (FP32 pairs for TN, FP64 for NN) and
  // widened, and its padding columns cleared, only when it is stored to LDS:
  // nothing waits for the loads before the next step's MFMAs have been issued
  typedef typename std::conditional<TN, float2, double2>::type Raw;
  auto load_thin_full = [&](int k0, Raw (&x)[TEL]) {
#pragma unroll
    for (int e = 0; e < TEL; ++e) {
      const int idx = tid + e * 256;
      const int kk = idx % OKSTEP, nn = idx / OKSTEP;
      const int64_t off = (int64_t)f * a.strideB + (int64_t)(k0 + kk) * a.ldb + (n0 + (nn < nc ? nn : 0));
      x[e] = reinterpret_cast<const Raw*>(a.B)[off];
    }
  };

  auto load_thin = [&](int k0, Raw (&x)[TEL]) {
#pragma unroll
    for (int e = 0; e < TEL; ++e) {
      const int idx = tid + e * 256;
      const int kk = idx % OKSTEP, nn = idx / OKSTEP;
      Raw v{};
      if (k0 + kk < ke && nn < nc) v = reinterpret_cast<const Raw*>(a.B)[(int64_t)f * a.strideB + (int64_t)(k0 + kk) * a.ldb + (n0 + nn)];
      x[e] = v;
    }
  };
  auto store_thin = [&](double* buf, const Raw (&x)[TEL]) {
#pragma unroll
    for (int e = 0; e < TEL; ++e) {
      const int idx = tid + e * 256;
      const int kk = idx % OKSTEP, nn = idx / OKSTEP;
      const bool ok = nn < nc;
      const double xr = ok ? (double)x[e].x : 0.0, xi = ok ? (double)x[e].y : 0.0;
      double* row0 = buf + (2 * nn) * OSTRIDE + 2 * kk;
      double* row1 = row0 + OSTRIDE;
      if (TN) {
        *reinterpret_cast<double2*>(row0) = make_double2(xr, xi);
        *reinterpret_cast<double2*>(row1) = make_double2(xi, -xr);
      } else {
        *reinterpret_cast<double2*>(row0) = make_double2(xr, -xi);
        *reinterpret_cast<double2*>(row1) = make_double2(xi, xr);
      }
    }
  };

  f64x4 acc[TT];
#pragma unroll
  for (int i = 0; i < TT; ++i) acc[i] = f64x4{0.0, 0.0, 0.0, 0.0};

  // NN with upper-triangular B: in the K step starting at complex row k0,
  // thin tiles i < (k0 - n0) / 8 see only zeros of B and are skipped (exact)
  // TN with `upper`: thin tiles whose columns all lie below the wave's first
  // output row (n0 + 8 i + 8 <= first column of this wave) give only entries
  // below the diagonal, which the consumer does not read
  auto tile0 = [&](int k0) {
    if (TN) {
      if (!a.upper) return 0;
      const int cmin = bt * 64 + wave * 16;
      return cmin > n0 ? (cmin - n0) / 8 : 0;
    }
    return (a.triu && k0 > n0) ? (k0 - n0) / 8 : 0;
  };
  auto compute = [&](const double* buf, const float (&v)[4], int istart) {
    const double bv[4] = {(double)v[0], (double)v[1], (double)v[2], (double)v[3]};
#pragma unroll
    for (int i = 0; i < TT; ++i) {
      if (i < tt && i >= istart) {
        const double* rowp = buf + (16 * i + r16) * OSTRIDE + 4 * q4;
        const double2 w0 = *reinterpret_cast<const double2*>(rowp);
        const double2 w1 = *reinterpret_cast<const double2*>(rowp + 2);
        const double w[4] = {w0.x, w0.y, w1.x, w1.y};
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(w[b], bv[b], acc[i], 0, 0, 0);
      }
    }
  };

  // main loop over the full K steps (LDS double buffer, next step's tall
  // operand in registers; the thin block is requested first because loads
  // complete in issue order), unrolled by two so that the two register sets
  // of the tall operand swap roles instead of being copied (a copy would wait
  // for the loads in flight); then a guarded ragged step
  const int nfull = (ke - kb) / OKSTEP;
  const bool tail = kb + nfull * OKSTEP < ke;
  float bA[4], bB[4];
  Raw tx[TEL];
  if (nfull > 0) {
    load_big_full(kb, bA);
    load_thin_full(kb, tx);
    store_thin(olds, tx);
  }
  __syncthreads();
  auto step = [&](int s, const float (&cur)[4], float (&nxt)[4]) {
    const int sn = s + 1 < nfull ? s + 1 : s;
    load_thin_full(kb + sn * OKSTEP, tx);
    load_big_full(kb + sn * OKSTEP, nxt);
    compute(olds + (s & 1) * BUF, cur, tile0(kb + s * OKSTEP));
    if (s + 1 < nfull) store_thin(olds + ((s + 1) & 1) * BUF, tx);
    __syncthreads();
  };
  for (int s = 0; s < nfull; s += 2) {
    step(s, bA, bB);
    if (s + 1 >= nfull) break;
    step(s + 1, bB, bA);
  }
  if (tail) {
    const int k0 = kb + nfull * OKSTEP;
    load_thin(k0, tx);
    store_thin(olds + (nfull & 1) * BUF, tx);
    load_big(k0, bA);
    __syncthreads();
    compute(olds + (nfull & 1) * BUF, bA, tile0(k0));
  }

  // Lanes q4 and q4 ^ 1 hold the real and the imaginary parts of the same
  // four columns n = n0 + 8 i + q4 / 2 + 2 r; after one exchange the even lane
  // stores r = 0, 1 and the odd lane r = 2, 3 as whole complex numbers.
  if (!colok) return;  // the partner lane (same column) returns too
  const bool odd = q4 & 1;
#pragma unroll
  for (int i = 0; i < TT; ++i) {
    if (i < tt) {
      double other[4];
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) other[rr] = __shfl_xor(acc[i][rr], 16, 64);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int rr = odd ? 2 + h : h;
        const double re = odd ? other[rr] : acc[i][rr];
        const double im = odd ? acc[i][rr] : other[rr];
        const int n = n0 + 8 * i + (q4 >> 1) + 2 * rr;
        if (n >= a.N) continue;
        if (TN) {
          double2* out = static_cast<double2*>(a.C) + (((int64_t)sp * a.batch + f) * a.M * a.N + (int64_t)col * a.N + n);
          *out = make_double2(re, im);
        } else {
          float2* out = static_cast<float2*>(a.C) + ((int64_t)f * a.strideC + (int64_t)col * a.ldc + n);
          double vr = a.alpha * re, vi = a.alpha * im;
          if (a.beta != 0.0) {
            const float2 o = *out;
            vr += a.beta * (double)o.x;
            vi += a.beta * (double)o.y;
          }
          *out = make_float2((float)vr, (float)vi);
        }
      }
    }
  }
}

// TN product of a square block with itself, upper triangle only, N <= 120
// (the block Grams): with one 64-row tile per wave the upper-triangle skip
// leaves the waves unequal (14, 12, 10, 8 thin tiles for N = 110, and a second
// row tile of mostly padding).  Here wave w owns the row groups w and 7 - w
// (16 rows each), 2 tt - 14 <= 16 thin tiles in all, and one workgroup per
// slice and split covers the whole triangle.  Accumulator slot s holds thin
// tile s of group w when 2 w <= s < tt, else the next tile of group 7 - w.
__global__ __launch_bounds__(256, 2) void ogemm_tn_pair_kernel(const OArgs a) {
  constexpr int TT = 16;
  constexpr int ROWS = TT * 16;
  constexpr int BUF = ROWS * OSTRIDE;
  constexpr int NCH = TT * 8;
  constexpr int TEL = OKSTEP * NCH / 256;
  extern __shared__ __align__(16) double olds[];

  const int id = blockIdx.x;
  const int t = (id & 7) * a.per + (id >> 3);
  if (t >= a.total) return;
  const int sp = t % a.nsplit;
  const int f = t / a.nsplit;
  const int kb = sp * a.kchunk;
  const int ke = min(a.K, kb + a.kchunk);
  const int nc = a.N;
  const int tt = (2 * nc + 15) / 16;

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: slot choices branch on scalars
  const int q4 = lane >> 4, r16 = lane & 15;
  const float* Xf = a.X + (int64_t)f * a.strideX;
  const int ga = wave, gb = 7 - wave;
  const int cola = 16 * ga + r16, colb = 16 * gb + r16;
  const bool oka = cola < a.M, okb = colb < a.M;
  const int cla = oka ? cola : a.M - 1, clb = okb ? colb : a.M - 1;

  auto load_big = [&](int k0, int col, bool ok, bool full, float (&v)[4]) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int i = k0 + 2 * q4 + c;
      float2 x = make_float2(0.f, 0.f);
      if (ok && (full || i < ke)) x = *reinterpret_cast<const float2*>(Xf + (int64_t)i * a.lx + 2 * col);
      v[2 * c] = x.x;
      v[2 * c + 1] = x.y;
    }
  };
  auto load_big_full = [&](int k0, int col, float (&v)[4]) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const float2 x = *reinterpret_cast<const float2*>(Xf + (int64_t)(k0 + 2 * q4 + c) * a.lx + 2 * col);
      v[2 * c] = x.x;
      v[2 * c + 1] = x.y;
    }
  };
  // full steps: every load issued, unconditionally, so that the next step's
  // loads stay in flight across this step's MFMAs.  Padding columns nn >= N
  // read column N - 1 instead of zeros: a thin row only reaches the output
  // rows it forms itself, and rows n >= N are never stored.
  // held as loaded (FP32 pairs), widened when stored to LDS
  auto load_thin_full = [&](int k0, float2 (&x)[TEL]) {
#pragma unroll
    for (int e = 0; e < TEL; ++e) {
      const int idx = tid + e * 256;
      const int kk = idx % OKSTEP, nn = min(idx / OKSTEP, nc - 1);
      x[e] = reinterpret_cast<const float2*>(a.B)[(int64_t)f * a.strideB + (int64_t)(k0 + kk) * a.ldb + nn];
    }
  };
  auto load_thin = [&](int k0, float2 (&x)[TEL]) {
#pragma unroll
    for (int e = 0; e < TEL; ++e) {
      const int idx = tid + e * 256;
      const int kk = idx % OKSTEP, nn = idx / OKSTEP;
      float2 v = make_float2(0.f, 0.f);
      if (k0 + kk < ke && nn < nc) v = reinterpret_cast<const float2*>(a.B)[(int64_t)f * a.strideB + (int64_t)(k0 + kk) * a.ldb + nn];
      x[e] = v;
    }
  };
  auto store_thin = [&](double* buf, const float2 (&x)[TEL]) {
#pragma unroll
    for (int e = 0; e < TEL; ++e) {
      const int idx = tid + e * 256;
      const int kk = idx % OKSTEP, nn = idx / OKSTEP;
      const double xr = (double)x[e].x, xi = (double)x[e].y;
      double* row0 = buf + (2 * nn) * OSTRIDE + 2 * kk;
      double* row1 = row0 + OSTRIDE;
      *reinterpret_cast<double2*>(row0) = make_double2(xr, xi);
      *reinterpret_cast<double2*>(row1) = make_double2(xi, -xr);
    }
  };
  // slot s -> (group b?, thin tile); tile >= tt: unused slot
  auto slot_tile = [&](int s, bool& useb) {
    if (s >= 2 * ga && s < tt) {
      useb = false;
      return s;
    }
    useb = true;
    const int idx = s < 2 * ga ? s : 2 * ga + (s - tt);
    return 2 * gb + idx;
  };

  f64x4 acc[TT];
#pragma unroll
  for (int i = 0; i < TT; ++i) acc[i] = f64x4{0.0, 0.0, 0.0, 0.0};
  auto compute = [&](const double* buf, const float (&va)[4], const float (&vb)[4]) {
    // register vectors, selected whole (a select between two arrays would
    // become a select between their addresses, i.e. private memory)
    const f64x4 dav = {(double)va[0], (double)va[1], (double)va[2], (double)va[3]};
    const f64x4 dbv = {(double)vb[0], (double)vb[1], (double)vb[2], (double)vb[3]};
#pragma unroll
    for (int s = 0; s < TT; ++s) {
      bool useb;
      const int tile = slot_tile(s, useb);
      if (tile < tt) {
        const double* rowp = buf + (16 * tile + r16) * OSTRIDE + 4 * q4;
        const double2 w0 = *reinterpret_cast<const double2*>(rowp);
        const double2 w1 = *reinterpret_cast<const double2*>(rowp + 2);
        const double w[4] = {w0.x, w0.y, w1.x, w1.y};
        const f64x4 bv = useb ? dbv : dav;
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(w[bb], bv[bb], acc[s], 0, 0, 0);
      }
    }
  };

  const int nfull = (ke - kb) / OKSTEP;
  const bool tail = kb + nfull * OKSTEP < ke;
  // unrolled by two: the register sets swap roles rather than being copied
  float aA[4], bA[4], aB[4], bB[4];
  float2 tx[TEL];
  if (nfull > 0) {
    load_big_full(kb, cla, aA);
    load_big_full(kb, clb, bA);
    load_thin_full(kb, tx);
    store_thin(olds, tx);
  }
  __syncthreads();
  auto step = [&](int s, const float (&ca)[4], const float (&cb)[4], float (&na)[4], float (&nb)[4]) {
    const int sn = s + 1 < nfull ? s + 1 : s;
    load_thin_full(kb + sn * OKSTEP, tx);
    load_big_full(kb + sn * OKSTEP, cla, na);
    load_big_full(kb + sn * OKSTEP, clb, nb);
    compute(olds + (s & 1) * BUF, ca, cb);
    if (s + 1 < nfull) store_thin(olds + ((s + 1) & 1) * BUF, tx);
    __syncthreads();
  };
  for (int s = 0; s < nfull; s += 2) {
    step(s, aA, bA, aB, bB);
    if (s + 1 >= nfull) break;
    step(s + 1, aB, bB, aA, bA);
  }
  if (tail) {
    const int k0 = kb + nfull * OKSTEP;
    load_thin(k0, tx);
    store_thin(olds + (nfull & 1) * BUF, tx);
    load_big(k0, cla, oka, false, aA);
    load_big(k0, clb, okb, false, bA);
    __syncthreads();
    compute(olds + (nfull & 1) * BUF, aA, bA);
  }

  // lanes q4 and q4 ^ 1 hold the real and the imaginary parts of the same
  // columns (same row pair): one exchange, then whole complex numbers
  const bool odd = q4 & 1;
#pragma unroll
  for (int s = 0; s < TT; ++s) {
    bool useb;
    const int tile = slot_tile(s, useb);
    if (tile >= tt) continue;
    double other[4];
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) other[rr] = __shfl_xor(acc[s][rr], 16, 64);
    const int col = useb ? colb : cola;
    if (!(useb ? okb : oka)) continue;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int rr = odd ? 2 + h : h;
      const double re = odd ? other[rr] : acc[s][rr];
      const double im = odd ? acc[s][rr] : other[rr];
      const int n = 8 * tile + (q4 >> 1) + 2 * rr;
      if (n >= a.N) continue;
      double2* out = static_cast<double2*>(a.C) + (((int64_t)sp * a.batch + f) * a.M * a.N + (int64_t)col * a.N + n);
      *out = make_double2(re, im);
    }
  }
}

// part[e] = sum_s part[s * total + e] in a fixed order (slot 0 in place).
__global__ void opart_reduce_kernel(double2* part, int nsplit, int64_t total) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    double2 v = part[e];
    for (int j = 1; j < nsplit; ++j) {
      const double2 w = part[(int64_t)j * total + e];
      v.x += w.x;
      v.y += w.y;
    }
    part[e] = v;
  }
}

template <bool TN, int TT, bool XVEC>
hipError_t olaunch_tta(const OArgs& a, hipStream_t s) {
  const size_t lds = (size_t)2 * TT * 16 * OSTRIDE * sizeof(double);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)ogemm_kernel<TN, TT, XVEC>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    (void)hipGetLastError();
    attr = true;
  }
  hipLaunchKernelGGL((ogemm_kernel<TN, TT, XVEC>), dim3(8 * a.per), dim3(256), lds, s, a);
  return hipGetLastError();
}

template <bool TN, int TT>
hipError_t olaunch_tt(const OArgs& a, hipStream_t s) {
  if (!TN && a.xvec) return olaunch_tta<TN, TT, true>(a, s);
  return olaunch_tta<TN, TT, false>(a, s);
}

template <bool TN>
hipError_t olaunch(const OArgs& a, int TT, hipStream_t s) {
  switch (TT) {
    case 4: return olaunch_tt<TN, 4>(a, s);
    case 8: return olaunch_tt<TN, 8>(a, s);
    default: return olaunch_tt<TN, 16>(a, s);
  }
}

int othin_tiles(int N) {
  const int nn = N < 128 ? N : 128;
  if (nn <= 32) return 4;
  if (nn <= 64) return 8;
  return 16;
}

// TN thin tiles: an upper-triangle product wider than one 128-column chunk
// (the Gram of C, m = 440) takes 64-column chunks, so the chunks that straddle
// the diagonal waste less (28 of 49 tiles computed at m = 440, against 19 of
// 28 twice as wide): 3.55 -> 3.22 ms for that Gram at 4096 x 4096 x 64.
int tn_thin_tiles(int N, bool upper) { return (upper && N > 128) ? 8 : othin_tiles(N); }

void fill_grid(OArgs& a, int TT) {
  a.nthin = (a.N + 8 * TT - 1) / (8 * TT);
  a.nbig = (a.M + 63) / 64;
  const int64_t total = (int64_t)a.nbig * a.nthin * a.nsplit * a.batch;
  a.total = (int)total;
  a.per = (a.total + 7) / 8;
}

}  // namespace

namespace {

// Concurrent workgroup slots: two 256-thread workgroups per CU (the kernel's
// occupancy), times the device's CU count.
int ogemm_slots() {
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

// Workgroups of a TN launch that do work (the others skip tiles strictly
// below the diagonal of a square upper-only product).
int64_t tn_live_tiles(int M, int N, int batch, bool upper) {
  const int TT = tn_thin_tiles(N, upper && M == N), NCH = 8 * TT;
  const int nthin = (N + NCH - 1) / NCH, nbig = (M + 63) / 64;
  int64_t live = 0;
  for (int bt = 0; bt < nbig; ++bt)
    for (int tc = 0; tc < nthin; ++tc) live += (upper && M == N && bt * 64 > tc * NCH + NCH - 1) ? 0 : 1;
  return live * batch;
}

}  // namespace

// Split of the contraction for a TN product: the smallest makespan in K steps
// over the device's workgroup slots, rounds x (steps per split + a fixed
// per-workgroup cost), plus the reduction of the partials.
int ogemm_tn_split(int M, int K, int N, int batch, bool upper) {
  const int64_t live = tn_live_tiles(M, N, batch, upper);
  const int64_t slots = ogemm_slots();
  int best = 1;
  double bcost = 1e300;
  for (int ns = 1; ns <= 16; ++ns) {
    int kc = (K + ns - 1) / ns;
    kc = (kc + OKSTEP - 1) / OKSTEP * OKSTEP;
    if (ns > 1 && kc < 16 * OKSTEP) break;  // keep at least 16 steps per split
    const int nsx = (K + kc - 1) / kc;
    const int64_t rounds = (live * nsx + slots - 1) / slots;
    const double cost = (double)rounds * (kc / OKSTEP + 6) + (nsx > 1 ? 0.5 * nsx : 0.0);
    if (cost < bcost - 1e-9) {
      bcost = cost;
      best = nsx;
    }
  }
  return best;
}

namespace {

// Split of the paired upper-triangle kernel (one workgroup per slice and
// split): the same makespan model.
int ogemm_tn_pair_split(int K, int batch) {
  const int64_t slots = ogemm_slots();
  int best = 1;
  double bcost = 1e300;
  for (int ns = 1; ns <= 32; ++ns) {
    int kc = (K + ns - 1) / ns;
    kc = (kc + OKSTEP - 1) / OKSTEP * OKSTEP;
    if (ns > 1 && kc < 16 * OKSTEP) break;
    const int nsx = (K + kc - 1) / kc;
    const int64_t rounds = ((int64_t)batch * nsx + slots - 1) / slots;
    const double cost = (double)rounds * (kc / OKSTEP + 6) + (nsx > 1 ? 0.5 * nsx : 0.0);
    if (cost < bcost - 1e-9) {
      bcost = cost;
      best = nsx;
    }
  }
  return best;
}

}  // namespace

size_t ogemm_tn_part_bytes(int M, int K, int N, int batch) {
  int ns = std::max(ogemm_tn_split(M, K, N, batch, false), ogemm_tn_split(M, K, N, batch, true));
  if (M == N && N > 64 && N <= 120) ns = std::max(ns, ogemm_tn_pair_split(K, batch));
  return (size_t)ns * batch * M * N * 16;
}

hipError_t ogemm_tn(const float* X, int64_t lx, int64_t strideX, const float* Y, int64_t ly, int64_t strideY,
                    double* part, int M, int N, int K, int batch, hipStream_t s, bool upper) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  OArgs a{};
  a.X = X;
  a.lx = 2 * lx;
  a.strideX = 2 * strideX;
  a.B = Y;
  a.ldb = ly;
  a.strideB = strideY;
  a.nsum = 1;
  a.C = part;
  a.M = M;
  a.K = K;
  a.N = N;
  a.batch = batch;
  a.nsplit = ogemm_tn_split(M, K, N, batch, upper && M == N);
  int kc = (K + a.nsplit - 1) / a.nsplit;
  kc = (kc + OKSTEP - 1) / OKSTEP * OKSTEP;
  a.kchunk = kc < OKSTEP ? OKSTEP : kc;
  a.xvec = 0;
  a.upper = (upper && M == N) ? 1 : 0;
  const int TT = tn_thin_tiles(N, a.upper != 0);
  hipError_t e;
  if (a.upper && N > 64 && N <= 120) {
    a.nsplit = ogemm_tn_pair_split(K, batch);
    kc = (K + a.nsplit - 1) / a.nsplit;
    kc = (kc + OKSTEP - 1) / OKSTEP * OKSTEP;
    a.kchunk = kc < OKSTEP ? OKSTEP : kc;
    a.nsplit = (K + a.kchunk - 1) / a.kchunk;
    a.nbig = 1;
    a.nthin = 1;
    a.total = a.nsplit * batch;
    a.per = (a.total + 7) / 8;
    const size_t lds = (size_t)2 * 16 * 16 * OSTRIDE * sizeof(double);
    static bool attr = false;
    if (!attr) {
      (void)hipFuncSetAttribute((const void*)ogemm_tn_pair_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds);
      (void)hipGetLastError();
      attr = true;
    }
    hipLaunchKernelGGL(ogemm_tn_pair_kernel, dim3(8 * a.per), dim3(256), lds, s, a);
    e = hipGetLastError();
  } else {
    fill_grid(a, TT);
    e = olaunch<true>(a, TT, s);
  }
  if (e != hipSuccess || a.nsplit <= 1) return e;
  const int64_t total = (int64_t)batch * M * N;
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(opart_reduce_kernel, dim3(blocks), dim3(256), 0, s, (double2*)part, a.nsplit, total);
  return hipGetLastError();
}

hipError_t ogemm_nn(const float* X, int64_t lx, int64_t strideX, const double* B, int64_t ldb, int64_t strideB,
                    int nsum, int64_t bsum_stride, float* C, int64_t ldc, int64_t strideC, int M, int N, int K,
                    int batch, double alpha, double beta, hipStream_t s, bool b_triu) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  if (nsum != 1) return hipErrorInvalidValue;  // callers pass a single (summed) B
  OArgs a{};
  a.X = X;
  a.lx = 2 * lx;
  a.strideX = 2 * strideX;
  a.B = B;
  a.ldb = ldb;
  a.strideB = strideB;
  a.nsum = nsum < 1 ? 1 : nsum;
  a.bsum_stride = bsum_stride;
  a.C = C;
  a.ldc = ldc;
  a.strideC = strideC;
  a.alpha = alpha;
  a.beta = beta;
  a.M = M;
  a.K = K;
  a.N = N;
  a.batch = batch;
  a.nsplit = 1;
  a.kchunk = (K + OKSTEP - 1) / OKSTEP * OKSTEP;
  a.xvec = ((lx & 1) == 0 && (strideX & 1) == 0 && ((uintptr_t)X & 15) == 0) ? 1 : 0;
  a.triu = b_triu ? 1 : 0;
  const int TT = othin_tiles(N);
  fill_grid(a, TT);
  // Slices past the last full round of workgroup slots would run as a nearly
  // empty extra round: they go to a second launch with narrower thin chunks
  // (more, shorter workgroups).
  const int64_t slots = ogemm_slots();
  const int64_t per_slice = (int64_t)a.nbig * a.nthin;
  const int64_t full = (int64_t)a.total / slots * slots;
  const int fsplit = (int)(full / per_slice);
  if (TT > 4 && fsplit >= 1 && fsplit < batch && (a.total - full) * 2 < slots) {
    OArgs b = a;
    b.batch = fsplit;
    fill_grid(b, TT);
    hipError_t e = olaunch<false>(b, TT, s);
    if (e != hipSuccess) return e;
    OArgs r = a;
    r.X = X + 2 * strideX * fsplit;
    r.B = B + 2 * strideB * fsplit;  // complex doubles
    r.C = C + 2 * strideC * fsplit;
    r.batch = batch - fsplit;
    fill_grid(r, 4);
    return olaunch<false>(r, 4, s);
  }
  return olaunch<false>(a, TT, s);
}

}  // namespace tsvd
