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

    // Right-looking Cholesky, lower: G + shift I = L L^H.
    int bad = 0, rescued = 0;
    for (int j = 0; j < b; ++j) {
      if (shift > 0 && !(L[tri(j, j)].re > shift)) rescued = 1;  // the shift carries this pivot
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
    if (tid == 0 && rescued) atomicAdd(&info[INFO_CHOL_SHIFTED], 1);
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
}

hipError_t chol_inv_blocked(const double* Gpart, int nsum, int64_t part_stride, double* Rinv, int b, int batch,
                            double shift_coef, int* info, hipStream_t s, int mode);

hipError_t chol_inv_ex(const double* Gpart, int nsum, int64_t part_stride, double* Rinv, void* gscratch, int b,
                       int batch, double shift_coef, int* info, hipStream_t s, int mode) {
  if (batch <= 0 || b <= 0) return hipSuccess;
  if (b > 1024) return hipErrorInvalidValue;
  if (b <= 128) return chol_inv_blocked(Gpart, nsum, part_stride, Rinv, b, batch, shift_coef, info, s, mode);
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

// ---------------------------------------------------------------------------
// Blocked variant for b <= 128: the lower triangle is kept in LDS as 16 x 16
// tiles (tile (I, J), I >= J, rows padded to 17 entries against bank
// conflicts); rows and columns beyond b are padded with the identity.
// Factorisation, per tile column K: one wave factors the diagonal tile and
// replaces it by its inverse X_KK = L_KK^{-1}; the panel tiles become
// A_IK X_KK^H; the trailing tiles lose A_IK A_JK^H.  Inverse, per tile row I:
// S_IJ = sum_{K=J}^{I-1} L_IK X_KJ, then X_IJ = -X_II S_IJ.  About 6 nb
// barrier phases instead of 2 b, with tile products spread over 4 waves.
// ---------------------------------------------------------------------------
namespace tsvd {
namespace {

constexpr int TSZ = 16;
constexpr int TRS = 17;               // padded row stride of a tile (complex)
constexpr int TEL2 = TSZ * TRS;       // complex elements per stored tile

__device__ __forceinline__ int tix(int I, int J) { return (I * (I + 1) / 2 + J) * TEL2; }
__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}
__device__ __forceinline__ cx<double> cmad(cx<double> acc, cx<double> a, cx<double> b) {
  acc.re += a.re * b.re - a.im * b.im;
  acc.im += a.re * b.im + a.im * b.re;
  return acc;
}
// acc += a * conj(b)
__device__ __forceinline__ cx<double> cmadc(cx<double> acc, cx<double> a, cx<double> b) {
  acc.re += a.re * b.re + a.im * b.im;
  acc.im += a.im * b.re - a.re * b.im;
  return acc;
}

// Invert the lower triangular 16 x 16 tile T in place (one wave; lane c < 16
// forms column c of the inverse by forward substitution in registers).
__device__ void tile_inverse(cx<double>* T, int lane) {
  cx<double> x[TSZ];
  const int c = lane & 15;
#pragma unroll
  for (int i = 0; i < TSZ; ++i) {
    cx<double> s{i == c ? 1.0 : 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < i; ++k) {
      const cx<double> l = T[i * TRS + k];
      s.re -= l.re * x[k].re - l.im * x[k].im;
      s.im -= l.re * x[k].im + l.im * x[k].re;
    }
    const cx<double> d = T[i * TRS + i];
    const double rden = 1.0 / (d.re * d.re + d.im * d.im);
    const cx<double> inv{d.re * rden, -d.im * rden};
    x[i] = (i < c) ? cx<double>{0.0, 0.0} : cx<double>{s.re * inv.re - s.im * inv.im, s.re * inv.im + s.im * inv.re};
  }
  wsync();
  if (lane < TSZ) {
#pragma unroll
    for (int i = 0; i < TSZ; ++i) T[i * TRS + c] = x[i];
  }
  wsync();
}

// Value of x in lane l (l uniform), through the scalar unit.
__device__ __forceinline__ double lane_bcast(double x, int l) {
  const long long v = __double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Cholesky of the Hermitian 16 x 16 tile T (lower part used) in place (one
// wave).  Returns bit 0 on a non-positive or non-finite pivot in a row <
// nvalid, bit 1 when such a row's pivot is at most `thr` (thr > 0: twice the
// shift that was added to the diagonal, i.e. the shift carries the pivot).
// Lane i (mod 16) holds row i in registers for the whole factorisation; the
// pivot and the entries L_jk of column k reach the other rows by lane
// broadcast, so a column costs no LDS round trip or wave barrier.  Every
// entry sees the same operations in the same order as the column-by-column
// right-looking form: scale column k by 1 / sqrt(pivot), then
// A_ij -= L_ik conj(L_jk) for k < j <= i.
__device__ int tile_cholesky(cx<double>* T, int lane, int nvalid, double thr) {
  const int i = lane & 15;
  cx<double> r[TSZ];
#pragma unroll
  for (int j = 0; j < TSZ; ++j) r[j] = T[i * TRS + j];
  int bad = 0;
#pragma unroll
  for (int k = 0; k < TSZ; ++k) {
    const double d = lane_bcast(r[k].re, k);
    if (thr > 0 && k < nvalid && !(d > thr)) bad |= 2;
    double piv = 1.0;
    if (d > 0 && isfinite(d))
      piv = sqrt(d);
    else if (k < nvalid)
      bad |= 1;
    const double inv = 1.0 / piv;
    if (i > k) {
      r[k].re *= inv;
      r[k].im *= inv;
    } else if (i == k) {
      r[k] = cx<double>{piv, 0.0};
    }
#pragma unroll
    for (int j = k + 1; j < TSZ; ++j) {
      const double lr = lane_bcast(r[k].re, j), li = lane_bcast(r[k].im, j);
      if (j <= i) {
        r[j].re -= r[k].re * lr + r[k].im * li;
        r[j].im -= r[k].im * lr - r[k].re * li;
      }
    }
  }
  wsync();
  if (lane < TSZ) {
#pragma unroll
    for (int j = 0; j < TSZ; ++j) T[i * TRS + j] = r[j];
  }
  wsync();
  return bad;
}

// Waves of the blocked kernel: the panel, trailing and inverse tile work is
// spread over them (one tile per wave at a time); 8 waves keep two per SIMD.
constexpr int CB_W = 8, CB_NT = 64 * CB_W, CB_SLOTS = (8 + CB_W - 1) / CB_W;

template <int NT>
__global__ __launch_bounds__(CB_NT) void chol_blk_kernel(const cx<double>* __restrict__ Gpart, int nsum,
                                                       int64_t part_stride, cx<double>* __restrict__ Rinv, int b,
                                                       double shift_coef, int* info, int mode) {
  extern __shared__ __align__(16) unsigned char smem[];
  cx<double>* L = reinterpret_cast<cx<double>*>(smem);
  __shared__ double red[CB_W];
  const int f = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const cx<double>* G = Gpart + (int64_t)f * b * b;
  constexpr int BP = NT * TSZ;

  // ---- load: lower triangle (i >= j) of the padded matrix into tiles ----
  if (mode != 0) {
    // modes 1 and 2 need the upper triangle of the summed partials: read it
    // row by row (coalesced) and store its conjugate transpose, L(i, j) =
    // conj(G(j, i)) for i >= j (mode 2 keeps the diagonal real); padding rows
    // b .. BP - 1 take the identity
#pragma unroll 2
    for (int e = tid; e < b * b; e += CB_NT) {
      const int r = e / b, cc = e - r * b;
      if (cc >= r) {
        cx<double> g{0.0, 0.0};
        for (int s = 0; s < nsum; ++s) {
          const cx<double> x = G[s * part_stride + e];
          g.re += x.re;
          g.im += x.im;
        }
        L[tix(cc >> 4, r >> 4) + (cc & 15) * TRS + (r & 15)] = cx<double>{g.re, (mode == 2 && cc == r) ? 0.0 : -g.im};
      }
    }
    for (int e = tid; e < (BP - b) * BP; e += CB_NT) {
      const int i = b + e / BP, j = e % BP;
      if (j <= i) L[tix(i >> 4, j >> 4) + (i & 15) * TRS + (j & 15)] = cx<double>{i == j ? 1.0 : 0.0, 0.0};
    }
  }
  for (int e = tid; mode == 0 && e < BP * BP; e += CB_NT) {
    const int i = e / BP, j = e % BP;
    if (j > i) continue;
    cx<double> v{(i == j && i >= b) ? 1.0 : 0.0, 0.0};
    if (i < b && j < b) {
      v = cx<double>{0.0, 0.0};
      for (int s = 0; s < nsum; ++s) {
        const cx<double>* Gs = G + s * part_stride;
        const cx<double> g = Gs[(int64_t)i * b + j];
        const cx<double> h = Gs[(int64_t)j * b + i];
        v.re += 0.5 * (g.re + h.re);
        v.im += 0.5 * (g.im - h.im);
      }
    }
    L[tix(i >> 4, j >> 4) + (i & 15) * TRS + (j & 15)] = v;
  }
  __syncthreads();

  int bad = 0;
  if (mode == 1) {
    // invert the diagonal tiles (one wave each)
    for (int K = wave; K < NT; K += CB_W) tile_inverse(L + tix(K, K), lane);
    __syncthreads();
  } else {
    double tr = 0;
    for (int i = tid; i < b; i += CB_NT) tr += L[tix(i >> 4, i >> 4) + (i & 15) * (TRS + 1)].re;
    tr = block_sum<CB_NT>(tr, red);
    const double shift = shift_coef * tr;
    for (int i = tid; i < b; i += CB_NT) L[tix(i >> 4, i >> 4) + (i & 15) * (TRS + 1)].re += shift;
    __syncthreads();
    // Look-ahead: the diagonal tile of step K + 1 is factored (and inverted)
    // by wave 0 during step K's trailing update, right after wave 0 has
    // applied that update to it, while the other waves update the rest.
    if (wave == 0) {
      bad |= tile_cholesky(L, lane, b, 2.0 * shift);
      tile_inverse(L, lane);  // X_00 = L_00^{-1}
    }
    __syncthreads();
    for (int K = 0; K < NT; ++K) {
      const cx<double>* D = L + tix(K, K);  // X_KK
      // panel: A_IK <- A_IK X_KK^H (one tile per wave at a time).  The
      // triangular tiles hold exact zeros above the diagonal, so every inner
      // product below runs over all 16 terms: the extra terms add exact
      // zeros after (or before) the nonzero ones, and the fixed trip count
      // lets the loads of a whole row issue at once.
      // Lane (q, c) forms rows r = 4 u + q of column c: the column operand is
      // read once per k for its four rows.
      const int q = lane >> 4, c = lane & 15;
      for (int I = K + 1 + wave; I < NT; I += CB_W) {
        cx<double>* P = L + tix(I, K);
        cx<double> out[4] = {};
#pragma unroll 4
        for (int k = 0; k < TSZ; ++k) {
          const cx<double> d = D[c * TRS + k];
#pragma unroll
          for (int u = 0; u < 4; ++u) out[u] = cmadc(out[u], P[(4 * u + q) * TRS + k], d);
        }
        wsync();
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = lane + 64 * u;
          P[(e >> 4) * TRS + (e & 15)] = out[u];
        }
        wsync();
      }
      __syncthreads();
      // trailing: A_IJ -= A_IK A_JK^H, K < J <= I.  Pair 0 is the next
      // diagonal tile (K + 1, K + 1): wave 0 updates it alone and then
      // factors it; waves 1 .. CB_W - 1 take the other pairs.
      const int m = NT - K - 1;
      const int npairs = m * (m + 1) / 2;
      const int pfirst = wave == 0 ? 0 : wave;
      const int plast = wave == 0 ? min(npairs, 1) : npairs;
      const int pstep = wave == 0 ? 1 : CB_W - 1;
      for (int pidx = pfirst; pidx < plast; pidx += pstep) {
        int I = 0, rem = pidx;
        while (rem >= I + 1) {
          rem -= I + 1;
          ++I;
        }
        const int Ig = K + 1 + I, Jg = K + 1 + rem;
        const cx<double>* AI = L + tix(Ig, K);
        const cx<double>* AJ = L + tix(Jg, K);
        cx<double>* T = L + tix(Ig, Jg);
        cx<double> acc[4] = {};
#pragma unroll 4
        for (int k = 0; k < TSZ; ++k) {
          const cx<double> aj = AJ[c * TRS + k];
#pragma unroll
          for (int u = 0; u < 4; ++u) acc[u] = cmadc(acc[u], AI[(4 * u + q) * TRS + k], aj);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int r = 4 * u + q;
          if (Ig == Jg && c > r) continue;
          cx<double> v = T[r * TRS + c];
          v.re -= acc[u].re;
          v.im -= acc[u].im;
          T[r * TRS + c] = v;
        }
      }
      if (wave == 0 && npairs > 0) {
        cx<double>* Dn = L + tix(K + 1, K + 1);
        wsync();  // the lanes' updates of the tile are visible to the whole wave
        bad |= tile_cholesky(Dn, lane, b - (K + 1) * TSZ, 2.0 * shift);
        tile_inverse(Dn, lane);  // X_{K+1,K+1}
      }
      __syncthreads();
    }
    if (tid == 0 && (bad & 1)) atomicAdd(&info[INFO_CHOL_BREAKDOWN], 1);
    if (tid == 0 && (bad & 2)) atomicAdd(&info[INFO_CHOL_SHIFTED], 1);
  }
  // wave 0 carries `bad`; other waves never set it
  (void)bad;

  // ---- inverse: row by row, X_IJ = -X_II sum_{K=J}^{I-1} L_IK X_KJ ----
  // (lane (q, c) forms rows r = 4 u + q of column c, as in the factorisation)
  const int q = lane >> 4, c = lane & 15;
  for (int I = 1; I < NT; ++I) {
    // phase A: S_IJ into registers (tiles J < I spread over the waves)
    cx<double> sreg[CB_SLOTS][4];
#pragma unroll
    for (int slot = 0; slot < CB_SLOTS; ++slot) {
      const int J = wave + CB_W * slot;
      if (J >= I) continue;
#pragma unroll
      for (int u = 0; u < 4; ++u) sreg[slot][u] = cx<double>{0.0, 0.0};
      for (int K = J; K < I; ++K) {
        const cx<double>* LI = L + tix(I, K);
        const cx<double>* XK = L + tix(K, J);
        // X_JJ (K == J) is lower triangular, its zeros stored
#pragma unroll 4
        for (int k = 0; k < TSZ; ++k) {
          const cx<double> x = XK[k * TRS + c];
#pragma unroll
          for (int u = 0; u < 4; ++u) sreg[slot][u] = cmad(sreg[slot][u], LI[(4 * u + q) * TRS + k], x);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int slot = 0; slot < CB_SLOTS; ++slot) {
      const int J = wave + CB_W * slot;
      if (J >= I) continue;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = lane + 64 * u;
        L[tix(I, J) + (e >> 4) * TRS + (e & 15)] = sreg[slot][u];
      }
    }
    __syncthreads();
    // phase B: X_IJ = -X_II S_IJ (X_II lower triangular)
    const cx<double>* XI = L + tix(I, I);
#pragma unroll
    for (int slot = 0; slot < CB_SLOTS; ++slot) {
      const int J = wave + CB_W * slot;
      if (J >= I) continue;
      const cx<double>* S = L + tix(I, J);
      cx<double> acc[4] = {};
#pragma unroll 4
      for (int k = 0; k < TSZ; ++k) {
        const cx<double> sv = S[k * TRS + c];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] = cmad(acc[u], XI[(4 * u + q) * TRS + k], sv);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) sreg[slot][u] = cx<double>{-acc[u].re, -acc[u].im};
    }
    __syncthreads();
#pragma unroll
    for (int slot = 0; slot < CB_SLOTS; ++slot) {
      const int J = wave + CB_W * slot;
      if (J >= I) continue;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = lane + 64 * u;
        L[tix(I, J) + (e >> 4) * TRS + (e & 15)] = sreg[slot][u];
      }
    }
    __syncthreads();
  }

  // ---- R^{-1} = X^H (upper triangular), b x b row-major ----
  cx<double>* out = Rinv + (int64_t)f * b * b;
  for (int e = tid; e < b * b; e += CB_NT) {
    const int r = e / b, c = e % b;
    cx<double> v{0.0, 0.0};
    if (c >= r) {
      const cx<double> x = L[tix(c >> 4, r >> 4) + (c & 15) * TRS + (r & 15)];
      v = cx<double>{x.re, -x.im};
    }
    out[e] = v;
  }
}

}  // namespace

bool chol_blocked_ok(int b) { return b <= 128; }

hipError_t chol_inv_blocked(const double* Gpart, int nsum, int64_t part_stride, double* Rinv, int b, int batch,
                            double shift_coef, int* info, hipStream_t s, int mode) {
  if (batch <= 0 || b <= 0) return hipSuccess;
  if (b > 128) return hipErrorInvalidValue;
  const int nt = (b + TSZ - 1) / TSZ;
  const size_t lds = (size_t)nt * (nt + 1) / 2 * TEL2 * sizeof(cx<double>);
  static bool attr = false;
  if (!attr) {
    const void* fns[8] = {(const void*)chol_blk_kernel<1>, (const void*)chol_blk_kernel<2>,
                          (const void*)chol_blk_kernel<3>, (const void*)chol_blk_kernel<4>,
                          (const void*)chol_blk_kernel<5>, (const void*)chol_blk_kernel<6>,
                          (const void*)chol_blk_kernel<7>, (const void*)chol_blk_kernel<8>};
    for (const void* fn : fns) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 157 * 1024);
    (void)hipGetLastError();
    attr = true;
  }
  const cx<double>* G = (const cx<double>*)Gpart;
  cx<double>* R = (cx<double>*)Rinv;
  switch (nt) {
#define TSVD_CHOL_CASE(n)                                                                                        \
  case n:                                                                                                        \
    hipLaunchKernelGGL(chol_blk_kernel<n>, dim3(batch), dim3(CB_NT), lds, s, G, nsum, part_stride, R, b, shift_coef, \
                       info, mode);                                                                              \
    break;
    TSVD_CHOL_CASE(1)
    TSVD_CHOL_CASE(2)
    TSVD_CHOL_CASE(3)
    TSVD_CHOL_CASE(4)
    TSVD_CHOL_CASE(5)
    TSVD_CHOL_CASE(6)
    TSVD_CHOL_CASE(7)
    TSVD_CHOL_CASE(8)
#undef TSVD_CHOL_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace tsvd
