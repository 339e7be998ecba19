// Top-k eigenpairs of a per-slice m x m Hermitian positive semidefinite
// matrix in FP64: the small decomposition behind the per-slice SVD of
// C_f = Q_f^H A_f in Alg. 2.  With C_f C_f^H = W diag(lambda) W^H, the left
// singular vectors of C_f are W, sigma = sqrt(lambda), and the right singular
// vectors are C_f^H W diag(1/sigma).
//
// Four kernels, all batched over the Fourier slices:
//  1. tridiag   one workgroup per slice: symmetrised sum of the split-K
//               partials, then Householder reduction G = H T H^H,
//               H = H_0 ... H_{m-2}, H_j = I - tau_j v_j v_j^H (complex
//               reflectors with real beta, so T is real symmetric).  Each step
//               touches the trailing matrix once: the rank-2 update of step s
//               and the matrix-vector product of step s+1 share one pass.  The
//               trailing matrix moves into LDS as soon as it fits.
//  2. bisect    one wave per eigenvalue: 64-way multisection on Sturm counts
//               of T for the k largest eigenvalues.
//  3. invit     one wave per cluster of close eigenvalues: inverse iteration
//               on the pivoted LU of T - lambda I (in LDS), members of a
//               cluster re-orthogonalised against each other.
//  4. backxf    W = H Z, several workgroups per slice, each owning 8 columns
//               of W in LDS.
#include <algorithm>

#include "common.h"
#include "kernels.h"


namespace tsvd {

constexpr int TRI_PMAX = 8;  // workgroups per slice of the blocked tridiagonalisation, at most

static inline size_t heig_per_slice(int m, int k) {
  (void)k;
  const size_t mp = (size_t)(m + 31) / 32 * 32;
  // A (m x m), tau (m), d and e (m each), the partial products exchanged by the
  // workgroups of a slice (2 x TRI_PMAX x mp) and their barrier counters
  size_t b = (size_t)16 * m * m + (size_t)16 * m + (size_t)16 * m;
  b = (b + 255) & ~(size_t)255;
  b += (size_t)2 * TRI_PMAX * mp * 16 + 256;
  return (b + 255) & ~(size_t)255;
}
size_t heig_scratch_bytes(int m, int k) { return heig_per_slice(m, k); }

__device__ __forceinline__ cx<double> cmulc(cx<double> a, cx<double> b) {
  return cx<double>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
__device__ __forceinline__ cx<double> cjmul(cx<double> a, cx<double> b) {
  return cx<double>{a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}

struct HeigView {
  cx<double>* A;  // m x m working matrix (global)
  cx<double>* tau;
  double* d;
  double* e;
  cx<double>* ypg;  // 2 x TRI_PMAX x mp partial products of the slice's workgroups
  unsigned* sync;   // barrier counter and abort flag of the slice's workgroups
  double* fscale;   // partial sums of ||G||_F^2 (PREP_WG of them): the fixed-point scale of the symv sums
};
__device__ __forceinline__ HeigView heig_view(unsigned char* scratch, size_t per_slice, int f, int m) {
  HeigView v;
  unsigned char* base = scratch + (size_t)f * per_slice;
  v.A = reinterpret_cast<cx<double>*>(base);
  v.tau = v.A + (size_t)m * m;
  v.d = reinterpret_cast<double*>(v.tau + m);
  v.e = v.d + m;
  const size_t off = (((size_t)16 * m * m + (size_t)32 * m) + 255) & ~(size_t)255;
  v.ypg = reinterpret_cast<cx<double>*>(base + off);
  const size_t mp = (size_t)(m + 31) / 32 * 32;
  v.sync = reinterpret_cast<unsigned*>(base + off + (size_t)2 * TRI_PMAX * mp * 16);
  v.fscale = reinterpret_cast<double*>(v.sync + 2);
  return v;
}

// ---------------------------------------------------------------------------
// 1. Householder tridiagonalisation
// ---------------------------------------------------------------------------
// View of the working matrix: element (r, c) at p[(r - off) * ld + (c - off)].
// One instantiation per memory space keeps LDS accesses as LDS instructions.
struct MatView {
  cx<double>* p;
  int ld, off;
  __device__ __forceinline__ cx<double>* at(int r, int c) const { return p + (int64_t)(r - off) * ld + (c - off); }
};

struct TriShared {
  double* red;  // 2 * (NT / 64) doubles
  cx<double>* tau;
  cx<double>* scale;
  int* skip;
  cx<double>* ppart;  // TRI_G x m partial sums of p
};

#ifndef TSVD_TRI_NT
#define TSVD_TRI_NT 512
#endif
#ifndef TSVD_TRI_NB
#define TSVD_TRI_NB 8
#endif
constexpr int TRI_NT = TSVD_TRI_NT;  // threads per tridiagonalisation workgroup
constexpr int TRI_G = 8;     // at most this many thread groups share one column

// Block-wide sum of a complex value (one reduction for both parts).
__device__ __forceinline__ cx<double> block_sum_cx(cx<double> v, double* red) {
  v.re = wave_sum(v.re);
  v.im = wave_sum(v.im);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    red[2 * w] = v.re;
    red[2 * w + 1] = v.im;
  }
  __syncthreads();
  cx<double> r{0, 0};
#pragma unroll
  for (int i = 0; i < TRI_NT / 64; ++i) {
    r.re += red[2 * i];
    r.im += red[2 * i + 1];
  }
  return r;
}

// Reflector of step s from row s (the conjugate of column s below the
// diagonal), given s2 = the squared norm of its entries after the first:
// writes v (length m - s - 1, v[0] = 1) to `dst` and to row s of the global
// matrix, and records d[s], e[s], tau[s].
__device__ __forceinline__ void tri_reflector_from(const MatView& B, int s, int m, double s2, cx<double>* dst,
                                                   const HeigView& hv, const TriShared& sh) {
  const int tid = threadIdx.x;
  const int L = m - s - 1;
  const cx<double>* row = B.at(s, s + 1);
  if (tid == 0) {
    hv.d[s] = B.at(s, s)->re;
    const double ar = row[0].re, ai = -row[0].im;
    if (s2 == 0.0 && ai == 0.0) {
      *sh.skip = 1;
      hv.e[s] = ar;
      *sh.tau = cx<double>{0, 0};
    } else {
      *sh.skip = 0;
      const double beta = -copysign(sqrt(ar * ar + ai * ai + s2), ar);
      *sh.tau = cx<double>{(beta - ar) / beta, -ai / beta};
      const double dr = ar - beta, di = ai;
      const double den = dr * dr + di * di;
      *sh.scale = cx<double>{dr / den, -di / den};
      hv.e[s] = beta;
    }
    hv.tau[s] = *sh.tau;
  }
  __syncthreads();
  const bool skip = *sh.skip != 0;
  const cx<double> scale = *sh.scale;
  cx<double>* grow = hv.A + (int64_t)s * m + (s + 1);
  for (int i = tid; i < L; i += TRI_NT) {
    cx<double> v;
    if (i == 0) {
      v = cx<double>{1.0, 0.0};
    } else if (skip) {
      v = cx<double>{0.0, 0.0};
    } else {
      const cx<double> a = row[i];
      v = cmulc(cx<double>{a.re, -a.im}, scale);
    }
    dst[i] = v;
    grow[i] = v;
  }
  __syncthreads();
}

__device__ __forceinline__ void tri_reflector(const MatView& B, int s, int m, cx<double>* dst, const HeigView& hv,
                                              const TriShared& sh) {
  const int L = m - s - 1;
  const cx<double>* row = B.at(s, s + 1);
  double s2 = 0;
  for (int i = 1 + threadIdx.x; i < L; i += TRI_NT) {
    const cx<double> a = row[i];
    s2 += a.re * a.re + a.im * a.im;
  }
  s2 = block_sum_cx(cx<double>{s2, 0.0}, sh.red).re;
  tri_reflector_from(B, s, m, s2, dst, hv, sh);
}

// (a) w_s = p_s - (tau_s / 2) (p_s^H v_s) v_s, in place over p_s.
__device__ __forceinline__ void tri_w(int L, const cx<double>* vb, cx<double>* wb, const TriShared& sh) {
  const int tid = threadIdx.x;
  const cx<double> tau = *sh.tau;
  cx<double> acc{0, 0};
  for (int i = tid; i < L; i += TRI_NT) {
    const cx<double> t = cjmul(wb[i], vb[i]);
    acc.re += t.re;
    acc.im += t.im;
  }
  acc = block_sum_cx(acc, sh.red);
  const cx<double> a2 = cmulc(cx<double>{-0.5 * tau.re, -0.5 * tau.im}, acc);
  const bool zero = (tau.re == 0.0 && tau.im == 0.0);
  for (int i = tid; i < L; i += TRI_NT) {
    if (zero) {
      wb[i] = cx<double>{0, 0};
    } else {
      const cx<double> t = cmulc(a2, vb[i]);
      wb[i].re += t.re;
      wb[i].im += t.im;
    }
  }
  __syncthreads();
}

// Last step (trailing size 1): d[m-1].
__device__ __forceinline__ void tri_last(const MatView& B, int m, const cx<double>* vb, const cx<double>* wb,
                                         const HeigView& hv) {
  if (threadIdx.x == 0) {
    const cx<double> v = vb[0], w = wb[0];
    hv.d[m - 1] = B.at(m - 1, m - 1)->re - 2.0 * (v.re * w.re + v.im * w.im);
    hv.e[m - 1] = 0.0;
  }
}

// (c) row s+1 of the step-s update (and the norm for the next reflector),
// (d) the reflector of step s+1, (e) the rest of the step-s update of
// A[s+2:, s+2:] fused with p_{s+1} = tau_{s+1} A' v_{s+1}; the rows of each
// column are split over up to TRI_G thread groups.
__device__ __forceinline__ void tri_cde(const MatView& B, int s, int m, const cx<double>* vb, const cx<double>* wb,
                                        cx<double>* vn, cx<double>* pn, const HeigView& hv, const TriShared& sh) {
  const int tid = threadIdx.x;
  const int L = m - s - 1;
  double s2 = 0;
  {
    cx<double>* row = B.at(s + 1, s + 1);
    const cx<double> v0 = vb[0], w0 = wb[0];
    for (int c = tid; c < L; c += TRI_NT) {
      const cx<double> vc = vb[c], wc = wb[c];
      cx<double> a = row[c];
      a.re -= (v0.re * wc.re + v0.im * wc.im) + (w0.re * vc.re + w0.im * vc.im);
      a.im -= (v0.im * wc.re - v0.re * wc.im) + (w0.im * vc.re - w0.re * vc.im);
      row[c] = a;
      if (c >= 2) s2 += a.re * a.re + a.im * a.im;  // entries of row s+1 after its first off-diagonal
    }
  }
  s2 = block_sum_cx(cx<double>{s2, 0.0}, sh.red).re;
  tri_reflector_from(B, s + 1, m, s2, vn, hv, sh);
  const int Ln = L - 1;
  if (Ln <= 0) return;
  const cx<double> taun = *sh.tau;
  int G = TRI_NT / Ln;
  if (G > TRI_G) G = TRI_G;
  if (G < 1) G = 1;
  constexpr int NB = TSVD_TRI_NB;  // rows per batch; the next batch is loaded while this one is updated
  const int64_t ld = B.ld;
  for (int t = tid; t < G * Ln || (G == 1 && t < Ln); t += TRI_NT) {
    const int g = G > 1 ? t / Ln : 0;
    const int cc = G > 1 ? t - g * Ln : t;
    const int c = s + 2 + cc;
    const cx<double> vc = vb[cc + 1], wc = wb[cc + 1];
    double ar = 0, ai = 0;
    cx<double>* colp = B.at(s + 2, c);
    auto upd = [&](cx<double> x, int r) {
      const cx<double> vr = vb[r + 1], wr = wb[r + 1];
      x.re -= (vr.re * wc.re + vr.im * wc.im) + (wr.re * vc.re + wr.im * vc.im);
      x.im -= (vr.im * wc.re - vr.re * wc.im) + (wr.im * vc.re - wr.re * vc.im);
      colp[(int64_t)r * ld] = x;
      const cx<double> tt = cjmul(x, vn[r]);
      ar += tt.re;
      ai += tt.im;
    };
    // rows g, g + G, g + 2G, ... of this column
    const int nrows = (Ln - g + G - 1) / G;
    const int nfull = nrows / NB;
    int q = 0;
    if (nfull > 0) {
      cx<double> a[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) a[u] = colp[(int64_t)(g + u * G) * ld];
      for (int bt = 0; bt < nfull - 1; ++bt, q += NB) {
        cx<double> an[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) an[u] = colp[(int64_t)(g + (q + NB + u) * G) * ld];
#pragma unroll
        for (int u = 0; u < NB; ++u) upd(a[u], g + (q + u) * G);
#pragma unroll
        for (int u = 0; u < NB; ++u) a[u] = an[u];
      }
#pragma unroll
      for (int u = 0; u < NB; ++u) upd(a[u], g + (q + u) * G);
      q += NB;
    }
    for (; q < nrows; ++q) upd(colp[(int64_t)(g + q * G) * ld], g + q * G);
    if (G > 1)
      sh.ppart[g * m + cc] = cx<double>{ar, ai};
    else
      pn[cc] = cmulc(taun, cx<double>{ar, ai});
  }
  __syncthreads();
  if (G > 1) {
    for (int cc = tid; cc < Ln; cc += TRI_NT) {
      cx<double> acc{0, 0};
      for (int g = 0; g < G; ++g) {
        acc.re += sh.ppart[g * m + cc].re;
        acc.im += sh.ppart[g * m + cc].im;
      }
      pn[cc] = cmulc(taun, acc);
    }
    __syncthreads();
  }
}

// A = Hermitian part of the sum of the nsum partials (or the Hermitian
// extension of their upper triangle), written to the slice's working matrix.
template <int NT>
__device__ __forceinline__ void tri_load_hermitian(const cx<double>* __restrict__ G, int nsum, int64_t part_stride,
                                                   int m, int upper_only, cx<double>* A) {
  const int tid = threadIdx.x;
  // sum of the partials (partial index outermost: independent loads in flight)
  const int mm = m * m;
  for (int s = 0; s < nsum; ++s) {
    const cx<double>* Gs = G + s * part_stride;
#pragma unroll 8
    for (int t = tid; t < mm; t += NT) {
      const cx<double> g = Gs[t];
      if (s == 0) {
        A[t] = g;
      } else {
        cx<double> a = A[t];
        a.re += g.re;
        a.im += g.im;
        A[t] = a;
      }
    }
  }
  __syncthreads();
  // Hermitian average (upper triangle from the lower one, diagonal real), or
  // the Hermitian extension of the upper triangle when only that is valid
  for (int t = tid; t < mm; t += NT) {
    const int i = t / m, c = t - (t / m) * m;
    if (c > i) continue;
    const cx<double> g = A[t], h = A[(int64_t)c * m + i];
    const cx<double> lo = upper_only ? cx<double>{h.re, i == c ? 0.0 : -h.im}
                                     : cx<double>{0.5 * (g.re + h.re), i == c ? 0.0 : 0.5 * (g.im - h.im)};
    A[t] = lo;
    A[(int64_t)c * m + i] = cx<double>{lo.re, -lo.im};
  }
  __syncthreads();
}

__global__ __launch_bounds__(TRI_NT) void heig_tridiag_kernel(const cx<double>* __restrict__ Gpart, int nsum,
                                                           int64_t part_stride, int m, unsigned char* scratch,
                                                           size_t per_slice, int Lsw, int upper_only) {
  extern __shared__ __align__(16) unsigned char smem[];
  cx<double>* vbuf0 = reinterpret_cast<cx<double>*>(smem);
  cx<double>* vbuf1 = vbuf0 + m;
  cx<double>* wbuf0 = vbuf1 + m;
  cx<double>* wbuf1 = wbuf0 + m;
  cx<double>* ppart = wbuf1 + m;          // TRI_G x m partial sums
  cx<double>* Tl = ppart + TRI_G * m;     // LDS copy of the trailing matrix
  __shared__ double red[2 * (TRI_NT / 64)];
  __shared__ cx<double> s_tau, s_scale;
  __shared__ int s_skip;
  const TriShared sh{red, &s_tau, &s_scale, &s_skip, ppart};
  const int tid = threadIdx.x;
  const int f = blockIdx.x;
  const HeigView hv = heig_view(scratch, per_slice, f, m);
  cx<double>* A = hv.A;
  const cx<double>* G = Gpart + (int64_t)f * m * m;

  tri_load_hermitian<TRI_NT>(G, nsum, part_stride, m, upper_only, A);
  if (m == 1) {
    if (tid == 0) {
      hv.d[0] = A[0].re;
      hv.e[0] = 0.0;
      hv.tau[0] = cx<double>{0, 0};
    }
    return;
  }
  const MatView Bg{A, m, 0};
  int cur = 0;  // which of the two vector buffers holds v_s / p_s
  auto vb = [&](int which) { return which ? vbuf1 : vbuf0; };
  auto wb = [&](int which) { return which ? wbuf1 : wbuf0; };

  // step 0: reflector and p_0 = tau_0 A[1:, 1:] v_0 (global)
  tri_reflector(Bg, 0, m, vbuf0, hv, sh);
  {
    const int L = m - 1;
    const cx<double> tau = s_tau;
    for (int c = tid; c < L; c += TRI_NT) {
      double ar = 0, ai = 0;
#pragma unroll 4
      for (int r = 0; r < L; ++r) {
        const cx<double> t = cjmul(*Bg.at(r + 1, c + 1), vbuf0[r]);
        ar += t.re;
        ai += t.im;
      }
      wbuf0[c] = cmulc(tau, cx<double>{ar, ai});
    }
    __syncthreads();
  }
  // global phase
  int s = 0;
  bool done = false;
  for (; s < m - 1; ++s) {
    const int L = m - s - 1;
    tri_w(L, vb(cur), wb(cur), sh);
    if (s == m - 2) {
      tri_last(Bg, m, vb(cur), wb(cur), hv);
      done = true;
      break;
    }
    if (L <= Lsw) break;
    tri_cde(Bg, s, m, vb(cur), wb(cur), vb(cur ^ 1), wb(cur ^ 1), hv, sh);
    cur ^= 1;
  }
  if (done) return;
  // LDS phase: the trailing matrix A[s+1:, s+1:] (w_s already formed)
  const int L0 = m - s - 1;
  for (int r = tid / 32; r < L0; r += TRI_NT / 32)
    for (int c = tid % 32; c < L0; c += 32) Tl[r * L0 + c] = A[(int64_t)(s + 1 + r) * m + (s + 1 + c)];
  __syncthreads();
  const MatView Bl{Tl, L0, s + 1};
  tri_cde(Bl, s, m, vb(cur), wb(cur), vb(cur ^ 1), wb(cur ^ 1), hv, sh);
  cur ^= 1;
  for (++s; s < m - 1; ++s) {
    const int L = m - s - 1;
    tri_w(L, vb(cur), wb(cur), sh);
    if (s == m - 2) {
      tri_last(Bl, m, vb(cur), wb(cur), hv);
      break;
    }
    tri_cde(Bl, s, m, vb(cur), wb(cur), vb(cur ^ 1), wb(cur ^ 1), hv, sh);
    cur ^= 1;
  }
}

// ---------------------------------------------------------------------------
// 1b. Blocked tridiagonalisation for larger m (panels of NB reflectors).
// The same reflectors as the unblocked kernel, but within a panel the trailing
// matrix is only read: step i forms y = A_tr v_i from the matrix as it stood
// at the start of the panel and corrects it with the panel's earlier
// reflectors, y -= V (W^H v) + W (V^H v); the panel's 2 NB rank-one terms
// A -= V W^H + W V^H are applied once at its end.  Only the lower triangle is
// read or written: a 32 x 32 tile below the diagonal feeds both y_R += A v_C
// and y_C += A^H v_R.  Each wave takes whole tiles (the next one is loaded
// while the current one is used), each lane a 4 x 4 block (rows
// 4 (lane / 8) + q, columns lane % 8 + 8 p); row and column sums are
// finished with three lane exchanges each and added into y in LDS.  The
// panel's V and W stay in LDS.  The trailing matrix is read about once per
// step at half size, against a read and a write of the full matrix per step in
// the unblocked form.  The waves' additions into y land in an order that
// depends on timing, so they are made in 64-bit fixed point (integer addition
// is associative): a contribution x is added as rint(x 2^62 / S) with S a power
// of two >= m ||G||_F.  Every partial sum of a row of the trailing matrix times
// v is below S in modulus (|a_rc| <= ||G||_2 <= ||G||_F, |v_c| <= 1), and
// the rounding, below 2^-61 m ||G||_F per contribution, stays under the FP64
// error of the product; the results are bitwise reproducible.
// ---------------------------------------------------------------------------
constexpr int T2_NT = 512;
constexpr int T2_W = T2_NT / 64;

__device__ __forceinline__ cx<double> cadd(cx<double> a, cx<double> b) { return cx<double>{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cx<double> shfl_xor_cx(cx<double> v, int mask) {
  return cx<double>{__shfl_xor(v.re, mask, 64), __shfl_xor(v.im, mask, 64)};
}
// a += x * y
__device__ __forceinline__ void cfma(cx<double>& a, cx<double> x, cx<double> y) {
  a.re = fma(x.re, y.re, fma(-x.im, y.im, a.re));
  a.im = fma(x.re, y.im, fma(x.im, y.re, a.im));
}
// a += conj(x) * y
__device__ __forceinline__ void cfmac(cx<double>& a, cx<double> x, cx<double> y) {
  a.re = fma(x.re, y.re, fma(x.im, y.im, a.re));
  a.im = fma(x.re, y.im, fma(-x.im, y.re, a.im));
}

template <int NW = T2_W, bool LEAD_SYNC = true>
__device__ __forceinline__ cx<double> block_sum2(cx<double> v, double* red) {
  v.re = wave_sum(v.re);
  v.im = wave_sum(v.im);
  const int w = threadIdx.x >> 6;
  if (LEAD_SYNC) __syncthreads();  // (skipped when red has not been read since the last barrier)
  if ((threadIdx.x & 63) == 0) {
    red[2 * w] = v.re;
    red[2 * w + 1] = v.im;
  }
  __syncthreads();
  cx<double> r{0, 0};
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    r.re += red[2 * i];
    r.im += red[2 * i + 1];
  }
  return r;
}

// Sum of a 4-vector over the eight lanes that differ only in lane bits X0, X1,
// X2 (three exchanges, halving the vector each time): the result is the total
// of element 2 [lane & X0] + [lane & X1]; the two lanes differing in X2 hold
// the same total.
template <int X0, int X1, int X2>
__device__ __forceinline__ cx<double> reduce4(const cx<double> (&y)[4], int lane) {
  const bool h0 = lane & X0, h1 = lane & X1;
  const cx<double> k0 = h0 ? y[2] : y[0], k1 = h0 ? y[3] : y[1];
  const cx<double> s0 = h0 ? y[0] : y[2], s1 = h0 ? y[1] : y[3];
  const cx<double> t0 = cadd(k0, shfl_xor_cx(s0, X0)), t1 = cadd(k1, shfl_xor_cx(s1, X0));
  const cx<double> kk = h1 ? t1 : t0, ss = h1 ? t0 : t1;
  const cx<double> u = cadd(kk, shfl_xor_cx(ss, X1));
  return cadd(u, shfl_xor_cx(u, X2));
}

// tile t of the lower triangle of tiles with first tile row / column J0 (row-major order)
__device__ __forceinline__ void tri_tile(int t, int J0, int& I, int& J) {
  int a = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((a + 1) * (a + 2) / 2 <= t) ++a;
  while (a * (a + 1) / 2 > t) --a;
  J = t - a * (a + 1) / 2 + J0;
  I = a + J0;
}

// The lane's 4 x 4 block: rows r0 + q, columns c0 + 8 p (eight lanes of a row
// group read one contiguous 128-byte segment per access).  Rows are clamped
// into the matrix; columns past m - 1 (last tile column only) read the next
// row, or for the last row the vectors stored after the matrix, and are masked.
__device__ __forceinline__ void load_block(const cx<double>* A, int m, int r0, int c0, cx<double> (&a)[4][4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const cx<double>* rp = A + (int64_t)min(r0 + q, m - 1) * m + c0;
#pragma unroll
    for (int p = 0; p < 4; ++p) a[q][p] = rp[8 * p];
  }
}

// y_R += A_blk v_C and y_C += A_blk^H v_R for the lane's block; MASK handles
// the tiles on the diagonal, at the first trailing column or past row m - 1.
template <bool MASK>
__device__ __forceinline__ void symv_block(const cx<double> (&a)[4][4], const cx<double>* vcur, int r0, int c0,
                                           int m, int cmin, cx<double> (&yR)[4], cx<double> (&yC)[4]) {
  cx<double> vr[4], vc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    vr[q] = vcur[r0 + q];
    vc[q] = vcur[c0 + 8 * q];
    yR[q] = yC[q] = cx<double>{0, 0};
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      cx<double> x = a[q][p];
      if (MASK) {
        const int r = r0 + q, c = c0 + 8 * p;
        const bool ok = r < m && c >= cmin && r >= c;
        if (!ok) x = cx<double>{0, 0};
        if (r == c) x.im = 0.0;
        cfma(yR[q], x, vc[p]);
        if (r == c) x = cx<double>{0, 0};
        cfmac(yC[p], x, vr[q]);
      } else {
        cfma(yR[q], x, vc[p]);
        cfmac(yC[p], x, vr[q]);
      }
    }
  }
}

// A_blk -= V_R W_C^H + W_R V_C^H over the panel's k < pw terms
__device__ __forceinline__ void rank_block(cx<double> (&a)[4][4], const cx<double>* Vl, const cx<double>* Wl, int MP,
                                           int pw, int r0, int c0) {
  for (int k = 0; k < pw; ++k) {
    cx<double> vr[4], wr[4], vc[4], wc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      vr[q] = Vl[k * MP + r0 + q];
      wr[q] = Wl[k * MP + r0 + q];
      vc[q] = Vl[k * MP + c0 + 8 * q];
      wc[q] = Wl[k * MP + c0 + 8 * q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const cx<double> nv{-vr[q].re, -vr[q].im}, nw{-wr[q].re, -wr[q].im};
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        // a -= v_r conj(w_c) + w_r conj(v_c)  ==  a += conj(w_c) (-v_r) + conj(v_c) (-w_r)
        cfmac(a[q][p], wc[p], nv);
        cfmac(a[q][p], vc[p], nw);
      }
    }
  }
}

// The slice's matrix, lower triangle only: A = Hermitian part of the sum of
// the nsum partials (or the Hermitian extension of their upper triangle),
// rows p, p + P, ... of it (the workgroup's share).
__device__ __forceinline__ void tri_load_lower(const cx<double>* __restrict__ G, int nsum, int64_t part_stride,
                                               int m, int upper_only, cx<double>* A, int p, int P) {
  for (int i = p; i < m; i += P) {
    for (int c = threadIdx.x; c <= i; c += T2_NT) {
      cx<double> g{0, 0}, h{0, 0};
      for (int s = 0; s < nsum; ++s) {
        const cx<double>* Gs = G + s * part_stride;
        const cx<double> x = Gs[(int64_t)i * m + c], y = Gs[(int64_t)c * m + i];
        g.re += x.re;
        g.im += x.im;
        h.re += y.re;
        h.im += y.im;
      }
      const cx<double> lo = upper_only ? cx<double>{h.re, i == c ? 0.0 : -h.im}
                                       : cx<double>{0.5 * (g.re + h.re), i == c ? 0.0 : 0.5 * (g.im - h.im)};
      A[(int64_t)i * m + c] = lo;
    }
  }
}

// Barrier over the P workgroups of one slice (P > 1; they are co-resident by
// cooperative launch).  ctr[0] counts arrivals, ctr[1] is set once a wait
// runs past its bound: every later wait of the slice then returns at once,
// the kernel finishes with wrong values and the nonfinite counter says so.
__device__ __forceinline__ void group_sync(unsigned* ctr, unsigned& gen, int P, int* info) {
  // every wave waits until its own global stores have reached the L2 (s_waitcnt
  // vmcnt(0)); the one release below then writes the L2 back for the group
  if (P > 1) __builtin_amdgcn_s_waitcnt(0x0F70);
  __syncthreads();
  if (P > 1) {
    ++gen;
    if (threadIdx.x == 0) {
      __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned target = gen * (unsigned)P;
      unsigned spins = 0;
      while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (__hip_atomic_load(ctr + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
        __builtin_amdgcn_s_sleep(1);
        if (++spins == (1u << 22)) {  // about a second: only reachable if the group is not co-resident
          __hip_atomic_store(ctr + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          atomicAdd(&info[INFO_NONFINITE], 1);
          break;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // after the relaxed polls
    }
    __syncthreads();
  }
}

// Per slice, PREP_WG workgroups (blockIdx.y): the barrier counters cleared and
// the partial sums of ||G||_F^2 over the rows r = y mod PREP_WG of the summed
// partials (their upper triangle counted twice when only it is valid); the
// tridiagonalisation adds the PREP_WG partials in order and takes the power of
// two S >= m ||G||_F as the fixed-point scale of its symv sums.
constexpr int PREP_WG = 8;
__global__ __launch_bounds__(256) void heig_prep_kernel(const cx<double>* __restrict__ Gpart, int nsum,
                                                        int64_t part_stride, int m, int upper_only,
                                                        unsigned char* scratch, size_t per_slice) {
  __shared__ double red[4];
  const int f = blockIdx.x, y = blockIdx.y;
  const HeigView hv = heig_view(scratch, per_slice, f, m);
  const cx<double>* G = Gpart + (int64_t)f * m * m;
  double acc = 0.0;
  // four rows per pass keep several loads of each thread in flight
  for (int r0 = y; r0 < m; r0 += 4 * PREP_WG) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = r0 + u * PREP_WG;
      if (r >= m) continue;
      for (int c = (upper_only ? r : 0) + (int)threadIdx.x; c < m; c += 256) {
        const int64_t t = (int64_t)r * m + c;
        cx<double> g{0, 0};
        for (int s = 0; s < nsum; ++s) {
          const cx<double> x = G[s * part_stride + t];
          g.re += x.re;
          g.im += x.im;
        }
        acc += (upper_only && c != r ? 2.0 : 1.0) * (g.re * g.re + g.im * g.im);
      }
    }
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    hv.fscale[y] = red[0] + red[1] + red[2] + red[3];
    if (y == 0) {
      hv.sync[0] = 0;
      hv.sync[1] = 0;
    }
  }
}

// S = 2^e >= m ||G||_F from the prep kernel's partial sums (fixed order).
__device__ __forceinline__ double tri_fix_scale(const HeigView& hv, int m) {
  double fro2 = 0.0;
  for (int y = 0; y < PREP_WG; ++y) fro2 += hv.fscale[y];
  const double bound = (double)m * sqrt(fro2);
  if (!(bound > 0.0) || !isfinite(bound)) return 1.0;
  int e = 0;
  (void)frexp(bound, &e);  // bound < 2^e
  return ldexp(1.0, e);
}

// Lighter barrier for data exchanged only through device-coherent accesses
// (agent-scope atomic loads and stores, which bypass the XCD's L2): each wave
// waits for its own accesses to complete, then the arrival count is bumped
// and polled without any cache writeback or invalidation.
__device__ __forceinline__ void group_sync_coherent(unsigned* ctr, unsigned& gen, int P, int* info) {
  if (P <= 1) {
    __syncthreads();
    return;
  }
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's coherent stores are complete
  __syncthreads();
  ++gen;
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned target = gen * (unsigned)P;
    unsigned spins = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(ctr + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
      __builtin_amdgcn_s_sleep(1);
      if (++spins == (1u << 22)) {
        __hip_atomic_store(ctr + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        atomicAdd(&info[INFO_NONFINITE], 1);
        break;
      }
    }
  }
  __syncthreads();
}

template <int NB>
__global__ __launch_bounds__(T2_NT) void heig_tri2_kernel(const cx<double>* __restrict__ Gpart, int nsum,
                                                          int64_t part_stride, int m, int MP, unsigned char* scratch,
                                                          size_t per_slice, int upper_only, int P,
                                                          int* __restrict__ info) {
  extern __shared__ __align__(16) unsigned char smem[];
  cx<double>* vcur = reinterpret_cast<cx<double>*>(smem);  // MP: v of the current step (0 outside its range)
  cx<double>* y = vcur + MP;                                // MP: A_tr v
  cx<double>* col = y + MP;                                 // MP: the updated column of the step
  cx<double>* Vl = col + MP;                                // NB x MP: the panel's reflectors
  cx<double>* Wl = Vl + NB * MP;                            // NB x MP: their update vectors
  cx<double>* xs = Wl + NB * MP;                            // 2 NB: W^H v and V^H v
  __shared__ double red[2 * T2_W];
  __shared__ cx<double> s_tau, s_scale;
  __shared__ int s_skip;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int f = blockIdx.x / P, pg = blockIdx.x - f * P;  // slice, workgroup within the slice
  const bool lead = pg == 0;                             // writes the slice's outputs
  const HeigView hv = heig_view(scratch, per_slice, f, m);
  cx<double>* A = hv.A;
  unsigned* ctr = hv.sync;
  unsigned gen = 0;
  // fixed-point scale factors of the symv sums (powers of two: exact)
  const double fsc = tri_fix_scale(hv, m);
  const double to_fix = ldexp(1.0, 62) / fsc, from_fix = fsc * ldexp(1.0, -62);
  unsigned long long* yq = reinterpret_cast<unsigned long long*>(y);
  tri_load_lower(Gpart + (int64_t)f * m * m, nsum, part_stride, m, upper_only, A, pg, P);
  for (int r = tid; r < (2 * NB + 3) * MP; r += T2_NT) vcur[r] = cx<double>{0, 0};
  const int la = lane >> 3, lb = lane & 7;
  const int T = MP / 32;
  const int w0 = pg * T2_W + wv, wstep = P * T2_W;  // this wave's first tile and tile stride
  group_sync(ctr, gen, P, info);

  // The trailing matrix is only read within a panel, so a step's column and
  // its first symv tiles are requested early: the column one step ahead, the
  // tiles before the column update.  Row indices are clamped into the matrix.
  cx<double> colnext[2];
  for (int j0 = 0; j0 < m - 1; j0 += NB) {
    const int pw = min(NB, m - 1 - j0);
    for (int ii = 0; ii < pw; ++ii) {
      const int i = j0 + ii;
      cx<double> colv[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        if (ii == 0) colv[u] = A[(int64_t)min(i + tid + u * T2_NT, m - 1) * m + i];
        else colv[u] = colnext[u];
      }
      if (ii + 1 < pw) {
#pragma unroll
        for (int u = 0; u < 2; ++u) colnext[u] = A[(int64_t)min(i + 1 + tid + u * T2_NT, m - 1) * m + i + 1];
      }
      const int sJ0 = (i + 1) >> 5, snT = T - sJ0;
      const int sntile = snT * (snT + 1) / 2;
      auto stile_rc = [&](int t, int& r0, int& c0) {
        int I, J;
        tri_tile(min(t, sntile - 1), sJ0, I, J);
        r0 = 32 * I + 4 * la;
        c0 = 32 * J + lb;
      };
      cx<double> a0[4][4], a1[4][4];
      {
        int r0, c0;
        stile_rc(w0, r0, c0);
        load_block(A, m, r0, c0, a0);
      }
      // (1) column i (rows i..m-1) brought up to date with the panel's earlier terms
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int r = i + tid + u * T2_NT;
        if (r >= m) continue;
        cx<double> a = colv[u];
        for (int k = 0; k < ii; ++k) {
          const cx<double> vr = Vl[k * MP + r], wr = Wl[k * MP + r];
          const cx<double> vi = Vl[k * MP + i], wi = Wl[k * MP + i];
          // a -= v_r conj(w_i) + w_r conj(v_i)
          a.re -= (vr.re * wi.re + vr.im * wi.im) + (wr.re * vi.re + wr.im * vi.im);
          a.im -= (vr.im * wi.re - vr.re * wi.im) + (wr.im * vi.re - wr.re * vi.im);
        }
        col[r] = a;
      }
      __syncthreads();
      // (2) reflector from alpha = col[i+1], x = col[i+2..m-1]
      double s2 = 0;
      for (int r = i + 2 + tid; r < m; r += T2_NT) s2 += col[r].re * col[r].re + col[r].im * col[r].im;
      s2 = block_sum2(cx<double>{s2, 0.0}, red).re;
      if (tid == 0) {
        const double ar = col[i + 1].re, ai = col[i + 1].im;
        double ei;
        if (s2 == 0.0 && ai == 0.0) {
          s_skip = 1;
          ei = ar;
          s_tau = cx<double>{0, 0};
        } else {
          s_skip = 0;
          const double beta = -copysign(sqrt(ar * ar + ai * ai + s2), ar);
          s_tau = cx<double>{(beta - ar) / beta, -ai / beta};
          const double dr = ar - beta, di = ai;
          const double den = dr * dr + di * di;
          s_scale = cx<double>{dr / den, -di / den};
          ei = beta;
        }
        if (lead) {
          hv.d[i] = col[i].re;
          hv.e[i] = ei;
          hv.tau[i] = s_tau;
        }
      }
      __syncthreads();
      const bool skip = s_skip != 0;
      const cx<double> tau = s_tau, scale = s_scale;
      // v (v[i+1] = 1) into LDS, into the panel and into row i of A; y = 0
      for (int r = i + 1 + tid; r < m; r += T2_NT) {
        cx<double> v;
        if (r == i + 1)
          v = cx<double>{1.0, 0.0};
        else if (skip)
          v = cx<double>{0.0, 0.0};
        else
          v = cmulc(col[r], scale);
        vcur[r] = v;
        Vl[ii * MP + r] = v;
        if (lead) A[(int64_t)i * m + r] = v;
        y[r] = cx<double>{0, 0};
      }
      if (tid == 0) vcur[i] = cx<double>{0, 0};
      __syncthreads();
      // (3a) x1 = W^H v, x2 = V^H v over rows i+1..m-1 (one wave per product)
      for (int dd = wv; dd < 2 * ii; dd += T2_W) {
        const cx<double>* X = (dd < ii ? Wl + dd * MP : Vl + (dd - ii) * MP);
        cx<double> acc{0, 0};
        for (int r = i + 1 + lane; r < m; r += 64) cfmac(acc, X[r], vcur[r]);
        acc.re = wave_sum(acc.re);
        acc.im = wave_sum(acc.im);
        if (lane == 0) xs[dd] = acc;
      }
      // (3b) y = A_tr v over the lower triangle of rows / columns >= i+1
      {
        const int J0 = sJ0, ntile = sntile;
        auto process = [&](const cx<double>(&a)[4][4], int t) {
          int I, J;
          tri_tile(t, J0, I, J);
          const int r0 = 32 * I + 4 * la, c0 = 32 * J + lb;
          cx<double> yR[4], yC[4];
          if (I > J && 32 * J >= i + 1 && 32 * I + 32 <= m)
            symv_block<false>(a, vcur, r0, c0, m, i + 1, yR, yC);
          else
            symv_block<true>(a, vcur, r0, c0, m, i + 1, yR, yC);
          const cx<double> sr = reduce4<4, 2, 1>(yR, lane);
          const cx<double> sc = reduce4<32, 16, 8>(yC, lane);
          auto fix = [&](double x) { return (unsigned long long)(long long)rint(x * to_fix); };
          if (!(lane & 1)) {
            const int q = ((lane >> 2) & 1) * 2 + ((lane >> 1) & 1);
            atomicAdd(&yq[2 * (r0 + q)], fix(sr.re));
            atomicAdd(&yq[2 * (r0 + q) + 1], fix(sr.im));
          }
          if (!(la & 1)) {
            const int p = ((la >> 2) & 1) * 2 + ((la >> 1) & 1);
            atomicAdd(&yq[2 * (c0 + 8 * p)], fix(sc.re));
            atomicAdd(&yq[2 * (c0 + 8 * p) + 1], fix(sc.im));
          }
        };
        // two tile buffers (the first requested at the start of the step);
        // the next tile is in flight while one is used
        int r0, c0;
        for (int t = w0; t < ntile; t += 2 * wstep) {
          stile_rc(t + wstep, r0, c0);
          load_block(A, m, r0, c0, a1);
          process(a0, t);
          if (t + wstep >= ntile) break;
          stile_rc(t + 2 * wstep, r0, c0);
          load_block(A, m, r0, c0, a0);
          process(a1, t + wstep);
        }
      }
      __syncthreads();
      // the fixed-point sums back to FP64 (each thread converts its own rows)
      for (int r = i + 1 + tid; r < m; r += T2_NT) {
        const long long qr = (long long)yq[2 * r], qi = (long long)yq[2 * r + 1];
        y[r] = cx<double>{(double)qr * from_fix, (double)qi * from_fix};
      }
      __syncthreads();
      if (P > 1) {
        // partial products of the slice's workgroups, summed in workgroup order
        // (double buffered by step parity: a workgroup is at most one exchange ahead)
        double* yb = reinterpret_cast<double*>(hv.ypg + (int64_t)((i & 1) * P) * MP);
        for (int r = i + 1 + tid; r < m; r += T2_NT) {
          double* d = yb + 2 * ((int64_t)pg * MP + r);
          __hip_atomic_store(d, y[r].re, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(d + 1, y[r].im, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        group_sync_coherent(ctr, gen, P, info);
        for (int r = i + 1 + tid; r < m; r += T2_NT) {
          cx<double> acc{0, 0};
          for (int q = 0; q < P; ++q) {
            const double* d = yb + 2 * ((int64_t)q * MP + r);
            acc.re += __hip_atomic_load(d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            acc.im += __hip_atomic_load(d + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
          y[r] = acc;
        }
        __syncthreads();
      }
      // (4) y -= V x1 + W x2; w = tau y; w += alpha v with alpha = -tau (w^H v) / 2
      //     (rows i+1..m-1, at most two per thread)
      cx<double> wl[2];
      cx<double> dot{0, 0};
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int r = i + 1 + tid + u * T2_NT;
        wl[u] = cx<double>{0, 0};
        if (r < m) {
          cx<double> yy = y[r];
          for (int k = 0; k < ii; ++k) {
            const cx<double> nx1{-xs[k].re, -xs[k].im}, nx2{-xs[ii + k].re, -xs[ii + k].im};
            cfma(yy, Vl[k * MP + r], nx1);
            cfma(yy, Wl[k * MP + r], nx2);
          }
          wl[u] = cmulc(tau, yy);
          cfmac(dot, wl[u], vcur[r]);
        }
      }
      dot = block_sum2(dot, red);
      const cx<double> alpha = cmulc(cx<double>{-0.5 * tau.re, -0.5 * tau.im}, dot);
      const bool zero = tau.re == 0.0 && tau.im == 0.0;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int r = i + 1 + tid + u * T2_NT;
        if (r < m) {
          cx<double> w = wl[u];
          cfma(w, alpha, vcur[r]);
          Wl[ii * MP + r] = zero ? cx<double>{0, 0} : w;
        }
      }
      __syncthreads();
    }
    // (5) A -= V W^H + W V^H on the lower triangle of rows / columns >= j0 + pw
    const int rs = j0 + pw;
    if (rs < m) {
      const int J0 = rs >> 5, nT = T - J0;
      const int ntile = nT * (nT + 1) / 2;
      auto tile_rc = [&](int t, int& r0, int& c0) {
        int I, J;
        tri_tile(min(t, ntile - 1), J0, I, J);
        r0 = 32 * I + 4 * la;
        c0 = 32 * J + lb;
      };
      auto process = [&](cx<double>(&a)[4][4], int t) {
        int I, J;
        tri_tile(t, J0, I, J);
        const int r0 = 32 * I + 4 * la, c0 = 32 * J + lb;
        rank_block(a, Vl, Wl, MP, pw, r0, c0);
        if (I > J && 32 * J >= rs && 32 * I + 32 <= m) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            cx<double>* rp = A + (int64_t)(r0 + q) * m + c0;
#pragma unroll
            for (int p = 0; p < 4; ++p) rp[8 * p] = a[q][p];
          }
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
#pragma unroll
            for (int p = 0; p < 4; ++p) {
              const int r = r0 + q, c = c0 + 8 * p;
              if (r < m && c >= rs && r >= c) A[(int64_t)r * m + c] = a[q][p];
            }
          }
        }
      };
      cx<double> a0[4][4], a1[4][4];
      int r0, c0;
      tile_rc(w0, r0, c0);
      load_block(A, m, r0, c0, a0);
      for (int t = w0; t < ntile; t += 2 * wstep) {
        tile_rc(t + wstep, r0, c0);
        load_block(A, m, r0, c0, a1);
        process(a0, t);
        if (t + wstep >= ntile) break;
        tile_rc(t + 2 * wstep, r0, c0);
        load_block(A, m, r0, c0, a0);
        process(a1, t + wstep);
      }
    }
    group_sync(ctr, gen, P, info);
  }
  if (tid == 0 && lead) {
    hv.d[m - 1] = A[(int64_t)(m - 1) * m + (m - 1)].re;
    hv.e[m - 1] = 0.0;
  }
}

// Register-resident form for several co-resident workgroups per slice.  The
// 32 x 32 tiles of the lower triangle are dealt out once: tile t (row-major
// over the triangle) belongs to workgroup t mod P, and within it to wave
// (t / P) mod RES_W, slot (t / P) / RES_W (at most RES_SLOTS per wave).  A wave keeps
// its tiles in registers for the whole reduction, in the 4 x 4 lane blocks of
// symv_block, so the trailing matrix is never read from or written to memory:
// every step applies the rank-2 update of the previous reflector in place.
// Per step i, one exchange between the workgroups of the slice:
//   - every workgroup adds its share of y = A_tr v (fixed point, as above) into
//     one slice-wide sum with agent-scope integer atomics, which are exact and
//     order-free, so y is the same in every workgroup and bit for bit the same
//     from run to run;
//   - the owners of column i + 1 publish it as it stands before this step's
//     update; after the exchange every workgroup applies the update to that one
//     column itself, so the next reflector needs no second exchange.
// The reflectors, w and the column update are repeated identically in every
// workgroup (same operands, same operations).  Sums and columns rotate through
// three buffers, so a buffer is cleared or rewritten only after every
// workgroup has passed the exchange that last read it.
// Four waves per workgroup, one per SIMD, so that each may hold up to 512
// registers (the tiles that do not fit the 256 vector registers sit in the
// accumulation registers); four tile slots per wave.
constexpr int RES_NT = 256;
constexpr int RES_W = RES_NT / 64;
constexpr int RES_SLOTS = 4;

// symv_block for the resident tiles with fewer live registers: the column
// operand is read once, the row operand one row of the lane block at a time.
template <bool MASK>
__device__ __forceinline__ void symv_res(const cx<double> (&a)[4][4], const cx<double>* vcur, int r0, int c0, int m,
                                         int cmin, cx<double> (&yR)[4], cx<double> (&yC)[4]) {
  cx<double> vc[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    vc[p] = vcur[c0 + 8 * p];
    yC[p] = cx<double>{0, 0};
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const cx<double> vr = vcur[r0 + q];
    yR[q] = cx<double>{0, 0};
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      cx<double> x = a[q][p];
      if (MASK) {
        const int r = r0 + q, c = c0 + 8 * p;
        const bool ok = r < m && c >= cmin && r >= c;
        if (!ok) x = cx<double>{0, 0};
        if (r == c) x.im = 0.0;
        cfma(yR[q], x, vc[p]);
        if (r == c) x = cx<double>{0, 0};
        cfmac(yC[p], x, vr);
      } else {
        cfma(yR[q], x, vc[p]);
        cfmac(yC[p], x, vr);
      }
    }
  }
}

__global__ __launch_bounds__(RES_NT, 1) void heig_trires_kernel(const cx<double>* __restrict__ Gpart, int nsum,
                                                            int64_t part_stride, int m, int MP,
                                                            unsigned char* scratch, size_t per_slice, int upper_only,
                                                            int P, int* __restrict__ info) {
  __shared__ cx<double> col[1024];    // column i (rows >= i), replicated
  __shared__ cx<double> vcur[1024];   // v of the step (0 outside rows i + 1 .. m - 1)
  __shared__ cx<double> wv_[1024];    // w of the step (0 outside)
  __shared__ unsigned long long yq[2 * 1024];  // this workgroup's share of y, fixed point
  __shared__ double red[2 * RES_W];
  __shared__ double red2[2][RES_W];  // per-wave partials of the next step's ||x||^2, by step parity
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int f = blockIdx.x / P, pg = blockIdx.x - f * P;
  const bool lead = pg == 0;
  const HeigView hv = heig_view(scratch, per_slice, f, m);
  cx<double>* Vout = hv.A;  // row i receives v_i (read by the back-transformation)
  unsigned* ctr = hv.sync;
  unsigned gen = 0;
  const double fsc = tri_fix_scale(hv, m);
  const double to_fix = ldexp(1.0, 62) / fsc, from_fix = fsc * ldexp(1.0, -62);
  // exchange buffers: three fixed-point sums (2 u64 per row) and three columns
  unsigned long long* ysum = reinterpret_cast<unsigned long long*>(hv.ypg);
  cx<double>* colx = hv.ypg + 3 * MP;
  const int T = MP / 32, NT = T * (T + 1) / 2;
  const int la = lane >> 3, lb = lane & 7;
  const cx<double>* G = Gpart + (int64_t)f * m * m;
  auto gram = [&](int r, int c) {  // A(r, c), r >= c, from the partials
    cx<double> g{0, 0}, h{0, 0};
    for (int s = 0; s < nsum; ++s) {
      const cx<double>* Gs = G + s * part_stride;
      const cx<double> x = Gs[(int64_t)r * m + c], y = Gs[(int64_t)c * m + r];
      g.re += x.re;
      g.im += x.im;
      h.re += y.re;
      h.im += y.im;
    }
    return upper_only ? cx<double>{h.re, r == c ? 0.0 : -h.im}
                      : cx<double>{0.5 * (g.re + h.re), r == c ? 0.0 : 0.5 * (g.im - h.im)};
  };
  // this wave's tiles
  int tI[RES_SLOTS], tJ[RES_SLOTS];
  bool tok[RES_SLOTS];
  cx<double> a[RES_SLOTS][4][4];
#pragma unroll
  for (int sl = 0; sl < RES_SLOTS; ++sl) {
    const int t = (sl * RES_W + wv) * P + pg;
    tok[sl] = t < NT;
    tri_tile(tok[sl] ? t : 0, 0, tI[sl], tJ[sl]);
    const int r0 = 32 * tI[sl] + 4 * la, c0 = 32 * tJ[sl] + lb;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const int r = r0 + q, c = c0 + 8 * p;
        a[sl][q][p] = (tok[sl] && r < m && c <= r) ? gram(r, c) : cx<double>{0, 0};
      }
  }
  for (int r = tid; r < MP; r += RES_NT) {
    col[r] = r < m ? gram(r, 0) : cx<double>{0, 0};
    vcur[r] = wv_[r] = cx<double>{0, 0};
    yq[2 * r] = yq[2 * r + 1] = 0ull;
    if (lead) {
      __hip_atomic_store(&ysum[2 * r], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&ysum[2 * r + 1], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  group_sync_coherent(ctr, gen, P, info);

  for (int i = 0; i < m - 1; ++i) {
    const int buf = i % 3;
    unsigned long long* ys = ysum + (int64_t)buf * 2 * MP;
    cx<double>* cxb = colx + (int64_t)buf * MP;
    // (1) reflector from alpha = col[i + 1], x = col[i + 2 .. m - 1] (every workgroup)
    double s2 = 0;
    if (i == 0) {
      for (int r = i + 2 + tid; r < m; r += RES_NT) s2 += col[r].re * col[r].re + col[r].im * col[r].im;
      s2 = block_sum2<RES_W>(cx<double>{s2, 0.0}, red).re;
    } else {
      // formed with the column update of the previous step
#pragma unroll
      for (int w = 0; w < RES_W; ++w) s2 += red2[i & 1][w];
    }
    // every thread forms the same reflector from the same operands
    const double ar = col[i + 1].re, ai = col[i + 1].im;
    const bool skip = s2 == 0.0 && ai == 0.0;
    cx<double> tau{0, 0}, scale{0, 0};
    double ei = ar;
    if (!skip) {
      const double beta = -copysign(sqrt(ar * ar + ai * ai + s2), ar);
      tau = cx<double>{(beta - ar) / beta, -ai / beta};
      const double dr = ar - beta, di = ai;
      const double den = dr * dr + di * di;
      scale = cx<double>{dr / den, -di / den};
      ei = beta;
    }
    if (lead && tid == 0) {
      hv.d[i] = col[i].re;
      hv.e[i] = ei;
      hv.tau[i] = tau;
    }
    for (int r = tid; r < MP; r += RES_NT) {
      cx<double> v{0, 0};
      if (r == i + 1)
        v = cx<double>{1.0, 0.0};
      else if (r > i + 1 && r < m && !skip)
        v = cmulc(col[r], scale);
      vcur[r] = v;
      wv_[r] = cx<double>{0, 0};
      if (lead && r > i && r < m) Vout[(int64_t)i * m + r] = v;
      yq[2 * r] = yq[2 * r + 1] = 0ull;
    }
    __syncthreads();
    // (2) this workgroup's share of y = A_tr v over its resident tiles
    const int J0 = (i + 1) >> 5;
#pragma unroll
    for (int sl = 0; sl < RES_SLOTS; ++sl) {
      if (tok[sl] && tJ[sl] >= J0) {
        const int r0 = 32 * tI[sl] + 4 * la, c0 = 32 * tJ[sl] + lb;
        cx<double> yR[4], yC[4];
        if (tI[sl] > tJ[sl] && 32 * tJ[sl] >= i + 1 && 32 * tI[sl] + 32 <= m)
          symv_res<false>(a[sl], vcur, r0, c0, m, i + 1, yR, yC);
        else
          symv_res<true>(a[sl], vcur, r0, c0, m, i + 1, yR, yC);
        const cx<double> sr = reduce4<4, 2, 1>(yR, lane);
        const cx<double> sc = reduce4<32, 16, 8>(yC, lane);
        auto fix = [&](double x) { return (unsigned long long)(long long)rint(x * to_fix); };
        if (!(lane & 1)) {
          const int q = ((lane >> 2) & 1) * 2 + ((lane >> 1) & 1);
          atomicAdd(&yq[2 * (r0 + q)], fix(sr.re));
          atomicAdd(&yq[2 * (r0 + q) + 1], fix(sr.im));
        }
        if (!(la & 1)) {
          const int p = ((la >> 2) & 1) * 2 + ((la >> 1) & 1);
          atomicAdd(&yq[2 * (c0 + 8 * p)], fix(sc.re));
          atomicAdd(&yq[2 * (c0 + 8 * p) + 1], fix(sc.im));
        }
      }
    }
    // column i + 1 as it stands before this step's update, from its owners
    const int Jn = (i + 1) >> 5;
#pragma unroll
    for (int sl = 0; sl < RES_SLOTS; ++sl) {
      if (tok[sl] && tJ[sl] == Jn) {
        const int r0 = 32 * tI[sl] + 4 * la, c0 = 32 * tJ[sl] + lb;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          if (c0 + 8 * p != i + 1) continue;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = r0 + q;
            if (r >= i + 1 && r < m) {
              double* d = reinterpret_cast<double*>(cxb + r);
              __hip_atomic_store(d, a[sl][q][p].re, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              __hip_atomic_store(d + 1, a[sl][q][p].im, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
          }
        }
      }
    }
    __syncthreads();
    // (3) add the share into the slice-wide sum; clear the sum of step i + 1
    unsigned long long* ysn = ysum + (int64_t)((i + 1) % 3) * 2 * MP;
    for (int r = i + 1 + tid; r < m; r += RES_NT) {
      const unsigned long long qr = yq[2 * r], qi = yq[2 * r + 1];
      if (qr) __hip_atomic_fetch_add(&ys[2 * r], qr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (qi) __hip_atomic_fetch_add(&ys[2 * r + 1], qi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (lead)
      for (int r = i + 2 + tid; r < m; r += RES_NT) {
        __hip_atomic_store(&ysn[2 * r], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ysn[2 * r + 1], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    group_sync_coherent(ctr, gen, P, info);
    // (4) y, then w = tau y + alpha v with alpha = -tau (w^H v) / 2 (rows i+1..m-1)
    cx<double> wl[2], cn[2];
    cx<double> dot{0, 0};
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int r = i + 1 + tid + u * RES_NT;
      wl[u] = cn[u] = cx<double>{0, 0};
      if (r < m) {
        const long long qr = (long long)__hip_atomic_load(&ys[2 * r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const long long qi = (long long)__hip_atomic_load(&ys[2 * r + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const double* d = reinterpret_cast<const double*>(cxb + r);
        cn[u] = cx<double>{__hip_atomic_load(d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                           __hip_atomic_load(d + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)};
        const cx<double> yy{(double)qr * from_fix, (double)qi * from_fix};
        wl[u] = cmulc(tau, yy);
        cfmac(dot, wl[u], vcur[r]);
      }
    }
    dot = block_sum2<RES_W, false>(dot, red);
    const cx<double> alpha = cmulc(cx<double>{-0.5 * tau.re, -0.5 * tau.im}, dot);
    const bool zero = tau.re == 0.0 && tau.im == 0.0;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int r = i + 1 + tid + u * RES_NT;
      if (r < m) {
        cx<double> w = wl[u];
        cfma(w, alpha, vcur[r]);
        wv_[r] = zero ? cx<double>{0, 0} : w;
      }
    }
    __syncthreads();
    // (5) A -= v w^H + w v^H on the resident tiles (v and w vanish outside the
    // trailing rows, so the finished rows and columns are left as they are)
#pragma unroll
    for (int sl = 0; sl < RES_SLOTS; ++sl) {
      if (tok[sl] && tJ[sl] >= J0) {
        const int r0 = 32 * tI[sl] + 4 * la, c0 = 32 * tJ[sl] + lb;
        cx<double> vc[4], wc[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          vc[p] = vcur[c0 + 8 * p];
          wc[p] = wv_[c0 + 8 * p];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const cx<double> vr = vcur[r0 + q], wr = wv_[r0 + q];
          const cx<double> nv{-vr.re, -vr.im}, nw{-wr.re, -wr.im};
#pragma unroll
          for (int p = 0; p < 4; ++p) {
            cfmac(a[sl][q][p], wc[p], nv);
            cfmac(a[sl][q][p], vc[p], nw);
          }
        }
      }
    }
    // (6) column i + 1 after this step's update, in every workgroup, and the
    // per-wave partial sums of ||col[i + 3 ..]||^2 for the next reflector
    const cx<double> vi = vcur[i + 1], wi = wv_[i + 1];
    double s2n = 0;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int r = i + 1 + tid + u * RES_NT;
      if (r < m) {
        cx<double> x = cn[u];
        const cx<double> nv{-vcur[r].re, -vcur[r].im}, nw{-wv_[r].re, -wv_[r].im};
        cfmac(x, wi, nv);
        cfmac(x, vi, nw);
        if (r == i + 1) x.im = 0.0;
        col[r] = x;
        if (r >= i + 3) s2n += x.re * x.re + x.im * x.im;
      }
    }
    s2n = wave_sum(s2n);
    if (lane == 0) red2[(i + 1) & 1][wv] = s2n;
    __syncthreads();
  }
  if (tid == 0 && lead) {
    hv.d[m - 1] = col[m - 1].re;
    hv.e[m - 1] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// 2. eigenvalues by multisection (one wave per eigenvalue)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int sturm_count(const double* d, const double* e2, int m, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0;
  for (int i = 1; i < m; ++i) {
    // e2 / q with the hardware reciprocal refined by one Newton step (a
    // relative perturbation of e2 at rounding level: the count stays the
    // exact count of a nearby tridiagonal matrix)
    double r = __builtin_amdgcn_rcp(q);
    r = r * fma(-q, r, 2.0);
    q = (d[i] - x) - e2[i - 1] * r;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0;
  }
  return cnt;
}

__device__ __forceinline__ double wave_min(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Gershgorin interval of T (widened), pivmin and ||T|| for one wave.
__device__ void tri_bounds(const double* d, const double* e, int m, double* gl, double* gu, double* pivmin,
                           double* tnorm) {
  const int lane = threadIdx.x & 63;
  double lo = 1e300, hi = -1e300, em = 0;
  for (int i = lane; i < m; i += 64) {
    const double r = fabs(e[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0);
    lo = fmin(lo, d[i] - r);
    hi = fmax(hi, d[i] + r);
    em = fmax(em, e[i] * e[i]);
  }
  lo = wave_min(lo);
  hi = wave_max(hi);
  em = wave_max(em);
  const double eps = 2.220446049250313e-16;
  const double tn = fmax(fabs(lo), fabs(hi));
  *pivmin = 2.2250738585072014e-308 * fmax(1.0, em);
  *tnorm = tn;
  *gl = lo - 2.0 * eps * tn * m - 2.0 * (*pivmin);
  *gu = hi + 2.0 * eps * tn * m + 2.0 * (*pivmin);
}

__global__ __launch_bounds__(256) void heig_bisect_kernel(int m, int k, unsigned char* scratch, size_t per_slice,
                                                          double* __restrict__ lambda_out, int* info) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* d = reinterpret_cast<double*>(smem);
  double* e = d + m;
  double* e2 = e + m;
  const int f = blockIdx.x;
  HeigView hv = heig_view(scratch, per_slice, f, m);
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    d[i] = hv.d[i];
    e[i] = hv.e[i];
    e2[i] = hv.e[i] * hv.e[i];
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int t = blockIdx.y * (blockDim.x >> 6) + wave;
  if (t >= k) return;
  double lo, hi, pivmin, tnorm;
  tri_bounds(d, e, m, &lo, &hi, &pivmin, &tnorm);
  const int idx = m - 1 - t;
  const double eps = 2.220446049250313e-16;
  for (int it = 0; it < 64; ++it) {
    if (hi - lo <= 2.0 * eps * fmax(fabs(lo), fabs(hi)) + 4.0 * pivmin) break;
    const double x = lo + (hi - lo) * (double)(lane + 1) / 65.0;
    const int cnt = sturm_count(d, e2, m, x, pivmin);
    const unsigned long long above = __ballot(cnt > idx);  // lanes whose point lies above lambda_idx
    const int p = above ? __ffsll((long long)above) - 1 : 64;  // first such lane
    const double xp = __shfl(x, p < 64 ? p : 63, 64);
    const double xm = __shfl(x, p > 0 ? p - 1 : 0, 64);
    const double nlo = p > 0 ? xm : lo;
    const double nhi = p < 64 ? xp : hi;
    if (nlo == lo && nhi == hi) break;
    lo = nlo;
    hi = nhi;
  }
  if (lane == 0) {
    const double lv = 0.5 * (lo + hi);
    lambda_out[(int64_t)f * k + t] = lv;
    if (!isfinite(lv)) atomicAdd(&info[INFO_NONFINITE], 1);
  }
}

// ---------------------------------------------------------------------------
// 3. eigenvectors of T by inverse iteration (one wave per cluster)
// ---------------------------------------------------------------------------
// Order LDS traffic between the lanes of one wave (the wave runs in lockstep;
// this keeps the compiler from moving LDS accesses across the point).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Waves (eigenvectors) per workgroup of the inverse iteration.  The LU
// factors and the iterate live in registers (NCH 64-entry chunks per lane);
// LDS holds T (2 m doubles) and one m-vector per wave for the residual.
constexpr int INVIT_NW = 4;

// Value of v held by lane j (j uniform across the wave): two v_readlane_b32.
// The dependent chains of the inverse iteration walk through a 64-entry chunk
// that the lanes fetched from LDS in parallel, at register latency.
__device__ __forceinline__ double lane_get(double v, int j) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffull), j);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), j);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ double hash_uniform(uint32_t a, uint32_t b) {
  uint32_t h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  h *= 0x297A2D39u;
  h ^= h >> 15;
  return (double)h * (2.0 / 4294967296.0) - 1.0;
}

template <int NCH>
__global__ __launch_bounds__(256) void heig_invit_kernel(int m, int k, unsigned char* scratch, size_t per_slice,
                                                         const double* __restrict__ lambda,
                                                         cx<double>* __restrict__ Wout, int* info,
                                                         double vfloor_rel) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* d = reinterpret_cast<double*>(smem);
  double* e = d + m;
  const int f = blockIdx.x;
  const int nw = blockDim.x >> 6;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* zs = e + m + (size_t)wave * m;  // this wave's iterate, for the residual
  HeigView hv = heig_view(scratch, per_slice, f, m);
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    d[i] = hv.d[i];
    e[i] = hv.e[i];
  }
  __syncthreads();
  const int t0 = blockIdx.y * nw + wave;
  if (t0 >= k) return;
  const double* lam = lambda + (int64_t)f * k;
  cx<double>* W = Wout + (int64_t)f * m * k;
  double gl, gu, pivmin, tnorm;
  tri_bounds(d, e, m, &gl, &gu, &pivmin, &tnorm);
  const double eps = 2.220446049250313e-16;
  // Eigenvalues closer than ortol form a cluster whose vectors are computed
  // in sequence and re-orthogonalised against each other; vectors of
  // eigenvalues further apart are computed independently (in parallel), with
  // a contamination of about eps * ||T|| / gap <= 2e-7 by their neighbours.
  const double ortol = 1e-9 * tnorm;
  // eigenvalues at or below vfloor_rel * lambda_0 (when vfloor_rel > 0) get a
  // zero vector and are not computed: a caller that discards them saves the
  // inverse iterations of a large cluster near zero
  const bool use_floor = vfloor_rel > 0.0;
  const double vfloor = vfloor_rel * lam[0];
  if (use_floor && !(lam[t0] > vfloor)) {
    for (int i = lane; i < m; i += 64) W[(int64_t)i * k + t0] = cx<double>{0.0, 0.0};
    return;
  }
  if (t0 > 0 && lam[t0 - 1] - lam[t0] < ortol) return;  // not the head of its cluster
  int t1 = t0 + 1;
  while (t1 < k && lam[t1 - 1] - lam[t1] < ortol && !(use_floor && !(lam[t1] > vfloor))) ++t1;
  const double tinyp = eps * fmax(tnorm, 1e-300);
  for (int t = t0; t < t1; ++t) {
    const double lv = lam[t];
    // pivoted LU of T - lambda I; entry 64 c + lane of the factors (reciprocal
    // pivot, the two entries right of it, multiplier, row swap) stays in this
    // lane's registers, chunk c.  The recurrence runs, uniform, in every lane.
    double r0[NCH], r1[NCH], r2[NCH], rmu[NCH], rsw[NCH], Z[NCH];
    double pc = d[0] - lv, qc = (m > 1) ? e[0] : 0.0, rc = 0.0;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      r0[c] = 1.0;
      r1[c] = r2[c] = rmu[c] = rsw[c] = 0.0;
      const int base = 64 * c;
      if (base < m - 1) {
        const int i = base + lane;
        const int cnt = min(64, m - 1 - base);
        const double ei_l = i < m - 1 ? e[i] : 0.0;
        const double an_l = i < m - 1 ? d[i + 1] - lv : 0.0;
        const double en_l = i + 1 < m - 1 ? e[i + 1] : 0.0;
        double o0 = 1.0, o1 = 0.0, o2 = 0.0, om = 0.0, os = 0.0;
        for (int j = 0; j < cnt; ++j) {
          const double ei = lane_get(ei_l, j);
          const double an = lane_get(an_l, j);
          const double en = lane_get(en_l, j);
          double s0, s1, s2, sm, ss;
          if (fabs(pc) >= fabs(ei)) {
            double piv = pc;
            if (fabs(piv) < tinyp) piv = copysign(tinyp, piv == 0.0 ? 1.0 : piv);
            const double mu = ei / piv;
            s0 = piv;
            s1 = qc;
            s2 = rc;
            sm = mu;
            ss = 0.0;
            pc = an - mu * qc;
            qc = en - mu * rc;
            rc = 0.0;
          } else {
            const double mu = pc / ei;
            s0 = ei;
            s1 = an;
            s2 = en;
            sm = mu;
            ss = 1.0;
            const double npc = qc - mu * an;
            const double nqc = rc - mu * en;
            pc = npc;
            qc = nqc;
            rc = 0.0;
          }
          if (lane == j) {
            o0 = s0;
            o1 = s1;
            o2 = s2;
            om = sm;
            os = ss;
          }
        }
        if (lane < cnt) {
          r0[c] = 1.0 / o0;  // the solves multiply by the reciprocal pivots
          r1[c] = o1;
          r2[c] = o2;
          rmu[c] = om;
          rsw[c] = os;
        }
      }
    }
    if (fabs(pc) < tinyp) pc = copysign(tinyp, pc == 0.0 ? 1.0 : pc);
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      if (64 * c + lane == m - 1) {
        r0[c] = 1.0 / pc;
        r1[c] = r2[c] = 0.0;
      }
      const int i = 64 * c + lane;
      Z[c] = i < m ? hash_uniform((uint32_t)t, (uint32_t)i) : 0.0;
    }
    for (int it = 0; it < 4; ++it) {
      // forward elimination with the row swaps and multipliers, then back
      // substitution, uniform in every lane over the chunks; z[i + 1] of
      // step i is the next lane's entry (or lane 0 of the next chunk)
      double zc = lane_get(Z[0], 0);
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        const int base = 64 * c;
        if (base < m - 1) {
          const int cnt = min(64, m - 1 - base);
          const double znext = c + 1 < NCH ? lane_get(Z[c + 1 < NCH ? c + 1 : c], 0) : 0.0;
          double out = 0.0;
          for (int j = 0; j < cnt; ++j) {
            double zn = j < 63 ? lane_get(Z[c], j + 1) : znext;
            if (lane_get(rsw[c], j) != 0.0) {
              const double tmp = zc;
              zc = zn;
              zn = tmp;
            }
            if (lane == j) out = zc;
            zc = zn - lane_get(rmu[c], j) * zc;
          }
          if (lane < cnt) Z[c] = out;
        }
      }
#pragma unroll
      for (int c = 0; c < NCH; ++c)
        if (64 * c + lane == m - 1) Z[c] = zc;
      double z1 = 0.0, z2 = 0.0;
#pragma unroll
      for (int c = NCH - 1; c >= 0; --c) {
        const int base = 64 * c;
        if (base < m) {
          const int cnt = min(64, m - base);
          double out = 0.0;
          for (int j = cnt - 1; j >= 0; --j) {
            const double v = (lane_get(Z[c], j) - lane_get(r1[c], j) * z1 - lane_get(r2[c], j) * z2) *
                             lane_get(r0[c], j);
            if (lane == j) out = v;
            z2 = z1;
            z1 = v;
          }
          if (lane < cnt) Z[c] = out;
        }
      }
      // re-orthogonalise against the earlier members of the cluster
      for (int t2 = t0; t2 < t; ++t2) {
        double cc = 0;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          const int i = 64 * c + lane;
          if (i < m) cc += Z[c] * W[(int64_t)i * k + t2].re;
        }
        cc = wave_sum(cc);
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          const int i = 64 * c + lane;
          if (i < m) Z[c] -= cc * W[(int64_t)i * k + t2].re;
        }
      }
      double nrm = 0;
#pragma unroll
      for (int c = 0; c < NCH; ++c) nrm += Z[c] * Z[c];
      nrm = wave_sum(nrm);
      nrm = nrm > 0 ? 1.0 / sqrt(nrm) : 0.0;
#pragma unroll
      for (int c = 0; c < NCH; ++c) Z[c] *= nrm;
    }
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const int i = 64 * c + lane;
      if (i < m) zs[i] = Z[c];
    }
    wave_sync();
    double res = 0;
    for (int i = lane; i < m; i += 64) {
      double y = (d[i] - lv) * zs[i];
      if (i > 0) y += e[i - 1] * zs[i - 1];
      if (i + 1 < m) y += e[i] * zs[i + 1];
      res = fmax(res, fabs(y));
    }
    res = wave_max(res);
    if (lane == 0 && !(res <= 1e3 * m * eps * fmax(tnorm, 1e-300))) atomicAdd(&info[INFO_EIG_NOCONV], 1);
    for (int i = lane; i < m; i += 64) W[(int64_t)i * k + t] = cx<double>{zs[i], 0.0};
    wave_sync();
    __threadfence();
  }
}

// ---------------------------------------------------------------------------
// 4. back-transformation W = H_0 ... H_{m-2} Z (8 columns per workgroup)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void heig_backxf_kernel(int m, int k, unsigned char* scratch, size_t per_slice,
                                                          cx<double>* __restrict__ Wout) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NC = 8;
  cx<double>* Wl = reinterpret_cast<cx<double>*>(smem);  // m x NC
  cx<double>* vl = Wl + (size_t)m * NC;                   // m
  __shared__ cx<double> sc[NC];
  const int f = blockIdx.x;
  const int c0 = blockIdx.y * NC;
  const int tid = threadIdx.x;
  HeigView hv = heig_view(scratch, per_slice, f, m);
  cx<double>* W = Wout + (int64_t)f * m * k;
  for (int idx = tid; idx < m * NC; idx += 256) {
    const int r = idx / NC, g = idx % NC;
    Wl[idx] = (c0 + g < k) ? W[(int64_t)r * k + c0 + g] : cx<double>{0, 0};
  }
  __syncthreads();
  const int g = tid >> 5, l32 = tid & 31;
  constexpr int PF = 4;  // v elements per thread held in registers (m <= 1024)
  cx<double> nxt[PF];
  auto fetch = [&](int j) {
    const int L = m - j - 1;
    const cx<double>* vg = hv.A + (int64_t)j * m + (j + 1);
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int i = tid + u * 256;
      nxt[u] = i < L ? vg[i] : cx<double>{0, 0};
    }
  };
  if (m >= 2) fetch(m - 2);
  for (int j = m - 2; j >= 0; --j) {
    const cx<double> tau = hv.tau[j];
    const int L = m - j - 1;
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int i = tid + u * 256;
      if (i < L) vl[i] = nxt[u];
    }
    if (j > 0) fetch(j - 1);
    if (tau.re == 0.0 && tau.im == 0.0) continue;
    __syncthreads();
    double sr = 0, si = 0;
    for (int i = l32; i < L; i += 32) {
      const cx<double> t = cjmul(vl[i], Wl[(j + 1 + i) * NC + g]);
      sr += t.re;
      si += t.im;
    }
    for (int o = 16; o > 0; o >>= 1) {
      sr += __shfl_xor(sr, o, 64);
      si += __shfl_xor(si, o, 64);
    }
    if (l32 == 0) sc[g] = cmulc(tau, cx<double>{sr, si});
    __syncthreads();
    for (int idx = tid; idx < L * NC; idx += 256) {
      const int i = idx / NC, gg = idx % NC;
      const cx<double> t = cmulc(vl[i], sc[gg]);
      cx<double>& w = Wl[(j + 1 + i) * NC + gg];
      w.re -= t.re;
      w.im -= t.im;
    }
    __syncthreads();
  }
  for (int idx = tid; idx < m * NC; idx += 256) {
    const int r = idx / NC, gg = idx % NC;
    if (c0 + gg < k) W[(int64_t)r * k + c0 + gg] = Wl[idx];
  }
}

// Back-transformation with the columns in registers: each half-wave owns one
// of the workgroup's 8 columns of W (rows l32 + 32 s), so the product with a
// reflector and the update need only lane exchanges.  The reflectors pass
// through LDS in groups of NB (double-buffered by group; the next group is
// fetched into registers while the current one is applied), one workgroup
// barrier per group: the NB reflectors of a group are applied in order
// with no barrier between them, since no half-wave reads another's column.
template <int S, int NB>
__global__ __launch_bounds__(256) void heig_backxf2_kernel(int m, int k, unsigned char* scratch, size_t per_slice,
                                                           cx<double>* __restrict__ Wout) {
  extern __shared__ __align__(16) unsigned char smem[];
  cx<double>* vbuf = reinterpret_cast<cx<double>*>(smem);  // 2 groups x NB x m
  const int f = blockIdx.x;
  const int tid = threadIdx.x, g = tid >> 5, l32 = tid & 31;
  const int col = blockIdx.y * 8 + g;
  const bool colok = col < k;
  HeigView hv = heig_view(scratch, per_slice, f, m);
  cx<double>* W = Wout + (int64_t)f * m * k;
  cx<double> w[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int r = l32 + 32 * s;
    w[s] = (colok && r < m) ? W[(int64_t)r * k + col] : cx<double>{0, 0};
  }
  constexpr int PF = 4;  // reflector entries per thread and reflector (m <= 1024)
  // reflectors j0 .. 0 in descending order; group q holds j = j0 - q NB - u, u < NB
  const int j0 = m - 2;
  const int ng = (j0 + NB) / NB;
  cx<double> pre[NB][PF];
  auto fetch = [&](int q) {
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int j = j0 - q * NB - u;
      const int L = m - j - 1;
      const cx<double>* vg = hv.A + (int64_t)(j >= 0 ? j : 0) * m + (j + 1);
#pragma unroll
      for (int p = 0; p < PF; ++p) {
        const int i = tid + p * 256;
        pre[u][p] = (j >= 0 && i < L) ? vg[i] : cx<double>{0, 0};
      }
    }
  };
  auto stage = [&](int q) {
    cx<double>* vb = vbuf + (size_t)(q & 1) * NB * m;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int j = j0 - q * NB - u;
      const int L = m - j - 1;
#pragma unroll
      for (int p = 0; p < PF; ++p) {
        const int i = tid + p * 256;
        if (j >= 0 && i < L) vb[(size_t)u * m + i] = pre[u][p];
      }
    }
  };
  auto apply = [&](int j, const cx<double>* vb) {
    const cx<double> tau = hv.tau[j];
    if (tau.re == 0.0 && tau.im == 0.0) return;
    // rows r = j + 1 + i of the reflector; row r of W sits in w[(r - l32) / 32].
    // The lane's entries of the reflector are read from LDS once, for both
    // the product and the update.
    cx<double> vv[S];
    double sr = 0, si = 0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int i = l32 + 32 * s - j - 1;
      vv[s] = (i >= 0 && i < m - j - 1) ? vb[i] : cx<double>{0, 0};
      const cx<double> t = cjmul(vv[s], w[s]);
      sr += t.re;
      si += t.im;
    }
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) {
      sr += __shfl_xor(sr, o, 64);
      si += __shfl_xor(si, o, 64);
    }
    const cx<double> sc = cmulc(tau, cx<double>{sr, si});
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const cx<double> t = cmulc(vv[s], sc);
      w[s].re -= t.re;
      w[s].im -= t.im;
    }
  };
  if (ng > 0) {
    fetch(0);
    stage(0);
    if (ng > 1) fetch(1);
  }
  __syncthreads();
  for (int q = 0; q < ng; ++q) {
    const cx<double>* vb = vbuf + (size_t)(q & 1) * NB * m;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int j = j0 - q * NB - u;
      if (j >= 0) apply(j, vb + (size_t)u * m);
    }
    if (q + 1 < ng) {
      stage(q + 1);
      if (q + 2 < ng) fetch(q + 2);
    }
    __syncthreads();
  }
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int r = l32 + 32 * s;
    if (colok && r < m) W[(int64_t)r * k + col] = w[s];
  }
}

hipError_t heig_topk(const double* Gpart, int nsum, int64_t part_stride, int m, int k, int batch, double* lambda,
                     double* W, void* scratch, int* info, hipStream_t s, int stages, bool upper_only,
                     double vfloor_rel) {
  if (batch <= 0) return hipSuccess;
  if (m > 1024 || k > m || k < 1) return hipErrorInvalidValue;
  static bool attr_set = false;
  if (!attr_set) {
    // dynamic LDS limits, leaving room for each kernel's static LDS
    (void)hipFuncSetAttribute((const void*)heig_tridiag_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              152 * 1024);
    (void)hipFuncSetAttribute((const void*)heig_tri2_kernel<8>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              152 * 1024);
    (void)hipFuncSetAttribute((const void*)heig_tri2_kernel<4>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              152 * 1024);
    (void)hipFuncSetAttribute((const void*)heig_backxf_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              152 * 1024);
    (void)hipGetLastError();
    attr_set = true;
  }
  const size_t per = heig_per_slice(m, k);
  unsigned char* sc = (unsigned char*)scratch;
  // 1. tridiagonalisation: vectors (4 m) + trailing matrix in LDS (Lsw^2)
  const size_t lds_total = 150 * 1024;
  const size_t vec_bytes = (size_t)(4 + TRI_G) * m * sizeof(cx<double>);
  int Lsw = 0;
  if (lds_total > vec_bytes) {
    Lsw = (int)sqrt((double)(lds_total - vec_bytes) / sizeof(cx<double>));
    if (Lsw > m - 1) Lsw = m - 1;
  }
  const size_t sm1 = vec_bytes + (size_t)Lsw * Lsw * sizeof(cx<double>);
  hipError_t e = hipSuccess;
  // blocked form when the matrix spans a few tiles and its panel fits in LDS
  const int MP = (m + 31) / 32 * 32;
  auto sm2 = [&](int nb) { return ((size_t)(2 * nb + 3) * MP + 2 * nb) * sizeof(cx<double>); };
  const bool blocked = m >= 64 && m <= 2 * T2_NT + 1;
  if ((stages & HEIG_TRIDIAG) && blocked && sm2(4) <= lds_total) {
    const int nb = sm2(8) <= lds_total ? 8 : 4;
    const size_t sm = sm2(nb);
    const void* fn = nb == 8 ? (const void*)heig_tri2_kernel<8> : (const void*)heig_tri2_kernel<4>;
    hipLaunchKernelGGL(heig_prep_kernel, dim3(batch, PREP_WG), dim3(256), 0, s, (const cx<double>*)Gpart, nsum,
                       part_stride, m, upper_only ? 1 : 0, sc, per);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // several co-resident workgroups per slice for large m when the slices
    // leave CUs idle (cooperative launch guarantees co-residency)
    int P = 1;
    if (m >= 256) {
      static int coop = -1, cus = 0;
      if (coop < 0) {
        int dev = 0;
        coop = 0;
        if (hipGetDevice(&dev) == hipSuccess) {
          (void)hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
          (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        }
        (void)hipGetLastError();
      }
      if (coop > 0 && cus > 0) P = std::min(TRI_PMAX, cus / batch);
      if (P < 2) P = 1;
    }
    const cx<double>* G = (const cx<double>*)Gpart;
    int nsum_a = nsum, m_a = m, mp_a = MP, up = upper_only ? 1 : 0;
    int64_t ps = part_stride;
    unsigned char* sc_a = sc;
    size_t per_a = per;
    int* info_a = info;
    // the register-resident form when the slice's tiles fit RES_SLOTS per wave
    const int NTt = (MP / 32) * (MP / 32 + 1) / 2;
    bool done = false;
    if (P > 1 && MP <= 2 * RES_NT && NTt <= RES_SLOTS * RES_W * P) {
      void* args[] = {(void*)&G, (void*)&nsum_a, (void*)&ps, (void*)&m_a, (void*)&mp_a, (void*)&sc_a, (void*)&per_a,
                      (void*)&up, (void*)&P, (void*)&info_a};
      if (hipLaunchCooperativeKernel((const void*)heig_trires_kernel, dim3(batch * P), dim3(RES_NT), args, 0, s) ==
          hipSuccess)
        done = true;
      else
        (void)hipGetLastError();  // not co-resident: the streaming form below
    }
    if (!done && P > 1) {
      void* args[] = {(void*)&G, (void*)&nsum_a, (void*)&ps, (void*)&m_a, (void*)&mp_a, (void*)&sc_a, (void*)&per_a,
                      (void*)&up, (void*)&P, (void*)&info_a};
      if (hipLaunchCooperativeKernel(fn, dim3(batch * P), dim3(T2_NT), args, (unsigned)sm, s) != hipSuccess) {
        (void)hipGetLastError();  // not co-resident at this size: one workgroup per slice
        P = 1;
      }
    }
    if (P == 1) {
      if (nb == 8)
        hipLaunchKernelGGL(heig_tri2_kernel<8>, dim3(batch), dim3(T2_NT), sm, s, G, nsum_a, ps, m_a, mp_a, sc_a, per_a,
                           up, 1, info_a);
      else
        hipLaunchKernelGGL(heig_tri2_kernel<4>, dim3(batch), dim3(T2_NT), sm, s, G, nsum_a, ps, m_a, mp_a, sc_a, per_a,
                           up, 1, info_a);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
  } else if (stages & HEIG_TRIDIAG) {
    hipLaunchKernelGGL(heig_tridiag_kernel, dim3(batch), dim3(TRI_NT), sm1, s, (const cx<double>*)Gpart, nsum,
                       part_stride, m, sc, per, Lsw, upper_only ? 1 : 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // 2. eigenvalues: 4 waves (eigenvalues) per workgroup
  if (stages & HEIG_BISECT) {
    hipLaunchKernelGGL(heig_bisect_kernel, dim3(batch, (k + 3) / 4), dim3(256), (size_t)3 * m * sizeof(double), s,
                       m, k, sc, per, lambda, info);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // 3. eigenvectors: LU factors and iterates in registers (NCH chunks of 64
  // entries per lane), T and one m-vector per wave in LDS
  if (stages & HEIG_INVIT) {
    const int nw = INVIT_NW;
    const size_t sm3 = (size_t)(2 + nw) * m * sizeof(double);
    const dim3 g3(batch, (k + nw - 1) / nw), b3(64 * nw);
    if (m <= 128)
      hipLaunchKernelGGL(heig_invit_kernel<2>, g3, b3, sm3, s, m, k, sc, per, lambda, (cx<double>*)W, info, vfloor_rel);
    else if (m <= 256)
      hipLaunchKernelGGL(heig_invit_kernel<4>, g3, b3, sm3, s, m, k, sc, per, lambda, (cx<double>*)W, info, vfloor_rel);
    else if (m <= 512)
      hipLaunchKernelGGL(heig_invit_kernel<8>, g3, b3, sm3, s, m, k, sc, per, lambda, (cx<double>*)W, info, vfloor_rel);
    else
      hipLaunchKernelGGL(heig_invit_kernel<16>, g3, b3, sm3, s, m, k, sc, per, lambda, (cx<double>*)W, info,
                         vfloor_rel);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // 4. back-transformation
  const size_t sm4 = ((size_t)m * 8 + m) * sizeof(cx<double>);
  if (stages & HEIG_BACKXF) {
    // two LDS groups of NB reflectors: 4 up to m = 448 (56 KB), 2 above
    const size_t sm5a = (size_t)2 * 4 * m * sizeof(cx<double>), sm5b = (size_t)2 * 2 * m * sizeof(cx<double>);
    const dim3 g5(batch, (k + 7) / 8);
    if (m <= 8 * 32)
      hipLaunchKernelGGL((heig_backxf2_kernel<8, 4>), g5, dim3(256), sm5a, s, m, k, sc, per, (cx<double>*)W);
    else if (m <= 14 * 32)
      hipLaunchKernelGGL((heig_backxf2_kernel<14, 4>), g5, dim3(256), sm5a, s, m, k, sc, per, (cx<double>*)W);
    else if (m <= 20 * 32)
      hipLaunchKernelGGL((heig_backxf2_kernel<20, 2>), g5, dim3(256), sm5b, s, m, k, sc, per, (cx<double>*)W);
    else
      hipLaunchKernelGGL(heig_backxf_kernel, dim3(batch, (k + 7) / 8), dim3(256), sm4, s, m, k, sc, per,
                         (cx<double>*)W);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace tsvd
