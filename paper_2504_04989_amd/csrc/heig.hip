// Top-k eigenpairs of a per-slice m x m Hermitian positive semidefinite
// matrix in FP64: the small decomposition behind the per-slice SVD of
// C_f = Q_f^H A_f in Alg. 2.  With C_f C_f^H = W diag(lambda) W^H, the left
// singular vectors of C_f are W, sigma = sqrt(lambda), and the right singular
// vectors are C_f^H W diag(1/sigma).
//
// One 256-thread workgroup per Fourier slice:
//  1. sum the split-K partials and symmetrise, G = (S + S^H) / 2;
//  2. Householder reduction to a real symmetric tridiagonal matrix,
//     G = H T H^H, H = H_0 ... H_{m-2}, H_j = I - tau_j v_j v_j^H
//     (complex reflectors with real beta, so T is real);
//  3. the k largest eigenvalues of T by bisection on Sturm counts (each
//     thread one eigenvalue);
//  4. their eigenvectors by inverse iteration on the pivoted LU of T - lambda I,
//     re-orthogonalised within clusters of close eigenvalues;
//  5. back-transformation W = H Z.
// The matrix lives in global scratch (L2-resident at these sizes); vectors
// and the tridiagonal live in LDS.
#include "common.h"
#include "kernels.h"

namespace tsvd {

static inline size_t heig_per_slice(int m, int k) {
  size_t b = (size_t)16 * m * m + (size_t)16 * m + (size_t)48 * k * m;
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

__device__ __forceinline__ int sturm_count(const double* d, const double* e2, int m, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0;
  for (int i = 1; i < m; ++i) {
    q = (d[i] - x) - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0;
  }
  return cnt;
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

__global__ __launch_bounds__(256) void heig_kernel(const cx<double>* __restrict__ Gpart, int nsum, int64_t part_stride,
                                                   int m, int k, double* __restrict__ lambda_out,
                                                   cx<double>* __restrict__ Wout, unsigned char* scratch,
                                                   size_t per_slice, int* info) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* d = reinterpret_cast<double*>(smem);
  double* e = d + m;
  double* e2 = e + m;
  cx<double>* v = reinterpret_cast<cx<double>*>(e2 + m);
  cx<double>* p = v + m;
  int* rank = reinterpret_cast<int*>(p + m);
  int* cstart = rank + k;
  __shared__ double red[8];
  __shared__ cx<double> s_tau, s_scale;
  __shared__ int s_skip, s_maxrank;
  __shared__ double s_gl, s_gu, s_pivmin, s_tnorm;

  const int f = blockIdx.x;
  const int tid = threadIdx.x;
  cx<double>* A = reinterpret_cast<cx<double>*>(scratch + (size_t)f * per_slice);
  cx<double>* tau_g = A + (size_t)m * m;
  double* lu = reinterpret_cast<double*>(tau_g + m);
  const cx<double>* G = Gpart + (int64_t)f * m * m;
  double* lam = lambda_out + (int64_t)f * k;
  cx<double>* W = Wout + (int64_t)f * m * k;

  // 1. symmetrised sum of the partials
  for (int64_t t = tid; t < (int64_t)m * m; t += 256) {
    const int i = (int)(t / m), c = (int)(t % m);
    double re = 0, im = 0, re2 = 0, im2 = 0;
    for (int s = 0; s < nsum; ++s) {
      const cx<double> g = G[s * part_stride + (int64_t)i * m + c];
      const cx<double> h = G[s * part_stride + (int64_t)c * m + i];
      re += g.re;
      im += g.im;
      re2 += h.re;
      im2 += h.im;
    }
    A[t] = cx<double>{0.5 * (re + re2), i == c ? 0.0 : 0.5 * (im - im2)};
  }
  __syncthreads();

  // 2. Householder tridiagonalisation (lower form; row j keeps v_j afterwards).
  for (int j = 0; j < m - 1; ++j) {
    const int L = m - j - 1;
    cx<double>* rowj = A + (int64_t)j * m + (j + 1);  // conj of column j below the diagonal
    double s2 = 0;
    for (int r = 1 + tid; r < L; r += 256) {
      const cx<double> a = rowj[r];
      s2 += a.re * a.re + a.im * a.im;
    }
    s2 = block_sum<256>(s2, red);
    if (tid == 0) {
      d[j] = A[(int64_t)j * m + j].re;
      const double ar = rowj[0].re, ai = -rowj[0].im;  // alpha = conj(row entry)
      if (s2 == 0.0 && ai == 0.0) {
        s_skip = 1;
        e[j] = ar;
        s_tau = cx<double>{0, 0};
      } else {
        s_skip = 0;
        const double beta = -copysign(sqrt(ar * ar + ai * ai + s2), ar);
        s_tau = cx<double>{(beta - ar) / beta, -ai / beta};
        // scale = 1 / (alpha - beta)
        const double dr = ar - beta, di = ai;
        const double den = dr * dr + di * di;
        s_scale = cx<double>{dr / den, -di / den};
        e[j] = beta;
      }
      tau_g[j] = s_tau;
    }
    __syncthreads();
    if (s_skip) {
      for (int r = tid; r < L; r += 256) rowj[r] = cx<double>{r == 0 ? 1.0 : 0.0, 0.0};
      __syncthreads();
      continue;
    }
    const cx<double> tau = s_tau, scale = s_scale;
    for (int r = tid; r < L; r += 256) {
      cx<double> vr;
      if (r == 0) {
        vr = cx<double>{1.0, 0.0};
      } else {
        const cx<double> a = rowj[r];
        vr = cmulc(cx<double>{a.re, -a.im}, scale);
      }
      v[r] = vr;
      rowj[r] = vr;
    }
    __syncthreads();
    // p = tau * A22 v, with A22[c][r] = conj(A22[r][c]) (coalesced row reads)
    cx<double>* A22 = A + (int64_t)(j + 1) * m + (j + 1);
    for (int c = tid; c < L; c += 256) {
      double ar = 0, ai = 0;
      for (int r = 0; r < L; ++r) {
        const cx<double> a = A22[(int64_t)r * m + c];
        const cx<double> t = cjmul(a, v[r]);
        ar += t.re;
        ai += t.im;
      }
      p[c] = cmulc(tau, cx<double>{ar, ai});
    }
    __syncthreads();
    double pr = 0, pi = 0;
    for (int c = tid; c < L; c += 256) {
      const cx<double> t = cjmul(p[c], v[c]);
      pr += t.re;
      pi += t.im;
    }
    pr = block_sum<256>(pr, red);
    pi = block_sum<256>(pi, red + 4);
    const cx<double> alpha2 = cmulc(cx<double>{-0.5 * tau.re, -0.5 * tau.im}, cx<double>{pr, pi});
    for (int c = tid; c < L; c += 256) {
      const cx<double> t = cmulc(alpha2, v[c]);
      p[c].re += t.re;
      p[c].im += t.im;
    }
    __syncthreads();
    // A22 -= v w^H + w v^H
    for (int r = 0; r < L; ++r) {
      const cx<double> vr = v[r], wr = p[r];
      cx<double>* row = A22 + (int64_t)r * m;
      for (int c = tid; c < L; c += 256) {
        const cx<double> wc = p[c], vc = v[c];
        cx<double> a = row[c];
        // v_r conj(w_c) + w_r conj(v_c)
        a.re -= (vr.re * wc.re + vr.im * wc.im) + (wr.re * vc.re + wr.im * vc.im);
        a.im -= (vr.im * wc.re - vr.re * wc.im) + (wr.im * vc.re - wr.re * vc.im);
        row[c] = a;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    d[m - 1] = A[(int64_t)(m - 1) * m + (m - 1)].re;
    e[m - 1] = 0.0;
  }
  __syncthreads();
  for (int i = tid; i < m; i += 256) e2[i] = e[i] * e[i];
  __syncthreads();

  // 3. Gershgorin interval and bisection for the k largest eigenvalues.
  __syncthreads();
  double lo = 1e300, hi = -1e300, emax = 0;
  for (int i = tid; i < m; i += 256) {
    const double r = fabs(e[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0);
    lo = fmin(lo, d[i] - r);
    hi = fmax(hi, d[i] + r);
    emax = fmax(emax, e2[i]);
  }
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off, 64));
    hi = fmax(hi, __shfl_xor(hi, off, 64));
    emax = fmax(emax, __shfl_xor(emax, off, 64));
  }
  if ((tid & 63) == 0) {
    red[tid >> 6] = lo;
    red[4 + (tid >> 6)] = hi;
  }
  __syncthreads();
  if (tid == 0) {
    double l = red[0], h = red[4];
    for (int w = 1; w < 4; ++w) {
      l = fmin(l, red[w]);
      h = fmax(h, red[4 + w]);
    }
    s_gl = l;
    s_gu = h;
  }
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = emax;
  __syncthreads();
  if (tid == 0) {
    const double em = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    const double eps0 = 2.220446049250313e-16;
    const double tnorm = fmax(fabs(s_gl), fabs(s_gu));
    s_pivmin = 2.2250738585072014e-308 * fmax(1.0, em);
    s_tnorm = tnorm;
    s_gl -= 2.0 * eps0 * tnorm * m + 2.0 * s_pivmin;
    s_gu += 2.0 * eps0 * tnorm * m + 2.0 * s_pivmin;
  }
  __syncthreads();
  const double eps = 2.220446049250313e-16;
  const double pivmin = s_pivmin, tnorm = s_tnorm;
  for (int t = tid; t < k; t += 256) {
    const int idx = m - 1 - t;
    double a = s_gl, b = s_gu;
    for (int it = 0; it < 256; ++it) {
      if (b - a <= 2.0 * eps * fmax(fabs(a), fabs(b)) + 4.0 * pivmin) break;
      const double mid = 0.5 * (a + b);
      if (mid <= a || mid >= b) break;
      if (sturm_count(d, e2, m, mid, pivmin) <= idx)
        a = mid;
      else
        b = mid;
    }
    const double lv = 0.5 * (a + b);
    lam[t] = lv;
    if (!isfinite(lv)) atomicAdd(&info[INFO_NONFINITE], 1);
  }
  __syncthreads();

  // 4. clusters (descending order) and inverse iteration.
  if (tid == 0) {
    const double ortol = 1e-7 * tnorm;
    int mr = 0;
    int start = 0, r = 0;
    for (int t = 0; t < k; ++t) {
      if (t > 0 && lam[t - 1] - lam[t] < ortol) {
        ++r;
      } else {
        start = t;
        r = 0;
      }
      rank[t] = r;
      cstart[t] = start;
      mr = r > mr ? r : mr;
    }
    s_maxrank = mr;
  }
  __syncthreads();
  for (int round = 0; round <= s_maxrank; ++round) {
    for (int t = tid; t < k; t += 256) {
      if (rank[t] != round) continue;
      double* mult = lu + (size_t)t * 6 * m;
      double* swp = mult + m;
      double* u0 = swp + m;
      double* u1 = u0 + m;
      double* u2 = u1 + m;
      double* z = u2 + m;
      const double lv = lam[t];
      const double tinyp = eps * fmax(tnorm, 1e-300);
      // pivoted LU of T - lambda I
      double pc = d[0] - lv, qc = (m > 1) ? e[0] : 0.0, rc = 0.0;
      for (int i = 0; i < m - 1; ++i) {
        const double ei = e[i];
        const double an = d[i + 1] - lv;
        const double en = (i + 1 < m - 1) ? e[i + 1] : 0.0;
        if (fabs(pc) >= fabs(ei)) {
          double piv = pc;
          if (fabs(piv) < tinyp) piv = copysign(tinyp, piv == 0.0 ? 1.0 : piv);
          const double mu = ei / piv;
          u0[i] = piv;
          u1[i] = qc;
          u2[i] = rc;
          mult[i] = mu;
          swp[i] = 0.0;
          pc = an - mu * qc;
          qc = en - mu * rc;
          rc = 0.0;
        } else {
          const double mu = pc / ei;
          u0[i] = ei;
          u1[i] = an;
          u2[i] = en;
          mult[i] = mu;
          swp[i] = 1.0;
          const double npc = qc - mu * an;
          const double nqc = rc - mu * en;
          pc = npc;
          qc = nqc;
          rc = 0.0;
        }
      }
      if (fabs(pc) < tinyp) pc = copysign(tinyp, pc == 0.0 ? 1.0 : pc);
      u0[m - 1] = pc;
      u1[m - 1] = 0.0;
      u2[m - 1] = 0.0;
      // start vector
      double nrm = 0;
      for (int i = 0; i < m; ++i) {
        z[i] = hash_uniform((uint32_t)t, (uint32_t)i);
        nrm += z[i] * z[i];
      }
      nrm = 1.0 / sqrt(nrm);
      for (int i = 0; i < m; ++i) z[i] *= nrm;
      for (int it = 0; it < 5; ++it) {
        // forward: apply the row operations
        for (int i = 0; i < m - 1; ++i) {
          if (swp[i] != 0.0) {
            const double tmp = z[i];
            z[i] = z[i + 1];
            z[i + 1] = tmp;
          }
          z[i + 1] -= mult[i] * z[i];
        }
        // back substitution with the three upper diagonals
        for (int i = m - 1; i >= 0; --i) {
          double s = z[i];
          if (i + 1 < m) s -= u1[i] * z[i + 1];
          if (i + 2 < m) s -= u2[i] * z[i + 2];
          z[i] = s / u0[i];
        }
        // re-orthogonalise against earlier members of the cluster
        for (int t2 = cstart[t]; t2 < t; ++t2) {
          const double* z2 = lu + (size_t)t2 * 6 * m + 5 * (size_t)m;
          double c = 0;
          for (int i = 0; i < m; ++i) c += z[i] * z2[i];
          for (int i = 0; i < m; ++i) z[i] -= c * z2[i];
        }
        nrm = 0;
        for (int i = 0; i < m; ++i) nrm += z[i] * z[i];
        nrm = (nrm > 0) ? 1.0 / sqrt(nrm) : 0.0;
        for (int i = 0; i < m; ++i) z[i] *= nrm;
      }
      // residual check ||(T - lambda) z||_inf
      double res = 0;
      for (int i = 0; i < m; ++i) {
        double y = (d[i] - lv) * z[i];
        if (i > 0) y += e[i - 1] * z[i - 1];
        if (i + 1 < m) y += e[i] * z[i + 1];
        res = fmax(res, fabs(y));
      }
      if (!(res <= 1e3 * m * eps * fmax(tnorm, 1e-300))) atomicAdd(&info[INFO_EIG_NOCONV], 1);
      for (int i = 0; i < m; ++i) W[(int64_t)i * k + t] = cx<double>{z[i], 0.0};
    }
    __syncthreads();
  }

  // 5. back-transformation W = H_0 ... H_{m-2} Z
  for (int j = m - 2; j >= 0; --j) {
    const cx<double> tau = tau_g[j];
    if (tau.re == 0.0 && tau.im == 0.0) continue;
    const int L = m - j - 1;
    const cx<double>* vj = A + (int64_t)j * m + (j + 1);
    for (int r = tid; r < L; r += 256) v[r] = vj[r];
    __syncthreads();
    cx<double>* Wj = W + (int64_t)(j + 1) * k;
    for (int c = tid; c < k; c += 256) {
      double sr = 0, si = 0;
      for (int r = 0; r < L; ++r) {
        const cx<double> t = cjmul(v[r], Wj[(int64_t)r * k + c]);
        sr += t.re;
        si += t.im;
      }
      p[c] = cmulc(tau, cx<double>{sr, si});
    }
    __syncthreads();
    for (int64_t idx = tid; idx < (int64_t)L * k; idx += 256) {
      const int r = (int)(idx / k), c = (int)(idx % k);
      const cx<double> t = cmulc(v[r], p[c]);
      cx<double> w = Wj[idx];
      w.re -= t.re;
      w.im -= t.im;
      Wj[idx] = w;
    }
    __syncthreads();
  }
}

hipError_t heig_topk(const double* Gpart, int nsum, int64_t part_stride, int m, int k, int batch, double* lambda,
                     double* W, void* scratch, int* info, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  if (m > 1024 || k > m || k < 1) return hipErrorInvalidValue;
  const size_t sm = (size_t)7 * m * sizeof(double) + (size_t)2 * k * sizeof(int);
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)heig_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);
    attr_set = true;
  }
  hipLaunchKernelGGL(heig_kernel, dim3(batch), dim3(256), sm, s, (const cx<double>*)Gpart, nsum, part_stride, m, k,
                     lambda, (cx<double>*)W, (unsigned char*)scratch, heig_per_slice(m, k), info);
  return hipGetLastError();
}

}  // namespace tsvd
