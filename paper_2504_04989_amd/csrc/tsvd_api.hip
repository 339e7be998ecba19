// C ABI of the randomized block Krylov truncated T-SVD (Alg. 2 of the paper;
// see include/tsvd_rbk.h for the contract of every entry point).
//
// Host side: validates arguments, carves the caller's workspace and enqueues
// the kernels on the caller's stream.  Per call, for all Fourier slices at
// once (each launch is batched over the n3/2 + 1 slices):
//   mode-3 DFT of A and Omega                       (Sec. 2, Alg. TP)
//   K_0 = A_f Om_f; block orthonormalisation         (Alg. 2 Krylov loop, T-QR)
//   for i = 1..q: T_i = A_f^H Q_{i-1}; W = A_f T_i;  re-orthogonalise W
//                 against Q_<i (two block Gram-Schmidt passes) and
//                 orthonormalise it (shifted CholeskyQR, three passes)
//   T_{q+1} = A_f^H Q_q, so that [T_1 .. T_{q+1}] = A_f^H Q_f = C_f^H
//   G_f = C_f C_f^H (FP64); top-k eigenpairs -> sigma, W_k  (T-SVD of C)
//   U_f = Q_f W_k; V_f = C_f^H W_k diag(1/sigma)      (lift and truncation)
//   phase convention; inverse DFT of U, S, V          (Alg. TP mirror)
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tsvd_rbk.h"
#include "common.h"
#include "kernels.h"

using namespace tsvd;

namespace {

thread_local std::string g_err;

int fail(int code, const char* msg) {
  g_err = msg;
  return code;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Plan {
  int64_t n1, n2, n3, k, b, q, m, F;
  bool power;  // Alg. 1: basis of the last power iterate only (m = b)
  int prec;
  DType dt;
  size_t cs;  // bytes of one complex element in the working precision
  int nsplit_blk, kchunk_blk;   // split-K for K = n1 products (block Grams, projections)
  int nsplit_g, kchunk_g;       // split-K for G = T^H T (K = n2)
  int nsplit_t, kchunk_t;       // split-K for the n2-row block Grams of Alg. 1
  int nsplit_r, kchunk_r;       // split-K for R_f = Q_f^H A_f (T-QR, FP64 path)
  bool tensor_op;               // T-QR / pseudoinverse: QR of A_f itself, r = m = min(n1, n2) in
                                // q + 1 column panels of width b <= 128
  int kmode;                    // Krylov-product arithmetic (KM_*) when dt == DT_F32
  bool asplit;                  // BF16x3 with A_f transformed straight into (hi, lo) bf16 pairs
                                // (KM_BF16X3_SPLIT; A_f is read only by the Krylov products)
  int ks_ax, ks_ahy;            // K splits of the Krylov products A X and A^H Y
  size_t kpart_bytes;           // their partials (K splits or tail splits)
  // workspace offsets (bytes)
  size_t o_canon, o_rout, o_xp;
  size_t o_cbuf, o_xbuf, o_uo, o_so, o_vo;  // completion: C^(n), X^(n) and the factors of L
  size_t o_lam1, o_w1, o_w1m, o_p, o_t1, o_lam2, o_w2, o_rk, o_split;  // FP64 small SVD, second pass
  size_t o_omsp;  // the spatial test tensor drawn from the seed (n2 x b x n3, storage type)
  size_t o_vr, o_sr;  // truncated basis: spatial V and S of its Ritz step (scratch outputs)
  // adjoint through the rank-k truncation: all eigenpairs of C C^H, four
  // m x m FP64 matrices, the modified cotangents U2 Pi + T H and T Pi
  size_t o_wall, o_lall, o_mm0, o_mm1, o_mm2, o_mm3, o_u2b, o_tp;
  size_t o_info, o_abar, o_obar, o_q, o_t, o_s0, o_s1, o_part, o_rinv, o_chol, o_lam, o_sig, o_wd, o_wds, o_heig,
      o_uf, o_vf, o_scx, o_us, o_gbar, o_dbar, o_wraw, o_qbar, o_u2, o_zbar, o_wbar, o_tbar, o_kpart, o_kpack,
      total;
};

size_t proj32_layout(int64_t ib, int64_t n1, int64_t b, int64_t F, int* nsplit, size_t* coef_off);

int split_for(int64_t K, int64_t tiles, int64_t batch, int* kchunk) {
  int64_t ns = (K + 127) / 128;
  int64_t cap = std::max<int64_t>(1, 1024 / std::max<int64_t>(1, tiles * batch));
  ns = std::min(ns, cap);
  if (ns < 1) ns = 1;
  int64_t kc = (K + ns - 1) / ns;
  kc = (kc + 15) / 16 * 16;
  ns = (K + kc - 1) / kc;
  if (ns < 1) ns = 1;
  *kchunk = (int)std::max<int64_t>(kc, 16);
  return (int)ns;
}

// Sizes the kernels address: one Fourier slice below 2^31 entries (per-slice
// row, column and tile indices are 32-bit; every offset across slices or
// into the whole tensor is 64-bit), the tensor below 2^36 entries (256 GiB
// in FP32, more than one device holds with its spectrum), for
// 1 <= n3 <= 4096, without overflowing on the way.
bool small_volume(int64_t n1, int64_t n2, int64_t n3) {
  const int64_t lim = (int64_t)1 << 31;
  if (n1 >= lim || n2 >= lim) return false;
  const int64_t a = n1 * n2;  // < 2^62
  return a < lim && a * n3 < ((int64_t)1 << 36);
}

// Alg. mp: per Fourier slice the Gram on the short side (A_f^H A_f when
// n1 >= n2, else A_f A_f^H; r = min(n1, n2)), all its eigenpairs, the
// sigma^-2-weighted projector Wg and the product with A_f^H.
int make_plan_tpinv(int64_t n1, int64_t n2, int64_t n3, int prec, Plan* p) {
  if (prec != TSVD_PREC_F64 && prec != TSVD_PREC_F32)
    return fail(TSVD_EINVAL, "the pseudoinverse takes TSVD_PREC_F64 or TSVD_PREC_F32");
  const int64_t r = std::min(n1, n2), K = std::max(n1, n2);
  if (r > 1024) return fail(TSVD_EINVAL, "min(n1, n2) must be <= 1024");
  if (n3 > 4096) return fail(TSVD_EINVAL, "n3 must be <= 4096");
  if (!small_volume(n1, n2, n3)) return fail(TSVD_EINVAL, "n1 * n2 must be < 2^31 and n1 * n2 * n3 < 2^36");
  *p = Plan{};
  p->n1 = n1;
  p->n2 = n2;
  p->n3 = n3;
  p->k = r;
  p->b = r;
  p->q = 0;
  p->m = r;
  p->F = n3 / 2 + 1;
  p->prec = prec;
  p->dt = prec == TSVD_PREC_F64 ? DT_F64 : DT_F32;
  p->cs = prec == TSVD_PREC_F64 ? 16 : 8;
  p->tensor_op = true;
  p->kmode = KM_F32;
  const int64_t F = p->F, tm = (r + 63) / 64;
  p->nsplit_g = split_for(K, tm * tm, F, &p->kchunk_g);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  const size_t cs = p->cs, rr = (size_t)r * r;
  p->o_info = take(256);
  p->o_abar = take((size_t)F * n1 * n2 * cs);
  size_t part = (size_t)p->nsplit_g * F * rr * 16;
  if (p->dt == DT_F32 && n1 >= n2) part = ogemm_tn_part_bytes((int)r, (int)n1, (int)r, (int)F);
  p->o_part = take(part);
  p->o_lam = take((size_t)F * r * 8);
  p->o_wd = take((size_t)F * rr * 16);
  p->o_wds = take((size_t)F * rr * 16);
  p->o_rinv = take((size_t)F * rr * 16);
  p->o_heig = take((size_t)F * heig_scratch_bytes((int)r, (int)r));
  p->o_xp = take((size_t)F * n2 * n1 * cs);
  p->total = o;
  return TSVD_OK;
}

int make_plan(int64_t n1, int64_t n2, int64_t n3, int64_t k, int64_t b, int64_t q, int prec, int op, Plan* p) {
  if (n1 < 1 || n2 < 1 || n3 < 1) return fail(TSVD_EINVAL, "n1, n2, n3 must be >= 1");
  if (op == TSVD_OP_TPINV) return make_plan_tpinv(n1, n2, n3, prec, p);
  // completion (Example 3): the approximation plan of the chosen method plus
  // the iterate buffers
  const bool completion = op == TSVD_OP_COMPLETE_RBK || op == TSVD_OP_COMPLETE_POWER;
  if (completion) op = op == TSVD_OP_COMPLETE_RBK ? TSVD_OP_APPROX : TSVD_OP_POWER_APPROX;
  // literal Krylov powers: the buffers of the approximation
  if (op == TSVD_OP_RBK_LITERAL) op = TSVD_OP_APPROX;
  const bool tensor_op = op == TSVD_OP_TQR;
  if (tensor_op) {
    // Alg. TQR: the QR of every slice A_f itself (r = min(n1, n2) columns);
    // k, b and q are not used
    if (prec != TSVD_PREC_F64 && prec != TSVD_PREC_F32)
      return fail(TSVD_EINVAL, "T-QR takes TSVD_PREC_F64 or TSVD_PREC_F32");
    if (std::min(n1, n2) > 1024) return fail(TSVD_EINVAL, "min(n1, n2) must be <= 1024");
    // the r = min(n1, n2) columns are orthonormalised in equal panels of at
    // most 128 columns (block Gram-Schmidt twice against the earlier panels,
    // shifted CholeskyQR per panel, as for the Krylov blocks)
    const int64_t r = std::min(n1, n2);
    int64_t npan = (r + 127) / 128;
    while (r % npan) ++npan;
    k = 1;
    b = r / npan;
    q = npan - 1;
  }
  if (b < 1 || q < 0) return fail(TSVD_EINVAL, "need b >= 1 and q >= 0");
  const bool power = op == TSVD_OP_POWER || op == TSVD_OP_POWER_APPROX;
  const bool ritz = op == TSVD_OP_RBK_RITZ;
  const bool abwd = op == TSVD_OP_APPROX_BWD;
  if (op == TSVD_OP_RBK || op == TSVD_OP_APPROX || power || ritz || abwd) {
    if (k < 1 || k > b) return fail(TSVD_EINVAL, "need 1 <= k <= b");
  } else {
    k = 1;
  }
  if (power && q > 4096) return fail(TSVD_EINVAL, "q must be <= 4096");
  // (b and q bounded before the product: m only matters up to 1024)
  const int64_t m = power ? b : ((b > 1024 || q > 1023) ? (int64_t)1025 : b * (q + 1));
  if (power) {
    if (m > std::min(n1, n2)) return fail(TSVD_EINVAL, "need b <= min(n1, n2)");
    if (m > 1024) return fail(TSVD_EINVAL, "b must be <= 1024");
  } else {
    if (m > std::min(n1, n2)) return fail(TSVD_EINVAL, "need m = b (q + 1) <= min(n1, n2)");
    if (m > 1024) return fail(TSVD_EINVAL, "m = b (q + 1) must be <= 1024");
  }
  if (n3 > 4096) return fail(TSVD_EINVAL, "n3 must be <= 4096");
  if (!small_volume(n1, n2, n3)) return fail(TSVD_EINVAL, "n1 * n2 must be < 2^31 and n1 * n2 * n3 < 2^36");
  if (prec != TSVD_PREC_F64 && prec != TSVD_PREC_F32 && prec != TSVD_PREC_BF16 && prec != TSVD_PREC_BF16X3)
    return fail(TSVD_EINVAL, "unknown precision mode");
  if (op < TSVD_OP_RBK || op > TSVD_OP_APPROX_BWD || op == TSVD_OP_COMPLETE_RBK || op == TSVD_OP_COMPLETE_POWER ||
      op == TSVD_OP_RBK_LITERAL)
    return fail(TSVD_EINVAL, "unsupported operation");
  p->power = power;
  p->tensor_op = tensor_op;
  p->n1 = n1;
  p->n2 = n2;
  p->n3 = n3;
  p->k = k;
  p->b = b;
  p->q = q;
  p->m = m;
  p->F = n3 / 2 + 1;
  p->prec = prec;
  p->dt = prec == TSVD_PREC_F64 ? DT_F64 : DT_F32;
  p->cs = prec == TSVD_PREC_F64 ? 16 : 8;
  const int64_t F = p->F;
  const int64_t tb = (b + 63) / 64;
  p->nsplit_blk = split_for(n1, tb * ((m + 63) / 64), F, &p->kchunk_blk);
  const int64_t tm = (m + 63) / 64;
  p->nsplit_g = split_for(n2, tm * tm, F, &p->kchunk_g);
  p->nsplit_t = split_for(n2, tb * tb, F, &p->kchunk_t);
  p->nsplit_r = split_for(n1, ((m + 63) / 64) * ((n2 + 63) / 64), F, &p->kchunk_r);
  p->kmode = prec == TSVD_PREC_BF16 ? KM_BF16 : (prec == TSVD_PREC_BF16X3 ? KM_BF16X3 : KM_F32);
  // the split form of A_f where nothing but the Krylov products reads it (not
  // the projection and its adjoint) and the transform has the split epilogue
  p->asplit = p->kmode == KM_BF16X3 && p->dt == DT_F32 && fft_reg_supported((int)n3, DT_F32) &&
              (op == TSVD_OP_RBK || op == TSVD_OP_APPROX || op == TSVD_OP_POWER || op == TSVD_OP_POWER_APPROX ||
               ritz);
  int kc_unused;
  if (p->kmode != KM_BF16) {
    p->ks_ax = p->dt == DT_F32 ? kgemm_split((int)n1, (int)n2, (int)b, (int)F, &kc_unused) : 1;
    p->ks_ahy = p->dt == DT_F32 ? kgemm_split((int)n2, (int)n1, (int)b, (int)F, &kc_unused) : 1;
  } else {
    p->ks_ax = kgemm_bf16_split((int)n1, (int)n2, (int)b, (int)F);
    p->ks_ahy = kgemm_bf16_split((int)n2, (int)n1, (int)b, (int)F);
  }

  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = align256(o + bytes);
    return r;
  };
  const size_t cs = p->cs;
  p->o_info = take(256);
  p->o_omsp = take(tensor_op ? 0 : (size_t)n2 * b * n3 * (p->dt == DT_F64 ? 8 : 4));
  p->o_abar = take((size_t)F * n1 * n2 * cs);
  p->o_obar = take(tensor_op ? 0 : (size_t)F * n2 * b * cs);
  p->o_q = take((size_t)F * n1 * m * cs);
  p->o_t = take(tensor_op ? 0 : (size_t)F * n2 * m * cs);
  // block scratch: n1-row Krylov blocks; Alg. 1 also orthonormalises the
  // n2-row half-step iterates A_f^H Q
  const int64_t srows = power ? std::max(n1, n2) : n1;
  p->o_s0 = take((size_t)F * srows * b * cs);
  p->o_s1 = take((size_t)F * srows * b * cs);
  size_t part = (size_t)p->nsplit_blk * F * m * b * 16;
  part = std::max(part, (size_t)p->nsplit_g * F * m * m * 16);
  if (power) part = std::max(part, (size_t)p->nsplit_t * F * b * b * 16);
  if (tensor_op) part = std::max(part, (size_t)p->nsplit_r * F * m * n2 * 16);
  if (p->dt == DT_F32) {
    // FP64-arithmetic products on FP32 blocks: block Grams (b x b), projections
    // (i b x b and b x i b), G = T^H T (m x m)
    part = ogemm_tn_part_bytes((int)m, (int)n2, (int)m, (int)F);
    // block Grams and projections against the i b earlier columns (Alg. 2
    // only; Alg. 1 orthonormalises each iterate on its own)
    for (int64_t i = 1; i <= (power ? 1 : std::max<int64_t>(q, 1)); ++i) {
      part = std::max(part, ogemm_tn_part_bytes((int)(i * b), (int)n1, (int)b, (int)F));
      part = std::max(part, ogemm_tn_part_bytes((int)b, (int)n1, (int)(i * b), (int)F));
    }
    if (power) {
      part = std::max(part, ogemm_tn_part_bytes((int)b, (int)n2, (int)b, (int)F));
    }
    if (tensor_op) {
      part = std::max(part, ogemm_tn_part_bytes((int)m, (int)n1, (int)n2, (int)F));
    }
    if (ritz) part = std::max(part, ogemm_tn_part_bytes((int)b, (int)n2, (int)b, (int)F));
    // the FP32 first projection pass of the stabilised recursion
    if (!power && !tensor_op)
      for (int64_t i = 1; i <= q; ++i) part = std::max(part, proj32_layout(i * b, n1, b, F, nullptr, nullptr));
  }
  if (ritz) part = std::max(part, (size_t)p->nsplit_t * F * b * b * 16);
  p->o_part = take(part);
  p->o_rinv = take((size_t)F * b * b * 16);
  p->o_chol = take(chol_uses_lds(b) ? 0 : (size_t)F * b * (b + 1) / 2 * 16);
  const bool need_svd = (op == TSVD_OP_RBK || op == TSVD_OP_APPROX || power || ritz);
  const int64_t ks = ritz ? b : k;  // columns of the small SVD's buffers
  p->o_lam = take(need_svd ? (size_t)F * ks * 8 : 0);
  p->o_sig = take(need_svd ? (size_t)F * ks * 8 : 0);
  p->o_wd = take(need_svd ? (size_t)F * m * ks * 16 : 0);
  p->o_wds = take(need_svd ? (size_t)F * m * ks * 16 : 0);
  p->o_heig = take(need_svd || abwd ? (size_t)F * heig_scratch_bytes((int)m, (int)(abwd ? m : ks)) : 0);
  p->o_canon = take(need_svd ? canon_scratch_bytes(n1, (int)ks, (int)F) : 0);
  const bool pass2 = need_svd && p->dt == DT_F64;
  p->o_lam1 = take(pass2 ? (size_t)F * ks * 8 : 0);
  p->o_w1 = take(pass2 ? (size_t)F * m * ks * 16 : 0);
  p->o_w1m = take(pass2 ? (size_t)F * m * ks * 16 : 0);
  p->o_p = take(pass2 ? (size_t)F * n2 * ks * 16 : 0);
  p->o_t1 = take(pass2 ? (size_t)F * n2 * m * 16 : 0);
  p->o_lam2 = take(pass2 ? (size_t)F * ks * 8 : 0);
  p->o_w2 = take(pass2 ? (size_t)F * m * ks * 16 : 0);
  p->o_rk = take(pass2 ? (size_t)F * ks * ks * 16 : 0);
  p->o_split = take(pass2 ? (size_t)F * 4 : 0);
  p->o_uf = take(need_svd ? (size_t)F * n1 * ks * cs : 0);
  p->o_vf = take(need_svd ? (size_t)F * n2 * ks * cs : 0);
  p->o_scx = take(need_svd ? (size_t)F * ks * cs : 0);
  const size_t es0 = p->dt == DT_F64 ? 8 : 4;
  p->o_vr = take(ritz ? (size_t)n2 * b * n3 * es0 : 0);
  p->o_sr = take(ritz ? (size_t)b * n3 * es0 : 0);
  p->o_wall = take(abwd ? (size_t)F * m * m * 16 : 0);
  p->o_lall = take(abwd ? (size_t)F * m * 8 : 0);
  p->o_mm0 = take(abwd ? (size_t)F * m * m * 16 : 0);
  p->o_mm1 = take(abwd ? (size_t)F * m * m * 16 : 0);
  p->o_mm2 = take(abwd ? (size_t)F * m * m * 16 : 0);
  p->o_mm3 = take(abwd ? (size_t)F * m * m * 16 : 0);
  p->o_u2b = take(abwd ? (size_t)F * n2 * m * cs : 0);
  p->o_tp = take(abwd ? (size_t)F * n2 * m * cs : 0);
  p->o_us = take(op == TSVD_OP_APPROX || op == TSVD_OP_POWER_APPROX ? (size_t)F * n1 * k * cs : 0);
  p->o_rout = take(tensor_op ? (size_t)F * m * n2 * cs : 0);
  p->o_xp = take(0);
  const bool bwd = op == TSVD_OP_PROJ_BWD || abwd;
  p->o_gbar = take(bwd ? (size_t)F * n1 * n2 * cs : 0);
  p->o_dbar = take(bwd ? (size_t)F * n1 * n2 * cs : 0);
  p->o_wraw = take(bwd ? (size_t)F * n1 * m * cs : 0);
  p->o_qbar = take(bwd ? (size_t)F * n1 * m * cs : 0);
  p->o_u2 = take(bwd ? (size_t)F * n2 * m * cs : 0);
  p->o_zbar = take(bwd ? (size_t)F * n1 * b * cs : 0);
  p->o_wbar = take(bwd ? (size_t)F * n1 * b * cs : 0);
  p->o_tbar = take(bwd ? (size_t)F * n2 * b * cs : 0);
  {
    size_t kp = std::max(p->ks_ax > 1 ? (size_t)p->ks_ax * F * n1 * b * 8 : 0,
                         p->ks_ahy > 1 ? (size_t)p->ks_ahy * F * n2 * b * 8 : 0);
    if (p->dt == DT_F32 && p->kmode != KM_BF16) {
      // unsplit products split their last, partial round of tiles along K
      if (p->ks_ax == 1) kp = std::max(kp, kgemm_part_bytes((int)n1, (int)n2, (int)b, (int)F, 1));
      if (p->ks_ahy == 1) kp = std::max(kp, kgemm_part_bytes((int)n2, (int)n1, (int)b, (int)F, 1));
    }
    if (tensor_op) kp = 0;
    p->kpart_bytes = kp;
    p->o_kpart = take(kp);
    const bool bfm = p->dt == DT_F32 && p->kmode == KM_BF16;
    p->o_kpack = take(bfm ? std::max(kgemm_bf16_pack_bytes(p->kmode, (int)n2, (int)b, (int)F),
                                     kgemm_bf16_pack_bytes(p->kmode, (int)n1, (int)b, (int)F))
                          : 0);
  }
  const size_t es = p->dt == DT_F64 ? 8 : 4;
  p->o_cbuf = take(completion ? (size_t)n1 * n2 * n3 * es : 0);
  p->o_xbuf = take(completion ? (size_t)n1 * n2 * n3 * es : 0);
  p->o_uo = take(completion ? (size_t)n1 * k * n3 * es : 0);
  p->o_so = take(completion ? (size_t)k * n3 * es : 0);
  p->o_vo = take(completion ? (size_t)n2 * k * n3 * es : 0);
  p->total = o;
  return TSVD_OK;
}

struct Ctx {
  const Plan& p;
  unsigned char* ws;
  hipStream_t s;
  template <typename T = void>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(ws + off);
  }
  int* info() const { return at<int>(p.o_info); }
};

#define HIPCHK(x)                                                            \
  do {                                                                       \
    hipError_t e_ = (x);                                                     \
    if (e_ != hipSuccess) {                                                  \
      char b_[256];                                                          \
      snprintf(b_, sizeof b_, "HIP error %d (%s) at %s:%d", (int)e_,         \
               hipGetErrorString(e_), __FILE__, __LINE__);                   \
      return fail(TSVD_EHIP, b_);                                            \
    }                                                                        \
  } while (0)

// ---- opt-in per-kernel-class event timer (tsvd_diag_timing*) -------------
enum KClass { K_FFT_A = 0, K_FFT_OMEGA, K_GEMM_KRYLOV, K_GEMM_ORTH, K_CHOL, K_HEIG_TRI, K_GEMM_LIFT, K_FFT_INV, K_MISC,
              K_HEIG_BISECT, K_HEIG_INVIT, K_HEIG_BACKXF, K_NCLASS };
struct Timer {
  std::mutex mu;
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  double ms[K_NCLASS] = {};
  long long count[K_NCLASS] = {};
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};
Timer g_timer;

struct Timed {
  int cls;
  hipStream_t s;
  hipEvent_t a = nullptr;
  Timed(int c, hipStream_t st) : cls(c), s(st) {
    if (!g_timer.on) return;
    std::lock_guard<std::mutex> l(g_timer.mu);
    a = g_timer.get();
    if (a) (void)hipEventRecord(a, s);
  }
  ~Timed() {
    if (!a) return;
    std::lock_guard<std::mutex> l(g_timer.mu);
    hipEvent_t b = g_timer.get();
    if (!b) return;
    (void)hipEventRecord(b, s);
    g_timer.pending.push_back({cls, {a, b}});
  }
};

GemmDesc gd() {
  GemmDesc d{};
  d.b_nsum = 1;
  d.nsplit = 1;
  d.alpha = 1.0;
  d.beta = 0.0;
  return d;
}

// part (M x N per slice, FP64) = X^H Y over K rows, X (K x M, ld lx) and Y
// (K x N, ld ly) in the working dtype.  *nsum receives the number of partial
// results (spaced F * M * N) whose sum is the product.
int inner_products(const Ctx& c, const void* X, int64_t lx, int M, const void* Y, int64_t ly, int N, int64_t K,
                   int64_t strideX, int64_t strideY, int nsplit, int kchunk, double* part, int* nsum,
                   int cls = K_GEMM_ORTH, bool upper = false) {
  const Plan& p = c.p;
  if (p.dt == DT_F32) {
    Timed tm_(cls, c.s);
    HIPCHK(ogemm_tn(static_cast<const float*>(X), lx, strideX, static_cast<const float*>(Y), ly, strideY, part, M, N,
                    (int)K, (int)p.F, c.s, upper));
    *nsum = 1;
    return TSVD_OK;
  }
  GemmDesc d = gd();
  d.A = X;
  d.lda = lx;
  d.strideA = strideX;
  d.ta = p.dt;
  d.a_conj = true;
  d.B = Y;
  d.ldb = ly;
  d.strideB = strideY;
  d.tb = p.dt;
  d.C = part;
  d.ldc = N;
  d.strideC = (int64_t)M * N;
  d.tc = DT_F64;
  d.M = M;
  d.N = N;
  d.K = (int)K;
  d.batch = (int)p.F;
  d.nsplit = nsplit;
  d.kchunk = kchunk;
  d.c_split_stride = p.F * M * N;
  d.compute = DT_F64;
  {
    Timed tm_(cls, c.s);
    HIPCHK(zgemm(d, c.s));
  }
  *nsum = nsplit;
  return TSVD_OK;
}

// dst (rows x b, ld ldd) = src (rows x b, ld lds) * Rinv   (FP64 arithmetic)
int apply_rinv(const Ctx& c, const void* src, int64_t lds, void* dst, int64_t ldd, int64_t rows) {
  const Plan& p = c.p;
  if (p.dt == DT_F32) {
    Timed tm_(K_GEMM_ORTH, c.s);
    HIPCHK(ogemm_nn(static_cast<const float*>(src), lds, rows * lds, c.at<double>(p.o_rinv), p.b, p.b * p.b, 1, 0,
                    static_cast<float*>(dst), ldd, rows * ldd, (int)rows, (int)p.b, (int)p.b, (int)p.F, 1.0, 0.0,
                    c.s, true));
    return TSVD_OK;
  }
  GemmDesc d = gd();
  d.A = src;
  d.lda = lds;
  d.strideA = rows * lds;
  d.ta = p.dt;
  d.B = c.at(p.o_rinv);
  d.ldb = p.b;
  d.strideB = p.b * p.b;
  d.tb = DT_F64;
  d.C = dst;
  d.ldc = ldd;
  d.strideC = rows * ldd;
  d.tc = p.dt;
  d.M = (int)rows;
  d.N = (int)p.b;
  d.K = (int)p.b;
  d.batch = (int)p.F;
  d.compute = DT_F64;
  {
    Timed tm_(K_GEMM_ORTH, c.s);
    HIPCHK(zgemm(d, c.s));
  }
  return TSVD_OK;
}

// One CholeskyQR pass over a rows x b block (rows = n1 for the Krylov blocks,
// n2 for Alg. 1's half-step iterates): dst = src R^{-1}, G = src^H src (+ shift).
int cholqr_pass(const Ctx& c, const void* src, int64_t lds, void* dst, int64_t ldd, bool shifted, int64_t rows) {
  const Plan& p = c.p;
  double* part = c.at<double>(p.o_part);
  int nsum = 1;
  // the Gram is Hermitian: on the FP32 path (b <= 128) only its upper triangle is formed
  const bool upper = p.dt == DT_F32 && chol_blocked_ok((int)p.b);
  const bool long_rows = rows == p.n1;
  int r = inner_products(c, src, lds, (int)p.b, src, lds, (int)p.b, rows, rows * lds, rows * lds,
                         long_rows ? p.nsplit_blk : p.nsplit_t, long_rows ? p.kchunk_blk : p.kchunk_t, part, &nsum,
                         K_GEMM_ORTH, upper);
  if (r) return r;
  const double u = 1.1102230246251565e-16;
  const double shift = shifted ? 11.0 * ((double)rows * p.b + (double)p.b * (p.b + 1)) * u : 0.0;
  {
    Timed tm_(K_CHOL, c.s);
    HIPCHK(chol_inv_ex(part, nsum, p.F * p.b * p.b, c.at<double>(p.o_rinv), c.at(p.o_chol), (int)p.b, (int)p.F,
                       shift, c.info(), c.s, upper ? 2 : 0));
  }
  return apply_rinv(c, src, lds, dst, ldd, rows);
}

// W (n1 x b, ld b) -= Q_<i (Q_<i^H W), Q_<i = first i*b columns of Q.
int project_out(const Ctx& c, void* W, int i) {
  const Plan& p = c.p;
  if (i == 0) return TSVD_OK;
  const int ib = (int)(i * p.b);
  double* part = c.at<double>(p.o_part);
  void* Q = c.at(p.o_q);
  int nsum = 1;
  int r = inner_products(c, Q, p.m, ib, W, p.b, (int)p.b, p.n1, p.n1 * p.m, p.n1 * p.b, p.nsplit_blk, p.kchunk_blk,
                         part, &nsum);
  if (r) return r;
  if (p.dt == DT_F32) {
    Timed tm_(K_GEMM_ORTH, c.s);
    HIPCHK(ogemm_nn(static_cast<const float*>(Q), p.m, p.n1 * p.m, part, p.b, (int64_t)ib * p.b, nsum,
                    p.F * ib * p.b, static_cast<float*>(W), p.b, p.n1 * p.b, (int)p.n1, (int)p.b, ib, (int)p.F, -1.0,
                    1.0, c.s));
    return TSVD_OK;
  }
  GemmDesc d = gd();
  d.A = Q;
  d.lda = p.m;
  d.strideA = p.n1 * p.m;
  d.ta = p.dt;
  d.B = part;
  d.ldb = p.b;
  d.strideB = (int64_t)ib * p.b;
  d.tb = DT_F64;
  d.b_nsum = nsum;
  d.b_sum_stride = p.F * ib * p.b;
  d.C = W;
  d.ldc = p.b;
  d.strideC = p.n1 * p.b;
  d.tc = p.dt;
  d.M = (int)p.n1;
  d.N = (int)p.b;
  d.K = ib;
  d.batch = (int)p.F;
  d.alpha = -1.0;
  d.beta = 1.0;
  d.compute = DT_F64;
  {
    Timed tm_(K_GEMM_ORTH, c.s);
    HIPCHK(zgemm(d, c.s));
  }
  return TSVD_OK;
}

// Bytes of o_part that project_out_f32 uses against ib earlier columns: the
// K-split partials of the coefficient product, then the coefficients.
size_t proj32_layout(int64_t ib, int64_t n1, int64_t b, int64_t F, int* nsplit, size_t* coef_off) {
  const int ns = kgemm_split_balanced((int)ib, (int)n1, (int)b, (int)F);
  const size_t off = align256(kgemm_part_bytes((int)ib, (int)n1, (int)b, (int)F, ns));
  if (nsplit) *nsplit = ns;
  if (coef_off) *coef_off = off;
  return off + (size_t)F * ib * b * 8;
}

// First of the two Gram-Schmidt passes of the Krylov recursion on FP32
// blocks, in FP32 arithmetic on the Krylov-product kernel:
// W -= Q_<i (Q_<i^H W), coefficients rounded to FP32.  Its rounding error,
// of the order of the rounding of the block's own FP32 Krylov product, is an
// FP32-level perturbation of the block; the second pass (FP64 arithmetic)
// removes whatever of it lies in the span of Q_<i, so the orthogonality of
// the basis is that of the FP64 pass.
int project_out_f32(const Ctx& c, void* W, int i) {
  const Plan& p = c.p;
  if (i == 0) return TSVD_OK;
  const int64_t ib = (int64_t)i * p.b;
  int ns = 1;
  size_t coef_off = 0;
  proj32_layout(ib, p.n1, p.b, p.F, &ns, &coef_off);
  unsigned char* base = c.at<unsigned char>(p.o_part);
  void* coef = base + coef_off;
  void* Q = c.at(p.o_q);
  Timed tm_(K_GEMM_ORTH, c.s);
  KGemmDesc k{};
  k.A = Q;
  k.lda = p.m;
  k.strideA = p.n1 * p.m;
  k.rows = (int)p.n1;
  k.cols = (int)ib;
  k.herm = true;
  k.X = W;
  k.ldx = p.b;
  k.strideX = p.n1 * p.b;
  k.C = coef;
  k.ldc = p.b;
  k.strideC = ib * p.b;
  k.N = (int)p.b;
  k.batch = (int)p.F;
  k.mode = KM_F32;
  k.nsplit = ns;
  k.part = base;
  k.part_bytes = coef_off;
  HIPCHK(kgemm(k, c.s));
  KGemmDesc u{};
  u.A = Q;
  u.lda = p.m;
  u.strideA = p.n1 * p.m;
  u.rows = (int)p.n1;
  u.cols = (int)ib;
  u.herm = false;
  u.X = coef;
  u.ldx = p.b;
  u.strideX = ib * p.b;
  u.C = W;
  u.ldc = p.b;
  u.strideC = p.n1 * p.b;
  u.N = (int)p.b;
  u.batch = (int)p.F;
  u.mode = KM_F32;
  u.nsplit = 1;
  u.sub = 1;
  HIPCHK(kgemm(u, c.s));
  return TSVD_OK;
}

// Shifted CholeskyQR3 of a rows x b block whose first pass has been done
// (result in S1): dst = orthonormal basis of its range.
int cholqr_finish(const Ctx& c, int64_t rows, void* dst, int64_t ldd) {
  const Plan& p = c.p;
  void* S0 = c.at(p.o_s0);
  void* S1 = c.at(p.o_s1);
  int r;
  if (p.dt == DT_F64) {
    // FP64 blocks can be far more ill-conditioned than FP32 ones, whose
    // rounding noise bounds the condition number near 1e8: a slice spectrum
    // that reaches the FP64 rounding level within one block gives
    // kappa >= 1/u.  One shifted pass then leaves kappa above u^{-1/2}
    // (rounding in W R^{-1}); two more bring it down before the unshifted
    // CholeskyQR2.
    if ((r = cholqr_pass(c, S1, p.b, S0, p.b, true, rows))) return r;
    if ((r = cholqr_pass(c, S0, p.b, S1, p.b, true, rows))) return r;
    if ((r = cholqr_pass(c, S1, p.b, S0, p.b, false, rows))) return r;
    return cholqr_pass(c, S0, p.b, dst, ldd, false, rows);
  }
  // FP32 storage with FP64 Grams.  The shifted pass maps sigma_j(W) to
  // sigma_j / sqrt(sigma_j^2 + s), so kappa(X1) <= sqrt(alpha) kappa(W) with
  // alpha = s / ||W||^2 <= 11 (rows b + b (b + 1)) 2^-53 b, and an FP32 block
  // has kappa(W) below about 1e8 (its rounding noise).  One unshifted pass
  // then leaves an FP64 orthogonality error of about 2^-53 kappa(X1)^2; when
  // that bound stays within 16 FP32 roundings (2^-20), below the FP32 rounding
  // of the block itself in the 2-norm, a second unshifted pass cannot improve
  // the stored result and is left out (rows * b up to about 6e6 at b = 110).
  const double u64 = 0x1p-53;
  const double alpha_max = 11.0 * ((double)rows * p.b + (double)p.b * (p.b + 1)) * u64 * (double)p.b;
  if (alpha_max * u64 * 1e16 <= 0x1p-20) return cholqr_pass(c, S1, p.b, dst, ldd, false, rows);
  if ((r = cholqr_pass(c, S1, p.b, S0, p.b, false, rows))) return r;
  return cholqr_pass(c, S0, p.b, dst, ldd, false, rows);
}

// Orthonormalise the block in S0 against Q_<i and write it to Q(:, i b : (i+1) b).
// first32: the first projection pass in FP32 arithmetic (FP32 blocks of the
// stabilised recursion, whose blocks are orthonormalised one by one).
int orth_block(const Ctx& c, int i, bool first32 = false) {
  const Plan& p = c.p;
  void* S0 = c.at(p.o_s0);
  void* S1 = c.at(p.o_s1);
  void* dst = c.at<unsigned char>(p.o_q) + (size_t)i * p.b * p.cs;
  int r;
  if ((r = (first32 && p.dt == DT_F32) ? project_out_f32(c, S0, i) : project_out(c, S0, i))) return r;
  if ((r = cholqr_pass(c, S0, p.b, S1, p.b, true, p.n1))) return r;
  if ((r = project_out(c, S1, i))) return r;
  return cholqr_finish(c, p.n1, dst, p.m);
}

// Orthonormalise an n2 x b block in place (ld b): Alg. 1's half-step iterate.
int orth_rows_n2(const Ctx& c, void* X) {
  const Plan& p = c.p;
  int r;
  if ((r = cholqr_pass(c, X, p.b, c.at(p.o_s1), p.b, true, p.n2))) return r;
  return cholqr_finish(c, p.n2, X, p.b);
}

// Out (M x N, ld ldc) = A_f (n1 x n2) * X (n2 x N, ld ldx): the big products.
int big_AX(const Ctx& c, const void* X, int64_t ldx, int64_t strideX, void* Out, int64_t ldo, int64_t strideO, int N) {
  const Plan& p = c.p;
  if (p.dt == DT_F32) {
    KGemmDesc k{};
    k.A = c.at(p.o_abar);
    k.lda = p.n2;
    k.strideA = p.n1 * p.n2;
    k.rows = (int)p.n1;
    k.cols = (int)p.n2;
    k.herm = false;
    k.X = X;
    k.ldx = ldx;
    k.strideX = strideX;
    k.C = Out;
    k.ldc = ldo;
    k.strideC = strideO;
    k.N = N;
    k.batch = (int)p.F;
    k.mode = p.asplit ? KM_BF16X3_SPLIT : p.kmode;
    k.nsplit = N == p.b ? p.ks_ax : 1;
    k.part = c.at(p.o_kpart);
    k.part_bytes = p.kpart_bytes;
    Timed tm_(K_GEMM_KRYLOV, c.s);
    if (p.kmode != KM_BF16 || N != p.b)
      HIPCHK(kgemm(k, c.s));
    else
      HIPCHK(kgemm_bf16(k, c.at(p.o_kpack), c.s));
    return TSVD_OK;
  }
  GemmDesc d = gd();
  d.A = c.at(p.o_abar);
  d.lda = p.n2;
  d.strideA = p.n1 * p.n2;
  d.ta = p.dt;
  d.B = X;
  d.ldb = ldx;
  d.strideB = strideX;
  d.tb = p.dt;
  d.C = Out;
  d.ldc = ldo;
  d.strideC = strideO;
  d.tc = p.dt;
  d.M = (int)p.n1;
  d.N = N;
  d.K = (int)p.n2;
  d.batch = (int)p.F;
  d.compute = p.dt;
  {
    Timed tm_(K_GEMM_KRYLOV, c.s);
    HIPCHK(zgemm(d, c.s));
  }
  return TSVD_OK;
}

// Out (n2 x N) = A_f^H * Y (n1 x N)
int big_AhY(const Ctx& c, const void* Y, int64_t ldy, int64_t strideY, void* Out, int64_t ldo, int64_t strideO,
            int N) {
  const Plan& p = c.p;
  if (p.dt == DT_F32) {
    KGemmDesc k{};
    k.A = c.at(p.o_abar);
    k.lda = p.n2;
    k.strideA = p.n1 * p.n2;
    k.rows = (int)p.n1;
    k.cols = (int)p.n2;
    k.herm = true;
    k.X = Y;
    k.ldx = ldy;
    k.strideX = strideY;
    k.C = Out;
    k.ldc = ldo;
    k.strideC = strideO;
    k.N = N;
    k.batch = (int)p.F;
    k.mode = p.asplit ? KM_BF16X3_SPLIT : p.kmode;
    k.nsplit = N == p.b ? p.ks_ahy : 1;
    k.part = c.at(p.o_kpart);
    k.part_bytes = p.kpart_bytes;
    Timed tm_(K_GEMM_KRYLOV, c.s);
    if (p.kmode != KM_BF16 || N != p.b)
      HIPCHK(kgemm(k, c.s));
    else
      HIPCHK(kgemm_bf16(k, c.at(p.o_kpack), c.s));
    return TSVD_OK;
  }
  GemmDesc d = gd();
  d.A = c.at(p.o_abar);
  d.lda = p.n2;
  d.strideA = p.n1 * p.n2;
  d.ta = p.dt;
  d.a_conj = true;
  d.B = Y;
  d.ldb = ldy;
  d.strideB = strideY;
  d.tb = p.dt;
  d.C = Out;
  d.ldc = ldo;
  d.strideC = strideO;
  d.tc = p.dt;
  d.M = (int)p.n2;
  d.N = N;
  d.K = (int)p.n1;
  d.batch = (int)p.F;
  d.compute = p.dt;
  {
    Timed tm_(K_GEMM_KRYLOV, c.s);
    HIPCHK(zgemm(d, c.s));
  }
  return TSVD_OK;
}

// Everything up to Q and T = C^H.
// Copy the raw block in S0 (n1 x b) to column block i of Wraw (n1 x m).
int save_raw(const Ctx& c, int i) {
  const Plan& p = c.p;
  HIPCHK(hipMemcpy2DAsync(c.at<unsigned char>(p.o_wraw) + (size_t)i * p.b * p.cs, (size_t)p.m * p.cs, c.at(p.o_s0),
                          (size_t)p.b * p.cs, (size_t)p.b * p.cs, (size_t)(p.F * p.n1), hipMemcpyDeviceToDevice, c.s));
  return TSVD_OK;
}

int krylov(const Ctx& c, const void* A, const void* Omega, bool keep_raw = false) {
  const Plan& p = c.p;
  const DType dt = p.dt;
  {
    Timed tm_(K_MISC, c.s);
    HIPCHK(zero_info(c.info(), c.s));
  }
  {
    Timed tm_(K_FFT_A, c.s);
    if (p.asplit)
      HIPCHK(fft_r2c_split(A, c.at(p.o_abar), p.n1 * p.n2, (int)p.n3, c.s));
    else
      HIPCHK(fft_r2c(A, c.at(p.o_abar), p.n1 * p.n2, (int)p.n3, dt, c.s));
  }
  {
    Timed tm_(K_FFT_OMEGA, c.s);
    HIPCHK(fft_r2c(Omega, c.at(p.o_obar), p.n2 * p.b, (int)p.n3, dt, c.s));
  }
  unsigned char* Q = c.at<unsigned char>(p.o_q);
  unsigned char* T = c.at<unsigned char>(p.o_t);
  int r;
  if ((r = big_AX(c, c.at(p.o_obar), p.b, p.n2 * p.b, c.at(p.o_s0), p.b, p.n1 * p.b, (int)p.b))) return r;
  if (p.power) {
    // Alg. 1, q power iterations with an orthonormalisation after every
    // product: T <- orth(A_f^H Q), Q <- orth(A_f T); the basis is the last
    // iterate's (same range as (A A^H)^q A Om in exact arithmetic, without
    // squaring the condition number at each step)
    if ((r = orth_block(c, 0))) return r;
    for (int i = 1; i <= p.q; ++i) {
      if ((r = big_AhY(c, Q, p.m, p.n1 * p.m, T, p.m, p.n2 * p.m, (int)p.b))) return r;
      if ((r = orth_rows_n2(c, T))) return r;
      if ((r = big_AX(c, T, p.m, p.n2 * p.m, c.at(p.o_s0), p.b, p.n1 * p.b, (int)p.b))) return r;
      if ((r = orth_block(c, 0))) return r;
    }
    return big_AhY(c, Q, p.m, p.n1 * p.m, T, p.m, p.n2 * p.m, (int)p.b);
  }
  if (keep_raw && (r = save_raw(c, 0))) return r;
  if ((r = orth_block(c, 0))) return r;
  for (int i = 1; i <= p.q; ++i) {
    const size_t col = (size_t)(i - 1) * p.b * p.cs;
    if ((r = big_AhY(c, Q + col, p.m, p.n1 * p.m, T + col, p.m, p.n2 * p.m, (int)p.b))) return r;
    if ((r = big_AX(c, T + col, p.m, p.n2 * p.m, c.at(p.o_s0), p.b, p.n1 * p.b, (int)p.b))) return r;
    if (keep_raw && (r = save_raw(c, i))) return r;
    if ((r = orth_block(c, i, true))) return r;
  }
  const size_t col = (size_t)p.q * p.b * p.cs;
  return big_AhY(c, Q + col, p.m, p.n1 * p.m, T + col, p.m, p.n2 * p.m, (int)p.b);
}

// Alg. 2 with the Krylov blocks exactly as written, K_0 = A_f Om_f,
// K_i = A_f (A_f^H K_{i-1}), none orthonormalised before the next product;
// then the T-QR of K = [K_0 .. K_q], block by block (each block projected off
// the earlier ones twice and orthonormalised by shifted CholeskyQR, the same
// span as one QR of K), and C_f^H = A_f^H Q_f.
int krylov_literal(const Ctx& c, const void* A, const void* Omega) {
  const Plan& p = c.p;
  {
    Timed tm_(K_MISC, c.s);
    HIPCHK(zero_info(c.info(), c.s));
  }
  {
    Timed tm_(K_FFT_A, c.s);
    if (p.asplit)
      HIPCHK(fft_r2c_split(A, c.at(p.o_abar), p.n1 * p.n2, (int)p.n3, c.s));
    else
      HIPCHK(fft_r2c(A, c.at(p.o_abar), p.n1 * p.n2, (int)p.n3, p.dt, c.s));
  }
  {
    Timed tm_(K_FFT_OMEGA, c.s);
    HIPCHK(fft_r2c(Omega, c.at(p.o_obar), p.n2 * p.b, (int)p.n3, p.dt, c.s));
  }
  unsigned char* Q = c.at<unsigned char>(p.o_q);
  unsigned char* T = c.at<unsigned char>(p.o_t);
  int r;
  if ((r = big_AX(c, c.at(p.o_obar), p.b, p.n2 * p.b, Q, p.m, p.n1 * p.m, (int)p.b))) return r;
  for (int i = 1; i <= p.q; ++i) {
    const size_t prev = (size_t)(i - 1) * p.b * p.cs, col = (size_t)i * p.b * p.cs;
    if ((r = big_AhY(c, Q + prev, p.m, p.n1 * p.m, T + prev, p.m, p.n2 * p.m, (int)p.b))) return r;
    if ((r = big_AX(c, T + prev, p.m, p.n2 * p.m, Q + col, p.m, p.n1 * p.m, (int)p.b))) return r;
  }
  for (int i = 0; i <= p.q; ++i) {
    {
      Timed tm_(K_MISC, c.s);
      HIPCHK(hipMemcpy2DAsync(c.at(p.o_s0), (size_t)p.b * p.cs, Q + (size_t)i * p.b * p.cs, (size_t)p.m * p.cs,
                              (size_t)p.b * p.cs, (size_t)(p.F * p.n1), hipMemcpyDeviceToDevice, c.s));
    }
    if ((r = orth_block(c, i))) return r;
  }
  for (int i = 0; i <= p.q; ++i) {
    const size_t col = (size_t)i * p.b * p.cs;
    if ((r = big_AhY(c, Q + col, p.m, p.n1 * p.m, T + col, p.m, p.n2 * p.m, (int)p.b))) return r;
  }
  return TSVD_OK;
}

// Small SVD of C_f = T_f^H via G = T^H T, lift, phase, inverse DFT.
int svd_and_lift(const Ctx& c, void* U, void* S, void* V) {
  const Plan& p = c.p;
  const DType dt = p.dt;
  double* part = c.at<double>(p.o_part);
  void* T = c.at(p.o_t);
  int nsum_g = 1;
  // G_f = T^H T is Hermitian: on the FP32 path only its upper triangle is formed
  const bool upper = p.dt == DT_F32;
  int r = inner_products(c, T, p.m, (int)p.m, T, p.m, (int)p.m, p.n2, p.n2 * p.m, p.n2 * p.m, p.nsplit_g,
                         p.kchunk_g, part, &nsum_g, K_GEMM_LIFT, upper);
  if (r) return r;
  double* lam = c.at<double>(p.o_lam);
  double* Wd = c.at<double>(p.o_wd);
  const int stage_cls[4][2] = {
      {HEIG_TRIDIAG, K_HEIG_TRI}, {HEIG_BISECT, K_HEIG_BISECT}, {HEIG_INVIT, K_HEIG_INVIT}, {HEIG_BACKXF, K_HEIG_BACKXF}};
  if (dt == DT_F32) {
    for (const auto& sc : stage_cls) {
      Timed tm_(sc[1], c.s);
      HIPCHK(heig_topk(part, nsum_g, p.F * p.m * p.m, (int)p.m, (int)p.k, (int)p.F, lam, Wd, c.at(p.o_heig),
                       c.info(), c.s, sc[0], upper));
    }
  } else {
    // FP64: the eigenvalues of the Gram carry an absolute error of order
    // m u lambda_0, which leaves sigma_j below about sqrt(m u) sigma_0
    // unresolved.  The first pass keeps its J leading eigenpairs (above
    // 1e-9 lambda_0 and a gap); the second pass projects them out of C^H,
    // T1 = T (I - W_J W_J^H), and takes the top eigenpairs of T1^H T1, whose
    // absolute error scales with the much smaller norm of the rest; they are
    // projected off W_J once more and fill the columns from J on.
    double* lam1 = c.at<double>(p.o_lam1);
    double* W1 = c.at<double>(p.o_w1);
    for (const auto& sc : stage_cls) {
      Timed tm_(sc[1], c.s);
      HIPCHK(heig_topk(part, nsum_g, p.F * p.m * p.m, (int)p.m, (int)p.k, (int)p.F, lam1, W1, c.at(p.o_heig),
                       c.info(), c.s, sc[0], false));
    }
    int* J = c.at<int>(p.o_split);
    void* W1m = c.at(p.o_w1m);
    {
      Timed tm_(K_MISC, c.s);
      HIPCHK(tail_split(lam1, W1, W1m, (int)p.m, (int)p.k, (int)p.F, 1e-9, 1.5, J, c.s));
    }
    auto z64 = [&](const void* A, int64_t lda, int64_t sa, bool ac, const void* B, int64_t ldb, int64_t sb, bool bc,
                   void* C, int64_t ldc, int64_t sc, int M, int N, int K, double alpha, double beta) -> int {
      GemmDesc d = gd();
      d.A = A;
      d.lda = lda;
      d.strideA = sa;
      d.ta = DT_F64;
      d.a_conj = ac;
      d.B = B;
      d.ldb = ldb;
      d.strideB = sb;
      d.tb = DT_F64;
      d.b_conj = bc;
      d.C = C;
      d.ldc = ldc;
      d.strideC = sc;
      d.tc = DT_F64;
      d.M = M;
      d.N = N;
      d.K = K;
      d.batch = (int)p.F;
      d.alpha = alpha;
      d.beta = beta;
      d.compute = DT_F64;
      Timed tm_(K_GEMM_LIFT, c.s);
      HIPCHK(zgemm(d, c.s));
      return TSVD_OK;
    };
    const int im = (int)p.m, ik = (int)p.k, in2 = (int)p.n2;
    void* P = c.at(p.o_p);
    void* T1 = c.at(p.o_t1);
    // P = T W1m (n2 x k); T1 = T - P W1m^H (n2 x m)
    if ((r = z64(T, p.m, p.n2 * p.m, false, W1m, p.k, p.m * p.k, false, P, p.k, p.n2 * p.k, in2, ik, im, 1.0, 0.0)))
      return r;
    HIPCHK(hipMemcpyAsync(T1, T, (size_t)p.F * p.n2 * p.m * 16, hipMemcpyDeviceToDevice, c.s));
    if ((r = z64(P, p.k, p.n2 * p.k, false, W1m, p.k, p.m * p.k, true, T1, p.m, p.n2 * p.m, in2, im, ik, -1.0, 1.0)))
      return r;
    int nsum2 = 1;
    r = inner_products(c, T1, p.m, im, T1, p.m, im, p.n2, p.n2 * p.m, p.n2 * p.m, p.nsplit_g, p.kchunk_g, part,
                       &nsum2, K_GEMM_LIFT);
    if (r) return r;
    double* lam2 = c.at<double>(p.o_lam2);
    double* W2 = c.at<double>(p.o_w2);
    for (const auto& sc : stage_cls) {
      Timed tm_(sc[1], c.s);
      HIPCHK(heig_topk(part, nsum2, p.F * p.m * p.m, im, ik, (int)p.F, lam2, W2, c.at(p.o_heig), c.info(), c.s,
                       sc[0], false));
    }
    // W2 -= W1m (W1m^H W2)
    void* Rk = c.at(p.o_rk);
    if ((r = z64(W1m, p.k, p.m * p.k, true, W2, p.k, p.m * p.k, false, Rk, p.k, p.k * p.k, ik, ik, im, 1.0, 0.0)))
      return r;
    if ((r = z64(W1m, p.k, p.m * p.k, false, Rk, p.k, p.k * p.k, false, W2, p.k, p.m * p.k, im, ik, ik, -1.0, 1.0)))
      return r;
    {
      Timed tm_(K_MISC, c.s);
      HIPCHK(tail_merge(lam1, W1, lam2, W2, J, im, ik, (int)p.F, lam, Wd, c.s));
    }
  }
  if (dt == DT_F32) {
    // FP32 lift products on the Krylov-product kernel (FP32 MFMA, FP32
    // accumulation, as the generic product computes them): thin operands W_k
    // and W_k Sigma^{-1} rounded to complex FP32 in the o_wds buffer
    unsigned char* wb = c.at<unsigned char>(p.o_wds);
    void* Wf = wb;
    void* Wsf = wb + (size_t)p.F * p.m * p.k * 8;
    {
      Timed tm_(K_MISC, c.s);
      HIPCHK(lift_operands_f32(Wd, lam, Wf, Wsf, (int)p.m, (int)p.k, (int)p.F, c.s));
    }
    for (int side = 0; side < 2; ++side) {
      const int64_t nb = side == 0 ? p.n1 : p.n2;
      KGemmDesc k{};
      k.A = side == 0 ? c.at(p.o_q) : T;
      k.lda = p.m;
      k.strideA = nb * p.m;
      k.rows = (int)nb;
      k.cols = (int)p.m;
      k.herm = false;
      k.X = side == 0 ? Wf : Wsf;
      k.ldx = p.k;
      k.strideX = p.m * p.k;
      k.C = c.at(side == 0 ? p.o_uf : p.o_vf);
      k.ldc = p.k;
      k.strideC = nb * p.k;
      k.N = (int)p.k;
      k.batch = (int)p.F;
      k.mode = KM_F32;
      k.nsplit = 1;
      k.part = c.at(p.o_kpart);
      k.part_bytes = p.kpart_bytes;
      Timed tm_(K_GEMM_LIFT, c.s);
      HIPCHK(kgemm(k, c.s));
    }
  } else {
    // U_f = Q_f W_k
    GemmDesc d = gd();
    d.A = c.at(p.o_q);
    d.lda = p.m;
    d.strideA = p.n1 * p.m;
    d.ta = dt;
    d.B = Wd;
    d.ldb = p.k;
    d.strideB = p.m * p.k;
    d.tb = DT_F64;
    d.C = c.at(p.o_uf);
    d.ldc = p.k;
    d.strideC = p.n1 * p.k;
    d.tc = dt;
    d.M = (int)p.n1;
    d.N = (int)p.k;
    d.K = (int)p.m;
    d.batch = (int)p.F;
    d.compute = dt;
    {
      Timed tm_(K_GEMM_LIFT, c.s);
      HIPCHK(zgemm(d, c.s));
    }
    // V_f = T_f W_k diag(1/sigma) with sigma_j = ||T_f w_j|| (the columns'
    // norms resolve small sigma_j far better than sqrt(lambda_j) of the Gram)
    d.A = T;
    d.strideA = p.n2 * p.m;
    d.B = Wd;
    d.C = c.at(p.o_vf);
    d.strideC = p.n2 * p.k;
    d.M = (int)p.n2;
    {
      Timed tm_(K_GEMM_LIFT, c.s);
      HIPCHK(zgemm(d, c.s));
    }
    {
      Timed tm_(K_MISC, c.s);
      HIPCHK(colnorm_sigma(c.at(p.o_vf), p.n2, (int)p.k, (int)p.F, c.at<double>(p.o_sig), c.at(p.o_scx), c.s));
    }
  }
  {
    Timed tm_(K_MISC, c.s);
    HIPCHK(canon_phase(c.at(p.o_uf), p.n1, c.at(p.o_vf), p.n2, (int)p.k, (int)p.F, dt, c.at(p.o_canon), c.s));
  }
  if (dt == DT_F32) {
    Timed tm_(K_MISC, c.s);
    HIPCHK(sigma_from_lambda(lam, c.at<double>(p.o_sig), c.at(p.o_scx), p.F * p.k, dt, c.s));
  }
  {
    Timed tm_(K_FFT_INV, c.s);
    HIPCHK(fft_c2r(c.at(p.o_uf), p.n1 * p.k, U, p.n1 * p.k, (int)p.n3, dt, c.s));
  }
  {
    Timed tm_(K_FFT_INV, c.s);
    HIPCHK(fft_c2r(c.at(p.o_vf), p.n2 * p.k, V, p.n2 * p.k, (int)p.n3, dt, c.s));
  }
  {
    Timed tm_(K_FFT_INV, c.s);
    HIPCHK(fft_c2r(c.at(p.o_scx), p.k, S, p.k, (int)p.n3, dt, c.s));
  }
  return TSVD_OK;
}


// X_f = (U_f diag(sigma)) V_f^H over A_f's buffer, then the inverse DFT to
// Xhat (the rank-k approximation U * S * V^T, Alg. TP).
int approx_tail(const Ctx& c, void* Xhat) {
  const Plan& p = c.p;
  {
    Timed tm_(K_MISC, c.s);
    HIPCHK(scale_cols_by(c.at(p.o_uf), c.at<double>(p.o_sig), c.at(p.o_us), p.n1, (int)p.k, (int)p.F, p.dt, c.s));
  }
  GemmDesc d = gd();
  d.A = c.at(p.o_us);
  d.lda = p.k;
  d.strideA = p.n1 * p.k;
  d.ta = p.dt;
  d.B = c.at(p.o_vf);
  d.ldb = p.k;
  d.strideB = p.n2 * p.k;
  d.tb = p.dt;
  d.b_conj = true;
  d.C = c.at(p.o_abar);
  d.ldc = p.n2;
  d.strideC = p.n1 * p.n2;
  d.tc = p.dt;
  d.M = (int)p.n1;
  d.N = (int)p.n2;
  d.K = (int)p.k;
  d.batch = (int)p.F;
  d.compute = p.dt;
  {
    Timed tm_(K_GEMM_LIFT, c.s);
    HIPCHK(zgemm(d, c.s));
  }
  {
    Timed tm_(K_FFT_INV, c.s);
    HIPCHK(fft_c2r(c.at(p.o_abar), p.n1 * p.n2, Xhat, p.n1 * p.n2, (int)p.n3, p.dt, c.s));
  }
  return TSVD_OK;
}

// Alg. TQR on the half spectrum: A_f -> Ā, Q_f = orthonormal basis of the
// first r = min(n1, n2) columns of A_f, one b-column panel after the other
// (each projected off the earlier panels and orthonormalised by shifted
// CholeskyQR, so span Q_f(:, 1:j) = span A_f(:, 1:j) at every panel end and
// the diagonal of R is real positive), R_f = Q_f^H A_f as FP64 partials
// (upper trapezoid valid).
int tqr_core(const Ctx& c, const void* A, int* nsum) {
  const Plan& p = c.p;
  {
    Timed tm_(K_MISC, c.s);
    HIPCHK(zero_info(c.info(), c.s));
  }
  {
    Timed tm_(K_FFT_A, c.s);
    HIPCHK(fft_r2c(A, c.at(p.o_abar), p.n1 * p.n2, (int)p.n3, p.dt, c.s));
  }
  int r;
  for (int i = 0; i <= p.q; ++i) {
    // panel i of A_f (row stride n2) into the staging block, then as a Krylov block
    {
      Timed tm_(K_MISC, c.s);
      HIPCHK(hipMemcpy2DAsync(c.at(p.o_s0), (size_t)p.b * p.cs,
                              c.at<unsigned char>(p.o_abar) + (size_t)i * p.b * p.cs, (size_t)p.n2 * p.cs,
                              (size_t)p.b * p.cs, (size_t)(p.F * p.n1), hipMemcpyDeviceToDevice, c.s));
    }
    if ((r = orth_block(c, i))) return r;
  }
  return inner_products(c, c.at(p.o_q), p.m, (int)p.m, c.at(p.o_abar), p.n2, (int)p.n2, p.n1, p.n1 * p.m,
                        p.n1 * p.n2, p.nsplit_r, p.kchunk_r, c.at<double>(p.o_part), nsum);
}

// Generic batched product C = alpha opA(A) opB(B) + beta C over the F slices
// (element strides and leading dimensions in complex elements).
struct Op {
  const void* p;
  int64_t ld, stride;
  DType t;
  bool conj;
};
int gemm(const Ctx& c, int cls, Op A, Op B, void* C, int64_t ldc, int64_t strideC, DType tc, int M, int N, int K,
         double alpha, double beta, DType compute, int b_nsum = 1, int64_t b_sum_stride = 0) {
  GemmDesc d = gd();
  d.A = A.p;
  d.lda = A.ld;
  d.strideA = A.stride;
  d.ta = A.t;
  d.a_conj = A.conj;
  d.B = B.p;
  d.ldb = B.ld;
  d.strideB = B.stride;
  d.tb = B.t;
  d.b_conj = B.conj;
  d.b_nsum = b_nsum;
  d.b_sum_stride = b_sum_stride;
  d.C = C;
  d.ldc = ldc;
  d.strideC = strideC;
  d.tc = tc;
  d.M = M;
  d.N = N;
  d.K = K;
  d.batch = (int)c.p.F;
  d.alpha = alpha;
  d.beta = beta;
  d.compute = compute;
  Timed tm_(cls, c.s);
  HIPCHK(zgemm(d, c.s));
  return TSVD_OK;
}

// Reverse pass of P(A) = Q Q^H A per Fourier slice (stabilised Krylov form):
//   direct term Q Q^H G; Qbar = (G A^H + A G^H) Q; for i = q..0:
//   Zbar_i = (I - Q_i Q_i^H) Qbar_i R_i^{-H} with R_i = Q_i^H W_i (the loss
//   depends on Q_i only through its range); for i >= 1:
//   Wbar_i = (I - Q_<i Q_<i^H) Zbar_i, Qbar_<i -= (Zbar_i W_i^H + W_i Zbar_i^H) Q_<i,
//   Abar += Wbar_i T_i^H, Tbar_i = A^H Wbar_i, Abar += Q_{i-1} Tbar_i^H,
//   Qbar_{i-1} += A Tbar_i; for i = 0: Abar += Zbar_0 Om^H.
int truncation_head(const Ctx& c, void* U2, void* Ub2, void* Tp);

int proj_backward_impl(const Ctx& c, const void* A, const void* Omega, const void* G, void* dA,
                       bool truncated = false) {
  const Plan& p = c.p;
  const DType dt = p.dt;
  int r = krylov(c, A, Omega, true);
  if (r) return r;
  {
    Timed tm_(K_FFT_A, c.s);
    HIPCHK(fft_r2c(G, c.at(p.o_gbar), p.n1 * p.n2, (int)p.n3, dt, c.s));
  }
  const int n1 = (int)p.n1, n2 = (int)p.n2, m = (int)p.m, b = (int)p.b;
  const int64_t s12 = p.n1 * p.n2, s1m = p.n1 * p.m, s2m = p.n2 * p.m, s1b = p.n1 * p.b, s2b = p.n2 * p.b;
  unsigned char* Q = c.at<unsigned char>(p.o_q);
  unsigned char* T = c.at<unsigned char>(p.o_t);
  unsigned char* Wr = c.at<unsigned char>(p.o_wraw);
  unsigned char* Qb = c.at<unsigned char>(p.o_qbar);
  void* Ab = c.at(p.o_abar);
  void* Gb = c.at(p.o_gbar);
  void* Db = c.at(p.o_dbar);
  void* U2 = c.at(p.o_u2);
  void* Zb = c.at(p.o_zbar);
  void* Wb = c.at(p.o_wbar);
  void* Tb = c.at(p.o_tbar);
  double* part = c.at<double>(p.o_part);
  const size_t cs = p.cs;
  // U2 = Gbar^H Q (= Y^H, Y = Q^H Gbar); Dbar = Q U2^H (= Q Q^H Gbar)
  if ((r = gemm(c, K_GEMM_KRYLOV, Op{Gb, n2, s12, dt, true}, Op{Q, m, s1m, dt, false}, U2, m, s2m, dt, n2, m, n1, 1.0,
                0.0, dt)))
    return r;
  // the rank-k truncation replaces U2 by Cbar^H = U2 Pi + T H and T by T Pi
  // (truncation_head); the projection keeps them
  void* Ub2 = U2;
  void* Tq = T;
  if (truncated) {
    Ub2 = c.at(p.o_u2b);
    Tq = c.at(p.o_tp);
    if ((r = truncation_head(c, U2, Ub2, Tq))) return r;
  }
  if ((r = gemm(c, K_GEMM_LIFT, Op{Q, m, s1m, dt, false}, Op{Ub2, m, s2m, dt, true}, Db, n2, s12, dt, n1, n2, m, 1.0,
                0.0, dt)))
    return r;
  // Qbar = Gbar T + Abar U2   (T = Abar^H Q)
  if ((r = gemm(c, K_GEMM_KRYLOV, Op{Gb, n2, s12, dt, false}, Op{Tq, m, s2m, dt, false}, Qb, m, s1m, dt, n1, m, n2,
                1.0, 0.0, dt)))
    return r;
  if ((r = gemm(c, K_GEMM_KRYLOV, Op{Ab, n2, s12, dt, false}, Op{Ub2, m, s2m, dt, false}, Qb, m, s1m, dt, n1, m, n2,
                1.0, 1.0, dt)))
    return r;
  const int ns = p.nsplit_blk, kc = p.kchunk_blk;
  int nsum = 1;
  for (int i = (int)p.q; i >= 0; --i) {
    unsigned char* Qi = Q + (size_t)i * b * cs;
    unsigned char* Qbi = Qb + (size_t)i * b * cs;
    unsigned char* Wi = Wr + (size_t)i * b * cs;
    // Qbar_i -= Q_i (Q_i^H Qbar_i)
    if ((r = inner_products(c, Qi, m, b, Qbi, m, b, p.n1, s1m, s1m, ns, kc, part, &nsum))) return r;
    if ((r = gemm(c, K_GEMM_ORTH, Op{Qi, m, s1m, dt, false}, Op{part, b, (int64_t)b * b, DT_F64, false}, Qbi, m, s1m,
                  dt, n1, b, b, -1.0, 1.0, DT_F64, nsum, p.F * b * b)))
      return r;
    // R_i = Q_i^H W_i, Rinv = R_i^{-1}
    if ((r = inner_products(c, Qi, m, b, Wi, m, b, p.n1, s1m, s1m, ns, kc, part, &nsum))) return r;
    {
      Timed tm_(K_CHOL, c.s);
      HIPCHK(chol_inv_ex(part, nsum, p.F * b * b, c.at<double>(p.o_rinv), c.at(p.o_chol), b, (int)p.F, 0.0, c.info(),
                         c.s, 1));
    }
    // Zbar = (I - Q_i Q_i^H) Qbar_i R_i^{-H}
    if ((r = gemm(c, K_GEMM_ORTH, Op{Qbi, m, s1m, dt, false}, Op{c.at(p.o_rinv), b, (int64_t)b * b, DT_F64, true},
                  Zb, b, s1b, dt, n1, b, b, 1.0, 0.0, DT_F64)))
      return r;
    if (i == 0) {
      // Dbar += Zbar_0 Om^H
      if ((r = gemm(c, K_GEMM_LIFT, Op{Zb, b, s1b, dt, false}, Op{c.at(p.o_obar), b, s2b, dt, true}, Db, n2, s12, dt,
                    n1, n2, b, 1.0, 1.0, dt)))
        return r;
      break;
    }
    const int ib = i * b;
    // Wbar = Zbar - Q_<i (Q_<i^H Zbar)
    HIPCHK(hipMemcpyAsync(Wb, Zb, (size_t)p.F * s1b * cs, hipMemcpyDeviceToDevice, c.s));
    if ((r = inner_products(c, Q, m, ib, Zb, b, b, p.n1, s1m, s1b, ns, kc, part, &nsum))) return r;
    if ((r = gemm(c, K_GEMM_ORTH, Op{Q, m, s1m, dt, false}, Op{part, b, (int64_t)ib * b, DT_F64, false}, Wb, b, s1b,
                  dt, n1, b, ib, -1.0, 1.0, DT_F64, nsum, p.F * ib * b)))
      return r;
    // Qbar_<i -= Zbar (W_i^H Q_<i) + W_i (Zbar^H Q_<i)
    if ((r = inner_products(c, Wi, m, b, Q, m, ib, p.n1, s1m, s1m, ns, kc, part, &nsum))) return r;
    if ((r = gemm(c, K_GEMM_ORTH, Op{Zb, b, s1b, dt, false}, Op{part, ib, (int64_t)b * ib, DT_F64, false}, Qb, m, s1m,
                  dt, n1, ib, b, -1.0, 1.0, DT_F64, nsum, p.F * b * ib)))
      return r;
    if ((r = inner_products(c, Zb, b, b, Q, m, ib, p.n1, s1b, s1m, ns, kc, part, &nsum))) return r;
    if ((r = gemm(c, K_GEMM_ORTH, Op{Wi, m, s1m, dt, false}, Op{part, ib, (int64_t)b * ib, DT_F64, false}, Qb, m, s1m,
                  dt, n1, ib, b, -1.0, 1.0, DT_F64, nsum, p.F * b * ib)))
      return r;
    unsigned char* Ti = T + (size_t)(i - 1) * b * cs;
    unsigned char* Qi1 = Q + (size_t)(i - 1) * b * cs;
    unsigned char* Qbi1 = Qb + (size_t)(i - 1) * b * cs;
    // Dbar += Wbar T_i^H
    if ((r = gemm(c, K_GEMM_LIFT, Op{Wb, b, s1b, dt, false}, Op{Ti, m, s2m, dt, true}, Db, n2, s12, dt, n1, n2, b, 1.0,
                  1.0, dt)))
      return r;
    // Tbar = Abar^H Wbar
    if ((r = gemm(c, K_GEMM_KRYLOV, Op{Ab, n2, s12, dt, true}, Op{Wb, b, s1b, dt, false}, Tb, b, s2b, dt, n2, b, n1,
                  1.0, 0.0, dt)))
      return r;
    // Dbar += Q_{i-1} Tbar^H
    if ((r = gemm(c, K_GEMM_LIFT, Op{Qi1, m, s1m, dt, false}, Op{Tb, b, s2b, dt, true}, Db, n2, s12, dt, n1, n2, b, 1.0,
                  1.0, dt)))
      return r;
    // Qbar_{i-1} += Abar Tbar
    if ((r = gemm(c, K_GEMM_KRYLOV, Op{Ab, n2, s12, dt, false}, Op{Tb, b, s2b, dt, false}, Qbi1, m, s1m, dt, n1, b, n2,
                  1.0, 1.0, dt)))
      return r;
  }
  {
    Timed tm_(K_FFT_INV, c.s);
    HIPCHK(fft_c2r(Db, s12, dA, s12, (int)p.n3, dt, c.s));
  }
  return TSVD_OK;
}

// Head of the adjoint through the rank-k truncation, X_f = Q Pi C with
// C = Q^H A_f = T^H and Pi = W_k W_k^H the projector onto the top-k
// eigenvectors of C C^H (Lemma mn38).  With Y = Q^H Gbar (U2 = Y^H):
// Cbar = Pi Y + H C and Qbar = Gbar C^H Pi + A_f Cbar^H, where H = W S W^H,
// S = N + N^H and N couples each eigenvector a of the top k with each c
// outside it: N_ac = M_ac / (lambda_a - lambda_c), N_ca = M_ca / (lambda_a -
// lambda_c), M = W^H (Y C^H) W.  Writes Ub2 = Cbar^H = U2 Pi + T H and
// Tp = T Pi (n2 x m each, working type); every m x m matrix is FP64.
int truncation_head(const Ctx& c, void* U2, void* Ub2, void* Tp) {
  const Plan& p = c.p;
  const DType dt = p.dt;
  const int n2 = (int)p.n2, m = (int)p.m, k = (int)p.k;
  const int64_t s2m = p.n2 * p.m, mm = p.m * p.m;
  void* T = c.at(p.o_t);
  double* part = c.at<double>(p.o_part);
  double* lam = c.at<double>(p.o_lall);
  void* W = c.at(p.o_wall);
  void* M0 = c.at(p.o_mm0);
  void* M1 = c.at(p.o_mm1);
  void* M2 = c.at(p.o_mm2);
  void* M3 = c.at(p.o_mm3);
  // all m eigenpairs of C C^H = T^H T (descending)
  const bool upper = dt == DT_F32;
  int nsum = 1;
  int r = inner_products(c, T, p.m, m, T, p.m, m, p.n2, s2m, s2m, p.nsplit_g, p.kchunk_g, part, &nsum, K_GEMM_LIFT,
                         upper);
  if (r) return r;
  const int stage_cls[4][2] = {
      {HEIG_TRIDIAG, K_HEIG_TRI}, {HEIG_BISECT, K_HEIG_BISECT}, {HEIG_INVIT, K_HEIG_INVIT}, {HEIG_BACKXF, K_HEIG_BACKXF}};
  for (const auto& sc : stage_cls) {
    Timed tm_(sc[1], c.s);
    HIPCHK(heig_topk(part, nsum, p.F * mm, m, m, (int)p.F, lam, (double*)W, c.at(p.o_heig), c.info(), c.s, sc[0],
                     upper));
  }
  // M = W^H (U2^H T) W
  if ((r = gemm(c, K_GEMM_LIFT, Op{U2, p.m, s2m, dt, true}, Op{T, p.m, s2m, dt, false}, M0, p.m, mm, DT_F64, m, m, n2,
                1.0, 0.0, DT_F64)))
    return r;
  if ((r = gemm(c, K_GEMM_LIFT, Op{M0, p.m, mm, DT_F64, false}, Op{W, p.m, mm, DT_F64, false}, M1, p.m, mm, DT_F64, m,
                m, m, 1.0, 0.0, DT_F64)))
    return r;
  if ((r = gemm(c, K_GEMM_LIFT, Op{W, p.m, mm, DT_F64, true}, Op{M1, p.m, mm, DT_F64, false}, M2, p.m, mm, DT_F64, m,
                m, m, 1.0, 0.0, DT_F64)))
    return r;
  // S = N + N^H (zero inside either group; a gap at the eigenvalues' rounding
  // level counts as a tie), H = W S W^H
  {
    Timed tm_(K_MISC, c.s);
    HIPCHK(gap_weights(M2, lam, m, k, (int)p.F, 8.0 * m * 0x1p-53, M0, c.info(), c.s));
  }
  if ((r = gemm(c, K_GEMM_LIFT, Op{W, p.m, mm, DT_F64, false}, Op{M0, p.m, mm, DT_F64, false}, M1, p.m, mm, DT_F64, m,
                m, m, 1.0, 0.0, DT_F64)))
    return r;
  if ((r = gemm(c, K_GEMM_LIFT, Op{M1, p.m, mm, DT_F64, false}, Op{W, p.m, mm, DT_F64, true}, M3, p.m, mm, DT_F64, m,
                m, m, 1.0, 0.0, DT_F64)))
    return r;
  // Pi = W_k W_k^H
  if ((r = gemm(c, K_GEMM_LIFT, Op{W, p.m, mm, DT_F64, false}, Op{W, p.m, mm, DT_F64, true}, M2, p.m, mm, DT_F64, m,
                m, k, 1.0, 0.0, DT_F64)))
    return r;
  // Ub2 = U2 Pi + T H; Tp = T Pi
  if ((r = gemm(c, K_GEMM_LIFT, Op{U2, p.m, s2m, dt, false}, Op{M2, p.m, mm, DT_F64, false}, Ub2, p.m, s2m, dt, n2, m,
                m, 1.0, 0.0, DT_F64)))
    return r;
  if ((r = gemm(c, K_GEMM_LIFT, Op{T, p.m, s2m, dt, false}, Op{M3, p.m, mm, DT_F64, false}, Ub2, p.m, s2m, dt, n2, m,
                m, 1.0, 1.0, DT_F64)))
    return r;
  return gemm(c, K_GEMM_LIFT, Op{T, p.m, s2m, dt, false}, Op{M2, p.m, mm, DT_F64, false}, Tp, p.m, s2m, dt, n2, m, m,
              1.0, 0.0, DT_F64);
}

// Alg. 2 with the basis truncated to its top b Ritz directions before the
// projection (the timing remark of Sec. 5, Ex. 1, read as Rayleigh-Ritz):
// Q_r = Q W_b (the lift of the first small SVD with b columns, phases as for
// U), Qr = its inverse transform; then the projection with the truncated
// basis, T_r = A_f^H Q_r (one b-column Krylov product), and the small SVD,
// lift, truncation to k and inverse transforms of Alg. 2 on (Q_r, T_r).
int ritz_body(const Ctx& c, const void* A, const void* Omega, void* Qr, void* U, void* S, void* V) {
  const Plan& p = c.p;
  int r = krylov(c, A, Omega);
  if (r) return r;
  // Ritz step: top-b eigenpairs of C C^H, Q_r = Q W_b into S0
  Plan p1 = p;
  p1.k = p.b;
  p1.o_uf = p.o_s0;
  Ctx c1{p1, c.ws, c.s};
  if ((r = svd_and_lift(c1, Qr, c.at(p.o_sr), c.at(p.o_vr)))) return r;
  // T_r = A_f^H Q_r (n2 x b, ld b) over T, which is no longer needed
  if ((r = big_AhY(c, c.at(p.o_s0), p.b, p.n1 * p.b, c.at(p.o_t), p.b, p.n2 * p.b, (int)p.b))) return r;
  // the small SVD of C_r = T_r^H with m = b
  Plan p2 = p;
  p2.m = p.b;
  p2.o_q = p.o_s0;
  p2.nsplit_g = p.nsplit_t;
  p2.kchunk_g = p.kchunk_t;
  Ctx c2{p2, c.ws, c.s};
  return svd_and_lift(c2, U, S, V);
}

bool aligned(const void* ptr, size_t a) { return ((uintptr_t)ptr % a) == 0; }

int check_ptrs(std::initializer_list<const void*> ptrs, const void* ws, size_t ws_bytes, const Plan& p) {
  for (const void* q : ptrs)
    if (!q || !aligned(q, 16)) return fail(TSVD_EINVAL, "null or misaligned (16 B) tensor pointer");
  if (!ws || !aligned(ws, 256)) return fail(TSVD_EINVAL, "null or misaligned (256 B) workspace");
  if (ws_bytes < p.total) return fail(TSVD_ENOMEM, "workspace smaller than tsvd_workspace_bytes()");
  return TSVD_OK;
}


// Omega == nullptr: the test tensor of Alg. 2 is drawn from `seed` into the
// workspace (the seed-taking entry points); otherwise the caller's tensor is used.
int resolve_omega(const Ctx& c, const void*& Omega, uint64_t seed) {
  if (Omega) return TSVD_OK;
  void* o = c.at(c.p.o_omsp);
  {
    Timed tm_(K_MISC, c.s);
    HIPCHK(omega_fill(o, c.p.n2 * c.p.b * c.p.n3, seed, c.p.dt, c.s));
  }
  Omega = o;
  return TSVD_OK;
}

int need_omega(const void* Omega) {
  if (!Omega || !aligned(Omega, 16)) return fail(TSVD_EINVAL, "null or misaligned (16 B) Omega");
  return TSVD_OK;
}

// Alg. 2 (op RBK / APPROX / RBK_LITERAL) or Alg. 1 (POWER / POWER_APPROX) on
// one tensor: Krylov (or power) basis, small SVD, lift, optional X_hat.
int svd_call(bool given, int op, const void* A, const void* Omega, uint64_t seed, int64_t n1, int64_t n2, int64_t n3, int64_t k,
             int64_t b, int64_t q, int prec, void* U, void* S, void* V, void* Xhat, void* ws, size_t ws_bytes,
             void* stream) {
  Plan p;
  int r = make_plan(n1, n2, n3, k, b, q, prec, op, &p);
  if (r) return r;
  if ((r = check_ptrs({A, U, S, V}, ws, ws_bytes, p))) return r;
  if (given && (r = need_omega(Omega))) return r;
  if ((op == TSVD_OP_APPROX || op == TSVD_OP_POWER_APPROX) && (!Xhat || !aligned(Xhat, 16)))
    return fail(TSVD_EINVAL, "null or misaligned (16 B) Xhat");
  if (Xhat && !aligned(Xhat, 16)) return fail(TSVD_EINVAL, "misaligned (16 B) Xhat");
  Ctx c{p, (unsigned char*)ws, (hipStream_t)stream};
  if ((r = resolve_omega(c, Omega, seed))) return r;
  if ((r = op == TSVD_OP_RBK_LITERAL ? krylov_literal(c, A, Omega) : krylov(c, A, Omega))) return r;
  if ((r = svd_and_lift(c, U, S, V))) return r;
  if (Xhat && (r = approx_tail(c, Xhat))) return r;
  g_err.clear();
  return TSVD_OK;
}

int complete_call(bool given, const void* M, const void* mask, const void* Omega, uint64_t seed, int64_t n1, int64_t n2,
                  int64_t n3, int64_t k, int64_t b, int64_t q, int64_t iters, int alg, int prec, void* C, void* ws,
                  size_t ws_bytes, void* stream) {
  if (alg != 1 && alg != 2) return fail(TSVD_EINVAL, "alg must be 1 (power iteration) or 2 (block Krylov)");
  if (iters < 0 || iters > 1000000) return fail(TSVD_EINVAL, "need 0 <= iters <= 1000000");
  Plan p;
  int r = make_plan(n1, n2, n3, k, b, q, prec, alg == 2 ? TSVD_OP_COMPLETE_RBK : TSVD_OP_COMPLETE_POWER, &p);
  if (r) return r;
  if ((r = check_ptrs({M, C}, ws, ws_bytes, p))) return r;
  if (!mask) return fail(TSVD_EINVAL, "null mask");
  if (given && (r = need_omega(Omega))) return r;
  Ctx c{p, (unsigned char*)ws, (hipStream_t)stream};
  // the same test tensor at every iteration
  if ((r = resolve_omega(c, Omega, seed))) return r;
  const int64_t n = n1 * n2 * n3;
  const unsigned char* T = static_cast<const unsigned char*>(mask);
  void* Cb = c.at(p.o_cbuf);
  {
    // C^(0) = T (.) M
    Timed tm_(K_MISC, c.s);
    HIPCHK(masked_merge(M, T, nullptr, iters == 0 ? C : Cb, n, p.dt, c.s));
  }
  for (int64_t it = 0; it < iters; ++it) {
    // X^(n) = L(C^(n)): the rank-k approximation of the chosen method
    if ((r = krylov(c, Cb, Omega))) return r;
    if ((r = svd_and_lift(c, c.at(p.o_uo), c.at(p.o_so), c.at(p.o_vo)))) return r;
    if ((r = approx_tail(c, c.at(p.o_xbuf)))) return r;
    // C^(n+1) = T (.) M + (1 - T) (.) X^(n)
    Timed tm_(K_MISC, c.s);
    HIPCHK(masked_merge(M, T, c.at(p.o_xbuf), it + 1 == iters ? C : Cb, n, p.dt, c.s));
  }
  g_err.clear();
  return TSVD_OK;
}

int proj_call(bool given, const void* A, const void* Omega, uint64_t seed, int64_t n1, int64_t n2, int64_t n3, int64_t b,
              int64_t q, int prec, void* P, void* ws, size_t ws_bytes, void* stream) {
  Plan p;
  int r = make_plan(n1, n2, n3, 1, b, q, prec, TSVD_OP_PROJ, &p);
  if (r) return r;
  if ((r = check_ptrs({A, P}, ws, ws_bytes, p))) return r;
  if (given && (r = need_omega(Omega))) return r;
  Ctx c{p, (unsigned char*)ws, (hipStream_t)stream};
  if ((r = resolve_omega(c, Omega, seed))) return r;
  if ((r = krylov(c, A, Omega))) return r;
  // P_f = Q_f C_f = Q_f T_f^H, written over A_f (no longer needed).
  GemmDesc d = gd();
  d.A = c.at(p.o_q);
  d.lda = p.m;
  d.strideA = p.n1 * p.m;
  d.ta = p.dt;
  d.B = c.at(p.o_t);
  d.ldb = p.m;
  d.strideB = p.n2 * p.m;
  d.tb = p.dt;
  d.b_conj = true;
  d.C = c.at(p.o_abar);
  d.ldc = p.n2;
  d.strideC = p.n1 * p.n2;
  d.tc = p.dt;
  d.M = (int)p.n1;
  d.N = (int)p.n2;
  d.K = (int)p.m;
  d.batch = (int)p.F;
  d.compute = p.dt;
  {
    Timed tm_(K_GEMM_LIFT, c.s);
    HIPCHK(zgemm(d, c.s));
  }
  {
    Timed tm_(K_FFT_INV, c.s);
    HIPCHK(fft_c2r(c.at(p.o_abar), p.n1 * p.n2, P, p.n1 * p.n2, (int)p.n3, p.dt, c.s));
  }
  g_err.clear();
  return TSVD_OK;
}

int proj_backward_call(bool given, const void* A, const void* Omega, uint64_t seed, const void* G, int64_t n1, int64_t n2,
                       int64_t n3, int64_t b, int64_t q, int prec, void* dA, void* ws, size_t ws_bytes, void* stream) {
  Plan p;
  int r = make_plan(n1, n2, n3, 1, b, q, prec, TSVD_OP_PROJ_BWD, &p);
  if (r) return r;
  if ((r = check_ptrs({A, G, dA}, ws, ws_bytes, p))) return r;
  if (given && (r = need_omega(Omega))) return r;
  Ctx c{p, (unsigned char*)ws, (hipStream_t)stream};
  if ((r = resolve_omega(c, Omega, seed))) return r;
  if ((r = proj_backward_impl(c, A, Omega, G, dA))) return r;
  g_err.clear();
  return TSVD_OK;
}

int approx_backward_call(bool given, const void* A, const void* Omega, uint64_t seed, const void* G, int64_t n1,
                         int64_t n2, int64_t n3, int64_t k, int64_t b, int64_t q, int prec, void* dA, void* ws,
                         size_t ws_bytes, void* stream) {
  Plan p;
  int r = make_plan(n1, n2, n3, k, b, q, prec, TSVD_OP_APPROX_BWD, &p);
  if (r) return r;
  if ((r = check_ptrs({A, G, dA}, ws, ws_bytes, p))) return r;
  if (given && (r = need_omega(Omega))) return r;
  Ctx c{p, (unsigned char*)ws, (hipStream_t)stream};
  if ((r = resolve_omega(c, Omega, seed))) return r;
  if ((r = proj_backward_impl(c, A, Omega, G, dA, true))) return r;
  g_err.clear();
  return TSVD_OK;
}

int ritz_call(bool given, const void* A, const void* Omega, uint64_t seed, int64_t n1, int64_t n2, int64_t n3,
              int64_t k, int64_t b, int64_t q, int prec, void* Qr, void* U, void* S, void* V, void* ws, size_t ws_bytes,
              void* stream) {
  Plan p;
  int r = make_plan(n1, n2, n3, k, b, q, prec, TSVD_OP_RBK_RITZ, &p);
  if (r) return r;
  if ((r = check_ptrs({A, Qr, U, S, V}, ws, ws_bytes, p))) return r;
  if (given && (r = need_omega(Omega))) return r;
  Ctx c{p, (unsigned char*)ws, (hipStream_t)stream};
  if ((r = resolve_omega(c, Omega, seed))) return r;
  if ((r = ritz_body(c, A, Omega, Qr, U, S, V))) return r;
  g_err.clear();
  return TSVD_OK;
}

// ---- scratch for the entry point that allocates nothing ----
// A file-scope device array: each device the library runs on holds its own
// copy until the process ends.  In host code its name stands for a host-side
// symbol, not a device address: the device address comes from
// hipGetSymbolAddress, once per device, and is the only handle used.
constexpr size_t kStaticScratchBytes = TSVD_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch (looked up on its first use
// on that device, with that device current).
int static_scratch(void** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(TSVD_EHIP, "device index beyond the scratch table");
  std::lock_guard<std::mutex> l(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(TSVD_EHIP, "hipGetSymbolAddress returned no address for the static scratch");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return TSVD_OK;
}

}  // namespace

extern "C" {

int tsvd_version(void) { return 100; }

const char* tsvd_last_error(void) { return g_err.c_str(); }

size_t tsvd_workspace_bytes(int64_t n1, int64_t n2, int64_t n3, int64_t k, int64_t b, int64_t q, int prec, int op) {
  Plan p;
  if (make_plan(n1, n2, n3, k, b, q, prec, op, &p)) return 0;
  return p.total;
}

int tsvd_omega(int64_t n2, int64_t b, int64_t n3, uint64_t seed, double* out_host) {
  if (n2 < 1 || b < 1 || n3 < 1 || !out_host) return fail(TSVD_EINVAL, "need n2, b, n3 >= 1 and a host buffer");
  if (n2 > ((int64_t)1 << 40) / b || n2 * b > ((int64_t)1 << 40) / n3)
    return fail(TSVD_EINVAL, "n2 * b * n3 must be <= 2^40");
  omega_host(out_host, n2 * b * n3, seed);
  g_err.clear();
  return TSVD_OK;
}

int tsvd_rbk(const void* A, int64_t n1, int64_t n2, int64_t n3, int64_t k, int64_t b, int64_t q, uint64_t seed,
             int prec, void* U, void* S, void* V, void* ws, size_t ws_bytes, void* stream) {
  return svd_call(false, TSVD_OP_RBK, A, nullptr, seed, n1, n2, n3, k, b, q, prec, U, S, V, nullptr, ws, ws_bytes, stream);
}

int tsvd_rbk_noalloc(const void* A, int64_t n1, int64_t n2, int64_t n3, int64_t k, int64_t b, int64_t q,
                     uint64_t seed, int prec, void* U, void* S, void* V, void* stream) {
  Plan p;
  int r = make_plan(n1, n2, n3, k, b, q, prec, TSVD_OP_RBK, &p);
  if (r) return r;
  if (p.total > kStaticScratchBytes) {
    char msg[160];
    snprintf(msg, sizeof msg, "tsvd_rbk_noalloc: these sizes need %zu bytes of scratch, beyond its %zu bytes; use "
             "tsvd_rbk with a workspace", p.total, kStaticScratchBytes);
    return fail(TSVD_ENOMEM, msg);
  }
  // pointer checks before the device is touched
  for (const void* ptr : {A, (const void*)U, (const void*)S, (const void*)V})
    if (!ptr || !aligned(ptr, 16)) return fail(TSVD_EINVAL, "null or misaligned (16 B) tensor pointer");
  void* ws = nullptr;
  if ((r = static_scratch(&ws))) return r;
  return svd_call(false, TSVD_OP_RBK, A, nullptr, seed, n1, n2, n3, k, b, q, prec, U, S, V, nullptr, ws,
                  kStaticScratchBytes, stream);
}

int tsvd_rbk_omega(const void* A, const void* Omega, int64_t n1, int64_t n2, int64_t n3, int64_t k, int64_t b,
                   int64_t q, int prec, void* U, void* S, void* V, void* ws, size_t ws_bytes, void* stream) {
  return svd_call(true, TSVD_OP_RBK, A, Omega, 0, n1, n2, n3, k, b, q, prec, U, S, V, nullptr, ws, ws_bytes, stream);
}

int tsvd_rbk_approx(const void* A, int64_t n1, int64_t n2, int64_t n3, int64_t k, int64_t b, int64_t q,
                    uint64_t seed, int prec, void* U, void* S, void* V, void* Xhat, void* ws, size_t ws_bytes,
                    void* stream) {
  return svd_call(false, TSVD_OP_APPROX, A, nullptr, seed, n1, n2, n3, k, b, q, prec, U, S, V, Xhat, ws, ws_bytes, stream);
}

int tsvd_rbk_approx_omega(const void* A, const void* Omega, int64_t n1, int64_t n2, int64_t n3, int64_t k, int64_t b,
                          int64_t q, int prec, void* U, void* S, void* V, void* Xhat, void* ws, size_t ws_bytes,
                          void* stream) {
  return svd_call(true, TSVD_OP_APPROX, A, Omega, 0, n1, n2, n3, k, b, q, prec, U, S, V, Xhat, ws, ws_bytes, stream);
}

int tsvd_power(const void* A, int64_t n1, int64_t n2, int64_t n3, int64_t k, int64_t b, int64_t q, uint64_t seed,
               int prec, void* U, void* S, void* V, void* ws, size_t ws_bytes, void* stream) {
  return svd_call(false, TSVD_OP_POWER, A, nullptr, seed, n1, n2, n3, k, b, q, prec, U, S, V, nullptr, ws, ws_bytes, stream);
}

int tsvd_power_omega(const void* A, const void* Omega, int64_t n1, int64_t n2, int64_t n3, int64_t k, int64_t b,
                     int64_t q, int prec, void* U, void* S, void* V, void* ws, size_t ws_bytes, void* stream) {
  return svd_call(true, TSVD_OP_POWER, A, Omega, 0, n1, n2, n3, k, b, q, prec, U, S, V, nullptr, ws, ws_bytes, stream);
}

int tsvd_power_approx(const void* A, int64_t n1, int64_t n2, int64_t n3, int64_t k, int64_t b, int64_t q,
                      uint64_t seed, int prec, void* U, void* S, void* V, void* Xhat, void* ws, size_t ws_bytes,
                      void* stream) {
  return svd_call(false, TSVD_OP_POWER_APPROX, A, nullptr, seed, n1, n2, n3, k, b, q, prec, U, S, V, Xhat, ws, ws_bytes,
                  stream);
}

int tsvd_power_approx_omega(const void* A, const void* Omega, int64_t n1, int64_t n2, int64_t n3, int64_t k,
                            int64_t b, int64_t q, int prec, void* U, void* S, void* V, void* Xhat, void* ws,
                            size_t ws_bytes, void* stream) {
  return svd_call(true, TSVD_OP_POWER_APPROX, A, Omega, 0, n1, n2, n3, k, b, q, prec, U, S, V, Xhat, ws, ws_bytes, stream);
}

int tsvd_rbk_literal(const void* A, int64_t n1, int64_t n2, int64_t n3, int64_t k, int64_t b, int64_t q,
                     uint64_t seed, int prec, void* U, void* S, void* V, void* Xhat, void* ws, size_t ws_bytes,
                     void* stream) {
  return svd_call(false, TSVD_OP_RBK_LITERAL, A, nullptr, seed, n1, n2, n3, k, b, q, prec, U, S, V, Xhat, ws, ws_bytes,
                  stream);
}

int tsvd_rbk_literal_omega(const void* A, const void* Omega, int64_t n1, int64_t n2, int64_t n3, int64_t k, int64_t b,
                           int64_t q, int prec, void* U, void* S, void* V, void* Xhat, void* ws, size_t ws_bytes,
                           void* stream) {
  return svd_call(true, TSVD_OP_RBK_LITERAL, A, Omega, 0, n1, n2, n3, k, b, q, prec, U, S, V, Xhat, ws, ws_bytes, stream);
}

int tsvd_rbk_ritz(const void* A, int64_t n1, int64_t n2, int64_t n3, int64_t k, int64_t b, int64_t q, uint64_t seed,
                  int prec, void* Qr, void* U, void* S, void* V, void* ws, size_t ws_bytes, void* stream) {
  return ritz_call(false, A, nullptr, seed, n1, n2, n3, k, b, q, prec, Qr, U, S, V, ws, ws_bytes, stream);
}

int tsvd_rbk_ritz_omega(const void* A, const void* Omega, int64_t n1, int64_t n2, int64_t n3, int64_t k, int64_t b,
                        int64_t q, int prec, void* Qr, void* U, void* S, void* V, void* ws, size_t ws_bytes,
                        void* stream) {
  return ritz_call(true, A, Omega, 0, n1, n2, n3, k, b, q, prec, Qr, U, S, V, ws, ws_bytes, stream);
}

int tsvd_rbk_approx_backward(const void* A, const void* G, int64_t n1, int64_t n2, int64_t n3, int64_t k, int64_t b,
                             int64_t q, uint64_t seed, int prec, void* dA, void* ws, size_t ws_bytes, void* stream) {
  return approx_backward_call(false, A, nullptr, seed, G, n1, n2, n3, k, b, q, prec, dA, ws, ws_bytes, stream);
}

int tsvd_rbk_approx_backward_omega(const void* A, const void* Omega, const void* G, int64_t n1, int64_t n2,
                                   int64_t n3, int64_t k, int64_t b, int64_t q, int prec, void* dA, void* ws,
                                   size_t ws_bytes, void* stream) {
  return approx_backward_call(true, A, Omega, 0, G, n1, n2, n3, k, b, q, prec, dA, ws, ws_bytes, stream);
}

int tsvd_tqr(const void* A, int64_t n1, int64_t n2, int64_t n3, int prec, void* Q, void* R, void* ws,
             size_t ws_bytes, void* stream) {
  Plan p;
  int r = make_plan(n1, n2, n3, 1, 1, 0, prec, TSVD_OP_TQR, &p);
  if (r) return r;
  if ((r = check_ptrs({A, Q, R}, ws, ws_bytes, p))) return r;
  Ctx c{p, (unsigned char*)ws, (hipStream_t)stream};
  int nsum = 1;
  if ((r = tqr_core(c, A, &nsum))) return r;
  {
    Timed tm_(K_MISC, c.s);
    HIPCHK(triu_store(c.at<double>(p.o_part), nsum, p.F * p.m * p.n2, (int)p.m, (int)p.n2, (int)p.F, c.at(p.o_rout),
                      p.dt, c.s));
  }
  {
    Timed tm_(K_FFT_INV, c.s);
    HIPCHK(fft_c2r(c.at(p.o_q), p.n1 * p.m, Q, p.n1 * p.m, (int)p.n3, p.dt, c.s));
  }
  {
    Timed tm_(K_FFT_INV, c.s);
    HIPCHK(fft_c2r(c.at(p.o_rout), p.m * p.n2, R, p.m * p.n2, (int)p.n3, p.dt, c.s));
  }
  g_err.clear();
  return TSVD_OK;
}

// Smallest relative cut-off the FP64 Gram resolves: its eigenvalues carry an
// absolute error of about (n1 + n2) u lambda_0 (u = 2^-53), so singular values
// below sqrt((n1 + n2) u) sigma_0 cannot be told from zero; the factor 4 keeps
// the kept values 16x above that level.
double tpinv_floor(int64_t n1, int64_t n2) { return 4.0 * std::sqrt(((double)n1 + (double)n2) * 0x1p-53); }

double tsvd_tpinv_default_rtol(int64_t n1, int64_t n2, int prec) {
  if (n1 < 1 || n2 < 1 || (prec != TSVD_PREC_F64 && prec != TSVD_PREC_F32)) return -1.0;
  const double eps = prec == TSVD_PREC_F64 ? 0x1p-52 : 0x1p-23;
  return std::max((double)std::max(n1, n2) * eps, tpinv_floor(n1, n2));
}

int tsvd_tpinv(const void* A, int64_t n1, int64_t n2, int64_t n3, double rtol, int prec, void* X, void* ws,
               size_t ws_bytes, void* stream) {
  Plan p;
  int r = make_plan(n1, n2, n3, 1, 1, 0, prec, TSVD_OP_TPINV, &p);
  if (r) return r;
  if (std::isnan(rtol)) return fail(TSVD_EINVAL, "rtol is NaN");
  if (rtol <= 0.0)
    rtol = tsvd_tpinv_default_rtol(n1, n2, prec);
  else if (rtol < tpinv_floor(n1, n2))
    return fail(TSVD_EINVAL, "rtol is below 4 sqrt((n1 + n2) 2^-53), the resolution of the FP64 Gram eigensolver");
  if ((r = check_ptrs({A, X}, ws, ws_bytes, p))) return r;
  Ctx c{p, (unsigned char*)ws, (hipStream_t)stream};
  const DType dt = p.dt;
  const int64_t rr = p.m, F = p.F, s12 = n1 * n2;
  const bool tall = n1 >= n2;
  {
    Timed tm_(K_MISC, c.s);
    HIPCHK(zero_info(c.info(), c.s));
  }
  void* Ab = c.at(p.o_abar);
  {
    Timed tm_(K_FFT_A, c.s);
    HIPCHK(fft_r2c(A, Ab, s12, (int)n3, dt, c.s));
  }
  // G_f on the short side: A_f^H A_f = V S^2 V^H (tall) or A_f A_f^H = U S^2 U^H
  double* part = c.at<double>(p.o_part);
  int nsum = 1;
  const bool upper = tall && dt == DT_F32;
  if (tall) {
    if ((r = inner_products(c, Ab, n2, (int)n2, Ab, n2, (int)n2, n1, s12, s12, p.nsplit_g, p.kchunk_g, part, &nsum,
                            K_GEMM_LIFT, upper)))
      return r;
  } else {
    GemmDesc d = gd();
    d.A = Ab;
    d.lda = n2;
    d.strideA = s12;
    d.ta = dt;
    d.B = Ab;
    d.ldb = n2;
    d.strideB = s12;
    d.tb = dt;
    d.b_conj = true;
    d.C = part;
    d.ldc = n1;
    d.strideC = n1 * n1;
    d.tc = DT_F64;
    d.M = (int)n1;
    d.N = (int)n1;
    d.K = (int)n2;
    d.batch = (int)F;
    d.nsplit = p.nsplit_g;
    d.kchunk = p.kchunk_g;
    d.c_split_stride = F * n1 * n1;
    d.compute = DT_F64;
    {
      Timed tm_(K_GEMM_LIFT, c.s);
      HIPCHK(zgemm(d, c.s));
    }
    nsum = p.nsplit_g;
  }
  // all r eigenpairs; those below a quarter of the cut-off get zero vectors
  double* lam = c.at<double>(p.o_lam);
  double* W = c.at<double>(p.o_wd);
  const double thr = rtol * rtol;
  const int stage_cls[4][2] = {
      {HEIG_TRIDIAG, K_HEIG_TRI}, {HEIG_BISECT, K_HEIG_BISECT}, {HEIG_INVIT, K_HEIG_INVIT}, {HEIG_BACKXF, K_HEIG_BACKXF}};
  for (const auto& sc : stage_cls) {
    Timed tm_(sc[1], c.s);
    HIPCHK(heig_topk(part, nsum, F * rr * rr, (int)rr, (int)rr, (int)F, lam, W, c.at(p.o_heig), c.info(), c.s, sc[0],
                     upper, 0.25 * thr));
  }
  // Wg = W diag(s^-2 over the kept values) W^H
  void* Ws = c.at(p.o_wds);
  void* Wg = c.at(p.o_rinv);
  {
    Timed tm_(K_MISC, c.s);
    HIPCHK(pinv_weights(W, lam, Ws, (int)rr, (int)rr, (int)F, thr, c.s));
  }
  if ((r = gemm(c, K_GEMM_LIFT, Op{Ws, rr, rr * rr, DT_F64, false}, Op{W, rr, rr * rr, DT_F64, true}, Wg, rr, rr * rr,
                DT_F64, (int)rr, (int)rr, (int)rr, 1.0, 0.0, DT_F64)))
    return r;
  // X_f^+ = V S^-2 V^H A_f^H = V S^+ U^H (tall), A_f^H U S^-2 U^H (wide)
  void* Xp = c.at(p.o_xp);
  if (tall)
    r = gemm(c, K_GEMM_LIFT, Op{Wg, rr, rr * rr, DT_F64, false}, Op{Ab, n2, s12, dt, true}, Xp, n1, s12, dt, (int)n2,
             (int)n1, (int)n2, 1.0, 0.0, DT_F64);
  else
    r = gemm(c, K_GEMM_LIFT, Op{Ab, n2, s12, dt, true}, Op{Wg, rr, rr * rr, DT_F64, false}, Xp, n1, s12, dt, (int)n2,
             (int)n1, (int)n1, 1.0, 0.0, DT_F64);
  if (r) return r;
  {
    Timed tm_(K_FFT_INV, c.s);
    HIPCHK(fft_c2r(Xp, s12, X, s12, (int)n3, dt, c.s));
  }
  g_err.clear();
  return TSVD_OK;
}

int tsvd_complete(const void* M, const void* mask, int64_t n1, int64_t n2, int64_t n3, int64_t k, int64_t b,
                  int64_t q, uint64_t seed, int64_t iters, int alg, int prec, void* C, void* ws, size_t ws_bytes,
                  void* stream) {
  return complete_call(false, M, mask, nullptr, seed, n1, n2, n3, k, b, q, iters, alg, prec, C, ws, ws_bytes, stream);
}

int tsvd_complete_omega(const void* M, const void* mask, const void* Omega, int64_t n1, int64_t n2, int64_t n3,
                        int64_t k, int64_t b, int64_t q, int64_t iters, int alg, int prec, void* C, void* ws,
                        size_t ws_bytes, void* stream) {
  return complete_call(true, M, mask, Omega, 0, n1, n2, n3, k, b, q, iters, alg, prec, C, ws, ws_bytes, stream);
}

int tsvd_proj(const void* A, int64_t n1, int64_t n2, int64_t n3, int64_t b, int64_t q, uint64_t seed, int prec,
              void* P, void* ws, size_t ws_bytes, void* stream) {
  return proj_call(false, A, nullptr, seed, n1, n2, n3, b, q, prec, P, ws, ws_bytes, stream);
}

int tsvd_proj_omega(const void* A, const void* Omega, int64_t n1, int64_t n2, int64_t n3, int64_t b, int64_t q,
                    int prec, void* P, void* ws, size_t ws_bytes, void* stream) {
  return proj_call(true, A, Omega, 0, n1, n2, n3, b, q, prec, P, ws, ws_bytes, stream);
}

int tsvd_proj_backward(const void* A, const void* G, int64_t n1, int64_t n2, int64_t n3, int64_t b, int64_t q,
                       uint64_t seed, int prec, void* dA, void* ws, size_t ws_bytes, void* stream) {
  return proj_backward_call(false, A, nullptr, seed, G, n1, n2, n3, b, q, prec, dA, ws, ws_bytes, stream);
}

int tsvd_proj_backward_omega(const void* A, const void* Omega, const void* G, int64_t n1, int64_t n2, int64_t n3,
                             int64_t b, int64_t q, int prec, void* dA, void* ws, size_t ws_bytes, void* stream) {
  return proj_backward_call(true, A, Omega, 0, G, n1, n2, n3, b, q, prec, dA, ws, ws_bytes, stream);
}

int tsvd_read_info(const void* ws, int32_t* info_host, void* stream) {
  if (!ws || !info_host) return fail(TSVD_EINVAL, "null pointer");
  hipError_t e = hipMemcpyAsync(info_host, ws, TSVD_INFO_COUNT * sizeof(int32_t), hipMemcpyDeviceToHost,
                                (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return fail(TSVD_EHIP, hipGetErrorString(e));
  if (info_host[TSVD_INFO_CHOL_BREAKDOWN] || info_host[TSVD_INFO_EIG_NOCONV] || info_host[TSVD_INFO_NONFINITE] ||
      info_host[TSVD_INFO_TRUNCATION_TIE]) {
    char msg[256];
    snprintf(msg, sizeof msg, "numerical failure on the device: %d Cholesky breakdowns, %d unconverged eigenvectors, "
             "%d non-finite values, %d ties at the rank-k cut (derivative undefined)",
             info_host[TSVD_INFO_CHOL_BREAKDOWN], info_host[TSVD_INFO_EIG_NOCONV], info_host[TSVD_INFO_NONFINITE],
             info_host[TSVD_INFO_TRUNCATION_TIE]);
    return fail(TSVD_ENUMERIC, msg);
  }
  g_err.clear();
  return TSVD_OK;
}

}  // extern "C"

#include "../../include/tsvd_rbk_diag.h"

extern "C" {

int tsvd_diag_omega(void* out, int64_t n, uint64_t seed, int dtype, void* stream) {
  if (!out || n < 0 || n > ((int64_t)1 << 40) || (dtype != 0 && dtype != 1)) return fail(TSVD_EINVAL, "bad arguments");
  HIPCHK(omega_fill(out, n, seed, dtype == 0 ? DT_F64 : DT_F32, (hipStream_t)stream));
  return TSVD_OK;
}

int tsvd_diag_fft_r2c(const void* X, void* Xb, int64_t ntubes, int64_t n3, int dtype, void* stream) {
  if (!X || !Xb || ntubes < 0 || n3 < 1 || n3 > 4096 || (dtype != 0 && dtype != 1))
    return fail(TSVD_EINVAL, "bad arguments");
  HIPCHK(fft_r2c(X, Xb, ntubes, (int)n3, dtype == 0 ? DT_F64 : DT_F32, (hipStream_t)stream));
  return TSVD_OK;
}

int tsvd_diag_fft_c2r(const void* Xb, void* X, int64_t ntubes, int64_t n3, int dtype, void* stream) {
  if (!X || !Xb || ntubes < 0 || n3 < 1 || n3 > 4096 || (dtype != 0 && dtype != 1))
    return fail(TSVD_EINVAL, "bad arguments");
  HIPCHK(fft_c2r(Xb, ntubes, X, ntubes, (int)n3, dtype == 0 ? DT_F64 : DT_F32, (hipStream_t)stream));
  return TSVD_OK;
}

size_t tsvd_diag_kgemm_ws_bytes(int herm, int64_t rows, int64_t cols, int64_t N, int64_t batch, int mode,
                                int nsplit) {
  if (rows < 1 || cols < 1 || N < 1 || batch < 1 || mode < KM_F32 || mode > KM_BF16X3_SPLIT || nsplit < 1 ||
      !small_volume(rows, cols, 1) || N >= (1 << 20) || batch > 65535)
    return 0;
  const int64_t M = herm ? cols : rows, K = herm ? rows : cols;
  size_t bytes = nsplit > 1 ? align256((size_t)nsplit * batch * M * N * 8) : 0;
  if (mode == KM_BF16) bytes += align256(kgemm_bf16_pack_bytes(mode, (int)K, (int)N, (int)batch));
  else if (nsplit == 1) bytes += align256(kgemm_part_bytes((int)M, (int)K, (int)N, (int)batch, 1));
  return bytes;
}

int tsvd_diag_kgemm(const void* A, int herm, const void* X, void* C, int64_t rows, int64_t cols, int64_t N,
                    int64_t batch, int mode, int nsplit, void* ws, size_t ws_bytes, void* stream) {
  const size_t need = tsvd_diag_kgemm_ws_bytes(herm, rows, cols, N, batch, mode, nsplit);
  if (!A || !X || !C || rows < 1 || cols < 1 || N < 1 || batch < 1 || mode < KM_F32 || mode > KM_BF16X3_SPLIT ||
      nsplit < 1 || nsplit > 64 || !small_volume(rows, cols, 1) || N >= (1 << 20) || batch > 65535)
    return fail(TSVD_EINVAL, "bad arguments");
  if (need > 0 && (!ws || ws_bytes < need || !aligned(ws, 256))) return fail(TSVD_ENOMEM, "workspace too small");
  const int64_t M = herm ? cols : rows, K = herm ? rows : cols;
  KGemmDesc d{};
  d.A = A;
  d.lda = cols;
  d.strideA = rows * cols;
  d.rows = (int)rows;
  d.cols = (int)cols;
  d.herm = herm != 0;
  d.X = X;
  d.ldx = N;
  d.strideX = K * N;
  d.C = C;
  d.ldc = N;
  d.strideC = M * N;
  d.N = (int)N;
  d.batch = (int)batch;
  d.mode = mode;
  d.nsplit = nsplit;
  unsigned char* w = static_cast<unsigned char*>(ws);
  d.part = nsplit > 1 ? w : nullptr;
  d.part_bytes = nsplit > 1 ? (size_t)nsplit * batch * M * N * 8 : 0;
  if (nsplit == 1 && mode != KM_BF16 && need > 0) {
    d.part = w;
    d.part_bytes = need;
  }
  void* pack = w + (nsplit > 1 ? align256((size_t)nsplit * batch * M * N * 8) : 0);
  if (mode == KM_BF16)
    HIPCHK(kgemm_bf16(d, pack, (hipStream_t)stream));
  else
    HIPCHK(kgemm(d, (hipStream_t)stream));
  return TSVD_OK;
}

int tsvd_diag_kgemm_sub(const void* A, const void* X, void* C, int64_t rows, int64_t cols, int64_t N,
                        int64_t batch, void* stream) {
  if (!A || !X || !C || rows < 1 || cols < 1 || N < 1 || batch < 1 || !small_volume(rows, cols, 1) ||
      !small_volume(rows, N, 1) || !small_volume(cols, N, 1) || N >= (1 << 20) || batch > 65535)
    return fail(TSVD_EINVAL, "bad arguments");
  KGemmDesc d{};
  d.A = A;
  d.lda = cols;
  d.strideA = rows * cols;
  d.rows = (int)rows;
  d.cols = (int)cols;
  d.herm = false;
  d.X = X;
  d.ldx = N;
  d.strideX = cols * N;
  d.C = C;
  d.ldc = N;
  d.strideC = rows * N;
  d.N = (int)N;
  d.batch = (int)batch;
  d.mode = KM_F32;
  d.nsplit = 1;
  d.sub = 1;
  HIPCHK(kgemm(d, (hipStream_t)stream));
  return TSVD_OK;
}

int tsvd_diag_split_bf16x3(const void* in, void* out, int64_t n, void* stream) {
  if (!in || !out || n < 1 || n >= ((int64_t)1 << 31) || !aligned(in, 8) || !aligned(out, 8))
    return fail(TSVD_EINVAL, "bad arguments");
  HIPCHK(split_bf16x3(in, out, n, (hipStream_t)stream));
  return TSVD_OK;
}

size_t tsvd_diag_heig_ws_bytes(int64_t m, int64_t k, int64_t batch) {
  if (m < 1 || m > 1024 || k < 1 || k > m || batch < 1 || batch > 65535) return 0;
  return 256 + align256((size_t)batch * heig_scratch_bytes((int)m, (int)k));
}

int tsvd_diag_heig(const void* G, int64_t m, int64_t k, int64_t batch, void* lambda, void* W, void* ws,
                   size_t ws_bytes, void* stream) {
  const size_t need = tsvd_diag_heig_ws_bytes(m, k, batch);
  if (!G || !lambda || !W || need == 0) return fail(TSVD_EINVAL, "bad arguments");
  if (!ws || ws_bytes < need || !aligned(ws, 256)) return fail(TSVD_ENOMEM, "workspace too small");
  const hipStream_t s = (hipStream_t)stream;
  unsigned char* w = static_cast<unsigned char*>(ws);
  int* info = reinterpret_cast<int*>(w);
  HIPCHK(zero_info(info, s));
  HIPCHK(heig_topk(static_cast<const double*>(G), 1, 0, (int)m, (int)k, (int)batch, static_cast<double*>(lambda),
                   static_cast<double*>(W), w + 256, info, s, HEIG_TRIDIAG | HEIG_BISECT | HEIG_INVIT | HEIG_BACKXF,
                   false));
  return TSVD_OK;
}

int tsvd_diag_zgemm(const void* A, int a_conj, const void* B, int b_conj, void* C, int64_t M, int64_t N, int64_t K,
                    int64_t batch, double alpha, double beta, int dtype, void* stream) {
  if (!A || !B || !C || M < 0 || N < 0 || K < 0 || batch < 0 || (dtype != 0 && dtype != 1) || (a_conj && b_conj) ||
      M >= (1 << 30) || N >= (1 << 30) || K >= (1 << 30) || batch > 65535)
    return fail(TSVD_EINVAL, "bad arguments");
  GemmDesc d = gd();
  const DType t = dtype == 0 ? DT_F64 : DT_F32;
  d.A = A;
  d.a_conj = a_conj != 0;
  d.lda = a_conj ? M : K;
  d.strideA = M * K;
  d.ta = t;
  d.B = B;
  d.b_conj = b_conj != 0;
  d.ldb = b_conj ? K : N;
  d.strideB = K * N;
  d.tb = t;
  d.C = C;
  d.ldc = N;
  d.strideC = M * N;
  d.tc = t;
  d.M = (int)M;
  d.N = (int)N;
  d.K = (int)K;
  d.batch = (int)batch;
  d.alpha = alpha;
  d.beta = beta;
  d.compute = t;
  HIPCHK(zgemm(d, (hipStream_t)stream));
  return TSVD_OK;
}

}  // extern "C"

extern "C" {

int tsvd_diag_timing(int enable) {
  std::lock_guard<std::mutex> l(g_timer.mu);
  for (auto& pe : g_timer.pending) {
    g_timer.pool.push_back(pe.second.first);
    g_timer.pool.push_back(pe.second.second);
  }
  g_timer.pending.clear();
  for (int i = 0; i < K_NCLASS; ++i) {
    g_timer.ms[i] = 0;
    g_timer.count[i] = 0;
  }
  g_timer.on = enable != 0;
  return TSVD_OK;
}

int tsvd_diag_timing_read(double* ms_out, int64_t* count_out, int nclass) {
  if (!ms_out || !count_out || nclass < 1) return fail(TSVD_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> l(g_timer.mu);
  for (auto& pe : g_timer.pending) {
    float ms = 0;
    hipError_t e = hipEventSynchronize(pe.second.second);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, pe.second.first, pe.second.second);
    if (e != hipSuccess) return fail(TSVD_EHIP, hipGetErrorString(e));
    g_timer.ms[pe.first] += ms;
    g_timer.count[pe.first] += 1;
    g_timer.pool.push_back(pe.second.first);
    g_timer.pool.push_back(pe.second.second);
  }
  g_timer.pending.clear();
  for (int i = 0; i < nclass; ++i) {
    ms_out[i] = i < K_NCLASS ? g_timer.ms[i] : 0.0;
    count_out[i] = i < K_NCLASS ? g_timer.count[i] : 0;
  }
  return TSVD_OK;
}

}  // extern "C"
