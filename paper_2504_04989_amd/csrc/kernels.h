// Host-side launch interface of the gfx950 kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tsvd {

enum DType { DT_F32 = 0, DT_F64 = 1 };

// Batched complex GEMM on interleaved complex storage:
//   C[f] = alpha * opA(A[f]) * opB(B[f]) + beta * C[f]      (f < batch)
// opA: a_conj == false -> A is M x K (row m at A + m * lda);
//      a_conj == true  -> A is stored K x M and opA = A^H.
// opB: b_conj == false -> B is K x N; b_conj == true -> B stored N x K, opB = B^H.
// b_nsum > 1: B is the sum of b_nsum matrices spaced b_sum_stride elements.
// nsplit > 1: the K range is cut into nsplit chunks of kchunk; chunk s writes
//   alpha * partial product to C + s * c_split_stride (beta must be 0).
// Element counts (lda, strides, ...) are in complex elements.
struct GemmDesc {
  const void* A; int64_t lda, strideA; DType ta; bool a_conj;
  const void* B; int64_t ldb, strideB; DType tb; bool b_conj; int b_nsum; int64_t b_sum_stride;
  void* C; int64_t ldc, strideC; DType tc;
  int M, N, K, batch;
  int nsplit, kchunk; int64_t c_split_stride;
  double alpha, beta;
  DType compute;
};
hipError_t zgemm(const GemmDesc& d, hipStream_t s);

// Krylov products C_f = op(A_f) X_f with the big FP32 complex slice A_f
// (rows x cols, row stride lda, slice stride strideA, complex elements) and a
// thin operand X_f (K x N, row stride ldx); herm: op = ^H (M = cols, K = rows),
// else identity (M = rows, K = cols).  C_f is M x N (row stride ldc).  Modes:
// FP32 MFMA, BF16 (one product), BF16x3 (hi/lo split, three products), FP32
// accumulation.  nsplit > 1 splits K; part must then hold
// nsplit * batch * M * N complex FP32 values (reduced in a fixed order).
// KM_BF16X3_SPLIT: BF16x3 with the big operand already stored as (hi, lo)
// bf16 pairs (fft_r2c_split's output form, 8 bytes per complex element); the
// thin operand is complex FP32 and split as it is staged, as in KM_BF16X3.
// Same products in the same order as KM_BF16X3: the results are bitwise equal.
enum KMode { KM_F32 = 0, KM_BF16 = 1, KM_BF16X3 = 2, KM_BF16X3_SPLIT = 3 };
struct KGemmDesc {
  const void* A; int64_t lda, strideA; int rows, cols; bool herm;
  const void* X; int64_t ldx, strideX;
  void* C; int64_t ldc, strideC;
  int N, batch, mode, nsplit;
  void* part;
  size_t part_bytes;  // size of part; a tail split is used only when it fits
  int sub;            // C -= op(A) X instead of C = op(A) X (no K split, no tail split)
};
hipError_t kgemm(const KGemmDesc& d, hipStream_t s);
// n complex FP32 values -> n (hi, lo) bf16 pairs (the KM_BF16X3_SPLIT form).
hipError_t split_bf16x3(const void* in, void* out, int64_t n, hipStream_t s);
// Bytes of d.part that kgemm uses: nsplit > 1 partials, or (nsplit == 1) the
// partials of the split remainder tiles (0 when there is no tail split).
size_t kgemm_part_bytes(int M, int K, int N, int batch, int nsplit);
// K split (and chunk) that gives the product enough workgroups to fill the chip.
int kgemm_split(int M, int K, int N, int batch, int* kchunk);
// K split (at most 16) of a product with few output tiles: the count that
// minimises rounds x (K steps per split + 6) over the device's workgroup
// slots (two per CU), a workgroup's fixed cost taken as 6 K steps.
int kgemm_split_balanced(int M, int K, int N, int batch);
// BF16 / BF16x3 modes on planar data: the thin operand is first packed into
// `pack` (kgemm_bf16_pack_bytes), partials (nsplit > 1) go to d.part.
hipError_t kgemm_bf16(const KGemmDesc& d, void* pack, hipStream_t s);
size_t kgemm_bf16_pack_bytes(int mode, int K, int N, int batch);
int kgemm_bf16_split(int M, int K, int N, int batch);

// FP64-arithmetic products on FP32-stored complex blocks.
// ogemm_tn: part[f] (M x N, FP64 complex, row-major) = X_f^H Y_f with X_f
//   (K x M, row stride lx) and Y_f (K x N, row stride ly); the K range is split
//   internally and the partial results are summed in a fixed order, so part
//   needs ogemm_tn_part_bytes() bytes and holds the sum in its first
//   batch * M * N entries on return.
// ogemm_nn: C_f (M x N, FP32, row stride ldc) = alpha X_f B_f + beta C_f with
//   X_f (M x K, row stride lx, FP32) and B_f (K x N, FP64, row stride ldb) the
//   sum of nsum matrices spaced bsum_stride complex elements; b_triu: B_f is
//   upper triangular with its zeros stored (their products are skipped).
size_t ogemm_tn_part_bytes(int M, int K, int N, int batch);
// upper = true (square products): only the entries on and above the
// diagonal are guaranteed; whole tiles below it are skipped.
hipError_t ogemm_tn(const float* X, int64_t lx, int64_t strideX, const float* Y, int64_t ly, int64_t strideY,
                    double* part, int M, int N, int K, int batch, hipStream_t s, bool upper = false);
hipError_t ogemm_nn(const float* X, int64_t lx, int64_t strideX, const double* B, int64_t ldb, int64_t strideB,
                    int nsum, int64_t bsum_stride, float* C, int64_t ldc, int64_t strideC, int M, int N, int K,
                    int batch, double alpha, double beta, hipStream_t s,
                    bool b_triu = false);

// Mode-3 real-to-half-spectrum DFT: X (ntubes x n3, tube-contiguous) ->
// Xb (F x ntubes complex, F = n3/2 + 1), slice-major.
hipError_t fft_r2c(const void* X, void* Xb, int64_t ntubes, int n3, DType t, hipStream_t s);
// Inverse: Xb (F x ntubes, slice stride `slice_stride` elements) -> X
// (ntubes x n3 real).  Imaginary parts of DC / Nyquist are ignored.
hipError_t fft_c2r(const void* Xb, int64_t slice_stride, void* X, int64_t ntubes, int n3, DType t, hipStream_t s);
// fft_r2c for FP32 data written as (hi, lo) bf16 pairs per complex value
// (hi = bf16(z), lo = bf16(z - hi), packed re | im << 16 each): the big
// operand of KM_BF16X3_SPLIT.  Only for the register-resident lengths
// (fft_reg_supported); hipErrorNotSupported otherwise.
bool fft_reg_supported(int n3, DType t);
hipError_t fft_r2c_split(const void* X, void* Xb, int64_t ntubes, int n3, hipStream_t s);

// Per-slice b x b Hermitian Gram (sum of nsum FP64 partials, partial s at
// Gpart + s * part_stride complex elements, slice f at + f * b * b) -> inverse
// of its shifted Cholesky factor R (G + shift_coef * trace(G) I = R^H R),
// upper triangular, FP64, b x b row-major per slice.  gscratch: b(b+1)/2
// complex doubles per slice, used when !chol_uses_lds(b).
inline bool chol_uses_lds(int64_t b) { return b * (b + 1) / 2 * 16 <= 120 * 1024; }
// mode 1: the partials sum to an upper triangular R instead; the kernel only
// inverts it (Rinv = R^{-1}).  mode 2 (b <= 128): only the upper triangle of
// the partials is valid; G is its Hermitian extension.
bool chol_blocked_ok(int b);  // the blocked factorisation (and mode 2) applies
hipError_t chol_inv_ex(const double* Gpart, int nsum, int64_t part_stride, double* Rinv, void* gscratch, int b,
                       int batch, double shift_coef, int* info, hipStream_t s, int mode = 0);

// Per-slice m x m Hermitian PSD matrix (sum of nsum FP64 partials): top-k
// eigenpairs.  lambda (batch x k, descending), W (batch x m x k complex FP64).
// `stages` selects which of the four launches to enqueue (they must run in
// this order on one stream, with the same arguments).
enum HeigStage { HEIG_TRIDIAG = 1, HEIG_BISECT = 2, HEIG_INVIT = 4, HEIG_BACKXF = 8, HEIG_ALL = 15 };
size_t heig_scratch_bytes(int m, int k);
// upper_only: only the entries on and above the diagonal of the summed
// partials are valid (the matrix is taken as their Hermitian extension).
// vfloor_rel > 0: eigenvalues lambda_j <= vfloor_rel * lambda_0 get a zero
// vector instead of an inverse iteration.
hipError_t heig_topk(const double* Gpart, int nsum, int64_t part_stride, int m, int k, int batch, double* lambda,
                     double* W, void* scratch, int* info, hipStream_t s, int stages = HEIG_ALL,
                     bool upper_only = false, double vfloor_rel = 0.0);

// Lift helpers.
// Wout (batch x m x k, dtype t) = W * diag(scale) where scale = sqrt(lambda)
// (scale_mode 0), 1/sqrt(lambda) (mode 1, 0 where lambda <= 0) or 1 (mode 2).
hipError_t scale_cols(const double* W, const double* lambda, void* Wout, int m, int k, int batch, int scale_mode,
                      DType t, hipStream_t s);
// Ws = W diag(g), g_c = 1 / lambda_c where lambda_c > thr * lambda_0 and
// lambda_c > 0, else 0 (FP64, batch x m x k, lambda descending per slice).
hipError_t pinv_weights(const double* W, const double* lambda, void* Ws, int m, int k, int batch, double thr,
                        hipStream_t s);
// Phase canonicalisation of (U_f, V_f) column pairs and sigma = sqrt(lambda).
size_t canon_scratch_bytes(int64_t n1, int k, int batch);
hipError_t lift_operands_f32(const double* W, const double* lambda, void* Wf, void* Wsf, int m, int k, int batch,
                             hipStream_t s);
hipError_t canon_phase(void* U, int64_t n1, void* V, int64_t n2, int k, int batch, DType t, void* scratch,
                       hipStream_t s);
// sigma = sqrt(max(lambda, 0)) (FP64) and (sigma, 0) as complex in dtype t.
hipError_t sigma_from_lambda(const double* lambda, double* sigma, void* scx, int64_t n, DType t, hipStream_t s);
// FP64: P (batch x n2 x k, = T_f W_k) -> sigma_j = ||P(:, j)||, V = P / sigma
// in place, sigma (FP64) and (sigma, 0) as complex double.
hipError_t colnorm_sigma(void* P, int64_t n2, int k, int batch, double* sigma, void* scx, hipStream_t s);
// U * diag(sigma): Uout (batch x n1 x k) = Uin * sigma (per slice).
hipError_t scale_cols_by(const void* Uin, const double* sigma, void* Uout, int64_t n1, int k, int batch, DType t,
                         hipStream_t s);
// R (batch x r x n, dtype t) = upper-trapezoidal part of the sum of nsum FP64
// partials (spaced part_stride complex elements); zeros below the diagonal.
hipError_t triu_store(const double* part, int nsum, int64_t part_stride, int r, int n, int batch, void* R, DType t,
                      hipStream_t s);
// C (n elements of dtype t) = mask ? M : X (X == nullptr: 0).
hipError_t masked_merge(const void* M, const unsigned char* mask, const void* X, void* C, int64_t n, DType t,
                        hipStream_t s);
// Second pass of the FP64 small SVD: the number J of the first pass's top-k
// eigenpairs (lam1, W1: m x k per slice) kept per slice, with W1m = W1 whose
// columns from J on are cleared; and the merge of the kept pairs with the
// second pass's (lam2, W2) into lambda and W (m x k).
// Adjoint through the rank-k truncation: per slice, S = N + N^H from
// M (m x m, FP64 complex) and the descending eigenvalues lambda (m):
// S_xy = (M_xy + conj(M_yx)) / (lambda_min(x,y) - lambda_max(x,y)) when
// exactly one of x, y is below k, else 0.  A gap at or below
// rel_tol * lambda_0 gives 0 there and counts in info[INFO_TIE].
hipError_t gap_weights(const void* M, const double* lambda, int m, int k, int batch, double rel_tol, void* S,
                       int* info, hipStream_t s);
hipError_t tail_split(const double* lam1, const void* W1, void* W1m, int m, int k, int batch, double tau,
                      double min_ratio, int* J, hipStream_t s);
hipError_t tail_merge(const double* lam1, const void* W1, const double* lam2, const void* W2, const int* J, int m,
                      int k, int batch, double* lam, void* W, hipStream_t s);
hipError_t zero_info(int* info, hipStream_t s);

// The seeded Gaussian test tensor of Alg. 2 (counter-based: Philox4x32-10 and
// a Box-Muller transform evaluated with a fixed sequence of IEEE double
// operations, identical on the host and the device): n values, element e of
// the stream at out[e], rounded once to dtype t on the device.
hipError_t omega_fill(void* out, int64_t n, uint64_t seed, DType t, hipStream_t s);
void omega_host(double* out, int64_t n, uint64_t seed);

}  // namespace tsvd
