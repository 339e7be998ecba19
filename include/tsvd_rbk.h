/*
 * tsvd_rbk.h -- C ABI of the MI355X (gfx950) randomized block Krylov
 * truncated T-SVD library (libtsvd_rbk.so).
 *
 * Method: M. Nobakht Kooshkghazi, S. Ahmadi-Asl, A. L. F. de Almeida,
 * "Randomized block Krylov method for approximation of truncated tensor SVD",
 * arXiv:2504.04989, Alg. 2 (proposed method) and the classical randomized
 * power-iteration method it is compared with (Alg. 1), with the T-product /
 * T-QR / T-SVD machinery of Sec. 2 (Alg. TP, Alg. TQR).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Tensors are real, C-contiguous (n1, n2, n3): element (i, j, t) sits at
 * (i * n2 + j) * n3 + t, so every tube X(i, j, :) is contiguous.  A tensor
 * written "p x r x n3" uses the same rule with (p, r, n3).
 *
 * Pointers named A, Omega, G, U, S, V, Xhat, P, Qr, dA and ws are DEVICE pointers
 * on the current HIP device.  The caller owns all of them; the library never
 * allocates or frees device memory and never keeps a pointer after return.
 * Inputs are read only.  Outputs may not alias inputs or each other.
 *
 * Element type of A, Omega, G and of every output: double for
 * TSVD_PREC_F64, float for the other precisions.  Every pointer must be
 * 16-byte aligned; ws must be 256-byte aligned.
 *
 * `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 * work is enqueued on it; the call returns without synchronising.  Results
 * are valid once the stream has reached the point of the call.
 *
 * Omega is the Gaussian test tensor of Alg. 2 (n2 x b x n3; the algorithm's
 * first line reads randn(n1, ...), but the product X * Omega needs n2 rows, as
 * in Alg. 1).  The entry points named after the paper's operations take a
 * 64-bit `seed` and draw Omega themselves, on the device, into the workspace
 * (tsvd_omega gives the same numbers on the host).  Each has an `_omega` twin
 * that takes Omega as a device tensor instead (for tests with arbitrary test
 * tensors).  The same (A, seed) or (A, Omega) always gives the same result.
 *
 * Parameters: k = target tubal rank (R in the paper), b = block width
 * (R + P: rank plus oversampling), q = number of Krylov steps.
 * m = b (q + 1) is the number of basis columns per Fourier slice (Alg. 2;
 * for Alg. 1, q counts power iterations and m = b).
 * Requirements (else TSVD_EINVAL, nothing enqueued):
 *   n1, n2, n3 >= 1;  1 <= k <= b;  q >= 0;  m <= min(n1, n2);
 *   n1 * n2 < 2^31;  n1 * n2 * n3 < 2^36;  m <= 1024;  n3 <= 4096;
 *   q <= 4096 for Alg. 1.
 *
 * Errors: every entry point returns a status.  TSVD_EINVAL (bad arguments),
 * TSVD_ENOMEM (ws_bytes below tsvd_workspace_bytes), TSVD_EHIP (a HIP launch
 * or runtime call failed; nothing more is enqueued).  Numerical events found
 * on the device (Cholesky shifts, a breakdown, an eigensolver that did not
 * converge, non-finite values) are counted in the workspace; the calls are
 * asynchronous, so they are reported by tsvd_read_info(), which returns
 * TSVD_ENUMERIC when a breakdown, an unconverged eigenvector or a non-finite
 * value was met.  tsvd_last_error() gives a message for the last non-zero
 * status returned on the calling thread.
 *
 * Internal precision: Gram matrices, Cholesky factors, re-orthogonalisation
 * coefficients and the small Hermitian eigenproblem are always FP64, and the
 * mode-3 transforms compute in FP64 (rounded once to the storage type).
 * `prec` names the storage type and the arithmetic of the Krylov products
 * A_f X and A_f^H Y (Alg. 2: the block Krylov space and C_f = Q_f^H A_f):
 *   TSVD_PREC_F64     FP64 storage, FP64 MFMA
 *   TSVD_PREC_F32     FP32 storage, FP32 MFMA
 *   TSVD_PREC_BF16    FP32 storage, products on BF16 MFMA (one product of the
 *                     bf16-rounded operands), FP32 accumulation
 *   TSVD_PREC_BF16X3  FP32 storage, each operand split x = hi + lo into two
 *                     bf16 numbers, hi*hi + hi*lo + lo*hi on BF16 MFMA, FP32
 *                     accumulation (about 16 significant bits per product)
 * The orthonormalisation products (block Grams, projections against the
 * earlier blocks, application of R^{-1}) and G_f = C_f C_f^H use FP64
 * arithmetic on the stored values in every mode; the lift (U_f = Q_f W_k,
 * V_f = C_f^H W_k / sigma) and the adjoint's other products use the storage
 * type's arithmetic.  With TSVD_PREC_F64 the small SVD takes a second pass
 * (the leading eigenpairs of G_f projected out, the rest solved again) so
 * that singular values far below sqrt(u) sigma_1 keep FP64 accuracy.
 */
#ifndef TSVD_RBK_H
#define TSVD_RBK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define TSVD_OK 0
#define TSVD_EINVAL 1
#define TSVD_ENOMEM 2
#define TSVD_EHIP 3
#define TSVD_ENUMERIC 4

/* precision of the transforms and of the large products */
#define TSVD_PREC_F64 0    /* see "Internal precision" above */
#define TSVD_PREC_F32 1
#define TSVD_PREC_BF16 2
#define TSVD_PREC_BF16X3 3

/* operations, for tsvd_workspace_bytes */
#define TSVD_OP_RBK 0
#define TSVD_OP_APPROX 1
#define TSVD_OP_PROJ 2
#define TSVD_OP_PROJ_BWD 3
#define TSVD_OP_POWER 4
#define TSVD_OP_POWER_APPROX 5
#define TSVD_OP_TQR 6     /* k, b, q ignored */
#define TSVD_OP_TPINV 7   /* k, b, q ignored */
#define TSVD_OP_COMPLETE_RBK 8    /* tsvd_complete with alg = 2 */
#define TSVD_OP_COMPLETE_POWER 9  /* tsvd_complete with alg = 1 */
#define TSVD_OP_RBK_LITERAL 10    /* tsvd_rbk_literal */
#define TSVD_OP_RBK_RITZ 11       /* tsvd_rbk_ritz */
#define TSVD_OP_APPROX_BWD 12     /* tsvd_rbk_approx_backward */

/* diagnostic counters returned by tsvd_read_info (int32 each) */
#define TSVD_INFO_CHOL_SHIFTED 0   /* shifted Cholesky passes whose shift rescued a
                                      pivot (unshifted pivot <= shift: the block
                                      is numerically rank deficient); not an
                                      error */
#define TSVD_INFO_CHOL_BREAKDOWN 1 /* pivots still non-positive after the shift */
#define TSVD_INFO_EIG_NOCONV 2     /* eigenvectors that did not converge        */
#define TSVD_INFO_NONFINITE 3      /* non-finite values met                     */
#define TSVD_INFO_TRUNCATION_TIE 4 /* tsvd_rbk_approx_backward: pairs of eigenvalues
                                      across the rank-k cut closer than their
                                      rounding level (derivative undefined) */
#define TSVD_INFO_COUNT 8

/* Library version (major * 10000 + minor * 100 + patch). */
int tsvd_version(void);

/* Message for the last non-zero status returned on this thread ("" if none).
 * The string is owned by the library and valid until the next call on the
 * same thread. */
const char* tsvd_last_error(void);

/* Bytes of device workspace needed by operation `op` (TSVD_OP_*) for these
 * sizes and precision; 0 if the arguments are invalid.  Pure host function. */
size_t tsvd_workspace_bytes(int64_t n1, int64_t n2, int64_t n3, int64_t k,
                            int64_t b, int64_t q, int prec, int op);

/* The seeded Gaussian test tensor of Alg. 2 (its first step, randn), on the
 * host: out_host (n2 x b x n3 doubles, host memory owned by the caller)
 * receives the tensor that the seed-taking entry points draw on the device
 * for the same (n2, b, n3, seed), bit for bit (the FP32 modes use these
 * values rounded to float).  Element e = (j b + c) n3 + t is value e of a
 * counter-based stream: pair e / 2 of Philox4x32-10 (Salmon et al., SC'11;
 * counter = pair index, key = seed) through a Box-Muller transform whose
 * logarithm, sine, cosine and square root are fixed sequences of IEEE double
 * operations.  n2 * b * n3 <= 2^40, else TSVD_EINVAL.  Pure host function. */
int tsvd_omega(int64_t n2, int64_t b, int64_t n3, uint64_t seed, double* out_host);

/* Alg. 2: randomized block Krylov truncated T-SVD.
 * In:  A (n1 x n2 x n3); the test tensor Omega (n2 x b x n3) is drawn from
 *      seed as tsvd_omega does, into the workspace.
 * Out: U (n1 x k x n3), S (k x n3: the k diagonal tubes of the f-diagonal
 *      S_R, row j is the tube S(j, j, :)), V (n2 x k x n3), with
 *      A ~ U * S * V^T (T-product, Sec. 2).
 * Per Fourier slice f = 0 .. n3/2 (conjugate symmetry gives the others,
 * Alg. TP): the block Krylov space [A_f Om_f, (A_f A_f^H) A_f Om_f, ...,
 * (A_f A_f^H)^q A_f Om_f] is built block by block, each block orthonormalised
 * against the earlier ones (same space as the literal powers in exact
 * arithmetic); C_f = Q_f^H A_f; top-k SVD of C_f; U_f = Q_f W_k,
 * V_f = right singular vectors.  Each column pair (U_f(:, j), V_f(:, j)) is
 * scaled by one unit phase so that the largest-modulus entry of U_f(:, j)
 * (first on ties) is real and positive. */
int tsvd_rbk(const void* A, int64_t n1, int64_t n2, int64_t n3, int64_t k,
             int64_t b, int64_t q, uint64_t seed, int prec, void* U, void* S,
             void* V, void* ws, size_t ws_bytes, void* stream);
/* tsvd_rbk for callers that cannot allocate (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and outputs as tsvd_rbk (same kernels, bit-identical results)
 * with no workspace argument and no allocation of any kind.  Its scratch is
 * a static device array of TSVD_NOALLOC_SCRATCH_BYTES (64 MiB) that
 * every device the library runs on holds until the process ends; sizes whose
 * tsvd_workspace_bytes(..., TSVD_OP_RBK) exceeds it return TSVD_ENOMEM with
 * nothing enqueued.  All calls on one device share that device's array and
 * it keeps the last call's contents (each call clears what it needs
 * cleared): calls that overlap on one device, on different streams or from
 * different threads, race and must be serialised by the caller.
 * tsvd_read_info does not apply (the scratch has no caller-visible handle). */
int tsvd_rbk_noalloc(const void* A, int64_t n1, int64_t n2, int64_t n3,
                     int64_t k, int64_t b, int64_t q, uint64_t seed, int prec,
                     void* U, void* S, void* V, void* stream);
#define TSVD_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* tsvd_rbk with the test tensor given: Omega (n2 x b x n3, device). */
int tsvd_rbk_omega(const void* A, const void* Omega, int64_t n1, int64_t n2,
                   int64_t n3, int64_t k, int64_t b, int64_t q, int prec,
                   void* U, void* S, void* V, void* ws, size_t ws_bytes,
                   void* stream);

/* Alg. 2 followed by the rank-k approximation Xhat = U * S * V^T
 * (n1 x n2 x n3), which equals Q * (Q^T * A)_k (Lemma mn38).  U, S and V
 * are written as in tsvd_rbk and may not be NULL. */
int tsvd_rbk_approx(const void* A, int64_t n1, int64_t n2, int64_t n3,
                    int64_t k, int64_t b, int64_t q, uint64_t seed, int prec,
                    void* U, void* S, void* V, void* Xhat, void* ws,
                    size_t ws_bytes, void* stream);
int tsvd_rbk_approx_omega(const void* A, const void* Omega, int64_t n1,
                          int64_t n2, int64_t n3, int64_t k, int64_t b,
                          int64_t q, int prec, void* U, void* S, void* V,
                          void* Xhat, void* ws, size_t ws_bytes, void* stream);

/* Alg. 2 with the Krylov blocks exactly as the algorithm writes them:
 * K_0 = A_f Om_f and K_i = A_f (A_f^H K_{i-1}), none orthonormalised before
 * the next product, then the T-QR of K = [K_0 .. K_q] (block by block, the
 * same span as one QR of K), C_f, small SVD, lift and phase as tsvd_rbk.  In
 * exact arithmetic it equals tsvd_rbk; in floating point each raw block K_i
 * carries only the directions whose sigma_j / sigma_1 exceeds about the
 * working precision to the power 1 / (2i + 1), so the later blocks add less
 * than tsvd_rbk's orthonormalised recursion does.  Offered for comparison.  The raw blocks grow like sigma_1^(2i): A should be
 * scaled so that sigma_1^(2q+1) stays within the working precision's range.
 * Xhat (n1 x n2 x n3) may be NULL; otherwise it receives U * S * V^T.
 * Workspace: tsvd_workspace_bytes(..., TSVD_OP_RBK_LITERAL). */
int tsvd_rbk_literal(const void* A, int64_t n1, int64_t n2, int64_t n3,
                     int64_t k, int64_t b, int64_t q, uint64_t seed, int prec,
                     void* U, void* S, void* V, void* Xhat, void* ws,
                     size_t ws_bytes, void* stream);
int tsvd_rbk_literal_omega(const void* A, const void* Omega, int64_t n1,
                           int64_t n2, int64_t n3, int64_t k, int64_t b,
                           int64_t q, int prec, void* U, void* S, void* V,
                           void* Xhat, void* ws, size_t ws_bytes, void* stream);

/* Alg. 2 with the basis truncated to k + p columns before the projection
 * (the timing remark of Sec. 5, Ex. 1: "Q truncated to k + p terms"), read as
 * a Rayleigh-Ritz reduction: per Fourier slice, the block Krylov basis Q_f
 * (n1 x m) of tsvd_rbk and C_f = Q_f^H A_f give the top b = k + p left
 * singular vectors W_b of C_f, and Q_r = Q_f W_b (n1 x b, columns in the
 * phase rule of tsvd_rbk); then Alg. 2's projection C_r = Q_r^H A_f (one more
 * b-column product over A_f), small SVD, lift and truncation to k run on Q_r.
 * The rank-k result equals tsvd_rbk's in exact arithmetic (the singular values
 * of C_r are the b largest of C_f).
 * Out: Qr (n1 x b x n3, the truncated basis as an orthonormal tensor,
 *      Qr^T * Qr = I), U, S, V as for tsvd_rbk.  Arguments, errors and
 * workspace (tsvd_workspace_bytes(..., TSVD_OP_RBK_RITZ)) otherwise as
 * tsvd_rbk; 1 <= k <= b. */
int tsvd_rbk_ritz(const void* A, int64_t n1, int64_t n2, int64_t n3, int64_t k,
                  int64_t b, int64_t q, uint64_t seed, int prec, void* Qr,
                  void* U, void* S, void* V, void* ws, size_t ws_bytes,
                  void* stream);
int tsvd_rbk_ritz_omega(const void* A, const void* Omega, int64_t n1,
                        int64_t n2, int64_t n3, int64_t k, int64_t b,
                        int64_t q, int prec, void* Qr, void* U, void* S,
                        void* V, void* ws, size_t ws_bytes, void* stream);

/* Alg. 1: classical randomized subspace method with q power iterations.
 * Same arguments, layouts and outputs as tsvd_rbk, but the basis Q_f
 * (n1 x b per Fourier slice) spans only the last power iterate
 * (A_f A_f^H)^q A_f Om_f; each iterate is orthonormalised before the next
 * multiplication (the same range as the literal powers in exact arithmetic).
 * Projection, small SVD, lift, truncation and phase rule as in tsvd_rbk. */
int tsvd_power(const void* A, int64_t n1, int64_t n2, int64_t n3, int64_t k,
               int64_t b, int64_t q, uint64_t seed, int prec, void* U,
               void* S, void* V, void* ws, size_t ws_bytes, void* stream);
int tsvd_power_omega(const void* A, const void* Omega, int64_t n1, int64_t n2,
                     int64_t n3, int64_t k, int64_t b, int64_t q, int prec,
                     void* U, void* S, void* V, void* ws, size_t ws_bytes,
                     void* stream);

/* Alg. 1 followed by the rank-k approximation Xhat = U * S * V^T
 * (n1 x n2 x n3), as tsvd_rbk_approx does for Alg. 2. */
int tsvd_power_approx(const void* A, int64_t n1, int64_t n2, int64_t n3,
                      int64_t k, int64_t b, int64_t q, uint64_t seed,
                      int prec, void* U, void* S, void* V, void* Xhat,
                      void* ws, size_t ws_bytes, void* stream);
int tsvd_power_approx_omega(const void* A, const void* Omega, int64_t n1,
                            int64_t n2, int64_t n3, int64_t k, int64_t b,
                            int64_t q, int prec, void* U, void* S, void* V,
                            void* Xhat, void* ws, size_t ws_bytes,
                            void* stream);

/* Alg. TQR: economy T-QR A = Q * R (Sec. 2).
 * In:  A (n1 x n2 x n3).  Out: Q (n1 x r x n3) with Q^T * Q = I, and
 * R (r x n2 x n3) whose Fourier slices are upper trapezoidal, r = min(n1, n2).
 * Per Fourier slice f = 0 .. n3/2: Q_f orthonormalises the first r columns of
 * A_f (shifted CholeskyQR, FP64 Grams and factors) and R_f = Q_f^H A_f, zero
 * below the diagonal; conjugate symmetry gives the other slices.  The
 * diagonal of every R_f is real and positive, which makes the factorisation
 * unique; the first r columns of each A_f must be linearly independent (a
 * breakdown is counted in TSVD_INFO_CHOL_BREAKDOWN).
 * prec: TSVD_PREC_F64 or TSVD_PREC_F32 (storage and the Q, R products; the
 * Grams are FP64).  Requirements: min(n1, n2) <= 1024, n3 <= 4096,
 * n1 * n2 < 2^31, n1 * n2 * n3 < 2^36.  Workspace:
 * tsvd_workspace_bytes(n1, n2, n3, 0, 0, 0, prec, TSVD_OP_TQR). */
int tsvd_tqr(const void* A, int64_t n1, int64_t n2, int64_t n3, int prec,
             void* Q, void* R, void* ws, size_t ws_bytes, void* stream);

/* Alg. mp: Moore-Penrose T-pseudoinverse X = A^+ (n2 x n1 x n3, Sec. 2), the
 * tensor with A*X*A = A, X*A*X = X and A*X, X*A symmetric, for any shape and
 * rank.  Per Fourier slice f = 0 .. n3/2 the Gram on the short side,
 * G_f = A_f^H A_f (n1 >= n2) or A_f A_f^H (n1 < n2), r = min(n1, n2), gives
 * all r eigenpairs (FP64 Hermitian eigensolver); a singular value
 * s_j = sqrt(lambda_j) counts as nonzero when s_j > rtol * s_1(A_f), and
 * X_f = W diag(s^-2 over those) W^H A_f^H (tall) or A_f^H W diag(...) W^H
 * (wide), which is V S^+ U^H, the matrix form of A^+ = V * S^+ * U^T
 * (S^+ inverts the nonzero tubes of S, Sec. 2); conjugate symmetry gives the
 * other slices (Alg. mp, second loop).
 * rtol: relative cut-off; rtol <= 0 takes tsvd_tpinv_default_rtol(n1, n2,
 * prec).  The Gram squares the spectrum, so singular values below about
 * sqrt((n1 + n2) 2^-53) s_1 are not resolved: an rtol below
 * 4 sqrt((n1 + n2) 2^-53) returns TSVD_EINVAL, and a kept singular value
 * s_j carries a relative error of about (n1 + n2) 2^-53 (s_1 / s_j)^2.
 * prec: TSVD_PREC_F64 or TSVD_PREC_F32 (storage and the final product; the
 * Gram, eigensolver and weights are FP64).  Requirements:
 * min(n1, n2) <= 1024, n3 <= 4096, n1 * n2 < 2^31, n1 * n2 * n3 < 2^36.  A
 * slice whose eigenvector iteration did not converge is counted in
 * TSVD_INFO_EIG_NOCONV.  Workspace: tsvd_workspace_bytes(n1, n2, n3, 0, 0,
 * 0, prec, TSVD_OP_TPINV). */
int tsvd_tpinv(const void* A, int64_t n1, int64_t n2, int64_t n3, double rtol,
               int prec, void* X, void* ws, size_t ws_bytes, void* stream);

/* Default relative cut-off of tsvd_tpinv: max(max(n1, n2) eps,
 * 4 sqrt((n1 + n2) 2^-53)) with eps the machine epsilon of the data
 * (2^-52 for TSVD_PREC_F64, 2^-23 for TSVD_PREC_F32), the usual matrix pinv
 * tolerance raised to what the FP64 Gram resolves.  Returns -1 for invalid
 * arguments.  Host only. */
double tsvd_tpinv_default_rtol(int64_t n1, int64_t n2, int prec);

/* Completion of Sec. 5, Example 3: alternate a rank-k approximation and the
 * data constraint,
 *   C^(0)   = T (.) M,
 *   X^(n)   = Alg. 2 (alg = 2) or Alg. 1 (alg = 1) rank-k approximation of
 *             C^(n) with test tensor Omega (the same Omega at every step),
 *   C^(n+1) = T (.) M + (1 - T) (.) X^(n),
 * and write C^(iters) to C (n1 x n2 x n3): observed entries equal M, missing
 * entries come from the last approximation.
 * M: the data (n1 x n2 x n3; entries where T is 0 are not read).  mask: T as
 * n1 x n2 x n3 bytes in the same layout (device pointer; 0 = missing,
 * non-zero = observed).  seed (Omega drawn once, used at every step), k, b,
 * q and prec as for tsvd_rbk / tsvd_power; tsvd_complete_omega takes Omega
 * (n2 x b x n3) instead.  iters in [0, 10^6].  Workspace:
 * tsvd_workspace_bytes(..., TSVD_OP_COMPLETE_RBK or TSVD_OP_COMPLETE_POWER).
 * tsvd_read_info reports the counters of the last iteration. */
int tsvd_complete(const void* M, const void* mask, int64_t n1, int64_t n2,
                  int64_t n3, int64_t k, int64_t b, int64_t q, uint64_t seed,
                  int64_t iters, int alg, int prec, void* C, void* ws,
                  size_t ws_bytes, void* stream);
int tsvd_complete_omega(const void* M, const void* mask, const void* Omega,
                        int64_t n1, int64_t n2, int64_t n3, int64_t k,
                        int64_t b, int64_t q, int64_t iters, int alg,
                        int prec, void* C, void* ws, size_t ws_bytes,
                        void* stream);

/* Projection P(A) = Q * Q^T * A (n1 x n2 x n3), Q the T-orthonormal basis of
 * the block Krylov tensor of Alg. 2 (the projector of Thm. mn44 and
 * Lemma mn38; no truncation), the test tensor drawn from seed. */
int tsvd_proj(const void* A, int64_t n1, int64_t n2, int64_t n3, int64_t b,
              int64_t q, uint64_t seed, int prec, void* P, void* ws,
              size_t ws_bytes, void* stream);
int tsvd_proj_omega(const void* A, const void* Omega, int64_t n1, int64_t n2,
                    int64_t n3, int64_t b, int64_t q, int prec, void* P,
                    void* ws, size_t ws_bytes, void* stream);

/* Adjoint of the projection: given G = dL/dP (n1 x n2 x n3), writes
 * dA = dL/dA (n1 x n2 x n3) for L(P(A)).  The Krylov blocks are recomputed
 * from A and Omega, not stored.  Derivative of the map defined by tsvd_proj;
 * for the real inner product sum_ijt x_ijt y_ijt (Sec. 2). */
int tsvd_proj_backward(const void* A, const void* G, int64_t n1, int64_t n2,
                       int64_t n3, int64_t b, int64_t q, uint64_t seed,
                       int prec, void* dA, void* ws, size_t ws_bytes,
                       void* stream);
int tsvd_proj_backward_omega(const void* A, const void* Omega, const void* G,
                             int64_t n1, int64_t n2, int64_t n3, int64_t b,
                             int64_t q, int prec, void* dA, void* ws,
                             size_t ws_bytes, void* stream);

/* Adjoint through the rank-k truncation: given G = dL/dXhat (n1 x n2 x n3),
 * writes dA = dL/dA (n1 x n2 x n3) for L(Xhat(A)), Xhat = U * S * V^T the
 * rank-k result of Alg. 2 with the test tensor of seed (= Q * (Q^T * A)_k,
 * Lemma mn38), real inner product sum_ijt x_ijt y_ijt.  Per Fourier slice
 * the truncation enters through the projector onto the top-k eigenvectors
 * of C_f C_f^H (all m eigenpairs are formed, FP64); the Krylov blocks are
 * recomputed from A and Omega.  The derivative exists where lambda_k >
 * lambda_{k+1} in every slice: eigenvalue pairs across the cut closer than
 * 8 m 2^-53 lambda_1 contribute nothing and are counted in
 * TSVD_INFO_TRUNCATION_TIE (tsvd_read_info then returns TSVD_ENUMERIC).
 * Arguments as tsvd_rbk (1 <= k <= b) plus G and dA (device, A's layout and
 * type); workspace tsvd_workspace_bytes(..., TSVD_OP_APPROX_BWD). */
int tsvd_rbk_approx_backward(const void* A, const void* G, int64_t n1,
                             int64_t n2, int64_t n3, int64_t k, int64_t b,
                             int64_t q, uint64_t seed, int prec, void* dA,
                             void* ws, size_t ws_bytes, void* stream);
int tsvd_rbk_approx_backward_omega(const void* A, const void* Omega,
                                   const void* G, int64_t n1, int64_t n2,
                                   int64_t n3, int64_t k, int64_t b, int64_t q,
                                   int prec, void* dA, void* ws,
                                   size_t ws_bytes, void* stream);

/* Copy the TSVD_INFO_COUNT diagnostic counters of the last call that used
 * workspace `ws` into info_host (host memory).  Synchronises `stream`.
 * Returns TSVD_ENUMERIC (counters still copied) when that call met a
 * Cholesky breakdown, an unconverged eigenvector or a non-finite value. */
int tsvd_read_info(const void* ws, int32_t* info_host, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* TSVD_RBK_H */
