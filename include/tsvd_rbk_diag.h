/*
 * tsvd_rbk_diag.h -- kernel-level entry points of libtsvd_rbk.so, exported so
 * that each building block of Alg. 2 can be checked on its own.  Same
 * conventions as tsvd_rbk.h (device pointers, caller-owned memory, stream
 * ordered, status codes, tsvd_last_error()).
 */
#ifndef TSVD_RBK_DIAG_H
#define TSVD_RBK_DIAG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Mode-3 DFT of real tubes (Sec. 2: fft(X, [], 3), unnormalised, omega =
 * exp(-2 pi i / n3)), first n3/2 + 1 frequencies only (Alg. TP).
 * X: ntubes x n3 real (tube-contiguous).  Xb: (n3/2 + 1) x ntubes complex,
 * interleaved (re, im), slice-major.  dtype: 0 = double, 1 = float. */
int tsvd_diag_fft_r2c(const void* X, void* Xb, int64_t ntubes, int64_t n3, int dtype, void* stream);

/* Inverse (ifft(., [], 3) with the 1/n3, Sec. 2) of a half spectrum completed
 * by conjugate symmetry (Alg. TP); imaginary parts of the DC and Nyquist
 * slices are ignored.  Xb: (n3/2 + 1) x ntubes complex; X: ntubes x n3 real. */
int tsvd_diag_fft_c2r(const void* Xb, void* X, int64_t ntubes, int64_t n3, int dtype, void* stream);

/* Batched complex product C[f] = alpha opA(A[f]) opB(B[f]) + beta C[f]
 * (the per-slice T-product of Sec. 2 / Alg. TP), all operands interleaved
 * complex row-major in the same dtype (0 = double, 1 = float).
 * a_conj = 0: A is M x K; 1: A is stored K x M and opA = A^H.
 * b_conj = 0: B is K x N; 1: B is stored N x K and opB = B^H.
 * Leading dimensions are the row lengths of the stored matrices. */
int tsvd_diag_zgemm(const void* A, int a_conj, const void* B, int b_conj, void* C, int64_t M, int64_t N, int64_t K,
                    int64_t batch, double alpha, double beta, int dtype, void* stream);

/* The Krylov-product kernels alone: C_f = op(A_f) X_f, FP32 complex, batch
 * slices.  A_f: rows x cols (contiguous slices); herm = 0: op = identity,
 * X_f is cols x N, C_f rows x N; herm = 1: op = ^H, X_f is rows x N, C_f
 * cols x N.  mode: 0 FP32 MFMA, 1 BF16 (one product), 2 BF16x3 (split
 * operands, three products), 3 BF16x3 with A already in (hi, lo) bf16 pair
 * form (tsvd_diag_split_bf16x3; X is complex FP32 as for the other modes),
 * bitwise equal to mode 2 on the unsplit A; FP32 accumulation.  nsplit > 1 splits the
 * contraction (partials reduced in a fixed order).  ws: device workspace of
 * tsvd_diag_kgemm_ws_bytes() bytes (256-byte aligned; may be NULL when that
 * is 0). */
size_t tsvd_diag_kgemm_ws_bytes(int herm, int64_t rows, int64_t cols, int64_t N, int64_t batch, int mode,
                                int nsplit);
int tsvd_diag_kgemm(const void* A, int herm, const void* X, void* C, int64_t rows, int64_t cols, int64_t N,
                    int64_t batch, int mode, int nsplit, void* ws, size_t ws_bytes, void* stream);

/* The Krylov-product kernel in its update form, C_f -= A_f X_f (the first
 * Gram-Schmidt pass of the stabilised recursion on FP32 blocks, Alg. 2, with
 * A_f the earlier basis columns and X_f their coefficients): A_f rows x cols,
 * X_f cols x N, C_f rows x N, FP32 complex, contiguous slices; FP32 MFMA with
 * FP32 accumulation, no split of the contraction.  Device pointers; C is
 * read and written; asynchronous on stream.  TSVD_EINVAL on bad sizes. */
int tsvd_diag_kgemm_sub(const void* A, const void* X, void* C, int64_t rows, int64_t cols, int64_t N,
                        int64_t batch, void* stream);

/* n complex FP32 values (interleaved re, im) -> n (hi, lo) bf16 pairs, the
 * operand form of mode 3 above: hi = bf16(z) and lo = bf16(z - hi) per part
 * (round to nearest even), stored as two 32-bit words re | im << 16 (8 bytes
 * per value, like the input).  in, out: device pointers, 8-byte aligned, may
 * not overlap partially (in == out is allowed).  Asynchronous on stream. */
int tsvd_diag_split_bf16x3(const void* in, void* out, int64_t n, void* stream);

/* The small Hermitian eigensolver alone (the per-slice SVD of C_f in Alg. 2
 * taken through C_f C_f^H, FP64): the k largest eigenvalues (descending) and
 * their eigenvectors of batch Hermitian m x m matrices G (interleaved
 * complex double, row-major, contiguous; the kernel uses the Hermitian part
 * (G + G^H) / 2).  lambda: batch x k doubles; W: batch x m x k complex
 * double, row-major.  ws: device workspace of tsvd_diag_heig_ws_bytes()
 * bytes, 256-byte aligned; its first TSVD_INFO_COUNT ints hold the
 * diagnostic counters (tsvd_read_info). */
size_t tsvd_diag_heig_ws_bytes(int64_t m, int64_t k, int64_t batch);
int tsvd_diag_heig(const void* G, int64_t m, int64_t k, int64_t batch, void* lambda, void* W, void* ws,
                   size_t ws_bytes, void* stream);

/* The seeded test tensor of Alg. 2 as the seed-taking entry points draw it on
 * the device: out (device, n values of dtype 0 = double / 1 = float) receives
 * values 0 .. n-1 of the stream that tsvd_omega writes on the host for the
 * same seed (FP32: those values rounded once). */
int tsvd_diag_omega(void* out, int64_t n, uint64_t seed, int dtype, void* stream);

/* Event timer over the kernels of the entry points in tsvd_rbk.h.
 * tsvd_diag_timing(1) clears the counters and starts recording a pair of HIP
 * events on the caller's stream around every launch; (0) stops.
 * tsvd_diag_timing_read synchronises on the recorded events and returns, per
 * kernel class, the summed duration in ms and the number of launches.
 * Classes: 0 mode-3 DFT of A, 1 DFT of Omega, 2 Krylov products
 * (A_f X and A_f^H Y), 3 orthonormalisation products, 4 Cholesky,
 * 5 tridiagonalisation of the small Hermitian eigenproblem, 6 Gram of C and
 * lift products, 7 inverse DFTs, 8 other, 9 eigenvalue bisection,
 * 10 inverse iteration, 11 eigenvector back-transformation. */
#define TSVD_DIAG_NCLASS 12
int tsvd_diag_timing(int enable);
int tsvd_diag_timing_read(double* ms_out, int64_t* count_out, int nclass);

#ifdef __cplusplus
}
#endif

#endif
