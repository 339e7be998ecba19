"""FP64 CPU oracle for the randomized block Krylov truncated T-SVD.

Paper: M. Nobakht Kooshkghazi, S. Ahmadi-Asl, A. L. F. de Almeida,
"Randomized block Krylov method for approximation of truncated tensor SVD"
(arXiv:2504.04989).

TEST INFRASTRUCTURE ONLY.  This module is imported by ``tests/``, by
``__graft_entry__.smoke()`` and by the ``cpu_baseline`` leg of ``bench.py``;
nothing in the library package imports, links or executes it, and it shares
no code with the HIP path.  It is deliberately plain: numpy in float64 /
complex128, explicit loops where the paper's definitions are loops, numpy's
matmul / norm as the only library primitives, no blocking and no reordering.

Every function names the passage of the paper it writes out.  The readings
taken where the paper is silent, ambiguous or garbled are listed at the end of
this docstring; each one is also recorded in the repository's design notes.

Pins (tests/test_oracle_*.py, all ``-m "not gpu"``):
  dft_mode3 / idft_mode3   impulse and pure-exponential closed forms, numpy.fft,
                           Parseval (eq. (eq_fou)), round trip, real DC/Nyquist
  tprod                    brute force fold(bcirc(X) unfold(Y)) (Def. T-product)
  ttranspose               (X*Y)^T = Y^T*X^T and bcirc(X^T) = bcirc(X)^T
  householder_qr           Q^H Q = I, QR = K, triangular R, numpy.linalg.qr
  jacobi_svd               numpy.linalg.svd singular values, W S Z^H = C
  rbk_tsvd                 m = n1 gives the exact truncated T-SVD; exact recovery
                           of a tubal-rank-r tensor (r <= k); n3 = 1 is the matrix
                           block Krylov method; Eckart-Young; Lemma mn38;
                           the Frobenius theorem of Sec. 4; monotone in q;
                           literal == stabilised Krylov form
  proj / proj_backward     central finite differences, torch CPU autograd,
                           Euler homogeneity
  approx_backward          central finite differences, torch CPU autograd
                           through QR and a Hermitian eigendecomposition,
                           Euler homogeneity, k = m equals proj_backward
  ritz_tsvd                the singular values of Q_r^T * A are the top r of
                           Q^T * A (Rayleigh-Ritz), the rank-k result equals
                           Alg. 2's, Q_r^T * Q_r = I and Q * Q^T * Q_r = Q_r
                           with spatial T-products, r = m spans Q
  tqr / tpinv              X = Q * R and Q^T * Q = I with spatial T-products,
                           triangular slices with a real non-negative
                           diagonal, numpy QR at n3 = 1; the four Penrose
                           conditions with spatial T-products (full rank,
                           rank deficient, wide), X^+ * X = I for full column
                           rank; at n3 = 1 a matrix with known singular values
                           gives V_r diag(1/s_r) U_r^H on either side of the
                           cut-off
  complete (Ex. 3)         full observation returns the data; with an exact
                           rank-k step the objective ||X - C|| never rises;
                           a tubal-rank-r tensor is recovered from half its
                           entries; observed entries equal the data
  power_tsvd (Alg. 1)      n3 = 1 is the matrix randomized subspace iteration
                           (numpy QR / SVD); b = n1 gives the exact truncated
                           T-SVD; exact recovery of a tubal-rank-r tensor;
                           q = 0 equals Alg. 2 at q = 0; the last iterate
                           computed with spatial T-products lies in range(Q_f);
                           literal == stabilised; Alg. 2's error <= Alg. 1's
                           for the same Omega and q (range(Y_q) in range(K))

Readings (where the paper is silent / ambiguous):
  R1  Omega has n2 rows (Alg. 2 draws randn(n1, ...) but X*Omega needs n2 rows,
      as in Alg. 1).
  R2  Omega is a real Gaussian tensor in the spatial domain, transformed like X.
  R3  Parameters are (k, b, q) with b = R + P (rank plus oversampling), k <= b.
  R4  DFT: omega = exp(-2 pi i / n), forward unnormalised, inverse carries 1/n3
      (Sec. 2, Def. of F_n).  Eq. (mn35) omits the 1/n3 of F^{-1}.  The half
      spectrum has n3//2 + 1 slices (= ceil((n3+1)/2)); the mirror index
      n3 - i + 2 (1-based) is (n3 - f) mod n3 (0-based).
  R5  "^T" in the Fourier domain is the per-slice conjugate transpose.
  R6  Krylov recursion: the parity reference is the stabilised form
      (orthonormalise each block and re-orthogonalise it against the earlier
      blocks before the next multiplication), which spans the same space as the
      literal powers of Alg. 2 in exact arithmetic; the literal form is kept as
      a cross-check (krylov="lit").
  R7  Economy T-QR, m = b (q + 1) <= min(n1, n2).
  R8  Only the top k singular triplets of each Fourier slice of C are kept.
  R9  Singular vectors carry an arbitrary phase; for comparison each column of
      U_f and V_f is multiplied by the conjugate phase of the largest-modulus
      entry of the U_f column (first such entry on ties).
  R10 Alg. 1 orthonormalises its last power iterate Y_q (its T-QR line names
      the Krylov tensor K, which Alg. 1 never forms); the parity reference
      orthonormalises after every product with A^H and with A (randomized
      subspace iteration), which spans the same range as the literal powers
      in exact arithmetic and never forms the squared spectrum; the literal
      form is kept as a cross-check (power="lit").  Alg. 1 shares Alg. 2's
      projection, small SVD, lift and rank-k truncation.
  R19 T-QR: qr(X_f, 0) fixes Q_f and R_f only up to one unit phase per column;
      the diagonal of R_f is taken real and non-negative (unique when the
      first r = min(n1, n2) columns of X_f are independent).  For n1 < n2 the
      economy QR orthonormalises the first n1 columns and R_f = Q_f^H X_f.
  R20 Completion (Example 3): the iteration starts from C^(0) = T (.) M (the
      missing entries zero), uses the same test tensor Omega in every call
      of L, and returns C^(iters), whose observed entries equal the data.
  R21 Alg. mp applies pinv to each Fourier slice without a tolerance; a
      singular value s_j of X_f counts as nonzero when s_j > rtol * s_1(X_f)
      (the usual relative rank cut-off of a matrix pinv), with
      rtol = max(n1, n2) * 2^-52 unless given.
  R23 "Q truncated to k + p terms" (the timing remark of Ex. 1): with the
      block order of Alg. 2 the first k + p columns of Q span only A*Omega, so
      the truncation is read as a Rayleigh-Ritz reduction: Q_r = Q W(:, 1:r),
      W the left singular vectors of C = Q^T * A per slice, r = k + p.  The
      rank-k result equals the full basis's in exact arithmetic.
  R24 Differentiating through the rank-k truncation: L = <G, X_hat(A)> with
      X_hat = Q * (Q^T * A)_k (Lemma mn38); the truncation enters through the
      projector onto the top-k eigenvectors of C C^H per slice, defined when
      lambda_k > lambda_{k+1} there.
"""
from __future__ import annotations

import numpy as np

EPS64 = 2.0 ** -53


# ---------------------------------------------------------------------------
# Sec. 2: DFT along mode 3, block diagonalisation, half spectrum
# ---------------------------------------------------------------------------

def twiddles(n: int) -> np.ndarray:
    """w[r] = omega^r, omega = exp(-2 pi i / n)  (Sec. 2, Def. of the DFT
    matrix F_n).  The four quarter points are set to their exact values so the
    DC and Nyquist rows of F_n are exactly real."""
    r = np.arange(n, dtype=np.float64)
    w = np.cos(2.0 * np.pi * r / n) - 1j * np.sin(2.0 * np.pi * r / n)
    w[0] = 1.0
    if n % 2 == 0:
        w[n // 2] = -1.0
    if n % 4 == 0:
        w[n // 4] = -1j
        w[3 * n // 4] = 1j
    return w


def dft_matrix(n: int) -> np.ndarray:
    """F_n with entries omega^(f t)  (Sec. 2, Def. of F_n)."""
    t = np.arange(n)
    return twiddles(n)[np.outer(t, t) % n]


def dft_mode3(X: np.ndarray, freqs=None) -> np.ndarray:
    """X_bar = fft(X, [], 3): the unnormalised DFT of every tube (Sec. 2),
    taken along the last axis.

    X_bar[i, j, f] = sum_t X[i, j, t] omega^(f t).  ``freqs`` restricts the
    output to the listed frequencies (same values, fewer of them)."""
    n3 = X.shape[-1]
    Fm = dft_matrix(n3)
    if freqs is not None:
        Fm = Fm[list(freqs), :]
    return np.tensordot(np.asarray(X), Fm, axes=([-1], [1]))


def idft_mode3(Xbar: np.ndarray) -> np.ndarray:
    """X = ifft(X_bar, [], 3) with F_n^{-1} = F_n^* / n  (Sec. 2)."""
    n3 = Xbar.shape[-1]
    Finv = np.conj(dft_matrix(n3)) / n3
    return np.tensordot(Xbar, Finv, axes=([-1], [1]))


def n_half(n3: int) -> int:
    """Number of Fourier slices computed, ceil((n3+1)/2) = n3//2 + 1
    (Alg. TP, first loop)."""
    return n3 // 2 + 1


def mirror(Xh: np.ndarray, n3: int) -> np.ndarray:
    """Complete a half spectrum by conjugate symmetry: slice n3 - f is
    conj(slice f)  (Alg. TP, second loop; 0-based index (n3 - f) mod n3)."""
    F = n_half(n3)
    full = np.zeros(Xh.shape[:-1] + (n3,), dtype=np.complex128)
    full[..., :F] = Xh
    for f in range(F, n3):
        full[..., f] = np.conj(Xh[..., n3 - f])
    return full


def real_part_checked(X: np.ndarray, rtol: float = 1e-12) -> np.ndarray:
    """Real part of an inverse transform that must be real; raises if the
    imaginary part is not at rounding level."""
    X = np.asarray(X)
    scale = max(float(np.max(np.abs(X.real))) if X.size else 0.0, 1e-300)
    im = float(np.max(np.abs(X.imag))) if X.size else 0.0
    if im > rtol * scale + 1e-300:
        raise ValueError(f"inverse DFT not real: max|Im| = {im:.3e}, max|Re| = {scale:.3e}")
    return np.ascontiguousarray(X.real)


# ---------------------------------------------------------------------------
# Sec. 2: bcirc / unfold / fold, T-product, T-transpose, identity, norms
# ---------------------------------------------------------------------------

def bcirc(X: np.ndarray) -> np.ndarray:
    """Block circulant matrix of X (Sec. 2): block (r, c) = X^{((r - c) mod n3)}."""
    n1, n2, n3 = X.shape
    B = np.zeros((n1 * n3, n2 * n3), dtype=X.dtype)
    for r in range(n3):
        for c in range(n3):
            B[r * n1:(r + 1) * n1, c * n2:(c + 1) * n2] = X[:, :, (r - c) % n3]
    return B


def unfold(X: np.ndarray) -> np.ndarray:
    """Stack the frontal slices vertically (Sec. 2, Def. of unfold)."""
    n1, n2, n3 = X.shape
    return np.concatenate([X[:, :, t] for t in range(n3)], axis=0)


def fold(M: np.ndarray, n1: int, n3: int) -> np.ndarray:
    """Inverse of ``unfold``."""
    return np.stack([M[t * n1:(t + 1) * n1, :] for t in range(n3)], axis=2)


def tprod_bcirc(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """T-product by its definition: fold(bcirc(X) . unfold(Y))  (Def. T-product)."""
    return fold(bcirc(X) @ unfold(Y), X.shape[0], X.shape[2])


def tprod(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """T-product in the Fourier domain (Alg. TP): transform both operands,
    multiply the first n3//2+1 frontal slices, mirror, inverse transform."""
    n3 = X.shape[2]
    F = n_half(n3)
    Xb, Yb = dft_mode3(X), dft_mode3(Y)
    Ch = np.empty((X.shape[0], Y.shape[1], F), dtype=np.complex128)
    for f in range(F):
        Ch[:, :, f] = Xb[:, :, f] @ Yb[:, :, f]
    return real_part_checked(idft_mode3(mirror(Ch, n3)))


def ttranspose(X: np.ndarray) -> np.ndarray:
    """Tensor transpose (Sec. 2): transpose every frontal slice and reverse the
    order of slices 2..n3."""
    n1, n2, n3 = X.shape
    T = np.empty((n2, n1, n3), dtype=X.dtype)
    T[:, :, 0] = X[:, :, 0].T
    for t in range(1, n3):
        T[:, :, t] = X[:, :, n3 - t].T
    return T


def identity_tensor(n: int, n3: int) -> np.ndarray:
    """Identity tensor: first frontal slice I_n, the others zero (Sec. 2)."""
    Id = np.zeros((n, n, n3))
    Id[:, :, 0] = np.eye(n)
    return Id


def fro(X: np.ndarray) -> float:
    """Frobenius norm (Def. mn3)."""
    return float(np.sqrt(np.sum(np.abs(X) ** 2)))


def relative_error(X: np.ndarray, Xt: np.ndarray) -> float:
    """e(X~) = ||X - X~||_F / ||X||_F  (Sec. 5, relative error)."""
    return fro(X - Xt) / fro(X)


def psnr(X: np.ndarray, Y: np.ndarray, peak: float = 255.0) -> float:
    """PSNR = 10 log10(peak^2 / MSE), MSE = ||X - Y||_F^2 / num(X)  (Sec. 5)."""
    mse = fro(X - Y) ** 2 / X.size
    return float(10.0 * np.log10(peak ** 2 / mse))


# ---------------------------------------------------------------------------
# Per-slice dense linear algebra: Householder QR, one-sided Jacobi SVD
# ---------------------------------------------------------------------------

def householder_qr(K: np.ndarray):
    """Economy QR, K = Q R with Q n x m orthonormal and R m x m upper
    triangular: the per-slice ``qr(X, 0)`` of Alg. TQR.

    Column j: x = R[j:, j]; beta = -exp(i arg x0) ||x||; v = x - beta e1 scaled
    so that v0 = 1; tau = (beta - x0) / beta (real); H_j = I - tau v v^H maps x
    to beta e1.  A zero column gives tau = 0 (H_j = I).  Q = H_0 ... H_{m-1}
    applied to the first m columns of the identity."""
    R = np.array(K, dtype=np.complex128)
    n, m = R.shape
    if m > n:
        raise ValueError("economy QR needs m <= n")
    vs, taus = [], []
    for j in range(m):
        x = R[j:, j].copy()
        nx = np.linalg.norm(x)
        if nx == 0.0:
            vs.append(np.zeros(n - j, dtype=np.complex128))
            taus.append(0.0)
            continue
        x0 = x[0]
        phase = x0 / abs(x0) if x0 != 0 else 1.0
        beta = -phase * nx
        v = x.copy()
        v[0] = x0 - beta
        v = v / v[0]
        tau = ((beta - x0) / beta).real
        R[j:, j:] -= tau * np.outer(v, v.conj() @ R[j:, j:])
        R[j, j] = beta
        R[j + 1:, j] = 0.0
        vs.append(v)
        taus.append(tau)
    Q = np.zeros((n, m), dtype=np.complex128)
    Q[:m, :m] = np.eye(m)
    for j in reversed(range(m)):
        v, tau = vs[j], taus[j]
        if tau != 0.0:
            Q[j:, :] -= tau * np.outer(v, v.conj() @ Q[j:, :])
    return Q, np.triu(R[:m, :m])


def jacobi_svd(C: np.ndarray, max_sweeps: int = 60, tol: float | None = None):
    """Thin SVD C = W diag(s) Z^H of an m x n matrix with m <= n, the per-slice
    T-SVD of Alg. 2 (Sec. 2: T-SVD by per-slice SVD in the Fourier domain).

    Steps: Householder QR C^H = Qc R (R m x m); one-sided (Hestenes) Jacobi on
    the columns of R with cyclic row ordering: for each pair (p, q),
    alpha = ||r_p||^2, beta = ||r_q||^2, gamma = r_p^H r_q = |gamma| e^{i phi};
    skip if |gamma| <= tol sqrt(alpha beta), otherwise apply the unitary
    J = [[c, s], [-s e^{-i phi}, c e^{-i phi}]] (zeta = (beta - alpha) / (2|gamma|),
    t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), c = 1/sqrt(1+t^2), s = c t) that
    makes the two columns orthogonal, to R and to the accumulator (initially I).
    Stop after a sweep without rotations.  Then s_j = ||r_j||,
    Zhat = R J diag(1/s), W = J, Z = Qc Zhat, sorted by decreasing s (ties keep
    the lower original index).  Returns (W, s, Z, sweeps)."""
    C = np.asarray(C, dtype=np.complex128)
    m, n = C.shape
    if m > n:
        raise ValueError("jacobi_svd expects a wide matrix (m <= n)")
    if tol is None:
        tol = m * EPS64
    Qc, R = householder_qr(C.conj().T)
    Y = R.copy()
    J = np.eye(m, dtype=np.complex128)
    sweeps = 0
    converged = False
    for sweep in range(max_sweeps):
        sweeps = sweep + 1
        rotated = False
        for p in range(m - 1):
            for q in range(p + 1, m):
                yp, yq = Y[:, p], Y[:, q]
                alpha = float(np.real(np.vdot(yp, yp)))
                beta = float(np.real(np.vdot(yq, yq)))
                gamma = np.vdot(yp, yq)
                ag = abs(gamma)
                if ag == 0.0 or ag <= tol * np.sqrt(alpha * beta):
                    continue
                rotated = True
                eph = np.conj(gamma / ag)          # e^{-i phi}
                zeta = (beta - alpha) / (2.0 * ag)
                t = (1.0 if zeta >= 0 else -1.0) / (abs(zeta) + np.sqrt(1.0 + zeta * zeta))
                c = 1.0 / np.sqrt(1.0 + t * t)
                s = c * t
                for M in (Y, J):
                    mp, mq = M[:, p].copy(), M[:, q].copy()
                    M[:, p] = c * mp - s * eph * mq
                    M[:, q] = s * mp + c * eph * mq
        if not rotated:
            converged = True
            break
    if not converged:
        raise RuntimeError(f"jacobi_svd: no convergence in {max_sweeps} sweeps")
    s = np.sqrt(np.real(np.sum(Y.conj() * Y, axis=0)))
    Zhat = np.zeros_like(Y)
    nz = s > 0
    Zhat[:, nz] = Y[:, nz] / s[nz]
    order = np.argsort(-s, kind="stable")
    W = J[:, order]
    s = s[order]
    Z = Qc @ Zhat[:, order]
    return W, s, Z, sweeps


def canonical_phase(Uf: np.ndarray, Vf: np.ndarray):
    """Reading R9: scale column j of Uf and Vf by the conjugate phase of Uf's
    largest-modulus entry in column j (first index on ties)."""
    Uf = Uf.copy()
    Vf = Vf.copy()
    for j in range(Uf.shape[1]):
        i = int(np.argmax(np.abs(Uf[:, j])))
        a = Uf[i, j]
        if a != 0:
            ph = np.conj(a) / abs(a)
            Uf[:, j] *= ph
            Vf[:, j] *= ph
    return Uf, Vf


# ---------------------------------------------------------------------------
# Alg. 2: randomized block Krylov truncated T-SVD, per Fourier slice
# ---------------------------------------------------------------------------

def krylov_basis(Af: np.ndarray, Of: np.ndarray, q: int, krylov: str = "stab"):
    """Orthonormal basis Q_f of the block Krylov space of Alg. 2 for one slice:
    K = [A Om, (A A^H) A Om, ..., (A A^H)^q A Om].

    krylov="lit": the blocks exactly as written (K_i = A (A^H K_{i-1})), then one
    Householder QR of K (Alg. 2, Krylov loop and T-QR).
    krylov="stab": Q_0 = qr(A Om); for i >= 1, W = A (A^H Q_{i-1}),
    Y = qr(W - Q_<i Q_<i^H W), Q_i = qr(Y - Q_<i Q_<i^H Y); Q = [Q_0 .. Q_q]
    (reading R6).  The second projection acts on the normalised block: when
    the new block lies numerically inside the earlier span (a spectrum that
    falls below the rounding level within the first blocks), two projections
    before normalising leave Q far from orthonormal, which the T-QR of the
    Krylov tensor excludes.
    Returns (Q, blocks) where blocks are the R factors / literal blocks."""
    if krylov == "lit":
        blocks = [Af @ Of]
        for _ in range(q):
            blocks.append(Af @ (Af.conj().T @ blocks[-1]))
        Q, R = householder_qr(np.concatenate(blocks, axis=1))
        return Q, R
    if krylov != "stab":
        raise ValueError(krylov)
    Q0, _ = householder_qr(Af @ Of)
    Qs = [Q0]
    for _ in range(q):
        W = Af @ (Af.conj().T @ Qs[-1])
        Qp = np.concatenate(Qs, axis=1)
        Y = W - Qp @ (Qp.conj().T @ W)
        Y, _ = householder_qr(Y)
        Y = Y - Qp @ (Qp.conj().T @ Y)
        Qi, _ = householder_qr(Y)
        Qs.append(Qi)
    return np.concatenate(Qs, axis=1), None


def _check_params(n1, n2, n3, k, b, q):
    if min(n1, n2, n3) < 1:
        raise ValueError("empty tensor")
    if not (1 <= k <= b) or q < 0:
        raise ValueError("need 1 <= k <= b and q >= 0")
    if b * (q + 1) > min(n1, n2):
        raise ValueError("need m = b (q + 1) <= min(n1, n2)")


def _truncated_slices(A, Omega, k, b, m, freqs, basis):
    """Shared tail of Alg. 1 and Alg. 2 in the Fourier domain: per slice f,
    Q_f = basis(A_f, Om_f) (n1 x m, orthonormal), C_f = Q_f^H A_f (projection),
    SVD of C_f, U_f = Q_f W(:, :k), S_f = s[:k], V_f = Z(:, :k) (lift and
    truncation), phases canonicalised (reading R9)."""
    n1, n2, n3 = A.shape
    if Omega.shape != (n2, b, n3):
        raise ValueError("Omega must be n2 x b x n3")
    if freqs is None:
        freqs = list(range(n_half(n3)))
    Ab = dft_mode3(A, freqs)
    Ob = dft_mode3(Omega, freqs)
    nf = len(freqs)
    out = {
        "freqs": list(freqs),
        "Uf": np.zeros((n1, k, nf), complex), "Sf": np.zeros((k, nf)),
        "Vf": np.zeros((n2, k, nf), complex), "Q": np.zeros((n1, m, nf), complex),
        "C": np.zeros((m, n2, nf), complex), "s_all": np.zeros((m, nf)),
    }
    for idx in range(nf):
        r = truncated_slice(Ab[:, :, idx], Ob[:, :, idx], k, basis)
        for key in ("Uf", "Vf", "Q", "C"):
            out[key][:, :, idx] = r[key]
        out["Sf"][:, idx] = r["Sf"]
        out["s_all"][:, idx] = r["s_all"]
    return out


def truncated_slice(Af: np.ndarray, Of: np.ndarray, k: int, basis):
    """One Fourier slice of the shared tail of Alg. 1 and Alg. 2: Q = basis(Af,
    Of), C = Q^H Af, C = W diag(s) Z^H (Jacobi SVD), U_f = Q W(:, :k),
    S_f = s[:k], V_f = Z(:, :k), phases canonicalised (reading R9)."""
    Q = basis(Af, Of)
    C = Q.conj().T @ Af
    W, s, Z, _ = jacobi_svd(C)
    Uf, Vf = canonical_phase(Q @ W[:, :k], Z[:, :k])
    return {"Uf": Uf, "Vf": Vf, "Sf": s[:k], "Q": Q, "C": C, "s_all": s}


def rbk_slice(Af: np.ndarray, Of: np.ndarray, k: int, b: int, q: int, krylov: str = "stab"):
    """Alg. 2 on one Fourier slice (Af n1 x n2, Of n2 x b): the per-slice body
    of rbk_slices for a slice whose DFT is already taken."""
    _check_params(Af.shape[0], Af.shape[1], 1, k, b, q)
    return truncated_slice(Af, Of, k, lambda A_, O_: krylov_basis(A_, O_, q, krylov)[0])


def _spatial_factors(sl: dict, n3: int) -> dict:
    """Mirror and inverse-transform the half-spectrum factors (Alg. TP)."""
    U = real_part_checked(idft_mode3(mirror(sl["Uf"], n3)))
    V = real_part_checked(idft_mode3(mirror(sl["Vf"], n3)))
    S = real_part_checked(idft_mode3(mirror(sl["Sf"].astype(np.complex128), n3)))
    sl.update(U=U, S=S, V=V)
    return sl


def rbk_slices(A: np.ndarray, Omega: np.ndarray, k: int, b: int, q: int,
               freqs=None, krylov: str = "stab"):
    """Alg. 2 in the Fourier domain for the requested slices (default: the
    n3//2 + 1 slices of the half spectrum).

    Per slice f: Krylov basis Q_f (Alg. 2 Krylov loop + T-QR), then the shared
    projection / small SVD / lift / truncation.  Returns a dict of per-slice
    arrays indexed like ``freqs``: Uf (n1,k,nf), Sf (k,nf), Vf (n2,k,nf),
    Q (n1,m,nf), C (m,n2,nf), s_all (m,nf) (all singular values of C_f)."""
    n1, n2, n3 = A.shape
    _check_params(n1, n2, n3, k, b, q)
    return _truncated_slices(A, Omega, k, b, b * (q + 1), freqs,
                             lambda Af, Of: krylov_basis(Af, Of, q, krylov)[0])


def rbk_tsvd(A: np.ndarray, Omega: np.ndarray, k: int, b: int, q: int,
             krylov: str = "stab"):
    """Alg. 2: U (n1 x k x n3), S (k x n3: the diagonal tubes of the f-diagonal
    S_R), V (n2 x k x n3) with A ~ U * S * V^T, plus the half-spectrum pieces.
    The mirror and inverse transform follow Alg. TP."""
    sl = rbk_slices(A, Omega, k, b, q, None, krylov)
    return _spatial_factors(sl, A.shape[2])


# ---------------------------------------------------------------------------
# Alg. 1: classical randomized subspace method with power iteration
# ---------------------------------------------------------------------------

def power_basis(Af: np.ndarray, Of: np.ndarray, q: int, power: str = "stab"):
    """Orthonormal basis Q_f (n1 x b) of range((A A^H)^q A Om) for one slice:
    only the last power iterate Y_q is used (Alg. 1).

    power="lit": Y_0 = A Om, Y_i = A (A^H Y_{i-1}) exactly as written, then one
    Householder QR of Y_q.
    power="stab": the same range with an orthonormalisation after every
    product (randomized subspace iteration, Halko, Martinsson and Tropp 2011,
    Alg. 4.4): Q_0 = qr(A Om), Qt_i = qr(A^H Q_{i-1}), Q_i = qr(A Qt_i)
    (reading R10)."""
    if power == "lit":
        Y = Af @ Of
        for _ in range(q):
            Y = Af @ (Af.conj().T @ Y)
        Q, _ = householder_qr(Y)
        return Q
    if power != "stab":
        raise ValueError(power)
    Qp, _ = householder_qr(Af @ Of)
    for _ in range(q):
        Qt, _ = householder_qr(Af.conj().T @ Qp)
        Qp, _ = householder_qr(Af @ Qt)
    return Qp


def power_slices(A: np.ndarray, Omega: np.ndarray, k: int, b: int, q: int,
                 freqs=None, power: str = "stab"):
    """Alg. 1 in the Fourier domain: basis of the last power iterate (m = b
    columns per slice), then the projection / small SVD / lift / truncation
    shared with Alg. 2.  Same dict layout as rbk_slices with m = b."""
    n1, n2, n3 = A.shape
    _check_params(n1, n2, n3, k, b, 0)
    if q < 0:
        raise ValueError("need q >= 0")
    return _truncated_slices(A, Omega, k, b, b, freqs,
                             lambda Af, Of: power_basis(Af, Of, q, power))


def power_tsvd(A: np.ndarray, Omega: np.ndarray, k: int, b: int, q: int,
               power: str = "stab"):
    """Alg. 1: U (n1 x k x n3), S (k x n3), V (n2 x k x n3) with
    A ~ U * S * V^T, plus the half-spectrum pieces."""
    sl = power_slices(A, Omega, k, b, q, None, power)
    return _spatial_factors(sl, A.shape[2])


def power_approx(A, Omega, k, b, q, power: str = "stab") -> np.ndarray:
    """Rank-k approximation U * S * V^T returned by Alg. 1."""
    n1, n2, n3 = A.shape
    return approx_from_slices(power_slices(A, Omega, k, b, q, None, power), n1, n2, n3)


def s_tensor(S: np.ndarray) -> np.ndarray:
    """f-diagonal k x k x n3 tensor from its k diagonal tubes."""
    k, n3 = S.shape
    T = np.zeros((k, k, n3))
    for j in range(k):
        T[j, j, :] = S[j, :]
    return T


def approx_from_slices(sl: dict, n1: int, n2: int, n3: int) -> np.ndarray:
    """X_hat = U * S * V^T assembled per slice as U_f S_f V_f^H (Alg. TP), then
    mirrored and inverse transformed; equals Q * (Q^T * A)_k (Lemma mn38)."""
    F = n_half(n3)
    Xh = np.zeros((n1, n2, F), complex)
    for f in range(F):
        Xh[:, :, f] = (sl["Uf"][:, :, f] * sl["Sf"][:, f]) @ sl["Vf"][:, :, f].conj().T
    return real_part_checked(idft_mode3(mirror(Xh, n3)))


def rbk_approx(A, Omega, k, b, q, krylov: str = "stab") -> np.ndarray:
    """Rank-k approximation X_hat = U_R * S_R * V_R^T returned by Alg. 2."""
    n1, n2, n3 = A.shape
    sl = rbk_slices(A, Omega, k, b, q, None, krylov)
    return approx_from_slices(sl, n1, n2, n3)


# ---------------------------------------------------------------------------
# Projection P(A) = Q * Q^T * A and its adjoint
# ---------------------------------------------------------------------------

def proj(A: np.ndarray, Omega: np.ndarray, b: int, q: int, krylov: str = "stab"):
    """P(A) = Q * Q^T * A with Q the T-QR basis of the block Krylov tensor of
    Alg. 2 (the orthogonal projection of Sec. 4, Thm. mn44 / Lemma mn38):
    per slice Q_f Q_f^H A_f, mirrored, inverse transformed."""
    n1, n2, n3 = A.shape
    _check_params(n1, n2, n3, 1, b, q)
    F = n_half(n3)
    Ab, Ob = dft_mode3(A, range(F)), dft_mode3(Omega, range(F))
    Ph = np.zeros((n1, n2, F), complex)
    for f in range(F):
        Q, _ = krylov_basis(Ab[:, :, f], Ob[:, :, f], q, krylov)
        Ph[:, :, f] = Q @ (Q.conj().T @ Ab[:, :, f])
    return real_part_checked(idft_mode3(mirror(Ph, n3)))


def _krylov_factors(A, Of, q):
    """The stabilised recursion (reading R6) with the factors its reverse pass
    needs: Q_0 R_0 = A Om; for i >= 1, T_i = A^H Q_{i-1}, W_i = A T_i,
    Z_i = (I - Q_<i Q_<i^H) W_i (twice), Q_i R_i = Z_i.  Returns the lists
    (Qs, Rs, Ts, Ws) with None in the unused i = 0 entries of Ts and Ws."""
    Q0, R0 = householder_qr(A @ Of)
    Qs, Rs, Ts, Ws = [Q0], [R0], [None], [None]
    for i in range(1, q + 1):
        T = A.conj().T @ Qs[i - 1]
        W = A @ T
        Qp = np.concatenate(Qs, axis=1)
        Z = W - Qp @ (Qp.conj().T @ W)
        Z = Z - Qp @ (Qp.conj().T @ Z)
        Qi, Ri = householder_qr(Z)
        Qs.append(Qi)
        Rs.append(Ri)
        Ts.append(T)
        Ws.append(W)
    return Qs, Rs, Ts, Ws


def _krylov_reverse(A, Of, Qs, Rs, Ts, Ws, Abar, Qbar_all):
    """Reverse pass of the stabilised recursion for a loss that depends on
    every block Q_i only through its range: given Abar (the direct part of
    dL/dA_f) and Qbar_all (dL/dQ, n1 x m), for i = q..1:
    Zbar_i = (I - Q_i Q_i^H) Qbar_i R_i^{-H}; Wbar_i = (I - Q_<i Q_<i^H) Zbar_i;
    Qbar_l -= (Zbar_i W_i^H + W_i Zbar_i^H) Q_l for l < i;
    Abar += Wbar_i T_i^H; Tbar_i = A^H Wbar_i; Abar += Q_{i-1} Tbar_i^H;
    Qbar_{i-1} += A Tbar_i.  Finally Zbar_0 = (I - Q_0 Q_0^H) Qbar_0 R_0^{-H}
    and Abar += Zbar_0 Om^H."""
    q = len(Qs) - 1
    b = Qs[0].shape[1]
    Qbar = [Qbar_all[:, i * b:(i + 1) * b].copy() for i in range(q + 1)]
    for i in range(q, 0, -1):
        Qi, Ri = Qs[i], Rs[i]
        X = Qbar[i] - Qi @ (Qi.conj().T @ Qbar[i])
        Zbar = np.linalg.solve(Ri, X.conj().T).conj().T        # X R^{-H}
        Qp = np.concatenate(Qs[:i], axis=1)
        Wbar = Zbar - Qp @ (Qp.conj().T @ Zbar)
        for l in range(i):
            Qbar[l] -= (Zbar @ (Ws[i].conj().T @ Qs[l]) + Ws[i] @ (Zbar.conj().T @ Qs[l]))
        Abar += Wbar @ Ts[i].conj().T
        Tbar = A.conj().T @ Wbar
        Abar += Qs[i - 1] @ Tbar.conj().T
        Qbar[i - 1] += A @ Tbar
    Q0, R0 = Qs[0], Rs[0]
    X = Qbar[0] - Q0 @ (Q0.conj().T @ Qbar[0])
    Zbar0 = np.linalg.solve(R0, X.conj().T).conj().T
    Abar += Zbar0 @ Of.conj().T
    return Abar


def _proj_slice_adjoint(Af, Of, Yb, q):
    """Adjoint of the per-slice map A_f -> Q Q^H A_f at A_f, applied to the
    cotangent Yb, for the real inner product <X, Y> = Re tr(X^H Y).

    Forward: the stabilised recursion (_krylov_factors).  Reverse: direct term
    Q Q^H Yb; Qbar = (Yb A^H + A Yb^H) Q; then the reverse recursion
    (_krylov_reverse), in which the loss depends on each Q_i only through its
    range (the gauge term of the QR adjoint vanishes)."""
    A = Af
    Qs, Rs, Ts, Ws = _krylov_factors(A, Of, q)
    Q = np.concatenate(Qs, axis=1)
    Abar = Q @ (Q.conj().T @ Yb)
    Qbar_all = Yb @ (A.conj().T @ Q) + A @ (Yb.conj().T @ Q)   # (Yb A^H + A Yb^H) Q
    return _krylov_reverse(A, Of, Qs, Rs, Ts, Ws, Abar, Qbar_all)


def proj_backward(A: np.ndarray, Omega: np.ndarray, G: np.ndarray, b: int, q: int):
    """dL/dA for L = <G, P(A)> (G = dL/dP): per-slice adjoint of the Fourier
    domain map applied to fft(G), mirrored, inverse transformed.  The 1/n3 of
    the inverse DFT and the conjugate mirror turn the per-slice adjoints into
    the spatial gradient: dL/dA = ifft(adjoint_f(fft(G)_f))."""
    n1, n2, n3 = A.shape
    _check_params(n1, n2, n3, 1, b, q)
    F = n_half(n3)
    Ab, Ob, Gb = dft_mode3(A, range(F)), dft_mode3(Omega, range(F)), dft_mode3(G, range(F))
    Dh = np.zeros((n1, n2, F), complex)
    for f in range(F):
        Dh[:, :, f] = _proj_slice_adjoint(Ab[:, :, f], Ob[:, :, f], Gb[:, :, f], q)
    return real_part_checked(idft_mode3(mirror(Dh, n3)))


def _approx_slice_adjoint(Af, Of, Yb, k, q):
    """Adjoint of the per-slice rank-k approximation of Alg. 2,
    A_f -> X_f = Q Pi C with C = Q^H A_f and Pi = W_k W_k^H the projector onto
    the top-k eigenvectors of G = C C^H (Lemma mn38: X_f = U_k U_k^H A_f with
    U_k = Q W_k), applied to the cotangent Yb, real inner product Re tr(X^H Y)
    (reading R24).

    With Y = Q^H Yb: the direct terms give Cbar = Pi Y and Qbar = Yb C^H Pi.
    Pi depends on G through the eigenvectors on either side of the cut: for
    a in the top k and c outside it, first-order perturbation theory gives
    dPi = sum w_c w_c^H dG w_a w_a^H / (lambda_a - lambda_c) + its conjugate
    transpose, so with M = W^H (Y C^H) W (Y C^H is the cotangent of Pi) the
    cotangent of G is W N W^H, N_ac = M_ac / (lambda_a - lambda_c) and
    N_ca = M_ca / (lambda_a - lambda_c) (zero inside either group), and
    G = C C^H adds (W (N + N^H) W^H) C to Cbar.  C = Q^H A_f then gives
    Abar = Q Cbar and Qbar += A_f Cbar^H.  X_f depends on Q only through its
    range, so the reverse recursion of the projection applies unchanged.
    Needs lambda_k - lambda_{k+1} above the eigenvalues' rounding level
    m 2^-53 lambda_1 (else ValueError)."""
    A = Af
    Qs, Rs, Ts, Ws = _krylov_factors(A, Of, q)
    Q = np.concatenate(Qs, axis=1)
    m = Q.shape[1]
    C = Q.conj().T @ A
    W, s, _, _ = jacobi_svd(C)
    lam = s * s
    if k < m and not lam[k - 1] - lam[k] > m * EPS64 * lam[0]:
        # a gap at the rounding level of the eigenvalues: the top-k subspace,
        # and with it the derivative, is not determined
        raise ValueError("the rank-k truncation needs lambda_k > lambda_{k+1}")
    Y = Q.conj().T @ Yb
    Wk = W[:, :k]
    Pi = Wk @ Wk.conj().T
    M = W.conj().T @ (Y @ C.conj().T) @ W
    N = np.zeros((m, m), dtype=np.complex128)
    for a in range(k):
        for c in range(k, m):
            N[a, c] = M[a, c] / (lam[a] - lam[c])
            N[c, a] = M[c, a] / (lam[a] - lam[c])
    H = W @ (N + N.conj().T) @ W.conj().T
    Cbar = Pi @ Y + H @ C
    Abar = Q @ Cbar
    Qbar_all = Yb @ (C.conj().T @ Pi) + A @ Cbar.conj().T
    return _krylov_reverse(A, Of, Qs, Rs, Ts, Ws, Abar, Qbar_all)


def approx_backward(A: np.ndarray, Omega: np.ndarray, G: np.ndarray, k: int, b: int, q: int):
    """dL/dA for L = <G, X_hat(A)>, X_hat = U * S * V^T the rank-k result of
    Alg. 2 (= Q * (Q^T * A)_k, Lemma mn38): per-slice adjoint of the Fourier
    domain map applied to fft(G), mirrored, inverse transformed (as for
    proj_backward)."""
    n1, n2, n3 = A.shape
    _check_params(n1, n2, n3, k, b, q)
    F = n_half(n3)
    Ab, Ob, Gb = dft_mode3(A, range(F)), dft_mode3(Omega, range(F)), dft_mode3(G, range(F))
    Dh = np.zeros((n1, n2, F), complex)
    for f in range(F):
        Dh[:, :, f] = _approx_slice_adjoint(Ab[:, :, f], Ob[:, :, f], Gb[:, :, f], k, q)
    return real_part_checked(idft_mode3(mirror(Dh, n3)))


# ---------------------------------------------------------------------------
# Sec. 5 (Ex. 1, timing remark): the basis truncated to k + p columns, read as
# a Rayleigh-Ritz reduction (reading R23)
# ---------------------------------------------------------------------------

def ritz_basis(Af: np.ndarray, Of: np.ndarray, q: int, r: int):
    """The block Krylov basis Q_f (n1 x m) of Alg. 2 reduced to its top r
    Ritz directions for A_f A_f^H: C = Q_f^H A_f = W diag(s) Z^H (Jacobi SVD),
    Q_r = Q_f W(:, :r), columns in the phase convention of reading R9.
    span Q_r is the r-dimensional subspace of span Q_f that captures the
    most of A_f (Rayleigh-Ritz)."""
    Q, _ = krylov_basis(Af, Of, q)
    W, _, _, _ = jacobi_svd(Q.conj().T @ Af)
    Qr, _ = canonical_phase(Q @ W[:, :r], np.zeros((1, r), dtype=np.complex128))
    return Qr


def ritz_slices(A: np.ndarray, Omega: np.ndarray, k: int, b: int, q: int, r: int | None = None, freqs=None):
    """Alg. 2 with Q truncated to r = k + p (default b) columns before the
    projection (reading R23): per slice Q_r = ritz_basis, then C_r = Q_r^H A_f,
    its SVD, lift and truncation exactly as for the full basis.  Same dict
    layout as rbk_slices, with Q the n1 x r truncated basis."""
    n1, n2, n3 = A.shape
    _check_params(n1, n2, n3, k, b, q)
    r = b if r is None else r
    if not k <= r <= b * (q + 1):
        raise ValueError("need k <= r <= m")
    return _truncated_slices(A, Omega, k, b, r, freqs, lambda Af, Of: ritz_basis(Af, Of, q, r))


def ritz_tsvd(A: np.ndarray, Omega: np.ndarray, k: int, b: int, q: int, r: int | None = None):
    """Spatial U, S, V of the truncated-basis variant, plus Qr: the truncated
    basis as an orthonormal n1 x r x n3 tensor (Qr^T * Qr = I)."""
    sl = ritz_slices(A, Omega, k, b, q, r)
    n3 = A.shape[2]
    sl = _spatial_factors(sl, n3)
    sl["Qr"] = real_part_checked(idft_mode3(mirror(sl["Q"], n3)))
    return sl


# ---------------------------------------------------------------------------
# Sec. 2: T-QR (Alg. TQR) and the Moore-Penrose pseudoinverse (Alg. mp)
# ---------------------------------------------------------------------------

def tqr(X: np.ndarray):
    """Alg. TQR: economy T-QR X = Q * R, Q (n1 x r x n3) with Q^T * Q = I,
    R (r x n2 x n3) with upper-trapezoidal Fourier slices, r = min(n1, n2).

    Per half-spectrum slice: Householder QR of the first r columns, R_f =
    Q_f^H X_f with the strictly lower part set to zero, then each pair
    (Q_f(:, j), R_f(j, :)) scaled by one unit phase so that R_f(j, j) is real
    and non-negative (reading R19); mirror (Alg. TQR, second loop); inverse
    DFT."""
    n1, n2, n3 = X.shape
    r = min(n1, n2)
    F = n_half(n3)
    Xb = dft_mode3(X, range(F))
    Qh = np.zeros((n1, r, F), complex)
    Rh = np.zeros((r, n2, F), complex)
    for f in range(F):
        Q, _ = householder_qr(Xb[:, :r, f])
        R = np.triu(Q.conj().T @ Xb[:, :, f])
        d = np.diag(R[:, :r])
        ph = np.ones(r, complex)
        nz = np.abs(d) > 0
        ph[nz] = np.conj(d[nz]) / np.abs(d[nz])
        Qh[:, :, f] = Q * np.conj(ph)[None, :]
        Rh[:, :, f] = R * ph[:, None]
    Q = real_part_checked(idft_mode3(mirror(Qh, n3)))
    R = real_part_checked(idft_mode3(mirror(Rh, n3)))
    return Q, R


def pinv_default_rtol(n1: int, n2: int) -> float:
    """Default relative cut-off of tpinv for FP64 data: max(n1, n2) times the
    FP64 machine epsilon 2^-52 (reading R21)."""
    return max(n1, n2) * 2.0 ** -52


def tpinv(X: np.ndarray, rtol: float | None = None) -> np.ndarray:
    """Alg. mp: Moore-Penrose pseudoinverse X^+ (n2 x n1 x n3).

    Every half-spectrum slice X_f = U diag(s) V^H (numpy's SVD, s descending)
    is inverted on its nonzero singular values, X_f^+ = V diag(s^+) U^H, the
    matrix form of A^+ = V * S^+ * U^T (Sec. 2: S^+ transposes S and inverts
    its nonzero tubes); s_j counts as nonzero when s_j > rtol * s_1 (reading
    R21; default pinv_default_rtol).  Mirror (Alg. mp, second loop), inverse
    DFT."""
    n1, n2, n3 = X.shape
    if rtol is None:
        rtol = pinv_default_rtol(n1, n2)
    F = n_half(n3)
    Xb = dft_mode3(X, range(F))
    Ch = np.zeros((n2, n1, F), complex)
    for f in range(F):
        U, s, Vh = np.linalg.svd(Xb[:, :, f], full_matrices=False)
        keep = s > rtol * s[0]
        sp = np.zeros_like(s)
        sp[keep] = 1.0 / s[keep]
        Ch[:, :, f] = (Vh.conj().T * sp[None, :]) @ U.conj().T
    return real_part_checked(idft_mode3(mirror(Ch, n3)))


def masked_loss(T: np.ndarray, M: np.ndarray, P: np.ndarray) -> float:
    """||M (.) (T - P)||_F^2, the completion data term of Ex. 3."""
    return float(np.sum((M * (T - P)) ** 2))


# ---------------------------------------------------------------------------
# Sec. 5, Example 3: completion by alternating a rank-R approximation and the
# data constraint
# ---------------------------------------------------------------------------

def complete(Mobs: np.ndarray, T: np.ndarray, Omega: np.ndarray, k: int, b: int, q: int, iters: int,
             alg: int = 2, history: bool = False):
    """Completion of Example 3: C^(0) = T (.) M (reading R20); then `iters`
    times X^(n) = L(C^(n)), the rank-k approximation of Alg. 2 (alg=2) or
    Alg. 1 (alg=1) with test tensor Omega, and C^(n+1) = T (.) M +
    (1 - T) (.) X^(n).  T is the 0/1 observation tensor.  Returns C^(iters)
    (and, with history, the values ||X^(n) - C^(n)||_F)."""
    L = rbk_approx if alg == 2 else power_approx
    C = T * Mobs
    hist = []
    for _ in range(iters):
        X = L(C, Omega, k, b, q)
        hist.append(fro(X - C))
        C = T * Mobs + (1.0 - T) * X
    return (C, hist) if history else C


# ---------------------------------------------------------------------------
# Reference truncated T-SVD (Sec. 2): per-slice full SVD, used as a pin
# ---------------------------------------------------------------------------

def exact_truncated_tsvd_slices(A: np.ndarray, k: int):
    """Truncated T-SVD of tubal rank k by the per-slice SVD in the Fourier
    domain (Sec. 2, T-SVD): returns (Uf, Sf, Vf, s_all) on the half spectrum."""
    n1, n2, n3 = A.shape
    F = n_half(n3)
    Ab = dft_mode3(A, range(F))
    r = min(n1, n2)
    Uf = np.zeros((n1, k, F), complex)
    Vf = np.zeros((n2, k, F), complex)
    Sf = np.zeros((k, F))
    s_all = np.zeros((r, F))
    for f in range(F):
        Af = Ab[:, :, f]
        if n1 <= n2:
            W, s, Z, _ = jacobi_svd(Af)
        else:
            Z, s, W, _ = jacobi_svd(Af.conj().T)
        u, v = canonical_phase(W[:, :k], Z[:, :k])
        Uf[:, :, f], Vf[:, :, f], Sf[:, f] = u, v, s[:k]
        s_all[:, f] = s[:r]
    return Uf, Sf, Vf, s_all
