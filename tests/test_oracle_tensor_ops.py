"""Pins for the oracle's T-QR (Alg. TQR) and T-pseudoinverse (Alg. mp), CPU only.

Both are checked in the spatial domain with the block-circulant T-product of
Sec. 2 (``tprod_bcirc``) and the slice-reversal transpose, independently of the
Fourier-domain code that computes them: X = Q * R with Q^T * Q = I for the
T-QR, and the four Penrose conditions for the pseudoinverse.
"""
import numpy as np
import pytest

from oracle import tsvd_oracle as O
from paper_2504_04989_amd import inputs

SHAPES = [(9, 6, 5), (7, 7, 4), (5, 8, 3), (6, 4, 1), (10, 3, 2)]


@pytest.mark.parametrize("shape", SHAPES)
def test_tqr_reconstructs_and_is_orthonormal(shape):
    n1, n2, n3 = shape
    r = min(n1, n2)
    X = inputs.random_tensor(shape, 41)
    Q, R = O.tqr(X)
    assert Q.shape == (n1, r, n3) and R.shape == (r, n2, n3)
    assert np.allclose(O.tprod_bcirc(Q, R), X, atol=1e-12 * np.abs(X).max())
    assert np.allclose(O.tprod_bcirc(O.ttranspose(Q), Q), O.identity_tensor(r, n3), atol=1e-12)
    Rb = np.fft.fft(R, axis=2)
    for f in range(n3):
        assert np.allclose(np.tril(Rb[:, :, f], -1), 0.0, atol=1e-12)
        d = np.diag(Rb[:, :r, f])
        assert np.all(np.abs(d.imag) <= 1e-12 * np.abs(d).max()) and np.all(d.real >= 0)


def test_tqr_n3_equal_one_is_matrix_qr():
    X = inputs.random_tensor((8, 5, 1), 42)
    Q, R = O.tqr(X)
    q, r = np.linalg.qr(X[:, :, 0])
    s = np.sign(np.diag(r))
    assert np.allclose(Q[:, :, 0], q * s, atol=1e-12)
    assert np.allclose(R[:, :, 0], r * s[:, None], atol=1e-12)


@pytest.mark.parametrize("shape", SHAPES)
def test_tpinv_penrose_conditions(shape):
    X = inputs.random_tensor(shape, 43)
    P = O.tpinv(X)
    assert P.shape == (shape[1], shape[0], shape[2])
    tp, tt = O.tprod_bcirc, O.ttranspose
    sc = np.abs(X).max() * np.abs(P).max()
    assert np.allclose(tp(tp(X, P), X), X, atol=1e-11 * np.abs(X).max() * max(1.0, sc))
    assert np.allclose(tp(tp(P, X), P), P, atol=1e-11 * np.abs(P).max() * max(1.0, sc))
    XP, PX = tp(X, P), tp(P, X)
    assert np.allclose(tt(XP), XP, atol=1e-11 * max(1.0, sc))
    assert np.allclose(tt(PX), PX, atol=1e-11 * max(1.0, sc))


def test_tpinv_rank_deficient():
    # tubal rank 2 < min(n1, n2): X^+ is not an inverse, the Penrose
    # conditions still hold
    X = inputs.exact_lowrank_tensor(9, 7, 4, 2, seed=44)
    P = O.tpinv(X)
    tp, tt = O.tprod_bcirc, O.ttranspose
    assert np.allclose(tp(tp(X, P), X), X, atol=1e-10 * np.abs(X).max())
    assert np.allclose(tp(tp(P, X), P), P, atol=1e-10 * np.abs(P).max())
    assert np.allclose(tt(tp(X, P)), tp(X, P), atol=1e-10)
    assert np.allclose(tt(tp(P, X)), tp(P, X), atol=1e-10)


def test_tpinv_full_column_rank_is_left_inverse():
    X = inputs.random_tensor((9, 4, 5), 45)
    assert np.allclose(O.tprod_bcirc(O.tpinv(X), X), O.identity_tensor(4, 5), atol=1e-11)


def _known_spectrum(n1, n2, s, seed):
    # n1 x n2 matrix U diag(s) V^T with Haar-orthonormal U, V (numpy QR of
    # Gaussian matrices)
    g = np.random.default_rng(seed)
    U, _ = np.linalg.qr(g.standard_normal((n1, len(s))))
    V, _ = np.linalg.qr(g.standard_normal((n2, len(s))))
    return U, np.asarray(s, float), V


@pytest.mark.parametrize("n1,n2", [(6, 4), (4, 6), (5, 5)])
def test_tpinv_cutoff_known_spectrum(n1, n2):
    # n3 = 1: X^+ = V_r diag(1/s_r) U_r^T over the singular values above
    # rtol * s_1, written out from the constructed factors (reading R21)
    U, s, V = _known_spectrum(n1, n2, [4.0, 2.0, 1e-3, 1e-9][: min(n1, n2)], 50 + n1)
    X = (U * s) @ V.T
    for rtol, r in ((1e-2, 2), (1e-5, 3), (1e-12, 4)):
        r = min(r, len(s))
        want = (V[:, :r] / s[:r]) @ U[:, :r].T
        got = O.tpinv(X[:, :, None], rtol=rtol)[:, :, 0]
        assert np.allclose(got, want, atol=1e-9 * np.abs(want).max()), (rtol, r)


def test_tpinv_default_cutoff_drops_rounding_level_values():
    # a rank-2 slice whose third singular value sits at rounding level: the
    # default cut-off max(n1, n2) 2^-52 s_1 treats it as zero
    U, s, V = _known_spectrum(7, 5, [3.0, 1.0, 1e-17], 60)
    X = (U * s) @ V.T
    want = (V[:, :2] / s[:2]) @ U[:, :2].T
    assert O.pinv_default_rtol(7, 5) == 7 * 2.0 ** -52
    assert np.allclose(O.tpinv(X[:, :, None])[:, :, 0], want, atol=1e-12)


def test_tpinv_wide_is_transpose_of_tall():
    # (X^T)^+ = (X^+)^T for the T-transpose, and the Penrose conditions
    X = inputs.random_tensor((4, 9, 5), 46)
    P = O.tpinv(X)
    assert np.allclose(O.ttranspose(O.tpinv(O.ttranspose(X))), P, atol=1e-11)
    tp = O.tprod_bcirc
    assert np.allclose(tp(X, P), O.identity_tensor(4, 5), atol=1e-11)
