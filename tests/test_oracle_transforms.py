"""Pins for the oracle's mode-3 DFT and T-algebra (CPU only).

Each check ties the oracle to something other than itself: closed forms,
numpy's FFT, Parseval's identity (eq. (eq_fou)) and the block-circulant
definitions of Sec. 2.
"""
import numpy as np
import pytest

from oracle import tsvd_oracle as O
from paper_2504_04989_amd.inputs import random_tensor


@pytest.mark.parametrize("n3", [1, 2, 3, 4, 5, 8, 12, 16, 200])
def test_dft_matches_numpy_fft(n3):
    X = random_tensor((3, 4, n3), seed=n3)
    ref = np.fft.fft(X, axis=2)
    got = O.dft_mode3(X)
    assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref))) * np.sqrt(n3)


@pytest.mark.parametrize("n3", [1, 5, 8, 16])
def test_dft_impulse_closed_form(n3):
    # DFT of a unit impulse at t0 is omega^(f t0) (Sec. 2, omega = exp(-2 pi i / n)).
    for t0 in range(n3):
        X = np.zeros((1, 1, n3))
        X[0, 0, t0] = 1.0
        f = np.arange(n3)
        ref = np.exp(-2j * np.pi * f * t0 / n3)
        assert np.allclose(O.dft_mode3(X)[0, 0], ref, atol=1e-14)


@pytest.mark.parametrize("n3", [4, 7, 16])
def test_dft_pure_exponential(n3):
    # x_t = exp(+2 pi i f0 t / n) transforms to n * delta(f - f0).
    t = np.arange(n3)
    for f0 in range(n3):
        X = np.exp(2j * np.pi * f0 * t / n3).reshape(1, 1, n3)
        ref = np.zeros(n3, complex)
        ref[f0] = n3
        assert np.allclose(O.dft_mode3(X)[0, 0], ref, atol=1e-12)


@pytest.mark.parametrize("n3", [1, 2, 6, 9, 16])
def test_round_trip_and_parseval(n3):
    X = random_tensor((5, 3, n3), seed=7 + n3)
    Xb = O.dft_mode3(X)
    back = O.idft_mode3(Xb)
    assert np.max(np.abs(back - X)) < 1e-14 * n3
    # eq. (eq_fou): ||X||_F^2 = (1/n3) sum_f ||Xbar_f||_F^2
    lhs = np.sum(X * X)
    rhs = np.sum(np.abs(Xb) ** 2) / n3
    assert abs(lhs - rhs) <= 1e-13 * lhs


@pytest.mark.parametrize("n3", [2, 4, 8, 16, 200])
def test_dc_and_nyquist_exactly_real(n3):
    X = random_tensor((4, 4, n3), seed=3)
    Xb = O.dft_mode3(X)
    assert np.all(Xb[:, :, 0].imag == 0)
    if n3 % 2 == 0:
        assert np.all(Xb[:, :, n3 // 2].imag == 0)


@pytest.mark.parametrize("n3", [1, 2, 5, 8])
def test_half_spectrum_mirror(n3):
    X = random_tensor((3, 2, n3), seed=11)
    Xb = O.dft_mode3(X)
    F = O.n_half(n3)
    assert F == int(np.ceil((n3 + 1) / 2))
    assert np.allclose(O.mirror(Xb[:, :, :F], n3), Xb, atol=1e-13)


@pytest.mark.parametrize("shape", [(3, 4, 2, 1), (3, 4, 2, 2), (4, 3, 5, 5), (2, 6, 3, 4), (5, 5, 5, 6)])
def test_tproduct_fourier_equals_bcirc_definition(shape):
    n1, n2, n4, n3 = shape
    X = random_tensor((n1, n2, n3), seed=1)
    Y = random_tensor((n2, n4, n3), seed=2)
    assert np.allclose(O.tprod(X, Y), O.tprod_bcirc(X, Y), atol=1e-12)


@pytest.mark.parametrize("n3", [1, 3, 4])
def test_transpose_identities(n3):
    X = random_tensor((4, 3, n3), seed=5)
    Y = random_tensor((3, 2, n3), seed=6)
    # (X*Y)^T = Y^T * X^T  (Sec. 2)
    assert np.allclose(O.ttranspose(O.tprod_bcirc(X, Y)),
                       O.tprod_bcirc(O.ttranspose(Y), O.ttranspose(X)), atol=1e-12)
    # bcirc(X^T) = bcirc(X)^T  (Lemma mn2)
    assert np.allclose(O.bcirc(O.ttranspose(X)), O.bcirc(X).T)
    # bcirc(X*Y) = bcirc(X) bcirc(Y)  (Lemma mn2)
    assert np.allclose(O.bcirc(O.tprod_bcirc(X, Y)), O.bcirc(X) @ O.bcirc(Y), atol=1e-12)
    # identity tensor
    Id = O.identity_tensor(4, n3)
    assert np.allclose(O.tprod_bcirc(Id, X), X)


@pytest.mark.parametrize("n3", [3, 4])
def test_transpose_is_slicewise_conjugate_transpose(n3):
    X = random_tensor((4, 3, n3), seed=9)
    Xb = O.dft_mode3(X)
    XTb = O.dft_mode3(O.ttranspose(X))
    for f in range(n3):
        assert np.allclose(XTb[:, :, f], Xb[:, :, f].conj().T, atol=1e-13)


@pytest.mark.parametrize("n3", [3, 4])
def test_block_diagonalisation(n3):
    # eq. (mn35) with the inverse DFT on the right: (F kron I) bcirc(X) (F^{-1} kron I) = bdiag(Xbar)
    n1, n2 = 3, 2
    X = random_tensor((n1, n2, n3), seed=4)
    Fm = O.dft_matrix(n3)
    L = np.kron(Fm, np.eye(n1))
    R = np.kron(np.conj(Fm) / n3, np.eye(n2))
    D = L @ O.bcirc(X) @ R
    Xb = O.dft_mode3(X)
    ref = np.zeros_like(D)
    for f in range(n3):
        ref[f * n1:(f + 1) * n1, f * n2:(f + 1) * n2] = Xb[:, :, f]
    assert np.allclose(D, ref, atol=1e-12)


def test_fourier_and_spatial_norms():
    X = random_tensor((4, 5, 6), seed=1)
    assert abs(O.fro(X) - np.linalg.norm(X)) < 1e-12
    assert O.relative_error(X, X) == 0.0
    assert abs(O.psnr(X, X + 1.0, peak=255.0) - 10 * np.log10(255.0 ** 2)) < 1e-9
