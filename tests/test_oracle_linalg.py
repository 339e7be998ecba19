"""Pins for the oracle's per-slice Householder QR and one-sided Jacobi SVD
(CPU only): invariants, numpy.linalg as an independent library routine, and
the orthogonal-tensor identity of Sec. 2."""
import numpy as np
import pytest

from oracle import tsvd_oracle as O
from paper_2504_04989_amd.inputs import random_tensor


def _cplx(shape, seed):
    return random_tensor(shape, seed) + 1j * random_tensor(shape, seed + 100)


@pytest.mark.parametrize("shape", [(6, 6), (9, 4), (30, 10), (5, 1)])
@pytest.mark.parametrize("complex_", [False, True])
def test_householder_qr_invariants_and_numpy(shape, complex_):
    K = _cplx(shape, 3) if complex_ else random_tensor(shape, 3)
    Q, R = O.householder_qr(K)
    m = shape[1]
    assert np.allclose(Q.conj().T @ Q, np.eye(m), atol=1e-13)
    assert np.allclose(Q @ R, K, atol=1e-13)
    assert np.allclose(R, np.triu(R))
    Qn, Rn = np.linalg.qr(K)
    # Same factorisation up to a unit-modulus scaling of each column.
    assert np.allclose(np.abs(np.diag(R)), np.abs(np.diag(Rn)), atol=1e-12)
    for j in range(m):
        ph = np.vdot(Q[:, j], Qn[:, j])
        assert abs(abs(ph) - 1) < 1e-12
        assert np.allclose(Q[:, j] * ph, Qn[:, j], atol=1e-12)
    if not complex_:
        assert np.all(Q.imag == 0) and np.all(R.imag == 0)


def test_householder_qr_rank_deficient_keeps_orthonormal_q():
    B = random_tensor((12, 3), 1)
    K = np.concatenate([B, B[:, :1] * 2.0, np.zeros((12, 1))], axis=1)
    Q, R = O.householder_qr(K)
    assert np.allclose(Q.conj().T @ Q, np.eye(5), atol=1e-13)
    assert np.allclose(Q @ R, K, atol=1e-13)


@pytest.mark.parametrize("shape", [(1, 1), (3, 3), (4, 9), (10, 25), (16, 16)])
@pytest.mark.parametrize("complex_", [False, True])
def test_jacobi_svd_vs_numpy(shape, complex_):
    C = _cplx(shape, 5) if complex_ else random_tensor(shape, 5)
    W, s, Z, sweeps = O.jacobi_svd(C)
    sn = np.linalg.svd(C, compute_uv=False)
    assert np.allclose(s, sn, atol=1e-13 * sn[0])
    assert np.all(np.diff(s) <= 0)
    assert np.allclose((W * s) @ Z.conj().T, C, atol=1e-12 * sn[0])
    m = shape[0]
    assert np.allclose(W.conj().T @ W, np.eye(m), atol=1e-12)
    assert np.allclose(Z.conj().T @ Z, np.eye(m), atol=1e-12)
    if not complex_:
        assert np.all(W.imag == 0) and np.all(Z.imag == 0)


def test_jacobi_svd_graded_spectrum():
    # Singular values over 10 decades: still relative-accurate at the top.
    rng = np.random.default_rng(0)
    m, n = 12, 20
    U, _ = np.linalg.qr(rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))
    V, _ = np.linalg.qr(rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m)))
    sv = np.logspace(0, -10, m)
    C = (U * sv) @ V.conj().T
    _, s, _, _ = O.jacobi_svd(C)
    assert np.allclose(s[:6], sv[:6], rtol=1e-10)


def test_tqr_gives_orthogonal_tensor():
    # Alg. TQR on a square tensor: Q^T * Q = Q * Q^T = I (Sec. 2, orthogonal tensor).
    n, n3 = 5, 4
    X = random_tensor((n, n, n3), 2)
    Xb = O.dft_mode3(X)
    F = O.n_half(n3)
    Qh = np.zeros((n, n, F), complex)
    for f in range(F):
        Qh[:, :, f], _ = O.householder_qr(Xb[:, :, f])
    Q = O.real_part_checked(O.idft_mode3(O.mirror(Qh, n3)))
    Id = O.identity_tensor(n, n3)
    assert np.allclose(O.tprod_bcirc(O.ttranspose(Q), Q), Id, atol=1e-12)
    assert np.allclose(O.tprod_bcirc(Q, O.ttranspose(Q)), Id, atol=1e-12)


def test_canonical_phase_makes_max_entry_real_positive():
    U = _cplx((7, 3), 1)
    V = _cplx((5, 3), 2)
    Uc, Vc = O.canonical_phase(U, V)
    for j in range(3):
        i = np.argmax(np.abs(Uc[:, j]))
        assert abs(Uc[i, j].imag) < 1e-15 and Uc[i, j].real > 0
    assert np.allclose(Uc @ Vc.conj().T, U @ V.conj().T)
