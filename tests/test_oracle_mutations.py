"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each case applies one textual mutation to a copy of the oracle's source
(a dropped conjugate, a wrong sign, a missing 1/n3, a wrong index, a dropped
adjoint term), loads the copy as a separate module and checks that the named
pin rejects it.  The oracle on disk is never modified.
"""
import inspect
import types

import numpy as np
import pytest

from oracle import tsvd_oracle
from paper_2504_04989_amd import inputs

SRC = inspect.getsource(tsvd_oracle)


def _mutant(old: str, new: str):
    assert SRC.count(old) == 1, f"mutation anchor not unique: {old!r}"
    mod = types.ModuleType("oracle_mutant")
    exec(compile(SRC.replace(old, new), "oracle_mutant", "exec"), mod.__dict__)
    return mod


# ---- pins, parameterised by the module under test -------------------------

def pin_dft(O):
    X = inputs.random_tensor((3, 2, 8), 1)
    assert np.allclose(O.dft_mode3(X), np.fft.fft(X, axis=2), atol=1e-12)


def pin_tprod(O):
    X = inputs.random_tensor((3, 4, 5), 1)
    Y = inputs.random_tensor((4, 2, 5), 2)
    assert np.allclose(O.tprod(X, Y), O.tprod_bcirc(X, Y), atol=1e-12)


def pin_qr(O):
    K = inputs.random_tensor((9, 4), 3) + 1j * inputs.random_tensor((9, 4), 4)
    Q, R = O.householder_qr(K)
    assert np.allclose(Q.conj().T @ Q, np.eye(4), atol=1e-12)
    assert np.allclose(Q @ R, K, atol=1e-12)


def pin_svd(O):
    C = inputs.random_tensor((5, 8), 5) + 1j * inputs.random_tensor((5, 8), 6)
    W, s, Z, _ = O.jacobi_svd(C, max_sweeps=30)
    assert np.allclose(s, np.linalg.svd(C, compute_uv=False), atol=1e-12)
    assert np.allclose((W * s) @ Z.conj().T, C, atol=1e-12)


def pin_krylov_spatial(O):
    A = inputs.random_tensor((9, 8, 5), 3)
    b, q = 2, 2
    Om = inputs.omega(8, b, 5, 3)
    Ks = [O.tprod_bcirc(A, Om)]
    for _ in range(q):
        Ks.append(O.tprod_bcirc(A, O.tprod_bcirc(O.ttranspose(A), Ks[-1])))
    Kb = np.fft.fft(np.concatenate(Ks, axis=1), axis=2)
    sl = O.rbk_slices(A, Om, 1, b, q)
    for f in range(3):
        Q = sl["Q"][:, :, f]
        assert np.allclose(Q.conj().T @ Q, np.eye(b * (q + 1)), atol=1e-12)
        res = Kb[:, :, f] - Q @ (Q.conj().T @ Kb[:, :, f])
        assert np.linalg.norm(res) < 1e-10 * np.linalg.norm(Kb[:, :, f])


def pin_power_spatial(O):
    A = inputs.random_tensor((9, 8, 5), 25)
    b, q = 3, 2
    Om = inputs.omega(8, b, 5, 25)
    Y = O.tprod_bcirc(A, Om)
    for _ in range(q):
        Y = O.tprod_bcirc(A, O.tprod_bcirc(O.ttranspose(A), Y))
    Yb = np.fft.fft(Y, axis=2)
    sl = O.power_slices(A, Om, 1, b, q)
    for f in range(3):
        Q = sl["Q"][:, :, f]
        res = Yb[:, :, f] - Q @ (Q.conj().T @ Yb[:, :, f])
        assert np.linalg.norm(res) < 1e-10 * np.linalg.norm(Yb[:, :, f])


def pin_tqr(O):
    X = inputs.random_tensor((7, 5, 4), 41)
    Q, R = O.tqr(X)
    assert np.allclose(O.tprod_bcirc(Q, R), X, atol=1e-12 * np.abs(X).max())
    assert np.allclose(O.tprod_bcirc(O.ttranspose(Q), Q), O.identity_tensor(5, 4), atol=1e-12)


def pin_tpinv(O):
    X = inputs.random_tensor((7, 5, 4), 43)
    P = O.tpinv(X)
    assert np.allclose(O.tprod_bcirc(O.tprod_bcirc(X, P), X), X, atol=1e-10)
    assert np.allclose(O.tprod_bcirc(P, X), O.identity_tensor(5, 4), atol=1e-10)


def pin_tpinv_cutoff(O):
    g = np.random.default_rng(51)
    U, _ = np.linalg.qr(g.standard_normal((6, 3)))
    V, _ = np.linalg.qr(g.standard_normal((4, 3)))
    s = np.array([4.0, 2.0, 1e-3])
    X = ((U * s) @ V.T)[:, :, None]
    want = (V[:, :2] / s[:2]) @ U[:, :2].T
    assert np.allclose(O.tpinv(X, rtol=1e-2)[:, :, 0], want, atol=1e-9)


def pin_complete(O):
    M = inputs.exact_lowrank_tensor(20, 24, 3, 2, seed=64)
    T = inputs.bernoulli_mask(M.shape, 0.6, 64)
    C = O.complete(M, T, inputs.omega(24, 4, 3, 64), 2, 4, 1, 60)
    assert np.array_equal(C[T == 1], M[T == 1])
    assert O.relative_error(M, C) < 0.1 * O.relative_error(M, T * M)


def pin_exact_tsvd(O):
    # m = n1: Alg. 2 must equal the truncated T-SVD computed with numpy's SVD.
    n1, n2, n3, k = 20, 24, 4, 5
    A = inputs.random_tensor((n1, n2, n3), 7)
    Om = inputs.omega(n2, 10, n3, 7)
    sl = O.rbk_tsvd(A, Om, k, 10, 1)
    Xh = O.approx_from_slices(sl, n1, n2, n3)
    Ab = np.fft.fft(A, axis=2)
    Xe = np.zeros_like(Ab)
    for f in range(n3):
        u, s, vh = np.linalg.svd(Ab[:, :, f])
        Xe[:, :, f] = (u[:, :k] * s[:k]) @ vh[:k]
    Xe = np.fft.ifft(Xe, axis=2).real
    assert np.linalg.norm(Xh - Xe) < 1e-11 * np.linalg.norm(Xe)


def pin_adjoint_fd(O):
    n1, n2, n3, b, q = 6, 5, 3, 2, 1
    A = inputs.random_tensor((n1, n2, n3), 2)
    Om = inputs.omega(n2, b, n3, 2)
    G = inputs.random_tensor((n1, n2, n3), 3)
    g = O.proj_backward(A, Om, G, b, q)
    h = 1e-6
    rng = np.random.default_rng(1)
    for _ in range(3):
        D = rng.standard_normal(A.shape)
        fd = (np.sum(G * O.proj(A + h * D, Om, b, q)) - np.sum(G * O.proj(A - h * D, Om, b, q))) / (2 * h)
        assert abs(fd - np.sum(g * D)) <= 1e-6 * abs(fd) + 1e-9


def pin_approx_adjoint_fd(O):
    n1, n2, n3, k, b, q = 7, 6, 3, 2, 3, 1
    A = inputs.random_tensor((n1, n2, n3), 12)
    Om = inputs.omega(n2, b, n3, 12)
    G = inputs.random_tensor((n1, n2, n3), 13)
    g = O.approx_backward(A, Om, G, k, b, q)
    h = 1e-6
    rng = np.random.default_rng(2)
    for _ in range(3):
        D = rng.standard_normal(A.shape)
        fd = (np.sum(G * O.rbk_approx(A + h * D, Om, k, b, q)) - np.sum(G * O.rbk_approx(A - h * D, Om, k, b, q))) / (2 * h)
        assert abs(fd - np.sum(g * D)) <= 1e-6 * abs(fd) + 1e-9


def pin_ritz(O):
    n1, n2, n3, k, b, q = 12, 10, 4, 3, 4, 1
    A = inputs.random_tensor((n1, n2, n3), 14)
    Om = inputs.omega(n2, b, n3, 14)
    sr = O.ritz_slices(A, Om, k, b, q)
    sf = O.rbk_slices(A, Om, k, b, q)
    assert np.allclose(sr["s_all"], sf["s_all"][:b], atol=1e-12 * sf["s_all"].max())
    assert np.allclose(O.approx_from_slices(sr, n1, n2, n3), O.approx_from_slices(sf, n1, n2, n3), atol=1e-12)


MUTATIONS = [
    ("dft sign", "- 1j * np.sin(2.0 * np.pi * r / n)", "+ 1j * np.sin(2.0 * np.pi * r / n)", pin_dft),
    ("mirror without conj", "full[..., f] = np.conj(Xh[..., n3 - f])", "full[..., f] = Xh[..., n3 - f]", pin_tprod),
    ("idft missing 1/n3", "Finv = np.conj(dft_matrix(n3)) / n3", "Finv = np.conj(dft_matrix(n3))", pin_tprod),
    ("householder tau", "tau = ((beta - x0) / beta).real", "tau = 0.5 * ((beta - x0) / beta).real", pin_qr),
    ("householder reflector without conj", "R[j:, j:] -= tau * np.outer(v, v.conj() @ R[j:, j:])",
     "R[j:, j:] -= tau * np.outer(v, v @ R[j:, j:])", pin_qr),
    ("jacobi rotation sign", "M[:, p] = c * mp - s * eph * mq", "M[:, p] = c * mp + s * eph * mq", pin_svd),
    ("jacobi phase", "eph = np.conj(gamma / ag)", "eph = gamma / ag", pin_svd),
    ("krylov transpose without conj", "W = Af @ (Af.conj().T @ Qs[-1])", "W = Af @ (Af.T @ Qs[-1])", pin_krylov_spatial),
    ("reorthogonalisation sign",
     "Y = W - Qp @ (Qp.conj().T @ W)\n        Y, _ = householder_qr(Y)\n        Y = Y - Qp @ (Qp.conj().T @ Y)",
     "Y = W + Qp @ (Qp.conj().T @ W)\n        Y, _ = householder_qr(Y)\n        Y = Y + Qp @ (Qp.conj().T @ Y)",
     pin_krylov_spatial),
    ("power iterate transpose without conj", "Qt, _ = householder_qr(Af.conj().T @ Qp)",
     "Qt, _ = householder_qr(Af.T @ Qp)", pin_power_spatial),
    ("power iteration one short", "    for _ in range(q):\n        Qt, _ =", "    for _ in range(q - 1):\n        Qt, _ =",
     pin_power_spatial),
    ("power basis without A^H", "Qt, _ = householder_qr(Af.conj().T @ Qp)", "Qt, _ = householder_qr(Qp[:Af.shape[1]])",
     pin_power_spatial),
    ("tqr phase applied twice to R", "Rh[:, :, f] = R * ph[:, None]", "Rh[:, :, f] = R * np.conj(ph)[:, None]",
     pin_tqr),
    ("tqr R without conj", "R = np.triu(Q.conj().T @ Xb[:, :, f])", "R = np.triu(Q.T @ Xb[:, :, f])", pin_tqr),
    ("tpinv conjugated", "Ch[:, :, f] = (Vh.conj().T * sp[None, :]) @ U.conj().T",
     "Ch[:, :, f] = ((Vh.conj().T * sp[None, :]) @ U.conj().T).conj()", pin_tpinv),
    ("tpinv cut-off against the smallest value", "keep = s > rtol * s[0]", "keep = s > rtol * s[-1]",
     pin_tpinv_cutoff),
    ("tpinv keeps every value", "keep = s > rtol * s[0]", "keep = s >= 0.0", pin_tpinv_cutoff),
    ("completion merge with the mask swapped", "C = T * Mobs + (1.0 - T) * X", "C = (1.0 - T) * Mobs + T * X",
     pin_complete),
    ("completion never updates C", "C = T * Mobs + (1.0 - T) * X", "C = T * Mobs + 0.0 * X", pin_complete),
    ("projection without conj", "C = Q.conj().T @ Af", "C = Q.T @ Af", pin_exact_tsvd),
    ("truncation off by one", "canonical_phase(Q @ W[:, :k], Z[:, :k])", "canonical_phase(Q @ W[:, :k], Z[:, 1:k + 1])", pin_exact_tsvd),
    ("lift with conj", "canonical_phase(Q @ W[:, :k], Z", "canonical_phase(Q @ W[:, :k].conj(), Z", pin_exact_tsvd),
    ("adjoint direct term dropped", "Abar = Q @ (Q.conj().T @ Yb)", "Abar = 0 * Yb", pin_adjoint_fd),
    ("adjoint Qbar term dropped", "Qbar_all = Yb @ (A.conj().T @ Q) + A @ (Yb.conj().T @ Q)",
     "Qbar_all = Yb @ (A.conj().T @ Q)", pin_adjoint_fd),
    ("adjoint reverse Krylov term dropped", "Abar += Qs[i - 1] @ Tbar.conj().T", "pass", pin_adjoint_fd),
    ("adjoint R^-H dropped", "Zbar0 = np.linalg.solve(R0, X.conj().T).conj().T", "Zbar0 = X", pin_adjoint_fd),
    ("truncation adjoint without the eigenvector term", "Cbar = Pi @ Y + H @ C", "Cbar = Pi @ Y",
     pin_approx_adjoint_fd),
    ("truncation adjoint gap sign", "N[c, a] = M[c, a] / (lam[a] - lam[c])", "N[c, a] = M[c, a] / (lam[c] - lam[a])",
     pin_approx_adjoint_fd),
    ("truncation adjoint Qbar without the projector", "Qbar_all = Yb @ (C.conj().T @ Pi) + A @ Cbar.conj().T",
     "Qbar_all = Yb @ C.conj().T + A @ Cbar.conj().T", pin_approx_adjoint_fd),
    ("truncated basis as the first r columns", "canonical_phase(Q @ W[:, :r], np.zeros",
     "canonical_phase(Q[:, :r] + 0 * W[:1, :r], np.zeros", pin_ritz),
    ("truncated basis from the smallest Ritz values", "canonical_phase(Q @ W[:, :r], np.zeros",
     "canonical_phase(Q @ W[:, -r:], np.zeros", pin_ritz),
]


@pytest.mark.parametrize("name,old,new,pin", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pin_rejects_planted_mistake(name, old, new, pin):
    pin(tsvd_oracle)                  # the real oracle passes the pin ...
    mutant = _mutant(old, new)
    with pytest.raises((AssertionError, ValueError, RuntimeError, np.linalg.LinAlgError)):
        pin(mutant)                   # ... and the planted mistake does not
