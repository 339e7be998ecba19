"""Kernel-level check of the small Hermitian eigensolver (the per-slice SVD of
C_f in Alg. 2 taken through C_f C_f^H, FP64): tridiagonalisation, bisection,
inverse iteration and back-transformation against LAPACK's eigh."""
import numpy as np
import pytest
import torch

from tests.gpu_util import load_api, host

pytestmark = pytest.mark.gpu
api = load_api()


def _gram(batch, m, seed, decay):
    """Hermitian PSD matrices B B^H with singular values of B decaying as
    (i + 1)^-decay (the spectrum shape of the Krylov Gram matrices)."""
    rng = np.random.default_rng(seed)
    out = np.empty((batch, m, m), dtype=np.complex128)
    for f in range(batch):
        U, _ = np.linalg.qr(rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))
        s = (np.arange(m) + 1.0) ** -decay
        out[f] = (U * s**2) @ U.conj().T
    return out


# m >= 256 with several workgroups per slice: the register-resident
# tridiagonalisation while the slice's tiles fit (440 / 448 over 33 slices is
# the 4096 x 4096 x 64 workload's shape; 256 and 300 exact and ragged tile
# counts), the streaming form beyond it (600 over 33 slices)
@pytest.mark.parametrize("m,k,batch", [(1, 1, 2), (2, 1, 3), (37, 10, 3), (120, 30, 5), (440, 100, 3),
                                       (256, 60, 33), (300, 64, 7), (440, 100, 33), (448, 90, 33), (600, 50, 33)])
def test_heig_vs_lapack(m, k, batch):
    print(f"[heig] m={m} k={k} batch={batch}", flush=True)
    G = _gram(batch, m, seed=m, decay=1.5)
    lam, W, info = api.diag_heig(torch.tensor(G, device="cuda"), k)
    lam, W = host(lam), host(W)
    assert info["eig_noconv"] == 0 and info["nonfinite"] == 0
    for f in range(batch):
        ref = np.linalg.eigvalsh(G[f])[::-1][:k]
        nrm = np.abs(ref[0])
        assert np.max(np.abs(lam[f] - ref)) <= 1e-13 * m * nrm
        Wf = W[f]
        # residual and orthonormality of the computed eigenvectors
        R = G[f] @ Wf - Wf * lam[f]
        assert np.max(np.linalg.norm(R, axis=0)) <= 1e-12 * m * nrm
        assert np.max(np.abs(Wf.conj().T @ Wf - np.eye(k))) <= 1e-10


def test_heig_clustered_and_degenerate():
    # repeated eigenvalues (an exact cluster) and a zero block
    m, k, batch = 64, 20, 2
    rng = np.random.default_rng(7)
    G = np.empty((batch, m, m), dtype=np.complex128)
    for f in range(batch):
        U, _ = np.linalg.qr(rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))
        lam = np.concatenate([np.full(8, 2.0), np.linspace(1.0, 0.5, 24), np.zeros(32)])
        G[f] = (U * lam) @ U.conj().T
    lam, W, info = api.diag_heig(torch.tensor(G, device="cuda"), k)
    lam, W = host(lam), host(W)
    assert info["eig_noconv"] == 0
    for f in range(batch):
        ref = np.linalg.eigvalsh(G[f])[::-1][:k]
        assert np.max(np.abs(lam[f] - ref)) <= 1e-12
        R = G[f] @ W[f] - W[f] * lam[f]
        assert np.max(np.linalg.norm(R, axis=0)) <= 1e-11
        assert np.max(np.abs(W[f].conj().T @ W[f] - np.eye(k))) <= 1e-10


def test_heig_repeats_bit_for_bit():
    """Two calls on the same matrices give the same eigenpairs bit for bit
    (the tridiagonalisation's sums are exact integer sums), at the 4096 x 4096
    x 64 workload's shape (m = 440 over 33 slices)."""
    G = torch.tensor(_gram(33, 440, seed=5, decay=1.5), device="cuda")
    l1, W1, _ = api.diag_heig(G, 100)
    l2, W2, _ = api.diag_heig(G, 100)
    assert torch.equal(l1, l2) and torch.equal(W1, W2)
