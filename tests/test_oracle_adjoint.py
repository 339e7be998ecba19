"""Pins for the oracle's projection P(A) = Q * Q^T * A and its adjoint (CPU only):
central finite differences, PyTorch CPU autograd through torch.fft and
torch.linalg.qr on the literal Krylov blocks, and Euler's identity for the
1-homogeneous map P."""
import numpy as np
import pytest
import torch

from oracle import tsvd_oracle as O
from paper_2504_04989_amd import inputs


def _loss(A, Om, G, b, q):
    return float(np.sum(G * O.proj(A, Om, b, q)))


def test_proj_is_projection_and_idempotent_on_its_range():
    A = inputs.random_tensor((12, 10, 5), 1)
    Om = inputs.omega(10, 2, 5, 1)
    P = O.proj(A, Om, 2, 1)
    # P(A) = Q*Q^T*A with Q T-orthonormal: A - P(A) is T-orthogonal to P(A)
    # (Lemma mn440 then gives the Pythagorean split).
    assert abs(O.fro(A) ** 2 - O.fro(P) ** 2 - O.fro(A - P) ** 2) < 1e-10 * O.fro(A) ** 2
    # m = n1 -> identity map
    A2 = inputs.random_tensor((10, 12, 5), 2)
    Om2 = inputs.omega(12, 5, 5, 1)
    assert np.allclose(O.proj(A2, Om2, 5, 1), A2, atol=1e-12)


def test_adjoint_full_finite_differences_small():
    n1, n2, n3, b, q = 6, 5, 4, 2, 1
    A = inputs.random_tensor((n1, n2, n3), 2)
    Om = inputs.omega(n2, b, n3, 2)
    G = inputs.random_tensor((n1, n2, n3), 3)
    g = O.proj_backward(A, Om, G, b, q)
    h = 1e-6 * np.abs(A).max()
    fd = np.zeros_like(A)
    for idx in np.ndindex(A.shape):
        E = np.zeros_like(A)
        E[idx] = h
        fd[idx] = (_loss(A + E, Om, G, b, q) - _loss(A - E, Om, G, b, q)) / (2 * h)
    assert np.linalg.norm(fd - g) <= 1e-6 * np.linalg.norm(g)


def test_adjoint_directional_finite_differences_masked_crop():
    n1, n2, n3, b, q = 40, 40, 8, 10, 2
    T, M, X0 = inputs.completion_problem(n1, n2, n3, 5, 0.3, seed=3)
    Om = inputs.omega(n2, b, n3, 3)
    P = O.proj(X0, Om, b, q)
    G = -2.0 * M * (T - P)                      # dL/dP of ||M (.) (T - P)||^2
    g = O.proj_backward(X0, Om, G, b, q)
    rng = np.random.default_rng(0)
    h = 1e-6 * np.abs(X0).max()
    for _ in range(4):
        D = rng.standard_normal(X0.shape)
        lp = O.masked_loss(T, M, O.proj(X0 + h * D, Om, b, q))
        lm = O.masked_loss(T, M, O.proj(X0 - h * D, Om, b, q))
        fd = (lp - lm) / (2 * h)
        an = float(np.sum(g * D))
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-12) + 1e-8


def _torch_proj(A, Om, b, q):
    """P(A) over the full spectrum (no conjugate mirror) with the literal
    Krylov blocks and torch's Householder QR."""
    Ab = torch.fft.fft(A.to(torch.complex128), dim=2)
    Ob = torch.fft.fft(Om.to(torch.complex128), dim=2)
    outs = []
    for f in range(A.shape[2]):
        Af, Of = Ab[:, :, f], Ob[:, :, f]
        blocks = [Af @ Of]
        for _ in range(q):
            blocks.append(Af @ (Af.conj().T @ blocks[-1]))
        Q, _ = torch.linalg.qr(torch.cat(blocks, dim=1))
        outs.append(Q @ (Q.conj().T @ Af))
    return torch.fft.ifft(torch.stack(outs, dim=2), dim=2).real


@pytest.mark.parametrize("shape,b,q", [((8, 7, 4), 2, 1), ((10, 9, 5), 3, 1), ((12, 12, 3), 2, 2)])
def test_adjoint_matches_torch_autograd(shape, b, q):
    A = inputs.random_tensor(shape, 4)
    Om = inputs.omega(shape[1], b, shape[2], 4)
    G = inputs.random_tensor(shape, 5)
    At = torch.tensor(A, dtype=torch.float64, requires_grad=True)
    P = _torch_proj(At, torch.tensor(Om), b, q)
    assert np.allclose(P.detach().numpy(), O.proj(A, Om, b, q), atol=1e-11)
    (P * torch.tensor(G)).sum().backward()
    g_ref = At.grad.numpy()
    g = O.proj_backward(A, Om, G, b, q)
    assert np.linalg.norm(g - g_ref) <= 1e-9 * np.linalg.norm(g_ref)


def test_adjoint_euler_homogeneity():
    A = inputs.random_tensor((14, 12, 6), 6)
    Om = inputs.omega(12, 3, 6, 6)
    G = inputs.random_tensor((14, 12, 6), 7)
    g = O.proj_backward(A, Om, G, 3, 2)
    P = O.proj(A, Om, 3, 2)
    assert abs(np.sum(g * A) - np.sum(G * P)) <= 1e-10 * abs(np.sum(G * P))
