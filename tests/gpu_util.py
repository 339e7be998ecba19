"""Helpers shared by the GPU parity tests (no method arithmetic here: only
transfers, norms and the comparison metrics)."""
import numpy as np
import pytest
import torch

DEV = "cuda"


def load_api():
    """The HIP binding.  Without a GPU the GPU tests are skipped; with a GPU a
    missing library is an error, never a silent skip."""
    try:
        from paper_2504_04989_amd import api
        return api
    except ImportError:
        if torch.cuda.is_available():
            raise
        pytest.skip("library not built and no GPU", allow_module_level=True)


def dev(x: np.ndarray, dtype=torch.float64) -> torch.Tensor:
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


def host(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


def rel_f(x, ref) -> float:
    """||x - ref||_F / ||ref||_F."""
    return float(np.linalg.norm((np.asarray(x) - np.asarray(ref)).ravel()) / np.linalg.norm(np.asarray(ref).ravel()))


def fourier_factors(U, S, V, freqs):
    """Fourier-domain factors of spatial outputs at the given frequencies
    (host numpy FFT; the GPU outputs are only transformed for comparison)."""
    Ub = np.fft.fft(U, axis=2)[:, :, freqs]
    Vb = np.fft.fft(V, axis=2)[:, :, freqs]
    Sb = np.fft.fft(S, axis=1)[:, freqs]
    return Ub, Sb, Vb


def unambiguous_phase_columns(Uf, rel_gap=1e-3):
    """Columns whose largest-modulus entry is separated from the runner-up, so
    the phase convention picks the same entry on both sides."""
    ok = []
    for j in range(Uf.shape[1]):
        a = np.sort(np.abs(Uf[:, j]))[::-1]
        ok.append(len(a) < 2 or a[0] - a[1] > rel_gap * a[0])
    return np.array(ok)


def fp32_twin_slice(A, Om, k, b, q, f):
    """The floor of FP32 arithmetic on one Fourier slice: the stabilised block
    Krylov method of Alg. 2 run entirely in complex64 with numpy / LAPACK
    primitives (QR, SVD), on the same inputs.  Returns (X_hat_f, sigma_1..k).
    Test infrastructure: it measures what a plain FP32 computation of the slice
    reaches, so that a GPU error can be told apart from the FP32 limit."""
    w = np.exp(-2j * np.pi * f * np.arange(A.shape[2]) / A.shape[2])
    return fp32_twin_slice_f(A @ w, Om @ w, k, b, q)


def _bf16(x):
    """Round float32 values to bfloat16 (nearest even), returned as float32."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(torch.bfloat16).to(torch.float32).numpy()


def _split16(z):
    """Complex64 z -> (hi, lo): hi = bf16(z), lo = bf16(z - hi) per real part."""
    z = np.asarray(z, dtype=np.complex64)
    hr, hi = _bf16(z.real), _bf16(z.imag)
    lr, li = _bf16(z.real - hr), _bf16(z.imag - hi)
    return (hr + 1j * hi).astype(np.complex64), (lr + 1j * li).astype(np.complex64)


def _x3(X, Y):
    """The three-product BF16 form of X @ Y: hi hi + hi lo + lo hi with
    float32 accumulation (complex64 products of bf16-valued operands)."""
    Xh, Xl = _split16(X)
    Yh, Yl = _split16(Y)
    return (Xh @ Yh) + (Xh @ Yl) + (Xl @ Yh)


def bf16x3_twin_slice_f(Af, Of, k, b, q):
    """fp32_twin_slice_f with every Krylov product (A Omega, A^H Q, A T and
    Q^H A) in the three-product BF16 form of the GPU's BF16x3 mode: the floor
    of that arithmetic (both operands held to 16 significant bits)."""
    Af = np.asarray(Af).astype(np.complex64)
    Of = np.asarray(Of).astype(np.complex64)
    Ah = np.ascontiguousarray(Af.conj().T)
    Qs = [np.linalg.qr(_x3(Af, Of))[0]]
    for _ in range(q):
        W = _x3(Af, _x3(Ah, Qs[-1]))
        Qp = np.concatenate(Qs, axis=1)
        W = W - Qp @ (Qp.conj().T @ W)
        W = W - Qp @ (Qp.conj().T @ W)
        Qs.append(np.linalg.qr(W)[0])
    Q = np.concatenate(Qs, axis=1)
    C = _x3(Ah, Q).conj().T
    W, s, Zh = np.linalg.svd(C, full_matrices=False)
    return ((Q @ W[:, :k]) * s[:k]) @ Zh[:k], s[:k].astype(np.float64)


def fp32_twin_slice_f(Af, Of, k, b, q):
    """fp32_twin_slice on a slice whose DFT is already taken (Af n1 x n2,
    Of n2 x b), rounded here to complex64."""
    Af = np.asarray(Af).astype(np.complex64)
    Of = np.asarray(Of).astype(np.complex64)
    Qs = [np.linalg.qr(Af @ Of)[0]]
    for _ in range(q):
        W = Af @ (Af.conj().T @ Qs[-1])
        Qp = np.concatenate(Qs, axis=1)
        W = W - Qp @ (Qp.conj().T @ W)
        W = W - Qp @ (Qp.conj().T @ W)
        Qs.append(np.linalg.qr(W)[0])
    Q = np.concatenate(Qs, axis=1)
    W, s, Zh = np.linalg.svd(Q.conj().T @ Af, full_matrices=False)
    return ((Q @ W[:, :k]) * s[:k]) @ Zh[:k], s[:k].astype(np.float64)
