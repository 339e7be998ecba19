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
