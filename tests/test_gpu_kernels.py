"""Kernel-level parity on the GPU: the mode-3 DFT kernels against the oracle's
plain DFT, and the batched complex MFMA product against a float64 product."""
import numpy as np
import pytest
import torch

from oracle import tsvd_oracle as O
from paper_2504_04989_amd import inputs
from tests.gpu_util import load_api, dev, host

pytestmark = pytest.mark.gpu
api = load_api()


@pytest.mark.parametrize("n3", [1, 2, 3, 5, 8, 12, 16, 32, 64, 200, 17, 49])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fft_r2c_c2r_vs_oracle(n3, prec):
    ntubes = 1000 + 3  # several workgroups and an odd tube count
    X = inputs.random_tensor((ntubes, n3), seed=n3)
    dt = torch.float64 if prec == "f64" else torch.float32
    Xd = dev(X, dt)
    Xb = host(api.diag_fft_r2c(Xd))
    Xh = X.astype(np.float32).astype(np.float64) if prec == "f32" else X
    ref = O.dft_mode3(Xh)[:, : n3 // 2 + 1].T          # (F, ntubes)
    tol = 1e-12 if prec == "f64" else 2e-6
    assert np.max(np.abs(Xb - ref)) <= tol * np.max(np.abs(ref))
    # DC and Nyquist exactly real
    assert np.all(Xb[0].imag == 0)
    if n3 % 2 == 0:
        assert np.all(Xb[n3 // 2].imag == 0)
    back = host(api.diag_fft_c2r(api.diag_fft_r2c(Xd), n3))
    assert np.max(np.abs(back - Xh)) <= (1e-13 if prec == "f64" else 2e-6) * np.max(np.abs(Xh)) * max(1, np.log2(n3 + 1))


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fft_c2r_vs_oracle_inverse(prec):
    n3, ntubes = 16, 257
    F = n3 // 2 + 1
    rng = np.random.default_rng(1)
    Xh = rng.standard_normal((F, ntubes)) + 1j * rng.standard_normal((F, ntubes))
    dt = torch.complex128 if prec == "f64" else torch.complex64
    got = host(api.diag_fft_c2r(torch.tensor(Xh, dtype=dt, device="cuda"), n3))
    Xh2 = Xh.astype(np.complex64).astype(np.complex128) if prec == "f32" else Xh.copy()
    Xh2[0].imag = 0
    Xh2[n3 // 2].imag = 0
    ref = O.real_part_checked(O.idft_mode3(O.mirror(Xh2.T, n3)))
    tol = 1e-13 if prec == "f64" else 2e-6
    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref))


def _cplx(shape, seed, dt):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return x, torch.tensor(x, dtype=dt, device="cuda")


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (70, 60, 1000), (1000, 60, 1000), (64, 64, 16), (33, 130, 47),
                                   (200, 7, 3)])
@pytest.mark.parametrize("mode", ["NN", "HN", "NH"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_zgemm_vs_float64(M, N, K, mode, prec):
    dt = torch.complex128 if prec == "f64" else torch.complex64
    batch = 3
    a_conj, b_conj = mode[0] == "H", mode[1] == "H"
    A, Ad = _cplx((batch, K, M) if a_conj else (batch, M, K), 1, dt)
    B, Bd = _cplx((batch, N, K) if b_conj else (batch, K, N), 2, dt)
    C0, Cd = _cplx((batch, M, N), 3, dt)
    got = host(api.diag_zgemm(Ad, Bd, a_conj, b_conj, Cd, alpha=-1.5, beta=0.5))
    if prec == "f32":
        A, B, C0 = (x.astype(np.complex64).astype(np.complex128) for x in (A, B, C0))
    opA = np.conj(np.transpose(A, (0, 2, 1))) if a_conj else A
    opB = np.conj(np.transpose(B, (0, 2, 1))) if b_conj else B
    ref = -1.5 * (opA @ opB) + 0.5 * C0
    tol = 1e-13 if prec == "f64" else 1e-5
    assert np.linalg.norm(got - ref) <= tol * np.linalg.norm(ref)
