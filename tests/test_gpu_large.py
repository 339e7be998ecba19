"""Tensors of more than 2^31 entries (9.2 GB in FP32): 1024 x 1100 x 2048
(1025 Fourier slices of 1.13e6 complex entries, the power-of-two DFT and
the Krylov products converting to BF16 on load) and 6000 x 6000 x 64 (33
slices of 3.6e7 entries, the register DFT that writes the BF16x3 split
pairs).  The offsets across slices and into the whole tensor pass 2^31, so
every kernel that addresses the input, its half spectrum or a slice's
factors beyond the first 2^31 entries takes its 64-bit path.

The input is the separable recipe: every Fourier slice is a rank-8 matrix
plus a multiple of one dense Gaussian matrix at 1e-3 of its scale, so the
rank-8 truncation is well separated from the rest.  The tensor is assembled
on the device from its factors (an FP32 product of the factor matrices);
the FP64 oracle forms each sampled slice from the same factors by linearity
of the mode-3 DFT (Sec. 2) and runs Alg. 2 on it with the same seeded test
tensor, rounded to FP32 as the library stores it."""
import numpy as np
import pytest
import torch

from oracle import tsvd_oracle as orc
from paper_2504_04989_amd import inputs
from tests.gpu_util import fourier_factors, host, load_api

R, K, B, Q = 8, 8, 12, 1
SEED = 31
DECAY, NOISE = 0.75, 1e-3
# DC, the first, two interior and the Nyquist slice
SHAPES = {(1024, 1100, 2048): [0, 1, 511, 1023, 1024], (6000, 6000, 64): [0, 1, 16, 31, 32]}
TOL = {"f32": 1e-5, "bf16x3": 1e-4}


def separable_slices(factors, freqs):
    """Fourier slices of the separable tensor at the given frequencies, from
    its factors: sum_c Sp_hat[f, c] G[:, c] H[:, c]^T + noise w_hat[f] Nz, with
    the oracle's DFT of the length-n3 factors (Sec. 2)."""
    G, H, Sp, Nz, w, noise = factors
    s_hat = orc.dft_mode3(np.ascontiguousarray(Sp.T)[None], freqs)[0]      # r x nf
    w_hat = orc.dft_mode3(w[None, None, :], freqs)[0, 0]                  # nf
    return [(G * s_hat[:, i]) @ H.T + noise * w_hat[i] * Nz for i in range(len(freqs))]


def test_separable_slices_match_the_dft_of_the_tensor():
    # the slice assembly above against the oracle's DFT of the whole tensor
    fac = inputs.separable_factors(12, 9, 10, 3, DECAY, NOISE, 4)
    A = inputs.separable_tensor(fac)
    freqs = [0, 1, 3, 5]
    Ab = orc.dft_mode3(A, freqs)
    for i, Af in enumerate(separable_slices(fac, freqs)):
        assert np.max(np.abs(Af - Ab[:, :, i])) <= 1e-13 * np.max(np.abs(Ab))


def _device_tensor(fac, shape):
    """A as FP32 on the device, (n1, n2, n3) with tubes contiguous: the
    (n1 n2) x r matrix of g_c(i) h_c(j) times Sp^T, plus noise Nz w^T."""
    n1, n2, n3 = shape
    G, H, Sp, Nz, w, noise = fac
    P = (G[:, None, :] * H[None, :, :]).reshape(n1 * n2, R)
    A = torch.empty((n1 * n2, n3), dtype=torch.float32, device="cuda")
    torch.mm(torch.from_numpy(P).float().cuda(), torch.from_numpy(np.ascontiguousarray(Sp.T)).float().cuda(), out=A)
    A.addr_(torch.from_numpy(Nz.ravel()).float().cuda(), torch.from_numpy(w).float().cuda(), alpha=noise)
    return A.view(n1, n2, n3)


_CACHE = {}


def _oracle(shape):
    """Factors, and the oracle's X_hat and sigma on the sampled slices."""
    if shape not in _CACHE:
        _CACHE.clear()
        n1, n2, n3 = shape
        fac = inputs.separable_factors(n1, n2, n3, R, DECAY, NOISE, SEED)
        Om = inputs.omega(n2, B, n3, SEED).astype(np.float32).astype(np.float64)
        Ob = orc.dft_mode3(Om, SHAPES[shape])
        del Om
        out = []
        for i, Af in enumerate(separable_slices(fac, SHAPES[shape])):
            sl = orc.rbk_slice(Af, Ob[:, :, i], K, B, Q)
            out.append(((sl["Uf"] * sl["Sf"]) @ sl["Vf"].conj().T, sl["Sf"], sl["s_all"]))
        _CACHE[shape] = (fac, out)
    return _CACHE[shape]


@pytest.mark.gpu
@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
@pytest.mark.parametrize("shape", list(SHAPES))
def test_tensor_beyond_2_pow_31_entries(shape, prec):
    api = load_api()
    n1, n2, n3 = shape
    freqs = SHAPES[shape]
    fac, ref = _oracle(shape)
    print(f"[large] {n1}x{n2}x{n3} ({n1 * n2 * n3:.3e} entries) k={K} b={B} q={Q} seed={SEED} prec={prec}",
          flush=True)
    A = _device_tensor(fac, shape)
    U, S, V = api.tsvd_rbk(A, SEED, K, B, Q, prec)
    torch.cuda.synchronize()
    del A
    U, S, V = (host(t).astype(np.float64) for t in (U, S, V))
    Ub, Sb, Vb = fourier_factors(U, S, V, freqs)
    for i, f in enumerate(freqs):
        Xo, so, s_all = ref[i]
        Xg = (Ub[:, :, i] * Sb[:, i].real) @ Vb[:, :, i].conj().T
        ex = np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo)
        es = np.max(np.abs(Sb[:, i].real - so) / so)
        print(f"[large] {prec} slice {f}: X rel {ex:.2e}, sigma rel max {es:.2e}, "
              f"sigma_k/sigma_1 {so[-1] / so[0]:.1e}, sigma_(k+1)/sigma_k {s_all[K] / so[-1]:.1e}", flush=True)
        assert ex <= TOL[prec]
        assert es <= TOL[prec]
