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
    if prec == "f64":
        assert np.max(np.abs(Xb - ref)) <= 1e-12 * np.max(np.abs(ref))
    else:
        # FP64 arithmetic inside, one rounding to FP32 on output: every element
        # is within half an FP32 ulp of the exact DFT (plus FP64 noise)
        err = np.abs(Xb.real - ref.real) + 1j * np.abs(Xb.imag - ref.imag)
        bound = 2.0 ** -24 * (np.abs(ref.real) + 1j * np.abs(ref.imag)) + 1e-12 * np.max(np.abs(ref))
        assert np.all(err.real <= bound.real) and np.all(err.imag <= bound.imag)
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


KG_CASES = [  # (batch, rows, cols, N, nsplit)
    (2, 70, 90, 5, 1),        # ragged tiles, tiny N
    (3, 130, 257, 60, 1),     # odd row stride: scalar big-operand loads
    (1, 33, 48, 128, 1),      # N = 128: one full thin chunk
    (2, 64, 64, 130, 1),      # N > 128: two thin chunks
    (2, 300, 520, 110, 3),    # split over K with a ragged last chunk
    (1, 16, 16, 1, 1),
]


@pytest.mark.parametrize("case", KG_CASES)
@pytest.mark.parametrize("herm", [False, True])
@pytest.mark.parametrize("mode", ["f32", "bf16x3", "bf16"])
def test_kgemm_vs_float64(case, herm, mode):
    """The Krylov-product kernel, op(A_f) X_f, against a float64 product of the
    same complex64 inputs."""
    batch, rows, cols, N, ns = case
    K = rows if herm else cols
    A, Ad = _cplx((batch, rows, cols), 1, torch.complex64)
    X, Xd = _cplx((batch, K, N), 2, torch.complex64)
    A, X = A.astype(np.complex64).astype(np.complex128), X.astype(np.complex64).astype(np.complex128)
    C = host(api.diag_kgemm(Ad, Xd, herm=herm, mode=mode, nsplit=ns))
    ref = (np.conj(np.swapaxes(A, 1, 2)) if herm else A) @ X
    err = np.linalg.norm((C - ref).ravel()) / np.linalg.norm(ref.ravel())
    tol = {"f32": 1e-6, "bf16x3": 2e-5, "bf16": 1e-2}[mode]
    assert err <= tol, f"rel err {err:.2e}"


@pytest.mark.parametrize("case", [(2, 70, 90, 5), (3, 200, 330, 110), (2, 4096, 110, 110), (1, 16, 1, 1),
                                  (33, 130, 220, 110)])
def test_kgemm_update_form_vs_float64(case):
    """The update form C_f -= A_f X_f (the first Gram-Schmidt pass of the
    recursion on FP32 blocks: A_f the earlier basis columns, ragged K = i b)
    against a float64 update of the same complex64 inputs; the inputs A, X
    are left as they were."""
    batch, rows, cols, N = case
    A, Ad = _cplx((batch, rows, cols), 1, torch.complex64)
    X, Xd = _cplx((batch, cols, N), 2, torch.complex64)
    C0, Cd = _cplx((batch, rows, N), 3, torch.complex64)
    A, X, C0 = (t.astype(np.complex64).astype(np.complex128) for t in (A, X, C0))
    api.diag_kgemm_sub(Ad, Xd, Cd)
    C = host(Cd)
    ref = C0 - A @ X
    scale = np.linalg.norm(C0.ravel()) + np.linalg.norm((A @ X).ravel())
    err = np.linalg.norm((C - ref).ravel()) / scale
    assert err <= 1e-6, f"rel err {err:.2e}"
    assert np.array_equal(host(Ad), A.astype(np.complex64)) and np.array_equal(host(Xd), X.astype(np.complex64))


@pytest.mark.parametrize("case", KG_CASES + [(33, 512, 520, 110, 1)])
@pytest.mark.parametrize("herm", [False, True])
def test_kgemm_presplit_bitwise_equals_bf16x3(case, herm):
    """BF16x3 with A given as (hi, lo) bf16 pairs and the thin operand split
    once per call gives the same products in the same order as the on-the-fly
    split: the results agree bit for bit (ragged tiles, K splits and the tail
    split of a 33-slice product included)."""
    batch, rows, cols, N, ns = case
    K = rows if herm else cols
    _, Ad = _cplx((batch, rows, cols), 11, torch.complex64)
    _, Xd = _cplx((batch, K, N), 12, torch.complex64)
    As = api.diag_split_bf16x3(Ad)
    c2 = api.diag_kgemm(Ad, Xd, herm=herm, mode="bf16x3", nsplit=ns)
    c3 = api.diag_kgemm(As, Xd, herm=herm, mode="bf16x3s", nsplit=ns)
    assert torch.equal(c2, c3)


def test_split_bf16x3_pairs():
    """The (hi, lo) pair form against its definition: hi = bf16(z), lo =
    bf16(z - hi) per part, round to nearest even (torch's bfloat16 cast)."""
    g = torch.Generator().manual_seed(13)
    Z = torch.complex(torch.randn(4097, generator=g), torch.randn(4097, generator=g))
    Z[0] = complex(0.0, -0.0)
    Z[1] = complex(3.0e38, -1.0e-30)
    P = api.diag_split_bf16x3(Z.cuda()).cpu()
    w = torch.view_as_real(P).contiguous().view(torch.int32).view(-1, 2)
    zr = torch.view_as_real(Z)
    hi = zr.to(torch.bfloat16)
    lo = (zr - hi.to(torch.float32)).to(torch.bfloat16)
    hb = hi.view(torch.int16).to(torch.int32) & 0xFFFF
    lb = lo.view(torch.int16).to(torch.int32) & 0xFFFF
    want_h = hb[:, 0] | (hb[:, 1] << 16)
    want_l = lb[:, 0] | (lb[:, 1] << 16)
    assert torch.equal(w[:, 0], want_h) and torch.equal(w[:, 1], want_l)


def test_kgemm_split_is_deterministic_and_matches_unsplit():
    A, Ad = _cplx((2, 200, 700), 3, torch.complex64)
    X, Xd = _cplx((2, 700, 40), 4, torch.complex64)
    c1 = host(api.diag_kgemm(Ad, Xd, nsplit=4))
    c2 = host(api.diag_kgemm(Ad, Xd, nsplit=4))
    c0 = host(api.diag_kgemm(Ad, Xd, nsplit=1))
    assert np.array_equal(c1, c2)
    assert np.linalg.norm((c1 - c0).ravel()) <= 1e-6 * np.linalg.norm(c0.ravel())


@pytest.mark.parametrize("herm", [False, True])
@pytest.mark.parametrize("mode", ["f32", "bf16x3"])
def test_kgemm_tail_split_vs_float64(herm, mode):
    """Enough tiles for two full rounds of the device's workgroup slots plus a
    remainder (1024 x 2048 slices, two thin chunks, 33 slices: 528 or 1056
    tiles on 256 CUs), which the kernel splits along K; checked against a
    float64 product and for run-to-run equality."""
    batch, rows, cols, N = 33, 1024, 2048, 224
    K = rows if herm else cols
    rng = np.random.default_rng(5)
    Ad = torch.complex(torch.tensor(rng.standard_normal((batch, rows, cols), dtype=np.float32)),
                       torch.tensor(rng.standard_normal((batch, rows, cols), dtype=np.float32))).cuda()
    Xd = torch.complex(torch.tensor(rng.standard_normal((batch, K, N), dtype=np.float32)),
                       torch.tensor(rng.standard_normal((batch, K, N), dtype=np.float32))).cuda()
    C1 = api.diag_kgemm(Ad, Xd, herm=herm, mode=mode)
    C2 = api.diag_kgemm(Ad, Xd, herm=herm, mode=mode)
    assert torch.equal(C1, C2)
    A64 = Ad.to(torch.complex128)
    opA = A64.transpose(1, 2).conj().contiguous() if herm else A64
    ref = torch.matmul(opA, Xd.to(torch.complex128).contiguous())
    err = (torch.linalg.norm((C1.to(torch.complex128) - ref).flatten()) / torch.linalg.norm(ref.flatten())).item()
    # FP32 accumulation over K = 1024 or 2048 complex terms: a few 1e-6
    tol = {"f32": 3e-6, "bf16x3": 3e-5}[mode]
    assert err <= tol, f"rel err {err:.2e}"
