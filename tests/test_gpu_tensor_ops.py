"""T-QR (Alg. TQR) and T-pseudoinverse (Alg. mp) on the HIP path (GPU).

Parity with the FP64 oracle (Q, R and A^+ element by element), plus the
spatial-domain identities X = Q * R, Q^T * Q = I and the Penrose conditions on
the GPU's own outputs.  T-QR tolerances: 1e-10 (FP64), 1e-5 (FP32); in FP32
the forward error of Q and R grows with the slices' condition number, so the
FP32 element-wise cases use tall Gaussian tensors (well conditioned).

The pseudoinverse goes through the FP64 Gram of each slice, whose eigenvalues
carry an absolute error of about (n1 + n2) 2^-53 lambda_1; a kept singular
value s_r then has a relative error of about (n1 + n2) 2^-53 kappa^2 with
kappa = s_1 / s_r, and FP32 data adds its own rounding, about 2^-24 kappa^2
relative on A^+.  The tolerance is ten times that model, floored at 1e-10
(FP64) and 1e-5 (FP32), with kappa taken over the kept values of every slice
from the oracle's SVDs; both sides use the same cut-off rtol.
"""
import numpy as np
import pytest
import torch

from oracle import tsvd_oracle as O
from paper_2504_04989_amd import inputs
from tests.gpu_util import load_api, dev, host, rel_f

pytestmark = pytest.mark.gpu
api = load_api()

TOL = {"f64": 1e-10, "f32": 1e-5}


def _cast(x, prec):
    return x if prec == "f64" else x.astype(np.float32).astype(np.float64)


def _dt(prec):
    return torch.float64 if prec == "f64" else torch.float32


CASES = [
    ((90, 60, 10), "f64"), ((90, 60, 10), "f32"),
    ((200, 40, 7), "f32"),              # odd n3
    ((64, 64, 9), "f64"),               # square
    ((40, 70, 6), "f64"),               # wide: r = n1, R is 40 x 70
    ((50, 30, 1), "f64"), ((50, 30, 1), "f32"),   # n3 = 1: the matrix QR
    ((60, 1, 5), "f64"),                # r = 1
    ((300, 150, 4), "f64"),             # r > 128: unblocked Cholesky
    ((1200, 200, 2), "f32"),            # r > 128, FP32
    ((333, 120, 3), "f32"),             # one 120-column panel over a ragged n1
]


@pytest.mark.parametrize("shape,prec", CASES)
def test_tqr_vs_oracle(shape, prec):
    print(f"[tqr] shape={shape} prec={prec}", flush=True)
    X = _cast(inputs.random_tensor(shape, 51), prec)
    ws = api.workspace(*shape, 0, 0, 0, prec, "tqr", "cuda")
    Q, R = api.tsvd_tqr(dev(X, _dt(prec)), prec, ws=ws)
    info = api.read_info(ws)
    Q, R = host(Q).astype(np.float64), host(R).astype(np.float64)
    Qo, Ro = O.tqr(X)
    tol = TOL[prec]
    assert info["chol_breakdown"] == 0 and info["nonfinite"] == 0
    assert rel_f(Q, Qo) <= tol, f"Q rel err {rel_f(Q, Qo):.3e}"
    assert rel_f(R, Ro) <= tol, f"R rel err {rel_f(R, Ro):.3e}"
    r = min(shape[:2])
    assert rel_f(O.tprod(Q, R), X) <= tol
    assert np.abs(O.tprod(O.ttranspose(Q), Q) - O.identity_tensor(r, shape[2])).max() <= tol


def _kappa(X, rtol):
    """Largest s_1 / s_r over the Fourier slices, s_r the smallest singular
    value above rtol * s_1 (the oracle's SVDs)."""
    n3 = X.shape[2]
    Xb = O.dft_mode3(X, range(O.n_half(n3)))
    kap = 1.0
    for f in range(Xb.shape[2]):
        sv = np.linalg.svd(Xb[:, :, f], compute_uv=False)
        if sv[0] == 0:
            continue
        kept = sv[sv > rtol * sv[0]]
        kap = max(kap, kept[0] / kept[-1])
    return kap


def _pinv_tol(shape, prec, kap):
    n1, n2 = shape[:2]
    if prec == "f64":
        return max(1e-10, 10 * (n1 + n2) * 2.0 ** -53 * kap ** 2)
    return max(1e-5, 10 * 2.0 ** -24 * kap ** 2)


def _slice_rank_mix(n1, n2, n3, seed):
    # X(:, :, t) = P + c_t Q with P of rank 1 and Q of rank 2: the DC slice
    # has rank 3 (when sum c_t != 0), every other slice rank 2
    g = np.random.default_rng(seed)
    P = np.outer(g.standard_normal(n1), g.standard_normal(n2))
    Q = g.standard_normal((n1, 2)) @ g.standard_normal((2, n2))
    c = g.standard_normal(n3)
    return P[:, :, None] + Q[:, :, None] * c[None, None, :]


PINV_CASES = [
    ("gauss", (90, 60, 10), "f64"), ("gauss", (90, 60, 10), "f32"),
    ("gauss", (200, 40, 7), "f32"),             # odd n3
    ("gauss", (64, 48, 9), "f64"),
    ("gauss", (40, 70, 6), "f64"), ("gauss", (40, 70, 6), "f32"),   # wide: Gram A A^H
    ("gauss", (50, 30, 1), "f64"), ("gauss", (50, 30, 1), "f32"),   # n3 = 1: the matrix pinv
    ("gauss", (60, 1, 5), "f64"), ("gauss", (1, 60, 5), "f64"),     # r = 1, tall and wide
    ("gauss", (300, 150, 4), "f64"),            # r > 128
    ("gauss", (1200, 200, 2), "f32"),
    ("gauss", (4096, 256, 8), "f32"),           # the timed shape's slices (n3 = 8)
    ("lowrank", (50, 40, 6), "f64"), ("lowrank", (50, 40, 6), "f32"),   # tubal rank 3
    ("lowrank", (30, 45, 5), "f64"),            # wide and rank deficient
    ("mix", (36, 28, 6), "f64"), ("mix", (36, 28, 6), "f32"),     # ranks differ across slices
    ("square", (48, 48, 4), "f64"),
]


def _pinv_input(kind, shape, seed):
    n1, n2, n3 = shape
    if kind == "lowrank":
        return inputs.exact_lowrank_tensor(n1, n2, n3, 3, seed=seed)
    if kind == "mix":
        return _slice_rank_mix(n1, n2, n3, seed)
    if kind == "square":
        # square slices kept away from singular: a scaled identity plus noise
        return inputs.random_tensor(shape, seed) * 0.1 + np.eye(n1)[:, :, None] * (np.arange(n3) == 0)[None, None, :]
    return inputs.random_tensor(shape, seed)


@pytest.mark.parametrize("kind,shape,prec", PINV_CASES)
def test_tpinv_vs_oracle_and_penrose(kind, shape, prec):
    print(f"[tpinv] kind={kind} shape={shape} prec={prec}", flush=True)
    X = _cast(_pinv_input(kind, shape, 52), prec)
    rtol = api.tpinv_default_rtol(shape[0], shape[1], prec)
    ws = api.workspace(*shape, 0, 0, 0, prec, "tpinv", "cuda")
    P = host(api.tsvd_tpinv(dev(X, _dt(prec)), 0.0, prec, ws=ws)).astype(np.float64)
    info = api.read_info(ws)
    assert info["eig_noconv"] == 0 and info["nonfinite"] == 0
    Po = O.tpinv(X, rtol=rtol)
    tol = _pinv_tol(shape, prec, _kappa(X, rtol))
    assert rel_f(P, Po) <= tol, f"A^+ rel err {rel_f(P, Po):.3e} (tol {tol:.1e})"
    if shape[0] * shape[1] > 400_000:
        return      # the Penrose products of the largest case take the oracle minutes
    tp, tt = O.tprod, O.ttranspose
    assert rel_f(tp(tp(X, P), X), X) <= tol
    assert rel_f(tp(tp(P, X), P), P) <= tol
    XP, PX = tp(X, P), tp(P, X)
    assert np.abs(tt(XP) - XP).max() <= tol * max(1.0, np.abs(XP).max())
    assert np.abs(tt(PX) - PX).max() <= tol * max(1.0, np.abs(PX).max())
    if kind == "gauss" and shape[0] >= shape[1]:
        assert np.abs(PX - O.identity_tensor(shape[1], shape[2])).max() <= 10 * tol


def test_tpinv_explicit_cutoff():
    # n3 = 1, singular values 4, 2, 1e-3: rtol = 1e-2 drops the third one on
    # both sides, rtol = 1e-4 keeps it
    g = np.random.default_rng(55)
    U, _ = np.linalg.qr(g.standard_normal((40, 3)))
    V, _ = np.linalg.qr(g.standard_normal((24, 3)))
    X = ((U * np.array([4.0, 2.0, 1e-3])) @ V.T)[:, :, None]
    for rtol in (1e-2, 1e-4):
        P = host(api.tsvd_tpinv(dev(X, torch.float64), rtol, "f64")).astype(np.float64)
        Po = O.tpinv(X, rtol=rtol)
        assert rel_f(P, Po) <= 1e-9, (rtol, rel_f(P, Po))


def test_tpinv_zero_tensor_and_rejections():
    X = np.zeros((20, 12, 4))
    P = host(api.tsvd_tpinv(dev(X, torch.float64), 0.0, "f64")).astype(np.float64)
    assert np.abs(P).max() == 0.0
    with pytest.raises(api.TsvdError):
        api.tsvd_tpinv(dev(X, torch.float64), 1e-12, "f64")      # below the Gram's resolution


def test_tqr_wide_fp32_backward():
    # wide FP32 tensor: the backward identities at the FP32 bar
    shape = (48, 80, 6)
    X = _cast(inputs.random_tensor(shape, 53), "f32")
    Q, R = api.tsvd_tqr(dev(X, torch.float32), "f32")
    Q, R = host(Q).astype(np.float64), host(R).astype(np.float64)
    assert rel_f(O.tprod(Q, R), X) <= 1e-5
    assert np.abs(O.tprod(O.ttranspose(Q), Q) - O.identity_tensor(48, 6)).max() <= 1e-5
