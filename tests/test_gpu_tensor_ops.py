"""T-QR (Alg. TQR) and T-pseudoinverse (Alg. mp) on the HIP path (GPU).

Parity with the FP64 oracle (Q, R and A^+ element by element), plus the
spatial-domain identities X = Q * R, Q^T * Q = I and the Penrose conditions on
the GPU's own outputs.  Tolerances: 1e-10 (FP64), 1e-5 (FP32).  In FP32 the
forward error of Q, R and A^+ grows with the slices' condition number, so the
FP32 element-wise cases use tall Gaussian tensors (well conditioned); the
backward identities hold for every shape.
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


@pytest.mark.parametrize("shape,prec", [c for c in CASES if c[0][0] >= c[0][1]])
def test_tpinv_vs_oracle_and_penrose(shape, prec):
    print(f"[tpinv] shape={shape} prec={prec}", flush=True)
    X = _cast(inputs.random_tensor(shape, 52), prec)
    ws = api.workspace(*shape, 0, 0, 0, prec, "tpinv", "cuda")
    P = host(api.tsvd_tpinv(dev(X, _dt(prec)), prec, ws=ws)).astype(np.float64)
    info = api.read_info(ws)
    assert info["chol_breakdown"] == 0 and info["nonfinite"] == 0
    Po = O.tpinv(X)
    tol = TOL[prec]
    assert rel_f(P, Po) <= tol, f"A^+ rel err {rel_f(P, Po):.3e}"
    tp, tt = O.tprod, O.ttranspose
    assert rel_f(tp(tp(X, P), X), X) <= tol
    assert rel_f(tp(tp(P, X), P), P) <= tol
    XP, PX = tp(X, P), tp(P, X)
    assert np.abs(tt(XP) - XP).max() <= tol * max(1.0, np.abs(XP).max())
    assert np.abs(PX - O.identity_tensor(shape[1], shape[2])).max() <= 10 * tol


def test_tqr_wide_fp32_backward():
    # wide FP32 tensor: the backward identities at the FP32 bar
    shape = (48, 80, 6)
    X = _cast(inputs.random_tensor(shape, 53), "f32")
    Q, R = api.tsvd_tqr(dev(X, torch.float32), "f32")
    Q, R = host(Q).astype(np.float64), host(R).astype(np.float64)
    assert rel_f(O.tprod(Q, R), X) <= 1e-5
    assert np.abs(O.tprod(O.ttranspose(Q), Q) - O.identity_tensor(48, 6)).max() <= 1e-5
