"""Python binding of libtsvd_rbk.so (ctypes; argument marshalling only).

Every step of the computation runs in the library's HIP kernels; torch only
supplies device memory and the current stream.  The names mirror the C ABI in
``include/tsvd_rbk.h``.  Importing this module loads the library and raises
if it has not been built (``python -m paper_2504_04989_amd.build``).
"""
from __future__ import annotations

import ctypes
import os

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib", "libtsvd_rbk.so")

TSVD_OK, TSVD_EINVAL, TSVD_ENOMEM, TSVD_EHIP, TSVD_ENUMERIC = 0, 1, 2, 3, 4
PREC = {"f64": 0, "f32": 1, "bf16": 2, "bf16x3": 3}
OP = {"rbk": 0, "approx": 1, "proj": 2, "proj_bwd": 3, "power": 4, "power_approx": 5, "tqr": 6, "tpinv": 7, "complete2": 8,
      "complete1": 9, "literal": 10}
INFO_NAMES = ("chol_shifted", "chol_breakdown", "eig_noconv", "nonfinite")
INFO_COUNT = 8

EXPORTS = ("tsvd_version", "tsvd_last_error", "tsvd_workspace_bytes", "tsvd_rbk", "tsvd_rbk_approx",
           "tsvd_power", "tsvd_power_approx", "tsvd_tqr", "tsvd_tpinv", "tsvd_complete",
           "tsvd_rbk_literal",
           "tsvd_proj", "tsvd_proj_backward", "tsvd_read_info", "tsvd_diag_fft_r2c", "tsvd_diag_fft_c2r",
           "tsvd_diag_zgemm", "tsvd_diag_kgemm", "tsvd_diag_kgemm_ws_bytes", "tsvd_diag_heig",
           "tsvd_diag_heig_ws_bytes", "tsvd_diag_timing", "tsvd_diag_timing_read")


class TsvdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"tsvd error {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with `python -m paper_2504_04989_amd.build`")
    lib = ctypes.CDLL(_LIB_PATH)
    i64, vp, sz = ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t
    lib.tsvd_version.restype = ctypes.c_int
    lib.tsvd_last_error.restype = ctypes.c_char_p
    lib.tsvd_workspace_bytes.restype = sz
    lib.tsvd_workspace_bytes.argtypes = [i64, i64, i64, i64, i64, i64, ctypes.c_int, ctypes.c_int]
    lib.tsvd_rbk.restype = ctypes.c_int
    lib.tsvd_rbk.argtypes = [vp, vp, i64, i64, i64, i64, i64, i64, ctypes.c_int, vp, vp, vp, vp, sz, vp]
    lib.tsvd_rbk_approx.restype = ctypes.c_int
    lib.tsvd_rbk_approx.argtypes = [vp, vp, i64, i64, i64, i64, i64, i64, ctypes.c_int, vp, vp, vp, vp, vp, sz, vp]
    lib.tsvd_power.restype = ctypes.c_int
    lib.tsvd_power.argtypes = [vp, vp, i64, i64, i64, i64, i64, i64, ctypes.c_int, vp, vp, vp, vp, sz, vp]
    lib.tsvd_power_approx.restype = ctypes.c_int
    lib.tsvd_power_approx.argtypes = [vp, vp, i64, i64, i64, i64, i64, i64, ctypes.c_int, vp, vp, vp, vp, vp, sz,
                                      vp]
    lib.tsvd_tqr.restype = ctypes.c_int
    lib.tsvd_tqr.argtypes = [vp, i64, i64, i64, ctypes.c_int, vp, vp, vp, sz, vp]
    lib.tsvd_tpinv.restype = ctypes.c_int
    lib.tsvd_tpinv.argtypes = [vp, i64, i64, i64, ctypes.c_int, vp, vp, sz, vp]
    lib.tsvd_rbk_literal.restype = ctypes.c_int
    lib.tsvd_rbk_literal.argtypes = [vp, vp, i64, i64, i64, i64, i64, i64, ctypes.c_int, vp, vp, vp, vp, vp, sz, vp]
    lib.tsvd_complete.restype = ctypes.c_int
    lib.tsvd_complete.argtypes = [vp, vp, vp, i64, i64, i64, i64, i64, i64, i64, ctypes.c_int, ctypes.c_int, vp, vp,
                                  sz, vp]
    lib.tsvd_proj.restype = ctypes.c_int
    lib.tsvd_proj.argtypes = [vp, vp, i64, i64, i64, i64, i64, ctypes.c_int, vp, vp, sz, vp]
    lib.tsvd_proj_backward.restype = ctypes.c_int
    lib.tsvd_proj_backward.argtypes = [vp, vp, vp, i64, i64, i64, i64, i64, ctypes.c_int, vp, vp, sz, vp]
    lib.tsvd_read_info.restype = ctypes.c_int
    lib.tsvd_read_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), vp]
    lib.tsvd_diag_fft_r2c.restype = ctypes.c_int
    lib.tsvd_diag_fft_r2c.argtypes = [vp, vp, i64, i64, ctypes.c_int, vp]
    lib.tsvd_diag_fft_c2r.restype = ctypes.c_int
    lib.tsvd_diag_fft_c2r.argtypes = [vp, vp, i64, i64, ctypes.c_int, vp]
    lib.tsvd_diag_timing.restype = ctypes.c_int
    lib.tsvd_diag_timing.argtypes = [ctypes.c_int]
    lib.tsvd_diag_timing_read.restype = ctypes.c_int
    lib.tsvd_diag_timing_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                          ctypes.c_int]
    lib.tsvd_diag_zgemm.restype = ctypes.c_int
    lib.tsvd_diag_zgemm.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int, vp, i64, i64, i64, i64, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_int, vp]
    lib.tsvd_diag_kgemm_ws_bytes.restype = sz
    lib.tsvd_diag_kgemm_ws_bytes.argtypes = [ctypes.c_int, i64, i64, i64, i64, ctypes.c_int, ctypes.c_int]
    lib.tsvd_diag_kgemm.restype = ctypes.c_int
    lib.tsvd_diag_kgemm.argtypes = [vp, ctypes.c_int, vp, vp, i64, i64, i64, i64, ctypes.c_int, ctypes.c_int, vp, sz,
                                    vp]
    lib.tsvd_diag_heig_ws_bytes.restype = sz
    lib.tsvd_diag_heig_ws_bytes.argtypes = [i64, i64, i64]
    lib.tsvd_diag_heig.restype = ctypes.c_int
    lib.tsvd_diag_heig.argtypes = [vp, i64, i64, i64, vp, vp, vp, sz, vp]
    return lib


lib = _load()


def _check(code: int):
    if code != TSVD_OK:
        raise TsvdError(code, lib.tsvd_last_error().decode())


def _prec_of(t: torch.Tensor, prec):
    if prec is None:
        return "f64" if t.dtype == torch.float64 else "f32"
    return prec


def _dtype_of(prec: str):
    return torch.float64 if prec == "f64" else torch.float32


def _stream(dev):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _check_in(t: torch.Tensor, dtype, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def workspace_bytes(n1, n2, n3, k, b, q, prec="f32", op="rbk") -> int:
    return int(lib.tsvd_workspace_bytes(n1, n2, n3, k, b, q, PREC[prec], OP[op]))


def workspace(n1, n2, n3, k, b, q, prec, op, device) -> torch.Tensor:
    nb = workspace_bytes(n1, n2, n3, k, b, q, prec, op)
    if nb == 0:
        raise TsvdError(TSVD_EINVAL, lib.tsvd_last_error().decode())
    return torch.empty(nb, dtype=torch.uint8, device=device)


def read_info(ws: torch.Tensor) -> dict:
    buf = (ctypes.c_int32 * INFO_COUNT)()
    _check(lib.tsvd_read_info(_ptr(ws), buf, _stream(ws.device)))
    return {name: int(buf[i]) for i, name in enumerate(INFO_NAMES)}


def tsvd_rbk(A: torch.Tensor, Omega: torch.Tensor, k: int, b: int, q: int, prec=None, ws=None, out=None):
    """Alg. 2: returns (U, S, V) with U (n1,k,n3), S (k,n3), V (n2,k,n3)."""
    prec = _prec_of(A, prec)
    dt = _dtype_of(prec)
    _check_in(A, dt, "A")
    _check_in(Omega, dt, "Omega")
    n1, n2, n3 = A.shape
    if tuple(Omega.shape) != (n2, b, n3):
        raise ValueError("Omega must have shape (n2, b, n3)")
    dev = A.device
    if ws is None:
        ws = workspace(n1, n2, n3, k, b, q, prec, "rbk", dev)
    if out is None:
        out = (torch.empty((n1, k, n3), dtype=dt, device=dev), torch.empty((k, n3), dtype=dt, device=dev),
               torch.empty((n2, k, n3), dtype=dt, device=dev))
    U, S, V = out
    _check(lib.tsvd_rbk(_ptr(A), _ptr(Omega), n1, n2, n3, k, b, q, PREC[prec], _ptr(U), _ptr(S), _ptr(V),
                        _ptr(ws), ws.numel(), _stream(dev)))
    return U, S, V


def tsvd_rbk_approx(A, Omega, k, b, q, prec=None, ws=None):
    """Alg. 2 plus X_hat = U * S * V^T: returns (U, S, V, X_hat)."""
    prec = _prec_of(A, prec)
    dt = _dtype_of(prec)
    _check_in(A, dt, "A")
    _check_in(Omega, dt, "Omega")
    n1, n2, n3 = A.shape
    if tuple(Omega.shape) != (n2, b, n3):
        raise ValueError("Omega must have shape (n2, b, n3)")
    dev = A.device
    if ws is None:
        ws = workspace(n1, n2, n3, k, b, q, prec, "approx", dev)
    U = torch.empty((n1, k, n3), dtype=dt, device=dev)
    S = torch.empty((k, n3), dtype=dt, device=dev)
    V = torch.empty((n2, k, n3), dtype=dt, device=dev)
    X = torch.empty((n1, n2, n3), dtype=dt, device=dev)
    _check(lib.tsvd_rbk_approx(_ptr(A), _ptr(Omega), n1, n2, n3, k, b, q, PREC[prec], _ptr(U), _ptr(S), _ptr(V),
                               _ptr(X), _ptr(ws), ws.numel(), _stream(dev)))
    return U, S, V, X


def tsvd_rbk_literal(A, Omega, k, b, q, prec=None, ws=None, approx=True):
    """Alg. 2 with the literal Krylov powers (no orthonormalisation between
    steps): returns (U, S, V, X_hat) (X_hat None when approx is False)."""
    prec = _prec_of(A, prec)
    dt = _dtype_of(prec)
    _check_in(A, dt, "A")
    _check_in(Omega, dt, "Omega")
    n1, n2, n3 = A.shape
    if tuple(Omega.shape) != (n2, b, n3):
        raise ValueError("Omega must have shape (n2, b, n3)")
    dev = A.device
    if ws is None:
        ws = workspace(n1, n2, n3, k, b, q, prec, "literal", dev)
    U = torch.empty((n1, k, n3), dtype=dt, device=dev)
    S = torch.empty((k, n3), dtype=dt, device=dev)
    V = torch.empty((n2, k, n3), dtype=dt, device=dev)
    X = torch.empty((n1, n2, n3), dtype=dt, device=dev) if approx else None
    _check(lib.tsvd_rbk_literal(_ptr(A), _ptr(Omega), n1, n2, n3, k, b, q, PREC[prec], _ptr(U), _ptr(S), _ptr(V),
                                _ptr(X), _ptr(ws), ws.numel(), _stream(dev)))
    return U, S, V, X


def tsvd_power(A: torch.Tensor, Omega: torch.Tensor, k: int, b: int, q: int, prec=None, ws=None):
    """Alg. 1 (q power iterations): returns (U, S, V) like tsvd_rbk."""
    prec = _prec_of(A, prec)
    dt = _dtype_of(prec)
    _check_in(A, dt, "A")
    _check_in(Omega, dt, "Omega")
    n1, n2, n3 = A.shape
    if tuple(Omega.shape) != (n2, b, n3):
        raise ValueError("Omega must have shape (n2, b, n3)")
    dev = A.device
    if ws is None:
        ws = workspace(n1, n2, n3, k, b, q, prec, "power", dev)
    U = torch.empty((n1, k, n3), dtype=dt, device=dev)
    S = torch.empty((k, n3), dtype=dt, device=dev)
    V = torch.empty((n2, k, n3), dtype=dt, device=dev)
    _check(lib.tsvd_power(_ptr(A), _ptr(Omega), n1, n2, n3, k, b, q, PREC[prec], _ptr(U), _ptr(S), _ptr(V),
                          _ptr(ws), ws.numel(), _stream(dev)))
    return U, S, V


def tsvd_power_approx(A, Omega, k, b, q, prec=None, ws=None):
    """Alg. 1 plus X_hat = U * S * V^T: returns (U, S, V, X_hat)."""
    prec = _prec_of(A, prec)
    dt = _dtype_of(prec)
    _check_in(A, dt, "A")
    _check_in(Omega, dt, "Omega")
    n1, n2, n3 = A.shape
    if tuple(Omega.shape) != (n2, b, n3):
        raise ValueError("Omega must have shape (n2, b, n3)")
    dev = A.device
    if ws is None:
        ws = workspace(n1, n2, n3, k, b, q, prec, "power_approx", dev)
    U = torch.empty((n1, k, n3), dtype=dt, device=dev)
    S = torch.empty((k, n3), dtype=dt, device=dev)
    V = torch.empty((n2, k, n3), dtype=dt, device=dev)
    X = torch.empty((n1, n2, n3), dtype=dt, device=dev)
    _check(lib.tsvd_power_approx(_ptr(A), _ptr(Omega), n1, n2, n3, k, b, q, PREC[prec], _ptr(U), _ptr(S),
                                 _ptr(V), _ptr(X), _ptr(ws), ws.numel(), _stream(dev)))
    return U, S, V, X


def tsvd_tqr(A: torch.Tensor, prec=None, ws=None):
    """Alg. TQR: returns (Q, R), Q (n1, r, n3), R (r, n2, n3), r = min(n1, n2)."""
    prec = _prec_of(A, prec)
    dt = _dtype_of(prec)
    _check_in(A, dt, "A")
    n1, n2, n3 = A.shape
    r = min(n1, n2)
    if ws is None:
        ws = workspace(n1, n2, n3, 0, 0, 0, prec, "tqr", A.device)
    Q = torch.empty((n1, r, n3), dtype=dt, device=A.device)
    R = torch.empty((r, n2, n3), dtype=dt, device=A.device)
    _check(lib.tsvd_tqr(_ptr(A), n1, n2, n3, PREC[prec], _ptr(Q), _ptr(R), _ptr(ws), ws.numel(),
                        _stream(A.device)))
    return Q, R


def tsvd_tpinv(A: torch.Tensor, prec=None, ws=None):
    """Alg. mp for slices of full column rank: returns A^+ (n2, n1, n3)."""
    prec = _prec_of(A, prec)
    dt = _dtype_of(prec)
    _check_in(A, dt, "A")
    n1, n2, n3 = A.shape
    if ws is None:
        ws = workspace(n1, n2, n3, 0, 0, 0, prec, "tpinv", A.device)
    X = torch.empty((n2, n1, n3), dtype=dt, device=A.device)
    _check(lib.tsvd_tpinv(_ptr(A), n1, n2, n3, PREC[prec], _ptr(X), _ptr(ws), ws.numel(), _stream(A.device)))
    return X


def tsvd_complete(M: torch.Tensor, mask: torch.Tensor, Omega: torch.Tensor, k: int, b: int, q: int, iters: int,
                  alg: int = 2, prec=None, ws=None):
    """Completion of Example 3: returns C^(iters) (n1, n2, n3).  mask: bool or
    uint8 tensor of M's shape (True / non-zero = observed)."""
    prec = _prec_of(M, prec)
    dt = _dtype_of(prec)
    _check_in(M, dt, "M")
    _check_in(Omega, dt, "Omega")
    n1, n2, n3 = M.shape
    if tuple(mask.shape) != tuple(M.shape) or mask.dtype not in (torch.bool, torch.uint8):
        raise ValueError("mask must be a bool / uint8 tensor of M's shape")
    if not mask.is_cuda or not mask.is_contiguous():
        raise ValueError("mask must be a contiguous device tensor")
    if tuple(Omega.shape) != (n2, b, n3):
        raise ValueError("Omega must have shape (n2, b, n3)")
    if ws is None:
        ws = workspace(n1, n2, n3, k, b, q, prec, "complete2" if alg == 2 else "complete1", M.device)
    C = torch.empty_like(M)
    _check(lib.tsvd_complete(_ptr(M), _ptr(mask), _ptr(Omega), n1, n2, n3, k, b, q, iters, alg, PREC[prec], _ptr(C),
                             _ptr(ws), ws.numel(), _stream(M.device)))
    return C


def tsvd_proj(A, Omega, b, q, prec=None, ws=None):
    """P(A) = Q * Q^T * A with Q the T-QR basis of the block Krylov tensor."""
    prec = _prec_of(A, prec)
    dt = _dtype_of(prec)
    _check_in(A, dt, "A")
    _check_in(Omega, dt, "Omega")
    n1, n2, n3 = A.shape
    dev = A.device
    if ws is None:
        ws = workspace(n1, n2, n3, 1, b, q, prec, "proj", dev)
    P = torch.empty_like(A)
    _check(lib.tsvd_proj(_ptr(A), _ptr(Omega), n1, n2, n3, b, q, PREC[prec], _ptr(P), _ptr(ws), ws.numel(),
                         _stream(dev)))
    return P


def tsvd_proj_backward(A, Omega, G, b, q, prec=None, ws=None):
    """dL/dA for L(P(A)) given G = dL/dP."""
    prec = _prec_of(A, prec)
    dt = _dtype_of(prec)
    for t, nm in ((A, "A"), (Omega, "Omega"), (G, "G")):
        _check_in(t, dt, nm)
    n1, n2, n3 = A.shape
    dev = A.device
    if ws is None:
        ws = workspace(n1, n2, n3, 1, b, q, prec, "proj_bwd", dev)
    dA = torch.empty_like(A)
    _check(lib.tsvd_proj_backward(_ptr(A), _ptr(Omega), _ptr(G), n1, n2, n3, b, q, PREC[prec], _ptr(dA), _ptr(ws),
                                  ws.numel(), _stream(dev)))
    return dA


class TProject(torch.autograd.Function):
    """A -> Q * Q^T * A with the hand-written adjoint; the Krylov blocks are
    recomputed in backward from (A, Omega), not stored."""

    @staticmethod
    def forward(ctx, A, Omega, b, q, prec=None):
        ctx.save_for_backward(A, Omega)
        ctx.b, ctx.q, ctx.prec = b, q, prec
        return tsvd_proj(A.detach().contiguous(), Omega.contiguous(), b, q, prec)

    @staticmethod
    def backward(ctx, G):
        A, Omega = ctx.saved_tensors
        dA = tsvd_proj_backward(A.detach().contiguous(), Omega.contiguous(), G.contiguous(), ctx.b, ctx.q, ctx.prec)
        return dA, None, None, None, None


# ---- kernel-level entry points (include/tsvd_rbk_diag.h) --------------------

def _dcode(t: torch.Tensor) -> int:
    return 0 if t.dtype in (torch.float64, torch.complex128) else 1


def diag_fft_r2c(X: torch.Tensor) -> torch.Tensor:
    """Half spectrum (F, ntubes) complex of the real tubes X (ntubes, n3)."""
    ntubes, n3 = X.shape
    cdt = torch.complex128 if X.dtype == torch.float64 else torch.complex64
    Xb = torch.empty((n3 // 2 + 1, ntubes), dtype=cdt, device=X.device)
    _check(lib.tsvd_diag_fft_r2c(_ptr(X), _ptr(Xb), ntubes, n3, _dcode(X), _stream(X.device)))
    return Xb


def diag_fft_c2r(Xb: torch.Tensor, n3: int) -> torch.Tensor:
    F, ntubes = Xb.shape
    assert F == n3 // 2 + 1
    rdt = torch.float64 if Xb.dtype == torch.complex128 else torch.float32
    X = torch.empty((ntubes, n3), dtype=rdt, device=Xb.device)
    _check(lib.tsvd_diag_fft_c2r(_ptr(Xb), _ptr(X), ntubes, n3, _dcode(Xb), _stream(Xb.device)))
    return X


def diag_zgemm(A, B, a_conj=False, b_conj=False, C=None, alpha=1.0, beta=0.0):
    """Batched complex product on the library's MFMA kernel (see tsvd_diag_zgemm)."""
    batch = A.shape[0]
    M = A.shape[2] if a_conj else A.shape[1]
    K = A.shape[1] if a_conj else A.shape[2]
    N = B.shape[1] if b_conj else B.shape[2]
    if C is None:
        C = torch.zeros((batch, M, N), dtype=A.dtype, device=A.device)
    _check(lib.tsvd_diag_zgemm(_ptr(A), int(a_conj), _ptr(B), int(b_conj), _ptr(C), M, N, K, batch, alpha, beta,
                               _dcode(A), _stream(A.device)))
    return C


KGEMM_MODE = {"f32": 0, "bf16": 1, "bf16x3": 2}


def diag_kgemm(A, X, herm=False, mode="f32", nsplit=1):
    """The Krylov-product kernel alone (see tsvd_diag_kgemm): op(A_f) X_f for
    complex64 tensors A (batch, rows, cols) and X (batch, K, N)."""
    batch, rows, cols = A.shape
    M = cols if herm else rows
    N = X.shape[2]
    C = torch.empty((batch, M, N), dtype=torch.complex64, device=A.device)
    nb = int(lib.tsvd_diag_kgemm_ws_bytes(int(herm), rows, cols, N, batch, KGEMM_MODE[mode], nsplit))
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=A.device)
    _check(lib.tsvd_diag_kgemm(_ptr(A), int(herm), _ptr(X), _ptr(C), rows, cols, N, batch, KGEMM_MODE[mode], nsplit,
                               _ptr(ws), ws.numel(), _stream(A.device)))
    return C


def diag_heig(G, k):
    """The small Hermitian eigensolver alone (see tsvd_diag_heig): the k
    largest eigenpairs of each complex128 matrix G (batch, m, m).  Returns
    (lambda (batch, k) descending, W (batch, m, k), info dict)."""
    batch, m, _ = G.shape
    lam = torch.empty((batch, k), dtype=torch.float64, device=G.device)
    W = torch.empty((batch, m, k), dtype=torch.complex128, device=G.device)
    nb = int(lib.tsvd_diag_heig_ws_bytes(m, k, batch))
    if nb == 0:
        raise TsvdError(TSVD_EINVAL, "bad eigensolver shape")
    ws = torch.empty(nb, dtype=torch.uint8, device=G.device)
    _check(lib.tsvd_diag_heig(_ptr(G), m, k, batch, _ptr(lam), _ptr(W), _ptr(ws), ws.numel(), _stream(G.device)))
    return lam, W, read_info(ws)


KERNEL_CLASSES = ("fft_A", "fft_omega", "gemm_krylov", "gemm_orth", "chol", "heig_tri", "gemm_lift", "fft_inv", "misc",
                  "heig_bisect", "heig_invit", "heig_backxf")


def diag_timing(enable: bool):
    _check(lib.tsvd_diag_timing(int(enable)))


def diag_timing_read() -> dict:
    n = len(KERNEL_CLASSES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    _check(lib.tsvd_diag_timing_read(ms, cnt, n))
    return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(KERNEL_CLASSES)}
