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
      "complete1": 9, "literal": 10, "ritz": 11, "approx_bwd": 12}
INFO_NAMES = ("chol_shifted", "chol_breakdown", "eig_noconv", "nonfinite", "truncation_tie")
INFO_COUNT = 8

EXPORTS = ("tsvd_version", "tsvd_last_error", "tsvd_workspace_bytes", "tsvd_omega",
           "tsvd_rbk", "tsvd_rbk_omega", "tsvd_rbk_noalloc", "tsvd_rbk_approx", "tsvd_rbk_approx_omega",
           "tsvd_power", "tsvd_power_omega", "tsvd_power_approx", "tsvd_power_approx_omega",
           "tsvd_rbk_literal", "tsvd_rbk_literal_omega", "tsvd_rbk_ritz", "tsvd_rbk_ritz_omega",
           "tsvd_rbk_approx_backward", "tsvd_rbk_approx_backward_omega", "tsvd_complete", "tsvd_complete_omega",
           "tsvd_tqr", "tsvd_tpinv", "tsvd_tpinv_default_rtol", "tsvd_proj", "tsvd_proj_omega", "tsvd_proj_backward",
           "tsvd_proj_backward_omega", "tsvd_read_info", "tsvd_diag_fft_r2c", "tsvd_diag_fft_c2r",
           "tsvd_diag_zgemm", "tsvd_diag_kgemm", "tsvd_diag_kgemm_ws_bytes", "tsvd_diag_kgemm_sub", "tsvd_diag_split_bf16x3", "tsvd_diag_heig",
           "tsvd_diag_heig_ws_bytes", "tsvd_diag_timing", "tsvd_diag_timing_read", "tsvd_diag_omega")


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
    u64, ci = ctypes.c_uint64, ctypes.c_int
    lib.tsvd_omega.restype = ci
    lib.tsvd_omega.argtypes = [i64, i64, i64, u64, vp]
    # (A, n1, n2, n3, k, b, q, seed, prec, U, S, V[, Xhat], ws, ws_bytes, stream) and the _omega twins
    # (A, Omega, n1, n2, n3, k, b, q, prec, U, S, V[, Xhat], ws, ws_bytes, stream)
    for name, nout in (("tsvd_rbk", 3), ("tsvd_rbk_approx", 4), ("tsvd_power", 3), ("tsvd_power_approx", 4),
                       ("tsvd_rbk_literal", 4)):
        f = getattr(lib, name)
        f.restype = ci
        f.argtypes = [vp, i64, i64, i64, i64, i64, i64, u64, ci] + [vp] * nout + [vp, sz, vp]
        f = getattr(lib, name + "_omega")
        f.restype = ci
        f.argtypes = [vp, vp, i64, i64, i64, i64, i64, i64, ci] + [vp] * nout + [vp, sz, vp]
    lib.tsvd_rbk_ritz.restype = ci
    lib.tsvd_rbk_ritz.argtypes = [vp, i64, i64, i64, i64, i64, i64, u64, ci] + [vp] * 4 + [vp, sz, vp]
    lib.tsvd_rbk_ritz_omega.restype = ci
    lib.tsvd_rbk_ritz_omega.argtypes = [vp, vp, i64, i64, i64, i64, i64, i64, ci] + [vp] * 4 + [vp, sz, vp]
    lib.tsvd_rbk_approx_backward.restype = ci
    lib.tsvd_rbk_approx_backward.argtypes = [vp, vp, i64, i64, i64, i64, i64, i64, u64, ci, vp, vp, sz, vp]
    lib.tsvd_rbk_approx_backward_omega.restype = ci
    lib.tsvd_rbk_approx_backward_omega.argtypes = [vp, vp, vp, i64, i64, i64, i64, i64, i64, ci, vp, vp, sz, vp]
    lib.tsvd_rbk_noalloc.restype = ci
    lib.tsvd_rbk_noalloc.argtypes = [vp, i64, i64, i64, i64, i64, i64, u64, ci, vp, vp, vp, vp]
    lib.tsvd_tqr.restype = ci
    lib.tsvd_tqr.argtypes = [vp, i64, i64, i64, ci, vp, vp, vp, sz, vp]
    lib.tsvd_tpinv.restype = ci
    lib.tsvd_tpinv.argtypes = [vp, i64, i64, i64, ctypes.c_double, ci, vp, vp, sz, vp]
    lib.tsvd_tpinv_default_rtol.restype = ctypes.c_double
    lib.tsvd_tpinv_default_rtol.argtypes = [i64, i64, ci]
    lib.tsvd_complete.restype = ci
    lib.tsvd_complete.argtypes = [vp, vp, i64, i64, i64, i64, i64, i64, u64, i64, ci, ci, vp, vp, sz, vp]
    lib.tsvd_complete_omega.restype = ci
    lib.tsvd_complete_omega.argtypes = [vp, vp, vp, i64, i64, i64, i64, i64, i64, i64, ci, ci, vp, vp, sz, vp]
    lib.tsvd_proj.restype = ci
    lib.tsvd_proj.argtypes = [vp, i64, i64, i64, i64, i64, u64, ci, vp, vp, sz, vp]
    lib.tsvd_proj_omega.restype = ci
    lib.tsvd_proj_omega.argtypes = [vp, vp, i64, i64, i64, i64, i64, ci, vp, vp, sz, vp]
    lib.tsvd_proj_backward.restype = ci
    lib.tsvd_proj_backward.argtypes = [vp, vp, i64, i64, i64, i64, i64, u64, ci, vp, vp, sz, vp]
    lib.tsvd_proj_backward_omega.restype = ci
    lib.tsvd_proj_backward_omega.argtypes = [vp, vp, vp, i64, i64, i64, i64, i64, ci, vp, vp, sz, vp]
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
    lib.tsvd_diag_split_bf16x3.restype = ctypes.c_int
    lib.tsvd_diag_split_bf16x3.argtypes = [vp, vp, i64, vp]
    lib.tsvd_diag_kgemm.restype = ctypes.c_int
    lib.tsvd_diag_kgemm.argtypes = [vp, ctypes.c_int, vp, vp, i64, i64, i64, i64, ctypes.c_int, ctypes.c_int, vp, sz,
                                    vp]
    lib.tsvd_diag_kgemm_sub.restype = ci
    lib.tsvd_diag_kgemm_sub.argtypes = [vp, vp, vp, i64, i64, i64, i64, vp]
    lib.tsvd_diag_omega.restype = ci
    lib.tsvd_diag_omega.argtypes = [vp, i64, u64, ci, vp]
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
    """Diagnostic counters of the last call that used `ws` (synchronises its
    stream).  "status" is TSVD_ENUMERIC when that call met a Cholesky
    breakdown, an unconverged eigenvector, a non-finite value or (adjoint of
    the truncation) a tie at the rank-k cut, else TSVD_OK."""
    buf = (ctypes.c_int32 * INFO_COUNT)()
    code = lib.tsvd_read_info(_ptr(ws), buf, _stream(ws.device))
    if code not in (TSVD_OK, TSVD_ENUMERIC):
        _check(code)
    out = {name: int(buf[i]) for i, name in enumerate(INFO_NAMES)}
    out["status"] = int(code)
    return out


def omega(n2: int, b: int, n3: int, seed: int):
    """The seeded test tensor (n2, b, n3) float64 on the host, as the
    seed-taking entry points draw it on the device (tsvd_omega)."""
    import numpy as np
    out = np.empty((n2, b, n3), dtype=np.float64)
    _check(lib.tsvd_omega(n2, b, n3, int(seed) & 0xFFFFFFFFFFFFFFFF, out.ctypes.data_as(ctypes.c_void_p)))
    return out


def _is_seed(Omega) -> bool:
    return isinstance(Omega, int) and not isinstance(Omega, bool)


def _omega_in(Omega, dt, n2: int, b: int, n3: int):
    """Validate a test-tensor argument: an int seed, or a contiguous device
    tensor of shape (n2, b, n3) in the working dtype."""
    if _is_seed(Omega):
        return
    if not isinstance(Omega, torch.Tensor):
        raise ValueError("Omega must be an int seed or a device tensor")
    _check_in(Omega, dt, "Omega")
    if tuple(Omega.shape) != (n2, b, n3):
        raise ValueError(f"Omega must have shape (n2, b, n3) = {(n2, b, n3)}, got {tuple(Omega.shape)}")


def _shape3(A: torch.Tensor, name="A"):
    if A.dim() != 3:
        raise ValueError(f"{name} must be a 3-way tensor (n1, n2, n3)")
    return tuple(int(x) for x in A.shape)


def _svd_call(name, op, A, Omega, k, b, q, prec, ws, out, with_x):
    prec = _prec_of(A, prec)
    dt = _dtype_of(prec)
    _check_in(A, dt, "A")
    n1, n2, n3 = _shape3(A)
    _omega_in(Omega, dt, n2, b, n3)
    dev = A.device
    if ws is None:
        ws = workspace(n1, n2, n3, k, b, q, prec, op, dev)
    if out is None:
        out = (torch.empty((n1, k, n3), dtype=dt, device=dev), torch.empty((k, n3), dtype=dt, device=dev),
               torch.empty((n2, k, n3), dtype=dt, device=dev))
    U, S, V = out
    for t, nm, shp in ((U, "U", (n1, k, n3)), (S, "S", (k, n3)), (V, "V", (n2, k, n3))):
        _check_in(t, dt, nm)
        if tuple(t.shape) != shp:
            raise ValueError(f"{nm} must have shape {shp}")
    X = torch.empty((n1, n2, n3), dtype=dt, device=dev) if with_x else None
    xs = [_ptr(X)] if name != "tsvd_rbk" and name != "tsvd_power" else []
    if _is_seed(Omega):
        f = getattr(lib, name)
        _check(f(_ptr(A), n1, n2, n3, k, b, q, int(Omega) & 0xFFFFFFFFFFFFFFFF, PREC[prec], _ptr(U), _ptr(S),
                 _ptr(V), *xs, _ptr(ws), ws.numel(), _stream(dev)))
    else:
        f = getattr(lib, name + "_omega")
        _check(f(_ptr(A), _ptr(Omega), n1, n2, n3, k, b, q, PREC[prec], _ptr(U), _ptr(S), _ptr(V), *xs, _ptr(ws),
                 ws.numel(), _stream(dev)))
    return U, S, V, X


def tsvd_rbk(A: torch.Tensor, Omega, k: int, b: int, q: int, prec=None, ws=None, out=None):
    """Alg. 2: returns (U, S, V) with U (n1,k,n3), S (k,n3), V (n2,k,n3).
    Omega: an int seed (the test tensor is drawn on the device) or a device
    tensor (n2, b, n3)."""
    return _svd_call("tsvd_rbk", "rbk", A, Omega, k, b, q, prec, ws, out, False)[:3]


NOALLOC_SCRATCH_BYTES = 64 << 20


def tsvd_rbk_noalloc(A: torch.Tensor, seed: int, k: int, b: int, q: int, prec=None, out=None):
    """tsvd_rbk through the entry point that allocates nothing (its scratch is
    the library's static device array of NOALLOC_SCRATCH_BYTES): returns
    (U, S, V).  Outputs are allocated here unless `out` is given."""
    prec = _prec_of(A, prec)
    dt = _dtype_of(prec)
    _check_in(A, dt, "A")
    n1, n2, n3 = _shape3(A)
    if not _is_seed(seed):
        raise ValueError("seed must be an int")
    dev = A.device
    if out is None:
        out = (torch.empty((n1, k, n3), dtype=dt, device=dev), torch.empty((k, n3), dtype=dt, device=dev),
               torch.empty((n2, k, n3), dtype=dt, device=dev))
    U, S, V = out
    for t, nm, shp in ((U, "U", (n1, k, n3)), (S, "S", (k, n3)), (V, "V", (n2, k, n3))):
        _check_in(t, dt, nm)
        if tuple(t.shape) != shp:
            raise ValueError(f"{nm} must have shape {shp}")
    _check(lib.tsvd_rbk_noalloc(_ptr(A), n1, n2, n3, k, b, q, int(seed) & 0xFFFFFFFFFFFFFFFF, PREC[prec], _ptr(U),
                                _ptr(S), _ptr(V), _stream(dev)))
    return U, S, V


def tsvd_rbk_approx(A, Omega, k, b, q, prec=None, ws=None):
    """Alg. 2 plus X_hat = U * S * V^T: returns (U, S, V, X_hat)."""
    return _svd_call("tsvd_rbk_approx", "approx", A, Omega, k, b, q, prec, ws, None, True)


def tsvd_rbk_literal(A, Omega, k, b, q, prec=None, ws=None, approx=True):
    """Alg. 2 with the literal Krylov powers (no orthonormalisation between
    steps): returns (U, S, V, X_hat) (X_hat None when approx is False)."""
    return _svd_call("tsvd_rbk_literal", "literal", A, Omega, k, b, q, prec, ws, None, approx)


def tsvd_rbk_ritz(A: torch.Tensor, Omega, k: int, b: int, q: int, prec=None, ws=None):
    """Alg. 2 with the basis truncated to its top b Ritz directions before the
    projection: returns (Qr, U, S, V), Qr (n1, b, n3) the truncated basis, U,
    S, V as tsvd_rbk (see tsvd_rbk_ritz in the C header)."""
    prec = _prec_of(A, prec)
    dt = _dtype_of(prec)
    _check_in(A, dt, "A")
    n1, n2, n3 = _shape3(A)
    _omega_in(Omega, dt, n2, b, n3)
    dev = A.device
    if ws is None:
        ws = workspace(n1, n2, n3, k, b, q, prec, "ritz", dev)
    Qr = torch.empty((n1, b, n3), dtype=dt, device=dev)
    U = torch.empty((n1, k, n3), dtype=dt, device=dev)
    S = torch.empty((k, n3), dtype=dt, device=dev)
    V = torch.empty((n2, k, n3), dtype=dt, device=dev)
    if _is_seed(Omega):
        _check(lib.tsvd_rbk_ritz(_ptr(A), n1, n2, n3, k, b, q, int(Omega) & 0xFFFFFFFFFFFFFFFF, PREC[prec], _ptr(Qr),
                                 _ptr(U), _ptr(S), _ptr(V), _ptr(ws), ws.numel(), _stream(dev)))
    else:
        _check(lib.tsvd_rbk_ritz_omega(_ptr(A), _ptr(Omega), n1, n2, n3, k, b, q, PREC[prec], _ptr(Qr), _ptr(U),
                                       _ptr(S), _ptr(V), _ptr(ws), ws.numel(), _stream(dev)))
    return Qr, U, S, V


def tsvd_rbk_approx_backward(A, Omega, G, k, b, q, prec=None, ws=None):
    """dL/dA for L(X_hat(A)) given G = dL/dX_hat (A's shape), X_hat the
    rank-k result of tsvd_rbk_approx (the derivative through the truncation)."""
    prec = _prec_of(A, prec)
    dt = _dtype_of(prec)
    _check_in(A, dt, "A")
    _check_in(G, dt, "G")
    n1, n2, n3 = _shape3(A)
    if tuple(G.shape) != (n1, n2, n3):
        raise ValueError(f"G must have A's shape {(n1, n2, n3)}, got {tuple(G.shape)}")
    _omega_in(Omega, dt, n2, b, n3)
    dev = A.device
    if ws is None:
        ws = workspace(n1, n2, n3, k, b, q, prec, "approx_bwd", dev)
    dA = torch.empty_like(A)
    if _is_seed(Omega):
        _check(lib.tsvd_rbk_approx_backward(_ptr(A), _ptr(G), n1, n2, n3, k, b, q, int(Omega) & 0xFFFFFFFFFFFFFFFF,
                                            PREC[prec], _ptr(dA), _ptr(ws), ws.numel(), _stream(dev)))
    else:
        _check(lib.tsvd_rbk_approx_backward_omega(_ptr(A), _ptr(Omega), _ptr(G), n1, n2, n3, k, b, q, PREC[prec],
                                                  _ptr(dA), _ptr(ws), ws.numel(), _stream(dev)))
    return dA


def tsvd_power(A: torch.Tensor, Omega, k: int, b: int, q: int, prec=None, ws=None):
    """Alg. 1 (q power iterations): returns (U, S, V) like tsvd_rbk."""
    return _svd_call("tsvd_power", "power", A, Omega, k, b, q, prec, ws, None, False)[:3]


def tsvd_power_approx(A, Omega, k, b, q, prec=None, ws=None):
    """Alg. 1 plus X_hat = U * S * V^T: returns (U, S, V, X_hat)."""
    return _svd_call("tsvd_power_approx", "power_approx", A, Omega, k, b, q, prec, ws, None, True)


def tsvd_tqr(A: torch.Tensor, prec=None, ws=None):
    """Alg. TQR: returns (Q, R), Q (n1, r, n3), R (r, n2, n3), r = min(n1, n2)."""
    prec = _prec_of(A, prec)
    dt = _dtype_of(prec)
    _check_in(A, dt, "A")
    n1, n2, n3 = _shape3(A)
    r = min(n1, n2)
    if ws is None:
        ws = workspace(n1, n2, n3, 0, 0, 0, prec, "tqr", A.device)
    Q = torch.empty((n1, r, n3), dtype=dt, device=A.device)
    R = torch.empty((r, n2, n3), dtype=dt, device=A.device)
    _check(lib.tsvd_tqr(_ptr(A), n1, n2, n3, PREC[prec], _ptr(Q), _ptr(R), _ptr(ws), ws.numel(),
                        _stream(A.device)))
    return Q, R


def tsvd_tpinv(A: torch.Tensor, rtol: float = 0.0, prec=None, ws=None):
    """Alg. mp: returns A^+ (n2, n1, n3) for any shape and rank; singular
    values s_j <= rtol * s_1 of a Fourier slice count as zero (rtol <= 0:
    tpinv_default_rtol)."""
    prec = _prec_of(A, prec)
    dt = _dtype_of(prec)
    _check_in(A, dt, "A")
    n1, n2, n3 = _shape3(A)
    if ws is None:
        ws = workspace(n1, n2, n3, 0, 0, 0, prec, "tpinv", A.device)
    X = torch.empty((n2, n1, n3), dtype=dt, device=A.device)
    _check(lib.tsvd_tpinv(_ptr(A), n1, n2, n3, float(rtol), PREC[prec], _ptr(X), _ptr(ws), ws.numel(),
                          _stream(A.device)))
    return X


def tpinv_default_rtol(n1: int, n2: int, prec: str) -> float:
    """The cut-off tsvd_tpinv takes for rtol <= 0."""
    return float(lib.tsvd_tpinv_default_rtol(n1, n2, PREC[prec]))


def tsvd_complete(M: torch.Tensor, mask: torch.Tensor, Omega, k: int, b: int, q: int, iters: int,
                  alg: int = 2, prec=None, ws=None):
    """Completion of Example 3: returns C^(iters) (n1, n2, n3).  mask: bool or
    uint8 tensor of M's shape (True / non-zero = observed).  Omega: int seed
    or device tensor (n2, b, n3)."""
    prec = _prec_of(M, prec)
    dt = _dtype_of(prec)
    _check_in(M, dt, "M")
    n1, n2, n3 = _shape3(M, "M")
    if tuple(mask.shape) != tuple(M.shape) or mask.dtype not in (torch.bool, torch.uint8):
        raise ValueError("mask must be a bool / uint8 tensor of M's shape")
    if not mask.is_cuda or not mask.is_contiguous():
        raise ValueError("mask must be a contiguous device tensor")
    _omega_in(Omega, dt, n2, b, n3)
    if ws is None:
        ws = workspace(n1, n2, n3, k, b, q, prec, "complete2" if alg == 2 else "complete1", M.device)
    C = torch.empty_like(M)
    if _is_seed(Omega):
        _check(lib.tsvd_complete(_ptr(M), _ptr(mask), n1, n2, n3, k, b, q, int(Omega) & 0xFFFFFFFFFFFFFFFF, iters,
                                 alg, PREC[prec], _ptr(C), _ptr(ws), ws.numel(), _stream(M.device)))
    else:
        _check(lib.tsvd_complete_omega(_ptr(M), _ptr(mask), _ptr(Omega), n1, n2, n3, k, b, q, iters, alg,
                                       PREC[prec], _ptr(C), _ptr(ws), ws.numel(), _stream(M.device)))
    return C


def tsvd_proj(A, Omega, b, q, prec=None, ws=None):
    """P(A) = Q * Q^T * A with Q the T-QR basis of the block Krylov tensor.
    Omega: int seed or device tensor (n2, b, n3)."""
    prec = _prec_of(A, prec)
    dt = _dtype_of(prec)
    _check_in(A, dt, "A")
    n1, n2, n3 = _shape3(A)
    _omega_in(Omega, dt, n2, b, n3)
    dev = A.device
    if ws is None:
        ws = workspace(n1, n2, n3, 1, b, q, prec, "proj", dev)
    P = torch.empty_like(A)
    if _is_seed(Omega):
        _check(lib.tsvd_proj(_ptr(A), n1, n2, n3, b, q, int(Omega) & 0xFFFFFFFFFFFFFFFF, PREC[prec], _ptr(P),
                             _ptr(ws), ws.numel(), _stream(dev)))
    else:
        _check(lib.tsvd_proj_omega(_ptr(A), _ptr(Omega), n1, n2, n3, b, q, PREC[prec], _ptr(P), _ptr(ws),
                                   ws.numel(), _stream(dev)))
    return P


def tsvd_proj_backward(A, Omega, G, b, q, prec=None, ws=None):
    """dL/dA for L(P(A)) given G = dL/dP (G has A's shape)."""
    prec = _prec_of(A, prec)
    dt = _dtype_of(prec)
    _check_in(A, dt, "A")
    _check_in(G, dt, "G")
    n1, n2, n3 = _shape3(A)
    if tuple(G.shape) != (n1, n2, n3):
        raise ValueError(f"G must have A's shape {(n1, n2, n3)}, got {tuple(G.shape)}")
    _omega_in(Omega, dt, n2, b, n3)
    dev = A.device
    if ws is None:
        ws = workspace(n1, n2, n3, 1, b, q, prec, "proj_bwd", dev)
    dA = torch.empty_like(A)
    if _is_seed(Omega):
        _check(lib.tsvd_proj_backward(_ptr(A), _ptr(G), n1, n2, n3, b, q, int(Omega) & 0xFFFFFFFFFFFFFFFF,
                                      PREC[prec], _ptr(dA), _ptr(ws), ws.numel(), _stream(dev)))
    else:
        _check(lib.tsvd_proj_backward_omega(_ptr(A), _ptr(Omega), _ptr(G), n1, n2, n3, b, q, PREC[prec], _ptr(dA),
                                            _ptr(ws), ws.numel(), _stream(dev)))
    return dA


class TProject(torch.autograd.Function):
    """A -> Q * Q^T * A with the hand-written adjoint; the Krylov blocks are
    recomputed in backward from (A, Omega), not stored.  Omega: int seed or
    device tensor (n2, b, n3)."""

    @staticmethod
    def forward(ctx, A, Omega, b, q, prec=None):
        if _is_seed(Omega):
            ctx.save_for_backward(A)
            ctx.seed = int(Omega)
        else:
            ctx.save_for_backward(A, Omega)
            ctx.seed = None
        ctx.b, ctx.q, ctx.prec = b, q, prec
        return tsvd_proj(A.detach().contiguous(), Omega if ctx.seed is not None else Omega.contiguous(), b, q, prec)

    @staticmethod
    def backward(ctx, G):
        if ctx.seed is not None:
            (A,) = ctx.saved_tensors
            Om = ctx.seed
        else:
            A, Om = ctx.saved_tensors
            Om = Om.contiguous()
        dA = tsvd_proj_backward(A.detach().contiguous(), Om, G.contiguous(), ctx.b, ctx.q, ctx.prec)
        return dA, None, None, None, None


class TApprox(torch.autograd.Function):
    """A -> X_hat(A), the rank-k result of Alg. 2, with the hand-written
    adjoint through the truncation; the Krylov blocks and the small SVD are
    recomputed in backward from (A, Omega).  Omega: int seed or device tensor
    (n2, b, n3)."""

    @staticmethod
    def forward(ctx, A, Omega, k, b, q, prec=None):
        if _is_seed(Omega):
            ctx.save_for_backward(A)
            ctx.seed = int(Omega)
        else:
            ctx.save_for_backward(A, Omega)
            ctx.seed = None
        ctx.k, ctx.b, ctx.q, ctx.prec = k, b, q, prec
        Om = Omega if ctx.seed is not None else Omega.contiguous()
        return tsvd_rbk_approx(A.detach().contiguous(), Om, k, b, q, prec)[3]

    @staticmethod
    def backward(ctx, G):
        if ctx.seed is not None:
            (A,) = ctx.saved_tensors
            Om = ctx.seed
        else:
            A, Om = ctx.saved_tensors
            Om = Om.contiguous()
        dA = tsvd_rbk_approx_backward(A.detach().contiguous(), Om, G.contiguous(), ctx.k, ctx.b, ctx.q, ctx.prec)
        return dA, None, None, None, None, None


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


KGEMM_MODE = {"f32": 0, "bf16": 1, "bf16x3": 2, "bf16x3s": 3}


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


def diag_kgemm_sub(A, X, C):
    """The Krylov-product kernel's update form (see tsvd_diag_kgemm_sub):
    C_f -= A_f X_f in place, complex64 tensors A (batch, rows, cols),
    X (batch, cols, N) and C (batch, rows, N)."""
    for name, t in (("A", A), ("X", X), ("C", C)):
        _check_in(t, torch.complex64, name)
    batch, rows, cols = A.shape
    N = X.shape[2]
    if tuple(X.shape) != (batch, cols, N) or tuple(C.shape) != (batch, rows, N):
        raise ValueError("A (batch, rows, cols), X (batch, cols, N) and C (batch, rows, N) do not match")
    _check(lib.tsvd_diag_kgemm_sub(_ptr(A), _ptr(X), _ptr(C), rows, cols, N, batch, _stream(A.device)))
    return C


def diag_split_bf16x3(Z):
    """Complex64 tensor -> the same number of (hi, lo) bf16 pairs (see
    tsvd_diag_split_bf16x3), held in a complex64 tensor of the same shape as
    opaque bits: the A operand of diag_kgemm(..., mode="bf16x3s")."""
    Z = Z.contiguous()
    out = torch.empty_like(Z)
    _check(lib.tsvd_diag_split_bf16x3(_ptr(Z), _ptr(out), Z.numel(), _stream(Z.device)))
    return out


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


def diag_omega(n: int, seed: int, dtype=torch.float64, device="cuda") -> torch.Tensor:
    """Values 0 .. n-1 of the seeded test-tensor stream, drawn on the device
    (see tsvd_diag_omega)."""
    out = torch.empty(n, dtype=dtype, device=device)
    _check(lib.tsvd_diag_omega(_ptr(out), n, int(seed) & 0xFFFFFFFFFFFFFFFF, 0 if dtype == torch.float64 else 1,
                               _stream(out.device)))
    return out


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
