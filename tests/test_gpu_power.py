"""Alg. 1 (classical randomized power iteration) on the HIP path (GPU).

Parity with the FP64 oracle element by element on well-conditioned inputs
(a low-tubal-rank tensor with geometric decay, where the squared spectrum of
the power iterates stays above the rounding level), and on the Sec. 5
Example 1 workload (n = 256, R = 45, P = 5, q = 2) on sampled Fourier slices:
singular values against the exact slice spectrum the inputs are built with,
X_hat slices against the oracle's, and the comparison the paper draws between
the two methods.  Tolerances: 1e-10 (FP64), 1e-5 (FP32), 1e-4 (BF16x3).
"""
import numpy as np
import pytest
import torch

from oracle import tsvd_oracle as O
from paper_2504_04989_amd import inputs
from tests.gpu_util import load_api, dev, fourier_factors, host, rel_f, unambiguous_phase_columns

pytestmark = pytest.mark.gpu
api = load_api()

TOL = {"f64": 1e-10, "f32": 1e-5, "bf16x3": 1e-4}


def _cast(x, prec):
    return x if prec == "f64" else x.astype(np.float32).astype(np.float64)


def _gpu(fn, A, Om, k, b, q, prec):
    dt = torch.float64 if prec == "f64" else torch.float32
    out = fn(dev(A, dt), dev(Om, dt), k, b, q, prec)
    torch.cuda.synchronize()
    return [host(t).astype(np.float64) for t in out]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape,k,b,q", [
    ((70, 90, 10), 8, 12, 2),     # ragged tiles, n1 < n2, even n3
    ((150, 97, 7), 6, 9, 3),      # n1 > n2, odd n3
    ((40, 33, 1), 3, 5, 1),       # n3 = 1: the matrix subspace iteration
    ((30, 40, 2), 4, 4, 0),       # DC + Nyquist only, q = 0, k = b
    ((65, 66, 17), 5, 8, 1),      # prime n3 > 13: direct DFT path
    ((36, 30, 6), 5, 10, 4),      # b (q + 1) = 50 > min(n1, n2): fine for Alg. 1
    ((130, 140, 4), 1, 1, 3),     # b = 1
])
def test_small_shapes(shape, k, b, q, prec):
    n1, n2, n3 = shape
    print(f"[power] shape={shape} k={k} b={b} q={q} prec={prec}", flush=True)
    A = _cast(inputs.lowrank_tensor(n1, n2, n3, min(n1, n2) // 2, ("geom", 0.8), 1e-3, 31), prec)
    Om = _cast(inputs.omega(n2, b, n3, 31), prec)
    U, S, V, X = _gpu(api.tsvd_power_approx, A, Om, k, b, q, prec)
    sl = O.power_tsvd(A, Om, k, b, q)
    Xo = O.approx_from_slices(sl, n1, n2, n3)
    tol = TOL[prec]
    assert rel_f(X, Xo) <= tol, f"X_hat rel err {rel_f(X, Xo):.3e}"
    Xf = O.tprod(O.tprod(U, O.s_tensor(S)), O.ttranspose(V))
    assert rel_f(Xf, Xo) <= tol
    F = n3 // 2 + 1
    Ub, Sb, Vb = fourier_factors(U, S, V, list(range(F)))
    s_err = np.max(np.abs(Sb.real - sl["Sf"]) / np.maximum(sl["Sf"], 1e-300))
    assert s_err <= tol, f"sigma rel err {s_err:.3e}"
    for f in range(F):
        ok = unambiguous_phase_columns(sl["Uf"][:, :, f])
        s_ext = np.r_[sl["s_all"][:, f], 0.0]
        gap = np.abs(np.diff(s_ext[: k + 1])) / s_ext[0]
        ok &= np.minimum(gap[:k], np.r_[1.0, gap[: k - 1]]) > 1e-3
        if ok.any():
            assert rel_f(Ub[:, ok, f], sl["Uf"][:, ok, f]) <= 1e3 * tol
            assert rel_f(Vb[:, ok, f], sl["Vf"][:, ok, f]) <= 1e3 * tol


def test_mixed_precision_bf16x3():
    n1, n2, n3, k, b, q = 96, 80, 8, 6, 10, 2
    A = _cast(inputs.lowrank_tensor(n1, n2, n3, 30, ("geom", 0.8), 1e-3, 32), "f32")
    Om = _cast(inputs.omega(n2, b, n3, 32), "f32")
    print(f"[power] bf16x3 shape={(n1, n2, n3)}", flush=True)
    X = _gpu(api.tsvd_power_approx, A, Om, k, b, q, "bf16x3")[3]
    Xo = O.power_approx(A, Om, k, b, q)
    assert rel_f(X, Xo) <= TOL["bf16x3"]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_q0_is_bitwise_alg2_q0(prec):
    # With no power iteration both methods run the same kernels on range(A Om).
    A = _cast(inputs.random_tensor((50, 44, 6), 33), prec)
    Om = _cast(inputs.omega(44, 7, 6, 33), prec)
    print(f"[power] q=0 bitwise prec={prec}", flush=True)
    a = _gpu(api.tsvd_power_approx, A, Om, 5, 7, 0, prec)
    r = _gpu(api.tsvd_rbk_approx, A, Om, 5, 7, 0, prec)
    for x, y in zip(a, r):
        assert np.array_equal(x, y)


def test_block_krylov_not_worse_than_power_iteration_gpu():
    # Sec. 3: range(Y_q) lies inside range(K) for the same Omega and q, so
    # Alg. 2's rank-k error is at most Alg. 1's; Example 1 spectra at a size
    # whose top-k spectrum the FP64 Gram resolves.
    n, n3, k, b, q = 96, 8, 6, 8, 2
    for decay in (("pow", -5.0), ("pow", -6.0), ("geom", 0.5)):
        A = inputs.spectrum_tensor(n, n, n3, decay, 34)
        Om = inputs.omega(n, b, n3, 34)
        print(f"[power] alg2 <= alg1 decay={decay}", flush=True)
        e1 = rel_f(_gpu(api.tsvd_power_approx, A, Om, k, b, q, "f64")[3], A)
        e2 = rel_f(_gpu(api.tsvd_rbk_approx, A, Om, k, b, q, "f64")[3], A)
        e1o = O.relative_error(A, O.power_approx(A, Om, k, b, q))
        e2o = O.relative_error(A, O.rbk_approx(A, Om, k, b, q))
        assert e2 <= e1 * (1 + 1e-9) + 1e-13
        assert abs(e1 - e1o) <= 1e-10 * e1o and abs(e2 - e2o) <= 1e-10 * e2o


# Example 1 asks for sigma_45 / sigma_1 = 5e-9 (m^-5), 1e-10 (m^-6) and 3e-14
# (0.5^m), below what one eigendecomposition of the FP64 Gram C_f C_f^H
# resolves (about sqrt(m u) sigma_1); the second pass of the FP64 small SVD
# (the leading eigenpairs projected out, the rest solved again) brings the GPU
# to the oracle's accuracy, which these checks hold it to.
@pytest.mark.parametrize("name", ["ex1_pow5_256", "ex1_pow6_256", "ex1_geom05_256"])
def test_example1_full_size_sampled_slices(name):
    A, Om, c = inputs.make_config(name)
    k, b, q = c["k"], c["b"], c["q"]
    print(f"[power] {name} full size", flush=True)
    n1, n2, n3 = A.shape
    outs = []
    for fn, op in ((api.tsvd_power_approx, "power_approx"), (api.tsvd_rbk_approx, "approx")):
        ws = api.workspace(n1, n2, n3, k, b, q, "f64", op, "cuda")
        outs.append(_gpu(lambda *a: fn(*a, ws=ws), A, Om, k, b, q, "f64"))
        info = api.read_info(ws)
        print(f"[power] {name} {op}: info {info}", flush=True)
        assert info["chol_breakdown"] == 0 and info["nonfinite"] == 0
    X1, X2 = outs
    sig = inputs._decay(c["decay"], min(A.shape[:2]))
    opt = np.sqrt(np.sum(sig[k:] ** 2) / np.sum(sig ** 2))
    e1, e2 = rel_f(X1[3], A), rel_f(X2[3], A)
    print(f"[power] {name}: alg1 {e1:.6e} alg2 {e2:.6e} optimum {opt:.6e}", flush=True)
    for e in (e1, e2):
        assert opt * (1 - 1e-6) - 1e-14 <= e <= opt * (1 + 1e-3) + 1e-12
    # Sec. 3: Alg. 2 is not worse than Alg. 1 (up to the rounding level)
    assert e2 <= e1 * (1 + 1e-6) + 1e-12
    freqs = [0, 1, 77, 128]
    Ab = np.fft.fft(A, axis=2)[:, :, freqs]
    for out, slices in ((X1, O.power_slices), (X2, O.rbk_slices)):
        U, S, V, X = out
        sl = slices(A, Om, k, b, q, freqs=freqs)
        Sb = np.fft.fft(S, axis=1)[:, freqs]
        Xb = np.fft.fft(X, axis=2)[:, :, freqs]
        for j, f in enumerate(freqs):
            # singular values against the exact spectrum the input is built with
            s = sig[:k]
            ds = np.max(np.abs(Sb[:, j].real - s))
            assert np.max(np.abs(sl["Sf"][:, j] - s)) <= 1e-10 * sig[0]
            Xo = (sl["Uf"][:, :, j] * sl["Sf"][:, j]) @ sl["Vf"][:, :, j].conj().T
            d = np.linalg.norm(Xb[:, :, j] - Xo) / np.linalg.norm(Ab[:, :, j])
            print(f"[power] {name} {slices.__name__} f={f}: max sigma err {ds / sig[0]:.2e} sigma_1, "
                  f"X_hat slice diff {d:.3e}", flush=True)
            assert ds <= 1e-10 * sig[0]
            assert d <= 1e-10
