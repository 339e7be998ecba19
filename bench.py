#!/usr/bin/env python
"""Throughput of the randomized block Krylov truncated T-SVD (Alg. 2) on one
MI355X: truncated T-SVDs per second with the input resident in HBM, for the
plain FP32 form and the mixed-precision forms (BF16x3 and BF16 Krylov
products, FP64 Gram / Cholesky / eigensolver), each checked against the FP64
oracle.

One step = one call of the seed-taking tsvd_rbk on the whole tensor (the
test tensor drawn on the device, mode-3 DFT, Krylov products,
orthonormalisation, small SVD, lift, inverse DFT) on seeded synthetic input
of the stated shape.  Each form is timed over K steps after W warmup steps.
`value` is the fastest form whose relative error against the FP64 oracle on
the 8 sampled Fourier slices is at most 1e-4; a form with no measured error
never qualifies.  Inside the timed region, HIP events on the library's stream
time every kernel class (roofline).  Side legs: the other workloads (1000^2 x
32 FP32, 512^2 x 200 in three precisions, the 2000^2 x 16 projection forward
and backward), Alg. 1 vs Alg. 2 on Example 1, the completion of Example 3 and
the T-QR / T-pseudoinverse.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--precs f32,bf16x3,bf16]
                    [--no-cpu-baseline] [--no-legs] [--no-alg1] [--no-completion] [--no-tqr]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

PEAK = {  # MI355X published peaks
    "hbm_gbs": 8000.0,
    "mfma_tflops": {"f32": 157.3, "f64": 78.6, "bf16": 2500.0},
    "valu_tflops": {"f32": 157.3, "f64": 78.6},
}
RELERR_GATE = 1e-4
METRIC = "truncated T-SVDs/s + MFMA util at rel-err<=1e-4: mixed-prec vs plain FP32"
C5_FREQS = [0, 5, 9, 14, 18, 23, 27, 32]   # the 8 sampled Fourier slices of the 4096 x 4096 x 64 workload


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def class_work(cls: str, c: dict, prec: str):
    """Algorithmic work of one step in a kernel class, as a dict:
    flops (algorithmic, complex products at 8 real flops per multiply-add),
    xf (MFMA flops the form executes per algorithmic flop: 3 for BF16x3),
    bytes (algorithmic HBM bytes, where stated), mfma / hbm peaks, and the
    bound of the algorithmic roofline: the resource whose time at its
    published peak is the larger (algorithmic flops / MFMA peak of the
    product's type against algorithmic bytes / HBM peak).  None for classes
    without a stated work."""
    n1, n2, n3, k, b, q = c["n1"], c["n2"], c["n3"], c["k"], c["b"], c["q"]
    F = n3 // 2 + 1
    m = b * (q + 1)
    es = 8 if prec == "f64" else 4
    hbm = PEAK["hbm_gbs"] * 1e9
    if cls == "gemm_krylov":   # (2q + 2) passes over A_f, b columns each
        launches = 2 * q + 2
        fl = launches * 8.0 * n1 * n2 * b * F
        # per launch: A_f read once (complex, 2 es bytes; BF16x3 keeps it as
        # (hi, lo) bf16 pairs of the same size, BF16 bulk needs one bf16 pair),
        # the thin block read and the result written (complex, 2 es bytes)
        ea = 4 if prec == "bf16" else 2 * es
        by = launches * (ea * n1 * n2 + 2 * es * (n1 + n2) * b) * F
        dt = "bf16" if prec in ("bf16", "bf16x3") else prec
        w = {"flops": fl, "xf": 3.0 if prec == "bf16x3" else 1.0, "bytes": by,
             "mfma_peak": PEAK["mfma_tflops"][dt] * 1e12, "hbm_peak": hbm,
             "note": "algorithmic flops 8 n1 n2 b F and bytes (A_f once, thin block, result) per launch" +
                     (" (BF16x3 executes 3 BF16 products per algorithmic one)" if prec == "bf16x3" else "")}
    elif cls == "fft_A":       # read the real tensor, write the half spectrum
        return {"flops": None, "xf": 1.0, "bytes": float(es * n1 * n2 * n3 + 2 * es * n1 * n2 * F),
                "mfma_peak": None, "hbm_peak": hbm, "bound": "hbm", "note": "algorithmic bytes"}
    elif cls == "gemm_orth":   # block CGS2 against earlier blocks + shifted CholeskyQR, FP64 arithmetic
        # CholeskyQR passes per block: shifted + 1 (FP32 storage, when the
        # FP64 orthogonality bound allows it, else + 2); FP64 adds two more
        # shifted passes
        # On FP32 storage the first projection pass (coefficients and update,
        # 16 n1 (i b) b flops against block i) runs in FP32 arithmetic on the
        # FP32 MFMA, the rest in FP64: the peak is the rate at which the mix
        # would run with every part at its own published peak.
        passes = 5 if prec == "f64" else cholqr_passes(n1, b)
        proj = sum(16.0 * n1 * (i * b) * b for i in range(1, q + 1))
        fl = 2 * proj + (q + 1) * passes * 8.0 * n1 * b * (b + 1)
        fl32 = 0.0 if prec == "f64" else proj
        p64, p32 = PEAK["mfma_tflops"]["f64"] * 1e12, PEAK["mfma_tflops"]["f32"] * 1e12
        peak = fl / ((fl - fl32) / p64 + fl32 / p32)
        w = {"flops": fl * F, "xf": 1.0, "bytes": None, "mfma_peak": peak,
             "hbm_peak": hbm, "note": "algorithmic flops (Hermitian Grams and W R^-1 counted as upper halves); "
                                      + ("FP64 arithmetic" if prec == "f64" else
                                         "first projection pass in FP32 arithmetic, the rest in FP64; peak = "
                                         "the mix's rate with each part at its published peak")}
    elif cls == "chol":        # b x b complex Cholesky + triangular inverse per slice, one per CholeskyQR pass
        passes = 5 if prec == "f64" else cholqr_passes(n1, b)
        return {"flops": passes * (q + 1) * F * (16.0 / 3.0 * b ** 3), "xf": 1.0, "bytes": None,
                "mfma_peak": PEAK["valu_tflops"]["f64"] * 1e12, "hbm_peak": hbm, "bound": "alu",
                "note": "algorithmic FP64 flops against the FP64 vector peak"}
    elif cls == "heig_tri":    # Householder tridiagonalisation of the m x m Hermitian G_f
        return {"flops": F * (16.0 / 3.0 * m ** 3), "xf": 1.0, "bytes": None,
                "mfma_peak": PEAK["valu_tflops"]["f64"] * 1e12, "hbm_peak": hbm, "bound": "alu",
                "note": "algorithmic FP64 flops against the FP64 vector peak"}
    elif cls == "gemm_lift":   # G = T^H T (Hermitian: upper half), U = Q W_k, V = T W_k
        w = {"flops": F * (4.0 * n2 * m * (m + 1) + 8.0 * (n1 + n2) * m * k), "xf": 1.0, "bytes": None,
             "mfma_peak": PEAK["mfma_tflops"]["f64"] * 1e12, "hbm_peak": hbm,
             "note": "algorithmic flops (Hermitian Gram counted as its upper half)"}
    else:
        return None
    t_mfma = w["flops"] / w["mfma_peak"]
    t_hbm = w["bytes"] / w["hbm_peak"] if w["bytes"] else 0.0
    w["bound"] = "hbm" if t_hbm > t_mfma else "mfma"
    return w


def cholqr_passes(rows: int, b: int) -> int:
    """CholeskyQR passes per FP32-stored block: the shifted pass plus one
    unshifted pass when the FP64 orthogonality bound of that pass stays within
    2^-20, else plus two (the library's rule for FP32 storage)."""
    u64 = 2.0 ** -53
    alpha = 11.0 * (rows * b + b * (b + 1)) * u64 * b
    return 2 if alpha * u64 * 1e16 <= 2.0 ** -20 else 3


def roofline_for(kernels: dict, c: dict, prec: str, workload: str):
    """Roofline of the dominant kernel class that has a stated algorithmic
    work.  bound = hbm: achieved = algorithmic bytes per step / that class's
    time per step against the HBM peak; bound = mfma or alu: algorithmic flops
    against the MFMA (or vector) peak of the class's arithmetic type.
    frac_mfma_executed gives the MFMA flops the form actually issues (3x the
    algorithmic flops for BF16x3) against the MFMA peak."""
    for cls, v in sorted(kernels.items(), key=lambda kv: -kv[1]["ms_per_step"]):
        w = class_work(cls, c, prec)
        if w is None:
            continue
        sec = v["ms_per_step"] * 1e-3
        if w["bound"] == "hbm":
            achieved, peak, unit = w["bytes"] / sec / 1e9, w["hbm_peak"] / 1e9, "GB/s"
        else:
            achieved, peak, unit = w["flops"] / sec / 1e12, w["mfma_peak"] / 1e12, "TFLOP/s"
        tr = profiled_traffic(cls, prec, workload)
        out = {"kernel": cls, "bound": w["bound"], "achieved": achieved, "peak": peak, "unit": unit,
               "frac": achieved / peak,
               "traffic": tr["bytes_per_launch"] if tr else None,
               "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
               "traffic_source": tr["source"] if tr else None, "work": w["note"],
               "launches_per_step": v["launches_per_step"], "avg_launch_ms": v["avg_launch_ms"]}
        if w["flops"] and w["mfma_peak"]:
            out["frac_mfma_executed"] = w["flops"] * w["xf"] / sec / w["mfma_peak"]
        if w["bytes"]:
            out["algorithmic_bytes_per_launch"] = w["bytes"] / v["launches_per_step"]
        return out
    return None


def kernel_figures(kernels: dict, c: dict, prec: str):
    """Krylov-product MFMA utilisation (algorithmic and executed flops against
    the MFMA peak of the form's type), their HBM rate over the algorithmic
    bytes, and the mode-3 DFT's HBM rate, from the timed kernel classes."""
    out = {}
    kry = kernels.get("gemm_krylov")
    if kry:
        w = class_work("gemm_krylov", c, prec)
        sec = kry["ms_per_step"] * 1e-3
        out["krylov_mfma_util"] = w["flops"] / sec / w["mfma_peak"]
        out["krylov_mfma_util_executed"] = w["flops"] * w["xf"] / sec / w["mfma_peak"]
        out["krylov_tflops_algorithmic"] = w["flops"] / sec / 1e12
        out["krylov_hbm_frac"] = w["bytes"] / sec / w["hbm_peak"]
        out["krylov_bound"] = w["bound"]
    fft = kernels.get("fft_A")
    if fft:
        w = class_work("fft_A", c, prec)
        gbs = w["bytes"] / (fft["ms_per_step"] * 1e-3) / 1e9
        out["fft_hbm"] = {"achieved_GBs": gbs, "peak_GBs": w["hbm_peak"] / 1e9, "frac": gbs * 1e9 / w["hbm_peak"],
                          "bytes_per_launch": w["bytes"], "ms_per_launch": fft["avg_launch_ms"]}
    return out


def profiled_traffic(cls: str, prec: str, workload: str):
    """HBM bytes per launch of a kernel class from the rocprofv3 counter
    summaries in profiles/ (FETCH_SIZE and WRITE_SIZE scaled by a device copy
    of known size), or None when no summary covers it or when a source file it
    was measured on has changed since."""
    import glob
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    for fn in sorted(glob.glob(os.path.join(root, "profiles", "*.md"))):
        for line in open(fn):
            if not line.startswith("traffic-record:"):
                continue
            rec = json.loads(line.split(":", 1)[1])
            if (rec["class"], rec["form"], rec["workload"]) != (cls, prec, workload):
                continue
            for src, digest in rec["sources_sha256"].items():
                path = os.path.join(root, src)
                if not os.path.exists(path) or hashlib.sha256(open(path, "rb").read()).hexdigest() != digest:
                    return None
            return {"bytes_per_launch": rec["bytes_per_launch"], "source": os.path.relpath(fn, root)}
    return None


def time_calls(api, fn, steps: int, warmup: int):
    """Warmup, then exactly `steps` timed calls bracketed by synchronisations,
    with the per-class HIP-event timer on; returns (ms per call, kernels)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    api.diag_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    timing = api.diag_timing_read()
    api.diag_timing(False)
    kernels = {}
    for cls, (tms, cnt) in timing.items():
        if cnt:
            kernels[cls] = {"ms_per_step": tms / steps, "launches_per_step": cnt / steps, "avg_launch_ms": tms / cnt}
    return ms, kernels


def slice_relerr(U, S, V, sl, freqs, idx=None):
    """Parseval-weighted relative error of X_hat = U * S * V^T on the sampled
    Fourier slices against the oracle's slices (idx: positions of freqs in
    the oracle's arrays).  Returns (weighted error, per-slice errors, per-slice
    largest relative singular-value errors)."""
    n3 = U.shape[2]
    idx = list(range(len(freqs))) if idx is None else idx
    w = np.exp(-2j * np.pi * np.outer(np.arange(n3), freqs) / n3)      # (n3, nf)
    Ub, Vb, Sb = U @ w, V @ w, (S @ w).real
    num = den = 0.0
    per, sig = [], []
    for i, (f, j) in enumerate(zip(freqs, idx)):
        Xg = (Ub[:, :, i] * Sb[:, i]) @ Vb[:, :, i].conj().T
        Xo = (sl["Uf"][:, :, j] * sl["Sf"][:, j]) @ sl["Vf"][:, :, j].conj().T
        d2, o2 = np.linalg.norm(Xg - Xo) ** 2, np.linalg.norm(Xo) ** 2
        wt = 1.0 if f == 0 or 2 * f == n3 else 2.0
        num += wt * d2
        den += wt * o2
        per.append(float(np.sqrt(d2 / o2)))
        sig.append(float(np.max(np.abs(Sb[:, i] - sl["Sf"][:, j]) / sl["Sf"][:, j])))
    return float(np.sqrt(num / den)), per, sig


def run_rbk_form(api, A64, c, prec, steps, warmup, workload):
    """Time tsvd_rbk (seed-taking) in one precision; returns (leg, outputs)."""
    import torch
    n1, n2, n3 = A64.shape
    k, b, q, seed = c["k"], c["b"], c["q"], c["seed"]
    dt = torch.float64 if prec == "f64" else torch.float32
    A = torch.from_numpy(A64.astype(np.float64 if prec == "f64" else np.float32)).to("cuda")
    ws = api.workspace(n1, n2, n3, k, b, q, prec, "rbk", "cuda")
    out = (torch.empty((n1, k, n3), dtype=dt, device="cuda"), torch.empty((k, n3), dtype=dt, device="cuda"),
           torch.empty((n2, k, n3), dtype=dt, device="cuda"))
    log(f"[bench] {workload} {prec}: {n1}x{n2}x{n3} k={k} b={b} q={q} seed={seed} workspace "
        f"{ws.numel() / 2**20:.1f} MiB")
    ms, kernels = time_calls(api, lambda: api.tsvd_rbk(A, seed, k, b, q, prec, ws=ws, out=out), steps, warmup)
    info = api.read_info(ws)
    log(f"[bench] {workload} {prec}: {ms:.3f} ms/step ({1e3 / ms:.2f} T-SVD/s); info {info}")
    for cls, v in sorted(kernels.items(), key=lambda kv: -kv[1]["ms_per_step"]):
        log(f"[bench]   {cls:12s} {v['ms_per_step']:.3f} ms/step  {v['launches_per_step']:.0f} launches  "
            f"{v['avg_launch_ms'] * 1e3:.1f} us/launch")
    leg = {"value": 1e3 / ms, "ms_per_step": ms, "roofline": roofline_for(kernels, c, prec, workload),
           "kernels": kernels, "numeric_info": info}
    leg.update(kernel_figures(kernels, c, prec))
    outs = tuple(t.cpu().numpy().astype(np.float64) for t in out)
    del A, ws, out
    torch.cuda.empty_cache()
    return leg, outs


def other_workloads(api, inputs, steps: int, warmup: int):
    """The other workloads: 1000 x 1000 x 32 (FP32), the 512 x 512 x 200
    hyperspectral tensor (FP32, BF16x3, BF16) and the 2000 x 2000 x 16
    projection forward + backward (FP32): per form the time per call, the
    roofline of its dominant class, the Krylov MFMA utilisation, the DFT's HBM
    rate and the error against the FP64 oracle on sampled slices (the oracle's
    time per slice beside it)."""
    import torch
    from oracle import tsvd_oracle as O
    res = {}
    for name, precs, freqs in (("c2_fp32_1000x1000x32", ["f32"], [0, 8, 16]),
                               ("c3_hyper_512x512x200", ["f32", "bf16x3", "bf16"], [0, 1, 7, 50, 100])):
        A64, Om64, c = inputs.make_config(name)
        A32 = A64.astype(np.float32).astype(np.float64)
        Om32 = Om64.astype(np.float32).astype(np.float64)
        t0 = time.perf_counter()
        sl = O.rbk_slices(A32, Om32, c["k"], c["b"], c["q"], freqs=freqs)
        t_or = (time.perf_counter() - t0) / len(freqs)
        legs = {}
        for prec in precs:
            leg, outs = run_rbk_form(api, A64, c, prec, steps, warmup, name)
            e, per, sig = slice_relerr(*outs, sl, freqs)
            leg.update(rel_err_vs_oracle=e, rel_err_slices=dict(zip(map(str, freqs), per)),
                       sigma_rel_err_slices=dict(zip(map(str, freqs), sig)))
            log(f"[bench] {name} {prec}: rel err vs FP64 oracle on slices {freqs}: {e:.2e}")
            legs[prec] = leg
        F = c["n3"] // 2 + 1
        res[name] = {"forms": legs, "oracle_seconds_per_slice": t_or, "oracle_seconds_extrapolated": t_or * F,
                     "sampled_slices": freqs}
    # the differentiation form: P(A) = Q * Q^T * A and its adjoint
    name = "c4_completion_2000x2000x16"
    A64, Om64, c = inputs.make_config(name)
    T, M = c["T"], c["M"]
    b, q, seed = c["b"], c["q"], c["seed"]
    n1, n2, n3 = A64.shape
    X = torch.from_numpy(A64.astype(np.float32)).to("cuda")
    Td, Md = torch.from_numpy(T.astype(np.float32)).to("cuda"), torch.from_numpy(M.astype(np.float32)).to("cuda")
    wf = api.workspace(n1, n2, n3, 1, b, q, "f32", "proj", "cuda")
    wb = api.workspace(n1, n2, n3, 1, b, q, "f32", "proj_bwd", "cuda")
    state = {}

    def fwd_bwd():
        P = api.tsvd_proj(X, seed, b, q, "f32", ws=wf)
        G = -2.0 * Md * (Td - P)
        state["P"], state["G"] = P, G
        state["dA"] = api.tsvd_proj_backward(X, seed, G, b, q, "f32", ws=wb)

    ms, kernels = time_calls(api, fwd_bwd, max(steps // 2, 3), 1)
    P, G, dA = (state[k].cpu().numpy().astype(np.float64) for k in ("P", "G", "dA"))
    lhs, rhs = float(np.sum(dA * A64.astype(np.float32))), float(np.sum(G * P))
    freqs = [0, 5]
    X32 = A64.astype(np.float32).astype(np.float64)
    Om32 = Om64.astype(np.float32).astype(np.float64)
    Ab, Ob, Gb = (O.dft_mode3(x, freqs) for x in (X32, Om32, G))
    Db = np.fft.fft(dA, axis=2)
    t0 = time.perf_counter()
    gerr = {}
    for j, f in enumerate(freqs):
        Df = O._proj_slice_adjoint(Ab[:, :, j], Ob[:, :, j], Gb[:, :, j], q)
        gerr[str(f)] = float(np.linalg.norm(Db[:, :, f] - Df) / np.linalg.norm(Df))
    t_or = (time.perf_counter() - t0) / len(freqs)
    log(f"[bench] {name} f32 forward + backward: {ms:.3f} ms; Euler rel {abs(lhs - rhs) / abs(rhs):.1e}; "
        f"gradient rel err vs oracle {gerr}")
    cfw = dict(c, k=1)
    kf = kernel_figures(kernels, cfw, "f32")
    res[name] = {"ms_per_fwd_bwd": ms, "fwd_bwd_per_s": 1e3 / ms, "kernels": kernels,
                 "fft_hbm": kf.get("fft_hbm"), "euler_rel": abs(lhs - rhs) / abs(rhs),
                 "gradient_rel_err_slices": gerr, "oracle_adjoint_seconds_per_slice": t_or}
    del X, Td, Md, wf, wb, state
    torch.cuda.empty_cache()
    return res


def compare_alg1_alg2(api, inputs, steps: int, warmup: int):
    """Sec. 5, Example 1: the power-iteration method (Alg. 1) and the block
    Krylov method (Alg. 2) on n x n x n tensors with prescribed slice spectra,
    R = 45, P = 5, q = 2, FP64.  Per spectrum: ms per call of each method (K
    timed calls after W warmups, input resident in HBM) and the relative
    Frobenius error of its rank-R approximation, beside the optimum."""
    import torch
    res = {}
    for name in inputs.EX1_CONFIGS:
        A64, _, c = inputs.make_config(name)
        k, b, q, seed = c["k"], c["b"], c["q"], c["seed"]
        n1, n2, n3 = A64.shape
        A = torch.from_numpy(A64).to("cuda")
        sig = inputs._decay(c["decay"], min(n1, n2))
        case = {"optimum_rel_err": float(np.sqrt(np.sum(sig[k:] ** 2) / np.sum(sig ** 2)))}
        for alg, fn, op in (("alg1", api.tsvd_power_approx, "power_approx"), ("alg2", api.tsvd_rbk_approx, "approx")):
            ws = api.workspace(n1, n2, n3, k, b, q, "f64", op, "cuda")
            for _ in range(warmup):
                out = fn(A, seed, k, b, q, "f64", ws=ws)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                out = fn(A, seed, k, b, q, "f64", ws=ws)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / steps
            err = float(torch.linalg.norm(out[3] - A) / torch.linalg.norm(A))
            case[alg] = {"ms_per_call": ms, "rel_err": err, "basis_columns": b if alg == "alg1" else b * (q + 1)}
            del ws, out
        log(f"[bench] {name}: alg1 {case['alg1']['ms_per_call']:.2f} ms err {case['alg1']['rel_err']:.4e}; "
            f"alg2 {case['alg2']['ms_per_call']:.2f} ms err {case['alg2']['rel_err']:.4e}; "
            f"optimum {case['optimum_rel_err']:.4e}")
        res[name] = case
        del A
        torch.cuda.empty_cache()
    return {"workload": "Example 1 spectra m^-5, m^-6, 0.5^m; n = 256; R = 45, P = 5, q = 2; f64", "cases": res}


def completion_runs(api, inputs):
    """Sec. 5, Example 3: completion of a 512 x 768 x 3 image stand-in with
    70% of the pixels missing, tubal rank 50, P = 10, q = 2, 100 iterations,
    with Alg. 2 and with Alg. 1 as the rank-50 step, FP32.  Per method: the
    time of the whole completion call with the data resident, ms per
    iteration and the PSNR of the result against the full image."""
    import torch
    name = "ex3_image_512x768x3"
    c = inputs.COMPLETION_CONFIGS[name]
    M64 = inputs.image_tensor(c["n1"], c["n2"], c["n3"], c["seed"])
    T = inputs.bernoulli_mask(M64.shape, c["keep"], c["seed"])
    M = torch.from_numpy(M64.astype(np.float32)).to("cuda")
    mask = torch.from_numpy(T != 0).to("cuda")
    k, b, q, iters, seed = c["k"], c["b"], c["q"], c["iters"], c["seed"]
    res = {}
    for alg in (2, 1):
        ws = api.workspace(c["n1"], c["n2"], c["n3"], k, b, q, "f32", f"complete{alg}", "cuda")
        api.tsvd_complete(M, mask, seed, k, b, q, 2, alg, "f32", ws=ws)   # warmup
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        C = api.tsvd_complete(M, mask, seed, k, b, q, iters, alg, "f32", ws=ws)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        mse = float(torch.mean((C.double() - M.double()) ** 2))
        ps = float(10 * np.log10(255.0 ** 2 / mse))
        res[f"alg{alg}"] = {"seconds": sec, "ms_per_iteration": sec * 1e3 / iters, "psnr_db": ps}
        log(f"[bench] {name} alg{alg}: {iters} iterations in {sec:.3f} s ({sec * 1e3 / iters:.2f} ms each), "
            f"PSNR {ps:.2f} dB")
        del ws, C
    mse0 = float(np.mean((T * M64 - M64) ** 2))
    return {"workload": "Example 3: 512 x 768 x 3 power-law image stand-in, 70% of pixels missing, R = 50, P = 10, "
                        "q = 2, 100 iterations, f32", "psnr_observed_db": float(10 * np.log10(255.0 ** 2 / mse0)),
            "runs": res}


def tqr_runs(api, inputs, steps: int, warmup: int):
    """T-QR (Alg. TQR) and the T-pseudoinverse (Alg. mp) of a tall Gaussian
    tensor, FP32, input resident: ms per call and the rate over the
    algorithmic HBM traffic (read A, write Q and R, or A^+)."""
    import torch
    n1, n2, n3 = 4096, 256, 64
    A = torch.from_numpy(inputs.random_tensor((n1, n2, n3), 81).astype(np.float32)).to("cuda")
    res = {}
    for op, fn, out_elems in (("tqr", api.tsvd_tqr, n1 * n2 * n3 + n2 * n2 * n3),
                              ("tpinv", api.tsvd_tpinv, n2 * n1 * n3)):
        ws = api.workspace(n1, n2, n3, 0, 0, 0, "f32", op, "cuda")
        for _ in range(warmup):
            fn(A, prec="f32", ws=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn(A, prec="f32", ws=ws)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        gb = 4.0 * (n1 * n2 * n3 + out_elems) / 1e9
        res[op] = {"ms_per_call": ms, "algorithmic_GB": gb, "GB_per_s": gb / (ms * 1e-3)}
        log(f"[bench] {op} {n1}x{n2}x{n3} f32: {ms:.3f} ms per call ({gb / (ms * 1e-3):.0f} GB/s algorithmic)")
        del ws
    return {"workload": f"Gaussian {n1} x {n2} x {n3}, f32", "calls": res}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c5_fp32_4096x4096x64")
    ap.add_argument("--precs", default=None,
                    help="comma-separated forms to time (default: f32,bf16x3,bf16; f64 for FP64 workloads)")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the FP64 oracle (then no form is gated and the headline is the plain FP32 form)")
    ap.add_argument("--no-legs", action="store_true", help="skip the other workloads (1000^2x32, 512^2x200, 2000^2x16)")
    ap.add_argument("--no-alg1", action="store_true", help="skip the Alg. 1 vs Alg. 2 comparison (Example 1)")
    ap.add_argument("--no-completion", action="store_true", help="skip the completion runs (Example 3)")
    ap.add_argument("--no-tqr", action="store_true", help="skip the T-QR / T-pseudoinverse timing")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB 5 times (HBM counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the Fourier slices of one tensor are processed by one device, and "
              "the frequency-sharded multi-GPU path is not built (see the design notes)", file=sys.stderr)
        print(json.dumps({"error": "only --gpus 1 is supported", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.calibrate_copy_mib:
        import torch
        n = args.calibrate_copy_mib * 2**20 // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 5}), flush=True)
        return

    from paper_2504_04989_amd import inputs

    t0 = time.perf_counter()
    A64, Om64, c = inputs.make_config(args.workload)
    log(f"[bench] generated {args.workload} in {time.perf_counter() - t0:.1f} s")
    precs = args.precs.split(",") if args.precs else (["f64"] if c["prec"] == "f64" else ["f32", "bf16x3", "bf16"])
    n1, n2, n3 = A64.shape
    k, b, q = c["k"], c["b"], c["q"]
    F = n3 // 2 + 1
    freqs = [f for f in C5_FREQS if f < F] if args.workload.startswith("c5") else sorted({0, F // 2, F - 1})

    # The FP64 oracle on the sampled slices runs in worker processes forked
    # now, before this process initialises the GPU, and overlaps the GPU legs.
    pool = None
    if not args.no_cpu_baseline:
        from oracle.pool import SlicePool
        cast = (lambda x: x) if precs == ["f64"] else (lambda x: x.astype(np.float32).astype(np.float64))
        pool = SlicePool(cast(A64), cast(Om64), k, b, q, freqs)
        log(f"[bench] FP64 oracle started on Fourier slices {freqs}: {pool.workers} workers x {pool.threads} "
            f"BLAS threads (DFT {pool.dft_seconds:.1f} s)")
    del Om64

    from paper_2504_04989_amd import api

    legs, outs = {}, {}
    for prec in precs:
        legs[prec], outs[prec] = run_rbk_form(api, A64, c, prec, args.steps, args.warmup, args.workload)
    del A64

    others = None if args.no_legs else other_workloads(api, inputs, max(args.steps // 2, 3), 1)
    alg12 = None if args.no_alg1 else compare_alg1_alg2(api, inputs, max(args.steps // 2, 3), 1)
    compl = None if args.no_completion else completion_runs(api, inputs)
    tqr = None if args.no_tqr else tqr_runs(api, inputs, max(args.steps // 2, 3), 1)

    base = None
    if pool is not None:
        sl = pool.get(progress=lambda msg: log(f"[bench] {msg}"))
        t_slice = sl["wall"] / len(freqs)
        base = {"value": 1.0 / (t_slice * F), "unit": "T-SVD/s", "cores": int(sl["threads"]), "kind": "oracle",
                "sample": f"FP64 oracle (plain numpy DFT, Householder QR, Jacobi SVD): mode-3 DFT at {len(freqs)} "
                          f"frequencies + Alg. 2 on Fourier slices {freqs} of {F} in {sl['wall']:.1f} s wall "
                          f"({sl['workers']} worker processes, {sl['threads']} threads in all; "
                          f"{np.mean(sl['seconds']):.1f} s per slice in a worker), extrapolated to all {F} slices: "
                          f"{t_slice * F:.0f} s per T-SVD"}
        for prec in precs:
            e, per, sig = slice_relerr(*outs[prec], sl, freqs)
            legs[prec]["rel_err_vs_oracle"] = e
            legs[prec]["rel_err_slices"] = dict(zip(map(str, freqs), per))
            legs[prec]["sigma_rel_err_slices"] = dict(zip(map(str, freqs), sig))
            log(f"[bench] {prec}: rel err vs FP64 oracle on slices {freqs}: {e:.2e} "
                f"(per slice {', '.join(f'{x:.1e}' for x in per)})")
        log(f"[bench] cpu baseline {base['value']:.4g} T-SVD/s ({base['sample']})")

    # headline: the fastest form whose measured error meets the gate; with no
    # measured error no form qualifies and the plain FP32 form is reported,
    # marked ungated
    gated = [p for p in precs if legs[p].get("rel_err_vs_oracle") is not None
             and legs[p]["rel_err_vs_oracle"] <= RELERR_GATE]
    if gated:
        best = max(gated, key=lambda p: legs[p]["value"])
    else:
        best = "f32" if "f32" in precs else precs[0]
    head = legs[best]
    res = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "T-SVD/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": best,
        "data": "synthetic",
        "config": {"workload": args.workload, "n1": n1, "n2": n2, "n3": n3, "k": k, "b": b, "q": q,
                   "seed": c["seed"], "form": best, "forms_timed": precs},
        "gate": {"rel_err_max": RELERR_GATE, "passed": bool(gated), "forms_passing": gated,
                 "rel_err_vs_oracle": head.get("rel_err_vs_oracle"), "sampled_slices": freqs},
        "roofline": head["roofline"],
        "krylov_mfma_util": head.get("krylov_mfma_util"),
        "krylov_mfma_util_executed": head.get("krylov_mfma_util_executed"),
        "fft_hbm": head.get("fft_hbm"),
        "forms": legs,
    }
    if "f32" in legs and best != "f32":
        res["speedup_vs_fp32"] = head["value"] / legs["f32"]["value"]
    if others is not None:
        res["other_workloads"] = others
    if alg12 is not None:
        res["alg1_vs_alg2"] = alg12
    if compl is not None:
        res["completion"] = compl
    if tqr is not None:
        res["tqr_tpinv"] = tqr
    if base is not None:
        res["cpu_baseline"] = base
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
