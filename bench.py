#!/usr/bin/env python
"""Throughput of the randomized block Krylov truncated T-SVD (Alg. 2) on one
MI355X: truncated T-SVDs per second with the input resident in HBM.

One step = one call of tsvd_rbk on the whole tensor (mode-3 DFT, Krylov
products, orthonormalisation, small SVD, lift, inverse DFT), seeded
synthetic input of the stated shape.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_work(cls: str, c: dict, prec: str):
    """Algorithmic work per launch of a kernel class: (amount, unit, bound, peak)."""
    n1, n2, n3, k, b, q = c["n1"], c["n2"], c["n3"], c["k"], c["b"], c["q"]
    F = n3 // 2 + 1
    m = b * (q + 1)
    es = 8 if prec == "f64" else 4
    if cls == "gemm_krylov":   # one pass over A_f for all slices, b right-hand columns
        return 8.0 * n1 * n2 * b * F / 1e12, "TFLOP/s", "mfma", PEAK["mfma_tflops"][prec]
    if cls == "fft_A":         # read the real tensor, write the half spectrum
        return (es * n1 * n2 * n3 + 2 * es * n1 * n2 * F) / 1e9, "GB/s", "hbm", PEAK["hbm_gbs"]
    if cls == "heig_tri":      # Householder tridiagonalisation of the m x m Hermitian G_f, FP64
        return F * (16.0 / 3.0 * m ** 3) / 1e12, "TFLOP/s", "alu", PEAK["valu_tflops"]["f64"]
    if cls == "chol":          # b x b complex Cholesky + triangular inverse, FP64, per slice
        return F * (16.0 / 3.0 * b ** 3) / 1e12, "TFLOP/s", "alu", PEAK["valu_tflops"]["f64"]
    return None   # classes whose launches differ in shape carry no per-launch figure


def cpu_baseline(A, Om, c, U, S, V, nslices):
    """The FP64 oracle on a bounded sample: the full mode-3 DFT of the input
    plus `nslices` Fourier slices of Alg. 2, extrapolated to all slices."""
    from oracle import tsvd_oracle as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    n1, n2, n3 = A.shape
    F = n3 // 2 + 1
    t0 = time.perf_counter()
    O.dft_mode3(A, range(F))
    t_dft = time.perf_counter() - t0
    freqs = sorted(set([0, F - 1] + list(np.linspace(0, F - 1, nslices).astype(int))))[:nslices]
    t0 = time.perf_counter()
    sl = O.rbk_slices(A, Om, c["k"], c["b"], c["q"], freqs=freqs)
    t_sl = (time.perf_counter() - t0) / len(freqs)
    t_job = t_dft + F * t_sl
    # parity spot check of the benchmarked output on the sampled slices
    Ub = np.fft.fft(U, axis=2)[:, :, freqs]
    Vb = np.fft.fft(V, axis=2)[:, :, freqs]
    Sb = np.fft.fft(S, axis=1)[:, freqs].real
    errs = []
    for i in range(len(freqs)):
        Xg = (Ub[:, :, i] * Sb[:, i]) @ Vb[:, :, i].conj().T
        Xo = (sl["Uf"][:, :, i] * sl["Sf"][:, i]) @ sl["Vf"][:, :, i].conj().T
        errs.append(float(np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo)))
    base = {"value": 1.0 / t_job, "unit": "T-SVD/s", "cores": int(cores), "kind": "oracle",
            "sample": f"full mode-3 DFT ({t_dft:.2f} s) + {len(freqs)} of {F} Fourier slices "
                      f"({t_sl:.2f} s each), extrapolated to {F} slices: {t_job:.1f} s per T-SVD"}
    return base, {"slices": freqs, "max_rel_err_xhat": max(errs)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2_fp32_1000x1000x32")
    ap.add_argument("--prec", default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-slices", type=int, default=2)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB 5 times (HBM counter calibration)")
    args = ap.parse_args()
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
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU (one Fourier-slice batch per device); "
                                   "multi-GPU frequency sharding is not built", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2504_04989_amd import api, inputs

    A64, Om64, c = inputs.make_config(args.workload)
    prec = args.prec or c["prec"]
    if prec not in ("f32", "f64"):
        prec = "f32"
    dt = torch.float64 if prec == "f64" else torch.float32
    npdt = np.float64 if prec == "f64" else np.float32
    A_h, Om_h = A64.astype(npdt), Om64.astype(npdt)
    A = torch.from_numpy(A_h).to("cuda")
    Om = torch.from_numpy(Om_h).to("cuda")
    n1, n2, n3 = A.shape
    k, b, q = c["k"], c["b"], c["q"]
    ws = api.workspace(n1, n2, n3, k, b, q, prec, "rbk", "cuda")
    out = (torch.empty((n1, k, n3), dtype=dt, device="cuda"), torch.empty((k, n3), dtype=dt, device="cuda"),
           torch.empty((n2, k, n3), dtype=dt, device="cuda"))
    log(f"[bench] workload {args.workload} {n1}x{n2}x{n3} k={k} b={b} q={q} prec={prec} "
        f"workspace {ws.numel() / 2**20:.1f} MiB")
    for _ in range(args.warmup):
        api.tsvd_rbk(A, Om, k, b, q, prec, ws=ws, out=out)
    torch.cuda.synchronize()
    log("[bench] warmup done")

    api.diag_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        api.tsvd_rbk(A, Om, k, b, q, prec, ws=ws, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timing = api.diag_timing_read()
    api.diag_timing(False)
    info = api.read_info(ws)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    log(f"[bench] {ms_per_step:.3f} ms/step; info {info}")

    kernels = {}
    for cls, (ms, cnt) in timing.items():
        if cnt:
            kernels[cls] = {"ms_per_step": ms / args.steps, "launches_per_step": cnt / args.steps,
                            "avg_launch_ms": ms / cnt}
    for cls, v in sorted(kernels.items(), key=lambda kv: -kv[1]["ms_per_step"]):
        log(f"[bench]   {cls:12s} {v['ms_per_step']:.3f} ms/step  {v['launches_per_step']:.0f} launches  "
            f"{v['avg_launch_ms'] * 1e3:.1f} us/launch")
    # roofline of the dominant kernel class that has a stated algorithmic work
    roof = None
    for cls, v in sorted(kernels.items(), key=lambda kv: -kv[1]["ms_per_step"]):
        w = kernel_work(cls, c, prec)
        if w is None:
            continue
        amount, unit, bound, peak = w
        achieved = amount / (v["avg_launch_ms"] * 1e-3)
        roof = {"kernel": cls, "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                "frac": achieved / peak, "traffic": None}
        break
    kry = kernels.get("gemm_krylov")
    mfma_util = None
    if kry:
        amount, _, _, peak = kernel_work("gemm_krylov", c, prec)
        mfma_util = amount / (kry["avg_launch_ms"] * 1e-3) / peak

    res = {
        "metric": "truncated T-SVDs/s at rel-err<=1e-4 vs the FP64 oracle",
        "value": 1e3 / ms_per_step,
        "unit": "T-SVD/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {"workload": args.workload, "n1": n1, "n2": n2, "n3": n3, "k": k, "b": b, "q": q,
                   "precision": prec},
        "roofline": roof,
        "krylov_gemm_mfma_frac": mfma_util,
        "kernels": kernels,
        "numeric_info": info,
    }
    if not args.no_cpu_baseline:
        U, S, V = (t.cpu().numpy().astype(np.float64) for t in out)
        log("[bench] cpu baseline: oracle on sampled slices")
        base, par = cpu_baseline(A_h.astype(np.float64), Om_h.astype(np.float64), c, U, S, V, args.cpu_slices)
        res["cpu_baseline"] = base
        res["parity_sample"] = par
        log(f"[bench] cpu baseline {base['value']:.4g} T-SVD/s; parity {par}")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
