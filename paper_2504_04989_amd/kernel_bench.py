"""Kernel-level timing of the library's hot kernels at a workload's shapes,
through the kernel entry points of the C ABI (include/tsvd_rbk_diag.h), on
data drawn on the device (no host generation, so a profiler pass is short).

    python -m paper_2504_04989_amd.kernel_bench krylov [--prec f32|bf16|bf16x3|bf16x3s] [--n 4096] [--f 33] [--N 110]
    python -m paper_2504_04989_amd.kernel_bench fft [--n 4096] [--n3 64]
    python -m paper_2504_04989_amd.kernel_bench orth [--n 4096] [--m 440] [--n3 64]

krylov: the Krylov products of Alg. 2, C_f = A_f X_f and C_f = A_f^H Y_f,
over f slices of an n x n complex FP32 A_f and N thin columns (the
4096 x 4096 x 64 workload: n = 4096, 33 slices, N = b = 110), each direction
timed over --reps launches after one warmup, with HIP events; prints the
time per launch and the rate in algorithmic flops (8 n^2 N f per launch).
bf16x3s: the BF16x3 form on A already split into (hi, lo) bf16 pairs, as
the split transform writes it for the Krylov basis (the thin operand is split
once per launch inside the timed call).
fft: the mode-3 real-to-half-spectrum DFT of n^2 real tubes of length n3
(FP32), timed likewise, with its algorithmic bytes (4 n^2 n3 + 8 n^2 F).
orth: the T-QR (Alg. TQR) of an n x m x n3 FP32 tensor, m = 440 orthonormalised
in four 110-column panels: the same orthonormalisation launches (block
Gram-Schmidt projections, shifted CholeskyQR, FP64 Grams and factors) as the
Krylov basis of the 4096 x 4096 x 64 workload (b = 110, q = 3), without the
small eigensolver.
Prints one JSON line per measurement.
"""
from __future__ import annotations

import argparse
import json

import torch

from . import api


def _time(fn, reps: int):
    fn()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


def krylov(n: int, F: int, N: int, prec: str, reps: int):
    g = torch.Generator(device="cuda").manual_seed(1)
    A = torch.randn((F, n, n), dtype=torch.complex64, device="cuda", generator=g)
    X = torch.randn((F, n, N), dtype=torch.complex64, device="cuda", generator=g)
    if prec == "bf16x3s":
        # the big operand as written by the split transform: (hi, lo) bf16 pairs
        A = api.diag_split_bf16x3(A)
    for herm in (False, True):
        ms = _time(lambda: api.diag_kgemm(A, X, herm=herm, mode=prec), reps)
        fl = 8.0 * n * n * N * F
        peak = {"f32": 157.3e12, "bf16": 2500e12, "bf16x3": 2500e12, "bf16x3s": 2500e12}[prec]
        ex = 3.0 if prec in ("bf16x3", "bf16x3s") else 1.0
        print(json.dumps({"kernel": "krylov", "op": "A^H Y" if herm else "A X", "prec": prec, "n": n, "slices": F,
                          "N": N, "ms_per_launch": ms, "tflops_algorithmic": fl / ms / 1e9,
                          "frac_algorithmic": fl / ms / 1e-3 / peak, "frac_executed": ex * fl / ms / 1e-3 / peak,
                          "GBs_operand": 8.0 * n * n * F / ms / 1e6}), flush=True)


def fft(n: int, n3: int, reps: int):
    X = torch.randn((n * n, n3), dtype=torch.float32, device="cuda")
    ms = _time(lambda: api.diag_fft_r2c(X), reps)
    F = n3 // 2 + 1
    gb = (4.0 * n * n * n3 + 8.0 * n * n * F) / 1e9
    print(json.dumps({"kernel": "fft_r2c", "n_tubes": n * n, "n3": n3, "ms_per_launch": ms, "GBs": gb / ms * 1e3,
                      "frac_hbm": gb / ms * 1e3 / 8000.0}), flush=True)


def orth(n: int, m: int, n3: int, reps: int):
    A = torch.randn((n, m, n3), dtype=torch.float32, device="cuda")
    ws = api.workspace(n, m, n3, 0, 0, 0, "f32", "tqr", "cuda")
    ms = _time(lambda: api.tsvd_tqr(A, "f32", ws=ws), reps)
    print(json.dumps({"kernel": "tqr", "n1": n, "n2": m, "n3": n3, "ms_per_call": ms}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["krylov", "fft", "orth"])
    ap.add_argument("--prec", default="bf16x3")
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--f", type=int, default=33)
    ap.add_argument("--N", type=int, default=110)
    ap.add_argument("--n3", type=int, default=64)
    ap.add_argument("--m", type=int, default=440)
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args()
    if a.what == "krylov":
        krylov(a.n, a.f, a.N, a.prec, a.reps)
    elif a.what == "orth":
        orth(a.n, a.m, a.n3, a.reps)
    else:
        fft(a.n, a.n3, a.reps)


if __name__ == "__main__":
    main()
