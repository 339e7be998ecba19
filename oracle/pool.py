"""Run the FP64 oracle's per-slice Alg. 2 on several Fourier slices in
parallel worker processes.

TEST INFRASTRUCTURE ONLY, like the rest of this package: used by ``tests/``
and by the ``cpu_baseline`` leg of ``bench.py``.  It adds no arithmetic: the
mode-3 DFT is ``dft_mode3`` at the requested frequencies and every slice is
``rbk_slice`` (the body of ``rbk_slices``) run unchanged in a worker.  Workers
are forked from the caller, which must not have initialised a GPU runtime;
each gets an equal share of the BLAS threads.
"""
from __future__ import annotations

import multiprocessing as mp
import os
import time

import numpy as np

from . import tsvd_oracle as O

_JOB: dict = {}


def _limit_threads(n: int):
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(limits=n)
    except Exception:  # pragma: no cover - threadpoolctl missing
        pass


def _work(i: int):
    Ab, Ob, k, b, q, extra = (_JOB[key] for key in ("Ab", "Ob", "k", "b", "q", "extra"))
    _limit_threads(_JOB["threads"])
    t0 = time.perf_counter()
    r = O.rbk_slice(Ab[:, :, i], Ob[:, :, i], k, b, q)
    sec = time.perf_counter() - t0
    out = {"Uf": r["Uf"], "Vf": r["Vf"], "Sf": r["Sf"], "s_all": r["s_all"], "seconds": sec}
    if extra is not None:
        out["extra"] = extra(Ab[:, :, i], Ob[:, :, i], k, b, q)
    return i, out


class SlicePool:
    """Start the oracle on `freqs` (DFT in the caller, one slice per task in
    `workers` forked processes); .get() waits and returns a dict of per-slice
    arrays indexed like freqs (Uf (n1,k,nf), Sf (k,nf), Vf (n2,k,nf), s_all
    (m,nf)), the per-slice seconds, the wall time and the thread count, plus
    "extra" (a list) when an extra per-slice function was given."""

    def __init__(self, A, Om, k, b, q, freqs, workers=None, threads=None, extra=None):
        ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        self.freqs = list(freqs)
        self.workers = max(1, min(workers or ncpu, len(self.freqs)))
        self.threads = max(1, threads or ncpu // self.workers)
        self.t0 = time.perf_counter()
        _JOB.update(Ab=O.dft_mode3(A, self.freqs), Ob=O.dft_mode3(Om, self.freqs), k=k, b=b, q=q, extra=extra,
                    threads=self.threads)
        self.dft_seconds = time.perf_counter() - self.t0
        self.shape = (A.shape[0], A.shape[1], k, b * (q + 1))
        self.pool = mp.get_context("fork").Pool(self.workers)
        self.res = self.pool.imap_unordered(_work, range(len(self.freqs)))

    def get(self, progress=None):
        """Wait for every slice; progress(message) is called as each ends."""
        rows = []
        for i, r in self.res:
            rows.append((i, r))
            if progress is not None:
                progress(f"oracle slice f={self.freqs[i]} done in {r['seconds']:.1f} s "
                         f"({len(rows)}/{len(self.freqs)}, {time.perf_counter() - self.t0:.0f} s since start)")
        self.pool.close()
        self.pool.join()
        _JOB.clear()
        n1, n2, k, m = self.shape
        nf = len(self.freqs)
        out = {"freqs": self.freqs, "Uf": np.zeros((n1, k, nf), complex), "Sf": np.zeros((k, nf)),
               "Vf": np.zeros((n2, k, nf), complex), "s_all": np.zeros((m, nf)), "seconds": [0.0] * nf,
               "wall": time.perf_counter() - self.t0, "dft_seconds": self.dft_seconds,
               "workers": self.workers, "threads": self.workers * self.threads}
        extra = [None] * nf
        for i, r in rows:
            out["Uf"][:, :, i], out["Vf"][:, :, i] = r["Uf"], r["Vf"]
            out["Sf"][:, i], out["s_all"][:, i] = r["Sf"], r["s_all"]
            out["seconds"][i] = r["seconds"]
            extra[i] = r.get("extra")
        if any(e is not None for e in extra):
            out["extra"] = extra
        return out
