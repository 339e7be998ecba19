"""Oracle slices of a full-size workload, computed once in a child process
and cached on disk for the GPU tests that sample it.

    python -m tests.oracle_slices WORKLOAD F1,F2,... OUT.npz

The child generates the workload (FP32-rounded, widened back to FP64, as the
GPU paths read it), runs the FP64 oracle on the listed Fourier slices in
parallel workers (oracle.pool) and, per slice, the plain FP32 computation of
the same slice (tests.gpu_util.fp32_twin_slice_f) that measures the FP32 floor,
and the same with the Krylov products in the three-product BF16 form
(tests.gpu_util.bf16x3_twin_slice_f), the floor of the BF16x3 mode.
It runs in its own process because the pool forks workers, which a test
process that has already initialised the GPU must not do."""
import hashlib
import os
import subprocess
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _twin(Af, Of, k, b, q):
    from tests.gpu_util import bf16x3_twin_slice_f, fp32_twin_slice_f
    Xt, st = fp32_twin_slice_f(Af, Of, k, b, q)
    Xt3, st3 = bf16x3_twin_slice_f(Af, Of, k, b, q)
    return {"Xt": Xt, "st": st, "Xt3": Xt3, "st3": st3}


def main(argv):
    name, freqs, out = argv[0], [int(x) for x in argv[1].split(",")], argv[2]
    sys.path.insert(0, ROOT)
    from oracle.pool import SlicePool
    from paper_2504_04989_amd import inputs
    t0 = time.perf_counter()
    A, Om, c = inputs.make_config(name)
    A = A.astype(np.float32).astype(np.float64)
    Om = Om.astype(np.float32).astype(np.float64)
    print(f"[oracle_slices] {name} generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    pool = SlicePool(A, Om, c["k"], c["b"], c["q"], freqs, extra=_twin)
    del A
    r = pool.get(progress=lambda msg: print(f"[oracle_slices] {msg}", file=sys.stderr, flush=True))
    print(f"[oracle_slices] {len(freqs)} slices in {r['wall']:.1f} s ({r['workers']} workers)", file=sys.stderr,
          flush=True)
    ex = r.pop("extra")
    np.savez(out + ".tmp.npz", Uf=r["Uf"], Sf=r["Sf"], Vf=r["Vf"], s_all=r["s_all"], freqs=np.array(freqs),
             Xt=np.stack([e["Xt"] for e in ex], axis=2), st=np.stack([e["st"] for e in ex], axis=1),
             Xt3=np.stack([e["Xt3"] for e in ex], axis=2), st3=np.stack([e["st3"] for e in ex], axis=1))
    os.replace(out + ".tmp.npz", out)


def _key(name, freqs):
    h = hashlib.sha256()
    for rel in ("oracle/tsvd_oracle.py", "oracle/pool.py", "paper_2504_04989_amd/inputs.py", "tests/gpu_util.py"):
        h.update(open(os.path.join(ROOT, rel), "rb").read())
    h.update(f"{name}:{freqs}".encode())
    return h.hexdigest()[:16]


class Pending:
    """The child that computes (or the cache file that holds) the slices."""

    def __init__(self, name, freqs):
        d = os.path.join(tempfile.gettempdir(), "tsvd_oracle_slices")
        os.makedirs(d, exist_ok=True)
        self.path = os.path.join(d, f"{name}_{_key(name, list(freqs))}.npz")
        self.proc = None
        if not os.path.exists(self.path):
            self.proc = subprocess.Popen([sys.executable, "-m", "tests.oracle_slices", name,
                                          ",".join(str(f) for f in freqs), self.path], cwd=ROOT)

    def get(self, timeout=1800):
        if self.proc is not None:
            rc = self.proc.wait(timeout)
            if rc != 0:
                raise RuntimeError(f"oracle slice child failed with status {rc}")
            self.proc = None
        with np.load(self.path) as z:
            return {k: z[k] for k in z.files}


if __name__ == "__main__":
    main(sys.argv[1:])
