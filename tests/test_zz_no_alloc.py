"""The entry point that allocates nothing (tsvd_rbk_noalloc: static device
scratch) against tsvd_rbk with a caller workspace, through the C ABI: two
calls in a row, the second on a smaller input, in FP64 and FP32; results
bit for bit equal (same kernels, same inputs).  Sizes beyond the scratch are
rejected before anything is enqueued."""
import numpy as np
import pytest
import torch

from paper_2504_04989_amd import inputs
from tests.gpu_util import load_api, dev

pytestmark = pytest.mark.gpu
api = load_api()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_matches_workspace_entry_point(prec):
    dt = torch.float64 if prec == "f64" else torch.float32
    cases = [((64, 64, 16), 5, 10, 2, 0), ((40, 36, 8), 3, 4, 2, 9)]   # the second is smaller
    for (n1, n2, n3), k, b, q, seed in cases:
        print(f"[noalloc] {prec} {n1}x{n2}x{n3} k={k} b={b} q={q} seed={seed}", flush=True)
        A = dev(inputs.lowrank_tensor(n1, n2, n3, 10, ("geom", 0.8), 1e-3, seed=n1 + seed), dt)
        assert api.workspace_bytes(n1, n2, n3, k, b, q, prec, "rbk") <= api.NOALLOC_SCRATCH_BYTES
        U0, S0, V0 = api.tsvd_rbk(A, seed, k, b, q, prec)
        U1, S1, V1 = api.tsvd_rbk_noalloc(A, seed, k, b, q, prec)
        torch.cuda.synchronize()
        for x, y in ((U0, U1), (S0, S1), (V0, V1)):
            assert torch.equal(x, y)
            assert bool(torch.isfinite(y).all())


def test_noalloc_rejects_sizes_beyond_the_scratch():
    n1, n2, n3 = 1024, 1024, 16
    assert api.workspace_bytes(n1, n2, n3, 10, 20, 1, "f32", "rbk") > api.NOALLOC_SCRATCH_BYTES
    A = torch.zeros((n1, n2, n3), dtype=torch.float32, device="cuda")
    with pytest.raises(api.TsvdError) as e:
        api.tsvd_rbk_noalloc(A, 1, 10, 20, 1, "f32")
    assert e.value.code == api.TSVD_ENOMEM and "scratch" in str(e.value)
    torch.cuda.synchronize()
