"""The seed-taking boundary on the GPU: the test tensor drawn on the device
equals the host stream bit for bit, the seed-taking entry points match the
FP64 oracle fed the independently generated stream, numerical events reach
tsvd_read_info, and the binding rejects mis-shaped tensors before any launch."""
import numpy as np
import pytest
import torch

from oracle import tsvd_oracle as O
from paper_2504_04989_amd import inputs
from tests.gpu_util import load_api, dev, host, rel_f

pytestmark = pytest.mark.gpu
api = load_api()


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (12345, 7), (1 << 20, 2**40 + 3), (4096 * 110 * 64, 4)])
def test_device_omega_equals_host_bitwise(n, seed):
    print(f"[seed] device Omega n={n} seed={seed}", flush=True)
    d64 = host(api.diag_omega(n, seed, torch.float64))
    h = api.omega(1, 1, n, seed).ravel()
    assert np.array_equal(d64, h)
    assert np.array_equal(d64, inputs.omega_counter(n, seed))
    d32 = host(api.diag_omega(n, seed, torch.float32))
    assert np.array_equal(d32, h.astype(np.float32))


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_seed_call_matches_oracle_and_omega_call(prec, tol):
    A, _, c = inputs.make_config("c1_fp64_64x64x16")
    k, b, q, seed = c["k"], c["b"], c["q"], c["seed"]
    dt = torch.float64 if prec == "f64" else torch.float32
    At = dev(A, dt)
    print(f"[seed] c1 {prec} seed={seed}", flush=True)
    U, S, V, X = api.tsvd_rbk_approx(At, seed, k, b, q, prec)
    Om = inputs.omega(64, b, 16, seed)
    Ain = A if prec == "f64" else A.astype(np.float32).astype(np.float64)
    Oin = Om if prec == "f64" else Om.astype(np.float32).astype(np.float64)
    Xo = O.rbk_approx(Ain, Oin, k, b, q)
    e = rel_f(host(X).astype(np.float64), Xo)
    print(f"[seed] X rel err vs oracle {e:.2e}", flush=True)
    assert e <= tol
    # the same bits as the call with the host-generated tensor
    U2, S2, V2, X2 = api.tsvd_rbk_approx(At, dev(Om, dt), k, b, q, prec)
    for a_, b_ in ((U, U2), (S, S2), (V, V2), (X, X2)):
        assert torch.equal(a_, b_)
    # the other seed-taking forms against their _omega twins
    Ut = api.tsvd_rbk(At, seed, k, b, q, prec)[0]
    assert torch.equal(Ut, U)
    P1 = api.tsvd_proj(At, seed, b, q, prec)
    P2 = api.tsvd_proj(At, dev(Om, dt), b, q, prec)
    assert torch.equal(P1, P2)
    G = dev(inputs.random_tensor(A.shape, 8), dt)
    assert torch.equal(api.tsvd_proj_backward(At, seed, G, b, q, prec),
                       api.tsvd_proj_backward(At, dev(Om, dt), G, b, q, prec))
    assert torch.equal(api.tsvd_power_approx(At, seed, k, b, q, prec)[3],
                       api.tsvd_power_approx(At, dev(Om, dt), k, b, q, prec)[3])
    assert torch.equal(api.tsvd_rbk_literal(At, seed, k, b, q, prec)[3],
                       api.tsvd_rbk_literal(At, dev(Om, dt), k, b, q, prec)[3])
    mask = torch.rand(A.shape, device="cuda") < 0.5
    assert torch.equal(api.tsvd_complete(At, mask, seed, k, b, q, 2, 2, prec),
                       api.tsvd_complete(At, mask, dev(Om, dt), k, b, q, 2, 2, prec))


def test_read_info_reports_numerical_failures():
    # counters written into a real workspace by the host, then read back:
    # TSVD_ENUMERIC for a breakdown, an unconverged eigenvector, a
    # non-finite value or a tie at the rank-k cut, TSVD_OK for a shift that
    # carried a pivot
    ws = api.workspace(64, 64, 16, 5, 10, 2, "f64", "rbk", "cuda")
    for counters, want in (([0, 0, 0, 0, 0], api.TSVD_OK), ([5, 0, 0, 0, 0], api.TSVD_OK),
                           ([0, 1, 0, 0, 0], api.TSVD_ENUMERIC), ([0, 0, 2, 0, 0], api.TSVD_ENUMERIC),
                           ([0, 0, 0, 3, 0], api.TSVD_ENUMERIC), ([0, 0, 0, 0, 1], api.TSVD_ENUMERIC)):
        pad = [0] * (api.INFO_COUNT - len(counters))
        ws[:32].view(torch.int32).copy_(torch.tensor(counters + pad, dtype=torch.int32))
        info = api.read_info(ws)
        assert info["status"] == want, (counters, info)
        assert [info[n] for n in api.INFO_NAMES] == counters


def test_exact_rank_input_takes_the_shifted_factorisation():
    # noiseless tubal rank 4 with b (q + 1) = 18 basis columns: the Krylov
    # blocks are numerically rank deficient, the shift carries their pivots
    # (counted), nothing breaks down and the tensor is recovered
    A = inputs.exact_lowrank_tensor(60, 50, 6, 4, seed=5)
    ws = api.workspace(60, 50, 6, 4, 6, 2, "f64", "approx", "cuda")
    U, S, V, X = api.tsvd_rbk_approx(dev(A), 5, 4, 6, 2, "f64", ws=ws)
    info = api.read_info(ws)
    print(f"[seed] exact rank: info {info}", flush=True)
    assert info["status"] == api.TSVD_OK
    assert info["chol_shifted"] > 0 and info["chol_breakdown"] == 0
    assert rel_f(host(X), A) <= 1e-10


def test_binding_rejects_misshaped_tensors_before_launch():
    A = torch.zeros((12, 10, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        api.tsvd_proj(A, torch.zeros((10, 3, 5), dtype=torch.float64, device="cuda"), 3, 1)
    with pytest.raises(ValueError):
        api.tsvd_proj_backward(A, 3, torch.zeros((12, 10, 5), dtype=torch.float64, device="cuda"), 3, 1)
    with pytest.raises(ValueError):
        api.tsvd_proj_backward(A, torch.zeros((10, 4, 4), dtype=torch.float64, device="cuda"),
                               torch.zeros_like(A), 3, 1)
    with pytest.raises(ValueError):
        api.TProject.apply(A, torch.zeros((9, 3, 4), dtype=torch.float64, device="cuda"), 3, 1)
    with pytest.raises(ValueError):
        api.tsvd_rbk(A, torch.zeros((10, 3, 4), dtype=torch.float32, device="cuda"), 2, 3, 1)
    torch.cuda.synchronize()
