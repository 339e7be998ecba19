"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/*.h, sizes workspaces and rejects bad arguments on the
host before anything is enqueued."""
import ctypes
import math
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2504_04989_amd", "lib", "libtsvd_rbk.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s+\*?\s*(tsvd_[a-z0-9_]+)\s*\(", src,
                             flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(LIB)
    names = _declared()
    assert "tsvd_rbk" in names and "tsvd_proj_backward" in names and "tsvd_diag_zgemm" in names
    for n in names:
        assert hasattr(lib, n), n


def test_binding_loads_and_names_match():
    from paper_2504_04989_amd import api
    for n in api.EXPORTS:
        assert hasattr(api.lib, n)
    assert api.lib.tsvd_version() >= 100


def test_workspace_sizes():
    from paper_2504_04989_amd import api
    ws = api.workspace_bytes(1000, 1000, 32, 50, 60, 2, "f32", "rbk")
    F = 17
    # at least the half spectrum of A plus Q and T = C^H
    assert ws >= F * 1000 * 1000 * 8 + 2 * F * 1000 * 180 * 8
    assert ws % 256 == 0
    assert api.workspace_bytes(64, 64, 16, 5, 10, 2, "f64", "rbk") > 0
    assert api.workspace_bytes(1000, 1000, 32, 50, 60, 2, "f32", "approx") >= ws


@pytest.mark.parametrize("args", [
    (0, 10, 4, 2, 3, 1),      # empty
    (10, 10, 4, 4, 3, 1),     # k > b
    (10, 10, 4, 2, 4, 2),     # m = 12 > 10
    (10, 10, 4, 2, 3, -1),    # q < 0
    (40, 40, 5000, 2, 3, 1),  # n3 too large
])
def test_invalid_sizes_rejected(args):
    from paper_2504_04989_amd import api
    assert api.workspace_bytes(*args, "f32", "rbk") == 0
    assert api.lib.tsvd_last_error().decode() != ""


def test_entry_points_reject_bad_pointers_without_touching_the_gpu():
    from paper_2504_04989_amd import api
    L = api.lib
    nul = ctypes.c_void_p(0)
    r = L.tsvd_rbk_omega(nul, nul, 10, 10, 4, 2, 3, 1, 1, nul, nul, nul, nul, 0, nul)
    assert r == api.TSVD_EINVAL
    r = L.tsvd_rbk_omega(nul, nul, 10, 10, 4, 5, 3, 1, 1, nul, nul, nul, nul, 0, nul)   # k > b
    assert r == api.TSVD_EINVAL and "k <= b" in L.tsvd_last_error().decode()
    r = L.tsvd_proj_omega(nul, nul, 10, 10, 4, 3, 1, 7, nul, nul, 0, nul)               # bad precision
    assert r == api.TSVD_EINVAL
    # aligned fake pointers but a workspace that is too small -> ENOMEM, nothing launched
    fake = ctypes.c_void_p(1 << 20)
    r = L.tsvd_rbk_omega(fake, fake, 10, 10, 4, 2, 3, 1, 1, fake, fake, fake, fake, 16, nul)
    assert r == api.TSVD_ENOMEM
    r = L.tsvd_diag_zgemm(nul, 0, nul, 0, nul, 4, 4, 4, 1, 1.0, 0.0, 1, nul)
    assert r == api.TSVD_EINVAL


def test_power_method_sizes_and_rejections():
    # Alg. 1 keeps m = b basis columns whatever q is: b (q + 1) > min(n1, n2)
    # is accepted, b > min(n1, n2) is not.
    from paper_2504_04989_amd import api
    assert api.workspace_bytes(10, 10, 4, 2, 4, 5, "f32", "power") > 0
    assert api.workspace_bytes(10, 10, 4, 2, 4, 5, "f32", "rbk") == 0
    assert api.workspace_bytes(10, 10, 4, 2, 11, 1, "f32", "power") == 0
    assert api.workspace_bytes(10, 10, 4, 5, 4, 1, "f32", "power") == 0          # k > b
    ws = api.workspace_bytes(256, 256, 256, 45, 50, 2, "f64", "power")
    assert 0 < ws < api.workspace_bytes(256, 256, 256, 45, 50, 2, "f64", "rbk")
    assert api.workspace_bytes(256, 256, 256, 45, 50, 2, "f64", "power_approx") > ws
    L = api.lib
    nul = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(1 << 20)
    assert L.tsvd_power_omega(nul, nul, 10, 10, 4, 2, 3, 1, 1, nul, nul, nul, nul, 0, nul) == api.TSVD_EINVAL
    r = L.tsvd_power_approx_omega(fake, fake, 10, 10, 4, 2, 3, 1, 1, fake, fake, fake, fake, fake, 16, nul)
    assert r == api.TSVD_ENOMEM
    r = L.tsvd_power_omega(fake, fake, 10, 10, 4, 2, 3, 5000, 1, fake, fake, fake, fake, 1 << 30, nul)   # q too large
    assert r == api.TSVD_EINVAL


def test_tensor_ops_sizes_and_rejections():
    from paper_2504_04989_amd import api
    assert api.workspace_bytes(30, 20, 8, 0, 0, 0, "f32", "tqr") > 0
    assert api.workspace_bytes(20, 30, 8, 0, 0, 0, "f64", "tqr") > 0          # wide: r = n1
    assert api.workspace_bytes(30, 20, 8, 0, 0, 0, "f64", "tpinv") > 0
    assert api.workspace_bytes(20, 30, 8, 0, 0, 0, "f64", "tpinv") > 0         # wide: Gram A A^H
    assert api.workspace_bytes(2000, 1100, 4, 0, 0, 0, "f32", "tpinv") == 0   # min(n1, n2) > 1024
    assert api.workspace_bytes(30, 20, 8, 0, 0, 0, "bf16", "tpinv") == 0
    assert api.workspace_bytes(30, 20, 8, 0, 0, 0, "bf16x3", "tqr") == 0      # FP64 / FP32 only
    assert api.workspace_bytes(2000, 1100, 4, 0, 0, 0, "f32", "tqr") == 0     # min(n1, n2) > 1024
    L = api.lib
    nul = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(1 << 20)
    assert L.tsvd_tqr(nul, 10, 8, 4, 1, nul, nul, nul, 0, nul) == api.TSVD_EINVAL
    assert L.tsvd_tqr(fake, 10, 8, 4, 1, fake, fake, fake, 16, nul) == api.TSVD_ENOMEM
    # rtol below 4 sqrt((n1 + n2) 2^-53), NaN rtol, null pointers
    assert L.tsvd_tpinv(fake, 8, 10, 4, 1e-12, 1, fake, fake, 1 << 30, nul) == api.TSVD_EINVAL
    assert "resolution" in api.lib.tsvd_last_error().decode()
    assert L.tsvd_tpinv(fake, 8, 10, 4, float("nan"), 1, fake, fake, 1 << 30, nul) == api.TSVD_EINVAL
    assert L.tsvd_tpinv(nul, 8, 10, 4, 0.0, 1, fake, fake, 1 << 30, nul) == api.TSVD_EINVAL
    assert L.tsvd_tpinv(fake, 8, 10, 4, 0.0, 1, fake, fake, 16, nul) == api.TSVD_ENOMEM


def test_tpinv_default_rtol():
    # max(max(n1, n2) eps, 4 sqrt((n1 + n2) 2^-53)), eps of the data type
    from paper_2504_04989_amd import api
    floor = lambda n1, n2: 4.0 * math.sqrt((n1 + n2) * 2.0 ** -53)
    assert api.tpinv_default_rtol(4096, 256, "f32") == 4096 * 2.0 ** -23
    assert api.tpinv_default_rtol(90, 60, "f64") == floor(90, 60)
    assert api.tpinv_default_rtol(3, 2, "f32") == max(3 * 2.0 ** -23, floor(3, 2))
    assert api.tpinv_default_rtol(0, 2, "f32") == -1.0
    assert api.tpinv_default_rtol(5, 2, "bf16") == -1.0


def test_completion_sizes_and_rejections():
    from paper_2504_04989_amd import api
    w2 = api.workspace_bytes(64, 96, 3, 5, 8, 2, "f32", "complete2")
    w1 = api.workspace_bytes(64, 96, 3, 5, 8, 2, "f32", "complete1")
    assert w2 > api.workspace_bytes(64, 96, 3, 5, 8, 2, "f32", "approx") and w1 > 0
    L = api.lib
    nul = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(1 << 20)
    args = (fake, fake, fake, 64, 96, 3, 5, 8, 2)
    assert L.tsvd_complete_omega(*args, 10, 3, 1, fake, fake, 1 << 40, nul) == api.TSVD_EINVAL      # bad alg
    assert L.tsvd_complete_omega(*args, -1, 2, 1, fake, fake, 1 << 40, nul) == api.TSVD_EINVAL      # iters < 0
    assert L.tsvd_complete_omega(*args, 10, 2, 1, fake, fake, 16, nul) == api.TSVD_ENOMEM
    assert L.tsvd_complete_omega(fake, nul, fake, 64, 96, 3, 5, 8, 2, 10, 2, 1, fake, fake, 1 << 40, nul) == api.TSVD_EINVAL


def test_literal_sizes_and_rejections():
    from paper_2504_04989_amd import api
    w = api.workspace_bytes(64, 64, 16, 5, 10, 2, "f64", "literal")
    assert w == api.workspace_bytes(64, 64, 16, 5, 10, 2, "f64", "approx") > 0
    L = api.lib
    nul = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(1 << 20)
    assert L.tsvd_rbk_literal_omega(fake, fake, 10, 10, 4, 2, 4, 2, 1, fake, fake, fake, nul, fake, 1 << 30, nul) \
        == api.TSVD_EINVAL                                                   # m = 12 > 10
    assert L.tsvd_rbk_literal_omega(fake, fake, 10, 10, 4, 2, 3, 1, 1, fake, fake, fake, nul, fake, 16, nul) \
        == api.TSVD_ENOMEM


def test_seed_entry_points_reject_bad_arguments_on_the_host():
    # the seed-taking forms validate like their _omega twins, before any launch
    from paper_2504_04989_amd import api
    L = api.lib
    nul = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(1 << 20)
    assert L.tsvd_rbk(nul, 10, 10, 4, 2, 3, 1, 7, 1, nul, nul, nul, nul, 0, nul) == api.TSVD_EINVAL
    assert L.tsvd_rbk(fake, 10, 10, 4, 2, 3, 1, 7, 1, fake, fake, fake, fake, 16, nul) == api.TSVD_ENOMEM
    assert L.tsvd_rbk_approx(fake, 10, 10, 4, 2, 3, 1, 7, 1, fake, fake, fake, nul, fake, 1 << 30, nul) \
        == api.TSVD_EINVAL                                                   # Xhat missing
    assert L.tsvd_proj(fake, 10, 10, 4, 3, 1, 7, 9, fake, fake, 1 << 30, nul) == api.TSVD_EINVAL   # bad precision
    assert L.tsvd_proj_backward(fake, nul, 10, 10, 4, 3, 1, 7, 1, fake, fake, 1 << 30, nul) == api.TSVD_EINVAL
    assert L.tsvd_complete(fake, fake, 64, 96, 3, 5, 8, 2, 7, 10, 3, 1, fake, fake, 1 << 40, nul) == api.TSVD_EINVAL
    assert L.tsvd_power(fake, 10, 10, 4, 2, 11, 1, 7, 1, fake, fake, fake, fake, 1 << 30, nul) == api.TSVD_EINVAL
    # the _omega twins need the tensor
    assert L.tsvd_rbk_omega(fake, nul, 10, 10, 4, 2, 3, 1, 1, fake, fake, fake, fake, 1 << 30, nul) \
        == api.TSVD_EINVAL
    assert "Omega" in L.tsvd_last_error().decode()


def test_seeded_omega_on_the_host_matches_the_input_generator():
    # tsvd_omega (the library's host copy of the generator the seed-taking
    # entry points run on the device) against the independent numpy
    # implementation of the same Philox4x32-10 / Box-Muller stream, bit for bit
    import numpy as np
    from paper_2504_04989_amd import api, inputs
    for shape, seed in (((7, 3, 5), 0), ((64, 10, 16), 0), ((33, 4, 9), 2**40 + 17), ((1, 1, 1), 5)):
        a = api.omega(*shape, seed)
        b = inputs.omega(*shape, seed)
        assert a.dtype == np.float64 and np.array_equal(a, b), (shape, seed)
    assert api.lib.tsvd_omega(0, 3, 4, 1, ctypes.c_void_p(1 << 20)) == api.TSVD_EINVAL
    assert api.lib.tsvd_omega(3, 3, 4, 1, ctypes.c_void_p(0)) == api.TSVD_EINVAL
    assert api.lib.tsvd_omega(1 << 20, 1 << 20, 2, 1, ctypes.c_void_p(1 << 20)) == api.TSVD_EINVAL   # > 2^40
