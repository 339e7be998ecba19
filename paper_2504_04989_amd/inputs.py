"""Seeded synthetic inputs for the randomized block Krylov T-SVD.

This module only draws random numbers and assembles test tensors; it holds
none of the method's arithmetic and imports neither the library binding nor
the oracle.  Both sides (the HIP library and the FP64 oracle) consume exactly
the arrays produced here.

Workload recipes (real tensors, C-contiguous (n1, n2, n3), tubes contiguous):

  lowrank      A = U * S * V^T (T-product) + noise * N(0, 1).  U (n1 x r x n3) and
               V (n2 x r x n3) i.i.d. N(0, 1); S f-diagonal with diagonal tubes
               S(i, i, :) = c_i g_i, g_i ~ N(0, I_n3), c_i the stated decay
               (i = 1..r).  The T-product is evaluated with numpy's FFT.
  hyperspectral sum of r separable Gaussian-bump spatial maps times smooth
               random spectral curves, min-max scaled to [0, 1], plus noise.
  completion   T = U * V^T of tubal rank r (N(0, 1) factors) and a Bernoulli
               keep-mask; the starting point X0 = M (.) T.
  image        power-law random fields in [0, 255] (n1 x n2 x 3), stand-ins for
               the photographs of Example 3, with Bernoulli or line masks.
  separable    A(i, j, t) = sum_c g_c(i) h_c(j) s_c(t) + noise N(i, j) w(t), all
               factors i.i.d. N(0, 1), s_c scaled by decay^c: drawn as factors
               only, for tensors of more than 2^31 entries that a test
               assembles on the device (separable_factors).
  spectrum     A = U * S * V^T with U, V orthogonal tensors (every Fourier slice
               unitary: numpy's QR of a complex Gaussian matrix, real at the DC
               and Nyquist slices) and S f-diagonal with tubes sigma_m e_1, so
               every Fourier slice of A has exactly the singular values
               sigma_1 >= sigma_2 >= ... (Sec. 5, Example 1: m^-5, m^-6, 0.5^m).

Draw order inside one seed: factors U, then S tubes, then V, then noise, then
the mask.  The Gaussian test tensor Omega (n2 x b x n3) comes from a separate
stream spawned from the same seed, so it does not depend on the data shape.
"""
from __future__ import annotations

import numpy as np

CONFIGS = {
    # name: shape, rank/decay recipe, method parameters, precision, seed
    "c1_fp64_64x64x16": dict(kind="lowrank", n1=64, n2=64, n3=16, r=10,
                             decay=("geom", 0.8), noise=1e-3, k=5, b=10, q=2,
                             seed=0, prec="f64"),
    "c2_fp32_1000x1000x32": dict(kind="lowrank", n1=1000, n2=1000, n3=32, r=200,
                                 decay=("geom", 0.95), noise=1e-4, k=50, b=60, q=2,
                                 seed=1, prec="f32"),
    "c3_hyper_512x512x200": dict(kind="hyperspectral", n1=512, n2=512, n3=200, r=30,
                                 noise=1e-3, k=30, b=40, q=3, seed=2, prec="bf16"),
    "c4_completion_2000x2000x16": dict(kind="completion", n1=2000, n2=2000, n3=16,
                                       r=20, keep=0.3, k=20, b=30, q=2, seed=3,
                                       prec="f32"),
    "c5_fp32_4096x4096x64": dict(kind="lowrank", n1=4096, n2=4096, n3=64, r=400,
                                 decay=("pow", -1.5), noise=1e-5, k=100, b=110, q=3,
                                 seed=4, prec="f32"),
}

# Sec. 5, Example 1: n x n x n tensors with prescribed slice spectra, R = 45,
# P = 5, q = 2 (the paper does not state n; 256 here).  Compared between the
# power-iteration method (Alg. 1) and the block Krylov method (Alg. 2).
EX1_CONFIGS = {
    "ex1_pow5_256": dict(kind="spectrum", n1=256, n2=256, n3=256, decay=("pow", -5.0),
                         k=45, b=50, q=2, seed=11, prec="f64"),
    "ex1_pow6_256": dict(kind="spectrum", n1=256, n2=256, n3=256, decay=("pow", -6.0),
                         k=45, b=50, q=2, seed=12, prec="f64"),
    "ex1_geom05_256": dict(kind="spectrum", n1=256, n2=256, n3=256, decay=("geom", 0.5),
                           k=45, b=50, q=2, seed=13, prec="f64"),
}


def _streams(seed: int):
    ss = np.random.SeedSequence(seed)
    data_ss, omega_ss = ss.spawn(2)
    return np.random.default_rng(data_ss), np.random.default_rng(omega_ss)


def _decay(spec, r: int) -> np.ndarray:
    i = np.arange(1, r + 1, dtype=np.float64)
    kind, val = spec
    if kind == "geom":
        return val ** i
    if kind == "pow":
        return i ** val
    raise ValueError(spec)


def _tprod_usvt(U: np.ndarray, s_tubes: np.ndarray | None, V: np.ndarray) -> np.ndarray:
    """U * S * V^T for f-diagonal S given by its diagonal tubes (r x n3), or
    U * V^T when s_tubes is None; evaluated slice-wise in the Fourier domain
    with numpy's real FFT."""
    n3 = U.shape[2]
    Ub = np.fft.rfft(U, axis=2)
    Vb = np.fft.rfft(V, axis=2)
    sb = np.fft.rfft(s_tubes, axis=1) if s_tubes is not None else None
    F = Ub.shape[2]
    Ab = np.empty((U.shape[0], V.shape[0], F), dtype=np.complex128)
    for f in range(F):
        Uf = Ub[:, :, f] if sb is None else Ub[:, :, f] * sb[:, f]
        Ab[:, :, f] = Uf @ Vb[:, :, f].conj().T
    return np.fft.irfft(Ab, n=n3, axis=2)


def lowrank_tensor(n1, n2, n3, r, decay, noise, seed):
    """A = U * S * V^T + noise * N(0, 1) (recipe ``lowrank``)."""
    rng, _ = _streams(seed)
    U = rng.standard_normal((n1, r, n3))
    s = _decay(decay, r)[:, None] * rng.standard_normal((r, n3))
    V = rng.standard_normal((n2, r, n3))
    A = _tprod_usvt(U, s, V)
    if noise:
        A += noise * rng.standard_normal((n1, n2, n3))
    return np.ascontiguousarray(A)


def exact_lowrank_tensor(n1, n2, n3, r, seed, decay=("geom", 0.8)):
    """Noiseless tensor of tubal rank <= r (recipe ``lowrank`` without noise)."""
    return lowrank_tensor(n1, n2, n3, r, decay, 0.0, seed)


def hyperspectral_tensor(n1, n2, n3, r, noise, seed):
    """Recipe ``hyperspectral``: A0(i, j, t) = sum_r g_r(i) h_r(j) s_r(t) with
    g_r, h_r Gaussian bumps (centres U[0, n), widths U[8, 64]) and s_r a sum
    of 2-3 Gaussian bumps over t (amplitude U[0.2, 1], width U[5, 40]);
    min-max scaled to [0, 1]; then noise * N(0, 1), no clipping."""
    rng, _ = _streams(seed)
    i = np.arange(n1, dtype=np.float64)
    j = np.arange(n2, dtype=np.float64)
    t = np.arange(n3, dtype=np.float64)
    G = np.empty((n1, r))
    H = np.empty((n2, r))
    Sp = np.zeros((n3, r))
    for c in range(r):
        ci, wi = rng.uniform(0, n1), rng.uniform(8, 64)
        cj, wj = rng.uniform(0, n2), rng.uniform(8, 64)
        G[:, c] = np.exp(-(i - ci) ** 2 / (2 * wi * wi))
        H[:, c] = np.exp(-(j - cj) ** 2 / (2 * wj * wj))
        for _ in range(int(rng.integers(2, 4))):
            a, ct, wt = rng.uniform(0.2, 1.0), rng.uniform(0, n3), rng.uniform(5, 40)
            Sp[:, c] += a * np.exp(-(t - ct) ** 2 / (2 * wt * wt))
    A = np.einsum("ic,jc,tc->ijt", G, H, Sp, optimize=True)
    A = (A - A.min()) / (A.max() - A.min())
    if noise:
        A += noise * rng.standard_normal((n1, n2, n3))
    return np.ascontiguousarray(A)


def separable_factors(n1, n2, n3, r, decay, noise, seed):
    """Recipe ``separable``: the factors of
    A(i, j, t) = sum_c G[i, c] H[j, c] Sp[t, c] + noise Nz[i, j] w[t]
    with G, H, Sp, Nz, w i.i.d. N(0, 1) (drawn in that order) and column c of
    Sp scaled by decay^c.  Every Fourier slice is a rank-r matrix plus a
    multiple of the one dense matrix Nz.  Returns (G, H, Sp, Nz, w, noise);
    the tensor itself is formed by the caller (separable_tensor for small
    shapes)."""
    rng, _ = _streams(seed)
    G = rng.standard_normal((n1, r))
    H = rng.standard_normal((n2, r))
    Sp = rng.standard_normal((n3, r)) * decay ** np.arange(r, dtype=np.float64)
    Nz = rng.standard_normal((n1, n2))
    w = rng.standard_normal(n3)
    return G, H, Sp, Nz, w, float(noise)


def separable_tensor(factors) -> np.ndarray:
    """The n1 x n2 x n3 tensor of separable_factors, on the host."""
    G, H, Sp, Nz, w, noise = factors
    A = np.einsum("ic,jc,tc->ijt", G, H, Sp, optimize=True) + noise * Nz[:, :, None] * w[None, None, :]
    return np.ascontiguousarray(A)


def _orthogonal_tensor(n: int, r: int, n3: int, rng) -> np.ndarray:
    """Real n x r x n3 tensor whose half-spectrum Fourier slices have
    orthonormal columns (numpy's QR of complex Gaussian matrices; real
    Gaussian at the DC slice and, for even n3, the Nyquist slice)."""
    F = n3 // 2 + 1
    Ub = np.empty((n, r, F), dtype=np.complex128)
    for f in range(F):
        G = rng.standard_normal((n, r))
        if not (f == 0 or (n3 % 2 == 0 and f == n3 // 2)):
            G = G + 1j * rng.standard_normal((n, r))
        Ub[:, :, f], _ = np.linalg.qr(G)
    return np.fft.irfft(Ub, n=n3, axis=2)


def spectrum_tensor(n1, n2, n3, decay, seed):
    """Recipe ``spectrum``: A = U * S * V^T, U and V orthogonal tensors, S
    f-diagonal with tubes sigma_m e_1 (m = 1..min(n1, n2)), so that every
    Fourier slice of A has the singular values sigma_m."""
    rng, _ = _streams(seed)
    r = min(n1, n2)
    U = _orthogonal_tensor(n1, r, n3, rng)
    V = _orthogonal_tensor(n2, r, n3, rng)
    s = np.zeros((r, n3))
    s[:, 0] = _decay(decay, r)
    return np.ascontiguousarray(_tprod_usvt(U, s, V))


def completion_problem(n1, n2, n3, r, keep, seed):
    """Recipe ``completion``: T = U * V^T (tubal rank r, N(0,1) factors),
    mask M ~ Bernoulli(keep) per entry, X0 = M (.) T.  Returns (T, M, X0)."""
    rng, _ = _streams(seed)
    U = rng.standard_normal((n1, r, n3))
    V = rng.standard_normal((n2, r, n3))
    T = _tprod_usvt(U, None, V)
    M = (rng.random((n1, n2, n3)) < keep).astype(np.float64)
    return np.ascontiguousarray(T), M, np.ascontiguousarray(M * T)


def image_tensor(n1, n2, n3, seed, alpha=1.6):
    """Recipe ``image``: a random image stand-in in [0, 255] with a power-law
    spectrum.  Each channel is white Gaussian noise whose 2-D Fourier
    amplitudes are scaled by 1 / (|f| + 1/max(n1, n2))^alpha (numpy FFT); the
    channels are mixed by a random positive matrix so that they are
    correlated, then the whole is min-max scaled to [0, 255].  alpha = 1.6
    leaves about 9% relative error in the best tubal-rank-50 approximation of
    a 512 x 768 x 3 image."""
    rng, _ = _streams(seed)
    fi = np.fft.fftfreq(n1)[:, None]
    fj = np.fft.fftfreq(n2)[None, :]
    filt = 1.0 / (np.sqrt(fi ** 2 + fj ** 2) + 1.0 / max(n1, n2)) ** alpha
    base = np.empty((n1, n2, n3))
    for c in range(n3):
        z = rng.standard_normal((n1, n2))
        base[:, :, c] = np.real(np.fft.ifft2(np.fft.fft2(z) * filt))
    mix = 0.5 + rng.random((n3, n3))
    img = np.einsum("ijc,dc->ijd", base, mix)
    img = (img - img.min()) / (img.max() - img.min()) * 255.0
    return np.ascontiguousarray(img)


def bernoulli_mask(shape, keep, seed):
    """0/1 observation tensor, each entry kept with probability `keep`
    (one draw per pixel, shared by the n3 channels)."""
    rng, _ = _streams(seed + 1000)
    m = (rng.random(shape[:2]) < keep).astype(np.float64)
    return np.ascontiguousarray(np.repeat(m[:, :, None], shape[2], axis=2))


def line_mask(shape, every, seed):
    """0/1 observation tensor with line segments missing on every `every`-th
    row and column (random offset): each segment covers a random 20-60% of
    its row or column (structured loss, Example 3).  Whole missing rows or
    columns would be unrecoverable by any low-rank model: a row with no
    observed entry stays zero in every rank-k approximation."""
    rng, _ = _streams(seed + 2000)
    n1, n2, n3 = shape
    m = np.ones((n1, n2))
    for i in range(int(rng.integers(0, every)), n1, every):
        ln = int(rng.uniform(0.2, 0.6) * n2)
        j0 = int(rng.integers(0, n2 - ln + 1))
        m[i, j0:j0 + ln] = 0.0
    for j in range(int(rng.integers(0, every)), n2, every):
        ln = int(rng.uniform(0.2, 0.6) * n1)
        i0 = int(rng.integers(0, n1 - ln + 1))
        m[i0:i0 + ln, j] = 0.0
    return np.ascontiguousarray(np.repeat(m[:, :, None], n3, axis=2))


def circle_mask(shape, count, seed, rmin=10.0, rmax=60.0, width=2.0):
    """0/1 observation tensor with `count` random circles missing: rings of
    radius U[rmin, rmax] and the given width around uniformly placed centres
    (structured loss, Example 3)."""
    rng, _ = _streams(seed + 3000)
    n1, n2, n3 = shape
    i = np.arange(n1, dtype=np.float64)[:, None]
    j = np.arange(n2, dtype=np.float64)[None, :]
    m = np.ones((n1, n2))
    for _ in range(count):
        ci, cj, r = rng.uniform(0, n1), rng.uniform(0, n2), rng.uniform(rmin, rmax)
        m[np.abs(np.sqrt((i - ci) ** 2 + (j - cj) ** 2) - r) < width / 2] = 0.0
    return np.ascontiguousarray(np.repeat(m[:, :, None], n3, axis=2))


# Sec. 5, Example 3: completion of 512 x 768 x 3 images with 70% of the pixels
# missing, tubal rank 50, P = 10, q = 2 (smooth random stand-ins for the
# missing Kodak images).
COMPLETION_CONFIGS = {
    "ex3_image_512x768x3": dict(n1=512, n2=768, n3=3, keep=0.3, k=50, b=60, q=2, iters=100, seed=21),
}


def philox4x32_10(ctr, key):
    """Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
    as easy as 1, 2, 3", SC'11), vectorised over counters.  ctr: uint32 array
    (..., 4); key: two uint32 words.  Ten rounds; each multiplies words 0 and 2
    by 0xD2511F53 and 0xCD9E8D57 (32 x 32 -> 64 bits), mixes the high halves
    with words 1 and 3 and the key, and the key is bumped by 0x9E3779B9 and
    0xBB67AE85 after every round.  Returns uint32 array (..., 4)."""
    c = [np.asarray(ctr[..., i], dtype=np.uint64) for i in range(4)]
    k0, k1 = np.uint64(int(key[0]) & 0xFFFFFFFF), np.uint64(int(key[1]) & 0xFFFFFFFF)
    mask = np.uint64(0xFFFFFFFF)
    for _ in range(10):
        p0 = np.uint64(0xD2511F53) * c[0]
        p1 = np.uint64(0xCD9E8D57) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & mask
        hi1, lo1 = p1 >> np.uint64(32), p1 & mask
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
        k0 = (k0 + np.uint64(0x9E3779B9)) & mask
        k1 = (k1 + np.uint64(0xBB67AE85)) & mask
    return np.stack([x.astype(np.uint32) for x in c], axis=-1)


def _unit(hi, lo):
    """Uniform in (0, 1): (2 x + 1) 2^-53 with the 52-bit integer
    x = (hi >> 6) 2^26 + (lo >> 6)."""
    x = (hi.astype(np.uint64) >> np.uint64(6) << np.uint64(26)) | (lo.astype(np.uint64) >> np.uint64(6))
    return (2 * x + 1).astype(np.float64) * 2.0 ** -53


def _log_unit(u):
    """ln u for u in (0, 1), as a fixed sequence of IEEE double operations:
    u = 2^e m with m in (sqrt(1/2), sqrt(2)], ln m = 2 atanh(s),
    s = (m - 1)/(m + 1), atanh by its Taylor series to s^21."""
    m, e = np.frexp(u)               # u = m 2^e, m in [0.5, 1)
    m = m * 2.0
    e = e - 1                        # m in [1, 2)
    big = m > float.fromhex("0x1.6a09e667f3bcdp+0")
    m = np.where(big, m * 0.5, m)
    e = np.where(big, e + 1, e)
    s = (m - 1.0) / (m + 1.0)
    s2 = s * s
    p = np.full_like(s, 1.0 / 21.0)
    for d in (19.0, 17.0, 15.0, 13.0, 11.0, 9.0, 7.0, 5.0, 3.0):
        p = p * s2 + 1.0 / d
    p = p * s2 + 1.0
    lm = 2.0 * s * p
    return e.astype(np.float64) * float.fromhex("0x1.62e42fefa39efp-1") + lm


def _sqrt_newton(x):
    """sqrt x: five Newton steps y <- (y + x / y) / 2 from the guess with
    the halved exponent (bits(x) >> 1) + 0x1ff8000000000000."""
    y = ((x.view(np.uint64) >> np.uint64(1)) + np.uint64(0x1FF8000000000000)).view(np.float64)
    for _ in range(5):
        y = 0.5 * (y + x / y)
    return y


def _sincos_2pi(u):
    """(cos 2 pi u, sin 2 pi u) for u in (0, 1): quadrant j = floor(4 u), the
    Taylor series of sin and cos of x = (pi/2)(4 u - j) to degree 25 and 24
    (Horner in x^2, alternating signs), rotated by j; a fixed sequence of IEEE
    double operations."""
    import math
    inv = {d: 1.0 / float(math.factorial(d)) for d in range(2, 26)}
    v = u * 4.0
    j = v.astype(np.int64)
    x = (v - j.astype(np.float64)) * float.fromhex("0x1.921fb54442d18p+0")
    x2 = x * x
    ps = np.full_like(x, inv[25])
    for d in range(23, 2, -2):                 # -1/23!, +1/21!, ..., -1/3!
        ps = ps * x2 - inv[d] if (d // 2) % 2 == 1 else ps * x2 + inv[d]
    pc = np.full_like(x, inv[24])
    for d in range(22, 1, -2):                 # -1/22!, +1/20!, ..., -1/2!
        pc = pc * x2 - inv[d] if (d // 2) % 2 == 1 else pc * x2 + inv[d]
    sn = x + x * x2 * ps
    cs = 1.0 + x2 * pc
    q = j & 3
    c = np.select([q == 0, q == 1, q == 2], [cs, -sn, -cs], sn)
    s = np.select([q == 0, q == 1, q == 2], [sn, cs, -sn], -cs)
    return c, s


def omega_counter(n: int, seed: int) -> np.ndarray:
    """The first n values of the seeded Gaussian stream of the test tensor
    Omega (Alg. 2 draws randn): element e takes pair p = e // 2 of a
    Box-Muller transform of Philox4x32-10(counter (p_lo, p_hi, 0, 0), key
    (seed_lo, seed_hi)), r cos(theta) for even e and r sin(theta) for odd e,
    with u1, u2 from the words (0, 1) and (2, 3), r = sqrt(-2 ln u1),
    theta = 2 pi u2."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    npairs = (n + 1) // 2
    out = np.empty(2 * npairs, dtype=np.float64)
    chunk = 1 << 22
    for p0 in range(0, npairs, chunk):
        p = np.arange(p0, min(npairs, p0 + chunk), dtype=np.uint64)
        ctr = np.zeros(p.shape + (4,), dtype=np.uint64)
        ctr[:, 0] = p & np.uint64(0xFFFFFFFF)
        ctr[:, 1] = p >> np.uint64(32)
        w = philox4x32_10(ctr, (seed & 0xFFFFFFFF, seed >> 32))
        u1 = _unit(w[:, 0], w[:, 1])
        u2 = _unit(w[:, 2], w[:, 3])
        r = _sqrt_newton(-2.0 * _log_unit(u1))
        c, s = _sincos_2pi(u2)
        out[2 * p0:2 * p0 + 2 * p.size:2] = r * c
        out[2 * p0 + 1:2 * p0 + 2 * p.size:2] = r * s
    return out[:n]


def omega(n2, b, n3, seed):
    """Gaussian test tensor Omega ~ N(0, 1), n2 x b x n3 (Alg. 2, first line,
    with n2 rows): element (j, c, t) is value (j b + c) n3 + t of the seeded
    counter-based stream (omega_counter)."""
    return np.ascontiguousarray(omega_counter(n2 * b * n3, seed).reshape(n2, b, n3))


def make_config(name: str):
    """(A, Omega, params) for a named workload; A and Omega are float64."""
    c = dict(CONFIGS[name] if name in CONFIGS else EX1_CONFIGS[name])
    kind = c["kind"]
    if kind == "lowrank":
        A = lowrank_tensor(c["n1"], c["n2"], c["n3"], c["r"], c["decay"], c["noise"], c["seed"])
    elif kind == "hyperspectral":
        A = hyperspectral_tensor(c["n1"], c["n2"], c["n3"], c["r"], c["noise"], c["seed"])
    elif kind == "spectrum":
        A = spectrum_tensor(c["n1"], c["n2"], c["n3"], c["decay"], c["seed"])
    elif kind == "completion":
        T, M, A = completion_problem(c["n1"], c["n2"], c["n3"], c["r"], c["keep"], c["seed"])
        c["T"], c["M"] = T, M
    else:
        raise ValueError(kind)
    Om = omega(c["n2"], c["b"], c["n3"], c["seed"])
    return A, Om, c


def random_tensor(shape, seed, dist="normal"):
    """Plain i.i.d. tensor for unit tests."""
    rng, _ = _streams(seed)
    if dist == "normal":
        return rng.standard_normal(shape)
    return rng.uniform(-1, 1, shape)
