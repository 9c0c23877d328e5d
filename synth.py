"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds no arithmetic of the method: it only draws matrices.  Both
the oracle and the HIP path receive the arrays it returns; neither imports
the other.

Recipe (NumPy ``default_rng`` / PCG64):
  * Haar-distributed orthonormal factors: Q of the QR of a standard-normal
    matrix, columns multiplied by sign(diag R) (Mezzadri 2007).
  * low-rank-structured A = (U * sigma) V^T in FP64 with U (m x c) and
    V (k x c) Haar factors drawn in that order from ``default_rng(seed)``,
    c = number of sigma_i >= 1e-9 sigma_1 (thin factors when the spectrum
    falls below that), then rounded once to binary32 (or bf16).
  * optional entrywise noise: the low-rank part is scaled to unit RMS entry
    and N(0, noise_var) noise from ``default_rng(seed + 200)`` is added.
  * B ~ N(0, 1) i.i.d. from ``default_rng(seed + 100)`` unless a seed is given.
  * Omega ~ N(0, 1) i.i.d. from ``default_rng(omega_seed)``, k x l, binary32.
"""

import numpy as np


def haar(n, cols, rng):
    G = rng.standard_normal((n, cols))
    Q, R = np.linalg.qr(G)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :]


def spectrum(kind, count, param):
    """sigma_i for i = 1..count: kind 'exp' -> exp(-i/param), 'pow' -> i^-param."""
    i = np.arange(1, count + 1, dtype=np.float64)
    if kind == "exp":
        return np.exp(-i / param)
    if kind == "pow":
        return i ** (-float(param))
    raise ValueError(kind)


def to_dtype(X, dtype):
    X = np.asarray(X, np.float64)
    if dtype == "fp32":
        return X.astype(np.float32)
    if dtype == "bf16":
        # round-to-nearest-even to 8 significant bits, kept in a float32 array
        b = X.astype(np.float32).view(np.uint32).astype(np.uint64)
        b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
        return b.astype(np.uint32).view(np.float32)
    raise ValueError(dtype)


def lowrank(m, k, sigma, seed, noise_var=0.0, dtype="fp32", info=None):
    """Return (A, sigma) with A = U diag(sigma) V^T (+ noise) as float32 data.

    With noise the low-rank part is first scaled to unit RMS entry; the
    returned sigma is scaled by the same factor, so it holds the singular
    values of the low-rank part of the returned A.  ``info`` (a dict, when
    given) receives that factor ("scale") and the Frobenius norm of the noise
    actually added ("noise_fro", 0 without noise)."""
    sigma = np.asarray(sigma, np.float64)
    c = int(np.sum(sigma >= 1e-9 * sigma[0]))
    c = max(1, min(c, m, k))
    rng = np.random.default_rng(seed)
    U = haar(m, c, rng)
    V = haar(k, c, rng)
    A = (U * sigma[:c][None, :]) @ V.T
    scale, noise_fro = 1.0, 0.0
    if noise_var > 0.0:
        scale = 1.0 / np.sqrt(np.mean(A * A))
        N = np.sqrt(noise_var) * np.random.default_rng(seed + 200).standard_normal((m, k))
        noise_fro = float(np.linalg.norm(N))
        A = A * scale + N
    if info is not None:
        info["scale"] = float(scale)
        info["noise_fro"] = noise_fro
    return to_dtype(A, dtype), sigma * scale


def gaussian(rows, cols, seed, dtype="fp32"):
    return to_dtype(np.random.default_rng(seed).standard_normal((rows, cols)), dtype)


def omega(k, l, seed):
    return np.random.default_rng(seed).standard_normal((k, l)).astype(np.float32)


def small_lramm_case(m=512, k=512, n=512, tau=32.0, seed=0, omega_seed=1):
    """Plain LRAMM small case: sigma_i = exp(-i/tau), Haar U, V from ``seed``,
    B ~ N(0,1) from seed + 100."""
    A, s = lowrank(m, k, spectrum("exp", min(m, k), tau), seed)
    B = gaussian(k, n, seed + 100)
    return A, B, s


def batch_shapes(count=64, lo=256, hi=8192, seed=7):
    """Uneven batch: (M, N, K) = round(exp(U(ln lo, ln hi))) drawn in the order
    M, N, K per product."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        v = np.exp(rng.uniform(np.log(lo), np.log(hi), size=3))
        out.append(tuple(int(round(x)) for x in v))
    return out
