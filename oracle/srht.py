"""Structured test matrix of the range finder: the subsampled randomised
Hadamard transform (SRHT) -- TEST INFRASTRUCTURE ONLY.

The paper puts the cost of its RSVD at O(mn log r) + O((m + n) r^2)
(Sec. 2.2, after Alg. 1), which is the cost of a structured random test
matrix (Halko, Martinsson & Tropp 2011, Sec. 4.6: Omega = sqrt(n / l) D F R
with D a random diagonal of unit entries, F a unitary transform with a fast
algorithm and R a uniformly random choice of l coordinates).  The real
variant here takes F = H / sqrt(k'), H the Sylvester-Hadamard matrix.

Definition (shared with the C ABI, both sides implementing it from here):
  k'  = the smallest power of two >= k; A is read as padded with k' - k zero
        columns (so only the first k rows of Omega matter);
  d_i = +1 when bit 0 of word x0 of Philox4x32-10 at counter (i, 0, 1, 0),
        key (seed mod 2^32, seed >> 32), is 0, else -1   (i < k');
  H   = the k' x k' Sylvester-Hadamard matrix, H[i][j] = (-1)^popcount(i & j);
  u_i = word x0 of Philox4x32-10 at counter (i, 0, 2, 0), same key;
  S   = the indices of the l smallest pairs (u_i, i) (lexicographic), listed
        in increasing index order;
  Omega = (D H)[0:k, S] / sqrt(l)     (k x l),
so that Y = A Omega = (A_pad D H)[:, S] / sqrt(l).  Over the full padded
height Omega^T Omega = (k' / l) I.

The sketch takes no operand codes.  In FP64 (the unquantised mode) it is
the product A Omega.  Otherwise, like every other stage output that feeds a
quantiser, it is a binary32 quantity, and its rounding is fixed here: the
radix-2 Walsh-Hadamard butterflies (u, w) -> (fl32(u + w), fl32(u - w)) on
index pairs (i, i + 2^s), i without bit s, for s = 0, 1, .., log2 k' - 1 in
that order, applied to the binary32 row of A times d; then each sampled
entry is multiplied by fl32(1 / sqrt(l)) with one rounding.  Power
iterations, when asked for, run as in lramm.py.

Pins (tests/test_oracle_srht.py): H against scipy.linalg.hadamard, the
identity Omega^T Omega = (k / l) I for k a power of two, S a set of l
distinct sorted indices whose selection frequencies and signs match their
probabilities over many seeds, ||A Omega||_F = ||A||_F when l = k = k', and
exact recovery of a rank-deficient A through the range finder; the binary32
transform equal to the FP64 product on integer inputs (every partial sum
exact) and within (log2 k' + 3) 2^-24 sum_i |a_i| / sqrt(l) of it on random
ones, and applying the binary32 butterflies twice giving k' times the input
on integers.
"""

import numpy as np

from .philox import MASK, philox4x32_10


def next_pow2(k):
    kp = 1
    while kp < k:
        kp *= 2
    return kp


def _words(seed, n, stream):
    """Word x0 of Philox4x32-10 at counters (i, 0, stream, 0), i < n."""
    i = np.arange(n, dtype=np.uint64)
    ctr = np.stack([i & np.uint64(MASK), np.zeros_like(i), np.full_like(i, stream), np.zeros_like(i)], axis=-1)
    return philox4x32_10(ctr, (seed & MASK, (seed >> 32) & MASK))[:, 0]


def srht_signs(seed, k):
    """d_0 .. d_{k'-1} as +-1.0."""
    w = _words(seed, next_pow2(k), 1)
    return np.where((w & 1) == 0, 1.0, -1.0)


def srht_samples(seed, k, l):
    """S: the l sampled coordinates of [0, k'), increasing."""
    kp = next_pow2(k)
    if not 1 <= l <= kp:
        raise ValueError("need 1 <= l <= k'")
    u = _words(seed, kp, 2).astype(np.int64)
    order = np.lexsort((np.arange(kp), u))      # by key, then by index
    return np.sort(order[:l])


def hadamard_entry(i, j):
    """H[i][j] = (-1)^popcount(i & j) for integer arrays i, j."""
    x = np.bitwise_and(np.asarray(i, np.int64), np.asarray(j, np.int64))
    par = np.zeros(np.broadcast(i, j).shape, np.int64)
    while np.any(x):
        par ^= x & 1
        x = x >> 1
    return 1.0 - 2.0 * par


def srht_omega(seed, k, l):
    """The k x l test matrix (D H)[0:k, S] / sqrt(l) in FP64."""
    d = srht_signs(seed, k)[:k]
    S = srht_samples(seed, k, l)
    H = hadamard_entry(np.arange(k)[:, None], S[None, :])
    return d[:, None] * H / np.sqrt(l)


def fwht_fp32(X):
    """Radix-2 Walsh-Hadamard transform of every row of X (k' columns, a
    power of two) in binary32, butterflies of bit s = 0, 1, .. in order."""
    Y = np.array(X, dtype=np.float32)
    kp = Y.shape[1]
    h = 1
    while h < kp:
        Y = Y.reshape(Y.shape[0], kp // (2 * h), 2, h)
        u = Y[:, :, 0, :].copy()
        w = Y[:, :, 1, :].copy()
        Y[:, :, 0, :] = u + w           # float32 + float32: one IEEE rounding
        Y[:, :, 1, :] = u - w
        Y = Y.reshape(-1, kp)
        h *= 2
    return Y


def srht_sketch(A, seed, l, precision="fp32"):
    """Y = A Omega: the FP64 product ("fp64") or the binary32 transform
    ("fp32", values returned as float64)."""
    A = np.asarray(A, np.float64)
    m, k = A.shape
    if precision == "fp64":
        return A @ srht_omega(seed, k, l)
    kp = next_pow2(k)
    X = np.zeros((m, kp), np.float32)
    X[:, :k] = A.astype(np.float32)
    X = X * srht_signs(seed, k).astype(np.float32)[None, :]   # exact sign flips
    T = fwht_fp32(X)
    S = srht_samples(seed, k, l)
    scale = np.float32(1.0 / np.sqrt(np.float64(l)))
    return (T[:, S] * scale).astype(np.float64)
