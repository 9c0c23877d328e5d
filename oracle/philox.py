"""Philox4x32-10 and the Gaussian test matrix -- TEST INFRASTRUCTURE ONLY.

The range finder samples A with a Gaussian test matrix (Sec. 2.2 lists
Gaussian sampling among the strategies; the library's default sketch uses
it).  When the caller does not pass Omega, the library draws it from a
counter-based generator so that any element can be recomputed independently.  Both sides
implement the same published generator from its definition:

  Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
  as 1, 2, 3", SC 2011): a 128-bit counter (x0..x3) and a 64-bit key (k0, k1);
  each of 10 rounds replaces the counter by
      (hi(M1*x2) ^ x1 ^ k0, lo(M1*x2), hi(M0*x0) ^ x3 ^ k1, lo(M0*x0))
  with M0 = 0xD2511F53, M1 = 0xCD9E8D57, and after every round bumps the key by
  the Weyl constants (0x9E3779B9, 0xBB67AE85).

Mapping to the k x l matrix Omega (a choice of this library, documented with
the C ABI): element Omega[i][j] has linear index e = j*k + i (row-major index
of Omega^T).  Philox is evaluated at counter (c mod 2^32, c >> 32, 0, 0) with
c = e >> 2 and key (seed mod 2^32, seed >> 32).  Its words form two
Box-Muller pairs: u1 = (x0 + 1) 2^-32 in (0, 1], u2 = x1 2^-32,
z0 = sqrt(-2 ln u1) cos(2 pi u2), z1 = sqrt(-2 ln u1) sin(2 pi u2), and the
same with (x2, x3) for z2, z3.  Element e takes z_(e mod 4), computed in FP64
and rounded once to binary32.

Pins (tests/test_oracle_philox.py): the published Random123 known-answer
vectors for Philox4x32-10, moments / normality of the generated matrix, and
Box-Muller closed forms (radius and angle of words with exact uniforms).
"""

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Vectorised Philox4x32-10.  ctr: (..., 4) uint32-valued; key: (2,)."""
    x = np.array(ctr, dtype=np.uint64) & MASK
    k0 = np.uint64(key[0] & MASK)
    k1 = np.uint64(key[1] & MASK)
    x0, x1, x2, x3 = (x[..., i].copy() for i in range(4))
    for _ in range(10):
        p0 = x0 * np.uint64(M0)          # < 2^64: exact in uint64
        p1 = x2 * np.uint64(M1)
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK)
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
        k0 = (k0 + np.uint64(W0)) & np.uint64(MASK)
        k1 = (k1 + np.uint64(W1)) & np.uint64(MASK)
    return np.stack([x0, x1, x2, x3], axis=-1).astype(np.uint32)


def box_muller(a, b):
    """Two standard normals from two uint32 words (FP64)."""
    u1 = (a.astype(np.float64) + 1.0) * 2.0**-32
    u2 = b.astype(np.float64) * 2.0**-32
    r = np.sqrt(-2.0 * np.log(u1))
    t = 2.0 * np.pi * u2
    return r * np.cos(t), r * np.sin(t)


def gaussian_omega(seed, k, l):
    """The k x l Gaussian test matrix of the library's seeded mode (binary32
    values returned as float64)."""
    total = k * l
    nctr = (total + 3) // 4
    c = np.arange(nctr, dtype=np.uint64)
    ctr = np.stack([c & np.uint64(MASK), c >> np.uint64(32),
                    np.zeros_like(c), np.zeros_like(c)], axis=-1)
    words = philox4x32_10(ctr, (seed & MASK, (seed >> 32) & MASK))
    z0, z1 = box_muller(words[:, 0], words[:, 1])
    z2, z3 = box_muller(words[:, 2], words[:, 3])
    z = np.stack([z0, z1, z2, z3], axis=-1).reshape(-1)[:total]
    omega_t = z.astype(np.float32).astype(np.float64).reshape(l, k)   # index e = j*k + i
    return omega_t.T.copy()
