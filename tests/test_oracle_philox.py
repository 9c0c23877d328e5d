"""Pins of the oracle's counter-based Gaussian generator: the published
Philox4x32-10 known-answer vectors and the distribution of the test matrix."""

import math
import os

import numpy as np
from scipy import stats

from oracle import philox as P

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_known_answer_vectors():
    n = 0
    for line in open(os.path.join(GOLD, "philox_kat.txt")):
        s = line.strip()
        if not s or s.startswith("#"):
            continue
        c, k, o = [[int(x, 16) for x in part.split()] for part in s.split("|")]
        out = P.philox4x32_10(np.array([c]), k)[0]
        assert [int(x) for x in out] == o
        n += 1
    assert n == 3


def test_gaussian_omega_distribution_and_mapping():
    k, l = 700, 37
    om = P.gaussian_omega(12345, k, l)
    assert om.shape == (k, l)
    assert np.all(om.astype(np.float32) == om)
    z = om.reshape(-1)
    assert abs(z.mean()) < 0.02 and abs(z.std() - 1) < 0.02
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # element (i, j) comes from counter e >> 2 with e = j*k + i, word pair e & 3
    i, j = 123, 17
    e = j * k + i
    w = P.philox4x32_10(np.array([[e >> 2, 0, 0, 0]]), (12345, 0))[0]
    pair = (w[0], w[1]) if (e & 3) < 2 else (w[2], w[3])
    zz = P.box_muller(np.array([pair[0]]), np.array([pair[1]]))[(e & 3) % 2][0]
    assert om[i, j] == float(np.float32(zz))
    # different seeds give different matrices
    assert not np.array_equal(om, P.gaussian_omega(12346, k, l))


def test_box_muller_closed_forms():
    """Words whose uniforms are exact (u1 = (a + 1) 2^-32, u2 = b 2^-32) give
    closed-form normals: radius sqrt(-2 ln u1), angle 2 pi u2, the first
    output on the cosine.  A swapped cosine and sine, a dropped factor 2 or an
    off-by-one in the word mapping fails one of these."""
    top = np.uint32(0xFFFFFFFF)
    # u1 = 1: radius 0 whatever the angle
    z0, z1 = P.box_muller(np.array([top, top]), np.array([0, 12345], np.uint32))
    assert np.all(z0 == 0.0) and np.all(z1 == 0.0)
    # u1 = 2^-32 (a = 0): radius sqrt(64 ln 2); u2 = 0: all on the first output
    r = math.sqrt(64.0 * math.log(2.0))
    z0, z1 = P.box_muller(np.array([0], np.uint32), np.array([0], np.uint32))
    assert abs(z0[0] - r) <= 1e-15 * r and z1[0] == 0.0
    # u1 = 1/2 (a = 2^31 - 1): radius sqrt(2 ln 2); quarter and half turns
    r = math.sqrt(2.0 * math.log(2.0))
    a = np.full(3, 2**31 - 1, np.uint32)
    z0, z1 = P.box_muller(a, np.array([2**30, 2**31, 3 * 2**30], np.uint32))
    assert np.allclose(z0, [0.0, -r, 0.0], atol=1e-15) and np.allclose(z1, [r, 0.0, -r], atol=1e-15)
    # random words: the pair's radius and angle are the two uniforms' images
    rng = np.random.default_rng(2)
    a = rng.integers(0, 2**32, 1000, dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, 2**32, 1000, dtype=np.uint64).astype(np.uint32)
    z0, z1 = P.box_muller(a, b)
    u1 = (a.astype(np.float64) + 1.0) / 2.0**32
    u2 = b.astype(np.float64) / 2.0**32
    assert np.allclose(z0**2 + z1**2, -2.0 * np.log(u1), rtol=1e-12, atol=1e-12)
    ang = np.mod(np.arctan2(z1, z0), 2.0 * np.pi)
    d = np.abs(ang - 2.0 * np.pi * u2)
    assert np.all(np.minimum(d, 2.0 * np.pi - d) <= 1e-9)
