"""Pins of the oracle's counter-based Gaussian generator: the published
Philox4x32-10 known-answer vectors and the distribution of the test matrix."""

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
