"""Pins of the oracle's structured test matrix (Halko et al. 2011, Sec. 4.6;
the paper's O(mn log r) RSVD cost, Sec. 2.2) against a library routine,
closed forms and sampling probabilities.  CPU only."""

import numpy as np
import scipy.linalg

import synth
from oracle import lramm as L
from oracle import srht as S


def test_hadamard_matches_scipy():
    for kp in (1, 2, 8, 64, 256):
        i = np.arange(kp)
        H = S.hadamard_entry(i[:, None], i[None, :])
        assert np.array_equal(H, scipy.linalg.hadamard(kp).astype(np.float64))


def test_next_pow2():
    assert [S.next_pow2(k) for k in (1, 2, 3, 64, 65, 4096, 4097)] == [1, 2, 4, 64, 128, 4096, 8192]


def test_columns_orthogonal_for_power_of_two_height():
    for k, l in ((64, 10), (256, 40), (512, 512)):
        Om = S.srht_omega(11, k, l)
        assert Om.shape == (k, l)
        assert np.max(np.abs(Om.T @ Om - (k / l) * np.eye(l))) <= 1e-12 * k / l


def test_full_sample_preserves_frobenius_norm():
    # l = k = k': Omega = D H / sqrt(k) is orthogonal
    rng = np.random.default_rng(3)
    A = rng.standard_normal((40, 128))
    Om = S.srht_omega(5, 128, 128)
    assert abs(np.linalg.norm(A @ Om) - np.linalg.norm(A)) <= 1e-12 * np.linalg.norm(A)


def test_samples_distinct_sorted_and_uniform():
    k, l, seeds = 100, 12, 400
    kp = S.next_pow2(k)
    counts = np.zeros(kp)
    plus = np.zeros(kp)
    for sd in range(seeds):
        s = S.srht_samples(sd, k, l)
        assert len(s) == l and np.all(np.diff(s) > 0) and s[0] >= 0 and s[-1] < kp
        counts[s] += 1
        plus += S.srht_signs(sd, k) > 0
    # each index drawn with probability l / k' (binomial, 400 trials): within 6 sd
    pr = l / kp
    sd_c = np.sqrt(seeds * pr * (1 - pr))
    assert np.max(np.abs(counts - seeds * pr)) <= 6 * sd_c
    assert np.max(np.abs(plus - seeds / 2)) <= 6 * np.sqrt(seeds / 4)


def test_sample_set_is_the_l_smallest_keys():
    # the set, not its construction: every unsampled key is at least the
    # largest sampled key (ties broken by index)
    k, l = 300, 37
    kp = S.next_pow2(k)
    u = S._words(9, kp, 2).astype(np.int64)
    s = S.srht_samples(9, k, l)
    chosen = np.zeros(kp, bool)
    chosen[s] = True
    worst = max((u[i], i) for i in s)
    assert all((u[i], i) > worst for i in np.nonzero(~chosen)[0])


def test_exact_recovery_through_range_finder():
    m, k, n, rk = 90, 200, 30, 15
    rng = np.random.default_rng(2)
    A = rng.standard_normal((m, rk)) @ rng.standard_normal((rk, k))
    B = rng.standard_normal((k, n))
    for q in (0, 1):
        out = L.lramm_forward(A, B, r=rk + 5, p=10, q=q, fmt=("fp64",) * 4, seed=4, sketch="srht")
        Qm = out["Q"]
        # rank(A) = 15 < l = 30: the sketch spans range(A); the extra Householder
        # columns are orthonormal completions
        assert np.linalg.norm(A - Qm @ (Qm.T @ A)) <= 1e-12 * np.linalg.norm(A)
        assert L.rel_fro(out["C"], A @ B) <= 1e-12


def test_srht_range_finder_close_to_gaussian():
    # same spectrum, same l: the two test matrices reach errors within a
    # small factor of each other and of the Eckart-Young floor
    m = k = 256
    A, sig = synth.lowrank(m, k, synth.spectrum("exp", 256, 12.0), 6)
    A = A.astype(np.float64)
    l = 50
    errs = {}
    for sk in ("gaussian", "srht"):
        out = L.lramm_forward(A, np.eye(k), r=40, p=10, q=0, fmt=("fp64",) * 4, seed=8, sketch=sk)
        Qm = out["Q"]
        errs[sk] = np.linalg.norm(A - Qm @ (Qm.T @ A))
    floor = L.tail(np.linalg.svd(A, compute_uv=False), l)
    for e in errs.values():
        assert floor <= e <= 30 * floor
    assert errs["srht"] <= 5 * errs["gaussian"]


def test_fp32_transform_exact_on_integers():
    # small integers: every partial sum of the butterflies is exact in binary32
    rng = np.random.default_rng(4)
    for k, l in ((7, 5), (100, 16), (1024, 64)):
        A = rng.integers(-50, 51, size=(9, k)).astype(np.float64)
        y32 = S.srht_sketch(A, 3, l, "fp32")
        y64 = S.srht_sketch(A, 3, l, "fp64")
        # both sides scale by 1/sqrt(l); compare before the (different) scalings
        sc = np.float32(1.0 / np.sqrt(np.float64(l)))
        assert np.array_equal(np.rint(y32 / np.float64(sc)), np.rint(y64 * np.sqrt(l)))


def test_fp32_transform_twice_is_kprime_times_input():
    rng = np.random.default_rng(5)
    X = rng.integers(-100, 101, size=(6, 256)).astype(np.float32)
    assert np.array_equal(S.fwht_fp32(S.fwht_fp32(X)), 256 * X)


def test_fp32_transform_within_rounding_bound():
    rng = np.random.default_rng(6)
    worst = 0.0
    for k, l in ((300, 40), (2048, 100), (5000, 272)):
        A = rng.standard_normal((12, k))
        A32 = A.astype(np.float32).astype(np.float64)
        y32 = S.srht_sketch(A32, 7, l, "fp32")
        y64 = S.srht_sketch(A32, 7, l, "fp64")
        p = int(np.log2(S.next_pow2(k)))
        bound = (p + 3) * 2.0**-24 * np.sum(np.abs(A32), axis=1)[:, None] / np.sqrt(l)
        err = np.abs(y32 - y64)
        assert np.all(err <= bound)
        worst = max(worst, float(np.max(err / bound)))
    assert worst > 1e-3          # binary32 rounding is really there
