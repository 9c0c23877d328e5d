"""Pins of the oracle's quantiser (paper Sec. 3.1; Theorems 4.1/4.2 of the
appendix) against hand-worked values, invariants and independent bit-level
constructions.  CPU only."""

import os
import struct

import numpy as np
import pytest

from oracle import quant as Q

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def f32(x):
    return np.asarray(x, np.float32).astype(np.float64)


def _hexf(h):
    return struct.unpack("<f", struct.pack("<I", int(h, 16)))[0]


def test_golden_examples():
    n = 0
    for line in open(os.path.join(GOLD, "quant_examples.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        fmt, vals, codes, d = [s.strip() for s in line.split("|")]
        v = f32([float(x) for x in vals.split()])
        c, dd = Q.quantize_rows(v[None, :], fmt)
        assert c[0].tolist() == [int(x) for x in codes.split()], line
        assert dd[0] == _hexf(d), line
        n += 1
    assert n == 4


def test_amax_maps_to_qmax_and_odd_symmetry():
    rng = np.random.default_rng(3)
    X = f32(rng.standard_normal((200, 97)) * np.exp(rng.uniform(-20, 20, (200, 1))))
    for fmt, qmax in (("int8", 127), ("int4", 7)):
        c, d = Q.quantize_rows(X, fmt)
        idx = np.argmax(np.abs(X), axis=1)
        top = c[np.arange(200), idx]
        assert np.all(np.abs(top) == qmax)
        assert np.all(np.sign(top) == np.sign(X[np.arange(200), idx]))
        cn, dn = Q.quantize_rows(-X, fmt)
        assert np.array_equal(cn, -c) and np.array_equal(dn, d)
        assert np.all(np.abs(c) <= qmax)


def test_power_of_two_scaling_invariance():
    rng = np.random.default_rng(4)
    X = f32(rng.standard_normal((50, 64)))
    c, d = Q.quantize_rows(X, "int8")
    for j in (-30, -3, 1, 17):
        cj, dj = Q.quantize_rows(X * 2.0**j, "int8")
        assert np.array_equal(cj, c)
        assert np.array_equal(dj, d * 2.0**j)


def test_elementwise_error_bound_and_theorem_4_2():
    rng = np.random.default_rng(5)
    X = f32(rng.uniform(-3, 3, (64, 300)))
    for fmt, qmax in (("int8", 127), ("int4", 7)):
        c, d = Q.quantize_rows(X, fmt)
        err = np.abs(X - c * d[:, None])
        assert np.all(err <= d[:, None] * (0.5 + 4 * qmax * 2.0**-24))
        # Theorem 4.2 (per-tensor form): ||A - A~||_F <= sqrt(mn) / lambda
        ct, dt = Q.quantize_tensor(X, fmt)
        lam = qmax / np.max(np.abs(X))
        assert np.linalg.norm(X - ct * dt) <= np.sqrt(X.size) / lam
        # Theorem 4.1: zero-mean error (RNE is unbiased on symmetric data)
        e = (X - c * d[:, None]) / d[:, None]
        assert abs(np.mean(e)) < 0.02


def test_requantise_is_idempotent():
    rng = np.random.default_rng(6)
    X = f32(rng.standard_normal((40, 128)))
    c, d = Q.quantize_rows(X, "int8")
    X2 = f32(c * d[:, None])
    c2, _ = Q.quantize_rows(X2, "int8")
    assert np.array_equal(c, c2)


def test_columns_are_transposed_rows():
    rng = np.random.default_rng(7)
    X = f32(rng.standard_normal((33, 20)))
    cc, dc = Q.quantize_cols(X, "int8")
    cr, dr = Q.quantize_rows(X.T, "int8")
    assert np.array_equal(cc, cr.T) and np.array_equal(dc, dr)


def test_non_finite_and_non_binary32_inputs_raise():
    with pytest.raises(ValueError):
        Q.quantize_rows(np.array([[1.0, np.nan]]), "int8")
    with pytest.raises(ValueError):
        Q.quantize_rows(np.array([[1.0, np.inf]]), "int8")
    with pytest.raises(ValueError):
        Q.quantize_rows(np.array([[0.1]]), "int8")      # 0.1 is not a binary32 value


def test_tiny_rows_quantise_to_zero():
    # amax so small that fl32(127 / amax) overflows -> zero codes, d = 0
    v = np.array([[2.0**-140, -2.0**-141]])
    c, d = Q.quantize_rows(v, "int8")
    assert c.tolist() == [[0, 0]] and d[0] == 0.0


def test_int4_packing_hand_worked():
    codes = np.array([[1, -1, 7, -7, 3]])
    p = Q.pack_int4(codes)
    # (1 | 0xF<<4) = 0xF1, (7 | 0x9<<4) = 0x97, (3 | 0<<4) = 0x03
    assert p.tolist() == [[0xF1, 0x97, 0x03]]
    assert np.array_equal(Q.unpack_int4(p, 5), codes)
    rng = np.random.default_rng(8)
    r = rng.integers(-7, 8, (9, 31))
    assert np.array_equal(Q.unpack_int4(Q.pack_int4(r), 31), r)


def _e4m3_grid():
    """All finite non-negative OCP e4m3 values from their bit patterns."""
    vals = []
    for e in range(16):
        for mnt in range(8):
            if e == 15 and mnt == 7:
                continue                     # the NaN pattern
            if e == 0:
                vals.append(mnt / 8.0 * 2.0**-6)
            else:
                vals.append((1 + mnt / 8.0) * 2.0 ** (e - 7))
    return np.array(sorted(set(vals)))


def test_e4m3_grid_and_ties():
    g = _e4m3_grid()
    assert g[-1] == 448.0 and len(g) == 127
    assert np.array_equal(Q.sat_rne_e4m3(g), g)
    assert np.array_equal(Q.sat_rne_e4m3(-g), -g)
    # midpoints go to the neighbour with an even mantissa
    lo, hi = g[:-1], g[1:]
    mid = (lo + hi) / 2
    r = Q.sat_rne_e4m3(mid)
    idx = np.arange(len(g))
    even = (idx % 8) % 2 == 0           # grid index parity == mantissa parity
    exp_ = np.where(even[:-1], lo, hi)
    assert np.array_equal(r, exp_)
    assert Q.sat_rne_e4m3(np.array([1e4, -500.0])).tolist() == [448.0, -448.0]


def test_bf16_matches_bit_rounding():
    rng = np.random.default_rng(9)
    x = rng.standard_normal(20000).astype(np.float32)
    # plant exact ties: low 16 bits = 0x8000
    b = x.view(np.uint32).copy()
    b[:1000] = (b[:1000] & 0xFFFF0000) | 0x8000
    x = b.view(np.float32)
    ref = []
    for v in x[:3000]:
        u = struct.unpack("<I", struct.pack("<f", float(v)))[0]
        keep, rest = u >> 16, u & 0xFFFF
        if rest > 0x8000 or (rest == 0x8000 and keep & 1):
            keep += 1
        ref.append(struct.unpack("<f", struct.pack("<I", keep << 16))[0])
    assert np.array_equal(Q.rne_bf16(x[:3000].astype(np.float64)), np.array(ref))
