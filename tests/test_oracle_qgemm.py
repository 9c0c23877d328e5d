"""Pins of the oracle's quantised GEMM (paper Sec. 3.1, Alg. 2; Sec. 3.3 size
invariance; appendix Theorem 4.3).  CPU only."""

import numpy as np
import pytest

from oracle import qgemm as G
from oracle import quant as Q


def f32(x):
    return np.asarray(x, np.float32).astype(np.float64)


def test_int_gemm_matches_python_integers():
    rng = np.random.default_rng(0)
    for (M, K, N) in [(1, 1, 1), (3, 7, 5), (9, 33, 4)]:
        L = rng.integers(-127, 128, (M, K))
        R = rng.integers(-127, 128, (K, N))
        acc = G.int_gemm(L, R)
        for i in range(M):
            for j in range(N):
                s = 0
                for k in range(K):
                    s += int(L[i, k]) * int(R[k, j])
                assert acc[i, j] == s


def test_int_gemm_matches_int64_matmul():
    rng = np.random.default_rng(1)
    L = rng.integers(-127, 128, (70, 4100))
    R = rng.integers(-127, 128, (4100, 50))
    assert np.array_equal(G.int_gemm(L, R), L @ R)


def test_int32_accumulator_bound():
    K = 133145                      # 133145 * 127^2 > 2^31 - 1
    L = np.full((1, K), 127)
    R = np.full((K, 1), 127)
    with pytest.raises(OverflowError):
        G.int_gemm(L, R)
    G.int_gemm(L[:, :133144], R[:133144])     # the largest K that fits


def test_epilogue_matches_float32_arithmetic():
    rng = np.random.default_rng(2)
    acc = rng.integers(-2**30, 2**30, (17, 13))
    dL = f32(rng.uniform(1e-4, 1e-1, 17))
    dR = f32(rng.uniform(1e-4, 1e-1, 13))
    Cin = f32(rng.standard_normal((17, 13)))
    out = G.epilogue(acc, dL, dR, alpha=0.75, beta=-1.25, Cin=Cin)
    for i in range(17):
        for j in range(13):
            c = (np.float32(acc[i, j]) * np.float32(dL[i])) * np.float32(dR[j])
            o = np.float32(0.75) * c + np.float32(-1.25) * np.float32(Cin[i, j])
            assert out[i, j] == float(np.float32(o))


def test_qgemm_composes_alg2_steps():
    rng = np.random.default_rng(3)
    L = f32(rng.standard_normal((40, 96)))
    R = f32(rng.standard_normal((96, 24)))
    p = G.qgemm(L, R, "int8", parts=True)
    Lc, dL = Q.quantize_rows(L, "int8")
    Rc, dR = Q.quantize_cols(R, "int8")
    ref = (np.float32(Lc @ Rc) * np.float32(dL)[:, None]) * np.float32(dR)[None, :]
    assert np.array_equal(p["out"], ref.astype(np.float64))
    # the result approximates the exact product at int8 resolution
    assert np.linalg.norm(p["out"] - L @ R) / np.linalg.norm(L @ R) < 0.03


def test_transposed_product_same_codes_and_accumulator():
    # the transposed product quantises the same vectors (rows of L are the
    # columns of L^T), so codes, scales and the exact accumulator agree; the
    # dequantised values then differ only by the order of the two scale
    # products, at most one binary32 rounding apart
    rng = np.random.default_rng(4)
    L = f32(rng.standard_normal((30, 64)))
    R = f32(rng.standard_normal((64, 20)))
    a = G.qgemm(L, R, "int8", parts=True)
    b = G.qgemm(R.T, L.T, "int8", parts=True)
    assert np.array_equal(a["acc"], b["acc"].T)
    assert np.array_equal(a["dL"], b["dR"]) and np.array_equal(a["dR"], b["dL"])
    # applying the factors in the swapped order reproduces a exactly
    swapped = G.fl32(G.fl32(G.fl32(b["acc"].T.astype(np.float64)) * b["dR"][:, None]) * b["dL"][None, :])
    assert np.array_equal(a["out"], swapped)
    ulp = np.spacing(np.abs(a["out"]).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(a["out"] - b["out"].T) <= ulp)


def test_relative_error_size_invariance():
    """Sec. 3.3: for fixed distributions the quantised-GEMM relative error
    does not depend on m, n, k."""
    errs = []
    for s in (256, 512, 1024):
        rng = np.random.default_rng(s)
        A = f32(rng.standard_normal((s, s)))
        B = f32(rng.standard_normal((s, s)))
        C = G.qgemm(A, B, "int8")
        errs.append(np.linalg.norm(C - A @ B) / np.linalg.norm(A @ B))
    errs = np.array(errs)
    assert np.max(errs) / np.min(errs) < 1.15


def test_theorem_4_3_upper_bound():
    """E||C - C~||_F <= k (s1 / l2 sqrt(n) + g1 / l1 sqrt(m) + sqrt(mn) / (l1 l2))
    with per-tensor lambdas (loose bound; checked on one draw)."""
    rng = np.random.default_rng(5)
    m, k, n = 64, 128, 96
    A = f32(rng.uniform(-1, 1, (m, k)))
    B = f32(rng.uniform(-1, 1, (k, n)))
    Ac, dA = Q.quantize_tensor(A, "int8")
    Bc, dB = Q.quantize_tensor(B, "int8")
    Ct = (Ac * dA) @ (Bc * dB)
    l1 = 127 / np.max(np.abs(A))
    l2 = 127 / np.max(np.abs(B))
    s1 = np.linalg.norm(A, 2)
    g1 = np.linalg.norm(B, 2)
    bound = k * (s1 / l2 * np.sqrt(n) + g1 / l1 * np.sqrt(m) + np.sqrt(m * n) / (l1 * l2))
    assert np.linalg.norm(A @ B - Ct) <= bound


def test_fp8_and_bf16_products():
    rng = np.random.default_rng(6)
    L = f32(rng.standard_normal((20, 64)))
    R = f32(rng.standard_normal((64, 12)))
    ex = L @ R
    e8 = np.linalg.norm(G.qgemm(L, R, "fp8") - ex) / np.linalg.norm(ex)
    eb = np.linalg.norm(G.qgemm(L, R, "bf16") - ex) / np.linalg.norm(ex)
    ei8 = np.linalg.norm(G.qgemm(L, R, "int8") - ex) / np.linalg.norm(ex)
    ei4 = np.linalg.norm(G.qgemm(L, R, "int4") - ex) / np.linalg.norm(ex)
    assert eb < e8 < ei4 and eb < ei8 < ei4
    assert eb < 5e-3


def test_bf16_product_hand_worked():
    """bf16 operands are the inputs rounded to nearest-even on the 8-bit
    significand, multiplied exactly, unit scales: 1 + 2^-8 is a tie and
    rounds down to 1, 1 + 3 2^-8 a tie that rounds up to 1 + 2^-6, so
    [1 + 2^-8, 3] . [1 + 3 2^-8, 2^-9] = 1 + 2^-6 + 3 2^-9 = 1 + 11 2^-9
    (truncation would give 1 + 7 2^-9, no rounding 1 + 11 2^-9 + 3 2^-16)."""
    L = np.array([[1.0 + 2.0**-8, 3.0]])
    R = np.array([[1.0 + 3.0 * 2.0**-8], [2.0**-9]])
    out = G.qgemm(L, R, "bf16", parts=True)
    assert out["out"][0, 0] == 1.0 + 11.0 * 2.0**-9
    assert np.all(np.asarray(out["dL"]) == 1.0) and np.all(np.asarray(out["dR"]) == 1.0)
    # the transposed layout: R's column is the quantised vector, not its row
    assert G.qgemm(R.T, L.T, "bf16")[0, 0] == 1.0 + 11.0 * 2.0**-9


def test_fp8_product_hand_worked():
    """fp8 e4m3: each row (column) is scaled so that its largest magnitude
    maps to 448, rounded to the e4m3 grid, and dequantised by amax / 448.
    Row [448, -3.5] keeps its values (scale 1); column [0.25, 2.75] maps to
    0.25 * 448 / 2.75 = 40.73, whose e4m3 neighbours are 40 and 44 (step 4
    in [32, 64)), so 40, and to 448.  The exact code product is
    448 * 40 - 3.5 * 448 = 16352."""
    L = np.array([[448.0, -3.5]])
    R = np.array([[0.25], [2.75]])
    out = G.qgemm(L, R, "fp8", parts=True)
    assert [float(x) for x in np.asarray(out["Lq"]).ravel()] == [448.0, -3.5]
    assert [float(x) for x in np.asarray(out["Rq"]).ravel()] == [40.0, 448.0]
    assert float(np.asarray(out["dL"]).ravel()[0]) == 1.0
    assert float(np.asarray(out["dR"]).ravel()[0]) == float(np.float32(2.75) / np.float32(448.0))
    assert float(out["acc"][0, 0]) == 16352.0
    assert abs(out["out"][0, 0] - 16352.0 * 2.75 / 448.0) <= 2.0**-23 * 100.375 * 2
