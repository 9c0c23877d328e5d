"""Pins of the oracle's one-sided LRAMM (paper Sec. 2.2 range finder / Alg. 1,
Sec. 3.2 chained quantised products, Sec. 3.3 error statements) against
closed forms, brute force and library routines.  CPU only."""

import math
import struct

import numpy as np
import pytest

import synth
from oracle import lramm as L
from oracle.qr import householder_qr


def _lowrank(m, k, sig, seed):
    A, s = synth.lowrank(m, k, sig, seed)
    return A.astype(np.float64), s


def test_exact_recovery_when_rank_at_most_l():
    m, k, n = 120, 110, 90
    sig = np.concatenate([np.linspace(3, 1, 20), np.zeros(90)])
    rng = np.random.default_rng(0)
    U, _ = np.linalg.qr(rng.standard_normal((m, 20)))
    V, _ = np.linalg.qr(rng.standard_normal((k, 20)))
    A = (U * sig[:20]) @ V.T
    B = rng.standard_normal((k, n))
    for q in (0, 1):
        out = L.lramm_forward(A, B, r=20, p=5, q=q, fmt=("fp64",) * 4, seed=3)
        Qm = out["Q"]
        assert np.linalg.norm(A - Qm @ (Qm.T @ A)) / np.linalg.norm(A) <= 1e-12
        assert L.rel_fro(out["C"], A @ B) <= 1e-12
        assert np.max(np.abs(Qm.T @ Qm - np.eye(25))) <= 1e-13


def test_eckart_young_floor():
    m = k = 200
    A, s = _lowrank(m, k, synth.spectrum("exp", 200, 15.0), 1)
    sv = np.linalg.svd(A, compute_uv=False)
    for q in (0, 1):
        for seed in range(5):
            out = L.lramm_forward(A, np.eye(k), r=30, p=6, q=q, fmt=("fp64",) * 4, seed=seed)
            Qm = out["Q"]
            res = np.linalg.norm(A - Qm @ (Qm.T @ A))
            assert res >= L.tail(sv, 36) * (1 - 1e-10)


def test_halko_average_case_bound_q0():
    """Halko, Martinsson, Tropp (2011), Thm 10.5: for a Gaussian sketch with
    r + p columns, E||A - QQ^T A||_F <= (1 + r/(p-1))^(1/2) (sum_{j>r} s_j^2)^(1/2)."""
    m = k = 160
    A, _ = _lowrank(m, k, synth.spectrum("pow", 160, 1.0), 2)
    sv = np.linalg.svd(A, compute_uv=False)
    r, p = 20, 5
    res = []
    for seed in range(24):
        out = L.lramm_forward(A, np.eye(k), r=r, p=p, q=0, fmt=("fp64",) * 4, seed=100 + seed)
        Qm = out["Q"]
        res.append(np.linalg.norm(A - Qm @ (Qm.T @ A)))
    assert np.mean(res) <= math.sqrt(1 + r / (p - 1)) * L.tail(sv, r)


def test_paper_rsvd_spectral_bound():
    """Paper eq. (rsvderror) / Theorem 3.2 (appendix): with a rank-2k
    factorisation, E||A - A_r|| <= [1 + 4 sqrt(2 min(m,n)/(k-1))]^(1/(2q+1)) s_{k+1}."""
    m = k = 150
    A, _ = _lowrank(m, k, synth.spectrum("exp", 150, 20.0), 3)
    sv = np.linalg.svd(A, compute_uv=False)
    kk = 15
    for q in (0, 1, 2):
        res = []
        for seed in range(10):
            out = L.lramm_forward(A, np.eye(k), r=kk, p=kk, q=q, fmt=("fp64",) * 4, seed=seed)
            Qm = out["Q"]
            res.append(np.linalg.norm(A - Qm @ (Qm.T @ A), 2))
        bound = (1 + 4 * math.sqrt(2 * min(m, k) / (kk - 1))) ** (1 / (2 * q + 1)) * sv[kk]
        assert np.mean(res) <= bound


def test_brute_force_full_svd_64():
    """64 x 64: with l = 64 the basis is complete and LRAMM equals A B; with a
    gapped spectrum and many power iterations the QB residual equals the
    truncated-SVD residual from LAPACK (Eckart-Young, Sec. 2.1)."""
    rng = np.random.default_rng(4)
    A = rng.standard_normal((64, 64))
    B = rng.standard_normal((64, 64))
    out = L.lramm_forward(A, B, r=60, p=4, q=0, fmt=("fp64",) * 4, seed=1)
    assert L.rel_fro(out["C"], A @ B) <= 1e-12
    U, _ = np.linalg.qr(rng.standard_normal((64, 64)))
    V, _ = np.linalg.qr(rng.standard_normal((64, 64)))
    s = np.concatenate([np.linspace(1.0, 0.5, 16), np.linspace(1e-3, 1e-4, 48)])
    Ag = (U * s) @ V.T
    out = L.lramm_forward(Ag, np.eye(64), r=12, p=4, q=12, fmt=("fp64",) * 4, seed=2)
    Qm = out["Q"]
    res = np.linalg.norm(Ag - Qm @ (Qm.T @ Ag))
    sv = np.linalg.svd(Ag, compute_uv=False)
    assert abs(res - L.tail(sv, 16)) <= 1e-10 * L.tail(sv, 16)


def test_error_falls_with_precision():
    A, s = _lowrank(256, 256, synth.spectrum("exp", 256, 24.0), 5)
    B = synth.gaussian(256, 192, 105).astype(np.float64)
    om = synth.omega(256, 60, 6).astype(np.float64)
    ref = L.lramm_forward(A, B, 50, 10, 1, ("fp64",) * 4, omega=om)["C"]
    errs = []
    for f in ("int4", "int8", "bf16"):
        C = L.lramm_forward(A, B, 50, 10, 1, (f,) * 4, omega=om)["C"]
        errs.append(L.rel_fro(C, ref))
    assert errs[0] > errs[1] > errs[2] > 0
    assert errs[2] < 1e-2 and errs[1] < 5e-2


def test_alpha_beta_applied_to_final_product():
    A, _ = _lowrank(64, 64, synth.spectrum("exp", 64, 8.0), 6)
    B = synth.gaussian(64, 40, 7).astype(np.float64)
    Cin = synth.gaussian(64, 40, 8).astype(np.float64)
    om = synth.omega(64, 20, 9).astype(np.float64)
    base = L.lramm_forward(A, B, 16, 4, 0, omega=om)["C"]
    ab = L.lramm_forward(A, B, 16, 4, 0, omega=om, alpha=0.5, beta=2.0, Cin=Cin)["C"]
    ref = (np.float32(0.5) * base.astype(np.float32)) + np.float32(2.0) * Cin.astype(np.float32)
    assert np.array_equal(ab, ref.astype(np.float64))


def test_argument_errors():
    A = np.zeros((10, 8))
    B = np.zeros((8, 5))
    with pytest.raises(ValueError):
        L.lramm_forward(A, B, 8, 1, 0, seed=0)          # l > min(m, k)
    with pytest.raises(ValueError):
        L.lramm_forward(A, B, 2, 1, 0, omega=np.zeros((8, 4)))
    with pytest.raises(ValueError):
        L.lramm_forward(A, np.zeros((7, 5)), 2, 1, 0, seed=0)


# ---------------------------------------------------------------------------
# brute force on a tiny case: pure Python floats/ints, binary32 rounding via
# struct, Gram-Schmidt QR -- no numpy in the arithmetic, no oracle code.

def _r32(x):
    return struct.unpack("<f", struct.pack("<f", x))[0]


def _quant(v, qmax=127):
    amax = max(abs(x) for x in v)
    if amax == 0:
        return [0] * len(v), 0.0
    lam = _r32(qmax / amax)
    return [max(-qmax, min(qmax, round(_r32(x * lam)))) for x in v], _r32(amax / qmax)


def _qmm(Lm, Rm, qmax=127):
    M, K, N = len(Lm), len(Rm), len(Rm[0])
    lq = [_quant(row, qmax) for row in Lm]
    rq = [_quant([Rm[t][j] for t in range(K)], qmax) for j in range(N)]
    out = []
    for i in range(M):
        row = []
        for j in range(N):
            acc = sum(lq[i][0][t] * rq[j][0][t] for t in range(K))
            row.append(_r32(_r32(_r32(float(acc)) * lq[i][1]) * rq[j][1]))
        out.append(row)
    return out


def _gs(Y):
    m, n = len(Y), len(Y[0])
    cols = [[Y[i][j] for i in range(m)] for j in range(n)]
    qs = []
    for c in cols:
        v = list(c)
        for _ in range(2):                      # classical GS, twice
            for qv in qs:
                d = sum(a * b for a, b in zip(qv, v))
                v = [a - d * b for a, b in zip(v, qv)]
        nv = math.sqrt(sum(a * a for a in v))
        qs.append([a / nv for a in v])
    return [[qs[j][i] for j in range(n)] for i in range(m)]


def _T(M):
    return [list(r) for r in zip(*M)]


def _f32m(M):
    return [[_r32(x) for x in r] for r in M]


def test_tiny_chain_against_pure_python():
    rng = np.random.default_rng(11)
    m, k, n, l = 9, 8, 7, 3
    A = np.float32(rng.standard_normal((m, k)) * np.exp(-np.arange(k) / 2.0)).astype(np.float64)
    B = np.float32(rng.standard_normal((k, n))).astype(np.float64)
    om = np.float32(rng.standard_normal((k, l))).astype(np.float64)
    out = L.lramm_forward(A, B, 2, 1, 1, ("int8",) * 4, omega=om)

    Al, Bl, Ol = A.tolist(), B.tolist(), om.tolist()
    Y = _qmm(Al, Ol)
    Qm = _gs(Y)
    Z = _qmm(_T(Al), _f32m(Qm))
    QZ = _gs(Z)
    Y = _qmm(Al, _f32m(QZ))
    Qm = _gs(Y)
    Bt = _qmm(_T(_f32m(Qm)), Al)
    T = _qmm(Bt, Bl)
    C = _qmm(_f32m(Qm), T)
    assert np.array_equal(out["Bt"], np.array(Bt))
    assert np.array_equal(out["T"], np.array(T))
    assert np.array_equal(out["C"], np.array(C))


def test_tiny_mixed_format_chain_against_pure_python():
    """The stage-to-format mapping: the sketch products in the first format,
    the power step's A^T Q and the projection in the second, G1 in the third,
    G2 in the fourth.  With int4 (q_max 7) and int8 (127) alternating, any
    stage that took another stage's format changes its codes."""
    rng = np.random.default_rng(12)
    m, k, n, l = 9, 8, 7, 3
    A = np.float32(rng.standard_normal((m, k)) * np.exp(-np.arange(k) / 2.0)).astype(np.float64)
    B = np.float32(rng.standard_normal((k, n))).astype(np.float64)
    om = np.float32(rng.standard_normal((k, l))).astype(np.float64)
    for fmt in (("int4", "int8", "int4", "int8"), ("int8", "int4", "int8", "int4")):
        qs, qp, q1, q2 = (7 if f == "int4" else 127 for f in fmt)
        out = L.lramm_forward(A, B, 2, 1, 1, fmt, omega=om)
        Al, Bl, Ol = A.tolist(), B.tolist(), om.tolist()
        Y = _qmm(Al, Ol, qs)
        Qm = _gs(Y)
        Z = _qmm(_T(Al), _f32m(Qm), qp)
        QZ = _gs(Z)
        Y = _qmm(Al, _f32m(QZ), qs)
        Qm = _gs(Y)
        Bt = _qmm(_T(_f32m(Qm)), Al, qp)
        T = _qmm(Bt, Bl, q1)
        C = _qmm(_f32m(Qm), T, q2)
        assert np.array_equal(out["Bt"], np.array(Bt)), fmt
        assert np.array_equal(out["T"], np.array(T)), fmt
        assert np.array_equal(out["C"], np.array(C)), fmt


def test_exact_recovery_with_dropped_sketch_columns():
    """rank(A) = 40 < l = 74: with the dropping orthonormalisation the sketch
    columns past the rank are dropped (zero Q columns, l - 40 of them in
    every orthonormalisation), Q still spans range(A), and the unquantised
    product recovers A B to 1e-12 (exact recovery)."""
    m = k = n = 256
    rng = np.random.default_rng(8)
    U, V = synth.haar(m, 40, rng), synth.haar(k, 40, rng)
    A = (U * synth.spectrum("exp", 40, 10.0)[None, :]) @ V.T      # rank 40 exactly, kept in FP64
    B = synth.gaussian(k, n, 108).astype(np.float64)
    om = synth.omega(k, 74, 9).astype(np.float64)
    ref = L.lramm_forward(A, B, 64, 10, 1, ("fp64",) * 4, omega=om, drop_dependent=True)
    assert all(len(d) == 74 - 40 for d in ref["dropped"])
    assert all(d == list(range(40, 74)) for d in ref["dropped"])
    Q = ref["Q"]
    assert not Q[:, 40:].any()
    assert L.rel_fro(Q @ (Q.T @ A), A) <= 1e-12
    assert L.rel_fro(ref["C"], A @ B) <= 1e-12
