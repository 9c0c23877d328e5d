"""Pins of the oracle's Householder QR (range-finder orthonormalisation,
paper Sec. 2.2) against invariants, LAPACK and a hand-worked example."""

import os

import numpy as np

from oracle.qr import householder_qr

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_blocks(path):
    blocks, cur, name = {}, None, None
    for line in open(path):
        s = line.strip()
        if not s or s.startswith("#"):
            continue
        if s.isalpha():
            name, cur = s, []
            blocks[name] = cur
        else:
            cur.append([float(x) for x in s.split()])
    return {k: np.array(v) for k, v in blocks.items()}


def test_hand_worked_3x2():
    b = _read_blocks(os.path.join(GOLD, "qr_3x2.txt"))
    Qh, Rh = householder_qr(b["Y"])
    assert np.allclose(Qh, b["Q"], atol=1e-15, rtol=0)
    assert np.allclose(Rh, b["R"], atol=1e-14, rtol=0)


def _check(Y, tol_orth=1e-13):
    Qh, Rh = householder_qr(Y)
    n = Y.shape[1]
    assert np.max(np.abs(Qh.T @ Qh - np.eye(n))) <= tol_orth
    assert np.linalg.norm(Qh @ Rh - Y) <= 1e-14 * np.linalg.norm(Y)
    assert np.array_equal(Rh, np.triu(Rh))
    assert np.all(np.diag(Rh) >= 0)
    return Qh, Rh


def test_invariants_and_lapack_agreement():
    rng = np.random.default_rng(0)
    for (m, n, cond) in [(300, 50, 1.0), (500, 74, 1e3), (257, 40, 1e6)]:
        U, _ = np.linalg.qr(rng.standard_normal((m, n)))
        V, _ = np.linalg.qr(rng.standard_normal((n, n)))
        s = np.logspace(0, -np.log10(cond), n)
        Y = (U * s) @ V.T
        Qh, Rh = _check(Y)
        Ql, Rl = np.linalg.qr(Y)
        sg = np.sign(np.diag(Rl))
        Ql, Rl = Ql * sg, Rl * sg[:, None]
        assert np.max(np.abs(Qh - Ql)) <= 1e-14 * cond * 50
        assert np.max(np.abs(Rh - Rl)) <= 1e-13 * np.max(np.abs(Rl)) * 50


def test_rank_deficient_stays_orthonormal():
    rng = np.random.default_rng(1)
    Y = rng.standard_normal((60, 10))
    Y[:, 3] = 0.0
    Y[:, 7] = Y[:, 1]
    Qh, Rh = householder_qr(Y)
    assert np.max(np.abs(Qh.T @ Qh - np.eye(10))) <= 1e-13
    assert np.linalg.norm(Qh @ Rh - Y) <= 1e-14 * np.linalg.norm(Y)
    assert Rh[3, 3] == 0.0 and abs(Rh[7, 7]) < 1e-13
