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


def test_dropping_qr_equals_plain_qr_at_full_rank():
    """With no dependent column the dropping variant is the plain QR."""
    from oracle.qr import householder_qr_dropping
    rng = np.random.default_rng(3)
    for (m, n, cond) in [(200, 40, 1.0), (300, 60, 1e4)]:
        U, _ = np.linalg.qr(rng.standard_normal((m, n)))
        V, _ = np.linalg.qr(rng.standard_normal((n, n)))
        Y = (U * np.logspace(0, -np.log10(cond), n)) @ V.T
        Q, R, dropped = householder_qr_dropping(Y, 64 * n * 2.0**-53)
        Qh, Rh = householder_qr(Y)
        assert dropped == []
        assert np.max(np.abs(Q - Qh)) <= 1e-14 * cond
        assert np.max(np.abs(np.diag(R) - np.diag(Rh))) <= 1e-13 * np.max(np.abs(Rh))


def test_dropping_qr_on_exactly_dependent_columns():
    """Columns that are exact integer combinations of earlier ones (and a
    zero column) are dropped; the kept columns of Q are LAPACK's thin QR of
    the kept columns of Y (signs fixed), the dropped ones are zero, and
    Q Q^T is the projector onto range(Y)."""
    from oracle.qr import householder_qr_dropping
    rng = np.random.default_rng(4)
    Y = rng.integers(-5, 6, (50, 8)).astype(np.float64)
    Y[:, 2] = Y[:, 0] + 2.0 * Y[:, 1]
    Y[:, 5] = 0.0
    Y[:, 7] = 3.0 * Y[:, 3] - Y[:, 6]
    Q, R, dropped = householder_qr_dropping(Y, 64 * 8 * 2.0**-53)
    assert dropped == [2, 5, 7]
    kept = [0, 1, 3, 4, 6]
    Ql, Rl = np.linalg.qr(Y[:, kept])
    Ql = Ql * np.sign(np.diag(Rl))[None, :]
    assert np.max(np.abs(Q[:, kept] - Ql)) <= 1e-14
    assert not Q[:, dropped].any()
    assert np.linalg.norm(Q @ (Q.T @ Y) - Y) <= 1e-13 * np.linalg.norm(Y)
    assert np.max(np.abs(Q[:, kept].T @ Q[:, kept] - np.eye(len(kept)))) <= 1e-14
