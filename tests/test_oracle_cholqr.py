"""Pins of the oracle's one-pass Cholesky QR against facts it does not
compute itself: orthogonal columns (a Hadamard basis), the one-column closed
form, the Cholesky factor from LAPACK, Householder QR within the first-order
forward error of a Cholesky-based QR, the orthogonality bound of Yamamoto et
al. (2015, Thm. 3.3), the residual bound of the triangular solves, and the dropped set and span on exactly dependent
integer columns."""

import numpy as np
import pytest
from scipy.linalg import hadamard

from oracle.qr import cholesky_qr, householder_qr, householder_qr_dropping

U = 2.0**-53


def _tol(n):
    return 64.0 * n * U


def _with_singular_values(rng, m, n, s):
    P, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (P * s[None, :]) @ V.T


def test_orthogonal_columns_exact():
    H = hadamard(64)[:, :8] / 8.0            # orthonormal columns
    d = np.arange(1.0, 9.0)
    Q, R, dropped = cholesky_qr(H * d[None, :], _tol(8))
    assert dropped == []
    assert np.max(np.abs(Q - H)) <= 4 * U
    assert np.max(np.abs(R - np.diag(d))) <= 8 * U * d.max()


def test_one_column_closed_form():
    x = np.array([[3.0], [4.0], [12.0]])
    Q, R, _ = cholesky_qr(x, _tol(1))
    assert np.allclose(Q[:, 0], x[:, 0] / 13.0, rtol=0, atol=2 * U)
    assert abs(R[0, 0] - 13.0) <= 16 * U * 13.0


def test_factor_is_lapack_cholesky():
    rng = np.random.default_rng(3)
    Y = _with_singular_values(rng, 300, 40, np.logspace(0, -3, 40))
    _, R, _ = cholesky_qr(Y, _tol(40))
    Rl = np.linalg.cholesky(Y.T @ Y).T
    # same matrix factored twice: first-order error cond(G) u ||R||
    assert np.max(np.abs(R - Rl)) <= 64 * 40 * U * 1e6 * np.max(np.abs(Rl))


@pytest.mark.parametrize("m,n,cond", [(500, 30, 1e2), (2000, 64, 1e4), (1000, 100, 1e6)])
def test_orthogonality_bound_and_householder_agreement(m, n, cond):
    rng = np.random.default_rng(int(np.log10(cond)) + n)
    s = np.logspace(0, -np.log10(cond), n)
    Y = _with_singular_values(rng, m, n, s)
    Q, R, dropped = cholesky_qr(Y, _tol(n))
    assert dropped == []
    k2 = s[0] / s[-1]
    d = 8.0 * k2 * np.sqrt(m * n * U + n * (n + 1) * U)
    E = np.linalg.norm(Q.T @ Q - np.eye(n), 2)
    if d < 1.0:
        assert E <= 5.0 / 64.0 * d * d
    # first-order forward error against the unique positive-diagonal QR:
    # the Gram and the Cholesky perturb R^T R by eps ||Y||_F^2 (eps =
    # (m + n + 1) u), which moves Q by at most sqrt(n / 2) eps kF^2, kF =
    # ||Y||_F / sigma_min; Householder adds O(m n u cond); factor 2 for the
    # terms of second order
    # the triangular solves' backward error (Higham, Accuracy and Stability
    # of Numerical Algorithms, Thm. 8.5: (R + dR) q_i = y_i, |dR| <= gamma_n
    # |R|) bounds the residual row by row
    gn = n * U / (1 - n * U)
    assert np.linalg.norm(Y - Q @ R) <= gn * np.linalg.norm(Q) * np.linalg.norm(R)
    Qh, _ = householder_qr(Y)
    kF = np.linalg.norm(Y) / s[-1]
    eps = (m + n + 1) * U
    bound = 2.0 * (np.sqrt(n / 2.0) * eps * kF**2 + m * n * U * k2)
    assert np.linalg.norm(Q - Qh) <= bound
    # one pass is visibly less orthogonal than Householder at cond 1e6 (the
    # oracle really stops after the first factorisation)
    if cond >= 1e6:
        assert E > 1e3 * np.linalg.norm(Qh.T @ Qh - np.eye(n), 2)


def test_dependent_integer_columns():
    rng = np.random.default_rng(11)
    Y = rng.integers(-4, 5, size=(40, 8)).astype(np.float64)
    Y[:, 3] = Y[:, 0] + Y[:, 1]
    Y[:, 6] = 2.0 * Y[:, 2]
    Q, R, dropped = cholesky_qr(Y, _tol(8))
    assert dropped == [3, 6]
    _, _, dropped_h = householder_qr_dropping(Y, _tol(8))
    assert dropped == dropped_h
    kept = [0, 1, 2, 4, 5, 7]
    assert np.all(Q[:, dropped] == 0.0) and np.all(R[dropped, :] == 0.0)
    assert np.max(np.abs(Q[:, kept].T @ Q[:, kept] - np.eye(6))) <= 1e-13
    assert np.max(np.abs(Q @ (Q.T @ Y) - Y)) <= 1e-12 * np.max(np.abs(Y))
    # the kept columns are the one-pass QR of the kept columns of Y
    Qk, _, dk = cholesky_qr(Y[:, kept], _tol(8))
    assert dk == [] and np.max(np.abs(Qk - Q[:, kept])) <= 1e-14
