"""Householder thin QR in FP64 -- TEST INFRASTRUCTURE ONLY.

The range finder of Sec. 2.2 needs a matrix Q with orthonormal columns that
spans the sketch Y.  The paper does not say how Q is formed (its CPU code used
Eigen); the oracle uses Householder reflections (Golub & Van Loan, Matrix
Computations, Sec. 5.2) and normalises signs so that diag(R) >= 0.  For a
full-column-rank Y the thin QR factorisation with positive diagonal is unique,
so any other backward-stable method (the GPU's Cholesky-based one) computes
the same Q up to rounding of order cond(Y) * 2^-53, without sharing an
algorithm with this one.

Rank-deficient Y: a column whose remaining norm is exactly zero gets no
reflector (R_jj = 0) and Q keeps the corresponding identity column pushed
through the later reflectors, so Q stays orthonormal.

Rank-deficient Y, second convention (``householder_qr_dropping``, used to
compare with the GPU's CholeskyQR, which zeroes the Q column of a pivot that
falls below 64 l 2^-53 times its Gram diagonal): a column whose unexplained
part is that small is left out entirely, so the kept columns are the QR of
the kept columns of Y and the dropped ones are zero.

Pins (tests/test_oracle_qr.py): ||Q^T Q - I||_max <= 1e-13,
||QR - Y||_F <= 1e-14 ||Y||_F, R upper triangular with a non-negative
diagonal, agreement with LAPACK's QR after the same sign normalisation, and a
hand-worked 3x2 example.
"""

import numpy as np


def householder_qr_dropping(Y, tol):
    """Thin QR that leaves out numerically dependent columns.

    Column j of Y is dependent when, after the reflectors of the columns kept
    before it, the part of it not yet in their span has squared norm at most
    ``tol`` times its own squared norm (R_jj^2 <= tol * ||y_j||^2, the same
    test as a Cholesky pivot against its Gram diagonal).  A dependent column
    gets no reflector and a zero column in Q (and a zero row in R); the kept
    columns of Q are the thin QR factor (positive diagonal) of the kept
    columns of Y, so span(Q) = span(Y) and Q Q^T is the projector onto it.
    Returns Q (m x n), R (n x n) and the list of dropped column indices."""
    W = np.array(Y, dtype=np.float64, copy=True)
    m, n = W.shape
    if n > m:
        raise ValueError("thin QR needs at least as many rows as columns")
    colnorm2 = np.sum(W * W, axis=0)
    vs, kept, dropped = [], [], []
    R = np.zeros((n, n))
    row = 0                                   # next reflector row
    for j in range(n):
        x = W[row:, j]
        r2 = float(np.dot(x, x))
        if r2 <= tol * colnorm2[j] or row >= m:
            dropped.append(j)
            continue
        normx = np.sqrt(r2)
        alpha = -normx if x[0] >= 0 else normx
        v = x.copy()
        v[0] -= alpha
        v /= np.sqrt(np.dot(v, v))
        W[row:, j:] -= 2.0 * np.outer(v, v @ W[row:, j:])
        vs.append((row, v))
        kept.append(j)
        row += 1
    nk = len(kept)
    Qk = np.zeros((m, nk))
    Qk[:nk, :nk] = np.eye(nk)
    for (r0, v) in reversed(vs):
        Qk[r0:, :] -= 2.0 * np.outer(v, v @ Qk[r0:, :])
    Rk = W[:nk, :]                            # rows of the kept reflectors, all columns
    s = np.sign(np.array([Rk[i, kept[i]] for i in range(nk)]))
    s[s == 0] = 1.0
    Qk = Qk * s[None, :]
    Rk = Rk * s[:, None]
    Q = np.zeros((m, n))
    for i, j in enumerate(kept):
        Q[:, j] = Qk[:, i]
        R[j, :] = np.where(np.arange(n) >= j, Rk[i, :], 0.0)
    return Q, R, dropped


def householder_qr(Y):
    """Thin QR of an m x n matrix (m >= n): returns Q (m x n), R (n x n)."""
    W = np.array(Y, dtype=np.float64, copy=True)
    m, n = W.shape
    if n > m:
        raise ValueError("thin QR needs at least as many rows as columns")
    vs = []
    for j in range(n):
        x = W[j:, j]
        normx = np.sqrt(np.dot(x, x))
        if normx == 0.0:
            vs.append(None)
            continue
        alpha = -normx if x[0] >= 0 else normx
        v = x.copy()
        v[0] -= alpha
        vnorm = np.sqrt(np.dot(v, v))
        if vnorm == 0.0:
            vs.append(None)
            continue
        v /= vnorm
        # apply H = I - 2 v v^T to the trailing columns
        W[j:, j:] -= 2.0 * np.outer(v, v @ W[j:, j:])
        vs.append(v)
    R = np.triu(W[:n, :])
    Q = np.zeros((m, n))
    Q[:n, :n] = np.eye(n)
    for j in reversed(range(n)):
        v = vs[j]
        if v is None:
            continue
        Q[j:, :] -= 2.0 * np.outer(v, v @ Q[j:, :])
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :], R * s[:, None]
