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

One pass of Cholesky QR (``cholesky_qr``, the cheaper orthonormalisation a
plan may ask for instead of the two-pass one): R from the Cholesky factor of
the Gram matrix Y^T Y, Q = Y R^-1, with the same dependent-column rule (a
pivot at most tol times its Gram diagonal drops the column: zero row of R,
zero column of Q, no part in later eliminations).  Its Q spans range(Y) but
is orthonormal only to about 2^-53 cond(Y)^2; Yamamoto, Nakatsukasa,
Yanagisawa and Fukaya (2015, Thm. 3.3) bound ||Q^T Q - I||_2 by (5/64) d^2,
d = 8 cond_2(Y) sqrt(m n u + n (n + 1) u), u = 2^-53, whenever d < 1.

Pins (tests/test_oracle_qr.py): ||Q^T Q - I||_max <= 1e-13,
||QR - Y||_F <= 1e-14 ||Y||_F, R upper triangular with a non-negative
diagonal, agreement with LAPACK's QR after the same sign normalisation, and a
hand-worked 3x2 example; for ``cholesky_qr`` (tests/test_oracle_cholqr.py):
exact on orthogonal columns, x / ||x|| for one column, Q^T Q - I within the
bound above, agreement with Householder QR within its first-order forward
error, and the dropped set and span of exactly dependent integer columns.
"""

import numpy as np
from scipy.linalg import solve_triangular


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


def cholesky_qr(Y, tol):
    """One pass of Cholesky QR in FP64: G = Y^T Y; the column-by-column
    Cholesky G = R^T R (pivot j: the Schur complement entry S_jj, accepted
    when it exceeds tol * G_jj, else column j is dropped and eliminates
    nothing); Q = Y R^-1 on the kept columns.  Returns Q (m x n), R (n x n)
    and the list of dropped column indices."""
    Y = np.asarray(Y, dtype=np.float64)
    m, n = Y.shape
    if n > m:
        raise ValueError("thin QR needs at least as many rows as columns")
    G = Y.T @ Y
    S = G.copy()
    R = np.zeros((n, n))
    dropped = []
    for j in range(n):
        piv = S[j, j]
        if not piv > tol * G[j, j]:
            dropped.append(j)
            continue
        R[j, j:] = S[j, j:] / np.sqrt(piv)
        S[j + 1:, j + 1:] -= np.outer(R[j, j + 1:], R[j, j + 1:])
    kept = [j for j in range(n) if j not in dropped]
    Q = np.zeros((m, n))
    if kept:
        Rk = R[np.ix_(kept, kept)]
        # Q_k R_k = Y_k: one triangular solve per row of Y (R_k^T q = y)
        Q[:, kept] = solve_triangular(Rk, Y[:, kept].T, trans="T", lower=False).T
    return Q, R, dropped
