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

Pins (tests/test_oracle_qr.py): ||Q^T Q - I||_max <= 1e-13,
||QR - Y||_F <= 1e-14 ||Y||_F, R upper triangular with a non-negative
diagonal, agreement with LAPACK's QR after the same sign normalisation, and a
hand-worked 3x2 example.
"""

import numpy as np


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
