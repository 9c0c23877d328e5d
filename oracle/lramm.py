"""One-sided LRAMM pipeline, frozen-Q backward and error metrics (FP64)
-- TEST INFRASTRUCTURE ONLY.

What is computed (paper references):
  * range finder (Sec. 2.2, two-stage method; Alg. 1's first step B <- Q* A):
    Y = A Omega with a Gaussian k x l test matrix, l = r + p, then Q = qr(Y)
    (Householder, or one pass of Cholesky QR when asked);
  * power (subspace) iterations, q of them (the paper's exponent q of
    Sec. 3.3 / eq. rsvderror; the procedure is the randomised subspace
    iteration of Halko, Martinsson & Tropp 2011, Alg. 4.4, which
    re-orthonormalises after every product):
        Z = A^T Q, Q_Z = qr(Z), Y = A Q_Z, Q = qr(Y);
  * projection B~ = Q^T A (Alg. 1, first line);
  * chained quantised products (Sec. 3.2, C = QM(QM(...))): T = QM(B~ B) and
    C = QM(Q T); every product is Alg. 2 (qgemm.py).  The product is formed as
    Q (B~ B), never (Q B~) B, which would be an m x k dense intermediate.
  * alpha/beta of Alg. 2 / Alg. 3 are applied to the final product only.

Every operand that enters a quantiser is binary32: the FP64 Q of the QR is
rounded once to binary32 (fl32(Q)) before quantisation; the products Y, Z,
B~ and T are binary32 outputs of the dequantising epilogue.

Stage formats: ``fmt`` = (sketch, proj, g1, g2).  ``sketch`` is used for
Y = A Omega and Y = A Q_Z, ``proj`` for Z = A^T Q and B~ = Q^T A, ``g1`` for
T = B~ B and ``g2`` for C = Q T.  ``"fp64"`` means no quantisation (the
paper's unquantised RSVD): an FP64 product, not rounded.

Rank: 1 <= l <= min(m, k).  No truncation back to r: the factorisation kept
is the rank-l QB form for which Halko's bounds are stated.

Backward (frozen Q, straight-through quantisation): the surrogate is
C = Q Q^T A B, so dA = Q Q^T dC B^T and dB = A^T Q Q^T dC, in FP64.

Pins: tests/test_oracle_lramm.py (exact recovery when rank(A) <= l, the
Eckart-Young floor, Halko's average-case bound, the brute-force 64 x 64 SVD
check, reduction to Alg. 2 when l = m = k, the chain's agreement with a
direct evaluation of Q(Q^T A)B, monotone convergence in bit width, pure
Python brute-force chains in one format and with int4 / int8 alternating
over the stages) and
tests/test_oracle_backward.py (central finite differences of the bilinear
surrogate).
"""

import numpy as np

from .quant import fl32
from .qgemm import qgemm
from .qr import cholesky_qr, householder_qr, householder_qr_dropping
from .philox import gaussian_omega
from .srht import srht_omega, srht_sketch

FORMATS = ("int8", "int4", "fp8", "bf16", "fp64")


def _product(L, R, fmt):
    """One stage product in the given format; returns binary32 (or FP64 for
    the unquantised format) values as float64."""
    if fmt == "fp64":
        return np.asarray(L, np.float64) @ np.asarray(R, np.float64)
    return qgemm(fl32(L), fl32(R), fmt)


def _q_operand(Q, fmt):
    """The operand form of an orthonormal factor: fl32 for quantised stages."""
    return Q if fmt == "fp64" else fl32(Q)


def range_finder(A, l, q, fs, fp, omega, drop_dependent=False, out=None, keep=True, y0=None, one_pass=False):
    """Q with l orthonormal columns spanning the sketch of A (Sec. 2.2,
    first stage): Y = A Omega in format fs (or y0 when given: the structured
    sketch, formed without operand codes), Q = qr(Y), then q subspace
    iterations Z = A^T Q (format fp), Q_Z = qr(Z), Y = A Q_Z (fs), Q = qr(Y).
    Intermediates go into ``out`` (when given, with ``keep``).  With
    ``one_pass`` every qr is one pass of Cholesky QR (qr.cholesky_qr, which
    drops dependent columns by the same rule) instead of Householder.
    Returns (Q, R) of the last orthonormalisation."""
    if out is None:
        out = {}
    tol = 64.0 * l * 2.0**-53

    def orth(X):
        if one_pass:
            Qd, Rd, dropped = cholesky_qr(X, tol)
            out.setdefault("dropped", []).append(dropped)
            return Qd, Rd
        if drop_dependent:
            Qd, Rd, dropped = householder_qr_dropping(X, tol)
            out.setdefault("dropped", []).append(dropped)
            return Qd, Rd
        return householder_qr(X)

    Y = _product(A, omega, fs) if y0 is None else y0
    Q, R = orth(Y)
    if keep:
        out.update(omega=omega, Y0=Y, Q0=Q)
    for it in range(q):
        Z = _product(A.T, _q_operand(Q, fp), fp)
        QZ, _ = orth(Z)
        Y = _product(A, _q_operand(QZ, fs), fs)
        Q, R = orth(Y)
        if keep:
            out[f"Z{it + 1}"] = Z
            out[f"QZ{it + 1}"] = QZ
            out[f"Y{it + 1}"] = Y
            out[f"Q{it + 1}"] = Q
    out["Y"] = Y
    return Q, R


def lramm_forward(A, B, r, p, q, fmt=("int8",) * 4, omega=None, seed=None,
                  alpha=1.0, beta=0.0, Cin=None, keep=True, drop_dependent=False, sketch="gaussian",
                  one_pass=False):
    """One-sided LRAMM.  A: m x k, B: k x n (binary32 values unless every
    stage is fp64).  Returns a dict with C and, with ``keep``, every
    intermediate (Omega, Y, Q, B~, T, and the power-iteration Z / Q_Z).

    ``sketch``: "gaussian" (Omega given or drawn from the seed, the first
    sketch in the sketch format) or "srht" (the structured test matrix of
    srht.py drawn from the seed: the first sketch is its FP64 product when the
    sketch format is "fp64", else its binary32 transform).

    ``drop_dependent``: orthonormalise with ``householder_qr_dropping`` at
    tolerance 64 l 2^-53 (a sketch column that the earlier ones already span
    to that accuracy gets a zero Q column instead of a completion vector);
    the basis then spans exactly the kept sketch columns.  This is the reading
    used for rank(A) < l, where the completion vectors of a plain Householder
    QR are arbitrary directions outside range(A) and would change the row
    scales of Q.

    ``one_pass``: orthonormalise with one pass of Cholesky QR (Q = Y R^-1,
    R the Cholesky factor of Y^T Y, same dropping rule): the cheaper basis,
    orthonormal only to about 2^-53 cond(Y)^2."""
    A = np.asarray(A, np.float64)
    B = np.asarray(B, np.float64)
    m, k = A.shape
    k2, n = B.shape
    if k2 != k:
        raise ValueError("inner dimensions differ")
    l = r + p
    if not (1 <= l <= min(m, k)):
        raise ValueError("need 1 <= r + p <= min(m, k)")
    fs, fp, f1, f2 = fmt
    for f in fmt:
        if f not in FORMATS:
            raise ValueError(f"unknown format {f!r}")
    y0 = None
    if sketch == "srht":
        if omega is not None or seed is None:
            raise ValueError("the structured sketch is drawn from the seed")
        omega = srht_omega(seed, k, l)
        y0 = srht_sketch(A, seed, l, "fp64" if fs == "fp64" else "fp32")
    elif sketch != "gaussian":
        raise ValueError(f"unknown sketch {sketch!r}")
    if omega is None:
        if seed is None:
            raise ValueError("pass omega or seed")
        omega = gaussian_omega(seed, k, l)
    omega = np.asarray(omega, np.float64)
    if omega.shape != (k, l):
        raise ValueError("omega must be k x l")

    out = {"l": l}
    Q, R = range_finder(A, l, q, fs, fp, omega, drop_dependent, out, keep, y0, one_pass)
    Bt = _product(_q_operand(Q, fp).T, A, fp)
    T = _product(Bt, B, f1)
    C = _product(_q_operand(Q, f2), T, f2)
    if f2 != "fp64":
        a = fl32(alpha)
        C = fl32(a * C)
        if beta != 0.0:
            C = fl32(C + fl32(fl32(beta) * np.asarray(Cin, np.float64)))
    else:
        C = alpha * C + (beta * np.asarray(Cin, np.float64) if beta != 0.0 else 0.0)
    out.update(Q=Q, R=R, Bt=Bt, T=T, C=C)
    return out


def lramm_backward(Q, A, B, dC):
    """Exact FP64 gradients of the frozen-Q surrogate C = Q Q^T A B."""
    Q = np.asarray(Q, np.float64)
    W = Q.T @ np.asarray(dC, np.float64)          # l x n
    dA = Q @ (W @ np.asarray(B, np.float64).T)     # m x k
    dB = np.asarray(A, np.float64).T @ (Q @ W)     # k x n
    return dA, dB


def surrogate(Q, A, B):
    """The frozen-Q forward map Q Q^T A B (FP64), for finite differences."""
    Q = np.asarray(Q, np.float64)
    return Q @ ((Q.T @ np.asarray(A, np.float64)) @ np.asarray(B, np.float64))


def rel_fro(X, Xref):
    d = np.linalg.norm(np.asarray(X, np.float64) - np.asarray(Xref, np.float64))
    nr = np.linalg.norm(np.asarray(Xref, np.float64))
    return d / nr if nr > 0 else d


def max_abs(X, Xref):
    return float(np.max(np.abs(np.asarray(X, np.float64) - np.asarray(Xref, np.float64))))


def tail(sigma, l):
    """Eckart-Young floor of a rank-l approximation in the Frobenius norm:
    (sum_{j > l} sigma_j^2)^(1/2) (Sec. 3.3, eq. svdfinq; Theorem 3.1)."""
    s = np.sort(np.asarray(sigma, np.float64))[::-1]
    return float(np.sqrt(np.sum(s[l:] ** 2)))


def error_report(C, A, B, sigma=None, l=None):
    """Relative Frobenius error (Sec. 3.3, E_r) and max-abs error against the
    exact FP64 product, with sigma_{l+1} and the rank-l tail when the
    spectrum of A is given."""
    Cex = np.asarray(A, np.float64) @ np.asarray(B, np.float64)
    rep = {"rel_fro": rel_fro(C, Cex), "max_abs": max_abs(C, Cex)}
    if sigma is not None and l is not None:
        s = np.sort(np.asarray(sigma, np.float64))[::-1]
        rep["sigma_next"] = float(s[l]) if l < len(s) else 0.0
        rep["tail"] = tail(s, l)
    return rep
