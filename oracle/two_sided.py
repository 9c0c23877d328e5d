"""Two-sided LRAMM, the paper's Alg. 3 (Sec. 3.2), in FP64 -- TEST
INFRASTRUCTURE ONLY.

Steps, in the paper's order and notation:
  1. rank-r RSVD of A and of B (Alg. 1 after the range finder of Sec. 2.2):
       Q = range of the sketch (oversampled to l = r + p columns, q subspace
       iterations, as in lramm.range_finder);  B~ = Q^T A;  SVD B~ = U' S V^T;
       U = Q U'; keep the first r triplets.
     A ~ U_r S_r V_r^T (m x k) and B ~ W_r G_r Z_r^T (k x n).
  2. the diagonal factors absorbed in floating point:
       U~ = U_r S_r (m x r),  Z~ = G_r Z_r^T (r x n);
  3. three chained quantised products (Alg. 2 each, bit budgets d1, d2, d3;
     the labels of Alg. 3's listing: E1 -> d1, E2 -> d2, E3 -> d3):
       E1 = QM(V_r^T W_r, d1)   (r x r, inner dimension k)
       E2 = QM(E1 Z~, d2)       (r x n, inner dimension r)
       E3 = QM(U~ E2, d3)       (m x n, inner dimension r)
  4. D = alpha E3 + beta C.

Readings where the paper is silent (listed in the design notes):
  * the RSVD uses the one-sided path's range finder (Gaussian sketch with
    oversampling p and q power iterations) and its per-stage formats
    (``rsvd_fmt`` = (sketch, projection); "fp64" is the unquantised RSVD);
  * singular vectors are made unique by a sign rule: in each column of U'
    the entry of largest magnitude (the first one on a tie) is positive, and
    the matching row of V^T takes the same sign;
  * quantisation per row of the left operand and per column of the right
    one, as everywhere (qgemm.py); "fp64" as a stage format skips it.

Also here: the direct quantised product DQd = QM(A B, d) that the paper
compares against (its DQ8 and DQ4).

Pins (tests/test_oracle_two_sided.py): exact recovery when both ranks are at
most r; the full-size case l = r = m = k = n reproduces A B; the truncated
factors reach the Eckart-Young error of the projected matrix; the
unquantised chain equals the product of the two rank-r approximations; the
sign rule.
"""

import numpy as np

from .lramm import _product, _q_operand, range_finder
from .philox import gaussian_omega


def sign_fix(Up, Vt):
    """Flip each singular pair so that the largest-magnitude entry of the
    column of Up is positive (first one on a tie)."""
    idx = np.argmax(np.abs(Up), axis=0)
    s = np.sign(Up[idx, np.arange(Up.shape[1])])
    s[s == 0] = 1.0
    return Up * s[None, :], Vt * s[:, None]


def rsvd(A, r, p, q, rsvd_fmt=("fp64", "fp64"), omega=None, seed=None):
    """Rank-r RSVD (Alg. 1) of A: (U_r, s_r, V_r^T, Q, B~, s_all)."""
    A = np.asarray(A, np.float64)
    m, k = A.shape
    l = r + p
    if not (1 <= r <= l <= min(m, k)):
        raise ValueError("need 1 <= r <= r + p <= min(m, k)")
    if omega is None:
        omega = gaussian_omega(seed, k, l)
    omega = np.asarray(omega, np.float64)
    fs, fp = rsvd_fmt
    Q, _ = range_finder(A, l, q, fs, fp, omega, keep=False)
    Bt = _product(_q_operand(Q, fp).T, A, fp)           # B <- Q* A
    Up, s, Vt = np.linalg.svd(Bt, full_matrices=False)  # U' S V* <- B
    Up, Vt = sign_fix(Up, Vt)
    U = Q @ Up[:, :r]                                    # U <- Q U'
    return U, s[:r], Vt[:r, :], Q, Bt, s


def lramm_two_sided(A, B, r, p, q, rsvd_fmt=("fp64", "fp64"), d=("int8", "int8", "int8"), omega_a=None,
                    omega_b=None, seed=None, alpha=1.0, beta=0.0, Cin=None):
    """Alg. 3.  A: m x k, B: k x n.  omega_a is k x l (sketch of A),
    omega_b is n x l (sketch of B, whose range is its column space in R^k).
    Returns a dict with D and the intermediate factors."""
    A = np.asarray(A, np.float64)
    B = np.asarray(B, np.float64)
    if A.shape[1] != B.shape[0]:
        raise ValueError("inner dimensions differ")
    l = r + p
    if omega_a is None:
        omega_a = gaussian_omega(seed, A.shape[1], l)
    if omega_b is None:
        omega_b = gaussian_omega(None if seed is None else seed + 1, B.shape[1], l)
    U, S, Vt, QA, BtA, sA = rsvd(A, r, p, q, rsvd_fmt, omega_a)
    W, G, Zt, QB, BtB, sB = rsvd(B, r, p, q, rsvd_fmt, omega_b)
    Ut = U * S[None, :]                 # U~ = U_r S_r
    Zs = G[:, None] * Zt                # Z~ = G_r Z_r^T
    d1, d2, d3 = d
    E1 = _product(Vt, W, d1)            # QM(V_r^T W_r, d1)
    E2 = _product(E1, Zs, d2)           # QM(E1 Z~, d2)
    E3 = _product(Ut, E2, d3)           # QM(U~ E2, d3)
    D = alpha * E3 + (beta * np.asarray(Cin, np.float64) if beta != 0.0 else 0.0)
    return {"D": D, "U": U, "S": S, "Vt": Vt, "W": W, "G": G, "Zt": Zt, "Ut": Ut, "Zs": Zs, "E1": E1,
            "E2": E2, "E3": E3, "QA": QA, "QB": QB, "BtA": BtA, "BtB": BtB, "sA": sA, "sB": sB}


def direct_quantised(A, B, d):
    """DQd: Alg. 2 on the full-size product (the paper's DQ8 / DQ4)."""
    return _product(np.asarray(A, np.float64), np.asarray(B, np.float64), d)
