"""Pins of the oracle's two-sided LRAMM (paper Alg. 3) against facts that do
not depend on it: exact recovery, the full-size case, Eckart-Young optimality
of the truncated factors, associativity of the unquantised chain, the sign
rule, and the expected ordering of bit budgets."""

import numpy as np

import synth
from oracle import two_sided as TS
from oracle.lramm import rel_fro


def _lowrank64(m, k, rank, seed, tau=8.0):
    rng = np.random.default_rng(seed)
    U, V = synth.haar(m, rank, rng), synth.haar(k, rank, rng)
    return (U * synth.spectrum("exp", rank, tau)[None, :]) @ V.T


def test_exact_recovery_when_both_ranks_at_most_r():
    m, k, n = 120, 100, 90
    A = _lowrank64(m, k, 12, 1)
    B = _lowrank64(k, n, 10, 2)
    rng = np.random.default_rng(3)
    out = TS.lramm_two_sided(A, B, 14, 6, 0, d=("fp64",) * 3, omega_a=rng.standard_normal((k, 20)),
                             omega_b=rng.standard_normal((n, 20)))
    assert rel_fro(out["D"], A @ B) <= 1e-12


def test_full_size_reproduces_the_product():
    """l = r = m = k = n: Q is square orthogonal, nothing is truncated."""
    rng = np.random.default_rng(4)
    A, B = rng.standard_normal((40, 40)), rng.standard_normal((40, 40))
    out = TS.lramm_two_sided(A, B, 40, 0, 0, d=("fp64",) * 3, omega_a=rng.standard_normal((40, 40)),
                             omega_b=rng.standard_normal((40, 40)))
    assert rel_fro(out["D"], A @ B) <= 1e-12


def test_truncation_reaches_eckart_young_within_the_range():
    """U~ V^T is the best rank-r approximation of Q Q^T A: its error equals
    the root sum of squares of the dropped singular values of B~."""
    m, k = 150, 130
    A = _lowrank64(m, k, 60, 5, tau=10.0)
    rng = np.random.default_rng(6)
    U, S, Vt, Q, Bt, s = TS.rsvd(A, 20, 10, 1, omega=rng.standard_normal((k, 30)))
    err = np.linalg.norm(Q @ Bt - (U * S[None, :]) @ Vt)
    assert abs(err - np.sqrt(np.sum(s[20:] ** 2))) <= 1e-10 * np.linalg.norm(A)
    # and U has orthonormal columns, V^T orthonormal rows
    assert np.max(np.abs(U.T @ U - np.eye(20))) <= 1e-12
    assert np.max(np.abs(Vt @ Vt.T - np.eye(20))) <= 1e-12


def test_unquantised_chain_is_the_product_of_the_approximations():
    """With fp64 stages D = (U~ V^T)(W Z~): E1..E3 chain the factors in the
    order of Alg. 3 (a transposed or swapped factor would break this)."""
    rng = np.random.default_rng(7)
    A = _lowrank64(80, 70, 30, 8)
    B = _lowrank64(70, 60, 30, 9)
    out = TS.lramm_two_sided(A, B, 12, 4, 1, d=("fp64",) * 3, omega_a=rng.standard_normal((70, 16)),
                             omega_b=rng.standard_normal((60, 16)))
    Aap = out["Ut"] @ out["Vt"]
    Bap = out["W"] @ out["Zs"]
    assert rel_fro(out["D"], Aap @ Bap) <= 1e-12
    assert out["E1"].shape == (12, 12) and out["E2"].shape == (12, 60) and out["E3"].shape == (80, 60)


def test_sign_rule():
    rng = np.random.default_rng(10)
    X = rng.standard_normal((30, 20))
    Up, s, Vt = np.linalg.svd(X, full_matrices=False)
    U2, V2 = TS.sign_fix(-Up, -Vt)
    U1, V1 = TS.sign_fix(Up, Vt)
    assert np.array_equal(U1, U2) and np.array_equal(V1, V2)
    assert np.all(U1[np.argmax(np.abs(U1), axis=0), np.arange(20)] > 0)
    assert np.allclose((U1 * s) @ V1, X, atol=1e-12)


def test_bit_budgets_order_errors():
    """On a low-rank product the error falls with the bit budget: 444 is
    worse than 884, which is worse than 888 (averaged over seeds), and all
    are worse than the unquantised chain."""
    m = k = n = 200
    errs = {key: [] for key in ("444", "884", "888", "fff")}
    for seed in range(4):
        A = _lowrank64(m, k, 40, 20 + seed, tau=6.0)
        B = _lowrank64(k, n, 40, 40 + seed, tau=6.0)
        Cex = A @ B
        rng = np.random.default_rng(60 + seed)
        oa, ob = rng.standard_normal((k, 50)), rng.standard_normal((n, 50))
        for key, d in (("444", ("int4",) * 3), ("884", ("int8", "int8", "int4")), ("888", ("int8",) * 3),
                       ("fff", ("fp64",) * 3)):
            errs[key].append(rel_fro(TS.lramm_two_sided(A, B, 40, 10, 0, d=d, omega_a=oa, omega_b=ob)["D"], Cex))
    mean = {key: np.mean(v) for key, v in errs.items()}
    assert mean["fff"] < mean["888"] < mean["884"] < mean["444"]
