"""GPU checks of the a-posteriori error estimate (||A - Q Q^T A||_F^2 =
||A||_F^2 - ||Q^T A||_F^2 for orthonormal Q; paper Alg. 1's B = Q* A and the
Frobenius error of Sec. 3.3) and of the rank ladder built on it, through the
C ABI.  The two norms are FP64 reductions checked against numpy; the
estimate against the exact range error of the GPU's own Q within the bound
that the projection's quantisation allows."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import lramm as OL  # noqa: E402

DEV = "cuda"

CASES = [
    # m, k, n, r, p, q, tau, fmt, io, trans_a, sketch
    (512, 512, 512, 64, 10, 1, 32.0, ("int8",) * 4, "fp32", False, "gaussian"),
    (700, 1536, 300, 90, 10, 0, 32.0, ("bf16",) * 4, "bf16", False, "gaussian"),
    (640, 384, 512, 100, 12, 0, 40.0, ("int8", "int8", "int4", "int4"), "fp32", True, "gaussian"),
    (1024, 2048, 512, 112, 16, 0, 64.0, ("bf16",) * 4, "bf16", False, "srht"),
]


@pytest.mark.parametrize("case", CASES)
def test_estimate_against_exact_range_error(lib, case):
    m, k, n, r, p, q, tau, fmt, io, ta, sketch = case
    print(f"estimate {m}x{k}x{n} r={r} p={p} q={q} {fmt} {io} trans_a={ta} {sketch}", flush=True)
    A, _ = synth.lowrank(m, k, synth.spectrum("exp", min(m, k), tau), 0, dtype=io)
    B = synth.gaussian(k, n, 100, dtype=io)
    dt = torch.bfloat16 if io == "bf16" else torch.float32
    Ad = torch.from_numpy(A).to(DEV).to(dt)
    Bd = torch.from_numpy(B).to(DEV).to(dt)
    As = Ad.t().contiguous().t() if ta else Ad        # transposed storage, same values
    plan = lib.LrammPlan(m, n, k, r, p, q, fmt, dt, dt, dt, 4, trans_a=ta, sketch=sketch, estimate=True)
    ws = plan.workspace()
    store, _ = lib.storage(As)
    plan.forward(store, Bd, ws)
    assert plan.status(ws) == 0
    est, a2, b2 = plan.error_estimate(ws)
    A64 = A.astype(np.float64)
    Qg, Btg = plan.factors(ws)
    Q = Qg.cpu().numpy()
    Bt = Btg.double().cpu().numpy()
    assert abs(a2 - np.sum(A64 ** 2)) <= 1e-12 * np.sum(A64 ** 2)
    assert abs(b2 - np.sum(Bt ** 2)) <= 1e-12 * np.sum(Bt ** 2)
    assert abs(est - np.sqrt(max(0.0, a2 - b2) / a2)) <= 1e-12
    # exact range error of the GPU's own Q, and how far the quantised
    # projection may move ||Bt||^2 from ||Q^T A||^2
    P = Q.T @ A64
    true = np.linalg.norm(A64 - Q @ P) / np.linalg.norm(A64)
    dev = np.linalg.norm(Bt - P) * (np.linalg.norm(Bt) + np.linalg.norm(P)) / a2
    print(f"estimate {est:.4e} exact {true:.4e} (allowed |est^2 - exact^2| {dev:.2e})")
    assert abs(est ** 2 - true ** 2) <= dev + 1e-12


def test_rank_ladder_stops_at_tolerance(lib):
    """auto_rank on sigma_i = exp(-i/40): the returned width meets the
    tolerance and the rung before it does not."""
    import paper_2405_16917_amd as L
    m = k = n = 1024
    A, sig = synth.lowrank(m, k, synth.spectrum("exp", m, 40.0), 2)
    B = synth.gaussian(k, n, 3)
    Ad, Bd = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
    tol = 3e-3
    C, l, est, tried = L.auto_rank(Ad, Bd, tol, p=16, q=1, fmt=("bf16",) * 4, l0=96)
    print("ladder", tried)
    assert est <= tol and l == tried[-1][0]
    assert len(tried) >= 2 and tried[-2][1] > tol
    # the Eckart-Young floor of the rung that met the tolerance is below it
    s = np.sort(sig)[::-1] * (np.linalg.norm(A) / np.linalg.norm(sig))
    assert OL.tail(s, l) / np.linalg.norm(A) <= tol
