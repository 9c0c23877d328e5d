"""The no-allocation CholeskyQR2 entry point (lramm_cholqr2_noalloc) against
lramm_cholqr2 through the C ABI: both run the same kernels, so Q and the
status flags must agree bit for bit, call after call, on the library's one
fixed scratch buffer (a smaller problem after a larger one, then the larger
one again, so stale scratch contents from the previous call are present)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle.qr import householder_qr  # noqa: E402

DEV = "cuda"


def _input(rows, l, cond, seed, dtype):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((rows, l)))
    V, _ = np.linalg.qr(rng.standard_normal((l, l)))
    Y = (U * np.logspace(0, -np.log10(cond), l)) @ V.T
    if dtype == torch.float32:
        Y = Y.astype(np.float32).astype(np.float64)
    return Y, torch.from_numpy(np.ascontiguousarray(Y)).to(DEV, dtype)


def test_noalloc_cholqr2_matches_workspace_entry(lib):
    lib.lramm_init()
    cases = [(4096, 272, 30.0, 1, torch.float32),     # one-launch Cholesky, odd block count
             (700, 40, 100.0, 2, torch.float64),      # smaller: half-live last block, FP64 input
             (4096, 272, 30.0, 1, torch.float32)]     # the first again, over the second's scratch
    for rows, l, cond, seed, dt in cases:
        print(f"noalloc case rows={rows} l={l} dtype={dt}", flush=True)
        Ynp, Y = _input(rows, l, cond, seed, dt)
        f_ref = torch.zeros(1, dtype=torch.int32, device=DEV)
        f_new = torch.zeros(1, dtype=torch.int32, device=DEV)
        Q_ref = lib.lramm_cholqr2(Y, l, flags=f_ref)
        Q_new = torch.full_like(Q_ref, float("nan"))
        lib.lramm_cholqr2_noalloc(Y, l, Q=Q_new, flags=f_new)
        torch.cuda.synchronize()
        assert torch.equal(Q_new, Q_ref)
        assert int(f_new.item()) == int(f_ref.item()) == 0
        Qg = Q_new.cpu().numpy()
        assert not Qg[:, l:].any()
        Qh, _ = householder_qr(Ynp)
        assert np.max(np.abs(Qg[:, :l] - Qh)) <= 2e-14 * cond * np.sqrt(l)

