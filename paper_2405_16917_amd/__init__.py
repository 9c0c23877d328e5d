"""LRAMM hot path on MI355X (gfx950): Python face of the HIP library.

    import paper_2405_16917_amd as lramm
    C = lramm.matmul(A, B, r=256, p=16, q=1)                 # forward only
    C = lramm.LRAMMFunction.apply(A, B, cfg)                 # differentiable

Every step runs in the library's HIP kernels (see include/lramm.h); this
package only marshals torch tensors, sizes and the current stream.
"""

import torch

from ._lib import (  # noqa: F401
    EXPORTS, LIB_PATH, LrammBatch, LrammError, LrammPlan, autotune_rank, load, lramm_cholqr2,
    lramm_cholqr2_workspace, lramm_cholqr2_noalloc, NOALLOC_SCRATCH_BYTES, E_SCRATCH,
    lramm_dense_gemm_nt, lramm_gemm_nt, lramm_gemm_nt_workspace, lramm_init, lramm_omega,
    lramm_pitch, lramm_quantize, FLAG_BREAKDOWN, FLAG_NONFINITE, FLAG_SQRTNEG, FLAG_STALL,
)


def matmul(A, B, r, p=16, q=1, fmt=("int8",) * 4, seed=0, omega=None, alpha=1.0, beta=0.0, out=None,
           out_dtype=None, return_plan=False, check=True):
    """C ~ alpha A B + beta out by LRAMM (one-sided, rank l = r + p).

    With ``check`` (the default) the device status word is read after the
    forward (this synchronises the stream): a non-finite input or a Cholesky
    wait past its bound raises LrammError instead of returning an invalid C."""
    m, k = A.shape
    n = B.shape[1]
    c_type = out.dtype if out is not None else (out_dtype or A.dtype)
    plan = LrammPlan(m, n, k, r, p, q, fmt, A.dtype, B.dtype, c_type, seed, alpha, beta)
    ws = plan.workspace(A.device)
    C = plan.forward(A, B, ws, C=out, omega=omega)
    if check:
        plan.status(ws)
    if return_plan:
        return C, plan, ws
    return C


class LRAMMConfig:
    """Settings of LRAMMFunction.  ``check``: read the device status word
    after each forward (synchronises the stream) and raise LrammError on a
    non-finite input or an invalid Cholesky factor."""

    def __init__(self, r, p=16, q=1, fmt=("int8",) * 4, seed=0, omega=None, recompute=False, check=True):
        self.r, self.p, self.q, self.fmt, self.seed, self.omega = r, p, q, fmt, seed, omega
        self.recompute = recompute
        self.check = check


class LRAMMFunction(torch.autograd.Function):
    """Forward: LRAMM.  Backward: gradient of the frozen-Q surrogate
    C = Q Q^T A B (quantisation straight-through): dA = Q Q^T dC B^T,
    dB = A^T Q Q^T dC, computed from Q in FP32 GEMMs.  With
    ``cfg.recompute`` the workspace holding Q is dropped after the forward
    and Q is recomputed bit-identically (same seed / Omega) in backward."""

    @staticmethod
    def forward(ctx, A, B, cfg):
        m, k = A.shape
        n = B.shape[1]
        plan = LrammPlan(m, n, k, cfg.r, cfg.p, cfg.q, cfg.fmt, A.dtype, B.dtype, A.dtype, cfg.seed)
        ws = plan.workspace(A.device)
        C = plan.forward(A, B, ws, omega=cfg.omega)
        if cfg.check:
            plan.status(ws)
        ctx.plan, ctx.cfg = plan, cfg
        ctx.ws = None if cfg.recompute else ws
        ctx.save_for_backward(A, B)
        return C

    @staticmethod
    def backward(ctx, dC):
        A, B = ctx.saved_tensors
        plan, ws = ctx.plan, ctx.ws
        if ws is None:
            ws = plan.workspace(A.device)
            plan.forward(A, B, ws, omega=ctx.cfg.omega)
        dA, dB = plan.backward(dC.contiguous().to(torch.float32), A, B, ws,
                               need_dA=ctx.needs_input_grad[0], need_dB=ctx.needs_input_grad[1])
        ctx.ws = None
        return dA, dB, None
