"""LRAMM hot path on MI355X (gfx950): Python face of the HIP library.

    import paper_2405_16917_amd as lramm
    C = lramm.matmul(A, B, r=256, p=16, q=1)                 # forward only
    C = lramm.LRAMMFunction.apply(A, B, cfg)                 # differentiable

Every step runs in the library's HIP kernels (see include/lramm.h); this
package only marshals torch tensors, sizes and the current stream.
"""

import torch

from ._lib import (  # noqa: F401
    EXPORTS, LIB_PATH, LrammBatch, LrammError, LrammPlan, LrammTsPlan, autotune_rank, load, lramm_cholqr2, storage,
    lramm_cholqr2_workspace, lramm_cholqr2_noalloc, lramm_r_factor, NOALLOC_SCRATCH_BYTES, E_SCRATCH,
    lramm_dense_gemm_nt, lramm_gemm_nt, lramm_gemm_nt_workspace, lramm_init, lramm_omega,
    lramm_pitch, lramm_quantize, lramm_srht_padded, lramm_srht_samples, lramm_srht_sketch, FLAG_BREAKDOWN, FLAG_NONFINITE, FLAG_SQRTNEG, FLAG_STALL,
)


def matmul(A, B, r, p=16, q=1, fmt=("int8",) * 4, seed=0, omega=None, alpha=1.0, beta=0.0, out=None,
           out_dtype=None, return_plan=False, check=True, side="left", sketch="gaussian", orth="cholqr2"):
    """C ~ alpha A B + beta out by LRAMM (one-sided, rank l = r + p).
    ``side="right"`` sketches B instead of A.  A or B may be transposed views
    (e.g. ``W.t()``): they are passed as transposed storage, not copied.
    ``sketch="srht"``: the first sketch uses the structured (subsampled
    randomised Hadamard) test matrix drawn from ``seed``.  ``orth="cholqr"``:
    one Cholesky QR pass per orthonormalisation instead of CholeskyQR2.

    With ``check`` (the default) the device status word is read after the
    forward (this synchronises the stream): a non-finite input or a Cholesky
    wait past its bound raises LrammError instead of returning an invalid C."""
    m, k = A.shape
    n = B.shape[1]
    As, ta = storage(A)
    Bs, tb = storage(B)
    c_type = out.dtype if out is not None else (out_dtype or A.dtype)
    plan = LrammPlan(m, n, k, r, p, q, fmt, A.dtype, B.dtype, c_type, seed, alpha, beta, trans_a=ta, trans_b=tb,
                     side=side, sketch=sketch, orth=orth)
    ws = plan.workspace(A.device)
    C = plan.forward(As, Bs, ws, C=out, omega=omega)
    if check:
        plan.status(ws)
    if return_plan:
        return C, plan, ws
    return C


def auto_rank(A, B, tol, p=16, q=1, fmt=("int8",) * 4, seed=0, l0=None, growth=1.5, l_max=None,
              sketch="gaussian", out_dtype=None):
    """The smallest sketch width on a geometric ladder whose a-posteriori
    estimate of ||A - Q Q^T A||_F / ||A||_F (lramm_error_estimate) is at
    most ``tol``.  The ladder starts at ``l0`` (default: the rank rule
    r = ceil(min(m, k) / 10) plus p) and grows by ``growth``, rounded up to
    a multiple of 32, up to ``l_max`` (default min(m, k, 1024)).  Returns
    (C, l, estimate, tried) with tried the (l, estimate) pairs in order; the
    last rung is returned even when it misses ``tol``."""
    m, k = A.shape
    n = B.shape[1]
    As, ta = storage(A)
    Bs, tb = storage(B)
    lim = min(m, k, 1024) if l_max is None else min(l_max, m, k)
    l = min(l0 if l0 is not None else autotune_rank(m, k) + p, lim)
    tried = []
    while True:
        pp = min(p, l - 1)
        plan = LrammPlan(m, n, k, l - pp, pp, q, fmt, A.dtype, B.dtype, out_dtype or A.dtype, seed,
                         trans_a=ta, trans_b=tb, sketch=sketch, estimate=True)
        ws = plan.workspace(A.device)
        C = plan.forward(As, Bs, ws)
        plan.status(ws)
        est = plan.error_estimate(ws)[0]
        tried.append((l, est))
        if est <= tol or l >= lim:
            return C, l, est, tried
        l = min(lim, -(-int(l * growth) // 32) * 32)


class LRAMMConfig:
    """Settings of LRAMMFunction.  ``side``: "left" sketches A, "right"
    sketches B (a low-rank weight on the right of activations).  ``check``:
    read the device status word after each forward (synchronises the stream)
    and raise LrammError on a non-finite input or an invalid Cholesky factor.
    ``orth``: "cholqr2" (two Cholesky QR passes) or "cholqr" (one)."""

    def __init__(self, r, p=16, q=1, fmt=("int8",) * 4, seed=0, omega=None, recompute=False, check=True,
                 side="left", sketch="gaussian", orth="cholqr2"):
        self.r, self.p, self.q, self.fmt, self.seed, self.omega = r, p, q, fmt, seed, omega
        self.orth = orth
        self.recompute = recompute
        self.check = check
        self.side = side
        self.sketch = sketch


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
        As, ta = storage(A)
        Bs, tb = storage(B)
        plan = LrammPlan(m, n, k, cfg.r, cfg.p, cfg.q, cfg.fmt, A.dtype, B.dtype, A.dtype, cfg.seed,
                         trans_a=ta, trans_b=tb, side=cfg.side, sketch=cfg.sketch, orth=cfg.orth)
        ws = plan.workspace(A.device)
        C = plan.forward(As, Bs, ws, omega=cfg.omega)
        if cfg.check:
            plan.status(ws)
        ctx.plan, ctx.cfg, ctx.trans = plan, cfg, (ta, tb)
        ctx.ws = None if cfg.recompute else ws
        ctx.save_for_backward(As, Bs)
        return C

    @staticmethod
    def backward(ctx, dC):
        As, Bs = ctx.saved_tensors
        plan, ws = ctx.plan, ctx.ws
        if ws is None:
            ws = plan.workspace(As.device)
            plan.forward(As, Bs, ws, omega=ctx.cfg.omega)
        dCs = dC.contiguous()
        if dCs.dtype != plan.c_type:
            dCs = dCs.to(plan.c_type)
        dA, dB = plan.backward(dCs, As, Bs, ws, need_dA=ctx.needs_input_grad[0], need_dB=ctx.needs_input_grad[1])
        ta, tb = ctx.trans
        ctx.ws = None
        # gradients in the layout of the inputs (transposed storage -> .t() view)
        return (dA.t() if (dA is not None and ta) else dA), (dB.t() if (dB is not None and tb) else dB), None
