"""Quantised GEMM, Alg. 2 of the paper (Sec. 3.1) -- TEST INFRASTRUCTURE ONLY.

Alg. 2 quantises both operands, forms the integer product, dequantises it and
returns alpha * D_F + beta * C.  The oracle writes those steps out:

  1. left operand quantised per row, right operand per column (quant.py);
  2. the integer product, exact.  Every partial sum of products of codes with
     |code| <= 127 is an integer of magnitude below K * 127^2, so an FP64
     matrix product is exact for K < 2^53 / 127^2; the function asserts the
     bound and also that every result fits the int32 accumulator
     (K * 127^2 < 2^31, i.e. K <= 133144 for int8);
  3. dequantisation by the row factor of the left operand, then by the column
     factor of the right operand, each product rounded to binary32:
     c_ij = fl32(fl32(fl32(acc_ij) * d_i) * d_j).  Alg. 2 does not fix the
     order; this is the reading the oracle takes (row factor first);
  4. alpha/beta: out = fl32(alpha * c) when beta == 0 (C is not read), else
     fl32(fl32(alpha * c) + fl32(beta * C)).

For fp8 operands the product of e4m3 values is also exact in FP64 (all
products are multiples of 2^-18 below 2^18), for bf16 operands it is the FP64
product of the bf16-rounded values.

Pins (tests/test_oracle_qgemm.py): the integer product equals brute-force
Python integer loops on small shapes and numpy int64 matmul on larger ones;
the epilogue equals an independent binary32 evaluation with numpy float32
scalars; hand-worked bf16 and fp8 products (rounding ties, the e4m3 grid and
the amax-to-448 scaling); the size-invariance of the relative error
(Sec. 3.3) and the Theorem 4.3 bound hold on random inputs.
"""

import numpy as np

from .quant import fl32, quantize_rows, quantize_cols

INT32_MAX = 2**31 - 1


def int_gemm(Lq, Rq):
    """Exact integer product of integer code matrices (M x K) @ (K x N)."""
    Lq = np.asarray(Lq, dtype=np.int64)
    Rq = np.asarray(Rq, dtype=np.int64)
    K = Lq.shape[1]
    lmax = int(np.max(np.abs(Lq))) if Lq.size else 0
    rmax = int(np.max(np.abs(Rq))) if Rq.size else 0
    bound = K * lmax * rmax
    assert bound < 2**53, "integer product would not be exact in FP64"
    acc = Lq.astype(np.float64) @ Rq.astype(np.float64)
    acc = acc.astype(np.int64)
    if acc.size and int(np.max(np.abs(acc))) > INT32_MAX:
        raise OverflowError("integer product exceeds the int32 accumulator")
    return acc


def epilogue(acc, dL, dR, alpha=1.0, beta=0.0, Cin=None):
    """Dequantising epilogue with the alpha/beta update of Alg. 2."""
    c = fl32(fl32(np.asarray(acc, np.float64)) * np.asarray(dL, np.float64)[:, None])
    c = fl32(c * np.asarray(dR, np.float64)[None, :])
    a = fl32(alpha)
    out = fl32(a * c)
    if beta != 0.0:
        b = fl32(beta)
        out = fl32(out + fl32(b * np.asarray(Cin, np.float64)))
    return out


def qgemm(L, R, fmt, alpha=1.0, beta=0.0, Cin=None, parts=False):
    """Alg. 2 on binary32 operands L (M x K) and R (K x N) in format ``fmt``.

    Returns the binary32 result (as float64) or, with ``parts``, a dict that
    also holds the codes, scales and the exact accumulator.
    """
    Lc, dL = quantize_rows(L, fmt)
    Rc, dR = quantize_cols(R, fmt)
    if fmt in ("int8", "int4"):
        acc = int_gemm(Lc, Rc)
    else:
        acc = np.asarray(Lc, np.float64) @ np.asarray(Rc, np.float64)
    out = epilogue(acc, dL, dR, alpha, beta, Cin)
    if parts:
        return {"out": out, "Lq": Lc, "dL": dL, "Rq": Rc, "dR": dR, "acc": acc}
    return out
