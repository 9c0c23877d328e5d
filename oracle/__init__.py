"""FP64 CPU oracle for the LRAMM hot path -- TEST INFRASTRUCTURE ONLY.

This package is the slow, plain, obviously-correct reference that the HIP path
is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  The product library never
imports, links or calls anything here, and nothing here imports the product.

Arithmetic is FP64.  Where the method rounds to binary32 (the quantiser rule,
the dequantising epilogue, the FP32 intermediates between stages) the oracle
computes the single IEEE operation in FP64 and rounds once to binary32; for
+, -, *, / and sqrt of binary32 operands this equals the directly rounded
binary32 result because 53 >= 2*24 + 2 (double rounding is innocuous).

Paper: arxiv 2405.16917, "LRAMM -- Low precision approximates GEMM via RSVD".

Modules
  quant   -- symmetric linear quantiser and its inverse (Sec. 3.1, eqs.
             Quantization / get_lambda / Dequantization)
  qgemm   -- quantised GEMM, Alg. 2 (Sec. 3.1), exact integer products
  qr      -- Householder thin QR (range-finder orthonormalisation, Sec. 2.2)
  philox  -- Philox4x32-10 counter RNG + Box-Muller for the Gaussian test matrix
  srht    -- the structured (subsampled randomised Hadamard) test matrix
  lramm   -- the one-sided LRAMM pipeline (randomised range finder, Sec. 2.2 /
             Alg. 1; chained quantised products, Sec. 3.2), the frozen-Q
             backward, and the error metrics (Sec. 3.3)

Parity status per function is stated in each module header.
"""

from . import quant, qgemm, qr, philox, srht, lramm  # noqa: F401
