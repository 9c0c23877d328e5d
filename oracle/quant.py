"""Symmetric linear quantiser (oracle, FP64) -- TEST INFRASTRUCTURE ONLY.

Paper Sec. 3.1: the integer code of a value is TypeCast(lambda * a) with
lambda = (2^(N-1) - 1) / a_max (eqs. Quantization and get_lambda), and the
value is recovered as a_int / lambda (eq. Dequantization).

Readings adopted where the paper is silent or loose (each listed in the design
notes of the repository):
  * rounding: TypeCast is taken as round-to-nearest, ties to even.  Truncation
    or floor would bias the error, contradicting the zero-mean error of
    Theorem 4.1 (appendix).
  * granularity: one a_max per vector.  A left GEMM operand is quantised per
    row, a right operand per column (the paper uses one a_max per matrix; the
    per-tensor variant is kept here as ``quantize_tensor``).
  * arithmetic: lambda = fl32(qmax / amax); code = clamp(rne(fl32(v * lambda)),
    -qmax, qmax); dequantisation multiplies by d = fl32(amax / qmax), a
    separately rounded reciprocal of lambda.
  * all-zero vector (a_max = 0, lambda undefined) and vectors so small that
    fl32(qmax / amax) overflows: every code is 0 and d = 0.
  * the code range is symmetric, +-(2^(N-1)-1): -128 / -8 never occur.

Extra formats used by the mixed-precision stages (not in the paper):
  * fp8 e4m3 (OCP: bias 7, 3 mantissa bits, max 448, no infinity):
    lambda = fl32(448 / amax), x = saturate(rne_e4m3(fl32(v * lambda))),
    d = fl32(amax / 448).
  * bf16: x = rne_bf16(v), d = 1 (no scaling).

Pins (tests/test_oracle_quant.py): hand-computed ties, the amax element maps
to +-qmax, odd symmetry, invariance under scaling by powers of two, the
per-element error bound, Theorem 4.2's Frobenius bound, idempotence after a
dequantise/requantise round trip, and e4m3 / bf16 grids checked against
independent bit-level constructions.
"""

import numpy as np

QMAX = {"int8": 127, "int4": 7}
FP8_MAX = 448.0


def fl32(x):
    """Round FP64 values to the nearest binary32 (ties to even); FP64 result."""
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def _check_finite(v):
    if not np.all(np.isfinite(v)):
        raise ValueError("quantiser input holds a non-finite value")


def rne_bf16(y):
    """Nearest bfloat16 value (8 significant bits, ties to even) of binary32 y."""
    y = np.asarray(y, dtype=np.float64)
    out = np.zeros_like(y)
    nz = y != 0
    f, e = np.frexp(y[nz])          # y = f * 2^e, 0.5 <= |f| < 1
    # spacing of the bf16 grid in the binade of y: 2^(e-1-7); subnormal floor 2^-133
    sp = np.ldexp(1.0, np.maximum(e - 8, -133))
    out[nz] = np.rint(y[nz] / sp) * sp
    return out


def sat_rne_e4m3(y):
    """Nearest OCP fp8 e4m3 value of y (ties to even), saturated to +-448."""
    y = np.asarray(y, dtype=np.float64)
    out = np.zeros_like(y)
    nz = y != 0
    f, e = np.frexp(y[nz])
    # 3 mantissa bits: spacing 2^(e-1-3) for normals (|y| >= 2^-6), 2^-9 below
    sp = np.ldexp(1.0, np.maximum(e - 4, -9))
    out[nz] = np.rint(y[nz] / sp) * sp
    return np.clip(out, -FP8_MAX, FP8_MAX)


def quantize_lastaxis(X, fmt):
    """Quantise each row of X (values must be binary32) independently.

    Returns (codes, d): for int8/int4 ``codes`` is an int64 array, for fp8
    the e4m3 values (float64), for bf16 the bf16 values; ``d`` (float64
    holding binary32 values) is the per-row dequantisation factor.
    """
    X = np.asarray(X, dtype=np.float64)
    _check_finite(X)
    if np.any(fl32(X) != X):
        raise ValueError("quantiser input must consist of binary32 values")
    rows = X.shape[0]
    if fmt == "bf16":
        return rne_bf16(X), np.ones(rows)
    if fmt in QMAX:
        qmax = float(QMAX[fmt])
    elif fmt == "fp8":
        qmax = FP8_MAX
    else:
        raise ValueError(f"unknown format {fmt!r}")
    amax = np.max(np.abs(X), axis=1) if X.shape[1] else np.zeros(rows)
    with np.errstate(divide="ignore", over="ignore"):
        lam = fl32(np.where(amax > 0, qmax / np.where(amax > 0, amax, 1.0), np.inf))
    live = np.isfinite(lam) & (amax > 0)
    lam_safe = np.where(live, lam, 0.0)
    y = fl32(X * lam_safe[:, None])          # one binary32 product per element
    if fmt == "fp8":
        codes = sat_rne_e4m3(y)
    else:
        codes = np.clip(np.rint(y), -qmax, qmax).astype(np.int64)
    d = np.where(live, fl32(amax / qmax), 0.0)
    codes[~live] = 0
    return codes, d


def quantize_rows(X, fmt):
    """Left-operand quantisation: one scale per row."""
    return quantize_lastaxis(X, fmt)


def quantize_cols(X, fmt):
    """Right-operand quantisation: one scale per column (codes keep X's shape)."""
    codes, d = quantize_lastaxis(np.asarray(X).T, fmt)
    return codes.T, d


def quantize_tensor(X, fmt):
    """The paper's per-matrix quantiser (one a_max for the whole matrix)."""
    X = np.asarray(X, dtype=np.float64)
    codes, d = quantize_lastaxis(X.reshape(1, -1), fmt)
    return codes.reshape(X.shape), float(d[0])


def dequantize_rows(codes, d):
    return codes.astype(np.float64) * d[:, None]


def dequantize_cols(codes, d):
    return codes.astype(np.float64) * d[None, :]


def pack_int4(codes):
    """Pack int4 codes two per byte along the last axis: element 2j in the low
    nibble, 2j+1 in the high nibble, two's complement.  An odd length is
    padded with a zero code."""
    c = np.asarray(codes, dtype=np.int64)
    if c.shape[-1] % 2:
        c = np.concatenate([c, np.zeros(c.shape[:-1] + (1,), np.int64)], axis=-1)
    lo = c[..., 0::2] & 0xF
    hi = c[..., 1::2] & 0xF
    return (lo | (hi << 4)).astype(np.uint8)


def unpack_int4(packed, n):
    p = np.asarray(packed, dtype=np.int64)
    lo = p & 0xF
    hi = (p >> 4) & 0xF
    out = np.empty(p.shape[:-1] + (2 * p.shape[-1],), np.int64)
    out[..., 0::2] = lo
    out[..., 1::2] = hi
    out = np.where(out >= 8, out - 16, out)
    return out[..., :n]
