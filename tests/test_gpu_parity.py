"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Integer work (quantiser codes, int32 accumulators, dequantised epilogue) is
compared bit for bit; the end-to-end LRAMM output within relative Frobenius
1e-5 of the oracle's own output at the same bit widths; Q within
1e-13 * cond(Y) of the oracle's Householder Q.
"""

import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import lramm as OL  # noqa: E402
from oracle import philox as OP  # noqa: E402
from oracle import qgemm as OG  # noqa: E402
from oracle import qr as OQR  # noqa: E402
from oracle import quant as OQ  # noqa: E402
from oracle import srht as OS  # noqa: E402
from oracle.qr import householder_qr  # noqa: E402

DEV = "cuda"


def g(x, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV, dtype)


def f32(x):
    return np.asarray(x, np.float32).astype(np.float64)


def bf16_round(x):
    return synth.to_dtype(x, "bf16").astype(np.float64)


def e4m3_value(b):
    """Value of OCP fp8 e4m3 bytes (sign, 4 exponent bits with bias 7, 3
    mantissa bits; exponent field 0 is subnormal, 2^-6 * m/8)."""
    b = np.asarray(b, np.int64)
    sign = np.where(b & 0x80, -1.0, 1.0)
    e = (b >> 3) & 0xF
    m = (b & 7).astype(np.float64)
    mag = np.where(e == 0, m / 8.0 * 2.0**-6, (1.0 + m / 8.0) * np.exp2(e - 7.0))
    assert not np.any((b & 0x7F) == 0x7F), "NaN code"
    return sign * mag


def codes_from(Xq, fmt, K):
    q = Xq.cpu().numpy() if hasattr(Xq, "cpu") else np.asarray(Xq)
    if fmt == "fp8":
        return e4m3_value(q[:, :K]), q
    if fmt == "int8":
        return q.view(np.int8)[:, :K].astype(np.int64), q
    if fmt == "int4":
        return OQ.unpack_int4(q, K), q
    if fmt == "bf16":
        u = q.view(np.uint16)[:, :K].astype(np.uint32) << 16
        return u.view(np.float32).astype(np.float64), q
    raise ValueError(fmt)


def pad_bytes(q, fmt, K):
    used = {"int8": K, "int4": (K + 1) // 2, "bf16": 2 * K, "fp8": K}[fmt]
    return q[:, used:]


# --------------------------------------------------------------- runtime --

def test_single_hip_runtime_and_library_loaded(lib):
    lib.lramm_init()
    maps = open("/proc/self/maps").read()
    hips = {l.split()[-1] for l in maps.splitlines() if "libamdhip64" in l}
    assert len(hips) == 1, hips
    assert lib.LIB_PATH in maps


# ------------------------------------------------------------- quantiser --

@pytest.mark.parametrize("fmt", ["int8", "int4", "fp8", "bf16"])
@pytest.mark.parametrize("shape", [(1, 1), (37, 50), (130, 257), (512, 512), (64, 4099)])
def test_quantize_rows_bit_exact(lib, fmt, shape):
    rng = np.random.default_rng(shape[0] * 1000 + shape[1] + len(fmt))
    X = f32(rng.standard_normal(shape) * np.exp(rng.uniform(-8, 8, (shape[0], 1))))
    X[0, :] = 0.0                                   # all-zero vector -> codes 0, d 0
    Xq, s = lib.lramm_quantize(g(X), fmt, transpose=False)
    torch.cuda.synchronize()
    codes, raw = codes_from(Xq, fmt, shape[1])
    ref_c, ref_d = OQ.quantize_rows(X, fmt)
    assert np.array_equal(codes, ref_c)
    assert np.array_equal(s.cpu().numpy().astype(np.float64), ref_d)
    assert not pad_bytes(raw, fmt, shape[1]).any()


@pytest.mark.parametrize("fmt", ["int8", "int4", "fp8", "bf16"])
@pytest.mark.parametrize("shape", [(1, 1), (50, 37), (257, 130), (512, 512), (4099, 70)])
def test_quantize_cols_bit_exact(lib, fmt, shape):
    rng = np.random.default_rng(shape[0] * 1000 + shape[1] + len(fmt) + 1)
    X = f32(rng.standard_normal(shape) * np.exp(rng.uniform(-8, 8, (1, shape[1]))))
    X[:, 0] = 0.0
    Xq, s = lib.lramm_quantize(g(X), fmt, transpose=True)
    torch.cuda.synchronize()
    codes, raw = codes_from(Xq, fmt, shape[0])
    ref_c, ref_d = OQ.quantize_cols(X, fmt)
    assert np.array_equal(codes, ref_c.T)
    assert np.array_equal(s.cpu().numpy().astype(np.float64), ref_d)
    assert not pad_bytes(raw, fmt, shape[0]).any()


@pytest.mark.parametrize("transpose", [False, True])
def test_quantize_bf16_and_f64_inputs(lib, transpose):
    rng = np.random.default_rng(5)
    Xb = bf16_round(rng.standard_normal((70, 90)))
    Xq, s = lib.lramm_quantize(g(Xb, torch.bfloat16), "int8", transpose=transpose)
    ref = OQ.quantize_cols(Xb, "int8") if transpose else OQ.quantize_rows(Xb, "int8")
    codes, _ = codes_from(Xq, "int8", 70 if transpose else 90)
    assert np.array_equal(codes, ref[0].T if transpose else ref[0])
    assert np.array_equal(s.cpu().numpy().astype(np.float64), ref[1])
    Xd = rng.standard_normal((70, 90))               # FP64 input is rounded once to binary32
    Xq, s = lib.lramm_quantize(g(Xd, torch.float64), "int8", transpose=transpose)
    ref = OQ.quantize_cols(f32(Xd), "int8") if transpose else OQ.quantize_rows(f32(Xd), "int8")
    codes, _ = codes_from(Xq, "int8", 70 if transpose else 90)
    assert np.array_equal(codes, ref[0].T if transpose else ref[0])


def test_quantize_flags_nonfinite(lib):
    X = torch.ones((8, 8), device=DEV)
    X[3, 4] = float("nan")
    flags = torch.zeros(1, dtype=torch.int32, device=DEV)
    lib.lramm_quantize(X, "int8", transpose=False, flags=flags)
    torch.cuda.synchronize()
    assert int(flags.item()) & lib.FLAG_NONFINITE
    flags.zero_()
    X[3, 4] = float("inf")
    lib.lramm_quantize(X, "int8", transpose=True, flags=flags)
    torch.cuda.synchronize()
    assert int(flags.item()) & lib.FLAG_NONFINITE


# ------------------------------------------------------------------ GEMM --

def _int_operands(rng, M, N, K, qmax):
    L = rng.integers(-qmax, qmax + 1, (M, K))
    R = rng.integers(-qmax, qmax + 1, (N, K))
    return L, R


def _pack(codes, fmt, K):
    pitch = {"int8": (K + 63) // 64 * 64, "int4": ((K + 1) // 2 + 63) // 64 * 64}[fmt]
    if fmt == "int8":
        buf = np.zeros((codes.shape[0], pitch), np.int8)
        buf[:, :K] = codes
        return buf.view(np.uint8)
    p = OQ.pack_int4(codes)
    buf = np.zeros((codes.shape[0], pitch), np.uint8)
    buf[:, :p.shape[1]] = p
    return buf


@pytest.mark.parametrize("fmt", ["int8", "int4"])
@pytest.mark.parametrize("MNK", [(1, 1, 1), (37, 53, 100), (129, 65, 300), (64, 64, 64), (256, 320, 4096),
                                 (300, 70, 8192), (512, 512, 512),
                                 # 128 x 64 and 64 x 128 tiles (skinny products at l = 272)
                                 (8192, 272, 1024), (272, 8192, 1024), (8192, 448, 640), (448, 8192, 520),
                                 # 256 x 256 tiles with 64-byte stages: whole and ragged M, N, K
                                 (4096, 4096, 2048), (4100, 4000, 2100),
                                 # one round of 128 .. 256 tiles over a long K: two K slices
                                 (416, 8192, 8192), (450, 4000, 8200)])
def test_gemm_int_bit_exact(lib, fmt, MNK):
    M, N, K = MNK
    rng = np.random.default_rng(M * 7 + N * 11 + K)
    qmax = 127 if fmt == "int8" else 7
    L, R = _int_operands(rng, M, N, K, qmax)
    dL = f32(rng.uniform(1e-3, 1e-1, M))
    dR = f32(rng.uniform(1e-3, 1e-1, N))
    Lq, Rq = g(_pack(L, fmt, K), torch.uint8), g(_pack(R, fmt, K), torch.uint8)
    acc = torch.empty((M, N), dtype=torch.int32, device=DEV)
    ws = torch.empty(max(1, lib.lramm_gemm_nt_workspace(M, N, K, fmt)), dtype=torch.uint8, device=DEV)
    C = lib.lramm_gemm_nt(M, N, K, fmt, Lq, g(dL), Rq, g(dR), acc_out=acc, ws=ws)
    ref_acc = OG.int_gemm(L, R.T)
    assert np.array_equal(acc.cpu().numpy().astype(np.int64), ref_acc)
    assert np.array_equal(C.cpu().numpy().astype(np.float64), OG.epilogue(ref_acc, dL, dR))
    # without split-K workspace: same bits
    C2 = lib.lramm_gemm_nt(M, N, K, fmt, Lq, g(dL), Rq, g(dR))
    assert torch.equal(C, C2)


def test_gemm_alpha_beta_and_bf16_out(lib):
    rng = np.random.default_rng(3)
    M, N, K = 200, 150, 333
    L, R = _int_operands(rng, M, N, K, 127)
    dL = f32(rng.uniform(1e-3, 1e-1, M))
    dR = f32(rng.uniform(1e-3, 1e-1, N))
    Cin = f32(rng.standard_normal((M, N)))
    Lq, Rq = g(_pack(L, "int8", K), torch.uint8), g(_pack(R, "int8", K), torch.uint8)
    C = g(Cin)
    lib.lramm_gemm_nt(M, N, K, "int8", Lq, g(dL), Rq, g(dR), alpha=0.5, beta=-1.5, C=C)
    ref = OG.epilogue(OG.int_gemm(L, R.T), dL, dR, 0.5, -1.5, Cin)
    assert np.array_equal(C.cpu().numpy().astype(np.float64), ref)
    Cb = lib.lramm_gemm_nt(M, N, K, "int8", Lq, g(dL), Rq, g(dR), ctype=torch.bfloat16)
    refb = bf16_round(OG.epilogue(OG.int_gemm(L, R.T), dL, dR))
    assert np.array_equal(Cb.float().cpu().numpy().astype(np.float64), refb)


@pytest.mark.parametrize("MNK", [(64, 64, 64), (100, 37, 257), (512, 512, 2048), (4100, 4000, 2100),
                                 (416, 8192, 8192)])
def test_gemm_bf16_operands(lib, MNK):
    M, N, K = MNK
    rng = np.random.default_rng(K)
    L = bf16_round(rng.standard_normal((M, K)))
    R = bf16_round(rng.standard_normal((N, K)))
    Lq, dL = lib.lramm_quantize(g(L), "bf16")
    Rq, dR = lib.lramm_quantize(g(R), "bf16")
    C = lib.lramm_gemm_nt(M, N, K, "bf16", Lq, dL, Rq, dR).double().cpu().numpy()
    ref = L @ R.T
    assert OL.rel_fro(C, ref) <= 1e-6 * np.sqrt(K / 64) + 1e-7


@pytest.mark.parametrize("MNK", [(3000, 2900, 300), (4096, 4096, 448), (2200, 4100, 1000)])
@pytest.mark.parametrize("c_bf16", [False, True])
def test_gemm_bf16_short_k(lib, MNK, c_bf16):
    """bf16 codes with K of at most 16 stages over at least 512 tiles of
    128 x 128 (the single-buffered kernel at three or four workgroups per CU,
    as in G2): every output within the FP32 accumulation bound, ragged M, N
    and K included."""
    M, N, K = MNK
    print(f"bf16 short-K GEMM {M}x{N}x{K} bf16 out {c_bf16}", flush=True)
    rng = np.random.default_rng(M + N + K)
    L = bf16_round(rng.standard_normal((M, K)))
    R = bf16_round(rng.standard_normal((N, K)) * np.exp(rng.uniform(-3, 3, (N, 1))))
    Lq, dL = lib.lramm_quantize(g(L), "bf16")
    Rq, dR = lib.lramm_quantize(g(R), "bf16")
    C = lib.lramm_gemm_nt(M, N, K, "bf16", Lq, dL, Rq, dR, ctype=torch.bfloat16 if c_bf16 else torch.float32)
    _check_product("short K", C.double().cpu().numpy(), L, dL.cpu().numpy().astype(np.float64), R,
                   dR.cpu().numpy().astype(np.float64), "bf16", c_bf16=c_bf16)


@pytest.mark.parametrize("MNK", [(1, 1, 1), (64, 64, 64), (100, 37, 257), (130, 200, 1000), (512, 512, 4096)])
def test_gemm_fp8_operands(lib, MNK):
    # fp8 products are exact in FP32, but the 32x32x64 MFMA adds the 64
    # products of one instruction at reduced precision (measured: up to about
    # 2^-16 of their absolute sum), then accumulates in FP32.  Bound: 2^-14 of
    # sum|a b| (code units) for the in-instruction sums, K 2^-24 of it for the
    # FP32 accumulation, plus the two roundings of the epilogue.
    M, N, K = MNK
    rng = np.random.default_rng(M + 3 * N + 5 * K)
    L = f32(rng.standard_normal((M, K)) * np.exp(rng.uniform(-4, 4, (M, 1))))
    R = f32(rng.standard_normal((N, K)) * np.exp(rng.uniform(-4, 4, (N, 1))))
    Lq, dL = lib.lramm_quantize(g(L), "fp8")
    Rq, dR = lib.lramm_quantize(g(R), "fp8")
    Lc, dLr = OQ.quantize_rows(L, "fp8")
    Rc, dRr = OQ.quantize_rows(R, "fp8")
    assert np.array_equal(dL.cpu().numpy().astype(np.float64), dLr)
    ref = OG.epilogue(Lc @ Rc.T, dLr, dRr)
    S = np.abs(Lc) @ np.abs(Rc).T
    bound = dLr[:, None] * dRr[None, :] * ((2.0**-14 + K * 2.0**-24) * S) + \
        3 * np.spacing(np.abs(ref).astype(np.float32))
    ws = torch.empty(max(1, lib.lramm_gemm_nt_workspace(M, N, K, "fp8")), dtype=torch.uint8, device=DEV)
    for w in (ws, None):
        C = lib.lramm_gemm_nt(M, N, K, "fp8", Lq, dL, Rq, dR, ws=w).double().cpu().numpy()
        assert np.all(np.abs(C - ref) <= bound), np.max(np.abs(C - ref) - bound)
    # the fp8 product approximates the exact one at e4m3 resolution
    if K >= 64:
        assert OL.rel_fro(C, L @ R.T) < 0.1


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float32])
def test_dense_comparator(lib, dtype):
    M, N, K = 256, 192, 512
    rng = np.random.default_rng(11)
    L = rng.standard_normal((M, K))
    R = rng.standard_normal((N, K))
    if dtype == torch.bfloat16:
        L, R = bf16_round(L), bf16_round(R)
    else:
        L, R = f32(L), f32(R)
    C = lib.lramm_dense_gemm_nt(g(L, dtype), g(R, dtype)).double().cpu().numpy()
    assert OL.rel_fro(C, L @ R.T) <= 1e-5


# ------------------------------------------------------------------ Omega --

@pytest.mark.parametrize("kl", [(512, 74), (1001, 37), (4096, 272)])
def test_omega_matches_oracle_philox(lib, kl):
    k, l = kl
    OmT = lib.lramm_omega(12345, k, l).cpu().numpy().astype(np.float64)
    ref = OP.gaussian_omega(12345, k, l)
    diff = OmT.T != ref
    # Box-Muller in FP64 on both sides, rounded once: a mismatch needs an FP64
    # result within a few ulps of a binary32 rounding boundary
    assert diff.sum() <= max(2, ref.size // 10**6)
    assert np.max(np.abs(OmT.T - ref)) <= 1e-6 * np.max(np.abs(ref))


# ---------------------------------------------------------------- CholQR2 --

# l' / 32 = 1 .. 32 blocks: odd and even block counts, the one-launch chain
# up to l' = 704 and the launch-per-two-panels schedule past it (l' = 736),
# up to the largest width the library takes (l' = 1024)
@pytest.mark.parametrize("case", [(100, 5, 10.0), (64, 32, 10.0),
                                  (300, 40, 1.0), (512, 74, 1e3), (1000, 96, 1e6), (2048, 272, 30.0),
                                  (700, 33, 10.0), (800, 128, 100.0), (2000, 200, 1e4), (4096, 528, 30.0),
                                  (2500, 700, 10.0), (1500, 736, 10.0), (2048, 1024, 10.0)])
def test_cholqr2_matches_householder(lib, case):
    rows, l, cond = case
    rng = np.random.default_rng(rows + l)
    U, _ = np.linalg.qr(rng.standard_normal((rows, l)))
    V, _ = np.linalg.qr(rng.standard_normal((l, l)))
    Y = f32((U * np.logspace(0, -np.log10(cond), l)) @ V.T)
    flags = torch.zeros(1, dtype=torch.int32, device=DEV)
    Q = lib.lramm_cholqr2(g(Y), l, flags=flags)
    torch.cuda.synchronize()
    Qg = Q.cpu().numpy()
    assert not Qg[:, l:].any()
    Qg = Qg[:, :l]
    Qh, Rh = householder_qr(Y)
    assert np.max(np.abs(Qg.T @ Qg - np.eye(l))) <= 1e-13
    assert np.max(np.abs(Qg - Qh)) <= 2e-14 * cond * np.sqrt(l)
    assert int(flags.item()) == 0
    _check_r_factor(lib, Y, Q, Qg, l, Qh, Rh)


def _check_r_factor(lib, Y, Q, Qg, l, Qh=None, Rh=None):
    """lramm_r_factor on the GPU's own Q: exact zeros below the diagonal,
    each entry within the FP64 summation bound of Q^T Y (rows terms), and,
    given Householder's factors, R within |(Q - Q_h)^T Y| of theirs plus the
    two computations' rounding (Householder's backward error, first order
    gamma_{rows l}, and the sum's)."""
    R = lib.lramm_r_factor(g(Y, torch.float64 if Y.dtype == np.float64 else torch.float32), Q, l).cpu().numpy()
    rows = Y.shape[0]
    assert not np.tril(R, -1).any()
    ref = np.triu(Qg.T @ Y)
    bound = np.triu(2.0 * rows * 2.0**-53 * (np.abs(Qg).T @ np.abs(Y)))
    assert np.all(np.abs(R - ref) <= bound)
    if Rh is not None:
        dq = np.linalg.norm(Qg - Qh, axis=0)[:, None] * np.linalg.norm(Y, axis=0)[None, :]
        tol = dq + 2.0 * rows * (l + 2) * 2.0**-53 * np.linalg.norm(Y, axis=0)[None, :]
        assert np.all(np.abs(R - Rh) <= np.triu(tol) + 1e-300)
    return R


def test_cholqr2_two_streams_at_once(lib):
    """Two one-launch Cholesky grids that fit the GPU together (l = 200 and
    272 on 2048 rows, on two streams): each result equals its single-stream
    result bit for bit and no flag (stall, breakdown) is raised."""
    rng = np.random.default_rng(77)
    Ys = [g(f32(rng.standard_normal((2048, l)))) for l in (200, 272)]
    single = []
    for Y in Ys:
        flags = torch.zeros(1, dtype=torch.int32, device=DEV)
        single.append(lib.lramm_cholqr2(Y, Y.shape[1], flags=flags))
        torch.cuda.synchronize()
        assert int(flags.item()) == 0
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs, flags = [], []
    for Y, st in zip(Ys, streams):
        f = torch.zeros(1, dtype=torch.int32, device=DEV)
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            outs.append(lib.lramm_cholqr2(Y, Y.shape[1], flags=f))
        flags.append(f)
    torch.cuda.synchronize()
    for Q, Q1, f in zip(outs, single, flags):
        assert int(f.item()) == 0
        assert torch.equal(Q, Q1)


# (l, dependent column): the first half of block 0, the half sweep of a last
# block whose second half is padding (l = 40: columns 32..39 live), and the
# second half of a block in the first, second and a later diagonal step
@pytest.mark.parametrize("l,dead", [(50, 7), (40, 35), (64, 20), (90, 52), (130, 115)])
def test_cholqr2_f64_input_and_rank_deficiency(lib, l, dead):
    rng = np.random.default_rng(9)
    Y = rng.standard_normal((400, l))
    Y[:, dead] = 0.0
    flags = torch.zeros(1, dtype=torch.int32, device=DEV)
    Q = lib.lramm_cholqr2(g(Y, torch.float64), l, flags=flags)
    torch.cuda.synchronize()
    Qg = Q.cpu().numpy()[:, :l]
    assert int(flags.item()) & lib.FLAG_BREAKDOWN
    assert not Qg[:, dead].any()
    keep = [j for j in range(l) if j != dead]
    assert np.max(np.abs(Qg[:, keep].T @ Qg[:, keep] - np.eye(l - 1))) <= 1e-13
    # span is kept: Y = Q Q^T Y
    assert np.linalg.norm(Y - Qg @ (Qg.T @ Y)) <= 1e-12 * np.linalg.norm(Y)
    # the triangular factor: the dropped column's row is zero, Y = Q R
    R = _check_r_factor(lib, Y, Q, Qg, l)
    assert not R[dead].any()
    assert np.linalg.norm(Y - Qg @ R) <= 1e-12 * np.linalg.norm(Y)


# ------------------------------------------------------------- end to end --

def _run_forward(lib, A, B, r, p, q, fmt, omega=None, seed=0, alpha=1.0, beta=0.0, Cin=None,
                 a_type=torch.float32, c_type=torch.float32, sketch="gaussian", orth="cholqr2"):
    m, k = A.shape
    n = B.shape[1]
    plan = lib.LrammPlan(m, n, k, r, p, q, fmt, a_type, a_type, c_type, seed, alpha, beta, sketch=sketch,
                         orth=orth)
    ws = plan.workspace()
    C = g(Cin, c_type) if Cin is not None else None
    Ad, Bd = g(A, a_type), g(B, a_type)
    C = plan.forward(Ad, Bd, ws, C=C, omega=None if omega is None else g(omega))
    flags = plan.status(ws)
    return C.double().cpu().numpy(), plan, ws, flags, Ad


# Accumulation error of one product of codes, per element, in code units:
#   int8 / int4: none (exact integer sums);
#   bf16: products exact in FP32, K - 1 FP32 additions in any order:
#         |err| <= K 2^-24 sum|a b|;
#   fp8:  the same, plus the gfx950 32x32x64 f8f6f4 MFMA's own addition of the
#         64 products of one instruction, which is not IEEE-exact: 2^-14 of
#         their absolute sum (a hardware constant, 4x the largest deviation
#         seen on random operands by test_gemm_fp8_operands).
ACC_REL = {"int8": 0.0, "int4": 0.0, "bf16": 1.0, "fp8": 1.0}


def _check_product(name, out, Lc, dL, Rc, dR, fmt, col_first=False, alpha=1.0, c_bf16=False):
    """GPU output of one product against its own codes: bit-exact for the
    integer formats, within the accumulation bound (and two roundings of
    the epilogue) for bf16 / fp8.  c_bf16: the output was rounded to bf16."""
    acc = Lc @ Rc.T
    if fmt == "bf16":   # no scales (the product ignores them)
        dL, dR = np.ones(Lc.shape[0]), np.ones(Rc.shape[0])
    f1, f2 = (dR[None, :], dL[:, None]) if col_first else (dL[:, None], dR[None, :])
    ref = OQ.fl32(OQ.fl32(OQ.fl32(acc) * f1) * f2)
    if alpha != 1.0:
        ref = OQ.fl32(OQ.fl32(alpha) * ref)
    if c_bf16:
        ref = bf16_round(ref)
    if fmt in ("int8", "int4") and not c_bf16:
        assert np.array_equal(out, ref), f"{name}: {np.max(np.abs(out - ref))}"
        return
    K = Lc.shape[1]
    S = np.abs(Lc) @ np.abs(Rc).T
    eacc = ACC_REL[fmt] * (K * 2.0**-24 + (2.0**-14 if fmt == "fp8" else 0.0)) * S
    ulps = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    bound = eacc * np.abs(f1) * np.abs(f2) * abs(alpha) * (1 + 2.0**-22) + 3 * ulps
    if c_bf16:
        # the GPU rounds its own FP32 value to bf16: one bf16 ulp (at most
        # 2^-7 of the magnitude) apart when the two straddle a rounding point
        bound = bound + (np.abs(ref) + bound) * 2.0**-7
    bad = np.abs(out - ref) > bound
    assert not bad.any(), f"{name}: {bad.sum()} elements past the bound, worst {np.max(np.abs(out - ref) - bound)}"


def _raw(plan, ws, name, A=None, rows=None):
    """Codes (bytes, on the host; only the given rows), scales, K, format of
    one quantised operand of the last forward."""
    c, sc, K, f = plan.codes(ws, name, A)
    if rows is not None:
        c, sc = c[torch.as_tensor(rows, device=c.device)], sc[torch.as_tensor(rows, device=c.device)]
    # on the direct bf16 path the A_rows scales are not written (the codes
    # are A itself, scale 1): whatever bits they hold are never used
    with np.errstate(invalid="ignore"):
        return c.cpu().numpy(), sc.cpu().numpy().astype(np.float64), K, f


def _check_codes(name, raw, K, fmt, X_rows, mismatch=0):
    """Codes the GPU wrote for the vectors that are the rows of X_rows
    (binary32 values) equal the oracle quantiser's, bit for bit (up to
    ``mismatch`` codes, for inputs that the two sides compute independently)."""
    ref_c, ref_d = OQ.quantize_rows(X_rows, fmt)
    got = codes_from(raw, fmt, K)[0]
    assert np.sum(got != ref_c) <= mismatch, name
    assert not pad_bytes(raw, fmt, K).any(), name
    return got.astype(np.float64)


def one_pass_q_tol(Y):
    """Bound on ||Q_a - Q_b||_F for two one-pass Cholesky QRs of the same
    full-rank Y in FP64 with different rounding orders, each within the
    first-order forward error of the exact Q: the Gram and the Cholesky
    perturb R^T R by (m + l + 1) u ||Y||_F^2, which moves Q by at most
    sqrt(l / 2) (m + l + 1) u kF^2 (kF = ||Y||_F / sigma_min), the solves add
    m l u cond(Y); a factor 2 for second-order terms, 2 for two computations."""
    m, l = Y.shape
    sv = np.linalg.svd(Y, compute_uv=False)
    u = 2.0**-53
    kF = np.linalg.norm(Y) / sv[-1]
    return 4.0 * (np.sqrt(l / 2.0) * (m + l + 1) * u * kF**2 + m * l * u * sv[0] / sv[-1])


def check_stages(lib, plan, ws, A, B, C, fmt, q, Ad=None, omega=None, omega_mismatch=0, alpha=1.0, sample=None,
                 c_bf16=False, srht_seed=None, one_pass=False):
    """Every stage of the last forward on its own inputs (binary32 values as
    float64 arrays A, B; C the GPU output): the codes of each quantised
    operand against the oracle quantiser applied to the GPU's own input to
    that quantiser, each product against the exact product of those codes,
    and Q against Householder QR of the GPU's last sketch -- or, with
    ``sample`` (row / column indices), every product on those rows or columns
    of its output and Q's orthonormality and span at full size."""
    fs, fp, f1, f2 = fmt
    Y = plan.intermediate(ws, "Y").double().cpu().numpy()
    Qg = plan.intermediate(ws, "Q").cpu().numpy()
    Bt = plan.intermediate(ws, "Bt").double().cpu().numpy()
    Tt = plan.intermediate(ws, "Tt").double().cpu().numpy()
    l = Y.shape[1]
    rows = np.arange(A.shape[0]) if sample is None else sample
    cols = np.arange(A.shape[1]) if sample is None else sample
    ncols = np.arange(B.shape[1]) if sample is None else sample
    dec = lambda raw, f, K: codes_from(raw, f, K)[0].astype(np.float64)
    if srht_seed is not None and q == 0:
        # the structured sketch: bit for bit the binary32 transform
        ref = OS.srht_sketch(A[rows], srht_seed, l, "fp32")
        assert np.array_equal(Y[rows], ref), f"srht sketch: {np.sum(Y[rows] != ref)} entries differ"
    else:
        # sketch: A by rows x (Omega or Q_Z) by columns -> Y
        rawA, dLa, K, _ = _raw(plan, ws, "A_rows", Ad, rows)
        La = _check_codes("A rows", rawA, K, fs, A[rows])
        rawS, dRs, _, _ = _raw(plan, ws, "sketch_R")
        Rs = dec(rawS, fs, K)
        if q == 0 and omega is not None:
            _check_codes("Omega", rawS, K, fs, omega.T, omega_mismatch)
        _check_product("sketch", Y[rows], La, dLa, Rs, dRs, fs)
    # orthonormalisation of the GPU's own last sketch
    if one_pass:
        # one Cholesky QR pass, against the oracle's on the same Y
        Qo, _, dropped = OQR.cholesky_qr(Y, 64.0 * l * 2.0**-53)
        assert dropped == []
        d = np.linalg.norm(Qg - Qo)
        tol = one_pass_q_tol(Y)
        print(f"one-pass Q: ||Q_gpu - Q_oracle||_F = {d:.3e} (bound {tol:.3e}), "
              f"||Q^T Q - I||_max = {np.max(np.abs(Qg.T @ Qg - np.eye(l))):.3e}")
        assert d <= tol
    else:
        assert np.max(np.abs(Qg.T @ Qg - np.eye(l))) <= 1e-12
        if sample is None:
            Qh, _ = householder_qr(Y)
            assert np.max(np.abs(Qg - Qh)) <= 1e-11
        else:
            assert np.linalg.norm(Y - Qg @ (Qg.T @ Y)) <= 1e-12 * np.linalg.norm(Y)
    # projection: Q by columns x A by columns -> Bt (l x k)
    rawQc, dLq, Kq, _ = _raw(plan, ws, "Q_cols")
    Lq = _check_codes("Q cols", rawQc, Kq, fp, OQ.fl32(Qg).T)
    try:
        rawAc, dRa, _, _ = _raw(plan, ws, "A_cols", rows=cols)
        Ra = _check_codes("A cols", rawAc, Kq, fp, A.T[cols])
    except lib.LrammError as e:
        # bf16 A read in place (stored K-major): its values are the codes
        assert e.code == lib._lib.E_INVALID and fp == "bf16"
        Ra, dRa = A.T[cols], np.ones(len(cols))
    _check_product("projection", Bt[:, cols], Lq, dLq, Ra, dRa, fp)
    # G1: B by columns x Bt by rows -> T^T (n x l), T's row factor first
    try:
        rawBc, dLb, Kb, _ = _raw(plan, ws, "B_cols", rows=ncols)
        Lb = _check_codes("B cols", rawBc, Kb, f1, B.T[ncols])
    except lib.LrammError as e:
        assert e.code == lib._lib.E_INVALID and f1 == "bf16"
        Lb, dLb, Kb = B.T[ncols], np.ones(len(ncols)), B.shape[0]
    rawBt, dRb, _, _ = _raw(plan, ws, "Bt_rows")
    Rb = _check_codes("Bt rows", rawBt, Kb, f1, Bt)
    _check_product("G1", Tt[ncols], Lb, dLb, Rb, dRb, f1, col_first=True)
    # G2: Q by rows x T^T by rows -> C
    rawQr, dLr, Kl, _ = _raw(plan, ws, "Q_rows", rows=rows)
    Lr = _check_codes("Q rows", rawQr, Kl, f2, OQ.fl32(Qg)[rows])
    rawTt, dRt, _, _ = _raw(plan, ws, "Tt_rows")
    Rt = _check_codes("Tt rows", rawTt, Kl, f2, Tt)
    _check_product("G2", C[rows], Lr, dLr, Rt, dRt, f2, alpha=alpha, c_bf16=c_bf16)


CASES = [
    # m, k, n, r, p, q, tau, fmt[, noise]
    (512, 512, 512, 64, 10, 1, 32.0, ("int8",) * 4),     # the small plain-LRAMM configuration
    (512, 512, 512, 64, 10, 0, 32.0, ("int8",) * 4),
    (512, 512, 512, 64, 10, 2, 32.0, ("int8",) * 4),
    (300, 257, 190, 20, 5, 1, 12.0, ("int8",) * 4),      # ragged
    (640, 384, 512, 100, 12, 1, 40.0, ("int8", "int8", "int4", "int4")),
    (512, 512, 512, 64, 10, 1, 32.0, ("int4",) * 4),
    (2048, 4096, 512, 64, 16, 1, 64.0, ("int8",) * 4),   # long K: split-K products
    # the at-scale workload (4096^3, l = 272 on 128 x 64 tiles and the
    # one-launch Cholesky at l' = 288, entrywise noise)
    (4096, 4096, 4096, 256, 16, 1, 128.0, ("int8",) * 4, 1e-4),
]


@pytest.mark.parametrize("case", CASES)
def test_lramm_forward_matches_oracle(lib, case):
    m, k, n, r, p, q, tau, fmt = case[:8]
    noise = case[8] if len(case) > 8 else 0.0
    print(f"forward case {m}x{k}x{n} r={r} p={p} q={q} {fmt}", flush=True)
    A, s = synth.lowrank(m, k, synth.spectrum("exp", min(m, k), tau), 0, noise_var=noise)
    B = synth.gaussian(k, n, 100)
    om = synth.omega(k, r + p, 1)
    C, plan, ws, flags, Ad = _run_forward(lib, A, B, r, p, q, fmt, omega=om)
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    check_stages(lib, plan, ws, A64, B64, C, fmt, q, Ad=Ad, omega=om.astype(np.float64))
    ref = OL.lramm_forward(A64, B64, r, p, q, fmt, omega=om.astype(np.float64))
    err = OL.rel_fro(C, ref["C"])
    assert err <= 1e-5, err
    assert flags == 0
    Qg, Btg = plan.factors(ws)
    assert np.max(np.abs(Qg.cpu().numpy() - ref["Q"])) <= 1e-11
    assert OL.rel_fro(Btg.cpu().numpy(), ref["Bt"]) <= 1e-5


def test_lramm_bf16_input_l400_long_k(lib):
    """bf16 inputs, l = 400 (the one-launch Cholesky at l' = 416), K = 8192,
    int8 stages: against the independent oracle at 1e-5."""
    m, k, n, r, p, q = 2048, 8192, 1024, 384, 16, 0
    A, _ = synth.lowrank(m, k, synth.spectrum("exp", m, 64.0), 0, dtype="bf16")
    B = synth.gaussian(k, n, 100, dtype="bf16")
    om = synth.omega(k, r + p, 1)
    C, plan, ws, flags, Ad = _run_forward(lib, A, B, r, p, q, ("int8",) * 4, omega=om, a_type=torch.bfloat16)
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    check_stages(lib, plan, ws, A64, B64, C, ("int8",) * 4, q, Ad=Ad, omega=om.astype(np.float64))
    ref = OL.lramm_forward(A64, B64, r, p, q, ("int8",) * 4, omega=om.astype(np.float64))
    assert OL.rel_fro(C, ref["C"]) <= 1e-5
    assert flags == 0


ONE_PASS_CASES = [
    # m, k, n, r, p, q, tau, fmt, a dtype, sketch[, noise]
    (512, 512, 512, 64, 10, 1, 32.0, ("int8",) * 4, "fp32", "gaussian"),
    (300, 257, 190, 20, 5, 2, 12.0, ("int8",) * 4, "fp32", "gaussian"),
    (4096, 4096, 4096, 256, 16, 1, 128.0, ("int8",) * 4, "fp32", "gaussian", 1e-4),
    (2048, 8192, 1024, 384, 32, 0, 64.0, ("bf16",) * 4, "bf16", "srht"),
    # bf16 projection and G2: the last solve also writes Q's two code layouts
    # (l = 400 inside l' = 416, ragged rows, after a power step; the odd block
    # count takes the solve that forms the last block from the others)
    (1000, 3000, 700, 368, 32, 1, 48.0, ("bf16",) * 4, "fp32", "gaussian"),
    (3000, 1000, 500, 100, 28, 0, 24.0, ("int8", "bf16", "int8", "bf16"), "fp32", "gaussian"),
    # 8192 rows: the solve with two 16-row halves per workgroup, l = 400 inside l' = 416
    (8192, 2048, 512, 368, 32, 0, 64.0, ("bf16",) * 4, "bf16", "srht"),
]


@pytest.mark.parametrize("case", ONE_PASS_CASES)
def test_lramm_one_pass_matches_oracle(lib, case):
    """Plans with one Cholesky QR pass per orthonormalisation: every stage on
    its own inputs, Q against the oracle's one-pass QR of the GPU's own last
    sketch within the first-order bound, and C against the oracle forward
    that orthonormalises the same way (1e-5 for integer stages; equally good
    approximations of A B for bf16, whose products accumulate in FP32)."""
    m, k, n, r, p, q, tau, fmt, dt, sketch = case[:10]
    noise = case[10] if len(case) > 10 else 0.0
    print(f"one-pass forward {m}x{k}x{n} r={r} p={p} q={q} {fmt} {dt} {sketch}", flush=True)
    A, _ = synth.lowrank(m, k, synth.spectrum("exp", min(m, k), tau), 0, noise_var=noise, dtype=dt)
    B = synth.gaussian(k, n, 100, dtype=dt)
    a_type = torch.bfloat16 if dt == "bf16" else torch.float32
    om = synth.omega(k, r + p, 1) if sketch == "gaussian" else None
    C, plan, ws, flags, Ad = _run_forward(lib, A, B, r, p, q, fmt, omega=om, seed=21, a_type=a_type, sketch=sketch,
                                          orth="cholqr")
    assert flags == 0
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    check_stages(lib, plan, ws, A64, B64, C, fmt, q, Ad=Ad, omega=None if om is None else om.astype(np.float64),
                 srht_seed=21 if sketch == "srht" else None, one_pass=True)
    ref = OL.lramm_forward(A64, B64, r, p, q, fmt, omega=None if om is None else om.astype(np.float64), seed=21,
                           sketch=sketch, one_pass=True)
    err = OL.rel_fro(C, ref["C"])
    if all(f in ("int8", "int4") for f in fmt):
        assert err <= 1e-5, err
    else:
        Cex = A64 @ B64
        e_gpu, e_ref = OL.rel_fro(C, Cex), OL.rel_fro(ref["C"], Cex)
        print(f"one-pass {fmt}: rel-F vs oracle {err:.3e}; vs exact gpu {e_gpu:.3e} oracle {e_ref:.3e}")
        assert e_gpu <= 2.0 * e_ref and e_ref <= 2.0 * e_gpu, (e_gpu, e_ref)


@pytest.mark.parametrize("shape", ["rows", "block"])
def test_lramm_rank_below_l(lib, shape):
    """rank(A) = 40 < l = 74, with the dependence exact in every sketch: A has
    40 nonzero rows ("rows", q = 0: each column of Y = A Omega lies in those
    40 coordinates, so rounding cannot lift the rank), or a nonzero 40 x 40
    block ("block", q = 1: Z = A^T Q as well).  CholeskyQR drops l - 40
    columns of every orthonormalisation (zero Q columns, breakdown flag), and
    the result equals the oracle that leaves dependent sketch columns out
    the same way (not the completion vectors of a plain Householder QR, which
    would change Q's row scales)."""
    m = k = n = 512
    rng = np.random.default_rng(12)
    A = np.zeros((m, k), np.float32)
    if shape == "rows":
        A[:40, :] = rng.standard_normal((40, k)).astype(np.float32)
        q = 0
    else:
        A[:40, :40] = rng.standard_normal((40, 40)).astype(np.float32)
        q = 1
    B = synth.gaussian(k, n, 112)
    om = synth.omega(k, 74, 13)
    fmt = ("int8",) * 4
    C, plan, ws, flags, Ad = _run_forward(lib, A, B, 64, 10, q, fmt, omega=om)
    assert flags & lib.FLAG_BREAKDOWN
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    ref = OL.lramm_forward(A64, B64, 64, 10, q, fmt, omega=om.astype(np.float64), drop_dependent=True)
    assert all(len(d) == 74 - 40 for d in ref["dropped"])
    Qg = plan.factors(ws)[0].cpu().numpy()
    dead = ref["dropped"][-1]
    assert not Qg[:, dead].any()
    assert np.max(np.abs(Qg - ref["Q"])) <= 1e-11
    assert OL.rel_fro(C, ref["C"]) <= 1e-5
    keep = [j for j in range(74) if j not in dead]
    assert np.max(np.abs(Qg[:, keep].T @ Qg[:, keep] - np.eye(len(keep)))) <= 1e-12


FP_CASES = [
    # m, k, n, r, p, q, tau, fmt, io dtype, seeded Omega
    (512, 512, 512, 64, 10, 1, 32.0, ("bf16",) * 4, torch.float32, False),
    (512, 512, 512, 64, 10, 1, 32.0, ("fp8",) * 4, torch.float32, False),
    (300, 257, 190, 20, 5, 1, 12.0, ("fp8",) * 4, torch.float32, False),
    (640, 384, 512, 100, 12, 1, 40.0, ("int8", "int8", "fp8", "fp8"), torch.float32, False),
    (640, 384, 512, 100, 12, 0, 40.0, ("bf16", "bf16", "int8", "int8"), torch.float32, False),
    # bf16 inputs straight into the bf16 sketch, Omega generated on the GPU
    (1024, 2048, 512, 200, 16, 0, 48.0, ("bf16",) * 4, torch.bfloat16, True),
    (1024, 2048, 512, 120, 16, 1, 48.0, ("bf16",) * 4, torch.bfloat16, True),
    (700, 1536, 300, 90, 10, 0, 32.0, ("int8", "bf16", "bf16", "bf16"), torch.bfloat16, True),
    # projections summed over K slices whose slice sum also writes Bt's bf16
    # codes: a ragged k (1002, padded to 1024; scalar quads) and k % 4 == 0
    (4096, 1002, 300, 84, 16, 0, 32.0, ("bf16",) * 4, torch.float32, False),
    (4096, 1000, 300, 84, 16, 1, 32.0, ("int8", "bf16", "bf16", "bf16"), torch.bfloat16, True),
    # G1 as T = Bt_q B with B read in place, summed over 16 K slices whose sum
    # also writes T's column codes, transposed (n = 1000: a ragged last tile)
    (1024, 4096, 1000, 84, 16, 0, 32.0, ("bf16",) * 4, torch.bfloat16, True),
]


@pytest.mark.parametrize("case", FP_CASES)
def test_lramm_forward_fp_formats(lib, case):
    """Formats with FP32 accumulation: the MFMA's order of FP32 additions
    cannot be replayed, so every stage is checked on the GPU's own inputs
    (codes bit-exact, each product within its accumulation bound).  The end
    result against the independent oracle is reported, and both must be
    equally good approximations of the exact product (within a factor 2)."""
    m, k, n, r, p, q, tau, fmt, io, seeded = case
    dt = "bf16" if io == torch.bfloat16 else "fp32"
    A, s = synth.lowrank(m, k, synth.spectrum("exp", min(m, k), tau), 0, dtype=dt)
    B = synth.gaussian(k, n, 100, dtype=dt)
    om = None if seeded else synth.omega(k, r + p, 1)
    C, plan, ws, flags, Ad = _run_forward(lib, A, B, r, p, q, fmt, omega=om, seed=3, a_type=io)
    assert flags == 0
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    om64 = OP.gaussian_omega(3, k, r + p).astype(np.float32).astype(np.float64) if seeded else \
        om.astype(np.float64)
    check_stages(lib, plan, ws, A64, B64, C, fmt, q, Ad=Ad, omega=om64, omega_mismatch=2 if seeded else 0)
    ref = OL.lramm_forward(A64, B64, r, p, q, fmt, omega=om64)
    err = OL.rel_fro(C, ref["C"])
    Cex = A64 @ B64
    e_gpu, e_ref = OL.rel_fro(C, Cex), OL.rel_fro(ref["C"], Cex)
    print(f"fmt {fmt}: end-to-end rel-F vs oracle {err:.3e}; vs exact gpu {e_gpu:.3e} oracle {e_ref:.3e}")
    assert e_gpu <= 2.0 * e_ref and e_ref <= 2.0 * e_gpu, (e_gpu, e_ref)


def test_target_workload_sampled_stages(lib):
    """The headline workload at full size (8192^3 bf16, sigma_i = exp(-i/64),
    l = 448, q = 0, bf16 in every stage, Omega from the seed), in the launch
    configuration the bench times: every stage checked on 96 sampled rows /
    columns of its output against its own codes, and Q's orthonormality and
    span at full size."""
    m = k = n = 8192
    A, _ = synth.lowrank(m, k, synth.spectrum("exp", m, 64.0), 0, dtype="bf16")
    B = synth.gaussian(k, n, 100, dtype="bf16")
    fmt = ("bf16",) * 4
    plan = lib.LrammPlan(m, n, k, 416, 32, 0, fmt, torch.bfloat16, torch.bfloat16, torch.bfloat16, 1,
                         exclusive=True)
    ws = plan.workspace()
    Ad, Bd = g(A, torch.bfloat16), g(B, torch.bfloat16)
    C = plan.forward(Ad, Bd, ws)
    assert plan.status(ws) == 0
    rng = np.random.default_rng(5)
    sample = np.sort(rng.choice(8192, 96, replace=False))
    om = OP.gaussian_omega(1, k, 448).astype(np.float32).astype(np.float64)
    Cs = C.float().cpu().numpy().astype(np.float64)
    check_stages(lib, plan, ws, A.astype(np.float64), B.astype(np.float64), Cs, fmt, 0, Ad=Ad, omega=om,
                 omega_mismatch=3, sample=sample, c_bf16=True)


def test_headline_setting_sampled_stages(lib):
    """The bench's headline setting at full size: 8192^3 bf16, sigma_i =
    exp(-i/64), l = 416 (r = 384, p = 32), q = 0, bf16 in every stage, the
    structured sketch from seed 1 and one Cholesky QR pass, in the launch
    configuration the bench times (exclusive plan, bf16 C).  The sketch is
    the oracle's binary32 transform to the bit on 96 sampled rows; every
    product is checked on 96 sampled rows / columns against its own codes;
    Q's orthonormality (one-pass bound) and span are checked at full size."""
    m = k = n = 8192
    print("headline setting 8192^3 bf16 l 416 srht one pass", flush=True)
    A, _ = synth.lowrank(m, k, synth.spectrum("exp", m, 64.0), 0, dtype="bf16")
    B = synth.gaussian(k, n, 100, dtype="bf16")
    fmt = ("bf16",) * 4
    plan = lib.LrammPlan(m, n, k, 384, 32, 0, fmt, torch.bfloat16, torch.bfloat16, torch.bfloat16, 1,
                         exclusive=True, sketch="srht", orth="cholqr")
    ws = plan.workspace()
    Ad, Bd = g(A, torch.bfloat16), g(B, torch.bfloat16)
    C = plan.forward(Ad, Bd, ws)
    assert plan.status(ws) == 0
    rng = np.random.default_rng(6)
    sample = np.sort(rng.choice(8192, 96, replace=False))
    Cs = C.float().cpu().numpy().astype(np.float64)
    check_stages(lib, plan, ws, A.astype(np.float64), B.astype(np.float64), Cs, fmt, 0, Ad=Ad, sample=sample,
                 c_bf16=True, srht_seed=1, one_pass=True)


def test_lramm_seeded_omega_and_alpha_beta(lib):
    m = k = n = 384
    A, _ = synth.lowrank(m, k, synth.spectrum("exp", 384, 24.0), 3)
    B = synth.gaussian(k, n, 103)
    Cin = synth.gaussian(m, n, 7)
    C, *_ = _run_forward(lib, A, B, 48, 8, 1, ("int8",) * 4, seed=77, alpha=0.75, beta=0.5, Cin=Cin)
    ref = OL.lramm_forward(A.astype(np.float64), B.astype(np.float64), 48, 8, 1, seed=77, alpha=0.75, beta=0.5,
                           Cin=Cin.astype(np.float64))
    assert OL.rel_fro(C, ref["C"]) <= 1e-5


def test_lramm_bf16_io(lib):
    m = k = n = 512
    A, _ = synth.lowrank(m, k, synth.spectrum("exp", 512, 32.0), 0, dtype="bf16")
    B = synth.gaussian(k, n, 100, dtype="bf16")
    om = synth.omega(k, 74, 1)
    C, *_ = _run_forward(lib, A, B, 64, 10, 1, ("int8",) * 4, omega=om, a_type=torch.bfloat16,
                              c_type=torch.bfloat16)
    ref = OL.lramm_forward(A.astype(np.float64), B.astype(np.float64), 64, 10, 1, omega=om.astype(np.float64))
    assert OL.rel_fro(C, bf16_round(ref["C"])) <= 1e-5


def test_lramm_deterministic(lib):
    m = k = n = 512
    A, _ = synth.lowrank(m, k, synth.spectrum("exp", 512, 32.0), 0)
    B = synth.gaussian(k, n, 100)
    C1, *_ = _run_forward(lib, A, B, 64, 10, 1, ("int8",) * 4, seed=5)
    C2, *_ = _run_forward(lib, A, B, 64, 10, 1, ("int8",) * 4, seed=5)
    assert np.array_equal(C1, C2)


def test_lramm_nonfinite_input_flag(lib):
    A = np.ones((128, 128), np.float32)
    A[5, 6] = np.nan
    B = np.ones((128, 64), np.float32)
    plan = lib.LrammPlan(128, 64, 128, 16, 4, 0)
    ws = plan.workspace()
    plan.forward(g(A), g(B), ws)
    with pytest.raises(lib.LrammError):
        plan.status(ws)


@pytest.mark.parametrize("where", ["A_late_row", "B_late_col"])
def test_lramm_nonfinite_in_late_workgroup(lib, where):
    """A NaN in the last rows of A (quantised by the last workgroups of the
    row pass) or the last column of B is reported: the status word is cleared
    before any kernel that may set it.  matmul() raises on it by default."""
    m, k, n = 4096, 256, 192
    A = np.ones((m, k), np.float32)
    B = np.ones((k, n), np.float32)
    if where == "A_late_row":
        A[m - 3, k - 1] = np.nan
    else:
        B[k - 2, n - 1] = np.inf
    plan = lib.LrammPlan(m, n, k, 16, 4, 0)
    ws = plan.workspace()
    plan.forward(g(A), g(B), ws)
    with pytest.raises(lib.LrammError) as e:
        plan.status(ws)
    assert e.value.code == 5
    with pytest.raises(lib.LrammError):
        lib.matmul(g(A), g(B), 16, 4, 0)
    # a clean input on the same workspace reports nothing
    plan.forward(g(np.ones((m, k), np.float32)), g(np.ones((k, n), np.float32)), ws)
    assert plan.status(ws) & lib.FLAG_NONFINITE == 0


# ---------------------------------------------------------------- backward --

def test_backward_matches_exact_gradient(lib):
    m, k, n = 384, 320, 256
    A, _ = synth.lowrank(m, k, synth.spectrum("exp", 320, 24.0), 0)
    B = synth.gaussian(k, n, 100)
    om = synth.omega(k, 48, 1)
    At = g(A).requires_grad_(True)
    Bt = g(B).requires_grad_(True)
    cfg = lib.LRAMMConfig(r=40, p=8, q=1, omega=g(om))
    C = lib.LRAMMFunction.apply(At, Bt, cfg)
    dC = synth.gaussian(m, n, 9)
    C.backward(g(dC))
    ref = OL.lramm_forward(A.astype(np.float64), B.astype(np.float64), 40, 8, 1, omega=om.astype(np.float64))
    dA, dB = OL.lramm_backward(ref["Q"], A, B, dC)
    assert OL.rel_fro(At.grad.double().cpu().numpy(), dA) <= 1e-5
    assert OL.rel_fro(Bt.grad.double().cpu().numpy(), dB) <= 1e-5
    # recompute mode gives identical gradients
    At2 = g(A).requires_grad_(True)
    Bt2 = g(B).requires_grad_(True)
    cfg2 = lib.LRAMMConfig(r=40, p=8, q=1, omega=g(om), recompute=True)
    lib.LRAMMFunction.apply(At2, Bt2, cfg2).backward(g(dC))
    assert torch.equal(At.grad, At2.grad) and torch.equal(Bt.grad, Bt2.grad)


# ------------------------------------------------- side / transposed storage --

def test_transposed_storage_gives_identical_results(lib):
    """A and B passed as transposed storage (torch .t() views of their
    transposes) give the same C bit for bit: the quantisers read the stored
    rows or columns that hold the same vectors."""
    m, k, n = 384, 320, 256
    A, _ = synth.lowrank(m, k, synth.spectrum("exp", k, 24.0), 4)
    B = synth.gaussian(k, n, 104)
    om = g(synth.omega(k, 56, 5))
    Ad, Bd = g(A), g(B)
    C0 = lib.matmul(Ad, Bd, 48, 8, 1, omega=om)
    C1 = lib.matmul(g(A.T.copy()).t(), g(B.T.copy()).t(), 48, 8, 1, omega=om)
    assert torch.equal(C0, C1)


@pytest.mark.parametrize("trans", [(False, False), (True, True)])
def test_side_right_matches_oracle_on_transposed_problem(lib, trans):
    """side = right sketches B: the result is the one-sided method on
    C^T = B^T A^T (oracle run on (B^T, A^T), transposed back), bit for bit
    for int8 stages, with A and B given either way."""
    m, k, n = 512, 320, 384
    X = synth.gaussian(m, k, 6)
    W, _ = synth.lowrank(k, n, synth.spectrum("exp", min(k, n), 20.0), 7)
    ta, tb = trans
    Xd = g(X.T.copy()).t() if ta else g(X)
    Wd = g(W.T.copy()).t() if tb else g(W)
    # the transposed problem C^T = W^T X^T keeps the inner dimension k: Omega is k x l
    C = lib.matmul(Xd, Wd, 50, 8, 1, omega=g(synth.omega(k, 58, 8)), side="right").double().cpu().numpy()
    ref = OL.lramm_forward(W.T.astype(np.float64), X.T.astype(np.float64), 50, 8, 1,
                           omega=synth.omega(k, 58, 8).astype(np.float64))
    assert OL.rel_fro(C, ref["C"].T) <= 1e-5


def test_backward_side_right_bf16(lib):
    """side = right with bf16 activations and weight: the gradients of the
    frozen-Q surrogate C = A B Q Q^T, written in bf16, within half a bf16
    ulp per element (rel-F <= 2^-8) of the exact FP64 gradient taken with
    the oracle's Q (equal to the GPU's to 1e-11)."""
    m, k, n = 512, 256, 384
    X = synth.gaussian(m, k, 9, dtype="bf16")
    W, _ = synth.lowrank(k, n, synth.spectrum("exp", min(k, n), 16.0), 10, dtype="bf16")
    om = synth.omega(k, 40, 11)
    Xd = g(X, torch.bfloat16).requires_grad_(True)
    Wd = g(W, torch.bfloat16).requires_grad_(True)
    cfg = lib.LRAMMConfig(r=32, p=8, q=1, omega=g(om), side="right")
    C = lib.LRAMMFunction.apply(Xd, Wd, cfg)
    assert C.dtype == torch.bfloat16
    dC = synth.gaussian(m, n, 12, dtype="bf16")
    C.backward(g(dC, torch.bfloat16))
    X64, W64, dC64 = X.astype(np.float64), W.astype(np.float64), dC.astype(np.float64)
    ref = OL.lramm_forward(W64.T, X64.T, 32, 8, 1, omega=om.astype(np.float64))
    # the transposed problem's gradients: dA' = grad of W^T, dB' = grad of X^T
    dWt, dXt = OL.lramm_backward(ref["Q"], W64.T, X64.T, dC64.T)
    eX = OL.rel_fro(Xd.grad.double().cpu().numpy(), dXt.T)
    eW = OL.rel_fro(Wd.grad.double().cpu().numpy(), dWt.T)
    assert Xd.grad.dtype == torch.bfloat16 and Wd.grad.dtype == torch.bfloat16
    assert eX <= 2.0**-8 and eW <= 2.0**-8, (eX, eW)


def test_differentiable_layer_workload(lib):
    """The differentiable-layer workload: X 16384 x 4096 bf16 ~ N(0, 1) times
    W 4096 x 4096 = rank-256 part (sigma_i = exp(-i/64), unit-RMS entries) +
    entrywise noise of variance 1e-3, W sketched (side = right), r = 256,
    p = 16, q = 1, int8.  Forward against the oracle on the transposed
    problem (1e-5), backward against the exact frozen-Q gradient (bf16
    output: rel-F <= 2^-8)."""
    m, k, n = 16384, 4096, 4096
    X = synth.gaussian(m, k, 21, dtype="bf16")
    W, _ = synth.lowrank(k, n, synth.spectrum("exp", 256, 64.0), 22, noise_var=1e-3, dtype="bf16")
    om = synth.omega(k, 272, 23)
    Xd = g(X, torch.bfloat16).requires_grad_(True)
    Wd = g(W, torch.bfloat16).requires_grad_(True)
    cfg = lib.LRAMMConfig(r=256, p=16, q=1, omega=g(om), side="right")
    C = lib.LRAMMFunction.apply(Xd, Wd, cfg)
    dC = synth.gaussian(m, n, 24, dtype="bf16")
    C.backward(g(dC, torch.bfloat16))
    Cg = C.detach().double().cpu().numpy()
    del C
    X64, W64 = X.astype(np.float64), W.astype(np.float64)
    ref = OL.lramm_forward(W64.T, X64.T, 256, 16, 1, omega=om.astype(np.float64))
    assert OL.rel_fro(Cg, bf16_round(ref["C"].T)) <= 1e-5
    dWt, dXt = OL.lramm_backward(ref["Q"], W64.T, X64.T, dC.astype(np.float64).T)
    eX = OL.rel_fro(Xd.grad.double().cpu().numpy(), dXt.T)
    eW = OL.rel_fro(Wd.grad.double().cpu().numpy(), dWt.T)
    assert eX <= 2.0**-8 and eW <= 2.0**-8, (eX, eW)


# -------------------------------------------------------- two-sided Alg. 3 --

@pytest.mark.parametrize("d", [("int8", "int8", "int8"), ("int8", "int8", "int4"), ("int8", "int4", "int4"),
                               ("int4", "int4", "int4")])
def test_two_sided_matches_oracle(lib, d):
    """Alg. 3 on the GPU against the oracle's two-sided LRAMM: the small SVDs
    (singular values, signed U'), the FP64 factor products, and each of the
    three quantised products bit for bit on the GPU's own inputs; the end
    result against the independent oracle is reported."""
    from oracle import two_sided as TS
    m, k, n, r, p, q = 512, 384, 448, 40, 8, 1
    A, _ = synth.lowrank(m, k, synth.spectrum("exp", k, 12.0), 31)
    B, _ = synth.lowrank(k, n, synth.spectrum("exp", k, 14.0), 32)
    oa, ob = synth.omega(k, r + p, 33), synth.omega(n, r + p, 34)
    plan = lib.LrammTsPlan(m, n, k, r, p, q, ("int8", "int8"), d)
    ws = plan.workspace()
    D = plan.forward(g(A), g(B), ws, omega_a=g(oa), omega_b=g(ob)).double().cpu().numpy()
    assert plan.status(ws) == 0
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    ref = TS.lramm_two_sided(A64, B64, r, p, q, ("int8", "int8"), d, omega_a=oa.astype(np.float64),
                             omega_b=ob.astype(np.float64))
    v = {kk: plan.intermediate(ws, kk).double().cpu().numpy() for kk in
         ("Ut", "Vt", "W", "Zs", "E1", "E2", "SA", "SB", "UpA", "UpB")}
    assert np.max(np.abs(v["SA"][:, 0] - ref["S"]) / ref["S"][0]) <= 1e-12
    assert np.max(np.abs(v["SB"][:, 0] - ref["G"]) / ref["G"][0]) <= 1e-12
    Up_ref = np.linalg.svd(ref["BtA"], full_matrices=False)[0]
    Up_ref = TS.sign_fix(Up_ref, np.eye(Up_ref.shape[1]))[0][:, :r]
    assert np.max(np.abs(v["UpA"] - Up_ref)) <= 1e-9
    # factors: FP64 products rounded once to binary32
    for name, refv in (("Ut", ref["Ut"]), ("Vt", ref["Vt"]), ("W", ref["W"]), ("Zs", ref["Zs"])):
        assert OL.rel_fro(v[name], OQ.fl32(refv)) <= 1e-6, name
    # the chain, each product on the GPU's own operands: bit for bit
    from oracle.qgemm import qgemm
    assert np.array_equal(v["E1"], qgemm(v["Vt"], v["W"], d[0]))
    assert np.array_equal(v["E2"], qgemm(v["E1"], v["Zs"], d[1]))
    assert np.array_equal(D, qgemm(v["Ut"], v["E2"], d[2]))
    err = OL.rel_fro(D, ref["D"])
    Cex = A64 @ B64
    print(f"two-sided {d}: rel-F vs oracle {err:.2e}, vs exact gpu {OL.rel_fro(D, Cex):.3e} "
          f"oracle {OL.rel_fro(ref['D'], Cex):.3e}")
    assert err <= 1e-3
