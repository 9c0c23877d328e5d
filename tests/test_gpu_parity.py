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
from oracle import quant as OQ  # noqa: E402
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
    q = Xq.cpu().numpy()
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
                                 (4096, 4096, 2048), (4100, 4000, 2100)])
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


@pytest.mark.parametrize("MNK", [(64, 64, 64), (100, 37, 257), (512, 512, 2048), (4100, 4000, 2100)])
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

# l' / 32 = 1 .. 23 blocks: odd and even block counts, the one-launch chain
# up to l' = 704 and the launch-per-two-panels schedule past it (l' = 736)
@pytest.mark.parametrize("case", [(100, 5, 10.0), (64, 32, 10.0),
                                  (300, 40, 1.0), (512, 74, 1e3), (1000, 96, 1e6), (2048, 272, 30.0),
                                  (700, 33, 10.0), (800, 128, 100.0), (2000, 200, 1e4), (4096, 528, 30.0),
                                  (2500, 700, 10.0), (1500, 736, 10.0)])
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
    Qh, _ = householder_qr(Y)
    assert np.max(np.abs(Qg.T @ Qg - np.eye(l))) <= 1e-13
    assert np.max(np.abs(Qg - Qh)) <= 2e-14 * cond * np.sqrt(l)
    assert int(flags.item()) == 0


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


# ------------------------------------------------------------- end to end --

def _run_forward(lib, A, B, r, p, q, fmt, omega=None, seed=0, alpha=1.0, beta=0.0, Cin=None,
                 a_type=torch.float32, c_type=torch.float32):
    m, k = A.shape
    n = B.shape[1]
    plan = lib.LrammPlan(m, n, k, r, p, q, fmt, a_type, a_type, c_type, seed, alpha, beta)
    ws = plan.workspace()
    C = g(Cin, c_type) if Cin is not None else None
    C = plan.forward(g(A, a_type), g(B, a_type), ws, C=C, omega=None if omega is None else g(omega))
    flags = plan.status(ws)
    return C.double().cpu().numpy(), plan, ws, flags


CASES = [
    # m, k, n, r, p, q, tau, fmt
    (512, 512, 512, 64, 10, 1, 32.0, ("int8",) * 4),     # the small plain-LRAMM configuration
    (512, 512, 512, 64, 10, 0, 32.0, ("int8",) * 4),
    (512, 512, 512, 64, 10, 2, 32.0, ("int8",) * 4),
    (300, 257, 190, 20, 5, 1, 12.0, ("int8",) * 4),      # ragged
    (640, 384, 512, 100, 12, 1, 40.0, ("int8", "int8", "int4", "int4")),
    (512, 512, 512, 64, 10, 1, 32.0, ("int4",) * 4),
    (2048, 4096, 512, 64, 16, 1, 64.0, ("int8",) * 4),   # long K: split-K products
]


@pytest.mark.parametrize("case", CASES)
def test_lramm_forward_matches_oracle(lib, case):
    m, k, n, r, p, q, tau, fmt = case
    A, s = synth.lowrank(m, k, synth.spectrum("exp", min(m, k), tau), 0)
    B = synth.gaussian(k, n, 100)
    om = synth.omega(k, r + p, 1)
    C, plan, ws, flags = _run_forward(lib, A, B, r, p, q, fmt, omega=om)
    ref = OL.lramm_forward(A.astype(np.float64), B.astype(np.float64), r, p, q, fmt, omega=om.astype(np.float64))
    err = OL.rel_fro(C, ref["C"])
    assert err <= 1e-5, err
    assert flags == 0
    Qg, Btg = plan.factors(ws)
    Qg = Qg.cpu().numpy()
    assert np.max(np.abs(Qg - ref["Q"])) <= 1e-11
    assert OL.rel_fro(Btg.cpu().numpy(), ref["Bt"]) <= 1e-5


FP_CASES = [
    (512, 512, 512, 64, 10, 1, 32.0, ("bf16",) * 4),
    (512, 512, 512, 64, 10, 1, 32.0, ("fp8",) * 4),
    (300, 257, 190, 20, 5, 1, 12.0, ("fp8",) * 4),
    (640, 384, 512, 100, 12, 1, 40.0, ("int8", "int8", "fp8", "fp8")),
    (640, 384, 512, 100, 12, 0, 40.0, ("bf16", "bf16", "int8", "int8")),
]
# rel-F of one replayed stage (FP32 accumulation in the MFMA's own order;
# the fp8 MFMA adds within an instruction at reduced precision)
STAGE_TOL = {"int8": 1e-6, "int4": 1e-6, "bf16": 1e-5, "fp8": 1e-4}
# end to end against the independent oracle: the stage differences move
# values across quantiser rounding boundaries (one code step each), and the
# sketch directions that the quantisation noise dominates rotate with them;
# measured 1.2e-3 (bf16 stages) and 2.5e-2 (fp8 in every stage)
INDEP_TOL = {"int8": 1e-5, "int4": 1e-5, "bf16": 5e-3, "fp8": 6e-2}


@pytest.mark.parametrize("case", FP_CASES)
def test_lramm_forward_fp_formats(lib, case):
    """Formats with FP32 accumulation: every stage is replayed from the GPU's
    own input to that stage (the quantiser codes then agree bit for bit and
    only the accumulation order differs), and the end result is compared
    with the independent oracle at a looser tolerance."""
    m, k, n, r, p, q, tau, fmt = case
    A, s = synth.lowrank(m, k, synth.spectrum("exp", min(m, k), tau), 0)
    B = synth.gaussian(k, n, 100)
    om = synth.omega(k, r + p, 1)
    C, plan, ws, flags = _run_forward(lib, A, B, r, p, q, fmt, omega=om)
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    assert flags == 0
    l = r + p
    Y = plan.intermediate(ws, "Y").double().cpu().numpy()
    Qg = plan.intermediate(ws, "Q").cpu().numpy()
    Btg = plan.intermediate(ws, "Bt").double().cpu().numpy()
    Tg = plan.intermediate(ws, "Tt").double().cpu().numpy().T
    # orthonormalisation of the GPU's last sketch
    Qh, _ = householder_qr(Y)
    assert np.max(np.abs(Qg - Qh)) <= 1e-11
    assert np.max(np.abs(Qg.T @ Qg - np.eye(l))) <= 1e-12
    # the three products, each on the GPU's own operands
    assert OL.rel_fro(Btg, OL._product(Qg.T, A64, fmt[1])) <= STAGE_TOL[fmt[1]]
    assert OL.rel_fro(Tg, OL._product(Btg, B64, fmt[2])) <= STAGE_TOL[fmt[2]]
    assert OL.rel_fro(C, OL._product(Qg, Tg, fmt[3])) <= STAGE_TOL[fmt[3]]
    ref = OL.lramm_forward(A64, B64, r, p, q, fmt, omega=om.astype(np.float64))
    err = OL.rel_fro(C, ref["C"])
    print(f"fmt {fmt}: end-to-end rel-F vs oracle {err:.3e}")
    assert err <= max(INDEP_TOL[f] for f in fmt)
    # and the two are equally good approximations of the exact product
    Cex = A64 @ B64
    e_gpu, e_ref = OL.rel_fro(C, Cex), OL.rel_fro(ref["C"], Cex)
    assert abs(e_gpu - e_ref) <= 0.05 * e_ref, (e_gpu, e_ref)


def test_lramm_seeded_omega_and_alpha_beta(lib):
    m = k = n = 384
    A, _ = synth.lowrank(m, k, synth.spectrum("exp", 384, 24.0), 3)
    B = synth.gaussian(k, n, 103)
    Cin = synth.gaussian(m, n, 7)
    C, _, _, _ = _run_forward(lib, A, B, 48, 8, 1, ("int8",) * 4, seed=77, alpha=0.75, beta=0.5, Cin=Cin)
    ref = OL.lramm_forward(A.astype(np.float64), B.astype(np.float64), 48, 8, 1, seed=77, alpha=0.75, beta=0.5,
                           Cin=Cin.astype(np.float64))
    assert OL.rel_fro(C, ref["C"]) <= 1e-5


def test_lramm_bf16_io(lib):
    m = k = n = 512
    A, _ = synth.lowrank(m, k, synth.spectrum("exp", 512, 32.0), 0, dtype="bf16")
    B = synth.gaussian(k, n, 100, dtype="bf16")
    om = synth.omega(k, 74, 1)
    C, _, _, _ = _run_forward(lib, A, B, 64, 10, 1, ("int8",) * 4, omega=om, a_type=torch.bfloat16,
                              c_type=torch.bfloat16)
    ref = OL.lramm_forward(A.astype(np.float64), B.astype(np.float64), 64, 10, 1, omega=om.astype(np.float64))
    assert OL.rel_fro(C, bf16_round(ref["C"])) <= 1e-5


def test_lramm_deterministic(lib):
    m = k = n = 512
    A, _ = synth.lowrank(m, k, synth.spectrum("exp", 512, 32.0), 0)
    B = synth.gaussian(k, n, 100)
    C1, _, _, _ = _run_forward(lib, A, B, 64, 10, 1, ("int8",) * 4, seed=5)
    C2, _, _, _ = _run_forward(lib, A, B, 64, 10, 1, ("int8",) * 4, seed=5)
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
