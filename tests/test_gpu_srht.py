"""GPU parity of the structured sketch (subsampled randomised Hadamard
transform; Halko et al. 2011 Sec. 4.6, the paper's O(mn log r) RSVD cost in
Sec. 2.2) through the C ABI: the sample set and the signs bit for bit
against the oracle's Philox, the sketch bit for bit against the oracle's
binary32 transform (same butterfly order), and the forward with the
structured sketch against the oracle stage by stage and end to end."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import lramm as OL  # noqa: E402
from oracle import srht as OS  # noqa: E402

from test_gpu_parity import _run_forward, check_stages  # noqa: E402

DEV = "cuda"


def _bits_to_signs(bits, kp):
    w = bits.cpu().numpy().astype(np.uint32)
    b = (w[:, None] >> np.arange(32, dtype=np.uint32)[None, :]) & 1
    return np.where(b.reshape(-1)[:kp] == 1, -1.0, 1.0)


@pytest.mark.parametrize("skl", [(1, 2, 1), (3, 3, 2), (7, 300, 37), (11, 4096, 272), (5, 5000, 448),
                                 (9, 8192, 448), (13, 32768, 1000), (2, 600, 1024), (4, 64, 64)])
def test_samples_and_signs_bit_exact(lib, skl):
    seed, k, l = skl
    print(f"srht samples seed {seed} k {k} l {l}", flush=True)
    S, bits = lib.lramm_srht_samples(seed, k, l)
    torch.cuda.synchronize()
    assert np.array_equal(S.cpu().numpy(), OS.srht_samples(seed, k, l))
    kp = OS.next_pow2(k)
    assert np.array_equal(_bits_to_signs(bits, kp), OS.srht_signs(seed, k))


@pytest.mark.parametrize("mkl", [(5, 2, 1), (3, 3, 2), (37, 100, 16), (64, 300, 37), (16, 512, 64),
                                 (9, 1000, 200), (33, 2048, 100), (40, 4096, 272), (20, 5000, 448),
                                 (24, 8192, 448), (8, 16384, 500), (4, 32768, 1000),
                                 # many samples: the last transform round runs over every element
                                 (12, 1000, 1000), (6, 8192, 4096), (7, 2, 2)])
@pytest.mark.parametrize("dtype", ["fp32", "bf16"])
def test_sketch_bit_exact(lib, mkl, dtype):
    """Few samples (l * (2^w - 1) < k' * w for the last round's w bits) take the
    output loop's restricted last round, many take the full round; both are
    the oracle's butterflies to the bit."""
    m, k, l = mkl
    print(f"srht sketch {m}x{k} l {l} {dtype}", flush=True)
    rng = np.random.default_rng(m + k)
    A = synth.to_dtype(rng.standard_normal((m, k)) * 3.0, dtype)
    Ad = torch.from_numpy(A).to(DEV).to(torch.bfloat16 if dtype == "bf16" else torch.float32)
    S, bits = lib.lramm_srht_samples(17, k, l)
    Y = lib.lramm_srht_sketch(Ad, l, S, bits)
    ref = OS.srht_sketch(A.astype(np.float64), 17, l, "fp32")
    got = Y.double().cpu().numpy()
    assert np.array_equal(got, ref), f"{np.sum(got != ref)} entries differ"


def test_sketch_padded_leading_dimensions(lib):
    """A and Y with leading dimensions past their widths (unaligned rows)."""
    m, k, l = 13, 1000, 50
    rng = np.random.default_rng(1)
    A = rng.standard_normal((m, k + 3)).astype(np.float32)
    Ad = torch.from_numpy(A).to(DEV)[:, :k]
    S, bits = lib.lramm_srht_samples(4, k, l)
    Y = torch.full((m, l + 5), 7.0, device=DEV)
    lib.lramm_srht_sketch(Ad, l, S, bits, Y=Y[:, :l])
    got = Y.double().cpu().numpy()
    assert np.array_equal(got[:, :l], OS.srht_sketch(A[:, :k].astype(np.float64), 4, l, "fp32"))
    assert np.all(got[:, l:] == 7.0)


@pytest.mark.parametrize("case", [(20000, 300, 37, "fp32", 0), (5000, 4096, 272, "bf16", 0),
                                  (3000, 1000, 50, "fp32", 3), (2500, 2048, 2048, "bf16", 0)])
def test_sketch_many_rows(lib, case):
    """Many rows (one workgroup each), aligned and unaligned, with the
    pruned and the full last round."""
    m, k, l, dtype, pad = case
    print(f"srht sketch {m}x{k} l {l} {dtype} ld pad {pad}", flush=True)
    rng = np.random.default_rng(m + l)
    A = synth.to_dtype(rng.standard_normal((m, k + pad)), dtype)
    Ad = torch.from_numpy(A).to(DEV).to(torch.bfloat16 if dtype == "bf16" else torch.float32)[:, :k]
    S, bits = lib.lramm_srht_samples(6, k, l)
    Y = lib.lramm_srht_sketch(Ad, l, S, bits).double().cpu().numpy()
    ref = OS.srht_sketch(A[:, :k].astype(np.float64), 6, l, "fp32")
    assert np.array_equal(Y, ref), f"{np.sum(Y != ref)} entries differ"


def test_target_shape_sketch_bit_exact(lib):
    """8192 x 8192 bf16 rows at l = 448 (the headline sketch) in full."""
    m = k = 8192
    l = 448
    rng = np.random.default_rng(3)
    A = synth.to_dtype(rng.standard_normal((m, k)), "bf16")
    Ad = torch.from_numpy(A).to(DEV).to(torch.bfloat16)
    S, bits = lib.lramm_srht_samples(1, k, l)
    Y = lib.lramm_srht_sketch(Ad, l, S, bits).double().cpu().numpy()
    del Ad
    ref = OS.srht_sketch(A, 1, l, "fp32")
    assert np.array_equal(Y, ref)


SRHT_CASES = [
    # m, k, n, r, p, q, tau, fmt, a dtype
    (512, 512, 512, 64, 10, 0, 32.0, ("int8",) * 4, "fp32"),
    (512, 512, 512, 64, 10, 1, 32.0, ("int8",) * 4, "fp32"),
    (300, 257, 190, 20, 5, 0, 12.0, ("int8",) * 4, "fp32"),          # ragged, k' = 512
    (640, 384, 512, 100, 12, 0, 40.0, ("int8", "int8", "int4", "int4"), "fp32"),
    (1024, 2048, 512, 112, 16, 0, 64.0, ("bf16",) * 4, "bf16"),
    (2048, 4096, 512, 240, 16, 0, 64.0, ("bf16",) * 4, "bf16"),
    # the projection and G1 read A and B in place over K = 4096 and 6144 in
    # two K slices (144 tiles each)
    (4096, 6144, 6144, 368, 16, 0, 64.0, ("bf16",) * 4, "bf16"),
]


@pytest.mark.parametrize("case", SRHT_CASES)
def test_forward_with_structured_sketch(lib, case):
    m, k, n, r, p, q, tau, fmt, dt = case
    print(f"srht forward {m}x{k}x{n} r={r} p={p} q={q} {fmt} {dt}", flush=True)
    A, _ = synth.lowrank(m, k, synth.spectrum("exp", min(m, k), tau), 0, dtype=dt)
    B = synth.gaussian(k, n, 100, dtype=dt)
    a_type = torch.bfloat16 if dt == "bf16" else torch.float32
    C, plan, ws, flags, Ad = _run_forward(lib, A, B, r, p, q, fmt, seed=21, a_type=a_type, sketch="srht")
    assert flags == 0
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    check_stages(lib, plan, ws, A64, B64, C, fmt, q, Ad=Ad, srht_seed=21)
    ref = OL.lramm_forward(A64, B64, r, p, q, fmt, seed=21, sketch="srht")
    if q == 0:
        Qg, Btg = plan.factors(ws)
        assert np.max(np.abs(Qg.cpu().numpy() - ref["Q"])) <= 1e-11
    err = OL.rel_fro(C, ref["C"])
    if all(f in ("int8", "int4") for f in fmt):
        assert err <= 1e-5, err
    else:
        # FP32-accumulated products: the stages above are the parity check;
        # end to end both sides must be equally good approximations
        Cex = A64 @ B64
        e_gpu, e_ref = OL.rel_fro(C, Cex), OL.rel_fro(ref["C"], Cex)
        print(f"srht {fmt}: end-to-end rel-F vs oracle {err:.3e}; vs exact gpu {e_gpu:.3e} oracle {e_ref:.3e}")
        assert e_gpu <= 2.0 * e_ref and e_ref <= 2.0 * e_gpu, (e_gpu, e_ref)
