"""Host-side checks of the C ABI (no GPU): the library loads, exports every
symbol include/lramm.h declares, and host-checkable argument errors return
the documented status codes without launching anything."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lramm.h")
LIB = os.path.join(ROOT, "paper_2405_16917_amd", "liblramm.so")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"LRAMM_API\s+[\w\s\*]*?\b(lramm_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    import paper_2405_16917_amd._lib as L
    return L.load()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 17
    for n in names:
        assert hasattr(lib, n), n
    import paper_2405_16917_amd._lib as L
    assert sorted(L.EXPORTS) == names


def test_status_strings_and_pitch(lib):
    import paper_2405_16917_amd._lib as L
    assert lib.lramm_status_string(0) == b"ok"
    assert lib.lramm_status_string(3).startswith(b"sketch width")
    assert lib.lramm_status_string(L.E_STALL).startswith(b"a Cholesky wait")
    assert L.FLAG_STALL == 0x8
    assert lib.lramm_pitch(272, 0) == 320      # int8: 272 bytes -> 64-byte multiple
    assert lib.lramm_pitch(272, 1) == 192      # int4: 136 bytes -> 192
    assert lib.lramm_pitch(100, 3) == 256      # bf16: 200 bytes -> 128-byte multiple
    assert lib.lramm_pitch(1, 0) == 64


def _desc(L, **kw):
    d = L.Desc()
    d.m, d.n, d.k, d.r, d.p, d.q = 512, 512, 512, 64, 10, 1
    d.fmt_sketch = d.fmt_proj = d.fmt_g1 = d.fmt_g2 = L.INT8
    d.a_type = d.b_type = d.c_type = L.F32
    d.seed, d.alpha, d.beta, d.flags = 0, 1.0, 0.0, 0
    for k, v in kw.items():
        setattr(d, k, v)
    return d


def _create(lib, d):
    h = ctypes.c_void_p()
    code = lib.lramm_plan_create(ctypes.byref(d), ctypes.byref(h))
    return code, h


def test_plan_validation(lib):
    import paper_2405_16917_amd._lib as L
    code, h = _create(lib, _desc(L))
    assert code == L.OK
    sz = ctypes.c_size_t()
    assert lib.lramm_workspace_bytes(h, ctypes.byref(sz)) == L.OK and sz.value > 512 * 512
    lib.lramm_plan_destroy(h)
    assert _create(lib, _desc(L, r=600, p=0))[0] == L.E_RANK          # l > min(m, k)
    assert _create(lib, _desc(L, r=0, p=0))[0] == L.E_RANK            # l < 1
    assert _create(lib, _desc(L, m=0))[0] == L.E_SHAPE
    assert _create(lib, _desc(L, fmt_g2=7))[0] == L.E_UNSUPPORTED
    assert _create(lib, _desc(L, flags=16))[0] == L.E_INVALID
    # the error estimate: only for plans that form the norms
    code, h = _create(lib, _desc(L))
    out = (ctypes.c_double * 3)()
    assert lib.lramm_error_estimate(h, ctypes.c_void_p(256), None, out) == L.E_INVALID
    lib.lramm_plan_destroy(h)
    code, h = _create(lib, _desc(L, flags=L.PLAN_ESTIMATE | L.PLAN_SRHT))
    assert code == L.OK
    lib.lramm_plan_destroy(h)
    # the structured sketch: A' row-major and k' <= 32768 only
    code, h = _create(lib, _desc(L, flags=L.PLAN_SRHT))
    assert code == L.OK
    lib.lramm_plan_destroy(h)
    assert _create(lib, _desc(L, flags=L.PLAN_SRHT, trans_a=1))[0] == L.E_UNSUPPORTED
    # one Cholesky QR pass: any combination with the other flags
    code, h = _create(lib, _desc(L, flags=L.PLAN_ONE_PASS | L.PLAN_SRHT | L.PLAN_ESTIMATE | L.PLAN_EXCLUSIVE))
    assert code == L.OK
    lib.lramm_plan_destroy(h)
    assert _create(lib, _desc(L, k=200000))[0] == L.E_OVERFLOW        # K * 127^2 > 2^31
    assert lib.lramm_plan_create(None, None) == L.E_INVALID


def test_stage_argument_errors(lib):
    import paper_2405_16917_amd._lib as L
    # null device pointers / bad shapes are caught on the host
    assert lib.lramm_quantize(4, 4, None, 4, L.F32, L.INT8, 0, None, 64, None, None, None) == L.E_INVALID
    assert lib.lramm_quantize(4, 4, 1, 3, L.F32, L.INT8, 0, 16, 64, 1, None, None) == L.E_SHAPE
    assert lib.lramm_quantize(4, 4, 1, 4, L.F32, L.INT8, 0, 16, 32, 1, None, None) == L.E_SHAPE
    assert lib.lramm_gemm_nt(4, 4, 64, 9, 16, 64, 1, 16, 64, 1, 1.0, 0.0, 1, 4, 0, None, 0, None, 0,
                             None) == L.E_UNSUPPORTED
    assert lib.lramm_gemm_nt(4, 4, 64, L.INT8, 16, 32, 1, 16, 64, 1, 1.0, 0.0, 1, 4, 0, None, 0, None, 0,
                             None) == L.E_SHAPE
    assert lib.lramm_gemm_nt(4, 4, 200000, L.INT8, 16, 200064, 1, 16, 200064, 1, 1.0, 0.0, 1, 4, 0, None, 0,
                             None, 0, None) == L.E_OVERFLOW
    assert lib.lramm_cholqr2(10, 20, 1, 20, L.F32, 1, 32, 1, 1 << 30, None, None) == L.E_RANK
    assert lib.lramm_cholqr2(100, 20, 1, 20, L.F32, 1, 20, 1, 1 << 30, None, None) == L.E_SHAPE
    assert lib.lramm_cholqr2(100, 20, 1, 20, L.F32, 1, 32, 1, 10, None, None) == L.E_WORKSPACE
    assert lib.lramm_dense_gemm_nt(64, 64, 60, L.BF16, 1, 64, 1, 64, 1, 64, None) == L.E_SHAPE
    assert lib.lramm_omega(0, 10, 3, None, 10, None) == L.E_INVALID


def test_noalloc_cholqr2_host_checks(lib):
    """The no-allocation CholeskyQR2 rejects, on the host, problems whose
    workspace exceeds its fixed scratch (every l <= 768 fits at any row
    count, l = 800 does not at large row counts), and the usual argument
    errors, without touching the GPU."""
    import paper_2405_16917_amd._lib as L
    cap = L.NOALLOC_SCRATCH_BYTES
    for rows in (768, 4096, 65536, 1 << 22):
        assert lib.lramm_cholqr2_workspace_min(rows, 768) <= cap
        assert lib.lramm_cholqr2_workspace_min(rows, 768) <= lib.lramm_cholqr2_workspace(rows, 768)
    assert lib.lramm_cholqr2_workspace_min(1 << 20, 800) > cap
    assert lib.lramm_cholqr2_noalloc(1 << 20, 800, 1, 800, L.F32, 1, 800, None, None) == L.E_SCRATCH
    assert lib.lramm_cholqr2_noalloc(10, 20, 1, 20, L.F32, 1, 32, None, None) == L.E_RANK
    assert lib.lramm_cholqr2_noalloc(100, 20, 1, 20, L.F32, 1, 20, None, None) == L.E_SHAPE
    assert lib.lramm_cholqr2_noalloc(100, 20, None, 20, L.F32, 1, 32, None, None) == L.E_INVALID
    assert lib.lramm_cholqr2_noalloc(0, 20, None, 20, L.F32, None, 32, None, None) == L.OK
    assert lib.lramm_status_string(L.E_SCRATCH).startswith(b"problem needs more scratch")


def test_r_factor_host_checks(lib):
    """lramm_r_factor's argument errors, returned on the host."""
    import paper_2405_16917_amd._lib as L
    assert lib.lramm_r_factor(-1, 4, 1, 4, L.F32, 1, 4, 1, 4, None) == L.E_SHAPE
    assert lib.lramm_r_factor(10, 0, None, 4, L.F32, None, 4, None, 4, None) == L.OK
    assert lib.lramm_r_factor(10, 4, None, 4, L.F32, 1, 4, 1, 4, None) == L.E_INVALID
    assert lib.lramm_r_factor(3, 4, 1, 4, L.F32, 1, 4, 1, 4, None) == L.E_RANK
    assert lib.lramm_r_factor(10, 4, 1, 3, L.F32, 1, 4, 1, 4, None) == L.E_SHAPE
    assert lib.lramm_r_factor(10, 4, 1, 4, L.F32, 1, 4, 1, 3, None) == L.E_SHAPE
    assert lib.lramm_r_factor(10, 4, 1, 4, L.BF16, 1, 4, 1, 4, None) == L.E_UNSUPPORTED


def test_one_launch_cholesky_admission(lib):
    """The one-launch Cholesky's grid (1 + (T-2)(T-1)/2 + T workgroups, T =
    ceil(l/32)) must fit the CUs less 16, or half of that unless the plan is
    exclusive, so that two default calls on different streams are resident
    together."""
    import paper_2405_16917_amd._lib as L
    grid = lambda T: 1 + (T - 2) * (T - 1) // 2 + T
    for l in range(1, 1025, 7):
        T = (l + 31) // 32
        for cus in (80, 256, 304):
            assert lib.lramm_chol_one_launch(l, cus, 0) == int(grid(T) <= (cus - 16) // 2)
            assert lib.lramm_chol_one_launch(l, cus, L.PLAN_EXCLUSIVE) == int(grid(T) <= cus - 16)
    # MI355X (256 CUs): shared up to l' = 480 (107 workgroups), exclusive up to 704 (233)
    assert lib.lramm_chol_one_launch(480, 256, 0) == 1 and lib.lramm_chol_one_launch(481, 256, 0) == 0
    assert lib.lramm_chol_one_launch(704, 256, L.PLAN_EXCLUSIVE) == 1
    assert lib.lramm_chol_one_launch(705, 256, L.PLAN_EXCLUSIVE) == 0
    assert lib.lramm_chol_one_launch(2000, 256, 0) == 0
    # the plan accepts the exclusive flag and nothing else
    assert _create(lib, _desc(L, flags=L.PLAN_EXCLUSIVE))[0] == L.OK
    assert _create(lib, _desc(L, flags=16))[0] == L.E_INVALID
    # the error estimate: only for plans that form the norms
    code, h = _create(lib, _desc(L))
    out = (ctypes.c_double * 3)()
    assert lib.lramm_error_estimate(h, ctypes.c_void_p(256), None, out) == L.E_INVALID
    lib.lramm_plan_destroy(h)
    code, h = _create(lib, _desc(L, flags=L.PLAN_ESTIMATE | L.PLAN_SRHT))
    assert code == L.OK
    lib.lramm_plan_destroy(h)
    # the structured sketch: A' row-major and k' <= 32768 only
    code, h = _create(lib, _desc(L, flags=L.PLAN_SRHT))
    assert code == L.OK
    lib.lramm_plan_destroy(h)
    assert _create(lib, _desc(L, flags=L.PLAN_SRHT, trans_a=1))[0] == L.E_UNSUPPORTED


def test_srht_host_checks(lib):
    """Sizes of the structured test matrix and the errors its entry points
    return before any launch."""
    import paper_2405_16917_amd._lib as L
    assert [lib.lramm_srht_padded(k) for k in (0, 1, 2, 3, 512, 513, 32768)] == [0, 1, 2, 4, 512, 1024, 32768]
    dummy = ctypes.c_void_p(16)
    assert lib.lramm_srht_samples(1, 1, 1, dummy, dummy, dummy, None) == L.E_UNSUPPORTED       # k < 2
    assert lib.lramm_srht_samples(1, 40000, 8, dummy, dummy, dummy, None) == L.E_UNSUPPORTED   # k' > 32768
    assert lib.lramm_srht_samples(1, 100, 0, dummy, dummy, dummy, None) == L.E_RANK
    assert lib.lramm_srht_samples(1, 100, 129, dummy, dummy, dummy, None) == L.E_RANK          # l > k'
    assert lib.lramm_srht_samples(1, 100, 8, None, dummy, dummy, None) == L.E_INVALID
    assert lib.lramm_srht_samples(1, 100, 8, dummy, dummy, None, None) == L.E_INVALID         # no key scratch
    assert lib.lramm_srht_sketch(4, 100, 8, dummy, 99, L.F32, dummy, dummy, dummy, 8, None) == L.E_SHAPE
    assert lib.lramm_srht_sketch(4, 100, 8, dummy, 100, L.F32, dummy, dummy, dummy, 7, None) == L.E_SHAPE
    assert lib.lramm_srht_sketch(4, 100, 8, dummy, 100, L.F64, dummy, dummy, dummy, 8, None) == L.E_UNSUPPORTED
