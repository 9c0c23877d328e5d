"""ctypes binding of ``liblramm.so`` (the C ABI of include/lramm.h).

Argument marshalling only: every function passes device pointers of torch
tensors, sizes and the current HIP stream straight to the library, which runs
every step of the path in its own kernels.  torch is imported first so that
the library binds to the HIP runtime torch already loaded (one runtime per
process).  There is no fallback: a missing library raises.
"""

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime before the library)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblramm.so")

# enums of include/lramm.h
(OK, E_INVALID, E_SHAPE, E_RANK, E_WORKSPACE, E_NONFINITE, E_BREAKDOWN, E_OVERFLOW, E_HIP, E_UNSUPPORTED, E_STALL,
 E_SCRATCH) = range(12)
NOALLOC_SCRATCH_BYTES = 24 << 20
F32, BF16, F64 = 0, 1, 2
INT8, INT4, FP8, BF16F = 0, 1, 2, 3
FLAG_NONFINITE, FLAG_BREAKDOWN, FLAG_SQRTNEG, FLAG_STALL = 0x1, 0x2, 0x4, 0x8
PLAN_EXCLUSIVE = 0x1
PLAN_SRHT = 0x2
PLAN_ESTIMATE = 0x4
PLAN_ONE_PASS = 0x8
ORTHS = {"cholqr2": 0, "cholqr": PLAN_ONE_PASS}
SKETCHES = {"gaussian": 0, "srht": PLAN_SRHT}

FMT = {"int8": INT8, "int4": INT4, "fp8": FP8, "bf16": BF16F}
DTYPE = {torch.float32: F32, torch.bfloat16: BF16, torch.float64: F64}

EXPORTS = (
    "lramm_init", "lramm_status_string", "lramm_plan_create", "lramm_plan_destroy",
    "lramm_workspace_bytes", "lramm_forward", "lramm_factors", "lramm_backward",
    "lramm_status_poll", "lramm_quantize", "lramm_pitch", "lramm_gemm_nt",
    "lramm_gemm_nt_workspace", "lramm_omega", "lramm_cholqr2",
    "lramm_cholqr2_workspace", "lramm_dense_gemm_nt", "lramm_plan_set_timing", "lramm_stage_times",
    "lramm_stage_name", "lramm_intermediate", "lramm_batch_create", "lramm_batch_destroy",
    "lramm_batch_workspace_bytes", "lramm_batched_forward", "lramm_batch_status_poll",
    "lramm_cholqr2_noalloc", "lramm_chol_one_launch", "lramm_codes",
    "lramm_ts_plan_create", "lramm_ts_plan_destroy", "lramm_ts_workspace_bytes", "lramm_ts_forward",
    "lramm_ts_intermediate", "lramm_ts_status_poll", "lramm_srht_padded", "lramm_srht_samples",
    "lramm_srht_sketch", "lramm_error_estimate", "lramm_cholqr2_workspace_min", "lramm_r_factor",
)
NSTAGES = 22


class LrammError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {_status_string(code)} (status {code})")


class TsDesc(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int64),
        ("r", ctypes.c_int32), ("p", ctypes.c_int32), ("q", ctypes.c_int32),
        ("fmt_sketch", ctypes.c_int32), ("fmt_proj", ctypes.c_int32),
        ("fmt_e1", ctypes.c_int32), ("fmt_e2", ctypes.c_int32), ("fmt_e3", ctypes.c_int32),
        ("a_type", ctypes.c_int32), ("b_type", ctypes.c_int32), ("c_type", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("alpha", ctypes.c_float), ("beta", ctypes.c_float),
        ("flags", ctypes.c_uint32), ("reserved", ctypes.c_int32),
    ]


class Desc(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int64),
        ("r", ctypes.c_int32), ("p", ctypes.c_int32), ("q", ctypes.c_int32),
        ("fmt_sketch", ctypes.c_int32), ("fmt_proj", ctypes.c_int32),
        ("fmt_g1", ctypes.c_int32), ("fmt_g2", ctypes.c_int32),
        ("a_type", ctypes.c_int32), ("b_type", ctypes.c_int32), ("c_type", ctypes.c_int32),
        ("reserved0", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("alpha", ctypes.c_float), ("beta", ctypes.c_float),
        ("flags", ctypes.c_uint32), ("reserved1", ctypes.c_uint32),
        ("trans_a", ctypes.c_int32), ("trans_b", ctypes.c_int32), ("side", ctypes.c_int32),
        ("reserved2", ctypes.c_int32),
    ]


_lib = None

P = ctypes.c_void_p
I64 = ctypes.c_int64
I32 = ctypes.c_int32
SZ = ctypes.c_size_t


def load(path=LIB_PATH):
    """Load the library (once) and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    sig = {
        "lramm_init": ([], I32),
        "lramm_status_string": ([I32], ctypes.c_char_p),
        "lramm_plan_create": ([ctypes.POINTER(Desc), ctypes.POINTER(P)], I32),
        "lramm_plan_destroy": ([P], None),
        "lramm_workspace_bytes": ([P, ctypes.POINTER(SZ)], I32),
        "lramm_forward": ([P, P, I64, P, I64, P, I64, P, I64, P, SZ, P], I32),
        "lramm_factors": ([P, P, ctypes.POINTER(P), ctypes.POINTER(I64), ctypes.POINTER(P),
                           ctypes.POINTER(I64)], I32),
        "lramm_intermediate": ([P, P, I32, ctypes.POINTER(P), ctypes.POINTER(I64), ctypes.POINTER(I64),
                                ctypes.POINTER(I64), ctypes.POINTER(I32)], I32),
        "lramm_backward": ([P, P, I64, P, I64, P, I64, P, I64, P, I64, P, SZ, P], I32),
        "lramm_status_poll": ([P, P, P, ctypes.POINTER(ctypes.c_uint32)], I32),
        "lramm_quantize": ([I64, I64, P, I64, I32, I32, I32, P, I64, P, P, P], I32),
        "lramm_r_factor": ([I64, I64, P, I64, I32, P, I64, P, I64, P], I32),
        "lramm_pitch": ([I64, I32], I64),
        "lramm_gemm_nt": ([I64, I64, I64, I32, P, I64, P, P, I64, P, ctypes.c_float, ctypes.c_float,
                           P, I64, I32, P, I64, P, SZ, P], I32),
        "lramm_gemm_nt_workspace": ([I64, I64, I64, I32], SZ),
        "lramm_omega": ([ctypes.c_uint64, I64, I64, P, I64, P], I32),
        "lramm_srht_padded": ([I64], I64),
        "lramm_error_estimate": ([P, P, P, ctypes.POINTER(ctypes.c_double)], I32),
        "lramm_srht_samples": ([ctypes.c_uint64, I64, I64, P, P, P, P], I32),
        "lramm_srht_sketch": ([I64, I64, I64, P, I64, I32, P, P, P, I64, P], I32),
        "lramm_cholqr2": ([I64, I64, P, I64, I32, P, I64, P, SZ, P, P], I32),
        "lramm_cholqr2_workspace": ([I64, I64], SZ),
        "lramm_cholqr2_workspace_min": ([I64, I64], SZ),
        "lramm_cholqr2_noalloc": ([I64, I64, P, I64, I32, P, I64, P, P], I32),
        "lramm_chol_one_launch": ([I64, I32, ctypes.c_uint32], I32),
        "lramm_codes": ([P, P, I32, ctypes.POINTER(P), ctypes.POINTER(I64), ctypes.POINTER(I64),
                         ctypes.POINTER(I64), ctypes.POINTER(P), ctypes.POINTER(I32)], I32),
        "lramm_ts_plan_create": ([ctypes.POINTER(TsDesc), ctypes.POINTER(P)], I32),
        "lramm_ts_plan_destroy": ([P], None),
        "lramm_ts_workspace_bytes": ([P, ctypes.POINTER(SZ)], I32),
        "lramm_ts_forward": ([P, P, I64, P, I64, P, I64, P, I64, P, I64, P, SZ, P], I32),
        "lramm_ts_intermediate": ([P, P, I32, ctypes.POINTER(P), ctypes.POINTER(I64), ctypes.POINTER(I64),
                                   ctypes.POINTER(I64), ctypes.POINTER(I32)], I32),
        "lramm_ts_status_poll": ([P, P, P, ctypes.POINTER(ctypes.c_uint32)], I32),
        "lramm_dense_gemm_nt": ([I64, I64, I64, I32, P, I64, P, I64, P, I64, P], I32),
        "lramm_plan_set_timing": ([P, I32], I32),
        "lramm_stage_times": ([P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I64)], I32),
        "lramm_stage_name": ([I32], ctypes.c_char_p),
        "lramm_batch_create": ([I32, ctypes.POINTER(P), I32, ctypes.c_uint32, ctypes.POINTER(P)], I32),
        "lramm_batch_destroy": ([P], None),
        "lramm_batch_workspace_bytes": ([P, ctypes.POINTER(SZ)], I32),
        "lramm_batched_forward": ([P, ctypes.POINTER(P), ctypes.POINTER(I64), ctypes.POINTER(P),
                                   ctypes.POINTER(I64), ctypes.POINTER(P), ctypes.POINTER(I64), P, SZ, P], I32),
        "lramm_batch_status_poll": ([P, P, P, ctypes.POINTER(ctypes.c_uint32)], I32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _status_string(code):
    if _lib is None:
        return "status"
    return _lib.lramm_status_string(code).decode()


def _check(code, where):
    if code != OK:
        raise LrammError(code, where)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _fmt(f):
    return FMT[f] if isinstance(f, str) else int(f)


# ----------------------------------------------------------------- stages --

def lramm_init():
    _check(load().lramm_init(), "lramm_init")


def lramm_pitch(K, fmt):
    return int(load().lramm_pitch(K, _fmt(fmt)))


def lramm_quantize(X, fmt, transpose=False, Xq=None, scales=None, flags=None):
    """Quantise the rows (transpose=False) or the columns (transpose=True,
    written transposed) of the 2-D tensor X.  Returns (Xq, scales)."""
    lib = load()
    rows, cols = X.shape
    K = rows if transpose else cols
    nvec = cols if transpose else rows
    pitch = lramm_pitch(K, fmt)
    if Xq is None:
        Xq = torch.empty((nvec, pitch), dtype=torch.uint8, device=X.device)
    if scales is None:
        scales = torch.empty(nvec, dtype=torch.float32, device=X.device)
    _check(lib.lramm_quantize(rows, cols, _ptr(X), X.stride(0), DTYPE[X.dtype], _fmt(fmt),
                              1 if transpose else 0, _ptr(Xq), Xq.stride(0), _ptr(scales),
                              _ptr(flags), _stream()), "lramm_quantize")
    return Xq, scales


def lramm_gemm_nt(M, N, K, fmt, Lq, dL, Rq, dR, alpha=1.0, beta=0.0, C=None, ctype=torch.float32,
                  acc_out=None, ws=None):
    """Quantised NT-GEMM: C = epi(Lq[:M] . Rq[:N]^T) on quantised rows."""
    lib = load()
    if C is None:
        C = torch.empty((M, N), dtype=ctype, device=Lq.device)
    wsz = 0 if ws is None else ws.numel() * ws.element_size()
    _check(lib.lramm_gemm_nt(M, N, K, _fmt(fmt), _ptr(Lq), Lq.stride(0), _ptr(dL), _ptr(Rq), Rq.stride(0),
                             _ptr(dR), alpha, beta, _ptr(C), C.stride(0), DTYPE[C.dtype], _ptr(acc_out),
                             0 if acc_out is None else acc_out.stride(0), _ptr(ws), wsz, _stream()),
           "lramm_gemm_nt")
    return C


def lramm_gemm_nt_workspace(M, N, K, fmt):
    return int(load().lramm_gemm_nt_workspace(M, N, K, _fmt(fmt)))


def lramm_omega(seed, k, l, device="cuda"):
    """Omega^T (l x k, FP32) of the seeded Gaussian test matrix."""
    out = torch.empty((l, k), dtype=torch.float32, device=device)
    _check(load().lramm_omega(seed, k, l, _ptr(out), out.stride(0), _stream()), "lramm_omega")
    return out


def lramm_srht_padded(k):
    return int(load().lramm_srht_padded(k))


def lramm_srht_samples(seed, k, l, device="cuda"):
    """(S [l int32], sign_bits [ceil(k'/32) int32 views of the uint32 words])
    of the structured test matrix."""
    kp = lramm_srht_padded(k)
    S = torch.empty(l, dtype=torch.int32, device=device)
    bits = torch.empty((kp + 31) // 32, dtype=torch.int32, device=device)
    keys = torch.empty(kp, dtype=torch.int32, device=device)
    _check(load().lramm_srht_samples(seed, k, l, _ptr(S), _ptr(bits), _ptr(keys), _stream()), "lramm_srht_samples")
    return S, bits


def lramm_srht_sketch(A, l, S, sign_bits, Y=None):
    """Y = A Omega (m x l FP32) with the structured test matrix given by
    (S, sign_bits) as lramm_srht_samples writes them."""
    m, k = A.shape
    if Y is None:
        Y = torch.empty((m, l), dtype=torch.float32, device=A.device)
    _check(load().lramm_srht_sketch(m, k, l, _ptr(A), A.stride(0), DTYPE[A.dtype], _ptr(S), _ptr(sign_bits),
                                    _ptr(Y), Y.stride(0), _stream()), "lramm_srht_sketch")
    return Y


def lramm_cholqr2_workspace(rows, l):
    return int(load().lramm_cholqr2_workspace(rows, l))


def lramm_cholqr2(Y, l=None, Q=None, ws=None, flags=None):
    """CholeskyQR2 of the first l columns of Y (FP32 or FP64) -> Q (FP64,
    leading dimension round_up(l, 32), padding columns zero)."""
    lib = load()
    rows = Y.shape[0]
    l = Y.shape[1] if l is None else l
    lw = (l + 31) // 32 * 32
    if Q is None:
        Q = torch.empty((rows, lw), dtype=torch.float64, device=Y.device)
    need = lramm_cholqr2_workspace(rows, l)
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=Y.device)
    _check(lib.lramm_cholqr2(rows, l, _ptr(Y), Y.stride(0), DTYPE[Y.dtype], _ptr(Q), Q.stride(0), _ptr(ws),
                             ws.numel(), _ptr(flags), _stream()), "lramm_cholqr2")
    return Q


def lramm_r_factor(Y, Q, l=None, R=None):
    """R = Q^T Y on and above the diagonal (zero below), l x l FP64: the
    triangular factor of Y = Q R for Q from lramm_cholqr2."""
    l = Y.shape[1] if l is None else l
    if R is None:
        R = torch.empty((l, l), dtype=torch.float64, device=Y.device)
    _check(load().lramm_r_factor(Y.shape[0], l, _ptr(Y), Y.stride(0), DTYPE[Y.dtype], _ptr(Q), Q.stride(0), _ptr(R),
                                 R.stride(0), _stream()), "lramm_r_factor")
    return R


def lramm_cholqr2_noalloc(Y, l=None, Q=None, flags=None):
    """lramm_cholqr2 on the library's fixed scratch (no workspace argument;
    the library allocates nothing).  Q must be given by callers that cannot
    allocate; it is created here only for convenience."""
    lib = load()
    rows = Y.shape[0]
    l = Y.shape[1] if l is None else l
    if Q is None:
        Q = torch.empty((rows, (l + 31) // 32 * 32), dtype=torch.float64, device=Y.device)
    _check(lib.lramm_cholqr2_noalloc(rows, l, _ptr(Y), Y.stride(0), DTYPE[Y.dtype], _ptr(Q), Q.stride(0),
                                     _ptr(flags), _stream()), "lramm_cholqr2_noalloc")
    return Q


def lramm_dense_gemm_nt(L, R, C=None):
    """Dense comparator: C = L . R^T (bf16 or fp32 operands, FP32 out)."""
    lib = load()
    M, K = L.shape
    N = R.shape[0]
    if C is None:
        C = torch.empty((M, N), dtype=torch.float32, device=L.device)
    dt = BF16 if L.dtype == torch.bfloat16 else F32
    _check(lib.lramm_dense_gemm_nt(M, N, K, dt, _ptr(L), L.stride(0), _ptr(R), R.stride(0), _ptr(C),
                                   C.stride(0), _stream()), "lramm_dense_gemm_nt")
    return C


# ------------------------------------------------------------------- plan --

def storage(X):
    """(tensor whose rows are stored contiguously, transposed flag) for a 2-D
    tensor or a transposed view of one: X itself when its rows are
    contiguous, else X.t() when that is (the ABI's transposed storage), else
    a contiguous copy."""
    if X.stride(1) == 1 and X.stride(0) >= X.shape[1]:
        return X, 0
    if X.stride(0) == 1 and X.stride(1) >= X.shape[0]:
        return X.t(), 1
    return X.contiguous(), 0


SIDES = {"left": 0, "right": 1, 0: 0, 1: 1}


class LrammPlan:
    """lramm_plan_create / lramm_forward / lramm_backward / lramm_factors /
    lramm_status_poll on one problem description.  A and B are passed as
    their storage: A row-major m x k (or k x m with trans_a), B k x n (or
    n x k with trans_b); ``side`` "right" sketches B instead of A;
    ``orth`` "cholqr" orthonormalises with one Cholesky QR pass instead of
    CholeskyQR2 (LRAMM_PLAN_ONE_PASS)."""

    def __init__(self, m, n, k, r, p=16, q=1, fmt=("int8",) * 4, a_type=torch.float32,
                 b_type=torch.float32, c_type=torch.float32, seed=0, alpha=1.0, beta=0.0, exclusive=False,
                 trans_a=False, trans_b=False, side="left", sketch="gaussian", estimate=False, orth="cholqr2"):
        lib = load()
        d = Desc()
        d.m, d.n, d.k, d.r, d.p, d.q = m, n, k, r, p, q
        d.fmt_sketch, d.fmt_proj, d.fmt_g1, d.fmt_g2 = (_fmt(f) for f in fmt)
        d.a_type, d.b_type, d.c_type = DTYPE[a_type], DTYPE[b_type], DTYPE[c_type]
        d.seed, d.alpha, d.beta = seed, alpha, beta
        d.flags = ((PLAN_EXCLUSIVE if exclusive else 0) | SKETCHES[sketch] | (PLAN_ESTIMATE if estimate else 0)
                   | ORTHS[orth])
        d.trans_a, d.trans_b, d.side = int(bool(trans_a)), int(bool(trans_b)), SIDES[side]
        self.desc = d
        self.c_type = c_type
        h = P()
        _check(lib.lramm_plan_create(ctypes.byref(d), ctypes.byref(h)), "lramm_plan_create")
        self._h = h
        sz = SZ()
        _check(lib.lramm_workspace_bytes(h, ctypes.byref(sz)), "lramm_workspace_bytes")
        self.ws_bytes = int(sz.value)
        self.l = r + p
        self.a_type, self.b_type = a_type, b_type

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.lramm_plan_destroy(self._h)
            self._h = None

    def workspace(self, device="cuda"):
        return torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)

    def _fdims(self):
        """(rows, cols) of the factor Q and of Bt: Q spans the sketched
        operand (m rows, or n with side 1)."""
        d = self.desc
        return (d.n, d.m) if d.side else (d.m, d.n)

    def forward(self, A, B, ws, C=None, omega=None):
        d = self.desc
        if C is None:
            C = torch.empty((d.m, d.n), dtype=self.c_type, device=A.device)
        _check(load().lramm_forward(self._h, _ptr(A), A.stride(0), _ptr(B), B.stride(0), _ptr(C), C.stride(0),
                                    _ptr(omega), 0 if omega is None else omega.stride(0), _ptr(ws),
                                    ws.numel(), _stream()), "lramm_forward")
        return C

    def error_estimate(self, ws):
        """(rel. Frobenius error estimate of the rank-l range, ||A'||_F^2,
        ||Bt||_F^2) after a forward of a plan made with estimate=True."""
        out = (ctypes.c_double * 3)()
        _check(load().lramm_error_estimate(self._h, _ptr(ws), _stream(), out), "lramm_error_estimate")
        return float(out[0]), float(out[1]), float(out[2])

    def factors(self, ws):
        """Views of (Q [m x l FP64], Bt [l x k FP32]) inside ws."""
        q, ldq, bt, ldbt = P(), I64(), P(), I64()
        _check(load().lramm_factors(self._h, _ptr(ws), ctypes.byref(q), ctypes.byref(ldq), ctypes.byref(bt),
                                    ctypes.byref(ldbt)), "lramm_factors")
        d = self.desc
        rows = self._fdims()[0]
        base = ws.data_ptr()
        qo, bo = q.value - base, bt.value - base
        Q = ws[qo:qo + rows * ldq.value * 8].view(torch.float64).view(rows, ldq.value)[:, :self.l]
        Bt = ws[bo:bo + self.l * ldbt.value * 4].view(torch.float32).view(self.l, ldbt.value)
        return Q, Bt

    VIEWS = {"Y": 0, "Q": 1, "Bt": 2, "Tt": 3, "T": 4}

    def intermediate(self, ws, name):
        """View of one FP intermediate ("Y", "Q", "Bt" or "Tt") inside ws.
        "Tt" is returned as a transposed view of T when the forward kept T."""
        ptr, rows, cols, ld, dt = P(), I64(), I64(), I64(), I32()
        code = load().lramm_intermediate(self._h, _ptr(ws), self.VIEWS[name], ctypes.byref(ptr), ctypes.byref(rows),
                                         ctypes.byref(cols), ctypes.byref(ld), ctypes.byref(dt))
        if code == E_INVALID and name == "Tt":
            return self.intermediate(ws, "T").t()
        _check(code, "lramm_intermediate")
        esz, tdt = (8, torch.float64) if dt.value == F64 else (4, torch.float32)
        off = ptr.value - ws.data_ptr()
        return ws[off:off + rows.value * ld.value * esz].view(tdt).view(rows.value, ld.value)[:, :cols.value]

    CODES = {"A_rows": 0, "sketch_R": 1, "Q_cols": 2, "A_cols": 3, "Bt_rows": 4, "B_cols": 5, "Q_rows": 6,
             "Tt_rows": 7}

    def codes(self, ws, name, A=None):
        """(codes uint8 [rows x pitch], scales float32 [rows], K, fmt name) of
        one quantised operand of the last forward (views into ws; "A_rows"
        on the direct bf16 path views A, which must then be passed)."""
        ptr, rows, K, pitch, sc, f = P(), I64(), I64(), I64(), P(), I32()
        _check(load().lramm_codes(self._h, _ptr(ws), self.CODES[name], ctypes.byref(ptr), ctypes.byref(rows),
                                  ctypes.byref(K), ctypes.byref(pitch), ctypes.byref(sc), ctypes.byref(f)),
               "lramm_codes")
        fname = {v: k for k, v in FMT.items()}[f.value]
        base = ws.data_ptr()
        nbytes = rows.value * pitch.value
        if base <= ptr.value < base + ws.numel():
            off = ptr.value - base
            codes = ws[off:off + nbytes].view(rows.value, pitch.value)
        else:
            if A is None or A.data_ptr() != ptr.value:
                raise ValueError("these codes are the input A itself: pass A")
            codes = A.view(torch.uint8).view(rows.value, -1)[:, :pitch.value]
        so = sc.value - base
        scales = ws[so:so + 4 * rows.value].view(torch.float32)
        return codes, scales, K.value, fname

    def backward(self, dC, A, B, ws, dA=None, dB=None, need_dA=True, need_dB=True):
        """Gradients of the frozen-Q surrogate; A, B, dA, dB are storage
        tensors (shapes and types as A and B are stored)."""
        if need_dA and dA is None:
            dA = torch.empty(A.shape, dtype=A.dtype, device=dC.device)
        if need_dB and dB is None:
            dB = torch.empty(B.shape, dtype=B.dtype, device=dC.device)
        _check(load().lramm_backward(self._h, _ptr(dC), dC.stride(0), _ptr(A), A.stride(0), _ptr(B),
                                     B.stride(0), _ptr(dA) if need_dA else None, dA.stride(0) if need_dA else 0,
                                     _ptr(dB) if need_dB else None, dB.stride(0) if need_dB else 0, _ptr(ws),
                                     ws.numel(), _stream()), "lramm_backward")
        return dA, dB

    def set_timing(self, enable=True):
        _check(load().lramm_plan_set_timing(self._h, 1 if enable else 0), "lramm_plan_set_timing")

    def stage_times(self):
        """{stage name: (total ms, launches)} recorded since the last call
        (synchronises the recorded events)."""
        lib = load()
        ms = (ctypes.c_double * NSTAGES)()
        cnt = (I64 * NSTAGES)()
        _check(lib.lramm_stage_times(self._h, ms, cnt), "lramm_stage_times")
        return {lib.lramm_stage_name(i).decode(): (ms[i], int(cnt[i])) for i in range(NSTAGES)}

    def status(self, ws):
        """Synchronise and return the device status flags (raises LrammError
        on a non-finite input or a Cholesky wait past its bound)."""
        f = ctypes.c_uint32()
        code = load().lramm_status_poll(self._h, _ptr(ws), _stream(), ctypes.byref(f))
        _check(code, "lramm_status_poll")
        return int(f.value)


class LrammTsPlan:
    """Two-sided LRAMM (the paper's Alg. 3): lramm_ts_plan_create /
    lramm_ts_forward / lramm_ts_intermediate / lramm_ts_status_poll.
    ``rsvd_fmt`` = formats of both RSVDs' sketch and projection, ``d`` =
    the budgets (d1, d2, d3) of E1, E2, E3."""

    VIEWS = {"Ut": 0, "Vt": 1, "W": 2, "Zs": 3, "E1": 4, "E2": 5, "SA": 6, "SB": 7, "UpA": 8, "UpB": 9}

    def __init__(self, m, n, k, r, p=8, q=1, rsvd_fmt=("int8", "int8"), d=("int8",) * 3, a_type=torch.float32,
                 b_type=torch.float32, c_type=torch.float32, seed=0, alpha=1.0, beta=0.0):
        lib = load()
        t = TsDesc()
        t.m, t.n, t.k, t.r, t.p, t.q = m, n, k, r, p, q
        t.fmt_sketch, t.fmt_proj = (_fmt(f) for f in rsvd_fmt)
        t.fmt_e1, t.fmt_e2, t.fmt_e3 = (_fmt(f) for f in d)
        t.a_type, t.b_type, t.c_type = DTYPE[a_type], DTYPE[b_type], DTYPE[c_type]
        t.seed, t.alpha, t.beta, t.flags = seed, alpha, beta, 0
        self.desc, self.c_type = t, c_type
        h = P()
        _check(lib.lramm_ts_plan_create(ctypes.byref(t), ctypes.byref(h)), "lramm_ts_plan_create")
        self._h = h
        sz = SZ()
        _check(lib.lramm_ts_workspace_bytes(h, ctypes.byref(sz)), "lramm_ts_workspace_bytes")
        self.ws_bytes = int(sz.value)

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.lramm_ts_plan_destroy(self._h)
            self._h = None

    def workspace(self, device="cuda"):
        return torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)

    def forward(self, A, B, ws, C=None, omega_a=None, omega_b=None):
        t = self.desc
        if C is None:
            C = torch.empty((t.m, t.n), dtype=self.c_type, device=A.device)
        _check(load().lramm_ts_forward(self._h, _ptr(A), A.stride(0), _ptr(B), B.stride(0), _ptr(C), C.stride(0),
                                       _ptr(omega_a), 0 if omega_a is None else omega_a.stride(0), _ptr(omega_b),
                                       0 if omega_b is None else omega_b.stride(0), _ptr(ws), ws.numel(), _stream()),
               "lramm_ts_forward")
        return C

    def intermediate(self, ws, name):
        ptr, rows, cols, ld, dt = P(), I64(), I64(), I64(), I32()
        _check(load().lramm_ts_intermediate(self._h, _ptr(ws), self.VIEWS[name], ctypes.byref(ptr),
                                            ctypes.byref(rows), ctypes.byref(cols), ctypes.byref(ld),
                                            ctypes.byref(dt)), "lramm_ts_intermediate")
        esz, tdt = (8, torch.float64) if dt.value == F64 else (4, torch.float32)
        off = ptr.value - ws.data_ptr()
        return ws[off:off + rows.value * ld.value * esz].view(tdt).view(rows.value, ld.value)[:, :cols.value]

    def status(self, ws):
        f = ctypes.c_uint32()
        _check(load().lramm_ts_status_poll(self._h, _ptr(ws), _stream(), ctypes.byref(f)), "lramm_ts_status_poll")
        return int(f.value)


BATCH_GRAPH = 0x1


def autotune_rank(m, k):
    """The paper's rank rule (Sec. 3.5): about a tenth of the smaller dimension
    of the sketched operand, r = ceil(min(m, k) / 10)."""
    return max(1, -(-min(m, k) // 10))


class LrammBatch:
    """lramm_batch_create / lramm_batched_forward over a list of LrammPlan."""

    def __init__(self, plans, nstreams=4, graph=False):
        lib = load()
        self.plans = list(plans)
        arr = (P * len(self.plans))(*[pl._h for pl in self.plans])
        h = P()
        _check(lib.lramm_batch_create(len(self.plans), arr, nstreams, BATCH_GRAPH if graph else 0, ctypes.byref(h)),
               "lramm_batch_create")
        self._h = h
        sz = SZ()
        _check(lib.lramm_batch_workspace_bytes(h, ctypes.byref(sz)), "lramm_batch_workspace_bytes")
        self.ws_bytes = int(sz.value)

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.lramm_batch_destroy(self._h)
            self._h = None

    def workspace(self, device="cuda"):
        return torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)

    def forward(self, As, Bs, Cs, ws):
        n = len(self.plans)
        assert len(As) == len(Bs) == len(Cs) == n
        ptrs = lambda ts: (P * n)(*[t.data_ptr() for t in ts])
        lds = lambda ts: (I64 * n)(*[t.stride(0) for t in ts])
        _check(load().lramm_batched_forward(self._h, ptrs(As), lds(As), ptrs(Bs), lds(Bs), ptrs(Cs), lds(Cs),
                                            _ptr(ws), ws.numel(), _stream()), "lramm_batched_forward")
        return Cs

    def status(self, ws):
        f = ctypes.c_uint32(0)
        code = load().lramm_batch_status_poll(self._h, _ptr(ws), _stream(), ctypes.byref(f))
        if code not in (OK, E_NONFINITE):
            _check(code, "lramm_batch_status_poll")
        return int(f.value)
