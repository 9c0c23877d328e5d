/*
 * lramm.h -- C ABI of the MI355X (gfx950) LRAMM hot path.
 *
 * LRAMM (arxiv 2405.16917) approximates C = A B by a randomised range finder
 * on A followed by low-precision quantised GEMMs on the low-rank factors
 * (paper Sec. 2.2, Alg. 1; Sec. 3.1, Alg. 2; Sec. 3.2, Alg. 3).  This library
 * computes the one-sided form
 *
 *     Y = A Omega            Gaussian sketch, Omega is k x l, l = r + p
 *     Q = orth(Y)            CholeskyQR2 with FP64 Gram/Cholesky/solve
 *     (q power iterations:  Z = A^T Q, Q_Z = orth(Z), Y = A Q_Z, Q = orth(Y))
 *     Bt = Q^T A             projection (Alg. 1, first line)
 *     T  = Bt B              first quantised product
 *     C  = alpha * Q T + beta * C        second quantised product
 *
 * where every product is Alg. 2: the left operand is quantised per row, the
 * right operand per column, the integer (or low-precision) product is
 * accumulated exactly in int32 (FP32 for fp8/bf16), and the result is
 * dequantised by the row factor, then the column factor, each product
 * rounded to binary32: c = fl32(fl32(fl32(acc) * d_row) * d_col).  (T is
 * formed transposed; its epilogue still applies T's row factor first.)
 *
 * Quantiser (paper Sec. 3.1, eqs. Quantization / get_lambda /
 * Dequantization), per vector v of binary32 values, qmax = 2^(N-1) - 1:
 *     amax = max |v_i|;  lambda = fl32(qmax / amax);
 *     code_i = clamp(rne(fl32(v_i * lambda)), -qmax, qmax);
 *     d = fl32(amax / qmax);  amax == 0 or lambda == inf  ->  codes 0, d = 0.
 * fp8 e4m3 uses qmax = 448 with saturating round-to-nearest-even; bf16 is a
 * plain round-to-nearest-even cast with d = 1.
 *
 * Conventions for every entry point
 *   - Matrices are row-major with a leading dimension in ELEMENTS, except
 *     quantised buffers whose leading dimension ("pitch") is in BYTES.
 *   - All matrix / vector pointers are DEVICE pointers owned by the caller.
 *     The library never allocates device memory after lramm_init(); scratch
 *     space comes from a caller-owned workspace whose size a query returns.
 *   - "stream" is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls are asynchronous on that stream.  Host-checkable argument errors
 *     return immediately without launching anything; conditions found on the
 *     GPU (non-finite input, Cholesky breakdown) set bits in a device status
 *     word that lramm_status_poll() reads.
 *   - No exception or abort crosses this ABI.  A plan is not re-entrant on
 *     concurrent streams.  Identical inputs, seed and plan give bit-identical
 *     results.
 *   - The Cholesky inside CholeskyQR2 (lramm_forward, lramm_cholqr2) runs
 *     as one launch whose workgroups wait on one another, and needs all of
 *     them on the GPU at once.  By default that launch is used only when its
 *     grid fits half of the compute units (less a margin), so two such calls
 *     overlapping on different streams are resident together; a plan with
 *     LRAMM_PLAN_EXCLUSIVE may use all of them.  More overlapping calls (or
 *     exclusive plans overlapping others) can keep each other's workgroups
 *     waiting: the waits are bounded, and an overrun sets LRAMM_FLAG_STALL
 *     (that result is not valid).  lramm_batched_forward on more than one
 *     stream uses launches whose workgroups never wait instead.
 */
#ifndef LRAMM_H
#define LRAMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define LRAMM_API __attribute__((visibility("default")))
#else
#define LRAMM_API
#endif

typedef enum {
  LRAMM_OK = 0,
  LRAMM_E_INVALID = 1,     /* null pointer, bad enum, bad flag            */
  LRAMM_E_SHAPE = 2,       /* sizes / leading dimensions inconsistent     */
  LRAMM_E_RANK = 3,        /* l = r + p outside [1, min(m, k)]            */
  LRAMM_E_WORKSPACE = 4,   /* workspace missing or too small              */
  LRAMM_E_NONFINITE = 5,   /* a quantiser met NaN / Inf (device flag)     */
  LRAMM_E_BREAKDOWN = 6,   /* Cholesky pivot dropped (device flag, non-fatal) */
  LRAMM_E_OVERFLOW = 7,    /* K too large for the int32 accumulator       */
  LRAMM_E_HIP = 8,         /* a HIP runtime call failed                   */
  LRAMM_E_UNSUPPORTED = 9, /* format / type combination not implemented   */
  LRAMM_E_STALL = 10,      /* a Cholesky wait ran past its bound (device
                              flag): the result is not valid             */
  LRAMM_E_SCRATCH = 11     /* problem larger than the fixed scratch of the
                              no-allocation entry point                  */
} lramm_status;

/* element types of A, B, C and of stage inputs */
typedef enum { LRAMM_F32 = 0, LRAMM_BF16 = 1, LRAMM_F64 = 2 } lramm_dtype;

/* operand format of one product stage (the paper's bit budgets d1..d3) */
typedef enum {
  LRAMM_INT8 = 0,    /* 8-bit symmetric, int32 accumulation                  */
  LRAMM_INT4 = 1,    /* 4-bit symmetric, stored two per byte                 */
  LRAMM_FP8 = 2,     /* OCP e4m3 scaled to 448, FP32 accumulation            */
  LRAMM_BF16F = 3    /* bfloat16 cast, FP32 accumulation                     */
} lramm_fmt;

/* device status word bits (lramm_status_poll) */
#define LRAMM_FLAG_NONFINITE 0x1u  /* a quantiser input held NaN or Inf       */
#define LRAMM_FLAG_BREAKDOWN 0x2u  /* CholeskyQR dropped a dependent column    */
#define LRAMM_FLAG_SQRTNEG   0x4u  /* a Cholesky pivot was negative / NaN      */
#define LRAMM_FLAG_STALL     0x8u  /* a wait inside the one-launch Cholesky ran
                                      past its bound: that factor is not valid */

/*
 * Problem description (paper Alg. 3 inputs A, B, C, r and the bit budgets;
 * Alg. 2's alpha, beta; plus oversampling p, power iterations q and seed).
 * A is m x k, B is k x n, C is m x n.  The sketch has l = r + p columns and
 * the factorisation keeps rank l (no truncation back to r).
 */
typedef struct {
  int64_t m, n, k;
  int32_t r, p, q;
  int32_t fmt_sketch;   /* lramm_fmt of Y = A Omega and Y = A Q_Z          */
  int32_t fmt_proj;     /* lramm_fmt of Z = A^T Q and Bt = Q^T A           */
  int32_t fmt_g1;       /* lramm_fmt of T = Bt B                           */
  int32_t fmt_g2;       /* lramm_fmt of C = Q T                            */
  int32_t a_type, b_type, c_type;   /* lramm_dtype: F32 or BF16            */
  int32_t reserved0;
  uint64_t seed;        /* Philox key when the caller passes no Omega      */
  float alpha, beta;
  uint32_t flags;       /* LRAMM_PLAN_EXCLUSIVE | _SRHT | _ESTIMATE | _ONE_PASS */
  uint32_t reserved1;
  /* Storage of A and B: 0 row-major as m x k (k x n), 1 stored as the
   * transpose, k x m (n x k) row-major.  C is always m x n row-major. */
  int32_t trans_a, trans_b;
  /* Which operand is sketched (paper Alg. 3 approximates either one):
   * 0 the left one, A (the formulas above); 1 the right one, B: the library
   * runs them on C^T = B^T A^T, i.e. with A := B^T, B := A^T, m <-> n, and
   * writes C (not C^T).  Q is then n x l and spans the row space of B. */
  int32_t side;
  int32_t reserved2;
} lramm_desc;

/* desc.flags: the caller runs no other CholeskyQR2 of this library on the
 * GPU while this plan's forward runs, so its one-launch Cholesky may use all
 * compute units (less a margin).  Without it the one-launch form is used
 * only when its grid fits half of them, so that two forwards on different
 * streams are always resident together; larger grids then use per-panel
 * launches whose workgroups never wait on each other. */
#define LRAMM_PLAN_EXCLUSIVE 0x1u
/* desc.flags: the first sketch Y = A Omega uses the structured test matrix
 * of lramm_srht_sketch (the subsampled randomised Hadamard transform; paper
 * Sec. 2.2, the O(mn log r) RSVD cost) instead of the Gaussian one: one pass
 * over A, no operand codes, FP32 arithmetic.  fmt_sketch then applies only
 * to the power iterations' Y = A Q_Z.  Needs A' (the sketched operand as the
 * library runs it) stored row-major (trans_a = 0, or side = 1 with
 * trans_b = 1), 2 <= k and k' <= 32768; lramm_forward's omega must be null.
 * Otherwise LRAMM_E_UNSUPPORTED (LRAMM_E_INVALID for a non-null omega). */
#define LRAMM_PLAN_SRHT 0x2u
/* desc.flags: the forward also forms ||A'||_F^2 (one more read of the
 * sketched operand, beside the orthonormalisation) and ||Bt||_F^2 (after
 * the projection), both in FP64 and deterministic, for
 * lramm_error_estimate. */
#define LRAMM_PLAN_ESTIMATE 0x4u
/* desc.flags: every orthonormalisation of the forward is one pass of
 * Cholesky QR (Gram, Cholesky, triangular solve in FP64) instead of
 * CholeskyQR2 -- the first of the two passes, with the same dependent-column
 * rule.  Q still spans range(Y) exactly as far as the factorisation goes,
 * but is orthonormal only to about 2^-53 cond(Y)^2 (Yamamoto, Nakatsukasa,
 * Yanagisawa & Fukaya 2015, Thm. 3.3: ||Q^T Q - I||_2 <= (5/64) d^2 with
 * d = 8 cond(Y) sqrt(m l u + l (l + 1) u) when d < 1), against the unit
 * roundoff level of the second pass.  The paper's range finder (Sec. 2.2)
 * asks only for an orthonormal basis of the sketch; a caller whose stage
 * formats quantise Q to 2^-8 (bf16) or coarser loses nothing measurable
 * while the sketch's condition number stays far below 2^26. */
#define LRAMM_PLAN_ONE_PASS 0x8u

typedef struct lramm_plan lramm_plan;   /* opaque, host memory */

/* Library set-up on the current device: checks the device is gfx950 and
 * looks up that device's address of the lramm_cholqr2_noalloc scratch.
 * Safe to call more than once.  Returns LRAMM_E_UNSUPPORTED on other
 * devices. */
LRAMM_API lramm_status lramm_init(void);

LRAMM_API const char* lramm_status_string(lramm_status s);

/* ------------------------------------------------------------------------
 * Plan / forward / backward.
 */

/* Validate the description and build the stage schedule and workspace
 * layout.  Host only; *out receives a plan owned by the caller. */
LRAMM_API lramm_status lramm_plan_create(const lramm_desc* desc, lramm_plan** out);
LRAMM_API void lramm_plan_destroy(lramm_plan* plan);

/* Bytes of device workspace lramm_forward / lramm_backward need. */
LRAMM_API lramm_status lramm_workspace_bytes(const lramm_plan* plan, size_t* bytes);

/* Forward pass (paper Alg. 3 in the one-sided form above).
 *   A: m x k (desc.a_type), lda >= k (trans_a: stored k x m, lda >= m).
 *   B: k x n (desc.b_type), ldb >= n (trans_b: stored n x k, ldb >= k).
 *   C: m x n (desc.c_type), ldc >= n; read when beta != 0.
 *   omega: optional k x l FP32 test matrix (ldo >= l); NULL draws it from
 *          Philox4x32-10 with key desc.seed (see lramm_omega).
 *   ws: device workspace of ws_bytes >= lramm_workspace_bytes().
 * After the call the workspace holds the factors (lramm_factors). */
LRAMM_API lramm_status lramm_forward(lramm_plan* plan, const void* A, int64_t lda,
                           const void* B, int64_t ldb, void* C, int64_t ldc,
                           const float* omega, int64_t ldo, void* ws,
                           size_t ws_bytes, void* stream);

/* Device views of the factors the last forward left in ws:
 *   Q: m x l FP64 with leading dimension *ldq (columns >= l are zero);
 *   Bt: l x k FP32 (the dequantised projection Q^T A), leading dim *ldbt.
 * With side 1 these are the factors of B^T: Q is n x l, Bt = Q^T B^T. */
LRAMM_API lramm_status lramm_factors(const lramm_plan* plan, const void* ws,
                           const double** Q, int64_t* ldq, const float** Bt,
                           int64_t* ldbt);

/* Device view of one FP intermediate the last forward left in ws, for
 * stage-by-stage replay against a reference (the FP32 values that feed each
 * quantiser; formats with FP32 accumulation cannot be compared bit for bit):
 *   LRAMM_VIEW_Y  (0): the last sketch Y = A Q_Z (or A Omega), m x l, FP32;
 *   LRAMM_VIEW_Q  (1): Q, m x l, FP64 (as lramm_factors);
 *   LRAMM_VIEW_BT (2): Bt = Q^T A, l x k, FP32;
 *   LRAMM_VIEW_TT (3): T^T = (Bt B)^T, n x l, FP32;
 *   LRAMM_VIEW_T  (4): T = Bt B, l x n, FP32 -- the form the forward keeps
 *                      when G1 read a bf16 B in place (then VIEW_TT is not
 *                      available, and the other way round).
 * *ptr points into ws; *ld is the leading dimension in elements, *dtype an
 * lramm_io value (LRAMM_F32 or LRAMM_F64).  Returns LRAMM_E_INVALID for an
 * unknown or unavailable view or NULL arguments. */
enum { LRAMM_VIEW_Y = 0, LRAMM_VIEW_Q = 1, LRAMM_VIEW_BT = 2, LRAMM_VIEW_TT = 3, LRAMM_VIEW_T = 4 };
LRAMM_API lramm_status lramm_intermediate(const lramm_plan* plan, const void* ws,
                           int32_t which, const void** ptr, int64_t* rows,
                           int64_t* cols, int64_t* ld, int32_t* dtype);

/* Device view of the quantised operands of one product of the last forward
 * on ws, for checking every product on its own operands:
 *   LRAMM_CODES_A_ROWS   (0): A by rows (sketch format), m x k -- A itself
 *                             when a bf16 A fed a bf16 sketch directly;
 *   LRAMM_CODES_SKETCH_R (1): right operand of the last sketch (Omega^T, or
 *                             Q_Z^T after power iterations), l x k;
 *   LRAMM_CODES_Q_COLS   (2): Q^T by rows (= Q by columns, proj format), l x m;
 *   LRAMM_CODES_A_COLS   (3): A^T by rows (proj format), k x m;
 *   LRAMM_CODES_BT_ROWS  (4): Bt by rows (g1 format), l x k;
 *   LRAMM_CODES_B_COLS   (5): B^T by rows (g1 format), n x k;
 *   LRAMM_CODES_Q_ROWS   (6): Q by rows (g2 format), m x l;
 *   LRAMM_CODES_TT_ROWS  (7): T^T by rows (g2 format), n x l.
 * Each is rows x pitch BYTES of codes in the layout lramm_quantize writes
 * (K codes per row, *fmt the lramm_fmt), with one FP32 scale per row (1 for
 * bf16; the A_ROWS scales are not written on the direct path).  Pointers
 * point into ws (or A). */
enum {
  LRAMM_CODES_A_ROWS = 0, LRAMM_CODES_SKETCH_R = 1, LRAMM_CODES_Q_COLS = 2, LRAMM_CODES_A_COLS = 3,
  LRAMM_CODES_BT_ROWS = 4, LRAMM_CODES_B_COLS = 5, LRAMM_CODES_Q_ROWS = 6, LRAMM_CODES_TT_ROWS = 7
};
LRAMM_API lramm_status lramm_codes(const lramm_plan* plan, const void* ws, int32_t which,
                           const void** codes, int64_t* rows, int64_t* K, int64_t* pitch,
                           const float** scales, int32_t* fmt);

/* Backward of C = Q Q^T A B with Q fixed and quantisation straight-through
 * (the gradient of the frozen-Q surrogate):
 *     W = Q^T dC,  dB = (Q^T A)^T W,  dA = Q (W B^T);
 * with side 1 the surrogate is C = A B Q Q^T, and the same formulas run on
 * the transposed problem (dA = dC Q Q^T B^T, dB = A^T dC Q Q^T).  Uses the Q
 * of the preceding lramm_forward on the same ws; all products on the FP32
 * MFMA with FP32 accumulation.  dC: m x n in desc.c_type (lddc); A, B as in
 * the forward (their types and storage); dA and dB are written in the type
 * and storage of A and B (leading dimensions ldda, lddb; bf16 rounded to
 * nearest even); either may be NULL to skip it. */
LRAMM_API lramm_status lramm_backward(lramm_plan* plan, const void* dC, int64_t lddc,
                            const void* A, int64_t lda, const void* B, int64_t ldb,
                            void* dA, int64_t ldda, void* dB, int64_t lddb, void* ws,
                            size_t ws_bytes, void* stream);

/* Synchronise the stream and read the device status word of ws.
 * *flags (nullable) receives the LRAMM_FLAG_* bits; the return value is
 * LRAMM_E_STALL if that bit is set, else LRAMM_E_NONFINITE if that bit is
 * set, else LRAMM_OK (breakdown is reported only through *flags). */
LRAMM_API lramm_status lramm_status_poll(const lramm_plan* plan, const void* ws,
                               void* stream, uint32_t* flags);

/* ------------------------------------------------------------------------
 * Uneven batch: many independent products C_i = alpha A_i B_i + beta C_i,
 * each described by its own plan (shapes, rank and formats per product; the
 * paper's rank rule r = ceil(min(M, K) / 10), Sec. 3.5, is one way to choose
 * them).  The batch owns nstreams (1..16) internal streams of default
 * priority; products are issued largest first, each to the least loaded
 * stream, and joined back into the caller's stream.  LRAMM_BATCH_GRAPH
 * (capture the sequence once and replay it as a HIP graph) is reserved and
 * currently returns LRAMM_E_UNSUPPORTED.  The plans must outlive the batch
 * and must not be used on other streams meanwhile.
 */
typedef struct lramm_batch lramm_batch;   /* opaque, host memory */
#define LRAMM_BATCH_GRAPH 0x1u

LRAMM_API lramm_status lramm_batch_create(int32_t count, lramm_plan* const* plans,
                           int32_t nstreams, uint32_t flags, lramm_batch** out);
LRAMM_API void lramm_batch_destroy(lramm_batch* batch);
/* One device workspace for the whole batch (each product gets a slice). */
LRAMM_API lramm_status lramm_batch_workspace_bytes(const lramm_batch* batch, size_t* bytes);
/* count-long arrays (host memory) of device pointers and leading dimensions,
 * in plan order; omega is always drawn from each plan's seed. */
LRAMM_API lramm_status lramm_batched_forward(lramm_batch* batch, const void* const* A,
                           const int64_t* lda, const void* const* B, const int64_t* ldb,
                           void* const* C, const int64_t* ldc, void* ws, size_t ws_bytes,
                           void* stream);
/* Synchronise and OR the status words of every product. */
LRAMM_API lramm_status lramm_batch_status_poll(const lramm_batch* batch, const void* ws,
                           void* stream, uint32_t* flags);

/* Stage timing, for measurement.  While enabled, lramm_forward records a
 * HIP event pair around every stage on the caller's stream (events are
 * created on the host at the first use and reused).  lramm_stage_times
 * synchronises those events, adds their elapsed times to per-stage totals
 * (milliseconds, launch counts) and clears the record; entries beyond
 * LRAMM_NSTAGES are ignored.  Stage names: lramm_stage_name(). */
#define LRAMM_NSTAGES 22
LRAMM_API lramm_status lramm_plan_set_timing(lramm_plan* plan, int32_t enable);
LRAMM_API lramm_status lramm_stage_times(lramm_plan* plan, double* ms,
                                         int64_t* counts);
LRAMM_API const char* lramm_stage_name(int32_t stage);

/* ------------------------------------------------------------------------
 * Stage entry points (each is one step of the forward, usable alone).
 */

/* Quantise a rows x cols matrix X (xtype F32, BF16 or F64; ldx elements).
 *   transpose == 0: each ROW is one vector (left-operand form);
 *       Xq is rows x pitch bytes, scales has rows entries, K = cols.
 *   transpose == 1: each COLUMN is one vector (right-operand form), stored
 *       transposed: Xq is cols x pitch bytes, scales has cols entries, K = rows.
 * int8/fp8/bf16: K codes per output row (bf16 takes 2 bytes each); int4: codes
 * packed two per byte along K (element 2j in the low nibble).  pitch must be
 * >= lramm_pitch(K, fmt); bytes past the codes up to the padded length are
 * written as zeros.  F64 inputs are rounded once to binary32 first.
 * flags: optional device word; LRAMM_FLAG_NONFINITE is or-ed in when X holds
 * NaN/Inf (the codes of such a vector are then unspecified). */
LRAMM_API lramm_status lramm_quantize(int64_t rows, int64_t cols, const void* X,
                            int64_t ldx, int32_t xtype, int32_t fmt,
                            int32_t transpose, void* Xq, int64_t pitch,
                            float* scales, uint32_t* flags, void* stream);

/* Padded byte length of one quantised vector of K elements (a multiple of
 * 64 bytes, zero-filled past the codes). */
LRAMM_API int64_t lramm_pitch(int64_t K, int32_t fmt);

/* Quantised NT-GEMM (Alg. 2): C[M x N] = epilogue(Lq[M x K] . Rq[N x K]^T)
 *   Lq, Rq: quantised rows with byte pitches ldl, ldr >= lramm_pitch(K, fmt),
 *           zero past K (as lramm_quantize writes them).
 *   dL (M), dR (N): dequantisation factors (ignored for bf16).
 *   C: FP32 or BF16 (ctype), ldc >= N;  c = fl32(fl32(fl32(acc) dL) dR);
 *      out = fl32(alpha c) [+ fl32(beta C_in)] (C_in read only if beta != 0).
 *      fp8 codes are OCP e4m3 multiplied on the 32x32x64 fp8 MFMA with FP32
 *      accumulation (each product is exact in FP32; the sums round in the
 *      hardware's order, so fp8 results match an FP64 sum only to FP32
 *      accumulation accuracy).
 *   acc_out: optional raw int32 accumulators (int8/int4 only), M x ld_acc.
 *   ws / ws_bytes: workspace for split-K partials (may be NULL / 0, then the
 *   library does not split K).  Returns LRAMM_E_OVERFLOW if K * qmax^2 could
 *   exceed the int32 accumulator, LRAMM_E_UNSUPPORTED if M * ldl or N * ldr
 *   reaches 2^31 bytes (operands are addressed with 32-bit offsets). */
LRAMM_API lramm_status lramm_gemm_nt(int64_t M, int64_t N, int64_t K, int32_t fmt,
                           const void* Lq, int64_t ldl, const float* dL,
                           const void* Rq, int64_t ldr, const float* dR,
                           float alpha, float beta, void* C, int64_t ldc,
                           int32_t ctype, int32_t* acc_out, int64_t ld_acc,
                           void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes lramm_gemm_nt may use for split-K on this shape. */
LRAMM_API size_t lramm_gemm_nt_workspace(int64_t M, int64_t N, int64_t K, int32_t fmt);

/* Gaussian test matrix (paper Sec. 2.2, Gaussian sampling), written
 * TRANSPOSED: OmegaT is l x k FP32 with leading dimension ldo >= k.
 * Element Omega[i][j] = OmegaT[j][i] has index e = j*k + i; it is word
 * (e mod 4) of Philox4x32-10 at counter (c mod 2^32, c >> 32, 0, 0),
 * c = e >> 2, key (seed mod 2^32, seed >> 32), turned into normals by the
 * Box-Muller transform in FP64 -- u1 = (x0 + 1) 2^-32, u2 = x1 2^-32,
 * z0 = sqrt(-2 ln u1) cos(2 pi u2), z1 = sqrt(-2 ln u1) sin(2 pi u2), same
 * for (x2, x3) -> (z2, z3) -- and rounded once to binary32. */
LRAMM_API lramm_status lramm_omega(uint64_t seed, int64_t k, int64_t l, float* OmegaT,
                         int64_t ldo, void* stream);

/* Structured test matrix (Halko, Martinsson & Tropp 2011, Sec. 4.6, real
 * form; paper Sec. 2.2, the O(mn log r) RSVD cost): with k' the smallest
 * power of two >= k,
 *     Omega = (D H)[0:k, S] / sqrt(l)     (k x l),
 * H the k' x k' Sylvester-Hadamard matrix, H[i][j] = (-1)^popcount(i & j),
 * D = diag(d_i), d_i = -1 when bit 0 of word x0 of Philox4x32-10 at counter
 * (i, 0, 1, 0) is set (else +1), and S the indices of the l smallest pairs
 * (x0 at counter (i, 0, 2, 0), i), in increasing order; key (seed mod 2^32,
 * seed >> 32) as for lramm_omega.
 * lramm_srht_padded: k' (0 for k < 1).
 * lramm_srht_samples: S (l int32, device) and the sign mask sign_bits
 * (ceil(k' / 32) uint32 words, device; bit i % 32 of word i / 32 set when
 * d_i = -1).  keys: k' uint32 of device scratch (the drawn keys; contents
 * unspecified on return).  Two launches: the keys and signs over k' / 256
 * workgroups, then the selection in one.  Needs 2 <= k, k' <= 32768 (else
 * LRAMM_E_UNSUPPORTED) and 1 <= l <= k' (else LRAMM_E_RANK); a null pointer
 * is LRAMM_E_INVALID.
 * lramm_srht_sketch: Y (m x l FP32, ldy >= l, device) = A Omega for A m x k
 * row-major (a_type F32 or BF16, lda >= k, device) from S and sign_bits as
 * lramm_srht_samples writes them: the fast Walsh-Hadamard transform of each
 * signed row in binary32, the sampled entries multiplied by fl32(1/sqrt(l)).
 * Each entry is within (log2 k' + 3) 2^-24 sum_i |A[r][i]| / sqrt(l) of the
 * exact value.  Same limits on k and l. */
/* A-posteriori error of the range finder after a forward of a plan created
 * with LRAMM_PLAN_ESTIMATE (else LRAMM_E_INVALID): with Q orthonormal,
 * ||A' - Q Q^T A'||_F^2 = ||A'||_F^2 - ||Q^T A'||_F^2 (paper Alg. 1,
 * B = Q* A; Sec. 3.3 states the rank-r error in the Frobenius norm), A' the
 * sketched operand.  Synchronises stream, then writes out[0] =
 * sqrt(max(0, ||A'||^2 - ||Bt||^2) / ||A'||^2) (Bt the projection as
 * computed, so quantised projection formats make it an estimate), out[1] =
 * ||A'||_F^2, out[2] = ||Bt||_F^2.  out: 3 doubles, host memory.  It is the
 * quantity a caller's rank choice can test against a tolerance. */
LRAMM_API lramm_status lramm_error_estimate(const lramm_plan* plan, const void* ws, void* stream,
                           double* out);

LRAMM_API int64_t lramm_srht_padded(int64_t k);
LRAMM_API lramm_status lramm_srht_samples(uint64_t seed, int64_t k, int64_t l, int32_t* S,
                         uint32_t* sign_bits, uint32_t* keys, void* stream);
LRAMM_API lramm_status lramm_srht_sketch(int64_t m, int64_t k, int64_t l, const void* A,
                         int64_t lda, int32_t a_type, const int32_t* S,
                         const uint32_t* sign_bits, float* Y, int64_t ldy, void* stream);

/* CholeskyQR2 of a rows x l matrix Y (ytype F32 or F64, ldy >= l):
 * Q (rows x l FP64, ldq >= round_up(l, 32)) with orthonormal columns spanning
 * range(Y) -- the thin QR factor with positive diagonal.  Gram matrices,
 * Cholesky factors and triangular solves are FP64.  A pivot whose square
 * falls to <= 64 l 2^-53 times its Gram diagonal marks a dependent column:
 * its Q column is zero and LRAMM_FLAG_BREAKDOWN is or-ed into *flags.
 * Columns l .. ldq-1 of Q are written as zero.  ws >= lramm_cholqr2_workspace. */
LRAMM_API lramm_status lramm_cholqr2(int64_t rows, int64_t l, const void* Y, int64_t ldy,
                           int32_t ytype, double* Q, int64_t ldq, void* ws,
                           size_t ws_bytes, uint32_t* flags, void* stream);
LRAMM_API size_t lramm_cholqr2_workspace(int64_t rows, int64_t l);
/* The triangular factor of the range finder's QR (paper Sec. 2.2, Alg. 1:
 * Y = Q R): R = Q^T Y on and above the diagonal, zero below, for the Q that
 * lramm_cholqr2 (or the forward, through lramm_factors) returned for Y.
 *   Y: rows x l, ytype F32 or F64, row-major, ldy >= l (device).
 *   Q: rows x l FP64, ldq >= l (device; columns past l are not read).
 *   R: l x l FP64, row-major, ldr >= l (device, caller-owned; columns past l
 *      are not written).  A column that lramm_cholqr2 dropped (its Q column
 *      is zero) gives a zero row of R.
 * Each entry is an FP64 sum over the rows in row order (bit-reproducible).
 * Returns LRAMM_E_SHAPE for negative sizes or short leading dimensions,
 * LRAMM_E_RANK for l > rows, LRAMM_E_INVALID for a null pointer,
 * LRAMM_E_UNSUPPORTED for another ytype; l = 0 does nothing.  Asynchronous
 * on stream. */
LRAMM_API lramm_status lramm_r_factor(int64_t rows, int64_t l, const void* Y, int64_t ldy,
                           int32_t ytype, const double* Q, int64_t ldq, double* R,
                           int64_t ldr, void* stream);
/* The least workspace lramm_cholqr2 runs in: with fewer bytes than
 * lramm_cholqr2_workspace (but at least these) it sums the FP64 Gram over
 * fewer row chunks -- the same arithmetic up to the order of the chunk sums. */
LRAMM_API size_t lramm_cholqr2_workspace_min(int64_t rows, int64_t l);

/* Host-only query of the schedule rule above: 1 when the Cholesky of an
 * l-column CholeskyQR2 runs as one launch on a GPU with compute_units CUs
 * (plan_flags 0 -- as for lramm_cholqr2 -- or LRAMM_PLAN_EXCLUSIVE), 0 when
 * it runs as per-panel launches.  The grid has 1 + (T-2)(T-1)/2 + T
 * workgroups for T = ceil(l / 32) blocks and is admitted when it is at most
 * compute_units - 16, or half of that without LRAMM_PLAN_EXCLUSIVE. */
LRAMM_API int32_t lramm_chol_one_launch(int64_t l, int32_t compute_units, uint32_t plan_flags);

/* CholeskyQR2 that allocates nothing, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Arguments, results and error codes are
 * those of lramm_cholqr2 (the same kernels: Q is bit-identical), without ws:
 * the scratch is one fixed buffer of LRAMM_NOALLOC_SCRATCH_BYTES inside the
 * library, one per GPU, held until the process ends and looked up by
 * lramm_init() (or by the first call on a device).  It runs on the current
 * device; stream must belong to it.
 *   - Returns LRAMM_E_SCRATCH when even the least CholeskyQR2 workspace
 *     (the Gram summed in one row chunk, about 5 l'^2 doubles) exceeds
 *     LRAMM_NOALLOC_SCRATCH_BYTES (every l <= 768 fits at any row count);
 *     below lramm_cholqr2_workspace(rows, l) it sums the Gram in fewer
 *     chunks (same results up to the order of the chunk sums).
 *   - Calls no hipMalloc / hipFree or other allocating routine.
 *   - All calls on one GPU share its buffer: calls that overlap in time on
 *     that GPU (several streams, several host threads) race and give wrong
 *     results; serialise them.  The buffer keeps the last call's contents;
 *     every word a call reads is written earlier in that call. */
#define LRAMM_NOALLOC_SCRATCH_BYTES (24u << 20)
LRAMM_API lramm_status lramm_cholqr2_noalloc(int64_t rows, int64_t l, const void* Y, int64_t ldy,
                           int32_t ytype, double* Q, int64_t ldq, uint32_t* flags,
                           void* stream);

/* ------------------------------------------------------------------------
 * Two-sided form, the paper's Alg. 3 (Sec. 3.2):
 *   rank-r RSVD of A and of B (Alg. 1 after the range finder above: Q from a
 *   sketch of l = r + p columns with q power iterations, Bt = Q^T A, small
 *   SVD Bt = U' S V^T, U = Q U', first r triplets kept), signs fixed so that
 *   the largest-magnitude entry of each column of U' is positive;
 *   U~ = U_A S_A (m x r), Z~ = G_B Z_B^T (r x n), computed in FP64 and
 *   rounded once to binary32, as are V_A^T (r x k) and W_B (k x r);
 *   E1 = QM(V_A^T W_B, d1), E2 = QM(E1 Z~, d2), D = alpha QM(U~ E2, d3) + beta C,
 * each QM the quantised product of Alg. 2.  The small SVD is the
 * eigen-decomposition of the FP64 Gram Bt Bt^T by Jacobi rotations, for
 * round_up(l, 2) <= 128 (else LRAMM_E_UNSUPPORTED).  A: m x k (a_type,
 * lda >= k), B: k x n (b_type, ldb >= n), C: m x n (c_type, ldc >= n);
 * omega_a (k x l, ldoa) and omega_b (n x l, ldob) may be NULL: then they
 * come from Philox with keys seed and seed + 1. */
typedef struct {
  int64_t m, n, k;
  int32_t r, p, q;
  int32_t fmt_sketch, fmt_proj;     /* lramm_fmt of both RSVDs' sketch / projection */
  int32_t fmt_e1, fmt_e2, fmt_e3;   /* the paper's bit budgets d1, d2, d3           */
  int32_t a_type, b_type, c_type;
  uint64_t seed;
  float alpha, beta;
  uint32_t flags;                   /* must be 0 */
  int32_t reserved;
} lramm_ts_desc;
typedef struct lramm_ts_plan lramm_ts_plan;
LRAMM_API lramm_status lramm_ts_plan_create(const lramm_ts_desc* desc, lramm_ts_plan** out);
LRAMM_API void lramm_ts_plan_destroy(lramm_ts_plan* plan);
LRAMM_API lramm_status lramm_ts_workspace_bytes(const lramm_ts_plan* plan, size_t* bytes);
LRAMM_API lramm_status lramm_ts_forward(lramm_ts_plan* plan, const void* A, int64_t lda, const void* B,
                           int64_t ldb, void* C, int64_t ldc, const float* omega_a, int64_t ldoa,
                           const float* omega_b, int64_t ldob, void* ws, size_t ws_bytes, void* stream);
/* Views of the two-sided intermediates (FP32 unless noted):
 *   LRAMM_TS_UT U~ (m x r), LRAMM_TS_VT V_A^T (r x k), LRAMM_TS_W W_B (k x r),
 *   LRAMM_TS_ZS Z~ (r x n), LRAMM_TS_E1 (r x r), LRAMM_TS_E2 (r x n),
 *   LRAMM_TS_SA / LRAMM_TS_SB singular values (r, FP64),
 *   LRAMM_TS_UPA / LRAMM_TS_UPB U' (l x r, FP64). */
enum { LRAMM_TS_UT = 0, LRAMM_TS_VT = 1, LRAMM_TS_W = 2, LRAMM_TS_ZS = 3, LRAMM_TS_E1 = 4, LRAMM_TS_E2 = 5,
       LRAMM_TS_SA = 6, LRAMM_TS_SB = 7, LRAMM_TS_UPA = 8, LRAMM_TS_UPB = 9 };
LRAMM_API lramm_status lramm_ts_intermediate(const lramm_ts_plan* plan, const void* ws, int32_t which,
                           const void** ptr, int64_t* rows, int64_t* cols, int64_t* ld,
                           int32_t* dtype);
/* Synchronise and OR the status words of both RSVDs and of the chain
 * (LRAMM_FLAG_BREAKDOWN also when Jacobi did not converge in 60 sweeps). */
LRAMM_API lramm_status lramm_ts_status_poll(const lramm_ts_plan* plan, const void* ws, void* stream,
                           uint32_t* flags);

/* Dense comparator GEMM (no quantisation, no vendor library):
 * C[M x N] = L[M x K] . R[N x K]^T with both operands K-contiguous.
 * dtype BF16: bf16 inputs (uint16 storage), FP32 accumulation, FP32 output.
 * dtype F32: FP32 inputs and output, FP32 accumulation.  ldl, ldr, ldc are
 * in elements; K must be a multiple of 64 and ldl, ldr multiples of 64. */
LRAMM_API lramm_status lramm_dense_gemm_nt(int64_t M, int64_t N, int64_t K,
                                 int32_t dtype, const void* L, int64_t ldl,
                                 const void* R, int64_t ldr, float* C,
                                 int64_t ldc, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LRAMM_H */
