// Internal helpers shared by the HIP sources of the LRAMM library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lramm.h"

namespace lramm {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef int v8i __attribute__((ext_vector_type(8)));

constexpr int kWave = 64;

#define LRAMM_HIP(expr)                              \
  do {                                               \
    hipError_t _e = (expr);                          \
    if (_e != hipSuccess) return LRAMM_E_HIP;        \
  } while (0)

#define LRAMM_TRY(expr)                              \
  do {                                               \
    lramm_status _s = (expr);                        \
    if (_s != LRAMM_OK) return _s;                   \
  } while (0)

static inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
static inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// Bytes of one quantised vector of K elements in format fmt: padded to 64
// bytes (128 for bf16, so that a padded row always holds whole 64-element
// tiles).
static inline int64_t pitch_bytes(int64_t K, int fmt) {
  int64_t raw = (fmt == LRAMM_INT4) ? ceil_div(K, 2) : (fmt == LRAMM_BF16F ? 2 * K : K);
  return round_up(raw > 0 ? raw : 1, fmt == LRAMM_BF16F ? 128 : 64);
}

// Elements one padded quantised vector holds.
static inline int64_t pitch_elems(int64_t pitch, int fmt) {
  return fmt == LRAMM_INT4 ? 2 * pitch : (fmt == LRAMM_BF16F ? pitch / 2 : pitch);
}

static inline int qmax_of(int fmt) {
  return fmt == LRAMM_INT8 ? 127 : (fmt == LRAMM_INT4 ? 7 : 448);
}

// ---------------------------------------------------------------- device ---

// Wavefront maximum of unsigned values (absmax bit patterns).
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = max(v, (unsigned)__shfl_xor((int)v, o, 64));
  return v;
}

// Largest |x| bit pattern: for non-negative floats the IEEE bits order like
// the values, so an unsigned max of |x| bits is the absmax (NaN/Inf compare
// above every finite value and are caught separately).
__device__ __forceinline__ unsigned abs_bits(float x) { return __float_as_uint(x) & 0x7fffffffu; }

// Quantiser parameters from the absmax (rule of the paper's Sec. 3.1 with the
// readings documented in lramm.h): lambda = fl32(qmax / amax),
// d = fl32(amax / qmax); zero / overflowing lambda -> all-zero codes, d = 0.
struct QParams {
  float lam;
  float d;
};

__device__ __forceinline__ QParams qparams(float amax, float qmax) {
  QParams p;
  if (!(amax > 0.0f) || !(amax <= 3.4028234663852886e38f)) {
    p.lam = 0.0f;
    p.d = 0.0f;
    return p;
  }
  float lam = __fdiv_rn(qmax, amax);
  if (!(lam <= 3.4028234663852886e38f)) {
    p.lam = 0.0f;
    p.d = 0.0f;
    return p;
  }
  p.lam = lam;
  p.d = __fdiv_rn(amax, qmax);
  return p;
}

// One code: clamp(rne(fl32(v * lam)), -qmax, qmax).
__device__ __forceinline__ int qcode(float v, float lam, float qmax) {
  float y = __fmul_rn(v, lam);
  y = __builtin_rintf(y);
  y = fminf(fmaxf(y, -qmax), qmax);
  return (int)y;
}

// OCP e4m3 (bias 7, max 448, no infinity): saturating round-to-nearest-even
// of a finite binary32 value, returned as the 8-bit pattern.
__device__ __forceinline__ uint32_t e4m3_bits(float y) {
  uint32_t sign = (__float_as_uint(y) >> 24) & 0x80u;
  float a = fabsf(y);
  if (a >= 448.0f) return sign | 0x7eu;            // saturate (S.1111.110 = 448)
  // spacing of the e4m3 grid in a's binade: 2^(e-3) for normals, 2^-9 below 2^-6
  int e;
  frexpf(a, &e);                                   // a = f 2^e, 0.5 <= f < 1
  int sp_exp = e - 4;
  if (sp_exp < -9) sp_exp = -9;
  float sp = ldexpf(1.0f, sp_exp);
  float qv = __builtin_rintf(a / sp) * sp;         // exact: a / sp is a power-of-2 scaling
  if (qv >= 448.0f) return sign | 0x7eu;
  if (qv == 0.0f) return sign;
  int qe;
  float qf = frexpf(qv, &qe);                      // qv = qf 2^qe
  int biased = qe - 1 + 7;
  if (biased <= 0) {                               // subnormal: value = m/8 * 2^-6
    uint32_t mant = (uint32_t)(qv * 512.0f);       // qv / 2^-9
    return sign | mant;
  }
  uint32_t mant = (uint32_t)((qf * 2.0f - 1.0f) * 8.0f);
  return sign | ((uint32_t)biased << 3) | mant;
}

// bf16 round-to-nearest-even of a finite binary32 value (16-bit pattern).
__device__ __forceinline__ uint16_t bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_float(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// Encode 4 consecutive values (elements c0..c0+3, c0 % 4 == 0) of one vector
// and store them at element offset c0 of the output row.
template <int FMT>
__device__ __forceinline__ void encode4(uint8_t* row, int64_t c0, const float v[4], bool live[4], float lam) {
  if constexpr (FMT == LRAMM_INT8) {
    uint32_t w = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int q = live[j] ? qcode(v[j], lam, 127.0f) : 0;
      w |= ((uint32_t)(q & 0xff)) << (8 * j);
    }
    *reinterpret_cast<uint32_t*>(row + c0) = w;
  } else if constexpr (FMT == LRAMM_INT4) {
    uint32_t w = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int q = live[j] ? qcode(v[j], lam, 7.0f) : 0;
      w |= ((uint32_t)(q & 0xf)) << (4 * j);
    }
    *reinterpret_cast<uint16_t*>(row + c0 / 2) = (uint16_t)w;
  } else if constexpr (FMT == LRAMM_FP8) {
    uint32_t w = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      uint32_t b = live[j] ? e4m3_bits(__fmul_rn(v[j], lam)) : 0u;
      w |= b << (8 * j);
    }
    *reinterpret_cast<uint32_t*>(row + c0) = w;
  } else {  // bf16
    uint32_t lo = (live[0] ? bf16_bits(v[0]) : 0u) | ((uint32_t)(live[1] ? bf16_bits(v[1]) : 0u) << 16);
    uint32_t hi = (live[2] ? bf16_bits(v[2]) : 0u) | ((uint32_t)(live[3] ? bf16_bits(v[3]) : 0u) << 16);
    uint2 w;
    w.x = lo;
    w.y = hi;
    *reinterpret_cast<uint2*>(row + 2 * c0) = w;
  }
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011): ten rounds of
// (hi(M1 x2) ^ x1 ^ k0, lo(M1 x2), hi(M0 x0) ^ x3 ^ k1, lo(M0 x0)), the key
// bumped by the Weyl constants after every round.
__device__ __forceinline__ void philox_round(uint32_t& x0, uint32_t& x1, uint32_t& x2, uint32_t& x3, uint32_t k0,
                                             uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  uint32_t hi0 = __umulhi(M0, x0), lo0 = M0 * x0;
  uint32_t hi1 = __umulhi(M1, x2), lo1 = M1 * x2;
  uint32_t n0 = hi1 ^ x1 ^ k0, n2 = hi0 ^ x3 ^ k1;
  x0 = n0;
  x1 = lo1;
  x2 = n2;
  x3 = lo0;
}

__device__ __forceinline__ void philox4x32_10(uint32_t ctr[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    philox_round(ctr[0], ctr[1], ctr[2], ctr[3], k0, k1);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

template <typename T>
__device__ __forceinline__ float load_as_f32(const T* p);
template <>
__device__ __forceinline__ float load_as_f32<float>(const float* p) { return *p; }
template <>
__device__ __forceinline__ float load_as_f32<uint16_t>(const uint16_t* p) { return bf16_to_float(*p); }
template <>
__device__ __forceinline__ float load_as_f32<double>(const double* p) { return (float)(*p); }

// Simple fill kernel (used instead of hipMemsetAsync so that sequences stay
// safe to capture in a graph).
__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, int64_t n);

lramm_status fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);

// ------------------------------------------------------------ host-side ---
// Internal launchers (no argument validation beyond what the kernels need;
// the C ABI layer validates).

// Column form (transpose = 1) with amax_ws: the column maxima go to that
// caller-zeroed buffer (abs bit patterns, cols entries) -- or are already
// there when amax_ready -- and the quantise pass writes the scales, saving the
// fill and scale launches.  With zero, zero_words words there are cleared
// too, by the row kernels themselves (one launch fewer for the caller).
lramm_status launch_quantize(int64_t rows, int64_t cols, const void* X, int64_t ldx, int xtype, int fmt,
                             int transpose, void* Xq, int64_t pitch, float* scales, uint32_t* flags,
                             hipStream_t s, uint32_t* amax_ws = nullptr, bool amax_ready = false,
                             uint32_t* zero = nullptr, int64_t zero_words = 0);

// Row codes (rows x rpitch, row scales) and transposed column codes (cols x
// cpitch, column scales) of X in one format from two reads of X (FP32 or
// BF16): the row and column maxima (into caller-zeroed rmax / cmax words;
// skipped for bf16), then both code matrices.  Bit-identical to the two
// separate quantisations.
lramm_status launch_quantize_both(int64_t rows, int64_t cols, const void* X, int64_t ldx, int xtype, int fmt,
                                  void* Rq, int64_t rpitch, float* rscales, void* Cq, int64_t cpitch,
                                  float* cscales, uint32_t* rmax, uint32_t* cmax, uint32_t* flags, hipStream_t s);

// km (bf16 only): bit 0 -- Lq is a bf16 matrix stored K-major (K rows of M
// elements, ldl bytes apart) instead of K-contiguous rows; bit 1 -- the same
// for Rq (K rows of N elements, ldr bytes apart).  Runs on the 128-row tiles.
// Optional second output of a bf16 product summed over K slices with the
// identity epilogue: C's bf16 row codes, or with ``transposed`` the codes of
// C's columns (one codes row per column of C), pitch and pe in elements, and
// unit scales.  *written tells whether they were formed (else the caller runs
// the quantiser on C).
struct CodesOut {
  uint16_t* codes;
  int64_t pitch;
  int64_t pe;
  float* scales;
  bool* written;
  bool transposed;
};
lramm_status launch_bf16_cols_from_parts(int64_t rows, int64_t cols, const float* parts, int nsplit, float* C,
                                         int64_t ldc, uint8_t* Xq, int64_t pitch, float* scales, hipStream_t s);
lramm_status launch_gemm_nt(int64_t M, int64_t N, int64_t K, int fmt, const void* Lq, int64_t ldl,
                            const float* dL, const void* Rq, int64_t ldr, const float* dR, float alpha,
                            float beta, void* C, int64_t ldc, int ctype, int32_t* acc_out, int64_t ld_acc,
                            void* ws, size_t ws_bytes, hipStream_t s, bool col_first = false, int km = 0,
                            const CodesOut* codes = nullptr);
size_t gemm_nt_workspace(int64_t M, int64_t N, int64_t K, int fmt);

lramm_status launch_omega(uint64_t seed, int64_t k, int64_t l, int64_t lrows, float* OmegaT, int64_t ldo,
                          hipStream_t s);
// Omega generated and quantised by rows of Omega^T in one launch (codes l x
// pitch, l scales), for k up to omega_quant_max_k(); LRAMM_E_UNSUPPORTED past it.
lramm_status launch_omega_quant(uint64_t seed, int64_t k, int64_t l, int fmt, uint8_t* Oq, int64_t pitch,
                                float* scales, hipStream_t s);
int64_t omega_quant_max_k();

// Structured test matrix (subsampled randomised Hadamard transform): k' =
// srht_padded(k) <= 32768 and k >= 2.  The sample set S (l int32, increasing)
// and the sign mask (ceil(k' / 32) words) from the seed, one workgroup; then
// Y (m x l, ldy) = (A_pad D H)[:, S] / sqrt(l) from A (m x k row-major, FP32
// or BF16), one workgroup per row.
int64_t srht_padded(int64_t k);
// zero (nullable): zero_words words cleared by the first launch on the way.
lramm_status launch_srht_samples(uint64_t seed, int64_t k, int64_t l, int32_t* S, uint32_t* sign_bits,
                                 uint32_t* keys, hipStream_t s, uint32_t* zero = nullptr, int64_t zero_words = 0);
lramm_status launch_srht(int64_t m, int64_t k, int64_t l, const void* A, int64_t lda, int a_type,
                         const uint32_t* sign_bits, const int32_t* S, float* Y, int64_t ldy, hipStream_t s);

// Squared Frobenius norm of a rows x cols matrix (FP32 or BF16, ldx) into
// *out (FP64, device), deterministic: partial sums per band of rows in part
// (sumsq_parts_max() doubles), then summed in index order.
lramm_status launch_sumsq(int64_t rows, int64_t cols, const void* X, int64_t ldx, int xtype, double* part,
                          double* out, hipStream_t s);
int sumsq_parts_max();

// Optional measurement hook: event pairs around individual launches.
struct TimingHook {
  void* ctx;
  void (*begin)(void* ctx, int stage);   // stage | (launches << 16): one event pair over that many launches
  void (*end)(void* ctx);
};
// sub-stage ids inside the orthonormalisation (continuing the forward's list)
enum { SUB_CHOL_GRAM = 17, SUB_CHOL_PANEL = 18, SUB_CHOL_SOLVE = 19, SUB_CHOL_SERIES = 20, SUB_CHOL_APPLY = 21 };

// How the Cholesky inside CholeskyQR2 may run.  Its one-launch form needs
// every workgroup of its grid resident at once, since they wait on each
// other:
//   CHAIN_OFF:       per-panel launches only (workgroups never wait), for
//                    callers that run several orthonormalisations at once;
//   CHAIN_SHARED:    one launch when its grid fits half of the compute units
//                    less a margin, so that two such grids issued on
//                    different streams are still resident together;
//   CHAIN_EXCLUSIVE: one launch when its grid fits all compute units less a
//                    margin; the caller runs no other one-launch Cholesky on
//                    the GPU meanwhile.
enum ChainMode { CHAIN_OFF = 0, CHAIN_SHARED = 1, CHAIN_EXCLUSIVE = 2 };
// The rule itself (host only): an l-column orthonormalisation on a GPU with
// compute_units CUs.
bool chain_admits(int64_t l, int compute_units, int chain_mode);

// colmax (nullable, caller-zeroed, ldq entries): column maxima of fl32(|Q|)
// as bit patterns, accumulated while Q is written.  passes = 1 stops after
// the first Cholesky QR pass (Q = Y R1^-1).
lramm_status launch_r_factor(int64_t rows, int64_t l, const void* Y, int64_t ldy, int ytype, const double* Q,
                             int64_t ldq, double* R, int64_t ldr, hipStream_t s);
// Optional output of a one-pass Cholesky QR: Q's bf16 codes in both layouts
// the bf16 products read (row codes, rows x rpitch elements, and the
// transposed codes, one row per column of Q, l x cpitch elements), each code
// bf16(fl32(q)), with unit scales.  *written tells whether they were formed.
struct QCodesOut {
  uint16_t* rows;
  int64_t rpitch;
  float* rscales;
  uint16_t* cols;
  int64_t cpitch;
  float* cscales;
  bool* written;
};
lramm_status launch_cholqr2(int64_t rows, int64_t l, const void* Y, int64_t ldy, int ytype, double* Q,
                            int64_t ldq, void* ws, size_t ws_bytes, uint32_t* flags, hipStream_t s,
                            const TimingHook* hook = nullptr, uint32_t* colmax = nullptr,
                            int chain_mode = CHAIN_SHARED, int passes = 2, const QCodesOut* qcodes = nullptr);
size_t cholqr2_workspace(int64_t rows, int64_t l);
// The least workspace CholeskyQR2 runs in (one row chunk of the Gram); with
// less than cholqr2_workspace it uses fewer chunks.
size_t cholqr2_workspace_min(int64_t rows, int64_t l);

lramm_status launch_dense_gemm_nt(int64_t M, int64_t N, int64_t K, int dtype, const void* L, int64_t ldl,
                                  const void* R, int64_t ldr, float* C, int64_t ldc, hipStream_t s);

// FP32 GEMM with either operand stored K-contiguous ("t" = transposed
// storage) or M/N-contiguous: C[M x N] = op(A) op(B), FP32 accumulation.
//   a_kmajor == 0: A stored M x K (lda, K contiguous)  -- A[i][k] = A[i*lda+k]
//   a_kmajor == 1: A stored K x M (lda, M contiguous)  -- A[i][k] = A[k*lda+i]
//   b_kmajor == 0: B stored N x K (ldb, K contiguous)  -- B[k][j] = B[j*ldb+k]
//   b_kmajor == 1: B stored K x N (ldb, N contiguous)  -- B[k][j] = B[k*ldb+j]
// a_type, b_type: LRAMM_F32, LRAMM_F64 or LRAMM_BF16 (converted to binary32
// on load); c_type: LRAMM_F32 or LRAMM_BF16 (rounded to nearest even).
lramm_status launch_gemm_f32(int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, int a_kmajor,
                             int a_type, const void* B, int64_t ldb, int b_kmajor, int b_type, void* C,
                             int64_t ldc, int c_type, hipStream_t s);

// Two-sided form: FP64 Gram of the rows of X (n x n, zero past rows), the
// small SVD from it by Jacobi (n even, <= jacobi_max_order()), and FP32
// results of FP64-accumulated products (operands FP32 or FP64, layouts as
// launch_gemm_f32).
lramm_status launch_rowgram(int rows, int cols, const void* X, int64_t ldx, int xtype, double* G, int n,
                            hipStream_t s);
int jacobi_max_order();
lramm_status launch_jacobi_svd(int n, int r, const double* G, double* V, double* Up, double* S, double* UpS,
                               double* UpSinv, uint32_t* flags, hipStream_t s);
lramm_status launch_gemm_f64acc(int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, int a_kmajor,
                                int a_type, const void* B, int64_t ldb, int b_kmajor, int b_type, float* C,
                                int64_t ldc, hipStream_t s);

}  // namespace lramm
