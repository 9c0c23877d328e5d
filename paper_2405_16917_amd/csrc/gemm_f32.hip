// FP32 GEMM on gfx950 MFMA (v_mfma_f32_32x32x2f32, FP32 accumulation) with
// either operand stored K-contiguous or M/N-contiguous.  It serves the
// frozen-Q backward (products with Q, Q^T, B^T and dC) and the dense FP32
// comparator.  Operands may be binary32, bf16 or FP64 (the orthonormal
// factor Q), each converted to binary32 on load; the output is binary32 or
// bf16 (round to nearest even).
//
// Tiling: 256 threads = 4 wavefronts (2 x 2), block tile 128 x 128, K stages
// of 16, double-buffered.  LDS holds both tiles K-major ([k][m], [k][n]) so an
// MFMA operand read is 32 consecutive floats per k (conflict-free).  Operand
// layout of v_mfma_f32_32x32x2f32: lane l supplies A[l % 32][l / 32] and
// B[l / 32][l % 32]; result as for the other 32 x 32 MFMAs.
#include "common.hpp"

namespace lramm {

constexpr int FBM = 128, FBN = 128, FBK = 16, FPAD = 4;

struct F32Args {
  int M, N, K;
  const void* A;
  int64_t lda;
  const void* B;
  int64_t ldb;
  void* C;
  int64_t ldc;
  int vec_a, vec_b;
  int c_bf16;
};

// four consecutive elements of type T as binary32 (vector load)
template <typename T>
__device__ __forceinline__ void load4v(const T* p, float v[4]) {
  if constexpr (sizeof(T) == 4) {
    float4 f = *reinterpret_cast<const float4*>(p);
    v[0] = f.x; v[1] = f.y; v[2] = f.z; v[3] = f.w;
  } else if constexpr (sizeof(T) == 8) {
    double2 a = *reinterpret_cast<const double2*>(p);
    double2 b = *reinterpret_cast<const double2*>(p + 2);
    v[0] = (float)a.x; v[1] = (float)a.y; v[2] = (float)b.x; v[3] = (float)b.y;
  } else {
    uint2 u = *reinterpret_cast<const uint2*>(p);
    v[0] = __uint_as_float(u.x << 16);
    v[1] = __uint_as_float(u.x & 0xffff0000u);
    v[2] = __uint_as_float(u.y << 16);
    v[3] = __uint_as_float(u.y & 0xffff0000u);
  }
}

template <typename T>
__device__ __forceinline__ float load1f(const T* p) {
  if constexpr (sizeof(T) == 2) return bf16_to_float(*p);
  else return (float)*p;
}

// Load a ROWSxFBK (kmajor == 0) or FBKxROWS (kmajor == 1) tile into registers
// as 2 float4 per thread, then scatter into LDS as [k][row].
template <int KMAJOR, typename T>
struct F32Tile {
  float v[2][4];
  __device__ __forceinline__ void load(const T* base, int64_t ld, int r0, int rtot, int k0, int ktot, int vec,
                                       int tid) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      int e = tid + 256 * i;
      if constexpr (KMAJOR == 0) {          // rows of K: row = e / 4, k = 4 (e % 4)
        int row = e >> 2, kq = (e & 3) * 4;
        int gr = r0 + row, gk = k0 + kq;
        const T* p = base + (int64_t)gr * ld + gk;
        if (vec && gr < rtot && gk + 3 < ktot) {
          load4v<T>(p, v[i]);
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) v[i][q] = (gr < rtot && gk + q < ktot) ? load1f<T>(p + q) : 0.0f;
        }
      } else {                              // K rows of contiguous ROWS: k = e / 32, row = 4 (e % 32)
        int kk = e >> 5, rq = (e & 31) * 4;
        int gk = k0 + kk, gr = r0 + rq;
        const T* p = base + (int64_t)gk * ld + gr;
        if (vec && gk < ktot && gr + 3 < rtot) {
          load4v<T>(p, v[i]);
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) v[i][q] = (gk < ktot && gr + q < rtot) ? load1f<T>(p + q) : 0.0f;
        }
      }
    }
  }
  __device__ __forceinline__ void store(float (*s)[FBM + FPAD], int tid) const {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      int e = tid + 256 * i;
      if constexpr (KMAJOR == 0) {
        int row = e >> 2, kq = (e & 3) * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) s[kq + q][row] = v[i][q];
      } else {
        int kk = e >> 5, rq = (e & 31) * 4;
        *reinterpret_cast<float4*>(&s[kk][rq]) = make_float4(v[i][0], v[i][1], v[i][2], v[i][3]);
      }
    }
  }
};

template <int AK, int BK_, typename TA, typename TB>
__global__ __launch_bounds__(256, 2) void gemm_f32_kernel(F32Args a) {
  __shared__ __attribute__((aligned(16))) float sA[2][FBK][FBM + FPAD];
  __shared__ __attribute__((aligned(16))) float sB[2][FBK][FBN + FPAD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int tiles_n = (a.N + FBN - 1) / FBN;
  const int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
  const int m0 = tm * FBM, n0 = tn * FBN;
  const int nst = (a.K + FBK - 1) / FBK;

  v16f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

  F32Tile<AK, TA> ta;
  F32Tile<BK_, TB> tb;
  const TA* Ap = reinterpret_cast<const TA*>(a.A);
  const TB* Bp = reinterpret_cast<const TB*>(a.B);
  if (nst > 0) {
    ta.load(Ap, a.lda, m0, a.M, 0, a.K, a.vec_a, tid);
    tb.load(Bp, a.ldb, n0, a.N, 0, a.K, a.vec_b, tid);
    ta.store(sA[0], tid);
    tb.store(sB[0], tid);
  }
  __syncthreads();
  const int ar = wm * 64 + (lane & 31), br = wn * 64 + (lane & 31), kl = lane >> 5;
  for (int st = 0; st < nst; ++st) {
    const int buf = st & 1;
    const bool more = st + 1 < nst;
    if (more) {
      ta.load(Ap, a.lda, m0, a.M, (st + 1) * FBK, a.K, a.vec_a, tid);
      tb.load(Bp, a.ldb, n0, a.N, (st + 1) * FBK, a.K, a.vec_b, tid);
    }
#pragma unroll
    for (int kk = 0; kk < FBK; kk += 2) {
      float av0 = sA[buf][kk + kl][ar], av1 = sA[buf][kk + kl][ar + 32];
      float bv0 = sB[buf][kk + kl][br], bv1 = sB[buf][kk + kl][br + 32];
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(av0, bv0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(av0, bv1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(av1, bv0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(av1, bv1, acc[1][1], 0, 0, 0);
    }
    if (more) {
      ta.store(sA[buf ^ 1], tid);
      tb.store(sB[buf ^ 1], tid);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int gn = n0 + wn * 64 + 32 * j + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int gm = m0 + wm * 64 + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (gm < a.M && gn < a.N) {
          const int64_t idx = (int64_t)gm * a.ldc + gn;
          if (a.c_bf16) reinterpret_cast<uint16_t*>(a.C)[idx] = bf16_bits(acc[i][j][r]);
          else reinterpret_cast<float*>(a.C)[idx] = acc[i][j][r];
        }
      }
    }
}

template <int AK, int BK_, typename TA, typename TB>
static void launch_f32_t(const F32Args& a, hipStream_t s) {
  int tiles = ((a.M + FBM - 1) / FBM) * ((a.N + FBN - 1) / FBN);
  hipLaunchKernelGGL((gemm_f32_kernel<AK, BK_, TA, TB>), dim3(tiles), dim3(256), 0, s, a);
}

template <typename TA, typename TB>
static void launch_f32_layouts(const F32Args& a, int a_kmajor, int b_kmajor, hipStream_t s) {
  // A stored M x K (a_kmajor == 0): loader KMAJOR 0; stored K x M: loader KMAJOR 1.
  // B stored N x K (b_kmajor == 0): loader KMAJOR 0; stored K x N: loader KMAJOR 1.
  if (!a_kmajor && !b_kmajor) launch_f32_t<0, 0, TA, TB>(a, s);
  else if (!a_kmajor && b_kmajor) launch_f32_t<0, 1, TA, TB>(a, s);
  else if (a_kmajor && !b_kmajor) launch_f32_t<1, 0, TA, TB>(a, s);
  else launch_f32_t<1, 1, TA, TB>(a, s);
}

template <typename TA>
static lramm_status launch_f32_b(const F32Args& a, int a_kmajor, int b_kmajor, int b_type, hipStream_t s) {
  switch (b_type) {
    case LRAMM_F32: launch_f32_layouts<TA, float>(a, a_kmajor, b_kmajor, s); break;
    case LRAMM_F64: launch_f32_layouts<TA, double>(a, a_kmajor, b_kmajor, s); break;
    case LRAMM_BF16: launch_f32_layouts<TA, uint16_t>(a, a_kmajor, b_kmajor, s); break;
    default: return LRAMM_E_UNSUPPORTED;
  }
  return LRAMM_OK;
}

static size_t esize(int t) { return t == LRAMM_F64 ? 8 : (t == LRAMM_BF16 ? 2 : 4); }

lramm_status launch_gemm_f32(int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, int a_kmajor, int a_type,
                             const void* B, int64_t ldb, int b_kmajor, int b_type, void* C, int64_t ldc, int c_type,
                             hipStream_t s) {
  if (M == 0 || N == 0) return LRAMM_OK;
  if (c_type != LRAMM_F32 && c_type != LRAMM_BF16) return LRAMM_E_UNSUPPORTED;
  F32Args a;
  a.M = (int)M;
  a.N = (int)N;
  a.K = (int)K;
  a.A = A;
  a.lda = lda;
  a.B = B;
  a.ldb = ldb;
  a.C = C;
  a.ldc = ldc;
  a.c_bf16 = c_type == LRAMM_BF16 ? 1 : 0;
  // 4-element vector loads need 4-element aligned rows
  a.vec_a = ((uintptr_t)A % (4 * esize(a_type)) == 0) && (lda % 4 == 0);
  a.vec_b = ((uintptr_t)B % (4 * esize(b_type)) == 0) && (ldb % 4 == 0);
  lramm_status st;
  switch (a_type) {
    case LRAMM_F32: st = launch_f32_b<float>(a, a_kmajor, b_kmajor, b_type, s); break;
    case LRAMM_F64: st = launch_f32_b<double>(a, a_kmajor, b_kmajor, b_type, s); break;
    case LRAMM_BF16: st = launch_f32_b<uint16_t>(a, a_kmajor, b_kmajor, b_type, s); break;
    default: return LRAMM_E_UNSUPPORTED;
  }
  if (st != LRAMM_OK) return st;
  LRAMM_HIP(hipGetLastError());
  return LRAMM_OK;
}

lramm_status launch_dense_gemm_nt(int64_t M, int64_t N, int64_t K, int dtype, const void* L, int64_t ldl,
                                  const void* R, int64_t ldr, float* C, int64_t ldc, hipStream_t s) {
  if (dtype == LRAMM_BF16) {
    return launch_gemm_nt(M, N, K, LRAMM_BF16F, L, 2 * ldl, nullptr, R, 2 * ldr, nullptr, 1.0f, 0.0f, C, ldc,
                          LRAMM_F32, nullptr, 0, nullptr, 0, s);
  }
  if (dtype == LRAMM_F32) {
    return launch_gemm_f32(M, N, K, L, ldl, 0, LRAMM_F32, R, ldr, 0, LRAMM_F32, C, ldc, LRAMM_F32, s);
  }
  return LRAMM_E_UNSUPPORTED;
}

}  // namespace lramm
