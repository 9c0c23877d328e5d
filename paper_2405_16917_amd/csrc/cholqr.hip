// CholeskyQR2 in FP64 for the range finder's orthonormalisation (paper
// Sec. 2.2: a matrix Q with orthonormal columns spanning the sketch).  For a
// rows x l matrix Y (FP32 or FP64):
//
//   pass(X):  G = X^T X (FP64)        Gram, split over row chunks, summed in
//                                      a fixed order (deterministic)
//             G = L L^T               blocked right-looking Cholesky, 32 x 32
//                                      panels, one launch per panel
//             Q = X L^-T              row-block forward substitution
//   Q1 = pass(Y); Q = pass(Q1)        (the second pass restores
//                                      orthogonality lost to cond(Y)^2 u)
//
// The thin QR factor with positive diagonal is unique, so Q equals the
// Householder Q of any other stable method to about cond(Y) * 2^-53.
//
// FP64 matrix work uses v_mfma_f64_16x16x4.  Operand layout: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; the 16 x 16 result puts
// D[4 r + l / 16][l % 16] in accumulator r of lane l (rows interleaved across
// the four lane groups, unlike the 32 x 32 MFMAs).
//
// Dependent columns (rank-deficient Y): a pivot whose square is at most
// 64 l 2^-53 times the original Gram diagonal is dropped -- its column of L
// and of Q become zero and LRAMM_FLAG_BREAKDOWN is raised.  Columns at or
// past l (tile padding) are dropped silently.
#include "common.hpp"

namespace lramm {

constexpr int NB = 32;   // panel width

__device__ __forceinline__ v4d mfma_f64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------------ Gram --
// part[chunk] (lw x lw, lower 32x32 tiles only) = X[rows of chunk]^T X[...]
template <typename T>
__global__ __launch_bounds__(256) void gram_kernel(int64_t rows, int lw, int ncols, const T* __restrict__ X,
                                                   int64_t ldx, double* __restrict__ part, int64_t rows_per_chunk) {
  __shared__ double red[4][NB][NB + 1];
  // lower-triangle tile index -> (ti, tj), ti >= tj
  int t = blockIdx.x, ti = 0;
  while (t > ti) {
    t -= ti + 1;
    ++ti;
  }
  const int tj = t;
  const int chunk = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)chunk * rows_per_chunk;
  int64_t r1 = r0 + rows_per_chunk;
  r1 = r1 < rows ? r1 : rows;
  const int a0 = ti * NB, b0 = tj * NB;
  const int li = lane & 15, lk = lane >> 4;

  v4d acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (v4d){0.0, 0.0, 0.0, 0.0};

  for (int64_t rb = r0 + 4 * wave; rb < r1; rb += 16) {
    int64_t r = rb + lk;
    double xa0 = 0, xa1 = 0, xb0 = 0, xb1 = 0;
    if (r < r1) {   // columns at or past ncols read as zero
      const T* row = X + r * ldx;
      if (a0 + li < ncols) xa0 = (double)row[a0 + li];
      if (a0 + 16 + li < ncols) xa1 = (double)row[a0 + 16 + li];
      if (b0 + li < ncols) xb0 = (double)row[b0 + li];
      if (b0 + 16 + li < ncols) xb1 = (double)row[b0 + 16 + li];
    }
    acc[0][0] = mfma_f64(xa0, xb0, acc[0][0]);
    acc[0][1] = mfma_f64(xa0, xb1, acc[0][1]);
    acc[1][0] = mfma_f64(xa1, xb0, acc[1][0]);
    acc[1][1] = mfma_f64(xa1, xb1, acc[1][1]);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[wave][16 * i + 4 * r + lk][16 * j + li] = acc[i][j][r];
  __syncthreads();
  double* out = part + (int64_t)chunk * lw * lw;
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    int i = e / NB, j = e % NB;
    double v = red[0][i][j];
    v += red[1][i][j];
    v += red[2][i][j];
    v += red[3][i][j];
    out[(int64_t)(a0 + i) * lw + b0 + j] = v;
  }
}

// G (lower tiles) = sum over chunks in order; diag0 = diag(G).
__global__ __launch_bounds__(256) void gram_reduce_kernel(int lw, int nchunks, const double* __restrict__ part,
                                                          double* __restrict__ G, double* __restrict__ diag0) {
  int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)lw * lw) return;
  int i = (int)(e / lw), j = (int)(e % lw);
  if ((i / NB) < (j / NB)) return;   // upper tiles are never read
  double s = 0.0;
  for (int c = 0; c < nchunks; ++c) s += part[(int64_t)c * lw * lw + e];
  G[e] = s;
  if (i == j) diag0[i] = s;
}

// -------------------------------------------------------------- Cholesky --
// Factor the 32 x 32 diagonal block held in sD (lower part) in place and
// build its inverse in sI.  256 threads.
__device__ void factor_diag(double (*sD)[NB + 1], double (*sI)[NB + 1], double* sPiv, const double* diag0, int col0,
                            int l_true, double tol, uint32_t* flags, bool report) {
  const int tid = threadIdx.x;
  for (int j = 0; j < NB; ++j) {
    if (tid == 0) {
      double a = sD[j][j];
      int col = col0 + j;
      double piv = 0.0;
      if (col < l_true) {
        double g0 = diag0[col];
        if (a > tol * g0 && a > 0.0) {
          piv = sqrt(a);
        } else if (report && flags) {
          atomicOr(flags, (a < -tol * g0 || a != a) ? (LRAMM_FLAG_BREAKDOWN | LRAMM_FLAG_SQRTNEG)
                                                    : LRAMM_FLAG_BREAKDOWN);
        }
      }
      *sPiv = piv;
    }
    __syncthreads();
    const double piv = *sPiv;
    const double inv = piv > 0.0 ? 1.0 / piv : 0.0;
    if (tid > j && tid < NB) sD[tid][j] *= inv;
    if (tid == j) sD[j][j] = piv;
    __syncthreads();
    for (int e = tid; e < NB * NB; e += 256) {
      int i = e / NB, c = e % NB;
      if (c > j && i >= c) sD[i][c] -= sD[i][j] * sD[c][j];
    }
    __syncthreads();
  }
  // inverse of the lower-triangular factor, one column per thread
  if (tid < NB) {
    const int c = tid;
    for (int i = 0; i < NB; ++i) {
      double v = 0.0;
      if (i >= c) {
        double s = (i == c) ? 1.0 : 0.0;
        for (int t2 = c; t2 < i; ++t2) s -= sD[i][t2] * sI[t2][c];
        double d = sD[i][i];
        v = d > 0.0 ? s / d : 0.0;
      }
      sI[i][c] = v;
    }
  }
  __syncthreads();
}

// dst (32 x 32, LDS) = src (32 x 32, global rows of ld) * Inv^T
__device__ __forceinline__ void times_inv_t(double (*dst)[NB + 1], const double* src, int64_t ld,
                                            double (*sI)[NB + 1], double (*tmp)[NB + 1]) {
  const int tid = threadIdx.x;
  for (int e = tid; e < NB * NB; e += 256) tmp[e / NB][e % NB] = src[(int64_t)(e / NB) * ld + (e % NB)];
  __syncthreads();
  for (int e = tid; e < NB * NB; e += 256) {
    int i = e / NB, c = e % NB;
    double s = 0.0;
    for (int t = 0; t <= c; ++t) s += tmp[i][t] * sI[c][t];   // Inv is lower: Inv[c][t] = 0 for t > c
    dst[i][c] = s;
  }
  __syncthreads();
}

// One panel step p of the right-looking blocked Cholesky on G (lw x lw, row
// major, lower tiles).  Block b covers tile (i, j) with p <= j <= i < T.
__global__ __launch_bounds__(256) void chol_step_kernel(int lw, int l_true, int p, double* __restrict__ G,
                                                        double* __restrict__ L, double* __restrict__ Dinv,
                                                        const double* __restrict__ diag0, double tol,
                                                        uint32_t* flags) {
  __shared__ double sD[NB][NB + 1];
  __shared__ double sI[NB][NB + 1];
  __shared__ double sT[NB][NB + 1];
  __shared__ double sLi[NB][NB + 1];
  __shared__ double sLj[NB][NB + 1];
  __shared__ double sPiv;
  const int T = lw / NB;
  int t = blockIdx.x, di = 0;
  while (t > di) {
    t -= di + 1;
    ++di;
  }
  const int i = p + di, j = p + t;   // p <= j <= i
  const int tid = threadIdx.x;

  const double* Gpp = G + (int64_t)p * NB * lw + p * NB;
  for (int e = tid; e < NB * NB; e += 256) sD[e / NB][e % NB] = Gpp[(int64_t)(e / NB) * lw + (e % NB)];
  __syncthreads();
  factor_diag(sD, sI, &sPiv, diag0, p * NB, l_true, tol, flags, i == p && j == p);

  if (i == p) {   // j == p: the diagonal block
    double* Lpp = L + (int64_t)p * NB * lw + p * NB;
    double* Dp = Dinv + (int64_t)p * NB * NB;
    for (int e = tid; e < NB * NB; e += 256) {
      int r = e / NB, c = e % NB;
      Lpp[(int64_t)r * lw + c] = c <= r ? sD[r][c] : 0.0;
      Dp[e] = sI[r][c];
    }
    // zero the strictly upper tiles of this block row of L
    for (int64_t e = tid; e < (int64_t)NB * (T - 1 - p) * NB; e += 256) {
      int r = (int)(e / ((T - 1 - p) * NB)), c = (int)(e % ((T - 1 - p) * NB));
      L[(int64_t)(p * NB + r) * lw + (p + 1) * NB + c] = 0.0;
    }
    return;
  }
  // L_ip = G_ip * Inv^T
  times_inv_t(sLi, G + (int64_t)i * NB * lw + p * NB, lw, sI, sT);
  if (j == p) {
    double* Lip = L + (int64_t)i * NB * lw + p * NB;
    for (int e = tid; e < NB * NB; e += 256) Lip[(int64_t)(e / NB) * lw + (e % NB)] = sLi[e / NB][e % NB];
    return;
  }
  // trailing update G_ij -= L_ip L_jp^T
  if (j == i) {
    for (int e = tid; e < NB * NB; e += 256) sLj[e / NB][e % NB] = sLi[e / NB][e % NB];
    __syncthreads();
  } else {
    times_inv_t(sLj, G + (int64_t)j * NB * lw + p * NB, lw, sI, sT);
  }
  double* Gij = G + (int64_t)i * NB * lw + j * NB;
  for (int e = tid; e < NB * NB; e += 256) {
    int r = e / NB, c = e % NB;
    double s = 0.0;
    for (int k = 0; k < NB; ++k) s += sLi[r][k] * sLj[c][k];
    Gij[(int64_t)r * lw + c] -= s;
  }
}

// ------------------------------------------------------------------ TRSM --
// Q[rows x lw] = X L^-T, 16 rows per block.  For each 32-column panel c:
//   W = X[:, c] - Q[:, <c] L[c, <c]^T      (K split over the 4 waves)
//   Q[:, c] = W Dinv_c^T
template <typename T>
__global__ __launch_bounds__(256) void trsm_kernel(int64_t rows, int lw, int ncols, const T* __restrict__ X,
                                                   int64_t ldx,
                                                   const double* __restrict__ L, const double* __restrict__ Dinv,
                                                   double* __restrict__ Q, int64_t ldq, int zero_to) {
  extern __shared__ double smem[];
  double* sQ = smem;                          // 16 x lw
  double* sW = smem + 16 * lw;                // 4 waves x 16 x 32 partials
  double* sX = sW + 4 * 16 * NB;              // 16 x 32 (W)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * 16;
  const int npanel = lw / NB;

  for (int c = 0; c < npanel; ++c) {
    const int c0 = c * NB;
    // partial products over t in [0, c0), K split across waves in steps of 4
    v4d acc0 = (v4d){0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
    for (int t0 = 4 * wave; t0 < c0; t0 += 16) {
      double a = sQ[li * lw + t0 + lk];
      double b0 = L[(int64_t)(c0 + li) * lw + t0 + lk];
      double b1 = L[(int64_t)(c0 + 16 + li) * lw + t0 + lk];
      acc0 = mfma_f64(a, b0, acc0);
      acc1 = mfma_f64(a, b1, acc1);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      sW[(wave * 16 + 4 * r + lk) * NB + li] = acc0[r];
      sW[(wave * 16 + 4 * r + lk) * NB + 16 + li] = acc1[r];
    }
    __syncthreads();
    for (int e = tid; e < 16 * NB; e += 256) {
      int r = e / NB, cc = e % NB;
      int64_t gr = row0 + r;
      double x = (gr < rows && c0 + cc < ncols) ? (double)X[gr * ldx + c0 + cc] : 0.0;
      double s = sW[(0 * 16 + r) * NB + cc];
      s += sW[(1 * 16 + r) * NB + cc];
      s += sW[(2 * 16 + r) * NB + cc];
      s += sW[(3 * 16 + r) * NB + cc];
      sX[r * NB + cc] = x - s;
    }
    __syncthreads();
    // Q[:, c] = W * Dinv_c^T  (waves 0, 1: one 16 x 16 output tile each)
    if (wave < 2) {
      const double* Dc = Dinv + (int64_t)c * NB * NB;
      v4d acc = (v4d){0.0, 0.0, 0.0, 0.0};
      for (int t0 = 0; t0 < NB; t0 += 4) {
        double a = sX[li * NB + t0 + lk];
        double b = Dc[(wave * 16 + li) * NB + t0 + lk];   // B[k][j] = Dinv[j][k]
        acc = mfma_f64(a, b, acc);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int rr = 4 * r + lk;
        sQ[rr * lw + c0 + wave * 16 + li] = acc[r];
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < 16 * zero_to; e += 256) {
    int r = e / zero_to, cc = e % zero_to;
    int64_t gr = row0 + r;
    if (gr < rows) Q[gr * ldq + cc] = cc < lw ? sQ[r * lw + cc] : 0.0;
  }
}

// ------------------------------------------------------------------ host --

struct CholWs {
  double *G, *L, *Dinv, *diag0, *part, *Q1;
  int nchunks;
  int64_t rows_per_chunk;
};

static void cholqr_layout(int64_t rows, int64_t l, int* lw_out, int* nchunks, int64_t* rpc) {
  int lw = (int)round_up(l, NB);
  int T = lw / NB;
  int ntri = T * (T + 1) / 2;
  int64_t nc = 512 / ntri;
  int64_t maxc = ceil_div(rows, 64);
  if (nc > maxc) nc = maxc;
  if (nc < 1) nc = 1;
  int64_t r = round_up(ceil_div(rows, nc), 16);
  nc = ceil_div(rows, r);
  if (nc < 1) nc = 1;
  *lw_out = lw;
  *nchunks = (int)nc;
  *rpc = r;
}

size_t cholqr2_workspace(int64_t rows, int64_t l) {
  int lw, nc;
  int64_t rpc;
  cholqr_layout(rows, l, &lw, &nc, &rpc);
  size_t sq = (size_t)lw * lw;
  size_t n = 2 * sq + (size_t)lw * NB + lw + (size_t)nc * sq + (size_t)rows * lw;
  return n * sizeof(double) + 256;
}

template <typename T>
static lramm_status one_pass(int64_t rows, int lw, int l_true, const T* X, int64_t ldx, double* Qout, int64_t ldq,
                             int zero_to, const CholWs& w, uint32_t* flags, hipStream_t s) {
  static bool attr_set = false;
  if (!attr_set) {
    LRAMM_HIP(hipFuncSetAttribute((const void*)trsm_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024));
    LRAMM_HIP(hipFuncSetAttribute((const void*)trsm_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024));
    attr_set = true;
  }
  const int Tn = lw / NB;
  const int ntri = Tn * (Tn + 1) / 2;
  hipLaunchKernelGGL((gram_kernel<T>), dim3(ntri, w.nchunks), dim3(256), 0, s, rows, lw, l_true, X, ldx, w.part,
                     w.rows_per_chunk);
  LRAMM_HIP(hipGetLastError());
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)ceil_div((int64_t)lw * lw, 256)), dim3(256), 0, s, lw,
                     w.nchunks, w.part, w.G, w.diag0);
  LRAMM_HIP(hipGetLastError());
  const double tol = 64.0 * (double)l_true * 0x1p-53;
  for (int p = 0; p < Tn; ++p) {
    int nb = (Tn - p) * (Tn - p + 1) / 2;
    hipLaunchKernelGGL(chol_step_kernel, dim3(nb), dim3(256), 0, s, lw, l_true, p, w.G, w.L, w.Dinv, w.diag0, tol,
                       flags);
    LRAMM_HIP(hipGetLastError());
  }
  size_t shm = (size_t)(16 * lw + 4 * 16 * NB + 16 * NB) * sizeof(double);
  hipLaunchKernelGGL((trsm_kernel<T>), dim3((unsigned)ceil_div(rows, 16)), dim3(256), shm, s, rows, lw, l_true, X,
                     ldx, w.L, w.Dinv, Qout, ldq, zero_to);
  LRAMM_HIP(hipGetLastError());
  return LRAMM_OK;
}

lramm_status launch_cholqr2(int64_t rows, int64_t l, const void* Y, int64_t ldy, int ytype, double* Q,
                            int64_t ldq, void* ws, size_t ws_bytes, uint32_t* flags, hipStream_t s) {
  if (rows == 0 || l == 0) return LRAMM_OK;
  int lw, nc;
  int64_t rpc;
  cholqr_layout(rows, l, &lw, &nc, &rpc);
  if (ws_bytes < cholqr2_workspace(rows, l)) return LRAMM_E_WORKSPACE;
  if ((size_t)(16 * lw + 5 * 16 * NB) * sizeof(double) > 160 * 1024) return LRAMM_E_UNSUPPORTED;
  uintptr_t base = round_up((int64_t)(uintptr_t)ws, 256);
  double* p = reinterpret_cast<double*>(base);
  size_t sq = (size_t)lw * lw;
  CholWs w;
  w.G = p;
  p += sq;
  w.L = p;
  p += sq;
  w.Dinv = p;
  p += (size_t)lw * NB;
  w.diag0 = p;
  p += lw;
  w.part = p;
  p += (size_t)nc * sq;
  w.Q1 = p;
  w.nchunks = nc;
  w.rows_per_chunk = rpc;
  // pass 1 on Y (columns at or past l are never read), pass 2 on Q1
  if (ytype == LRAMM_F32) {
    LRAMM_TRY(one_pass<float>(rows, lw, (int)l, (const float*)Y, ldy, w.Q1, lw, lw, w, flags, s));
  } else if (ytype == LRAMM_F64) {
    LRAMM_TRY(one_pass<double>(rows, lw, (int)l, (const double*)Y, ldy, w.Q1, lw, lw, w, flags, s));
  } else {
    return LRAMM_E_UNSUPPORTED;
  }
  int zero_to = (int)ldq;
  LRAMM_TRY(one_pass<double>(rows, lw, (int)l, w.Q1, lw, Q, ldq, zero_to, w, flags, s));
  return LRAMM_OK;
}

}  // namespace lramm
