// Kernels of the two-sided form (paper Sec. 3.2, Alg. 3) that the one-sided
// path does not have: the small SVD of Alg. 1 (B~ = U' S V^T for the l x k
// projection B~ = Q^T A) and the floating-point factor products around it.
//
// The small SVD goes through the l x l Gram matrix G = B~ B~^T (FP64): its
// eigenvectors are the left singular vectors U', its eigenvalues the squared
// singular values.  G is diagonalised by cyclic Jacobi rotations (Golub & Van
// Loan, Matrix Computations, Sec. 8.5) in one workgroup with G in LDS, l/2
// disjoint rotations at a time in round-robin (tournament) order.
#include "common.hpp"

namespace lramm {

// --------------------------------------------------------------- row Gram --
// G[i][j] = sum_t X[i][t] X[j][t] for the rows of X (rows x cols, FP32 or
// FP64, ldx), in FP64 with a fixed summation order; G is n x n (ldg = n),
// rows and columns at or past `rows` are zero.  One workgroup per 16 x 16
// tile of the lower triangle, written to both triangles.
template <typename T>
__global__ __launch_bounds__(256) void rowgram_kernel(int rows, int cols, const T* __restrict__ X, int64_t ldx,
                                                      double* __restrict__ G, int n) {
  __shared__ double xi[16][65], xj[16][65];
  // tile (ti, tj), ti >= tj, from the linear index of the lower triangle
  int t = blockIdx.x, ti = 0;
  while (t > ti) {
    t -= ti + 1;
    ++ti;
  }
  const int tj = t;
  const int tid = threadIdx.x, li = tid >> 4, lj = tid & 15;
  double acc = 0.0;
  for (int c0 = 0; c0 < cols; c0 += 64) {
    for (int e = tid; e < 16 * 64; e += 256) {
      const int r = e >> 6, c = e & 63;
      const int gi = ti * 16 + r, gj = tj * 16 + r, gc = c0 + c;
      xi[r][c] = (gi < rows && gc < cols) ? (double)X[(int64_t)gi * ldx + gc] : 0.0;
      xj[r][c] = (gj < rows && gc < cols) ? (double)X[(int64_t)gj * ldx + gc] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int c = 0; c < 64; ++c) acc = fma(xi[li][c], xj[lj][c], acc);
    __syncthreads();
  }
  const int gi = ti * 16 + li, gj = tj * 16 + lj;
  if (gi < n && gj < n) {
    G[(int64_t)gi * n + gj] = acc;
    G[(int64_t)gj * n + gi] = acc;
  }
}

// ------------------------------------------------------------ Jacobi eig --
constexpr int kJacMax = 128;                 // largest (even) order held in LDS
constexpr int kJacPitch = kJacMax + 1;

// Eigen-decomposition of the symmetric n x n G (n even, <= kJacMax) and the
// rank-r factors of the small SVD:
//   Up (n x r): eigenvectors of the r largest eigenvalues, largest first,
//       each signed so that its largest-magnitude entry (the first on a tie)
//       is positive;
//   S (r): sqrt of those eigenvalues (0 for a negative rounding residue);
//   UpS = Up diag(S), UpSinv = Up diag(1/S) (0 where S == 0).
// V (n x n, global) holds the accumulated rotations.  A pair (p, q) is
// rotated while |g_pq| > 2^-53 sqrt(|g_pp g_qq|); sweeps stop when none is,
// or after max_sweeps (then *flags gets LRAMM_FLAG_BREAKDOWN).
__global__ __launch_bounds__(512) void jacobi_eig_kernel(int n, int r, const double* __restrict__ G,
                                                         double* __restrict__ V, double* __restrict__ Up,
                                                         double* __restrict__ S, double* __restrict__ UpS,
                                                         double* __restrict__ UpSinv, int max_sweeps,
                                                         uint32_t* flags) {
  __shared__ double a[kJacMax * kJacPitch];
  __shared__ double cs[kJacMax / 2][2];
  __shared__ int pr[kJacMax / 2][2];
  __shared__ int pos[kJacMax];
  __shared__ int rank[kJacMax];
  __shared__ int rotated;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < n * n; e += nt) {
    const int i = e / n, j = e % n;
    a[i * kJacPitch + j] = G[e];
    V[e] = i == j ? 1.0 : 0.0;
  }
  for (int i = tid; i < n; i += nt) pos[i] = i;
  const int half = n / 2;
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int step = 0; step < n - 1; ++step) {
      // the rotations of this step: pairs (pos[i], pos[n - 1 - i])
      if (tid < half) {
        int p = pos[tid], q = pos[n - 1 - tid];
        if (p > q) {
          const int tmp = p;
          p = q;
          q = tmp;
        }
        const double app = a[p * kJacPitch + p], aqq = a[q * kJacPitch + q], apq = a[p * kJacPitch + q];
        double c = 1.0, s = 0.0;
        if (apq != 0.0 && fabs(apq) > 0x1p-53 * sqrt(fabs(app) * fabs(aqq))) {
          // symmetric 2 x 2 Schur decomposition: (J^T A J)_pq = 0 with
          // J_pp = J_qq = c, J_pq = s, J_qp = -s
          const double tau = (aqq - app) / (2.0 * apq);
          const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + tt * tt);
          s = tt * c;
          rotated = 1;
        }
        cs[tid][0] = c;
        cs[tid][1] = s;
        pr[tid][0] = p;
        pr[tid][1] = q;
      }
      __syncthreads();
      // rows: A <- J^T A
      for (int e = tid; e < half * n; e += nt) {
        const int i = e / n, j = e % n;
        const double c = cs[i][0], s = cs[i][1];
        if (s == 0.0) continue;
        const int p = pr[i][0], q = pr[i][1];
        const double ap = a[p * kJacPitch + j], aq = a[q * kJacPitch + j];
        a[p * kJacPitch + j] = c * ap - s * aq;
        a[q * kJacPitch + j] = s * ap + c * aq;
      }
      __syncthreads();
      // columns: A <- A J, V <- V J
      for (int e = tid; e < half * n; e += nt) {
        const int i = e / n, j = e % n;
        const double c = cs[i][0], s = cs[i][1];
        if (s == 0.0) continue;
        const int p = pr[i][0], q = pr[i][1];
        const double ap = a[j * kJacPitch + p], aq = a[j * kJacPitch + q];
        a[j * kJacPitch + p] = c * ap - s * aq;
        a[j * kJacPitch + q] = s * ap + c * aq;
        const double vp = V[(int64_t)j * n + p], vq = V[(int64_t)j * n + q];
        V[(int64_t)j * n + p] = c * vp - s * vq;
        V[(int64_t)j * n + q] = s * vp + c * vq;
      }
      // next pairing: position 0 stays, the others rotate by one
      int nxt = 0;
      if (tid < n) nxt = tid == 0 ? pos[0] : pos[tid == 1 ? n - 1 : tid - 1];
      __syncthreads();
      if (tid < n) pos[tid] = nxt;
      __syncthreads();
    }
    // every thread reads the flag before thread 0 may clear it for the next sweep
    const int rot = rotated;
    __syncthreads();
    if (!rot) break;
  }
  if (sweep == max_sweeps && tid == 0 && flags) atomicOr(flags, LRAMM_FLAG_BREAKDOWN);
  // order: rank of eigenvalue i = number of larger ones (earlier index on ties)
  for (int i = tid; i < n; i += nt) {
    const double di = a[i * kJacPitch + i];
    int rk = 0;
    for (int j = 0; j < n; ++j) {
      const double dj = a[j * kJacPitch + j];
      rk += (dj > di || (dj == di && j < i)) ? 1 : 0;
    }
    rank[i] = rk;
  }
  __syncthreads();
  // the first r: sign rule, singular values, scaled copies
  for (int i = tid; i < n; i += nt) {
    const int c = rank[i];
    if (c >= r) continue;
    int arg = 0;
    double best = -1.0;
    for (int j = 0; j < n; ++j) {
      const double v = fabs(V[(int64_t)j * n + i]);
      if (v > best) {
        best = v;
        arg = j;
      }
    }
    const double sg = V[(int64_t)arg * n + i] < 0.0 ? -1.0 : 1.0;
    const double lam = a[i * kJacPitch + i];
    const double sv = lam > 0.0 ? sqrt(lam) : 0.0;
    S[c] = sv;
    for (int j = 0; j < n; ++j) {
      const double u = sg * V[(int64_t)j * n + i];
      Up[(int64_t)j * r + c] = u;
      UpS[(int64_t)j * r + c] = u * sv;
      UpSinv[(int64_t)j * r + c] = sv > 0.0 ? u / sv : 0.0;
    }
  }
}

// ------------------------------------------- FP64-accumulated products --
// C[M x N] (binary32, rounded once) = op(A) op(B) with FP64 products and
// sums, for the small factor products of the two-sided form.  Operand
// layouts as launch_gemm_f32 (a_kmajor / b_kmajor), types FP32 or FP64.
template <typename TA, typename TB>
__global__ __launch_bounds__(256) void gemm_f64acc_kernel(int M, int N, int K, const TA* __restrict__ A,
                                                          int64_t lda, int a_kmajor, const TB* __restrict__ B,
                                                          int64_t ldb, int b_kmajor, float* __restrict__ C,
                                                          int64_t ldc) {
  __shared__ double sa[16][17], sb[16][17];
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
  const int row = blockIdx.y * 16 + ty, col = blockIdx.x * 16 + tx;
  double acc = 0.0;
  for (int k0 = 0; k0 < K; k0 += 16) {
    {
      const int gi = blockIdx.y * 16 + ty, gk = k0 + tx;   // A[gi][gk]
      double v = 0.0;
      if (gi < M && gk < K) v = (double)(a_kmajor ? A[(int64_t)gk * lda + gi] : A[(int64_t)gi * lda + gk]);
      sa[ty][tx] = v;
      const int gk2 = k0 + ty, gj = blockIdx.x * 16 + tx;   // B[gk2][gj]
      double w = 0.0;
      if (gk2 < K && gj < N) w = (double)(b_kmajor ? B[(int64_t)gk2 * ldb + gj] : B[(int64_t)gj * ldb + gk2]);
      sb[ty][tx] = w;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) acc = fma(sa[ty][kk], sb[kk][tx], acc);
    __syncthreads();
  }
  if (row < M && col < N) C[(int64_t)row * ldc + col] = (float)acc;
}

// ------------------------------------------------------------------ host --

lramm_status launch_rowgram(int rows, int cols, const void* X, int64_t ldx, int xtype, double* G, int n,
                            hipStream_t s) {
  const int T = n / 16 + (n % 16 ? 1 : 0);
  const dim3 grid((unsigned)(T * (T + 1) / 2));
  if (xtype == LRAMM_F32)
    hipLaunchKernelGGL(rowgram_kernel<float>, grid, dim3(256), 0, s, rows, cols, (const float*)X, ldx, G, n);
  else if (xtype == LRAMM_F64)
    hipLaunchKernelGGL(rowgram_kernel<double>, grid, dim3(256), 0, s, rows, cols, (const double*)X, ldx, G, n);
  else
    return LRAMM_E_UNSUPPORTED;
  LRAMM_HIP(hipGetLastError());
  return LRAMM_OK;
}

int jacobi_max_order() { return kJacMax; }

lramm_status launch_jacobi_svd(int n, int r, const double* G, double* V, double* Up, double* S, double* UpS,
                               double* UpSinv, uint32_t* flags, hipStream_t s) {
  if (n < 2 || n % 2 || n > kJacMax || r < 1 || r > n) return LRAMM_E_UNSUPPORTED;
  hipLaunchKernelGGL(jacobi_eig_kernel, dim3(1), dim3(512), 0, s, n, r, G, V, Up, S, UpS, UpSinv, 60, flags);
  LRAMM_HIP(hipGetLastError());
  return LRAMM_OK;
}

lramm_status launch_gemm_f64acc(int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, int a_kmajor,
                                int a_type, const void* B, int64_t ldb, int b_kmajor, int b_type, float* C,
                                int64_t ldc, hipStream_t s) {
  if (M == 0 || N == 0) return LRAMM_OK;
  const dim3 grid((unsigned)ceil_div(N, 16), (unsigned)ceil_div(M, 16));
#define F64ACC(TA, TB)                                                                                           \
  hipLaunchKernelGGL((gemm_f64acc_kernel<TA, TB>), grid, dim3(256), 0, s, (int)M, (int)N, (int)K,             \
                     (const TA*)A, lda, a_kmajor, (const TB*)B, ldb, b_kmajor, C, ldc)
  if (a_type == LRAMM_F64 && b_type == LRAMM_F64) F64ACC(double, double);
  else if (a_type == LRAMM_F64 && b_type == LRAMM_F32) F64ACC(double, float);
  else if (a_type == LRAMM_F32 && b_type == LRAMM_F64) F64ACC(float, double);
  else if (a_type == LRAMM_F32 && b_type == LRAMM_F32) F64ACC(float, float);
  else return LRAMM_E_UNSUPPORTED;
#undef F64ACC
  LRAMM_HIP(hipGetLastError());
  return LRAMM_OK;
}

}  // namespace lramm
