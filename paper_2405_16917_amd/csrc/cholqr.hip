// CholeskyQR2 in FP64 for the range finder's orthonormalisation (paper
// Sec. 2.2: a matrix Q with orthonormal columns spanning the sketch).  For a
// rows x l matrix Y (FP32 or FP64):
//
//   G1 = Y^T Y (FP64)                 Gram, split over row chunks, summed in
//                                      a fixed order (deterministic)
//   G1 = L L^T, X = L^-1              blocked right-looking Cholesky, 32 x 32
//                                      tiles, one launch per panel; the block
//                                      inverse is formed in the same launches
//   Q1 = Y X^T                         FP64 GEMM
//   G2 = Q1^T Q1 = I + E,  Q = Q1 (chol(G2))^-T   second pass, restoring the
//                                      orthogonality lost to cond(Y)^2 u (see
//                                      the second-pass section)
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
// G (lower tiles) = sum over chunks in order; diag0 = diag(G).
__global__ __launch_bounds__(256) void gram_reduce_kernel(int lw, int nchunks, const double* __restrict__ part,
                                                          double* __restrict__ G, double* __restrict__ diag0,
                                                          uint32_t* gate) {
  int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e == 0) *gate = 0u;   // second-pass gate of this orthonormalisation
  if (e >= (int64_t)lw * lw) return;
  int i = (int)(e / lw), j = (int)(e % lw);
  if ((i / NB) < (j / NB)) return;   // upper tiles are never read
  double s = 0.0;
  for (int c = 0; c < nchunks; ++c) s += part[(int64_t)c * lw * lw + e];
  G[e] = s;
  if (i == j) diag0[i] = s;
}

// ---------------------------------------------------- FP64 tile GEMM engine --
// A 64 x 64 output tile on 4 wavefronts (2 x 2, each 32 x 32 = 2 x 2 MFMA
// 16 x 16 sub-tiles) accumulating sum_k A(k, m) B(k, n) over [kbeg, kend).
// K advances in stages of 32, double-buffered in LDS, both operands stored
// K-major ([k][m]) so that an MFMA operand read is 16 consecutive doubles.
// Operands come from functors fa(k, m, valid), fb(k, n, valid) returning
// doubles: they load unconditionally from an in-range address and return zero
// when the element is outside the operand (no branches around the loads, so a
// stage's loads are all in flight together).  AK / BK: the operand is
// contiguous along k in memory (threads then walk k first, keeping global
// loads coalesced).
constexpr int FT = 64, FK = 32, FP = FT + 2;
struct F64Smem {
  double a[2][FK][FP];
  double b[2][FK][FP];
};

template <bool AK, bool BK, class FA, class FB>
__device__ __forceinline__ void f64_gemm_tile(const FA& fa, const FB& fb, int kbeg, int kend, v4d acc[2][2],
                                              F64Smem& sm) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1, li = lane & 15, lk = lane >> 4;
  double ra[8], rb[8];
  auto gload = [&](int kb) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = tid + 256 * i;
      const int ka = AK ? e % FK : e / FT, ma = AK ? e / FK : e % FT;
      const int kbb = BK ? e % FK : e / FT, nb = BK ? e / FK : e % FT;
      const bool va = kb + ka < kend, vb = kb + kbb < kend;
      ra[i] = fa(va ? kb + ka : kbeg, ma, va);
      rb[i] = fb(vb ? kb + kbb : kbeg, nb, vb);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = tid + 256 * i;
      const int ka = AK ? e % FK : e / FT, ma = AK ? e / FK : e % FT;
      const int kbb = BK ? e % FK : e / FT, nb = BK ? e / FK : e % FT;
      sm.a[buf][ka][ma] = ra[i];
      sm.b[buf][kbb][nb] = rb[i];
    }
  };
  const int nst = kend > kbeg ? (kend - kbeg + FK - 1) / FK : 0;
  if (nst == 0) return;
  gload(kbeg);
  sstore(0);
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int buf = st & 1;
    const bool more = st + 1 < nst;
    if (more) gload(kbeg + (st + 1) * FK);
#pragma unroll
    for (int kk = 0; kk < FK; kk += 4) {
      double av[2], bv[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        av[q] = sm.a[buf][kk + lk][wm * 32 + 16 * q + li];
        bv[q] = sm.b[buf][kk + lk][wn * 32 + 16 * q + li];
      }
#pragma unroll
      for (int si = 0; si < 2; ++si)
#pragma unroll
        for (int sj = 0; sj < 2; ++sj) acc[si][sj] = mfma_f64(av[si], bv[sj], acc[si][sj]);
    }
    if (more) sstore(buf ^ 1);
    __syncthreads();
  }
}

// Output coordinates of accumulator element (si, sj, r) of this lane.
__device__ __forceinline__ int f64_row(int si, int r) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return (wave >> 1) * 32 + 16 * si + 4 * r + (lane >> 4);
}
__device__ __forceinline__ int f64_col(int sj) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return (wave & 1) * 32 + 16 * sj + (lane & 15);
}

// Gram of a row chunk, 64 x 64 tiles (ta, tb), ta >= tb:
// out[a][b] = sum_{r in chunk} X[r][a] X[r][b]; columns >= ncols read as zero.
template <typename T>
__global__ __launch_bounds__(256, 2) void gram64_kernel(int64_t rows, int lw, int ncols, const T* __restrict__ X,
                                                        int64_t ldx, double* __restrict__ part,
                                                        int64_t rows_per_chunk) {
  __shared__ F64Smem sm;
  int t = blockIdx.x, ta = 0;
  while (t > ta) {
    t -= ta + 1;
    ++ta;
  }
  const int tb = t, a0 = ta * FT, b0 = tb * FT;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_chunk;
  const int64_t r1 = r0 + rows_per_chunk < rows ? r0 + rows_per_chunk : rows;
  auto fa = [&](int k, int m, bool v) -> double {
    const bool ok = v && a0 + m < ncols;
    const double x = (double)X[(r0 + k) * ldx + (ok ? a0 + m : 0)];
    return ok ? x : 0.0;
  };
  auto fb = [&](int k, int n, bool v) -> double {
    const bool ok = v && b0 + n < ncols;
    const double x = (double)X[(r0 + k) * ldx + (ok ? b0 + n : 0)];
    return ok ? x : 0.0;
  };
  v4d acc[2][2] = {{{0, 0, 0, 0}, {0, 0, 0, 0}}, {{0, 0, 0, 0}, {0, 0, 0, 0}}};
  f64_gemm_tile<false, false>(fa, fb, 0, (int)(r1 - r0), acc, sm);
  double* out = part + (int64_t)blockIdx.y * lw * lw;
#pragma unroll
  for (int si = 0; si < 2; ++si)
#pragma unroll
    for (int sj = 0; sj < 2; ++sj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = a0 + f64_row(si, r), j = b0 + f64_col(sj);
        if (i < lw && j < lw) out[(int64_t)i * lw + j] = acc[si][sj][r];
      }
}

// Q[r][c] = [Q1[r][c] +] sum_{k <= c} X[r][k] B(k, c) for the two solve
// products of CholeskyQR, 64 x 64 output tiles over (rows, lw):
//   APPLY == false:  B(k, c) = Linv[c][k]  (Q1 = X L^-T, X = Y in FP32/FP64)
//   APPLY == true :  B(k, c) = M[k][c]     (Q = Q1 + Q1 M, X = Q1)
// Columns in [lw, zero_to) of Q are written as zero.  When gate is non-null
// the kernel is skipped if (*gate & gate_mask) is set.
template <typename T, bool APPLY>
__global__ __launch_bounds__(256, 2) void solve_gemm_kernel(int64_t rows, int lw, int ncols, const T* __restrict__ X,
                                                            int64_t ldx, const double* __restrict__ B,
                                                            double* __restrict__ Q, int64_t ldq, int zero_to,
                                                            const uint32_t* gate, uint32_t gate_mask) {
  if (gate && (*gate & gate_mask)) return;
  __shared__ F64Smem sm;
  const int64_t r0 = (int64_t)blockIdx.x * FT;
  const int c0 = blockIdx.y * FT;
  if (c0 >= lw) {
    for (int e = threadIdx.x; e < FT * FT; e += 256) {
      const int64_t r = r0 + e / FT;
      const int c = c0 + e % FT;
      if (r < rows && c < zero_to) Q[r * ldq + c] = 0.0;
    }
    return;
  }
  auto fa = [&](int k, int m, bool v) -> double {
    const int64_t r = r0 + m;
    const bool ok = v && r < rows && k < ncols;
    const double x = (double)X[ok ? r * ldx + k : 0];
    return ok ? x : 0.0;
  };
  auto fb = [&](int k, int n, bool v) -> double {
    // both factors are triangular (Linv lower, M upper): B(k, c) = 0 for k > c,
    // and the blocks beyond the diagonal are never written, so never read them
    const int c = c0 + n;
    const bool ok = v && c < lw && k <= c;
    const double x = B[ok ? (APPLY ? (int64_t)k * lw + c : (int64_t)c * lw + k) : 0];
    return ok ? x : 0.0;
  };
  v4d acc[2][2] = {{{0, 0, 0, 0}, {0, 0, 0, 0}}, {{0, 0, 0, 0}, {0, 0, 0, 0}}};
  const int kend = c0 + FT < lw ? c0 + FT : lw;      // triangular: terms with k > c vanish
  if constexpr (APPLY) {
    f64_gemm_tile<true, false>(fa, fb, 0, kend, acc, sm);
  } else {
    f64_gemm_tile<true, true>(fa, fb, 0, kend, acc, sm);
  }
#pragma unroll
  for (int si = 0; si < 2; ++si)
#pragma unroll
    for (int sj = 0; sj < 2; ++sj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + f64_row(si, r);
        const int c = c0 + f64_col(sj);
        if (row < rows && c < zero_to) {
          double v = acc[si][sj][r];
          if constexpr (APPLY) v += (double)X[row * ldx + c];
          Q[row * ldq + c] = c < lw ? v : 0.0;
        }
      }
}

// -------------------------------------------------------------- Cholesky --
// Blocked right-looking Cholesky with 32 x 32 tiles.  Launch p updates every
// trailing tile (i, j), p < j <= i, with the panel p; the workgroup that
// finishes tile (p+1, p+1) then factors it, so the next launch finds L and
// its inverse for that diagonal block ready.  A diagonal block is factored by
// one wavefront with rows in registers (lane i owns row i) and cross-lane
// broadcasts by readlane, without barriers.

__device__ __forceinline__ double lane_bcast(double v, int lane) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Order LDS accesses of one wavefront (compiler barrier + LDS wait).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// One wavefront factors the 32 x 32 block S (LDS, pitch NB + 1) into L
// (written to Lout, row pitch ldl, zeros above the diagonal) and writes the
// inverse of L to Iout (32 x 32, row-major).  Lane i keeps row i in
// registers; after each column is scaled it is published in LDS (scratch)
// and read back by every lane as uniform-address (broadcast) loads.
// scratch: NB * (NB + 1) + 2 NB doubles of LDS private to this wavefront.
__device__ __attribute__((always_inline)) inline void factor_block_wave(const double* S, double* scratch,
                                                                        const double* diag0, int col0, int l_true,
                                                                        double tol, uint32_t* flags, double* Lout,
                                                                        int64_t ldl, double* Iout) {
  const int lane = threadIdx.x & 63;
  const int row = lane & 31;
  double* Ls = scratch;                      // L, pitch NB + 1
  double* colbuf = scratch + NB * (NB + 1);  // two column slots (double-buffered)
  // pivot thresholds, loaded once (lane j: column col0 + j; negative = padding column)
  const double thr = col0 + row < l_true ? tol * diag0[col0 + row] : -1.0;
  double a[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) a[k] = S[row * (NB + 1) + k];
  double inv[NB];
  uint32_t bad = 0;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const double d = lane_bcast(a[j], j);
    const double tj = lane_bcast(thr, j);
    double piv = 0.0, iv = 0.0;
    if (tj >= 0.0) {
      if (d > tj && d > 0.0) {
        // 1/sqrt(d): hardware estimate refined by two Newton steps (quadratic
        // convergence from ~2^-23 to full precision); piv = d / sqrt(d)
        double y = __builtin_amdgcn_rsq(d);
        y = y * fma(-0.5 * d * y, y, 1.5);
        y = y * fma(-0.5 * d * y, y, 1.5);
        iv = y;
        piv = d * y;
      } else {
        bad |= (d < -tj || d != d) ? (LRAMM_FLAG_BREAKDOWN | LRAMM_FLAG_SQRTNEG) : LRAMM_FLAG_BREAKDOWN;
      }
    }
    inv[j] = iv;
    a[j] = row > j ? a[j] * iv : (row == j ? piv : a[j]);
    double* col = colbuf + (j & 1) * NB;
    if (lane < NB) col[lane] = a[j];
    wave_lds_sync();
#pragma unroll
    for (int k = j + 1; k < NB; ++k) a[k] = fma(-a[j], col[k], a[k]);
  }
  if (lane < NB) {
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const double v = k <= row ? a[k] : 0.0;
      Ls[row * (NB + 1) + k] = v;
      Lout[(int64_t)row * ldl + k] = v;
    }
  }
  wave_lds_sync();
  // inverse, one column per lane: X[i][c] = (delta_ic - sum_t L[i][t] X[t][c]) / L[i][i],
  // the sum split over four independent partial sums
  double x[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    double p0 = row == i ? 1.0 : 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
#pragma unroll
    for (int t = 0; t < i; t += 4) {
      p0 = fma(-Ls[i * (NB + 1) + t], x[t], p0);
      if (t + 1 < i) p1 = fma(-Ls[i * (NB + 1) + t + 1], x[t + 1], p1);
      if (t + 2 < i) p2 = fma(-Ls[i * (NB + 1) + t + 2], x[t + 2], p2);
      if (t + 3 < i) p3 = fma(-Ls[i * (NB + 1) + t + 3], x[t + 3], p3);
    }
    x[i] = ((p0 + p1) + (p2 + p3)) * inv[i];
  }
  if (lane < NB) {
#pragma unroll
    for (int i = 0; i < NB; ++i) Iout[i * NB + row] = x[i];
  }
  if (lane == 0 && bad && flags) atomicOr(flags, bad);
}

// First diagonal block (one wavefront).
__global__ __launch_bounds__(64) void chol_first_kernel(int lw, int l_true, const double* __restrict__ G,
                                                        double* __restrict__ L, double* __restrict__ Dinv,
                                                        const double* __restrict__ diag0, double tol,
                                                        uint32_t* flags) {
  __shared__ double sS[NB * (NB + 1)];
  __shared__ double scratch[NB * (NB + 1) + 2 * NB];
  for (int e = threadIdx.x; e < NB * NB; e += 64) sS[(e / NB) * (NB + 1) + e % NB] = G[(int64_t)(e / NB) * lw + e % NB];
  __syncthreads();
  factor_block_wave(sS, scratch, diag0, 0, l_true, tol, flags, L, lw, Dinv);
}

// 32 x 32 tile product on 4 wavefronts: out = X Y^T (X, Y in LDS, pitch
// NB + 1); wave w computes the 16 x 16 sub-tile (w / 2, w % 2).
__device__ __forceinline__ v4d tile_xyt(const double (*X)[NB + 1], const double (*Y)[NB + 1], int wave, int li,
                                        int lk) {
  const int si = wave >> 1, sj = wave & 1;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < NB; kk += 4) acc = mfma_f64(X[16 * si + li][kk + lk], Y[16 * sj + li][kk + lk], acc);
  return acc;
}

// Block (p, j), j <= p, of X = L^-1 (lower triangular, 32 x 32 blocks):
//   X_pp = Dinv_p;  X_pj = -Dinv_p sum_{t=j}^{p-1} L_pt X_tj  (j < p).
// Needs row blocks 0..p-1 of X and row block p of L.  One workgroup.
__device__ void inverse_block(int lw, int p, int j, const double* __restrict__ L, const double* __restrict__ Dinv,
                              double* __restrict__ Xinv, double (*sS)[NB + 1]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4, si = wave >> 1, sj = wave & 1;
  const double* Dp = Dinv + (int64_t)p * NB * NB;
  double* Xpj = Xinv + (int64_t)p * NB * lw + j * NB;
  if (j == p) {
    for (int e = tid; e < NB * NB; e += 256) Xpj[(int64_t)(e / NB) * lw + e % NB] = Dp[e];
    return;
  }
  // S = sum_t L_pt X_tj  (sub-tile (si, sj) per wave)
  v4d acc = {0, 0, 0, 0};
  for (int t = j; t < p; ++t) {
    const double* Lpt = L + (int64_t)p * NB * lw + t * NB;
    const double* Xtj = Xinv + (int64_t)t * NB * lw + j * NB;
    double av[8], bv[8];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      av[kk] = Lpt[(int64_t)(16 * si + li) * lw + 4 * kk + lk];
      bv[kk] = Xtj[(int64_t)(4 * kk + lk) * lw + 16 * sj + li];
    }
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) acc = mfma_f64(av[kk], bv[kk], acc);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) sS[16 * si + 4 * r + lk][16 * sj + li] = acc[r];
  __syncthreads();
  // X_pj = -Dinv_p S
  v4d out = {0, 0, 0, 0};
#pragma unroll
  for (int kk = 0; kk < NB; kk += 4) out = mfma_f64(Dp[(16 * si + li) * NB + kk + lk], sS[kk + lk][16 * sj + li], out);
#pragma unroll
  for (int r = 0; r < 4; ++r) Xpj[(int64_t)(16 * si + 4 * r + lk) * lw + 16 * sj + li] = -out[r];
}

// Last row block of X = L^-1 (after the last panel launch).
__global__ __launch_bounds__(256) void inverse_row_kernel(int lw, int p, const double* __restrict__ L,
                                                          const double* __restrict__ Dinv, double* __restrict__ Xinv,
                                                          const uint32_t* gate, uint32_t gate_mask) {
  if (gate && !(*gate & gate_mask)) return;
  __shared__ double sS[NB][NB + 1];
  inverse_block(lw, p, blockIdx.x, L, Dinv, Xinv, sS);
}

// Launch p (0 <= p < T - 1): workgroup b owns trailing tile (i, j),
// p < j <= i < T.  It forms L_ip = G_ip Dinv_p^T and L_jp, writes L_ip when
// j == p + 1, updates G_ij -= L_ip L_jp^T, and the owner of (p+1, p+1)
// factors that block.  p + 1 further workgroups form row block p of
// X = L^-1, which is ready because row blocks < p of X and row block p of L
// were finished by earlier launches.
__global__ __launch_bounds__(256) void chol_panel_kernel(int lw, int l_true, int p, double* __restrict__ G,
                                                         double* __restrict__ L, double* __restrict__ Dinv,
                                                         double* __restrict__ Xinv, const double* __restrict__ diag0,
                                                         double tol, uint32_t* flags) {
  __shared__ double sD[NB][NB + 1];
  __shared__ double sGi[NB][NB + 1], sGj[NB][NB + 1];
  __shared__ double sLi[NB][NB + 1], sLj[NB][NB + 1];
  __shared__ double sS[NB][NB + 1];
  __shared__ double scratch[NB * (NB + 1) + 2 * NB];
  const int T = lw / NB;
  const int ntrail = (T - p - 1) * (T - p) / 2;
  if ((int)blockIdx.x >= ntrail) {   // inverse row block p (blocks past the trailing tiles)
    inverse_block(lw, p, blockIdx.x - ntrail, L, Dinv, Xinv, sS);
    return;
  }
  int t = blockIdx.x, di = 0;
  while (t > di) {
    t -= di + 1;
    ++di;
  }
  const int i = p + 1 + di, j = p + 1 + t;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const double* Dp = Dinv + (int64_t)p * NB * NB;
  const double* Gip = G + (int64_t)i * NB * lw + p * NB;
  const double* Gjp = G + (int64_t)j * NB * lw + p * NB;
  for (int e = tid; e < NB * NB; e += 256) {
    const int r = e / NB, c = e % NB;
    sD[r][c] = Dp[e];
    sGi[r][c] = Gip[(int64_t)r * lw + c];
    if (j != i) sGj[r][c] = Gjp[(int64_t)r * lw + c];
  }
  __syncthreads();
  {
    v4d li_acc = tile_xyt(sGi, sD, wave, li, lk);
#pragma unroll
    for (int r = 0; r < 4; ++r) sLi[16 * (wave >> 1) + 4 * r + lk][16 * (wave & 1) + li] = li_acc[r];
    if (j != i) {
      v4d lj_acc = tile_xyt(sGj, sD, wave, li, lk);
#pragma unroll
      for (int r = 0; r < 4; ++r) sLj[16 * (wave >> 1) + 4 * r + lk][16 * (wave & 1) + li] = lj_acc[r];
    }
  }
  __syncthreads();
  if (j == p + 1) {
    double* Lip = L + (int64_t)i * NB * lw + p * NB;
    for (int e = tid; e < NB * NB; e += 256) Lip[(int64_t)(e / NB) * lw + e % NB] = sLi[e / NB][e % NB];
  }
  const v4d upd = tile_xyt(sLi, j != i ? sLj : sLi, wave, li, lk);
  double* Gij = G + (int64_t)i * NB * lw + j * NB;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int rr = 16 * (wave >> 1) + 4 * r + lk, cc = 16 * (wave & 1) + li;
    const double v = Gij[(int64_t)rr * lw + cc] - upd[r];
    Gij[(int64_t)rr * lw + cc] = v;
    sS[rr][cc] = v;
  }
  if (i == p + 1 && j == p + 1) {
    __syncthreads();
    if (wave == 0)
      factor_block_wave(&sS[0][0], scratch, diag0, (p + 1) * NB, l_true, tol, flags,
                        L + (int64_t)(p + 1) * NB * lw + (p + 1) * NB, lw, Dinv + (int64_t)(p + 1) * NB * NB);
  }
}

// One wavefront: acc[si][sj] (16 x 16 sub-tiles) += X[32 x 32] Y[32 x 32]^T,
// X and Y row-major in global memory (L2-resident), K = 32.
__device__ __forceinline__ void wave_tile_xyt(const double* X, int64_t ldx, const double* Y, int64_t ldy, int li,
                                              int lk, v4d acc[2][2]) {
  double xv[2][8], yv[2][8];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      xv[s][kk] = X[(int64_t)(16 * s + li) * ldx + 4 * kk + lk];
      yv[s][kk] = Y[(int64_t)(16 * s + li) * ldy + 4 * kk + lk];
    }
#pragma unroll
  for (int kk = 0; kk < 8; ++kk)
#pragma unroll
    for (int si = 0; si < 2; ++si)
#pragma unroll
      for (int sj = 0; sj < 2; ++sj) acc[si][sj] = mfma_f64(xv[si][kk], yv[sj][kk], acc[si][sj]);
}

// The whole blocked Cholesky in one workgroup (no launches between panels).
// When gate is non-null the kernel does nothing unless (*gate & gate_mask).
__global__ __launch_bounds__(256) void chol_fused_kernel(int lw, int l_true, double* __restrict__ G,
                                                         double* __restrict__ L, double* __restrict__ Dinv,
                                                         const double* __restrict__ diag0, double tol,
                                                         uint32_t* flags, const uint32_t* gate, uint32_t gate_mask) {
  if (gate && !(*gate & gate_mask)) return;
  __shared__ double sS[NB][NB + 1];
  __shared__ double scratch[NB * (NB + 1) + 2 * NB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int T = lw / NB;
  for (int p = 0; p < T; ++p) {
    const double* Gpp = G + (int64_t)p * NB * lw + p * NB;
    for (int e = tid; e < NB * NB; e += 256) sS[e / NB][e % NB] = Gpp[(int64_t)(e / NB) * lw + e % NB];
    __syncthreads();
    double* Dp = Dinv + (int64_t)p * NB * NB;
    if (wave == 0)
      factor_block_wave(&sS[0][0], scratch, diag0, p * NB, l_true, tol, flags, L + (int64_t)p * NB * lw + p * NB,
                        lw, Dp);
    __syncthreads();
    // panel: L_ip = G_ip Dinv_p^T, one 32 x 32 tile per wavefront
    for (int i = p + 1 + wave; i < T; i += 4) {
      v4d acc[2][2] = {{{0, 0, 0, 0}, {0, 0, 0, 0}}, {{0, 0, 0, 0}, {0, 0, 0, 0}}};
      wave_tile_xyt(G + (int64_t)i * NB * lw + p * NB, lw, Dp, NB, li, lk, acc);
      double* Lip = L + (int64_t)i * NB * lw + p * NB;
#pragma unroll
      for (int si = 0; si < 2; ++si)
#pragma unroll
        for (int sj = 0; sj < 2; ++sj)
#pragma unroll
          for (int r = 0; r < 4; ++r) Lip[(int64_t)(16 * si + 4 * r + lk) * lw + 16 * sj + li] = acc[si][sj][r];
    }
    __syncthreads();
    // trailing update: G_ij -= L_ip L_jp^T for p < j <= i
    const int nt = (T - p - 1) * (T - p) / 2;
    for (int idx = wave; idx < nt; idx += 4) {
      int t = idx, di = 0;
      while (t > di) {
        t -= di + 1;
        ++di;
      }
      const int i = p + 1 + di, j = p + 1 + t;
      v4d acc[2][2] = {{{0, 0, 0, 0}, {0, 0, 0, 0}}, {{0, 0, 0, 0}, {0, 0, 0, 0}}};
      wave_tile_xyt(L + (int64_t)i * NB * lw + p * NB, lw, L + (int64_t)j * NB * lw + p * NB, lw, li, lk, acc);
      double* Gij = G + (int64_t)i * NB * lw + j * NB;
#pragma unroll
      for (int si = 0; si < 2; ++si)
#pragma unroll
        for (int sj = 0; sj < 2; ++sj)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            double* g = Gij + (int64_t)(16 * si + 4 * r + lk) * lw + 16 * sj + li;
            *g -= acc[si][sj][r];
          }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------ second pass series --
// After the first pass, G2 = Q1^T Q1 = I + E with |E| of order cond(Y)^2 u.
// Its Cholesky factor I + F (F lower triangular) and the solve factor
// (I + F)^-T are expanded in E: with F0 = tril_half(E) (strict lower part of
// E plus half its diagonal),
//     (I + F)^-T - I = M = -F0^T + tril_half(F0 F0^T)^T + (F0 F0)^T + O(|E|^3),
// so Q = Q1 (I + F)^-T = Q1 + Q1 M.  series_m_kernel builds M (upper
// triangular, 32 x 32 tiles (a, b), a <= b) and raises gate_bit when some
// |E_ij| exceeds tau, in which case the full second pass runs instead.

__device__ __forceinline__ double f0_at(const double* G2, int lw, int l_true, int i, int t) {
  // F0[i][t] for the lower triangle of E = G2 - I (zero outside l_true)
  if (i >= l_true || t >= l_true || t > i) return 0.0;
  const double g = G2[(int64_t)i * lw + t];
  return i == t ? 0.5 * (g - 1.0) : g;
}

__global__ __launch_bounds__(256) void series_m_kernel(int lw, int l_true, const double* __restrict__ G2,
                                                       double* __restrict__ M, uint32_t* gate, uint32_t gate_bit,
                                                       double tau) {
  __shared__ double sB[NB][NB + 1];   // F0 rows of block b, t-chunk
  __shared__ double sA[NB][NB + 1];   // F0 rows of block a, t-chunk
  __shared__ double sC[NB][NB + 1];   // F0 t-chunk rows, columns of block a
  int t = blockIdx.x, bb = 0;
  while (t > bb) {
    t -= bb + 1;
    ++bb;
  }
  const int ab = t;                   // tile (ab, bb) of M with ab <= bb
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int si = wave >> 1, sj = wave & 1;
  // gate test on the E tile (bb, ab) this block owns
  bool over = false;
  for (int e = tid; e < NB * NB; e += 256) {
    const int i = bb * NB + e / NB, j = ab * NB + e % NB;
    if (i < l_true && j < l_true && j <= i) {
      const double v = G2[(int64_t)i * lw + j] - (i == j ? 1.0 : 0.0);
      if (!(fabs(v) <= tau)) over = true;
    }
  }
  if (over) atomicOr(gate, gate_bit);
  // out[r][c] = M[ab*NB + r][bb*NB + c]: transposed accumulation of
  //   S1[b][a] = sum_t F0[b][t] F0[a][t]  (t <= a)  and  S2[b][a] = sum_t F0[b][t] F0[t][a]  (a <= t <= b)
  // sub-tile (si, sj) of the (bb, ab) orientation: rows b, columns a
  v4d s1 = {0, 0, 0, 0}, s2 = {0, 0, 0, 0};
  for (int tb = 0; tb <= bb; ++tb) {
    __syncthreads();
    for (int e = tid; e < NB * NB; e += 256) {
      const int r = e / NB, c = e % NB;
      sB[r][c] = f0_at(G2, lw, l_true, bb * NB + r, tb * NB + c);
      sA[r][c] = f0_at(G2, lw, l_true, ab * NB + r, tb * NB + c);
      sC[r][c] = f0_at(G2, lw, l_true, tb * NB + r, ab * NB + c);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < NB; kk += 4) {
      const double x = sB[16 * si + li][kk + lk];
      if (tb <= ab) s1 = mfma_f64(x, sA[16 * sj + li][kk + lk], s1);     // B[k][j] = F0[a j][t k]
      if (tb >= ab) s2 = mfma_f64(x, sC[kk + lk][16 * sj + li], s2);     // B[k][j] = F0[t k][a j]
    }
  }
  // write M[a][b] = -F0[b][a] + h(S1)[b][a] + S2[b][a]  (transpose of the (b, a) tile)
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int bi = bb * NB + 16 * si + 4 * r + lk;     // row index in the (b, a) orientation
    const int aj = ab * NB + 16 * sj + li;
    double v = 0.0;
    if (aj <= bi) {
      const double h1 = (aj < bi) ? s1[r] : 0.5 * s1[r];
      v = -f0_at(G2, lw, l_true, bi, aj) + h1 + s2[r];
    }
    M[(int64_t)aj * lw + bi] = v;
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
                                                   double* __restrict__ Q, int64_t ldq, int zero_to,
                                                   const uint32_t* gate, uint32_t gate_mask) {
  if (gate && !(*gate & gate_mask)) return;
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
  double *G, *L, *Dinv, *diag0, *part, *Q1, *M, *X;
  uint32_t* gate;
  int nchunks;
  int64_t rows_per_chunk;
};

constexpr uint32_t kGateFull = 1u;      // second pass needs the full Cholesky
constexpr double kSeriesTau = 1e-5;     // |E| bound of the second-pass expansion (error O(tau^3))

static void cholqr_layout(int64_t rows, int64_t l, int* lw_out, int* nchunks, int64_t* rpc) {
  const int lw = (int)round_up(l, NB);
  const int t64 = (int)ceil_div(lw, FT);
  const int ntri = t64 * (t64 + 1) / 2;
  int64_t nc = 384 / ntri;
  const int64_t maxc = ceil_div(rows, 64);
  if (nc > maxc) nc = maxc;
  if (nc < 1) nc = 1;
  const int64_t r = round_up(ceil_div(rows, nc), FK);
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
  const size_t sq = (size_t)lw * lw;
  const size_t n = 4 * sq + (size_t)lw * NB + lw + (size_t)nc * sq + (size_t)rows * lw + 32;
  return n * sizeof(double) + 256;
}

static lramm_status set_trsm_attr() {
  static bool done = false;
  if (!done) {
    LRAMM_HIP(hipFuncSetAttribute((const void*)trsm_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024));
    LRAMM_HIP(hipFuncSetAttribute((const void*)trsm_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024));
    done = true;
  }
  return LRAMM_OK;
}

struct HookScope {
  const TimingHook* h;
  HookScope(const TimingHook* hook, int stage) : h(hook) {
    if (h) h->begin(h->ctx, stage);
  }
  ~HookScope() {
    if (h) h->end(h->ctx);
  }
};

template <typename T>
static lramm_status gram(int64_t rows, int lw, int l_true, const T* X, int64_t ldx, const CholWs& w, hipStream_t s,
                         const TimingHook* hook) {
  const int t64 = (int)ceil_div(lw, FT);
  const int ntri = t64 * (t64 + 1) / 2;
  {
    HookScope hs(hook, SUB_CHOL_GRAM);
    hipLaunchKernelGGL((gram64_kernel<T>), dim3(ntri, w.nchunks), dim3(256), 0, s, rows, lw, l_true, X, ldx, w.part,
                       w.rows_per_chunk);
  }
  LRAMM_HIP(hipGetLastError());
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)ceil_div((int64_t)lw * lw, 256)), dim3(256), 0, s, lw,
                     w.nchunks, w.part, w.G, w.diag0, w.gate);
  LRAMM_HIP(hipGetLastError());
  return LRAMM_OK;
}

// Cholesky of w.G into w.L, w.Dinv and X = L^-1 (one launch per panel).
static lramm_status cholesky_inverse(int lw, int l_true, const CholWs& w, uint32_t* flags, hipStream_t s,
                                     const TimingHook* hook) {
  const double tol = 64.0 * (double)l_true * 0x1p-53;
  const int Tn = lw / NB;
  hipLaunchKernelGGL(chol_first_kernel, dim3(1), dim3(64), 0, s, lw, l_true, w.G, w.L, w.Dinv, w.diag0, tol, flags);
  LRAMM_HIP(hipGetLastError());
  for (int p = 0; p + 1 < Tn; ++p) {
    const int nb = (Tn - p - 1) * (Tn - p) / 2 + p + 1;
    HookScope hs(hook, SUB_CHOL_PANEL);
    hipLaunchKernelGGL(chol_panel_kernel, dim3(nb), dim3(256), 0, s, lw, l_true, p, w.G, w.L, w.Dinv, w.X, w.diag0,
                       tol, flags);
    LRAMM_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(inverse_row_kernel, dim3(Tn), dim3(256), 0, s, lw, Tn - 1, w.L, w.Dinv, w.X, nullptr, 0u);
  LRAMM_HIP(hipGetLastError());
  return LRAMM_OK;
}

template <typename T, bool APPLY>
static lramm_status solve_gemm(int64_t rows, int lw, int ncols, const T* X, int64_t ldx, const double* B, double* Q,
                               int64_t ldq, int zero_to, const uint32_t* gate, uint32_t mask, hipStream_t s,
                               const TimingHook* hook) {
  HookScope hs(hook, APPLY ? SUB_CHOL_APPLY : SUB_CHOL_SOLVE);
  dim3 grid((unsigned)ceil_div(rows, FT), (unsigned)ceil_div(zero_to, FT));
  hipLaunchKernelGGL((solve_gemm_kernel<T, APPLY>), grid, dim3(256), 0, s, rows, lw, ncols, X, ldx, B, Q, ldq,
                     zero_to, gate, mask);
  LRAMM_HIP(hipGetLastError());
  return LRAMM_OK;
}

lramm_status launch_cholqr2(int64_t rows, int64_t l, const void* Y, int64_t ldy, int ytype, double* Q,
                            int64_t ldq, void* ws, size_t ws_bytes, uint32_t* flags, hipStream_t s,
                            const TimingHook* hook) {
  if (rows == 0 || l == 0) return LRAMM_OK;
  int lw, nc;
  int64_t rpc;
  cholqr_layout(rows, l, &lw, &nc, &rpc);
  if (ws_bytes < cholqr2_workspace(rows, l)) return LRAMM_E_WORKSPACE;
  if ((size_t)(16 * lw + 5 * 16 * NB) * sizeof(double) > 160 * 1024) return LRAMM_E_UNSUPPORTED;
  LRAMM_TRY(set_trsm_attr());
  uintptr_t base = round_up((int64_t)(uintptr_t)ws, 256);
  double* p = reinterpret_cast<double*>(base);
  const size_t sq = (size_t)lw * lw;
  CholWs w;
  w.G = p;
  p += sq;
  w.L = p;
  p += sq;
  w.M = p;
  p += sq;
  w.X = p;
  p += sq;
  w.Dinv = p;
  p += (size_t)lw * NB;
  w.diag0 = p;
  p += lw;
  w.part = p;
  p += (size_t)nc * sq;
  w.Q1 = p;
  p += (size_t)rows * lw;
  w.gate = reinterpret_cast<uint32_t*>(p);
  w.nchunks = nc;
  w.rows_per_chunk = rpc;
  const int lt = (int)l;
  // pass 1 on Y (columns at or past l are never read): Q1 = Y L1^-T
  if (ytype == LRAMM_F32) {
    LRAMM_TRY(gram<float>(rows, lw, lt, (const float*)Y, ldy, w, s, hook));
    LRAMM_TRY(cholesky_inverse(lw, lt, w, flags, s, hook));
    LRAMM_TRY((solve_gemm<float, false>(rows, lw, lt, (const float*)Y, ldy, w.X, w.Q1, lw, lw, nullptr, 0, s, hook)));
  } else if (ytype == LRAMM_F64) {
    LRAMM_TRY(gram<double>(rows, lw, lt, (const double*)Y, ldy, w, s, hook));
    LRAMM_TRY(cholesky_inverse(lw, lt, w, flags, s, hook));
    LRAMM_TRY((solve_gemm<double, false>(rows, lw, lt, (const double*)Y, ldy, w.X, w.Q1, lw, lw, nullptr, 0, s, hook)));
  } else {
    return LRAMM_E_UNSUPPORTED;
  }
  // pass 2 on Q1: expansion of the near-identity factor, or (gated) the full pass
  const int zero_to = (int)ldq;
  LRAMM_TRY(gram<double>(rows, lw, lt, w.Q1, lw, w, s, hook));
  const int Tn = lw / NB;
  {
    HookScope hs(hook, SUB_CHOL_SERIES);
    hipLaunchKernelGGL(series_m_kernel, dim3(Tn * (Tn + 1) / 2), dim3(256), 0, s, lw, lt, w.G, w.M, w.gate,
                       kGateFull, kSeriesTau);
  }
  LRAMM_HIP(hipGetLastError());
  LRAMM_TRY((solve_gemm<double, true>(rows, lw, lw, w.Q1, lw, w.M, Q, ldq, zero_to, w.gate, kGateFull, s, hook)));
  // gated fallback: full Cholesky of G2 and triangular solve
  const double tol = 64.0 * (double)lt * 0x1p-53;
  hipLaunchKernelGGL(chol_fused_kernel, dim3(1), dim3(256), 0, s, lw, lt, w.G, w.L, w.Dinv, w.diag0, tol, flags,
                     w.gate, kGateFull);
  LRAMM_HIP(hipGetLastError());
  const size_t shm = (size_t)(16 * lw + 4 * 16 * NB + 16 * NB) * sizeof(double);
  hipLaunchKernelGGL((trsm_kernel<double>), dim3((unsigned)ceil_div(rows, 16)), dim3(256), shm, s, rows, lw, lt,
                     w.Q1, (int64_t)lw, w.L, w.Dinv, Q, ldq, zero_to, w.gate, kGateFull);
  LRAMM_HIP(hipGetLastError());
  return LRAMM_OK;
}

}  // namespace lramm
