// CholeskyQR2 in FP64 for the range finder's orthonormalisation (paper
// Sec. 2.2: a matrix Q with orthonormal columns spanning the sketch).  For a
// rows x l matrix Y (FP32 or FP64), l' = l rounded up to 32:
//
//   G1 = Y^T Y (FP64)                 32 x 32 lower tiles x row chunks, the
//                                      four wavefronts of a workgroup split
//                                      the chunk; partials summed in a fixed
//                                      order (deterministic)
//   G1 = L L^T, X = L^-1              blocked right-looking Cholesky, 32 x 32
//                                      tiles, one launch per panel; the block
//                                      inverse is formed in the same launches
//   Q1 = Y X^T                         tall-skinny FP64 product
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
// the four lane groups, unlike the 32 x 32 MFMAs).  The k index a lane feeds
// may be permuted freely as long as A and B use the same permutation: the
// tall-skinny kernels let lane group g feed k = k0 + 4 g + q in step q, so
// that each lane reads 4 consecutive elements of a row with one vector load.
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

// Four consecutive elements x[0..3] of a row as doubles (one vector load).
__device__ __forceinline__ void load4d(const float* p, double v[4]) {
  const float4 f = *reinterpret_cast<const float4*>(p);
  v[0] = f.x, v[1] = f.y, v[2] = f.z, v[3] = f.w;
}
__device__ __forceinline__ void load4d(const double* p, double v[4]) {
  const double4 d = *reinterpret_cast<const double4*>(p);
  v[0] = d.x, v[1] = d.y, v[2] = d.z, v[3] = d.w;
}

// v where ok, else zero, without letting the compiler move the load that
// produced v under a branch (a select of a loaded value may be turned into a
// conditional load followed by a full wait; a multiply keeps the load
// unconditional).  Callers load from a valid address either way.
__device__ __forceinline__ double keep_if(bool ok, double v) { return v * (ok ? 1.0 : 0.0); }

// Lower 32 x 32 tile t (row-major over the lower triangle) -> (i, j), i >= j.
__device__ __forceinline__ void lower_tile(int t, int& i, int& j) {
  int di = 0;
  while (t > di) {
    t -= di + 1;
    ++di;
  }
  i = di;
  j = t;
}

// ------------------------------------------------------------------ Gram --
// Partial Gram of one row chunk for one lower 32 x 32 tile (a, b), a >= b:
//   part[chunk][32a + i][32b + j] = sum_{r in chunk} X[r][32a + i] X[r][32b + j],
// columns >= ncols read as zero.  The four wavefronts take consecutive
// quarters of the chunk; a wavefront computes the whole 32 x 32 tile (2 x 2
// MFMA sub-tiles), four rows per step, each lane reading X[r][c..] of one
// row (16 consecutive columns per lane group: coalesced).  The quarters are
// summed in LDS in a fixed order.
template <typename T>
__global__ __launch_bounds__(256) void gram_kernel(int64_t rows, int lw, int ncols, const T* __restrict__ X,
                                                   int64_t ldx, double* __restrict__ part, int64_t rows_per_chunk) {
  __shared__ double red[4][NB][NB + 1];
  int ta, tb;
  lower_tile(blockIdx.x, ta, tb);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t c0 = (int64_t)blockIdx.y * rows_per_chunk;
  const int64_t c1 = c0 + rows_per_chunk < rows ? c0 + rows_per_chunk : rows;
  const int64_t per = ((c1 - c0 + 15) / 16) * 4;   // a quarter of the chunk, a multiple of 4 rows
  const int64_t w0 = c0 + wave * per;
  const int64_t w1 = w0 + per < c1 ? w0 + per : c1;
  // columns past ncols are read from column 0 (valid data) and their Gram
  // entries zeroed at the end, so the main loop needs no masks
  int ca[2], cb[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    ca[s] = ta * NB + 16 * s + li;
    cb[s] = tb * NB + 16 * s + li;
    ca[s] = ca[s] < ncols ? ca[s] : 0;
    cb[s] = cb[s] < ncols ? cb[s] : 0;
  }
  v4d acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (v4d){0.0, 0.0, 0.0, 0.0};
  auto mma = [&](const double (*a)[2], const double (*b)[2]) {
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
      for (int si = 0; si < 2; ++si)
#pragma unroll
        for (int sj = 0; sj < 2; ++sj) acc[si][sj] = mfma_f64(a[q][si], b[q][sj], acc[si][sj]);
  };
  // full groups of 32 rows (8 MFMA steps); the next group is loaded while
  // the current one is multiplied
  const int64_t nfull = w1 > w0 ? (w1 - w0) / 32 : 0;
  double av[8][2], bv[8][2];
  auto fetch = [&](int64_t r, double (*a)[2], double (*b)[2]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const T* xr = X + (r + 4 * q + lk) * ldx;
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        a[q][s] = (double)xr[ca[s]];
        b[q][s] = (double)xr[cb[s]];
      }
    }
  };
  if (nfull > 0) fetch(w0, av, bv);
  for (int64_t g = 0; g < nfull; ++g) {
    double an[8][2], bn[8][2];
    const bool more = g + 1 < nfull;
    if (more) fetch(w0 + 32 * (g + 1), an, bn);
    mma(av, bv);
    if (more) {
#pragma unroll
      for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int u = 0; u < 2; ++u) av[q][u] = an[q][u], bv[q][u] = bn[q][u];
    }
  }
  // the last partial group (rows past w1 contribute zero)
  const int64_t rt = w0 + 32 * nfull;
  if (rt < w1) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t rr = rt + 4 * q + lk;
      const bool ok = rr < w1;
      const T* xr = X + (ok ? rr : w0) * ldx;
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        av[q][s] = keep_if(ok, (double)xr[ca[s]]);
        bv[q][s] = keep_if(ok, (double)xr[cb[s]]);
      }
    }
    mma(av, bv);
  }
#pragma unroll
  for (int si = 0; si < 2; ++si)
#pragma unroll
    for (int sj = 0; sj < 2; ++sj)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[wave][16 * si + 4 * r + lk][16 * sj + li] = acc[si][sj][r];
  __syncthreads();
  double* out = part + (int64_t)blockIdx.y * lw * lw + (int64_t)ta * NB * lw + tb * NB;
#pragma unroll
  for (int u = 0; u < NB * NB / 256; ++u) {
    const int e = tid + 256 * u;
    const int i = e / NB, j = e % NB;
    const bool in = ta * NB + i < ncols && tb * NB + j < ncols;
    out[(int64_t)i * lw + j] = in ? (red[0][i][j] + red[1][i][j]) + (red[2][i][j] + red[3][i][j]) : 0.0;
  }
}

// G (lower tiles) = sum over chunks in order; diag0 = diag(G).
//   mode 0 (first pass): clears the second-pass gate of this orthonormalisation;
//   mode 1 (second pass): raises gate_bit when some |G_ij - delta_ij|, i, j < l_true,
//   exceeds tau (or is NaN).
__global__ __launch_bounds__(256) void gram_reduce_kernel(int lw, int l_true, int nchunks,
                                                          const double* __restrict__ part, double* __restrict__ G,
                                                          double* __restrict__ diag0, uint32_t* gate, int mode,
                                                          uint32_t gate_bit, double tau) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (mode == 0 && e == 0) *gate = 0u;
  if (e >= (int64_t)lw * lw) return;
  const int i = (int)(e / lw), j = (int)(e % lw);
  if ((i / NB) < (j / NB)) return;   // upper tiles are never read
  double s = 0.0;
  for (int c = 0; c < nchunks; ++c) s += part[(int64_t)c * lw * lw + e];
  G[e] = s;
  if (i == j) diag0[i] = s;
  if (mode == 1 && i < l_true && j <= i) {
    const double v = s - (i == j ? 1.0 : 0.0);
    if (!(fabs(v) <= tau)) atomicOr(gate, gate_bit);
  }
}

// ---------------------------------------------------- tall-skinny product --
// Q[r][c] = (ADD ? X[r][c] : 0) + sum_{k < kend(c)} X[r][k] W[c][k]  for c < lw,
// kend(c) = min(32 (c / 32 + 1), ncols): W is lower triangular by 32-blocks
// (the blocks above its diagonal are never read).  Columns [lw, zero_to) of
// Q are written as zero.
//   solve: X = Y, W = L^-1                 (Q1 = Y L^-T)
//   apply: X = Q1, W = M^T, ADD            (Q = Q1 + Q1 M)
// A workgroup owns 16 rows, staged once in LDS as FP64 (zero past ncols and
// past the last row).  Its eight wavefronts (two per SIMD) share the
// 32-column blocks, block c costing c + 1 units of K, by longest-first
// assignment to the least loaded wavefront (computed identically on every
// lane).  A wavefront computes a 16 x 32 block (2 MFMA sub-tiles) per step of
// 16 k: lane group g feeds k = 16 s + 4 g + q in MFMA q, reading its 4
// values of X from LDS and of W with one vector load per sub-tile; W is
// fetched four steps at a time, one group ahead of the MFMAs.
constexpr int TS_ROWS = 16, TS_WAVES = 8;

__host__ __device__ constexpr int ts_pitch(int lw) { return lw + 4; }

template <typename T, bool ADD>
__global__ __launch_bounds__(TS_WAVES * 64) void tsmul_kernel(int64_t rows, int lw, int ncols,
                                                              const T* __restrict__ X, int64_t ldx,
                                                              const double* __restrict__ W, double* __restrict__ Q,
                                                              int64_t ldq, int zero_to, int vec) {
  extern __shared__ double sA[];   // TS_ROWS x ts_pitch(lw)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int pitch = ts_pitch(lw);
  const int64_t r0 = (int64_t)blockIdx.x * TS_ROWS;
  // stage the row panel: 4 consecutive columns per thread
  const int q4 = lw / 4;
  for (int e = tid; e < TS_ROWS * q4; e += TS_WAVES * 64) {
    const int rr = e / q4, c = (e % q4) * 4;
    const int64_t gr = r0 + rr;
    const bool rok = gr < rows;
    const T* xr = X + (rok ? gr : rows - 1) * ldx;
    double v[4];
    if (vec && c + 4 <= ncols) {
      load4d(xr + c, v);
    } else {   // unaligned rows, or the row's last partial group: never read past column ncols
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = (double)xr[c + q < ncols ? c + q : 0];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) sA[rr * pitch + c + q] = (rok && c + q < ncols) ? v[q] : 0.0;
  }
  __syncthreads();
  const int Tb = lw / NB;
  int load[TS_WAVES];
#pragma unroll
  for (int u = 0; u < TS_WAVES; ++u) load[u] = 0;
  for (int c = Tb - 1; c >= 0; --c) {
    int w = 0;
#pragma unroll
    for (int u = 1; u < TS_WAVES; ++u)
      if (load[u] < load[w]) w = u;
    load[w] += c + 1;
    if (w != wave) continue;
    const int cb0 = c * NB;
    const int kend = cb0 + NB < ncols ? cb0 + NB : ncols;
    const int ksteps = (kend + 15) / 16;
    const int ngroups = (ksteps + 3) / 4;
    const double* w0p = W + (int64_t)(cb0 + li) * lw + 4 * lk;
    const double* w1p = W + (int64_t)(cb0 + 16 + li) * lw + 4 * lk;
    const double* ap = sA + li * pitch + 4 * lk;
    v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
    double b[2][4][4];
    auto fetch = [&](int g, double (*b0)[4], double (*b1)[4]) {
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        if (4 * g + st < ksteps) {   // uniform: never reads W past column 32 (c + 1)
          load4d(w0p + 16 * (4 * g + st), b0[st]);
          load4d(w1p + 16 * (4 * g + st), b1[st]);
        }
      }
    };
    fetch(0, b[0], b[1]);
    for (int g = 0; g < ngroups; ++g) {
      double bn[2][4][4];
      const bool more = g + 1 < ngroups;
      if (more) fetch(g + 1, bn[0], bn[1]);
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int ks = 4 * g + st;
        if (ks < ksteps) {
          double a[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) a[q] = ap[16 * ks + q];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            acc0 = mfma_f64(a[q], b[0][st][q], acc0);
            acc1 = mfma_f64(a[q], b[1][st][q], acc1);
          }
        }
      }
      if (more) {
#pragma unroll
        for (int st = 0; st < 4; ++st)
#pragma unroll
          for (int q = 0; q < 4; ++q) b[0][st][q] = bn[0][st][q], b[1][st][q] = bn[1][st][q];
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int rr = 4 * r + lk;
      const int64_t row = r0 + rr;
      if (row < rows) {
        double v0 = acc0[r], v1 = acc1[r];
        if constexpr (ADD) {
          v0 += sA[rr * pitch + cb0 + li];
          v1 += sA[rr * pitch + cb0 + 16 + li];
        }
        Q[row * ldq + cb0 + li] = v0;
        Q[row * ldq + cb0 + 16 + li] = v1;
      }
    }
  }
  const int zc = zero_to - lw;
  for (int e = tid; e < TS_ROWS * zc; e += TS_WAVES * 64) {
    const int64_t row = r0 + e / zc;
    if (row < rows) Q[row * ldq + lw + e % zc] = 0.0;
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
// inverse X = L^-1 to Iout (32 x 32, row-major), both in one right-looking
// sweep over the columns.  Lanes 0..31 keep row i = lane of the block, lanes
// 32..63 column c = lane - 32 of X (starting as the identity), in the same
// registers v[].  Step j: the pivot v[j] of lane j is read by readlane, the
// scaled column l_j = L[:, j] is published in LDS (scratch, one 32-slot row
// per column), and every lane applies
//   v[k] -= m l_kj   (k > j),   m = l_ij (row lanes) or X[j][c] = v[j] / l_jj (column lanes),
// i.e. the Cholesky update of row i and the same elimination on column c of
// X, reading l_kj from LDS (uniform-address loads).  Only the update of the
// next column (k = j + 1) is on the critical path, and it takes l_{j+1,j}
// from lane j + 1 by readlane; the other updates of column j are applied
// one step later, so their LDS loads are off the pivot chain.
// scratch: NB * NB + NB doubles of LDS private to this wavefront.
__device__ __attribute__((always_inline)) inline void factor_block_wave(const double* S, double* scratch,
                                                                        const double* diag0, int col0, int l_true,
                                                                        double tol, uint32_t* flags, double* Lout,
                                                                        int64_t ldl, double* Iout) {
  const int lane = threadIdx.x & 63;
  const int row = lane & 31;
  const bool fac = lane < NB;
  double* sthr = scratch + NB * NB;   // pivot thresholds (negative: padding column)
  if (fac) sthr[lane] = col0 + row < l_true ? tol * diag0[col0 + row] : -1.0;
  double v[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) v[k] = fac ? S[row * (NB + 1) + k] : (k == row ? 1.0 : 0.0);
  wave_lds_sync();
  uint32_t bad = 0;
  // the updates from column j - 1 (other than the next column's) are applied
  // one step late, after the pivot of column j, so that the LDS loads of
  // column j - 1 complete while that pivot is computed
  double cprev[NB];
  double mprev = 0.0;
#pragma unroll
  for (int k = 0; k < NB; ++k) cprev[k] = 0.0;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const double tj = sthr[j];
    const double d = lane_bcast(v[j], j);
    // 1/sqrt(d): hardware estimate refined by two Newton steps (quadratic
    // convergence from ~2^-23 to full precision); piv = d / sqrt(d)
    const double hd = 0.5 * d;
    double y = __builtin_amdgcn_rsq(d);
    y = y * fma(-hd * y, y, 1.5);
    y = y * fma(-hd * y, y, 1.5);
    const bool live = tj >= 0.0;
    const bool ok = live && d > tj && d > 0.0;
    const double iv = ok ? y : 0.0;
    bad |= (live && !ok) ? ((d < -tj || d != d) ? (LRAMM_FLAG_BREAKDOWN | LRAMM_FLAG_SQRTNEG) : LRAMM_FLAG_BREAKDOWN)
                         : 0u;
    // row lanes: l_ij (0 above the diagonal, d / sqrt(d) on it); column lanes: X[j][c]
    const double sc = v[j] * ((fac && row < j) ? 0.0 : iv);
    const double m = (fac && row == j) ? d * iv : sc;
    v[j] = m;
    double* col = scratch + j * NB;
    if (fac) col[lane] = m;
    wave_lds_sync();   // also keeps later columns' loads out of this step (register pressure)
    if (j + 1 < NB) {
      const double ln = lane_bcast(m, j + 1);       // l_{j+1, j}
      v[j + 1] = fma(-m, ln, v[j + 1]);
    }
    // late updates of column j - 1 (k >= j + 1), then the loads for column j
#pragma unroll
    for (int k = j + 1; k < NB; ++k) v[k] = fma(-mprev, cprev[k], v[k]);
#pragma unroll
    for (int k = j + 2; k < NB; ++k) cprev[k] = col[k];
    mprev = m;
  }
  if (fac) {
#pragma unroll
    for (int k = 0; k < NB; ++k) Lout[(int64_t)row * ldl + k] = k <= row ? v[k] : 0.0;
  } else {
#pragma unroll
    for (int k = 0; k < NB; ++k) Iout[k * NB + row] = v[k];
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
#pragma unroll
  for (int u = 0; u < NB * NB / 64; ++u) {
    const int e = threadIdx.x + 64 * u;
    sS[(e / NB) * (NB + 1) + e % NB] = G[(int64_t)(e / NB) * lw + e % NB];
  }
  __syncthreads();
  factor_block_wave(sS, scratch, diag0, 0, l_true, tol, flags, L, lw, Dinv);
}

// 32 x 32 tile product on 4 wavefronts: out = X Y^T (X, Y in LDS, pitch
// NB + 1); wave w computes the 16 x 16 sub-tile (w / 2, w % 2).
__device__ __forceinline__ v4d tile_xyt(const double (*X)[NB + 1], const double (*Y)[NB + 1], int wave, int li,
                                        int lk) {
  const int si = wave >> 1, sj = wave & 1;
  v4d a0 = {0.0, 0.0, 0.0, 0.0}, a1 = a0;   // two chains: half the dependent MFMA latency
#pragma unroll
  for (int kk = 0; kk < NB; kk += 8) {
    a0 = mfma_f64(X[16 * si + li][kk + lk], Y[16 * sj + li][kk + lk], a0);
    a1 = mfma_f64(X[16 * si + li][kk + 4 + lk], Y[16 * sj + li][kk + 4 + lk], a1);
  }
  return a0 + a1;
}

// Block (p, j), j <= p, of X = L^-1 (lower triangular, 32 x 32 blocks):
//   X_pp = Dinv_p;  X_pj = -Dinv_p sum_{t=j}^{p-1} L_pt X_tj  (j < p).
// Needs row blocks 0..p-1 of X and row block p of L.  One workgroup: the
// four wavefronts share the terms of the sum (t = j + w, j + w + 4, ...),
// each forming whole 32 x 32 products (2 x 2 MFMA sub-tiles) with all its
// loads issued together; the partial sums meet in LDS (red0..red3) in a
// fixed order, and each wavefront then forms one 16 x 16 sub-tile of the
// product with Dinv_p.
__device__ void inverse_block(int lw, int p, int j, const double* __restrict__ L, const double* __restrict__ Dinv,
                              double* __restrict__ Xinv, double (*sS)[NB + 1], double (*red0)[NB + 1],
                              double (*red1)[NB + 1], double (*red2)[NB + 1], double (*red3)[NB + 1]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4, si = wave >> 1, sj = wave & 1;
  const double* Dp = Dinv + (int64_t)p * NB * NB;
  double* Xpj = Xinv + (int64_t)p * NB * lw + j * NB;
  if (j == p) {
#pragma unroll
    for (int u = 0; u < NB * NB / 256; ++u) {
      const int e = tid + 256 * u;
      Xpj[(int64_t)(e / NB) * lw + e % NB] = Dp[e];
    }
    return;
  }
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
  for (int t = j + wave; t < p; t += 4) {
    const double* Lpt = L + (int64_t)p * NB * lw + t * NB;
    const double* Xtj = Xinv + (int64_t)t * NB * lw + j * NB;
    double av[2][8], bv[2][8];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk)
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        av[u][kk] = Lpt[(int64_t)(16 * u + li) * lw + 4 * kk + lk];
        bv[u][kk] = Xtj[(int64_t)(4 * kk + lk) * lw + 16 * u + li];
      }
#pragma unroll
    for (int kk = 0; kk < 8; ++kk)
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = mfma_f64(av[a][kk], bv[b][kk], acc[a][b]);
  }
  double (*mine)[NB + 1] = wave == 0 ? red0 : (wave == 1 ? red1 : (wave == 2 ? red2 : red3));
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) mine[16 * a + 4 * r + lk][16 * b + li] = acc[a][b][r];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < NB * NB / 256; ++u) {
    const int e = tid + 256 * u;
    const int r = e / NB, c = e % NB;
    sS[r][c] = (red0[r][c] + red1[r][c]) + (red2[r][c] + red3[r][c]);
  }
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
  __shared__ double red[4][NB][NB + 1];
  inverse_block(lw, p, blockIdx.x, L, Dinv, Xinv, sS, red[0], red[1], red[2], red[3]);
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
    inverse_block(lw, p, blockIdx.x - ntrail, L, Dinv, Xinv, sS, sGi, sGj, sLi, sLj);
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
  double* Gij = G + (int64_t)i * NB * lw + j * NB;
  // every load of this launch is issued here: the panel tiles, Dinv_p and
  // this thread's elements of the tile being updated
  double gij[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) gij[r] = Gij[(int64_t)(16 * (wave >> 1) + 4 * r + lk) * lw + 16 * (wave & 1) + li];
#pragma unroll
  for (int u = 0; u < NB * NB / 256; ++u) {
    const int e = tid + 256 * u;
    const int r = e / NB, c = e % NB;
    sD[r][c] = Dp[e];
    sGi[r][c] = Gip[(int64_t)r * lw + c];
    sGj[r][c] = Gjp[(int64_t)r * lw + c];
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
#pragma unroll
    for (int u = 0; u < NB * NB / 256; ++u) {
      const int e = tid + 256 * u;
      Lip[(int64_t)(e / NB) * lw + e % NB] = sLi[e / NB][e % NB];
    }
  }
  const v4d upd = tile_xyt(sLi, j != i ? sLj : sLi, wave, li, lk);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int rr = 16 * (wave >> 1) + 4 * r + lk, cc = 16 * (wave & 1) + li;
    const double v = gij[r] - upd[r];
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

// The whole blocked Cholesky of G in one workgroup (no launches between
// panels), used only by the gated fallback of the second pass.  sS and
// scratch are LDS buffers of the caller.
__device__ void chol_single_wg(int lw, int l_true, double* __restrict__ G, double* __restrict__ L,
                               double* __restrict__ Dinv, const double* __restrict__ diag0, double tol,
                               uint32_t* flags, double (*sS)[NB + 1], double* scratch) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int T = lw / NB;
  for (int p = 0; p < T; ++p) {
    const double* Gpp = G + (int64_t)p * NB * lw + p * NB;
#pragma unroll
    for (int u = 0; u < NB * NB / 256; ++u) {
      const int e = tid + 256 * u;
      sS[e / NB][e % NB] = Gpp[(int64_t)(e / NB) * lw + e % NB];
    }
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
// so Q = Q1 (I + F)^-T = Q1 + Q1 M.  The kernel writes W = M^T (lower
// triangular, the operand layout of tsmul_kernel) tile by tile:
//     W[b][a] = -F0[b][a] + h(S1)[b][a] + S2[b][a],   a <= b,
//     S1[b][a] = sum_{t <= a} F0[b][t] F0[a][t],  S2[b][a] = sum_{a <= t <= b} F0[b][t] F0[t][a],
// h halving the diagonal.  The 32-wide t blocks of both sums are shared
// round-robin by the four wavefronts and their partial tiles summed in LDS.
// When the Gram reduction raised the gate (some |E_ij| > tau) the expansion
// is not accurate enough: workgroup 0 then runs the full blocked Cholesky of
// G2 and its inverse X2 in one workgroup and writes W = X2 - I (so that
// Q1 + Q1 W^T = Q1 X2^T), and the other workgroups do nothing.

// F0 elements (i, t..t+3) of row i: tril_half(G2 - I), zero outside l_true.
__device__ __forceinline__ void f0_row4(const double* G2, int lw, int l_true, int i, int t, double v[4]) {
  const int ic = i < lw ? i : lw - 1;
  load4d(G2 + (int64_t)ic * lw + t, v);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int tq = t + q;
    const bool in = i < l_true && tq < l_true && tq <= i;
    const double g = tq == i ? 0.5 * (v[q] - 1.0) : v[q];
    v[q] = keep_if(in, g);
  }
}

__device__ __forceinline__ double f0_at(const double* G2, int lw, int l_true, int i, int t) {
  const bool in = i < l_true && t < l_true && t <= i;
  const double g = G2[in ? (int64_t)i * lw + t : 0];
  return keep_if(in, i == t ? 0.5 * (g - 1.0) : g);
}

// Gated fallback of the second pass, in one workgroup: W = chol(G2)^-1 - I.
// Kept out of line so that its register pressure does not spill the series
// path of the kernel below.
__device__ __noinline__ void series_fallback(int lw, int l_true, double* G2, double* Wout, double* L, double* Dinv,
                                             const double* diag0, double tol, uint32_t* flags,
                                             double (*red)[NB][NB + 1]) {
  const int tid = threadIdx.x;
  double (*sS)[NB + 1] = red[0];
  chol_single_wg(lw, l_true, G2, L, Dinv, diag0, tol, flags, sS, &red[1][0][0]);
  const int Tn = lw / NB;
  for (int p = 0; p < Tn; ++p) {
    for (int j = 0; j <= p; ++j) {
      inverse_block(lw, p, j, L, Dinv, Wout, sS, red[1], red[2], red[3], red[4]);
      __syncthreads();
    }
  }
  for (int i = tid; i < lw; i += 256) Wout[(int64_t)i * lw + i] -= 1.0;
}

__global__ __launch_bounds__(256) void series_kernel(int lw, int l_true, double* __restrict__ G2,
                                                     double* __restrict__ Wout, double* __restrict__ L,
                                                     double* __restrict__ Dinv, const double* __restrict__ diag0,
                                                     double tol, uint32_t* flags, const uint32_t* gate,
                                                     uint32_t gate_bit) {
  __shared__ double red[5][NB][NB + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  if (*gate & gate_bit) {
    // fallback: W = chol(G2)^-1 - I, all in workgroup 0
    if (blockIdx.x != 0) return;
    series_fallback(lw, l_true, G2, Wout, L, Dinv, diag0, tol, flags, red);
    return;
  }
  int bb, ab;
  lower_tile(blockIdx.x, bb, ab);     // tile (bb, ab) of W, ab <= bb
  // tasks: S1 over t blocks 0..ab, S2 over ab..bb
  const int n1 = ab + 1, n2 = bb - ab + 1;
  v4d s1[2][2], s2[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) s1[i][j] = s2[i][j] = (v4d){0.0, 0.0, 0.0, 0.0};
  for (int task = wave; task < n1 + n2; task += 4) {
    const bool first = task < n1;
    const int tb = first ? task : ab + (task - n1);
#pragma unroll
    for (int k0 = 0; k0 < NB; k0 += 16) {
      const int t = tb * NB + k0 + 4 * lk;
      double a[2][4], b[2][4];
#pragma unroll
      for (int s = 0; s < 2; ++s) f0_row4(G2, lw, l_true, bb * NB + 16 * s + li, t, a[s]);
      if (first) {
#pragma unroll
        for (int s = 0; s < 2; ++s) f0_row4(G2, lw, l_true, ab * NB + 16 * s + li, t, b[s]);
      } else {
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int q = 0; q < 4; ++q) b[s][q] = f0_at(G2, lw, l_true, t + q, ab * NB + 16 * s + li);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int si = 0; si < 2; ++si)
#pragma unroll
          for (int sj = 0; sj < 2; ++sj) {
            if (first) s1[si][sj] = mfma_f64(a[si][q], b[sj][q], s1[si][sj]);
            else s2[si][sj] = mfma_f64(a[si][q], b[sj][q], s2[si][sj]);
          }
    }
  }
  // per-wave h(S1) + S2 at each element of the (b, a) tile, then the fixed-order sum
#pragma unroll
  for (int si = 0; si < 2; ++si)
#pragma unroll
    for (int sj = 0; sj < 2; ++sj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rb = 16 * si + 4 * r + lk, ca = 16 * sj + li;
        const int bi = bb * NB + rb, aj = ab * NB + ca;
        const double h1 = aj < bi ? s1[si][sj][r] : 0.5 * s1[si][sj][r];
        red[wave][rb][ca] = h1 + s2[si][sj][r];
      }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < NB * NB / 256; ++u) {
    const int e = tid + 256 * u;
    const int rb = e / NB, ca = e % NB;
    const int bi = bb * NB + rb, aj = ab * NB + ca;
    double v = 0.0;
    if (aj <= bi)
      v = -f0_at(G2, lw, l_true, bi, aj) + ((red[0][rb][ca] + red[1][rb][ca]) + (red[2][rb][ca] + red[3][rb][ca]));
    Wout[(int64_t)bi * lw + aj] = v;
  }
}

// ------------------------------------------------------------------ host --

struct CholWs {
  double *G, *L, *Dinv, *diag0, *part, *Q1, *W, *X;
  uint32_t* gate;
  int nchunks;
  int64_t rows_per_chunk;
};

constexpr uint32_t kGateFull = 1u;      // second pass needs the full Cholesky
constexpr double kSeriesTau = 1e-5;     // |E| bound of the second-pass expansion (error O(tau^3))

// Row chunks of the Gram: about two workgroups per compute unit over the
// lower 32 x 32 tiles, each wavefront at least 4 rows.
static void cholqr_layout(int64_t rows, int64_t l, int* lw_out, int* nchunks, int64_t* rpc) {
  const int lw = (int)round_up(l, NB);
  const int Tn = lw / NB;
  const int ntri = Tn * (Tn + 1) / 2;
  int64_t nc = 512 / ntri;
  if (nc < 1) nc = 1;
  int64_t r = round_up(ceil_div(rows, nc), (int64_t)16);
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
static lramm_status gram(int64_t rows, int lw, int l_true, const T* X, int64_t ldx, const CholWs& w, int mode,
                         hipStream_t s, const TimingHook* hook) {
  const int Tn = lw / NB;
  const int ntri = Tn * (Tn + 1) / 2;
  {
    HookScope hs(hook, SUB_CHOL_GRAM);
    hipLaunchKernelGGL((gram_kernel<T>), dim3(ntri, w.nchunks), dim3(256), 0, s, rows, lw, l_true, X, ldx, w.part,
                       w.rows_per_chunk);
  }
  LRAMM_HIP(hipGetLastError());
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)ceil_div((int64_t)lw * lw, 256)), dim3(256), 0, s, lw,
                     l_true, w.nchunks, w.part, w.G, w.diag0, w.gate, mode, kGateFull, kSeriesTau);
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

template <typename T, bool ADD>
static lramm_status tsmul(int64_t rows, int lw, int ncols, const T* X, int64_t ldx, const double* W, double* Q,
                          int64_t ldq, int zero_to, hipStream_t s, const TimingHook* hook) {
  static bool attr_set = false;
  if (!attr_set) {   // up to 16 x 1028 doubles of LDS
    LRAMM_HIP(hipFuncSetAttribute((const void*)tsmul_kernel<T, ADD>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024));
    attr_set = true;
  }
  HookScope hs(hook, ADD ? SUB_CHOL_APPLY : SUB_CHOL_SOLVE);
  // 4-element vector loads need every row start aligned to 4 elements
  const int vec = ((uintptr_t)X % (4 * sizeof(T)) == 0 && ldx % 4 == 0) ? 1 : 0;
  const size_t shm = (size_t)TS_ROWS * ts_pitch(lw) * sizeof(double);
  hipLaunchKernelGGL((tsmul_kernel<T, ADD>), dim3((unsigned)ceil_div(rows, (int64_t)TS_ROWS)), dim3(TS_WAVES * 64),
                     shm, s, rows, lw, ncols, X, ldx, W, Q, ldq, zero_to, vec);
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
  uintptr_t base = round_up((int64_t)(uintptr_t)ws, 256);
  double* p = reinterpret_cast<double*>(base);
  const size_t sq = (size_t)lw * lw;
  CholWs w;
  w.G = p;
  p += sq;
  w.L = p;
  p += sq;
  w.W = p;
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
    LRAMM_TRY(gram<float>(rows, lw, lt, (const float*)Y, ldy, w, 0, s, hook));
    LRAMM_TRY(cholesky_inverse(lw, lt, w, flags, s, hook));
    LRAMM_TRY((tsmul<float, false>(rows, lw, lt, (const float*)Y, ldy, w.X, w.Q1, lw, lw, s, hook)));
  } else if (ytype == LRAMM_F64) {
    LRAMM_TRY(gram<double>(rows, lw, lt, (const double*)Y, ldy, w, 0, s, hook));
    LRAMM_TRY(cholesky_inverse(lw, lt, w, flags, s, hook));
    LRAMM_TRY((tsmul<double, false>(rows, lw, lt, (const double*)Y, ldy, w.X, w.Q1, lw, lw, s, hook)));
  } else {
    return LRAMM_E_UNSUPPORTED;
  }
  // pass 2 on Q1: expansion of the near-identity factor, or (gated) the full factor
  const int zero_to = (int)ldq;
  LRAMM_TRY(gram<double>(rows, lw, lt, w.Q1, lw, w, 1, s, hook));
  const int Tn = lw / NB;
  const double tol = 64.0 * (double)lt * 0x1p-53;
  {
    HookScope hs(hook, SUB_CHOL_SERIES);
    hipLaunchKernelGGL(series_kernel, dim3(Tn * (Tn + 1) / 2), dim3(256), 0, s, lw, lt, w.G, w.W, w.L, w.Dinv,
                       w.diag0, tol, flags, w.gate, kGateFull);
  }
  LRAMM_HIP(hipGetLastError());
  LRAMM_TRY((tsmul<double, true>(rows, lw, lw, w.Q1, lw, w.W, Q, ldq, zero_to, s, hook)));
  return LRAMM_OK;
}

}  // namespace lramm
