// CholeskyQR2 in FP64 for the range finder's orthonormalisation (paper
// Sec. 2.2: a matrix Q with orthonormal columns spanning the sketch).  For a
// rows x l matrix Y (FP32 or FP64), l' = l rounded up to 32:
//
//   G1 = Y^T Y (FP64)                 32 x 32 lower tiles x row chunks, the
//                                      four wavefronts of a workgroup split
//                                      the chunk; partials summed in a fixed
//                                      order (deterministic)
//   G1 = L L^T, X = L^-1              blocked right-looking Cholesky, 32 x 32
//                                      tiles, with the block inverse, in one
//                                      launch whose workgroups wait on progress
//                                      counters (one launch per two panels
//                                      when its grid cannot be resident)
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
// The first pass's column maxima of |Q1| are kept in kCmSlices copies, one
// per group of workgroups (the solve's workgroup index mod kCmSlices), so
// that a column's atomics spread over several words; readers take the
// maximum over the copies.
constexpr int kCmSlices = 8;
// The workspace's gate area (64 words): word 0 the second pass's gate, words
// kProgWord .. kProgWord + 2 the progress counters of the one-launch
// Cholesky, all cleared by the first pass's Gram reduction.
constexpr int kProgWord = 8;

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

// threadIdx.x as a value the compiler may not reuse or move: index
// arithmetic of the LDS tile helpers then stays where it is used, instead of
// being hoisted out of the long loops of the one-launch Cholesky and held in
// registers across them.
__device__ __forceinline__ int tid_x() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
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
  // full groups of 32 rows (8 MFMA steps) in three register buffers, loads
  // two groups ahead of the MFMAs; fetches past the last group re-read group
  // 0 (valid rows, unused) so that no load sits under a branch
  const int64_t nfull = w1 > w0 ? (w1 - w0) / 32 : 0;
  auto fetch = [&](int64_t g, double (*a)[2], double (*b)[2]) {
    const int64_t r = w0 + 32 * (g < nfull ? g : 0);
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
  if (nfull > 0) {
    double a0[8][2], b0[8][2], a1[8][2], b1[8][2], a2[8][2], b2[8][2];
    fetch(0, a0, b0);
    fetch(1, a1, b1);
    for (int64_t g = 0; g < nfull; g += 3) {
      fetch(g + 2, a2, b2);
      mma(a0, b0);
      if (g + 1 >= nfull) break;
      fetch(g + 3, a0, b0);
      mma(a1, b1);
      if (g + 2 >= nfull) break;
      fetch(g + 4, a1, b1);
      mma(a2, b2);
    }
  }
  // the last partial group (rows past w1 contribute zero)
  const int64_t rt = w0 + 32 * nfull;
  if (rt < w1) {
    double av[8][2], bv[8][2];
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

// The same partial Gram with 64 x 64 tiles: workgroup (tile (A, B) of the
// 64-column blocks, A >= B; row chunk), wavefront (wi, wj) computes the
// 32 x 32 tile (2A + wi, 2B + wj) over the whole chunk (none above the
// diagonal or past the last 32-block), so each workgroup reads its two
// 64-column bands once for four tiles instead of two 32-column bands for
// one.  Written to the same partial layout as gram_kernel.
template <typename T>
__global__ __launch_bounds__(256) void gram64_kernel(int64_t rows, int lw, int ncols, const T* __restrict__ X,
                                                     int64_t ldx, double* __restrict__ part, int64_t rows_per_chunk) {
  int A64, B64;
  lower_tile(blockIdx.x, A64, B64);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ta = 2 * A64 + (wave >> 1), tb = 2 * B64 + (wave & 1);
  const int Tn = lw / NB;
  if (ta >= Tn || tb >= Tn || ta < tb) return;   // no barrier below: idle wavefronts leave
  const int64_t w0 = (int64_t)blockIdx.y * rows_per_chunk;
  const int64_t w1 = w0 + rows_per_chunk < rows ? w0 + rows_per_chunk : rows;
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
  const int64_t nfull = w1 > w0 ? (w1 - w0) / 32 : 0;
  auto fetch = [&](int64_t g, double (*a)[2], double (*b)[2]) {
    const int64_t r = w0 + 32 * (g < nfull ? g : 0);
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
  if (nfull > 0) {
    double a0[8][2], b0[8][2], a1[8][2], b1[8][2], a2[8][2], b2[8][2];
    fetch(0, a0, b0);
    fetch(1, a1, b1);
    for (int64_t g = 0; g < nfull; g += 3) {
      fetch(g + 2, a2, b2);
      mma(a0, b0);
      if (g + 1 >= nfull) break;
      fetch(g + 3, a0, b0);
      mma(a1, b1);
      if (g + 2 >= nfull) break;
      fetch(g + 4, a1, b1);
      mma(a2, b2);
    }
  }
  const int64_t rt = w0 + 32 * nfull;
  if (rt < w1) {
    double av[8][2], bv[8][2];
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
  double* out = part + (int64_t)blockIdx.y * lw * lw + (int64_t)ta * NB * lw + tb * NB;
#pragma unroll
  for (int si = 0; si < 2; ++si)
#pragma unroll
    for (int sj = 0; sj < 2; ++sj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * si + 4 * r + lk, j = 16 * sj + li;
        const bool in = ta * NB + i < ncols && tb * NB + j < ncols;
        out[(int64_t)i * lw + j] = in ? acc[si][sj][r] : 0.0;
      }
}

// Second-pass gate bits (one word per orthonormalisation).
constexpr uint32_t kGateFull = 1u;    // |E| too large for the expansion: full Cholesky of G2
constexpr uint32_t kGatePass2 = 2u;   // the first pass is not yet orthonormal to the second pass's accuracy

// G (lower tiles) = sum over chunks in order; diag0 = diag(G).
//   mode 0 (first pass): clears the gate word and the first-pass column
//   maxima cm1 (kCmSlices x lw words) of this orthonormalisation;
//   mode 1 (second pass): with E = G - I over i, j < l_true, raises kGateFull
//   when some |E_ij| exceeds tau (or is NaN) and kGatePass2 when some |E_ij|
//   exceeds tau_skip (or is NaN); one atomic per wavefront at most.
__global__ __launch_bounds__(256) void gram_reduce_kernel(int lw, int l_true, int nchunks,
                                                          const double* __restrict__ part, double* __restrict__ G,
                                                          double* __restrict__ diag0, uint32_t* gate,
                                                          uint32_t* cm1, int mode, double tau, double tau_skip) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (mode == 0) {
    if (e == 0) *gate = 0u;
    if (e < 3) gate[kProgWord + e] = 0u;   // the Cholesky chain's progress counters
    if (cm1 && e < (int64_t)kCmSlices * lw) cm1[e] = 0u;
  }
  uint32_t bits = 0;
  if (e < (int64_t)lw * lw) {
    const int i = (int)(e / lw), j = (int)(e % lw);
    if ((i / NB) >= (j / NB)) {   // upper tiles are never read
      // the chunks in order, sixteen loads in flight (clamped, unused past the last chunk)
      double s = 0.0;
      const int64_t sq = (int64_t)lw * lw;
      for (int c0 = 0; c0 < nchunks; c0 += 16) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = part[(int64_t)(c0 + u < nchunks ? c0 + u : nchunks - 1) * sq + e];
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (c0 + u < nchunks) s += v[u];
      }
      G[e] = s;
      if (i == j) diag0[i] = s;
      if (mode == 1 && i < l_true && j <= i) {
        const double v = fabs(s - (i == j ? 1.0 : 0.0));
        if (!(v <= tau)) bits |= kGateFull;
        if (!(v <= tau_skip)) bits |= kGatePass2;
      }
    }
  }
  if (mode == 1) {
    const uint64_t full = __ballot(bits & kGateFull), pass2 = __ballot(bits & kGatePass2);
    const uint32_t wb = (full ? kGateFull : 0u) | (pass2 ? kGatePass2 : 0u);
    if ((threadIdx.x & 63) == 0 && wb) atomicOr(gate, wb);
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
// past the last row) before anything is written, so Q may be X itself (the
// apply step runs in place).  With a gate word, the apply step does nothing
// unless kGatePass2 is set.  Its eight wavefronts (two per SIMD) share the
// 32-column blocks, block c costing c + 1 units of K, by longest-first
// assignment to the least loaded wavefront (computed identically on every
// lane).  A wavefront computes a 16 x 32 block (2 MFMA sub-tiles) per step of
// 16 k: lane group g feeds k = 16 s + 4 g + q in MFMA q, reading its 4
// values of X from LDS and of W with one vector load per sub-tile; W is
// fetched four steps at a time, one group ahead of the MFMAs.
constexpr int TS_ROWS = 16, TS_WAVES = 8;

__host__ __device__ constexpr int ts_pitch(int lw) { return lw + 4; }
// LDS bytes of the solve with its last block formed from the others:
// staged rows, the other blocks' results, eight partial sums and the residual.
__host__ __device__ constexpr size_t ts_solve_last_lds(int lw) {
  return (size_t)(2 * TS_ROWS * ts_pitch(lw) + (TS_WAVES + 1) * TS_ROWS * NB) * sizeof(double);
}
// With STAGED, each wavefront passes its W rows through an LDS tile of 32
// rows x 16 k (pitch 18 doubles: the 16-byte reads of 8 consecutive rows hit
// distinct banks), so that the global loads read whole 128-byte rows.
constexpr int TS_WST = 32 * 18;
constexpr size_t ts_stage_lds() { return (size_t)TS_WAVES * TS_WST * sizeof(double); }

// RB: 16-row halves per workgroup (1 or 2).  With two, each wavefront feeds
// the same W fragments to both halves (W is read once per 32 rows, and four
// accumulators are in flight); the last-block solve needs RB = 1.
// Q's bf16 codes written beside Q (rows codes and the transposed codes; null
// rows: none), for a solve whose Q is final.
struct TsCodes {
  uint16_t* rows;
  int64_t rpitch;       // elements
  int rpe;              // elements per codes row (zero from lw on)
  float* rscales;
  uint16_t* cols;       // one row per column c < ncols
  int64_t cpitch;       // elements
  int64_t cpe;          // elements per transposed codes row (zero from rows on)
  float* cscales;
};

__device__ __forceinline__ void ts_put_codes(const TsCodes& tc, int64_t row, int col, int ncols, double v) {
  const uint16_t h = bf16_bits((float)v);
  tc.rows[row * tc.rpitch + col] = h;
  if (col < ncols) tc.cols[(int64_t)col * tc.cpitch + row] = h;
}

template <typename T, bool ADD, bool STAGED, int RB = 1>
__global__ __launch_bounds__(TS_WAVES * 64) void tsmul_kernel(int64_t rows, int lw, int ncols, const T* X,
                                                              int64_t ldx, const double* __restrict__ W, double* Q,
                                                              int64_t ldq, int zero_to, int vec,
                                                              uint32_t* __restrict__ colmax, int cm_stride,
                                                              const uint32_t* __restrict__ gate,
                                                              const double* __restrict__ Ltri,
                                                              const double* __restrict__ Dlast, TsCodes tc) {
  extern __shared__ double sA[];   // ROWS x ts_pitch(lw) [+ the last-block solve's buffers]
  constexpr int ROWS = TS_ROWS * RB;
  if (ADD && gate && !(*gate & kGatePass2)) return;   // second pass skipped: Q already holds Q1
  if (colmax) colmax += (blockIdx.x % kCmSlices) * cm_stride;   // this workgroup's copy (cm_stride 0: one copy)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int pitch = ts_pitch(lw);
  const int64_t r0 = (int64_t)blockIdx.x * ROWS;
  // stage the row panel: 4 consecutive columns per thread
  const int q4 = lw / 4;
  for (int e = tid; e < ROWS * q4; e += TS_WAVES * 64) {
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
  // last-block solve: block Tb - 1 of Q1 from the other blocks (below), so
  // row block Tb - 1 of W = L^-1 is never needed
  const bool solve_last = RB == 1 && !ADD && Ltri != nullptr;
  double* sQ = sA + TS_ROWS * pitch;              // the other blocks' results, same layout as sA
  int load[TS_WAVES];
#pragma unroll
  for (int u = 0; u < TS_WAVES; ++u) load[u] = 0;
  for (int c = (solve_last ? Tb - 2 : Tb - 1); c >= 0; --c) {
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
    const double* ap2 = ap + TS_ROWS * pitch;     // rows 16 .. 31 (RB = 2)
    v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = acc0, acc2 = acc0, acc3 = acc0;
    if constexpr (STAGED) {
      // 8 rows of 16 k (128 bytes each) per load instruction; a kstep's 32 x 16
      // tile goes through the wavefront's LDS tile into the MFMA layout.  The
      // next group of four ksteps is loaded while this one is multiplied
      // (past the last kstep the loads repeat it, unused).
      double* wst = sA + (solve_last ? 2 * TS_ROWS * pitch + (TS_WAVES + 1) * TS_ROWS * NB : ROWS * pitch) +
                    wave * TS_WST;
      typedef unsigned int v4u __attribute__((ext_vector_type(4)));
      const int lr = lane >> 3, lj = lane & 7;
      const double* wg = W + (int64_t)(cb0 + lr) * lw + 2 * lj;
      auto fetchg = [&](int g, v4u (*r)[4]) {
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const int ks = min(4 * g + st, ksteps - 1);
#pragma unroll
          for (int i = 0; i < 4; ++i) r[st][i] = *reinterpret_cast<const v4u*>(wg + (int64_t)(8 * i) * lw + 16 * ks);
        }
      };
      v4u rc[4][4], rn[4][4];
      fetchg(0, rc);
      for (int g = 0; g < ngroups; ++g) {
        fetchg(g + 1 < ngroups ? g + 1 : g, rn);
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const int ks = 4 * g + st;
          if (ks < ksteps) {
            // the wavefront rewrites its tile only after reading the previous
            // kstep from it (LDS keeps one wavefront's accesses in order)
#pragma unroll
            for (int i = 0; i < 4; ++i) *reinterpret_cast<v4u*>(wst + (8 * i + lr) * 18 + 2 * lj) = rc[st][i];
            double b0[4], b1[4];
            const double2 x0 = *reinterpret_cast<const double2*>(wst + li * 18 + 4 * lk);
            const double2 x1 = *reinterpret_cast<const double2*>(wst + li * 18 + 4 * lk + 2);
            const double2 y0 = *reinterpret_cast<const double2*>(wst + (16 + li) * 18 + 4 * lk);
            const double2 y1 = *reinterpret_cast<const double2*>(wst + (16 + li) * 18 + 4 * lk + 2);
            b0[0] = x0.x, b0[1] = x0.y, b0[2] = x1.x, b0[3] = x1.y;
            b1[0] = y0.x, b1[1] = y0.y, b1[2] = y1.x, b1[3] = y1.y;
            double a[4], a2[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) a[q] = ap[16 * ks + q];
            if constexpr (RB == 2) {
#pragma unroll
              for (int q = 0; q < 4; ++q) a2[q] = ap2[16 * ks + q];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              acc0 = mfma_f64(a[q], b0[q], acc0);
              acc1 = mfma_f64(a[q], b1[q], acc1);
              if constexpr (RB == 2) {
                acc2 = mfma_f64(a2[q], b0[q], acc2);
                acc3 = mfma_f64(a2[q], b1[q], acc3);
              }
            }
          }
        }
#pragma unroll
        for (int st = 0; st < 4; ++st)
#pragma unroll
          for (int i = 0; i < 4; ++i) rc[st][i] = rn[st][i];
      }
    } else {
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
          double a[4], a2[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) a[q] = ap[16 * ks + q];
          if constexpr (RB == 2) {
#pragma unroll
            for (int q = 0; q < 4; ++q) a2[q] = ap2[16 * ks + q];
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            acc0 = mfma_f64(a[q], b[0][st][q], acc0);
            acc1 = mfma_f64(a[q], b[1][st][q], acc1);
            if constexpr (RB == 2) {
              acc2 = mfma_f64(a2[q], b[0][st][q], acc2);
              acc3 = mfma_f64(a2[q], b[1][st][q], acc3);
            }
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
    }
    uint32_t m0 = 0, m1 = 0;   // column maxima of fl32(|Q|) over this wavefront's rows
    if (solve_last) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        sQ[(4 * r + lk) * pitch + cb0 + li] = acc0[r];
        sQ[(4 * r + lk) * pitch + cb0 + 16 + li] = acc1[r];
      }
    }
#pragma unroll
    for (int h = 0; h < RB; ++h)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = 16 * h + 4 * r + lk;
        const int64_t row = r0 + rr;
        if (row < rows) {
          double v0 = h ? acc2[r] : acc0[r], v1 = h ? acc3[r] : acc1[r];
          if constexpr (ADD) {
            v0 += sA[rr * pitch + cb0 + li];
            v1 += sA[rr * pitch + cb0 + 16 + li];
          }
          Q[row * ldq + cb0 + li] = v0;
          Q[row * ldq + cb0 + 16 + li] = v1;
          if (tc.rows) {
            ts_put_codes(tc, row, cb0 + li, ncols, v0);
            ts_put_codes(tc, row, cb0 + 16 + li, ncols, v1);
          }
          m0 = max(m0, __float_as_uint(fabsf((float)v0)));
          m1 = max(m1, __float_as_uint(fabsf((float)v1)));
        }
      }
    if (colmax) {
      // the four lane groups hold the same columns: combine, then one atomic per column
      m0 = max(m0, (uint32_t)__shfl_xor((int)m0, 16));
      m0 = max(m0, (uint32_t)__shfl_xor((int)m0, 32));
      m1 = max(m1, (uint32_t)__shfl_xor((int)m1, 16));
      m1 = max(m1, (uint32_t)__shfl_xor((int)m1, 32));
      if (lk == 0) {
        if (m0) atomicMax(colmax + cb0 + li, m0);
        if (m1) atomicMax(colmax + cb0 + 16 + li, m1);
      }
    }
  }
  if (solve_last) {
    // Q1_c = (Y_c - sum_{t<c} Q1_t L_{c,t}^T) Dinv_c^T, c = Tb - 1: wavefront w
    // takes the terms t = w, w + 8, ...; the partial sums meet in LDS in a
    // fixed order, then one wavefront applies Dinv_c
    double* red = sQ + TS_ROWS * pitch;             // TS_WAVES x 16 x 32
    double* sR = red + TS_WAVES * TS_ROWS * NB;     // 16 x 32
    __syncthreads();                                // every other block is in sQ
    const int c = Tb - 1, cb0 = c * NB;
    v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
    for (int t = wave; t < c; t += TS_WAVES) {
#pragma unroll
      for (int st = 0; st < 2; ++st) {
        const int k0 = t * NB + 16 * st + 4 * lk;
        double a[4], b0[4], b1[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] = sQ[li * pitch + k0 + q];
        load4d(Ltri + (int64_t)(cb0 + li) * lw + k0, b0);
        load4d(Ltri + (int64_t)(cb0 + 16 + li) * lw + k0, b1);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          acc0 = mfma_f64(a[q], b0[q], acc0);
          acc1 = mfma_f64(a[q], b1[q], acc1);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      red[(wave * TS_ROWS + 4 * r + lk) * NB + li] = acc0[r];
      red[(wave * TS_ROWS + 4 * r + lk) * NB + 16 + li] = acc1[r];
    }
    __syncthreads();
    for (int e = tid; e < TS_ROWS * NB; e += TS_WAVES * 64) {
      const int i = e / NB, j = e % NB;
      double v = 0.0;
#pragma unroll
      for (int w = 0; w < TS_WAVES; ++w) v += red[(w * TS_ROWS + i) * NB + j];
      sR[i * NB + j] = sA[i * pitch + cb0 + j] - v;
    }
    __syncthreads();
    if (wave == 0) {
      v4d o0 = {0.0, 0.0, 0.0, 0.0}, o1 = o0;
#pragma unroll
      for (int st = 0; st < 2; ++st) {
        const int k0 = 16 * st + 4 * lk;
        double a[4], b0[4], b1[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] = sR[li * NB + k0 + q];
        load4d(Dlast + (int64_t)li * NB + k0, b0);
        load4d(Dlast + (int64_t)(16 + li) * NB + k0, b1);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          o0 = mfma_f64(a[q], b0[q], o0);
          o1 = mfma_f64(a[q], b1[q], o1);
        }
      }
      uint32_t m0 = 0, m1 = 0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + 4 * r + lk;
        if (row < rows) {
          Q[row * ldq + cb0 + li] = o0[r];
          Q[row * ldq + cb0 + 16 + li] = o1[r];
          if (tc.rows) {
            ts_put_codes(tc, row, cb0 + li, ncols, o0[r]);
            ts_put_codes(tc, row, cb0 + 16 + li, ncols, o1[r]);
          }
          m0 = max(m0, __float_as_uint(fabsf((float)o0[r])));
          m1 = max(m1, __float_as_uint(fabsf((float)o1[r])));
        }
      }
      if (colmax) {
        m0 = max(m0, (uint32_t)__shfl_xor((int)m0, 16));
        m0 = max(m0, (uint32_t)__shfl_xor((int)m0, 32));
        m1 = max(m1, (uint32_t)__shfl_xor((int)m1, 16));
        m1 = max(m1, (uint32_t)__shfl_xor((int)m1, 32));
        if (lk == 0) {
          if (m0) atomicMax(colmax + cb0 + li, m0);
          if (m1) atomicMax(colmax + cb0 + 16 + li, m1);
        }
      }
    }
  }
  const int zc = zero_to - lw;
  for (int e = tid; e < ROWS * zc; e += TS_WAVES * 64) {
    const int64_t row = r0 + e / zc;
    if (row < rows) Q[row * ldq + lw + e % zc] = 0.0;
  }
  if (tc.rows) {
    // the row codes' padding past lw, the unit scales of the rows (and, in
    // workgroup 0, of the transposed codes)
    const int zr = tc.rpe - lw;
    for (int e = tid; e < ROWS * zr; e += TS_WAVES * 64) {
      const int64_t row = r0 + e / zr;
      if (row < rows) tc.rows[row * tc.rpitch + lw + e % zr] = 0;
    }
    for (int e = tid; e < ROWS; e += TS_WAVES * 64)
      if (r0 + e < rows) tc.rscales[r0 + e] = 1.0f;
    if (blockIdx.x == 0)
      for (int c = tid; c < ncols; c += TS_WAVES * 64) tc.cscales[c] = 1.0f;
    // the transposed codes' padding past the last row, by the last workgroup
    const int zt = (int)(tc.cpe - rows);
    if (r0 + ROWS >= rows && zt > 0)
      for (int e = tid; e < ncols * zt; e += TS_WAVES * 64) tc.cols[(int64_t)(e / zt) * tc.cpitch + rows + e % zt] = 0;
  }
}

// -------------------------------------------------------------- Cholesky --
// Blocked right-looking Cholesky with 32 x 32 tiles, two panels per launch.
// Launch p (p even) finds L and Dinv for the diagonal blocks p and p + 1 (and
// L_{p+1,p}) ready; every trailing tile (i, j), p + 2 <= j <= i, forms its own
// panel tiles L_{i,p}, L_{i,p+1} (and L_{j,.}) and applies both panels; the
// workgroup of tile (p+2, p+2) owns (p+3, p+2) and (p+3, p+3) too and
// factors the diagonal blocks p + 2 and p + 3 one after the other, so the
// next launch again finds two factored blocks.  Further workgroups form row
// blocks p and p + 1 of X = L^-1.  A diagonal block is factored by one
// wavefront with rows in registers (lane i owns row i).

__device__ __forceinline__ double lane_bcast(double v, int lane) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// LDS of one wavefront's block factorisation (doubles, 16-byte aligned):
// the published columns of L, one 64-slot row per column.
constexpr int kFactorScratch = NB * 64;

// Pivot threshold of column col: tol times its original Gram diagonal, +inf
// for padding columns (col >= l_true; diag0 is not read there).  Callers load
// the thresholds of a block into LDS at kernel start, so that the global
// load's latency overlaps the tile loads instead of the factorisation.
__device__ __forceinline__ double pivot_thr(const double* diag0, int col, int l_true, double tol) {
  return col < l_true ? tol * diag0[col] : __builtin_inf();
}

// One wavefront factors the 32 x 32 block S (LDS, pitch NB + 1) in place
// into L (the entries above the diagonal are left undefined: store the tile
// with tile_store_lower) and writes the inverse X = L^-1 to the LDS tile Xo
// (pitch NB + 1), both in one right-looking sweep over the columns.  Lanes 0..31 keep row i = lane of the block, lanes
// 32..63 column c = lane - 32 of X (starting as the identity), in the same
// registers v[].  Step j: the pivot v[j] of lane j is read by readlane, every
// lane scales its v[j] by 1 / l_jj (giving l_ij on the row lanes and X[j][c]
// on the column lanes), the scaled column is published in LDS, and every
// lane applies
//   v[k] -= m l_kj   (k > j),   m = the scaled v[j] of the lane,
// i.e. the Cholesky update of row i and the same elimination on column c of
// X, reading l_kj from LDS (uniform-address loads).  Only the update of the
// next column (k = j + 1) is on the critical path; it takes l_{j+1,j} from
// lane j + 1 by readlane, and the other updates of column j are applied one
// step later, once their LDS loads have returned.  The LDS column is read
// back by the wavefront that wrote it, so LDS keeps the order without a wait.
// A pivot is accepted when it exceeds its threshold thr[j] (LDS, see
// pivot_thr); otherwise 1 / l_jj is taken as zero and column j of L and row j
// of X vanish.  Dropped live pivots are
// classified after the sweep: the pivot is recomputed on its lane with the
// same operations in the same order (so it is bit-identical) and flags
// breakdown, plus a negative or NaN pivot.
// With NS < NB only the first NS columns are swept and the last NB - NS are
// taken as dropped (their columns of L and rows of X are zero), which is
// what the full sweep gives when those columns are padding (their
// thresholds are +inf).
// scratch: kFactorScratch doubles of LDS private to this wavefront.
template <int NEWTON = 2, int NS = NB>
__device__ __attribute__((always_inline)) inline void factor_block_wave(double* S, double* Xo, double* scratch,
                                                                        const double* thr_s, int col0, int l_true,
                                                                        uint32_t* flags) {
  const int lane = tid_x() & 63;
  const int row = lane & 31;
  const bool fac = lane < NB;
  const bool live_col = col0 + row < l_true;
  double v[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) v[k] = fac ? S[row * (NB + 1) + k] : (k == row ? 1.0 : 0.0);
  double cprev[NB];
  double mprev = 0.0;
#pragma unroll
  for (int k = 0; k < NB; ++k) cprev[k] = 0.0;
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    const double d = lane_bcast(v[j], j);
    const bool ok = d > thr_s[j];
    // 1/sqrt(d): hardware estimate (about 2^-23) refined by NEWTON Newton
    // steps, each squaring the relative error
    const double hd = 0.5 * d;
    double y = __builtin_amdgcn_rsq(d);
#pragma unroll
    for (int it = 0; it < NEWTON; ++it) y = y * fma(-hd * y, y, 1.5);
    const double iv = ok ? y : 0.0;      // zero for padding and dropped pivots
    // m = v[j] / l_jj on every lane: l_ij below the diagonal, l_jj = d / sqrt(d)
    // on it (v[j] of lane j is d), X[j][c] on the column lanes; rows above j
    // get values that are never read (their L entries are written as zero)
    const double m = v[j] * iv;
    v[j] = m;
    double* col = scratch + j * 64;
    col[lane] = m;                       // slots 32..63 are never read
    if (j + 1 < NS) {
      const double ln = lane_bcast(m, j + 1);       // l_{j+1, j}
      v[j + 1] = fma(-m, ln, v[j + 1]);
    }
#pragma unroll
    for (int k = j + 1; k < NS; ++k) v[k] = fma(-mprev, cprev[k], v[k]);
    // l_kj, k >= j + 2, for the delayed updates: 16-byte loads of aligned pairs
    int k0 = j + 2;
    if ((k0 & 1) && k0 < NS) cprev[k0++] = col[k0];
#pragma unroll
    for (int k = k0; k < NS; k += 2) {
      const double2 t = *reinterpret_cast<const double2*>(col + k);
      cprev[k] = t.x;
      cprev[k + 1] = t.y;
    }
    mprev = m;
  }
#pragma unroll
  for (int k = NS; k < NB; ++k) v[k] = 0.0;   // padding columns: dropped
  // a dropped pivot leaves l_jj = 0 (or NaN for a non-finite pivot)
  const bool suspect = fac && live_col && !(scratch[row * 64 + row] > 0.0);
  if (__ballot(suspect)) {
    uint32_t bad = 0;
    if (suspect) {
      // the pivot of column r = row as the sweep formed it: the updates of
      // columns 0 .. r-3 in order, then column r-1, then column r-2
      const double* Lc = scratch + row;    // L[row][k] = Lc[64 k]
      double d = S[row * (NB + 1) + row];
      for (int k = 0; k + 2 < row; ++k) d = fma(-Lc[64 * k], Lc[64 * k], d);
      if (row >= 1) d = fma(-Lc[64 * (row - 1)], Lc[64 * (row - 1)], d);
      if (row >= 2) d = fma(-Lc[64 * (row - 2)], Lc[64 * (row - 2)], d);
      const double thr = thr_s[row];
      if (!(d > thr)) bad = (d < -thr || d != d) ? (LRAMM_FLAG_BREAKDOWN | LRAMM_FLAG_SQRTNEG) : LRAMM_FLAG_BREAKDOWN;
    }
    if (bad && flags) atomicOr(flags, bad);
  }
  if (fac) {
#pragma unroll
    for (int k = 0; k < NB; ++k) S[row * (NB + 1) + k] = v[k];
  } else {
#pragma unroll
    for (int k = 0; k < NB; ++k) Xo[k * (NB + 1) + row] = v[k];
  }
}

// The diagonal block at column col0, swept over its first half only when
// its second half is padding (the last block of l' = l rounded up to 32).
template <int NEWTON = 2>
__device__ __attribute__((always_inline)) inline void factor_block(double* S, double* Xo, double* scratch,
                                                                   const double* thr_s, int col0, int l_true,
                                                                   uint32_t* flags) {
  if (l_true - col0 <= NB / 2)
    factor_block_wave<NEWTON, NB / 2>(S, Xo, scratch, thr_s, col0, l_true, flags);
  else
    factor_block_wave<NEWTON, NB>(S, Xo, scratch, thr_s, col0, l_true, flags);
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

typedef double Tile[NB][NB + 1];   // an LDS tile, padded rows

// Global 32 x 32 tile (row stride ld) -> LDS, all loads issued first.
__device__ __forceinline__ void tile_load(double (*dst)[NB + 1], const double* src, int64_t ld) {
  const int tid = tid_x();
  double v[NB * NB / 256];
#pragma unroll
  for (int u = 0; u < NB * NB / 256; ++u) {
    const int e = tid + 256 * u;
    v[u] = src[(int64_t)(e / NB) * ld + e % NB];
  }
#pragma unroll
  for (int u = 0; u < NB * NB / 256; ++u) {
    const int e = tid + 256 * u;
    dst[e / NB][e % NB] = v[u];
  }
}

__device__ __forceinline__ void tile_store(double* dst, int64_t ld, const double (*src)[NB + 1]) {
  const int tid = tid_x();
#pragma unroll
  for (int u = 0; u < NB * NB / 256; ++u) {
    const int e = tid + 256 * u;
    dst[(int64_t)(e / NB) * ld + e % NB] = src[e / NB][e % NB];
  }
}

// The lower triangle of an LDS tile, zeros above the diagonal.
__device__ __forceinline__ void tile_store_lower(double* dst, int64_t ld, const double (*src)[NB + 1]) {
  const int tid = tid_x();
#pragma unroll
  for (int u = 0; u < NB * NB / 256; ++u) {
    const int e = tid + 256 * u;
    const int r = e / NB, c = e % NB;
    dst[(int64_t)r * ld + c] = c <= r ? src[r][c] : 0.0;
  }
}

// The 16 x 16 sub-tile st = 2 (row half) + (column half) of an LDS tile, in
// accumulator layout, and the same sub-tile of a product X Y^T.
__device__ __forceinline__ void sub_put_at(double (*T)[NB + 1], int st, v4d v) {
  const int lane = tid_x() & 63;
#pragma unroll
  for (int r = 0; r < 4; ++r) T[16 * (st >> 1) + 4 * r + (lane >> 4)][16 * (st & 1) + (lane & 15)] = v[r];
}
__device__ __forceinline__ v4d sub_get_at(const double (*T)[NB + 1], int st) {
  const int lane = tid_x() & 63;
  v4d v;
#pragma unroll
  for (int r = 0; r < 4; ++r) v[r] = T[16 * (st >> 1) + 4 * r + (lane >> 4)][16 * (st & 1) + (lane & 15)];
  return v;
}
__device__ __forceinline__ v4d sub_xyt_at(const double (*X)[NB + 1], const double (*Y)[NB + 1], int st) {
  const int lane = tid_x() & 63;
  return tile_xyt(X, Y, st, lane & 15, lane >> 4);
}

// This wavefront's sub-tile (st = wave index).
__device__ __forceinline__ void sub_put(double (*T)[NB + 1], v4d v) { sub_put_at(T, tid_x() >> 6, v); }
__device__ __forceinline__ v4d sub_get(const double (*T)[NB + 1]) { return sub_get_at(T, tid_x() >> 6); }
__device__ __forceinline__ v4d sub_xyt(const double (*X)[NB + 1], const double (*Y)[NB + 1]) {
  return sub_xyt_at(X, Y, tid_x() >> 6);
}

// In place: T <- T Y^T (a product of two LDS tiles written over its left factor).
__device__ __forceinline__ void tile_mul_t_inplace(double (*T)[NB + 1], const double (*Y)[NB + 1]) {
  const v4d v = sub_xyt(T, Y);
  __syncthreads();
  sub_put(T, v);
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

// Row blocks r0 .. r0 + nrows - 1 of X = L^-1 (nrows 1 or 2); workgroup jc
// forms the blocks of column block jc in row order, so a row sees the one
// above it (same workgroup, after a barrier).
__device__ void inverse_rows(int lw, int r0, int nrows, int jc, const double* __restrict__ L,
                             const double* __restrict__ Dinv, double* __restrict__ Xinv, double (*sS)[NB + 1],
                             double (*r0b)[NB + 1], double (*r1b)[NB + 1], double (*r2b)[NB + 1],
                             double (*r3b)[NB + 1]) {
  for (int rr = r0; rr < r0 + nrows; ++rr) {
    if (jc <= rr) inverse_block(lw, rr, jc, L, Dinv, Xinv, sS, r0b, r1b, r2b, r3b);
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void inverse_rows_kernel(int lw, int r0, int nrows, const double* __restrict__ L,
                                                           const double* __restrict__ Dinv,
                                                           double* __restrict__ Xinv) {
  __shared__ double sS[NB][NB + 1];
  __shared__ double red[4][NB][NB + 1];
  inverse_rows(lw, r0, nrows, blockIdx.x, L, Dinv, Xinv, sS, red[0], red[1], red[2], red[3]);
}

// The first two diagonal blocks (one workgroup): factor G_00, form
// L_10 = G_10 Dinv_0^T, update G_11 and factor it.
__global__ __launch_bounds__(256) void chol_first2_kernel(int lw, int l_true, const double* __restrict__ G,
                                                          double* __restrict__ L, double* __restrict__ Dinv,
                                                          const double* __restrict__ diag0, double tol,
                                                          uint32_t* flags) {
  __shared__ Tile s00, s10, s11, sD;
  __shared__ __align__(16) double scratch[kFactorScratch];
  __shared__ double s_thr[2 * NB];   // pivot thresholds of blocks 0 and 1
  const int T = lw / NB;
  const int wave = threadIdx.x >> 6;
  const double thr = threadIdx.x < 2 * NB ? pivot_thr(diag0, threadIdx.x, l_true, tol) : 0.0;
  tile_load(s00, G, lw);
  if (T > 1) {
    tile_load(s10, G + (int64_t)NB * lw, lw);
    tile_load(s11, G + (int64_t)NB * lw + NB, lw);
  }
  if (threadIdx.x < 2 * NB) s_thr[threadIdx.x] = thr;
  __syncthreads();
  if (wave == 0) factor_block<1>(&s00[0][0], &sD[0][0], scratch, s_thr, 0, l_true, flags);
  __syncthreads();
  tile_store_lower(L, lw, s00);
  tile_store(Dinv, NB, sD);
  if (T == 1) return;
  tile_mul_t_inplace(s10, sD);                 // L_10
  __syncthreads();
  tile_store(L + (int64_t)NB * lw, lw, s10);
  sub_put(s11, sub_get(s11) - sub_xyt(s10, s10));
  __syncthreads();
  if (wave == 0) factor_block<1>(&s11[0][0], &sD[0][0], scratch, s_thr + NB, NB, l_true, flags);
  __syncthreads();
  tile_store_lower(L + (int64_t)NB * lw + NB, lw, s11);
  tile_store(Dinv + NB * NB, NB, sD);
}

// Launch p (p even, p + 2 < T).  Blocks 0 .. nt-1: trailing tiles (i, j),
// p + 2 <= j <= i < T, in lower-triangle order (tile 0 = (p+2, p+2) is the
// diagonal workgroup, tiles 1 and 2 = (p+3, p+2), (p+3, p+3) belong to it);
// blocks nt .. nt + p + 1: column block jc = b - nt of X row blocks p, p + 1.
__global__ __launch_bounds__(256) void chol_panel2_kernel(int lw, int l_true, int p, double* __restrict__ G,
                                                          double* __restrict__ L, double* __restrict__ Dinv,
                                                          double* __restrict__ Xinv,
                                                          const double* __restrict__ diag0, double tol,
                                                          uint32_t* flags) {
  __shared__ Tile sD0, sD1, sL10, sA0, sA1, sB0, sB1, sU, sV, sW, sX;
  __shared__ __align__(16) double scratch[kFactorScratch];
  __shared__ int s_cnt;   // wavefronts 1 and 2 of the diagonal workgroup meet on it
  __shared__ double s_thr[2 * NB];   // pivot thresholds of the diagonal workgroup's blocks
  const int T = lw / NB;
  const int R = T - p - 2;
  const int nt = R * (R + 1) / 2;
  const int b = blockIdx.x;
  if (b >= nt) {   // inverse row blocks p, p + 1
    inverse_rows(lw, p, 2, b - nt, L, Dinv, Xinv, sU, sA0, sA1, sB0, sB1);
    return;
  }
  int di, dj;
  lower_tile(b, di, dj);
  if (b == 1 || b == 2) return;   // owned by the diagonal workgroup
  const int i = p + 2 + di, j = p + 2 + dj;
  const int wave = threadIdx.x >> 6;
  const double* Dp = Dinv + (int64_t)p * NB * NB;
  const bool diag = b == 0;
  const double thr = diag && threadIdx.x < 2 * NB ? pivot_thr(diag0, i * NB + threadIdx.x, l_true, tol) : 0.0;
  // every load first: Dinv_p, Dinv_{p+1}, L_{p+1,p}, the panel tiles of rows i (and j)
  tile_load(sD0, Dp, NB);
  tile_load(sD1, Dp + NB * NB, NB);
  tile_load(sL10, L + (int64_t)(p + 1) * NB * lw + p * NB, lw);
  tile_load(sA0, G + (int64_t)i * NB * lw + p * NB, lw);
  tile_load(sA1, G + (int64_t)i * NB * lw + (p + 1) * NB, lw);
  const bool two = diag && i + 1 < T;          // the diagonal workgroup also owns row i + 1
  const bool other = !diag && j != i;          // a distinct row j
  if (other || two) {
    const int r = two ? i + 1 : j;
    tile_load(sB0, G + (int64_t)r * NB * lw + p * NB, lw);
    tile_load(sB1, G + (int64_t)r * NB * lw + (p + 1) * NB, lw);
  }
  tile_load(sU, G + (int64_t)i * NB * lw + j * NB, lw);                  // G_ij (G_ii for the diagonal)
  if (two) {
    tile_load(sV, G + (int64_t)(i + 1) * NB * lw + i * NB, lw);          // G_{i+1,i}
    tile_load(sW, G + (int64_t)(i + 1) * NB * lw + (i + 1) * NB, lw);    // G_{i+1,i+1}
  }
  if (threadIdx.x == 0) s_cnt = 0;
  if (diag && threadIdx.x < 2 * NB) s_thr[threadIdx.x] = thr;
  __syncthreads();
  if (diag) {
    // Row i: panel tiles and the update of G_ii, one 16 x 16 sub-tile per wavefront.
    {
      const v4d a = sub_xyt(sA0, sD0);
      __syncthreads();
      sub_put(sA0, a);
    }
    __syncthreads();
    sub_put(sA1, sub_get(sA1) - sub_xyt(sA0, sL10));
    __syncthreads();
    {
      const v4d a = sub_xyt(sA1, sD1);
      __syncthreads();
      sub_put(sA1, a);
    }
    __syncthreads();
    tile_store(L + (int64_t)i * NB * lw + p * NB, lw, sA0);
    tile_store(L + (int64_t)i * NB * lw + (p + 1) * NB, lw, sA1);
    // (G_ii - L_{i,p} L_{i,p}^T) - L_{i,p+1} L_{i,p+1}^T: the one-launch chain's
    // order, so that both schedules give the same factor bit for bit
    sub_put(sU, (sub_get(sU) - sub_xyt(sA0, sA0)) - sub_xyt(sA1, sA1));
    __syncthreads();
    if (wave == 0) {
      factor_block<1>(&sU[0][0], &sX[0][0], scratch, s_thr, i * NB, l_true, flags);
    } else if (two && wave <= 2) {
      // Meanwhile wavefronts 1 and 2 take row i + 1, rows 16 h .. 16 h + 15 each
      // (h = wave - 1): its panel tiles and G_{i+1,i} need only these rows and
      // the finished tiles of row i, so each wavefront updates its rows in
      // place with no barrier; G_{i+1,i+1} needs both halves of the panel
      // tiles and waits for the other wavefront on an LDS counter.  Wavefront
      // 3 has no part in it.
      const int h = wave - 1;
      v4d c0 = sub_xyt_at(sB0, sD0, 2 * h), c1 = sub_xyt_at(sB0, sD0, 2 * h + 1);
      sub_put_at(sB0, 2 * h, c0);
      sub_put_at(sB0, 2 * h + 1, c1);
      c0 = sub_get_at(sB1, 2 * h) - sub_xyt_at(sB0, sL10, 2 * h);
      c1 = sub_get_at(sB1, 2 * h + 1) - sub_xyt_at(sB0, sL10, 2 * h + 1);
      sub_put_at(sB1, 2 * h, c0);
      sub_put_at(sB1, 2 * h + 1, c1);
      c0 = sub_xyt_at(sB1, sD1, 2 * h);
      c1 = sub_xyt_at(sB1, sD1, 2 * h + 1);
      sub_put_at(sB1, 2 * h, c0);
      sub_put_at(sB1, 2 * h + 1, c1);
#pragma unroll
      for (int c = 0; c < 2; ++c)
        sub_put_at(sV, 2 * h + c,
                   (sub_get_at(sV, 2 * h + c) - sub_xyt_at(sB0, sA0, 2 * h + c)) - sub_xyt_at(sB1, sA1, 2 * h + c));
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      if ((threadIdx.x & 63) == 0) __hip_atomic_fetch_add(&s_cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      while (__hip_atomic_load(&s_cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < 2) __builtin_amdgcn_s_sleep(1);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      // the lower sub-tiles of G_{i+1,i+1} (the factor reads no entry above the diagonal)
      const int st0 = h == 0 ? 0 : 2;
      sub_put_at(sW, st0, (sub_get_at(sW, st0) - sub_xyt_at(sB0, sB0, st0)) - sub_xyt_at(sB1, sB1, st0));
      if (h == 0) sub_put_at(sW, 3, (sub_get_at(sW, 3) - sub_xyt_at(sB0, sB0, 3)) - sub_xyt_at(sB1, sB1, 3));
    }
    __syncthreads();
    tile_store_lower(L + (int64_t)i * NB * lw + i * NB, lw, sU);
    tile_store(Dinv + (int64_t)i * NB * NB, NB, sX);
    if (!two) return;
    tile_store(L + (int64_t)(i + 1) * NB * lw + p * NB, lw, sB0);
    tile_store(L + (int64_t)(i + 1) * NB * lw + (p + 1) * NB, lw, sB1);
    tile_mul_t_inplace(sV, sX);                  // L_{i+1,i}
    __syncthreads();
    tile_store(L + (int64_t)(i + 1) * NB * lw + i * NB, lw, sV);
    sub_put(sW, sub_get(sW) - sub_xyt(sV, sV));
    __syncthreads();
    // the Dinv tile of panel p is no longer read: it receives the inverse of block i + 1
    if (wave == 0) factor_block<1>(&sW[0][0], &sD0[0][0], scratch, s_thr + NB, (i + 1) * NB, l_true, flags);
    __syncthreads();
    tile_store_lower(L + (int64_t)(i + 1) * NB * lw + (i + 1) * NB, lw, sW);
    tile_store(Dinv + (int64_t)(i + 1) * NB * NB, NB, sD0);
    return;
  }
  // trailing tile (i, j): panel p: L_{r,p} = G_{r,p} Dinv_p^T for r = i (and j)
  {
    const v4d a = sub_xyt(sA0, sD0);
    const v4d c = other ? sub_xyt(sB0, sD0) : a;
    __syncthreads();
    sub_put(sA0, a);
    if (other) sub_put(sB0, c);
  }
  __syncthreads();
  // panel p + 1: L_{r,p+1} = (G_{r,p+1} - L_{r,p} L_{p+1,p}^T) Dinv_{p+1}^T
  sub_put(sA1, sub_get(sA1) - sub_xyt(sA0, sL10));
  if (other) sub_put(sB1, sub_get(sB1) - sub_xyt(sB0, sL10));
  __syncthreads();
  {
    const v4d a = sub_xyt(sA1, sD1);
    const v4d c = other ? sub_xyt(sB1, sD1) : a;
    __syncthreads();
    sub_put(sA1, a);
    if (other) sub_put(sB1, c);
  }
  __syncthreads();
  // G_ij -= L_{i,p} L_{j,p}^T + L_{i,p+1} L_{j,p+1}^T;  column p + 2 writes the panel tiles of row i
  const double (*J0)[NB + 1] = other ? sB0 : sA0;
  const double (*J1)[NB + 1] = other ? sB1 : sA1;
  const v4d g = sub_get(sU) - (sub_xyt(sA0, J0) + sub_xyt(sA1, J1));
  sub_put(sU, g);
  __syncthreads();
  tile_store(G + (int64_t)i * NB * lw + j * NB, lw, sU);
  if (j == p + 2) {
    tile_store(L + (int64_t)i * NB * lw + p * NB, lw, sA0);
    tile_store(L + (int64_t)i * NB * lw + (p + 1) * NB, lw, sA1);
  }
}

// ------------------------------------------------ one-launch Cholesky chain --
// The schedule of the launches above as one grid whose workgroups keep a
// role for the whole factorisation and wait for each other on three
// progress counters in global memory (prog[0..2]) instead of launch
// boundaries:
//   workgroup 0      the diagonal chain: blocks 0 and 1, then for p = 0, 2, ...
//                    the panel rows i = p + 2, p + 3 and their diagonal blocks
//                    (the diagonal workgroup's part of launch p); prog[0]
//                    counts its finished steps, prog[2] the steps whose Dinv_i
//                    and L_{i+1,i} are out (before block i + 1 is factored);
//   1 .. ntr         one trailing tile (i, j), 2 <= j <= i, each: the update
//                    of the tile by panels p, p + 1 for every p it trails
//                    (the tile stays in LDS between steps); prog[1] counts
//                    finished (tile, step) pairs;
//   ntr + 1 ..       one column block jc of X = L^-1, each: row blocks p and
//                    p + 1 once the diagonal blocks p, p + 1 are factored.
// Step p of a trailing tile needs diagonal step p - 2 (Dinv_p and L_{p+1,p}
// for its first half, Dinv_{p+1} for the rest) and trailing step p - 2 (the
// final panel tiles of its rows).  Diagonal step p + 2 needs trailing step
// p: wavefronts 1 - 3 of workgroup 0 wait for it and fetch that step's
// tiles while wavefront 0 factors the second block of step p.  Every
// workgroup must be resident at once: the host launches it only when the
// grid fits the compute units (one workgroup per CU by its LDS).  Every wait
// is bounded; an overrun raises LRAMM_FLAG_STALL (the factor is then not
// valid) instead of hanging.
constexpr uint32_t kChainSpin = 1u << 18;

__device__ __forceinline__ void chain_wait(const uint32_t* ctr, uint32_t target, uint32_t* flags) {
  uint32_t n = 0;
  while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    if (++n > kChainSpin) {
      if (flags && (threadIdx.x & 63) == 0) atomicOr(flags, LRAMM_FLAG_STALL);
      break;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// This workgroup's global writes so far made visible, then *ctr += 1: every
// wavefront's agent-scope release (its stores written back and complete)
// comes before the barrier, so the counter moves only after all of them.
__device__ __forceinline__ void chain_signal(uint32_t* ctr) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Trailing tiles of step p (p even): (i, j), p + 2 <= j <= i < T, less the
// ones the diagonal workgroup owns, (p+2, p+2) and, when p + 3 < T,
// (p+3, p+2), (p+3, p+3).  chain_done(p) = those of steps 0, 2, .., p.
__device__ __forceinline__ uint32_t chain_done(int T, int p) {
  uint32_t s = 0;
  for (int q = 0; q <= p; q += 2) {
    const int R = T - q - 2;
    if (R >= 1) s += (uint32_t)(R * (R + 1) / 2 - (R >= 2 ? 3 : 1));
  }
  return s;
}

// Global 32 x 32 tiles -> LDS by one wavefront: rows 2u, 2u + 1 per step,
// every load of the NT tiles issued before the first LDS write.
template <int NT>
__device__ __forceinline__ void tiles_load_wave(double (*d0)[NB + 1], const double* s0, double (*d1)[NB + 1],
                                                const double* s1, double (*d2)[NB + 1], const double* s2,
                                                int64_t ld) {
  const int lane = tid_x() & 63;
  const int r = lane >> 5, c = lane & 31;
  double v[NT][16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int64_t o = (int64_t)(2 * u + r) * ld + c;
    v[0][u] = s0[o];
    if (NT > 1) v[NT > 1 ? 1 : 0][u] = s1[o];
    if (NT > 2) v[NT > 2 ? 2 : 0][u] = s2[o];
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    d0[2 * u + r][c] = v[0][u];
    if (NT > 1) d1[2 * u + r][c] = v[NT > 1 ? 1 : 0][u];
    if (NT > 2) d2[2 * u + r][c] = v[NT > 2 ? 2 : 0][u];
  }
}

// LDS tile -> global by one wavefront (LOWER: zeros above the diagonal).
template <bool LOWER>
__device__ __forceinline__ void tile_store_wave(double* dst, int64_t ld, const double (*src)[NB + 1]) {
  const int lane = tid_x() & 63;
  const int r = lane >> 5, c = lane & 31;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int row = 2 * u + r;
    const double v = src[row][c];
    dst[(int64_t)row * ld + c] = (!LOWER || c <= row) ? v : 0.0;
  }
}

// T[st] -= (X Y^T)[st] for one 16 x 16 sub-tile, by one wavefront.
__device__ __forceinline__ void sub_sub_xyt(double (*T)[NB + 1], const double (*X)[NB + 1],
                                            const double (*Y)[NB + 1], int st) {
  sub_put_at(T, st, sub_get_at(T, st) - sub_xyt_at(X, Y, st));
}

// Spin (LDS) until *cnt >= target; workgroup-scope acquire.
__device__ __forceinline__ void lds_wait(const int* cnt, int target) {
  while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < target) __builtin_amdgcn_s_sleep(1);
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}
// Workgroup-scope release, then *cnt += 1 (one lane).
__device__ __forceinline__ void lds_post(int* cnt) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  if ((tid_x() & 63) == 0) __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// The next item of a work queue in LDS (the same value on every lane).
__device__ __forceinline__ int lds_claim(int* cnt) {
  int q = 0;
  if ((tid_x() & 63) == 0) q = __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  return __builtin_amdgcn_readfirstlane(q);
}

// Wavefronts 1 - 3 of a workgroup meet: each adds one to *cnt and waits
// for target (3, 6, .. for the first, second, .. meeting since *cnt was 0).
__device__ __forceinline__ void meet3(int* cnt, int target) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  if ((tid_x() & 63) == 0) __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < target) __builtin_amdgcn_s_sleep(1);
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// inv_end: X row blocks 0 .. inv_end - 1 are formed (T, or T - 1 when the
// solve forms the last block of Q1 itself).  prog[0..2] must be zero at the
// launch.
//
// A step of the diagonal workgroup (rows i = p + 2, i + 1; p = -2 for the
// first two blocks) finds in LDS what the previous step prepared on its idle
// wavefronts: L_{i,p}, L_{i+1,p} (final), A1' = G_{i,p+1} - L_{i,p} L_{p+1,p}^T,
// U' = G_ii - L_{i,p} L_{i,p}^T, the raw G tiles of row i + 1, L_{p+1,p} and
// Dinv_{p+1}.  On the critical path it forms only L_{i,p+1} = A1' Dinv_{p+1}^T
// and U' - L_{i,p+1} L_{i,p+1}^T, and factors block i on wavefront 0;
// meanwhile wavefronts 1 - 3 apply panel column p to row i + 1 (B1', V', W'),
// wavefronts 1 - 2 finish that row with Dinv_{p+1}, and wavefront 3 writes
// the finished panel tiles, waits for trailing step p and fetches the next
// G_{in+1,in}, G_{in+1,in+1}.  It then forms L_{i+1,i} and W and factors block
// i + 1; during that factorisation wavefronts 1 - 3 write this step's tiles
// (wavefront 1 publishes Dinv_i and L_{i+1,i}), fetch the rest of the next
// row pair's G tiles, form L_{in,i} (and L_{in+1,i}) and apply column i to
// the next row's A1' and U'.
__global__ __launch_bounds__(256) void chol_chain_kernel(int lw, int l_true, double* __restrict__ G,
                                                         double* __restrict__ L, double* __restrict__ Dinv,
                                                         double* __restrict__ Xinv,
                                                         const double* __restrict__ diag0, double tol,
                                                         uint32_t* flags, uint32_t* prog, int inv_end) {
  __shared__ Tile pool[12];
  __shared__ __align__(16) double lscratch[kFactorScratch];
  __shared__ int s_cnt, s_cnt3, s_item, s_itemd, s_find;
  __shared__ double lthr[2][2 * NB];
  const int T = lw / NB;
  const int ntr = T > 2 ? (T - 2) * (T - 1) / 2 : 0;
  const int b = blockIdx.x;
  const int tid = threadIdx.x, wave = tid >> 6;

  if (b > ntr) {
    // ---- column block jc of X
    const int jc = b - 1 - ntr;
    for (int p = 0; p < inv_end; p += 2) {
      // z = 0 opaque to the compiler (as in the diagonal chain below)
      int z = 0;
      asm volatile("" : "+s"(z));
      Tile* P = pool + z;
      const int lwz = lw + z;
      const int nrows = inv_end - p < 2 ? inv_end - p : 2;
      if (jc > p + nrows - 1) continue;
      chain_wait(&prog[0], (uint32_t)(p / 2 + 1), flags);
      inverse_rows(lwz, p, nrows, jc, L, Dinv, Xinv, P[7], P[3], P[4], P[5], P[6]);
    }
    return;
  }

  if (b > 0) {
    // ---- trailing tile (i, j)
    int di, dj;
    lower_tile(b - 1, di, dj);
    const int i = 2 + di, j = 2 + dj;
    const int p_last = ((j - 2) / 2) * 2;
    const bool owned_last = (j % 2 == 0) ? (i == j || i == j + 1) : (i == j);
    const int last = owned_last ? p_last - 2 : p_last;
    const bool other = j != i;
    for (int p = 0; p <= last; p += 2) {
      // z = 0 opaque to the compiler (as in the diagonal chain below)
      int z = 0;
      asm volatile("" : "+s"(z));
      Tile* P = pool + z;
      double (*sD0)[NB + 1] = P[0], (*sD1)[NB + 1] = P[1], (*sL10)[NB + 1] = P[2];
      double (*sA0)[NB + 1] = P[3], (*sA1)[NB + 1] = P[4], (*sB0)[NB + 1] = P[5];
      double (*sB1)[NB + 1] = P[6], (*sU)[NB + 1] = P[7];
      const int lwz = lw + z;
      // first half: Dinv_p and L_{p+1,p} (published before the diagonal
      // workgroup factors block p + 1), then Dinv_{p+1}
      chain_wait(&prog[2], (uint32_t)(p / 2 + 1), flags);
      if (p >= 2) chain_wait(&prog[1], chain_done(T, p - 2), flags);
      const double* Dp = Dinv + (int64_t)p * NB * NB;
      tile_load(sD0, Dp, NB);
      tile_load(sL10, L + (int64_t)(p + 1) * NB * lwz + p * NB, lwz);
      tile_load(sA0, G + (int64_t)i * NB * lwz + p * NB, lwz);
      tile_load(sA1, G + (int64_t)i * NB * lwz + (p + 1) * NB, lwz);
      if (other) {
        tile_load(sB0, G + (int64_t)j * NB * lwz + p * NB, lwz);
        tile_load(sB1, G + (int64_t)j * NB * lwz + (p + 1) * NB, lwz);
      }
      if (p == 0) tile_load(sU, G + (int64_t)i * NB * lwz + j * NB, lwz);
      __syncthreads();
      {
        const v4d a = sub_xyt(sA0, sD0);
        const v4d c = other ? sub_xyt(sB0, sD0) : a;
        __syncthreads();
        sub_put(sA0, a);
        if (other) sub_put(sB0, c);
      }
      __syncthreads();
      sub_put(sA1, sub_get(sA1) - sub_xyt(sA0, sL10));
      if (other) sub_put(sB1, sub_get(sB1) - sub_xyt(sB0, sL10));
      chain_wait(&prog[0], (uint32_t)(p / 2 + 1), flags);
      tile_load(sD1, Dp + NB * NB, NB);
      __syncthreads();
      {
        const v4d a = sub_xyt(sA1, sD1);
        const v4d c = other ? sub_xyt(sB1, sD1) : a;
        __syncthreads();
        sub_put(sA1, a);
        if (other) sub_put(sB1, c);
      }
      __syncthreads();
      const double (*J0)[NB + 1] = other ? sB0 : sA0;
      const double (*J1)[NB + 1] = other ? sB1 : sA1;
      sub_put(sU, sub_get(sU) - (sub_xyt(sA0, J0) + sub_xyt(sA1, J1)));
      __syncthreads();
      if (j == p + 2) {
        tile_store(L + (int64_t)i * NB * lwz + p * NB, lwz, sA0);
        tile_store(L + (int64_t)i * NB * lwz + (p + 1) * NB, lwz, sA1);
      }
      if (p == last) tile_store(G + (int64_t)i * NB * lwz + j * NB, lwz, sU);
      chain_signal(&prog[1]);
    }
    return;
  }

  // ---- the diagonal chain.  Slots A0 .. U keep their role; the others
  // change role between steps (Dinv_{i+1} becomes the next Dinv_{p+1}, the
  // next row pair's G_{in+1,in} and G_{in+1,in+1} the next V and W).
  enum { kA0 = 0, kA1 = 1, kB0 = 2, kB1 = 3, kU = 4 };
  int rD1 = 5, rD0 = 6, rX = 7, rV = 8, rW = 9, rPV = 10, rPW = 11, cur = 0;
  if (tid < 2 * NB) lthr[0][tid] = pivot_thr(diag0, tid, l_true, tol);
  tile_load(pool[kU], G, lw);
  if (T > 1) {
    tile_load(pool[rV], G + (int64_t)NB * lw, lw);
    tile_load(pool[rW], G + (int64_t)NB * lw + NB, lw);
  }
  for (int p = -2;; p += 2) {
    // z = 0, opaque to the compiler: the LDS tile addresses and row strides
    // below are then formed inside the loop instead of hundreds of address
    // values being hoisted out of it and held in registers across the chain
    int z = 0;
    asm volatile("" : "+s"(z));
    Tile* P = pool + z;
    double (*A0)[NB + 1] = P[kA0], (*A1)[NB + 1] = P[kA1], (*B0)[NB + 1] = P[kB0], (*B1)[NB + 1] = P[kB1];
    double (*U)[NB + 1] = P[kU], (*D1)[NB + 1] = P[rD1], (*D0)[NB + 1] = P[rD0], (*X)[NB + 1] = P[rX];
    double (*V)[NB + 1] = P[rV], (*W)[NB + 1] = P[rW], (*PV)[NB + 1] = P[rPV], (*PW)[NB + 1] = P[rPW];
    double* scratch = lscratch + z;
    double* thr = &lthr[cur][0] + z;
    double* thrn = &lthr[cur ^ 1][0] + z;
    const int lwz = lw + z;
    const int i = p + 2;
    const bool two = i + 1 < T;
    const int in = i + 2;                        // the next step's first row
    const bool two_n = in + 1 < T;
    const double* Gi = G + (int64_t)in * NB * lwz;
    const double* Gn = Gi + (int64_t)NB * lwz;
    if (tid == 0) {
      s_cnt = 0;
      s_cnt3 = 0;
      s_item = 0;
      s_itemd = 0;
      s_find = 0;
    }
    __syncthreads();
    if (p >= 0) {
      // L_{i,p+1} = A1' Dinv_{p+1}^T, then U = U' - L_{i,p+1} L_{i,p+1}^T
      {
        const v4d a = sub_xyt(A1, D1);
        __syncthreads();
        sub_put(A1, a);
      }
      __syncthreads();
      sub_put(U, sub_get(U) - sub_xyt(A1, A1));
      __syncthreads();
    }
    if (wave == 0) {
      factor_block<1>(&U[0][0], &X[0][0], scratch, thr, i * NB, l_true, flags);
    } else {
      // Wavefronts 1 - 3 first finish what the previous step left of row
      // i + 1 (PV still holds L_{p+1,p}): B1' = G_{i+1,p+1} - L_{i+1,p} L_{p+1,p}^T,
      // V' = G_{i+1,i} - L_{i+1,p} L_{i,p}^T, W' = G_{i+1,i+1} - L_{i+1,p} L_{i+1,p}^T
      // (lower sub-tiles), one 16 x 16 sub-tile per item claimed in turn;
      // wavefront 3 writes the finished panel tiles of rows i, i + 1 first.
      if (wave == 3 && p >= 0) {
        tile_store_wave<false>(L + (int64_t)i * NB * lwz + p * NB, lwz, A0);
        tile_store_wave<false>(L + (int64_t)i * NB * lwz + (p + 1) * NB, lwz, A1);
        if (two) tile_store_wave<false>(L + (int64_t)(i + 1) * NB * lwz + p * NB, lwz, B0);
      }
      const int ndef = (p >= 0 && two) ? 11 : 0;
      for (;;) {
        const int q = lds_claim(&s_itemd);
        if (q >= ndef) break;
        if (q < 4)
          sub_sub_xyt(B1, B0, PV, q);
        else if (q < 8)
          sub_sub_xyt(V, B0, A0, q - 4);
        else
          sub_sub_xyt(W, B0, B0, q == 8 ? 0 : q - 7);
        lds_post(&s_find);
      }
      lds_wait(&s_find, ndef);
      if (wave == 3) {
        // once trailing step p is done, the next row pair's G tiles that go to
        // free slots (the barrier after this factorisation passes the wait on
        // to the other wavefronts)
        if (two && in < T) {
          if (p >= 0) chain_wait(&prog[1], chain_done(T, p), flags);
          if (two_n) tiles_load_wave<2>(PV, Gn + in * NB, PW, Gn + (in + 1) * NB, PW, nullptr, lwz);
        }
      } else if (p >= 0 && two) {
        // wavefronts 1 and 2: row i + 1, rows 16 h .. 16 h + 15 each (h = wave
        // - 1): L_{i+1,p+1} = B1' Dinv_{p+1}^T and V' - L_{i+1,p+1} L_{i,p+1}^T
        // need only these rows; W needs both halves and waits for the other
        const int h = wave - 1;
        const v4d c0 = sub_xyt_at(B1, D1, 2 * h), c1 = sub_xyt_at(B1, D1, 2 * h + 1);
        sub_put_at(B1, 2 * h, c0);
        sub_put_at(B1, 2 * h + 1, c1);
        sub_sub_xyt(V, B1, A1, 2 * h);
        sub_sub_xyt(V, B1, A1, 2 * h + 1);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        if ((tid & 63) == 0) __hip_atomic_fetch_add(&s_cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        while (__hip_atomic_load(&s_cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < 2) __builtin_amdgcn_s_sleep(1);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        // the lower sub-tiles of W (the factor reads no entry above the diagonal)
        sub_sub_xyt(W, B1, B1, h == 0 ? 0 : 2);
        if (h == 0) sub_sub_xyt(W, B1, B1, 3);
      }
    }
    __syncthreads();
    if (!two) {
      tile_store_lower(L + (int64_t)i * NB * lwz + i * NB, lwz, U);
      tile_store(Dinv + (int64_t)i * NB * NB, NB, X);
      chain_signal(&prog[0]);
      return;
    }
    tile_mul_t_inplace(V, X);                    // L_{i+1,i}
    __syncthreads();
    sub_put(W, sub_get(W) - sub_xyt(V, V));
    __syncthreads();
    // the updates by the panel column i (V = L_{i+1,i}) of the next row that
    // its first products need: A1' and U' (lower sub-tiles), one 16 x 16
    // sub-tile per item, claimed by wavefronts 1 - 3 in turn; row in + 1's
    // share waits for the next step's first factorisation (V stays in the
    // slot that becomes its PV)
    auto stage2 = [&]() {
      for (;;) {
        const int q = lds_claim(&s_item);
        if (q >= 7) break;
        if (q < 4)
          sub_sub_xyt(A1, A0, V, q);
        else
          sub_sub_xyt(U, A0, A0, q == 4 ? 0 : q - 3);
      }
    };
    if (wave == 0) {
      factor_block<1>(&W[0][0], &D0[0][0], scratch, thr + NB, (i + 1) * NB, l_true, flags);
      tile_store_wave<true>(L + (int64_t)(i + 1) * NB * lwz + (i + 1) * NB, lwz, W);
      tile_store_wave<false>(Dinv + (int64_t)(i + 1) * NB * NB, NB, D0);
    } else {
      // this step's finished tiles, each written by the wavefront that
      // refills its slot below; wavefront 1 publishes Dinv_i and L_{i+1,i}
      // at once (the first half of trailing step p + 2 needs only these)
      const int pn = i;
      if (wave == 1) {
        tile_store_wave<false>(Dinv + (int64_t)i * NB * NB, NB, X);
        tile_store_wave<false>(L + (int64_t)(i + 1) * NB * lwz + i * NB, lwz, V);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if ((tid & 63) == 0) __hip_atomic_fetch_add(&prog[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else if (wave == 2) {
        tile_store_wave<true>(L + (int64_t)i * NB * lwz + i * NB, lwz, U);
        if (p >= 0) tile_store_wave<false>(L + (int64_t)(i + 1) * NB * lwz + (p + 1) * NB, lwz, B1);
      }
      if (in < T) {
        // the rest of the next step's G tiles (trailing step p was waited
        // for by wavefront 3 before the last barrier)
        if (wave == 3) {
          tiles_load_wave<2>(A0, Gi + pn * NB, A1, Gi + (pn + 1) * NB, A1, nullptr, lwz);
          thrn[tid - 192] = pivot_thr(diag0, in * NB + (tid - 192), l_true, tol);
        } else if (wave == 2) {
          if (two_n)
            tiles_load_wave<3>(U, Gi + in * NB, B0, Gn + pn * NB, B1, Gn + (pn + 1) * NB, lwz);
          else
            tiles_load_wave<1>(U, Gi + in * NB, U, nullptr, U, nullptr, lwz);
        }
        meet3(&s_cnt3, 3);
        // L_{in,pn} = G_{in,pn} Dinv_pn^T (and row in + 1), in place: every
        // product first, then the writes
        const int n1 = two_n ? 8 : 4;
        v4d r1[3];
#pragma unroll
        for (int u = 0; u < 3; ++u) {
          const int q = wave - 1 + 3 * u;
          if (q < n1) r1[u] = sub_xyt_at(q < 4 ? A0 : B0, X, q & 3);
        }
        meet3(&s_cnt3, 6);
#pragma unroll
        for (int u = 0; u < 3; ++u) {
          const int q = wave - 1 + 3 * u;
          if (q < n1) sub_put_at(q < 4 ? A0 : B0, q & 3, r1[u]);
        }
        meet3(&s_cnt3, 9);
        stage2();
      }
    }
    __syncthreads();
    if (in >= T) {
      chain_signal(&prog[0]);
      return;
    }
    // Dinv_{i+1} is the next step's Dinv_{p+1}; G_{in+1,in}, G_{in+1,in+1} its
    // V, W (their updates by panel column i still to come) and L_{i+1,i} its PV
    int t = rD1;
    rD1 = rD0;
    rD0 = t;
    t = rV;
    rV = rPV;
    rPV = t;
    t = rW;
    rW = rPW;
    rPW = t;
    cur ^= 1;
    chain_signal(&prog[0]);
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
// panels), used only by the gated fallback of the second pass.  sS, sX (one
// tile each) and scratch (kFactorScratch + NB doubles, 16-byte aligned: the
// factor's columns and the block's pivot thresholds) are LDS buffers of the
// caller.
__device__ void chol_single_wg(int lw, int l_true, double* __restrict__ G, double* __restrict__ L,
                               double* __restrict__ Dinv, const double* __restrict__ diag0, double tol,
                               uint32_t* flags, double (*sS)[NB + 1], double (*sX)[NB + 1], double* scratch) {
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
    double* thr = scratch + kFactorScratch;
    if (tid < NB) thr[tid] = pivot_thr(diag0, p * NB + tid, l_true, tol);
    __syncthreads();
    double* Dp = Dinv + (int64_t)p * NB * NB;
    if (wave == 0) factor_block(&sS[0][0], &sX[0][0], scratch, thr, p * NB, l_true, flags);
    __syncthreads();
    tile_store_lower(L + (int64_t)p * NB * lw + p * NB, lw, sS);
    tile_store(Dp, NB, sX);
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
  static_assert(kFactorScratch + NB <= 2 * NB * (NB + 1), "factor scratch and thresholds span red[1] and red[2]");
  chol_single_wg(lw, l_true, G2, L, Dinv, diag0, tol, flags, sS, red[3], &red[1][0][0]);
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
                                                     const uint32_t* __restrict__ cm1,
                                                     uint32_t* __restrict__ colmax) {
  __shared__ __align__(16) double red[5][NB][NB + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const uint32_t g = *gate;
  if (!(g & kGatePass2)) {
    // second pass skipped: Q is Q1, whose column maxima become the result's
    if (blockIdx.x == 0 && cm1 && colmax)
      for (int c = tid; c < l_true; c += 256) {
        uint32_t m = cm1[c];
#pragma unroll
        for (int q = 1; q < kCmSlices; ++q) m = max(m, cm1[(int64_t)q * lw + c]);
        colmax[c] = m;
      }
    return;
  }
  if (g & kGateFull) {
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
  double *G, *L, *Dinv, *diag0, *part, *W, *X;
  uint32_t* gate;
  uint32_t* prog;  // the chain kernel's three progress counters (gate + kProgWord)
  uint32_t* cm1;   // column maxima of fl32(|Q1|) (first pass), kCmSlices copies of lw words
  int nchunks;
  int64_t rows_per_chunk;
};

constexpr double kSeriesTau = 1e-5;     // |E| bound of the second-pass expansion (error O(tau^3))
// The second pass is skipped when every |E_ij| of the first pass is at most
// 2^-44, about the orthonormality the second pass itself reaches (l u for
// l of a few hundred): it would change Q by no more than its own rounding.
constexpr double kSkipTau = 0x1p-44;

// Row chunks of the Gram: about two workgroups per compute unit over the
// lower 32 x 32 tiles, each wavefront at least 4 rows.
// The Gram runs on 64 x 64 tiles (gram64_kernel) from four 32-blocks on.
static bool gram_wide(int lw) { return lw / NB >= 4; }

static size_t cholqr_bytes(int lw, int nc) {
  const size_t sq = (size_t)lw * lw;
  const size_t n = 4 * sq + (size_t)lw * NB + lw + (size_t)nc * sq + 32 + (size_t)kCmSlices * lw / 2 + 1;
  return n * sizeof(double) + 256;
}

// Row chunks of the Gram (at most 16, about two workgroups per compute unit
// over the lower tiles, each wavefront at least 4 rows), fewer when the
// partial sums must fit a workspace of budget bytes.
static void cholqr_layout(int64_t rows, int64_t l, int* lw_out, int* nchunks, int64_t* rpc,
                          size_t budget = (size_t)-1) {
  const int lw = (int)round_up(l, NB);
  const int Tn = lw / NB;
  const int T64 = (Tn + 1) / 2;
  const int ntri = gram_wide(lw) ? T64 * (T64 + 1) / 2 : Tn * (Tn + 1) / 2;
  int64_t want = 512 / ntri;
  if (want > 16) want = 16;
  while (want > 1 && cholqr_bytes(lw, (int)want) > budget) --want;
  if (want < 1) want = 1;
  int64_t r = round_up(ceil_div(rows, want), (int64_t)16);
  int64_t nc = ceil_div(rows, r);
  if (nc < 1) nc = 1;
  *lw_out = lw;
  *nchunks = (int)nc;
  *rpc = r;
}

size_t cholqr2_workspace(int64_t rows, int64_t l) {
  int lw, nc;
  int64_t rpc;
  cholqr_layout(rows, l, &lw, &nc, &rpc);
  return cholqr_bytes(lw, nc);
}

size_t cholqr2_workspace_min(int64_t rows, int64_t l) {
  (void)rows;
  return cholqr_bytes((int)round_up(l, NB), 1);
}

struct HookScope {
  const TimingHook* h;
  HookScope(const TimingHook* hook, int stage, int launches = 1) : h(hook) {
    if (h) h->begin(h->ctx, stage | (launches << 16));
  }
  ~HookScope() {
    if (h) h->end(h->ctx);
  }
};

template <typename T>
static lramm_status gram(int64_t rows, int lw, int l_true, const T* X, int64_t ldx, const CholWs& w, int mode,
                         hipStream_t s, const TimingHook* hook) {
  const int Tn = lw / NB;
  {
    HookScope hs(hook, SUB_CHOL_GRAM);
    if (gram_wide(lw)) {
      const int T64 = (Tn + 1) / 2;
      hipLaunchKernelGGL((gram64_kernel<T>), dim3(T64 * (T64 + 1) / 2, w.nchunks), dim3(256), 0, s, rows, lw, l_true,
                         X, ldx, w.part, w.rows_per_chunk);
    } else {
      hipLaunchKernelGGL((gram_kernel<T>), dim3(Tn * (Tn + 1) / 2, w.nchunks), dim3(256), 0, s, rows, lw, l_true, X,
                         ldx, w.part, w.rows_per_chunk);
    }
  }
  LRAMM_HIP(hipGetLastError());
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)ceil_div((int64_t)lw * lw, 256)), dim3(256), 0, s, lw,
                     l_true, w.nchunks, w.part, w.G, w.diag0, w.gate, w.cm1, mode, kSeriesTau, kSkipTau);
  LRAMM_HIP(hipGetLastError());
  return LRAMM_OK;
}

// Workgroups of the one-launch chain for Tn diagonal blocks: the diagonal
// chain, one per trailing tile (i, j), j >= 2, one per column block of L^-1.
static int chain_grid_of(int Tn) { return 1 + (Tn > 2 ? (Tn - 2) * (Tn - 1) / 2 : 0) + Tn; }

// Whether the chain's grid may be used: it must fit the compute units less a
// margin (its LDS allows one workgroup per CU), or half of that when two such
// grids may run at the same time.
bool chain_admits(int64_t l, int compute_units, int chain_mode) {
  const int Tn = (int)(round_up(l, NB) / NB);
  const int lim = compute_units - 16;
  if (chain_mode == CHAIN_EXCLUSIVE) return chain_grid_of(Tn) <= lim;
  if (chain_mode == CHAIN_SHARED) return chain_grid_of(Tn) <= lim / 2;
  return false;
}

static int device_compute_units() {
  static const int cus = [] {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return n;
  }();
  return cus;
}

// Cholesky of w.G into w.L, w.Dinv and X = L^-1: the one-launch chain, or
// (a grid too large to be resident at once) one launch per two panels.
// With skip_last_row (an odd block count whose last row block of X would
// need a launch of its own) that row block is left out: the solve forms the
// last block of Q1 from the others instead.
static lramm_status cholesky_inverse(int lw, int l_true, const CholWs& w, uint32_t* flags, hipStream_t s,
                                     const TimingHook* hook, bool skip_last_row, int chain_mode) {
  const double tol = 64.0 * (double)l_true * 0x1p-53;
  const int Tn = lw / NB;
  // one launch when every workgroup of the chain can be resident at once
  const int chain_grid = chain_grid_of(Tn);
  if (chain_admits(lw, device_compute_units(), chain_mode)) {
    const int inv_end = (skip_last_row && Tn % 2 == 1) ? Tn - 1 : Tn;
    {
      HookScope hs(hook, SUB_CHOL_PANEL, 1);
      hipLaunchKernelGGL(chol_chain_kernel, dim3(chain_grid), dim3(256), 0, s, lw, l_true, w.G, w.L, w.Dinv, w.X,
                         w.diag0, tol, flags, w.prog, inv_end);
    }
    LRAMM_HIP(hipGetLastError());
    return LRAMM_OK;
  }
  int p = 0;
  {
    // one timing pair over the whole chain of dependent launches
    HookScope hs(hook, SUB_CHOL_PANEL, 1 + (Tn - 1) / 2);
    hipLaunchKernelGGL(chol_first2_kernel, dim3(1), dim3(256), 0, s, lw, l_true, w.G, w.L, w.Dinv, w.diag0, tol,
                       flags);
    LRAMM_HIP(hipGetLastError());
    for (; p + 2 < Tn; p += 2) {
      const int R = Tn - p - 2;
      const int nb = R * (R + 1) / 2 + p + 2;
      hipLaunchKernelGGL(chol_panel2_kernel, dim3(nb), dim3(256), 0, s, lw, l_true, p, w.G, w.L, w.Dinv, w.X,
                         w.diag0, tol, flags);
      LRAMM_HIP(hipGetLastError());
    }
  }
  if (skip_last_row && Tn - p == 1) return LRAMM_OK;
  hipLaunchKernelGGL(inverse_rows_kernel, dim3(Tn), dim3(256), 0, s, lw, p, Tn - p, w.L, w.Dinv, w.X);
  LRAMM_HIP(hipGetLastError());
  return LRAMM_OK;
}

// Whether the tall-skinny product takes 32 rows per workgroup (RB = 2): the
// staged panel of 32 rows and the W tiles fit LDS, and 32-row workgroups
// still cover every CU (8192 x 416: 60 -> 49 us per solve with 32 rows;
// 4096 x 288: 22 us with 16 rows against 27 with 32).
static bool ts_two_halves(int64_t rows, int lw) {
  const int cus = device_compute_units();
  return (size_t)2 * TS_ROWS * ts_pitch(lw) * sizeof(double) + ts_stage_lds() <= (size_t)160 * 1024 &&
         ceil_div(rows, (int64_t)(2 * TS_ROWS)) >= (cus > 0 ? cus : 256);
}

template <typename T, bool ADD>
static lramm_status tsmul(int64_t rows, int lw, int ncols, const T* X, int64_t ldx, const double* W, double* Q,
                          int64_t ldq, int zero_to, hipStream_t s, const TimingHook* hook,
                          uint32_t* colmax = nullptr, const uint32_t* gate = nullptr,
                          const double* Ltri = nullptr, const double* Dlast = nullptr, int cm_stride = 0,
                          const TsCodes& tc = TsCodes{}) {
  constexpr size_t kMaxLds = 160 * 1024;
  static bool attr_set = false;
  if (!attr_set) {   // up to 160 KiB of LDS
    LRAMM_HIP(hipFuncSetAttribute((const void*)tsmul_kernel<T, ADD, false>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds));
    LRAMM_HIP(hipFuncSetAttribute((const void*)tsmul_kernel<T, ADD, true>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds));
    LRAMM_HIP(hipFuncSetAttribute((const void*)tsmul_kernel<T, ADD, true, 2>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds));
    attr_set = true;
  }
  HookScope hs(hook, ADD ? SUB_CHOL_APPLY : SUB_CHOL_SOLVE);
  // 4-element vector loads need every row start aligned to 4 elements
  const int vec = ((uintptr_t)X % (4 * sizeof(T)) == 0 && ldx % 4 == 0) ? 1 : 0;
  // 32 rows per workgroup when their panel and the W tiles fit
  const size_t shm2 = (size_t)2 * TS_ROWS * ts_pitch(lw) * sizeof(double);
  if (!Ltri && ts_two_halves(rows, lw)) {
    const dim3 grid2((unsigned)ceil_div(rows, (int64_t)(2 * TS_ROWS)));
    hipLaunchKernelGGL((tsmul_kernel<T, ADD, true, 2>), grid2, dim3(TS_WAVES * 64), shm2 + ts_stage_lds(), s, rows,
                       lw, ncols, X, ldx, W, Q, ldq, zero_to, vec, colmax, cm_stride, gate, Ltri, Dlast, tc);
    LRAMM_HIP(hipGetLastError());
    return LRAMM_OK;
  }
  size_t shm = (size_t)TS_ROWS * ts_pitch(lw) * sizeof(double);
  if (Ltri) shm = ts_solve_last_lds(lw);
  const dim3 grid((unsigned)ceil_div(rows, (int64_t)TS_ROWS)), block(TS_WAVES * 64);
  // W staged through LDS when the tiles fit beside the row panel
  if (shm + ts_stage_lds() <= kMaxLds)
    hipLaunchKernelGGL((tsmul_kernel<T, ADD, true>), grid, block, shm + ts_stage_lds(), s, rows, lw, ncols, X, ldx, W,
                       Q, ldq, zero_to, vec, colmax, cm_stride, gate, Ltri, Dlast, tc);
  else
    hipLaunchKernelGGL((tsmul_kernel<T, ADD, false>), grid, block, shm, s, rows, lw, ncols, X, ldx, W, Q, ldq,
                       zero_to, vec, colmax, cm_stride, gate, Ltri, Dlast, tc);
  LRAMM_HIP(hipGetLastError());
  return LRAMM_OK;
}

// R = Q^T Y on and above the diagonal, zero below: the triangular factor of
// Y = Q R for the orthonormal Q of a Cholesky QR of Y (R = Q^T Q R).  One
// workgroup per 32 x 32 tile of R; rows of Q and Y pass through LDS in chunks
// of 64, and each thread sums its 4 entries over the rows in row order
// (FP64 fused multiply-adds, the same order on every call).
constexpr int kRChunk = 64;

template <typename T>
__global__ __launch_bounds__(256) void r_factor_kernel(int64_t rows, int l, const double* __restrict__ Q, int64_t ldq,
                                                       const T* __restrict__ Y, int64_t ldy, double* __restrict__ R,
                                                       int64_t ldr) {
  __shared__ double sQ[kRChunk][33];
  __shared__ double sY[kRChunk][33];
  const int tb = (l + 31) / 32;
  const int bi = blockIdx.x / tb, bj = blockIdx.x % tb;
  const int t = threadIdx.x;
  const int a = t & 31, b0 = (t >> 5) * 4;   // entries (32 bi + a, 32 bj + b0 .. b0 + 3)
  const int gi = 32 * bi + a;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (bi <= bj) {
    for (int64_t r0 = 0; r0 < rows; r0 += kRChunk) {
      // stage 64 rows of Q's column block bi and Y's column block bj
      for (int e = t; e < kRChunk * 32; e += 256) {
        const int rr = e >> 5, c = e & 31;
        const int64_t row = r0 + rr;
        const int qc = 32 * bi + c, yc = 32 * bj + c;
        sQ[rr][c] = (row < rows && qc < l) ? Q[row * ldq + qc] : 0.0;
        sY[rr][c] = (row < rows && yc < l) ? (double)Y[row * ldy + yc] : 0.0;
      }
      __syncthreads();
#pragma unroll 4
      for (int rr = 0; rr < kRChunk; ++rr) {
        const double q = sQ[rr][a];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] = fma(q, sY[rr][b0 + u], acc[u]);
      }
      __syncthreads();
    }
  }
  if (gi < l)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int gj = 32 * bj + b0 + u;
      if (gj < l) R[(int64_t)gi * ldr + gj] = gi <= gj ? acc[u] : 0.0;
    }
}

lramm_status launch_r_factor(int64_t rows, int64_t l, const void* Y, int64_t ldy, int ytype, const double* Q,
                             int64_t ldq, double* R, int64_t ldr, hipStream_t s) {
  const int tb = (int)ceil_div(l, (int64_t)32);
  const dim3 grid((unsigned)(tb * tb));
  if (ytype == LRAMM_F32)
    hipLaunchKernelGGL(r_factor_kernel<float>, grid, dim3(256), 0, s, rows, (int)l, Q, ldq, (const float*)Y, ldy, R,
                       ldr);
  else if (ytype == LRAMM_F64)
    hipLaunchKernelGGL(r_factor_kernel<double>, grid, dim3(256), 0, s, rows, (int)l, Q, ldq, (const double*)Y, ldy,
                       R, ldr);
  else
    return LRAMM_E_UNSUPPORTED;
  LRAMM_HIP(hipGetLastError());
  return LRAMM_OK;
}

lramm_status launch_cholqr2(int64_t rows, int64_t l, const void* Y, int64_t ldy, int ytype, double* Q,
                            int64_t ldq, void* ws, size_t ws_bytes, uint32_t* flags, hipStream_t s,
                            const TimingHook* hook, uint32_t* colmax, int chain_mode, int passes,
                            const QCodesOut* qcodes) {
  if (qcodes) *qcodes->written = false;
  if (rows == 0 || l == 0) return LRAMM_OK;
  if (passes != 1 && passes != 2) return LRAMM_E_INVALID;
  int lw, nc;
  int64_t rpc;
  cholqr_layout(rows, l, &lw, &nc, &rpc, ws_bytes);
  if (ws_bytes < cholqr_bytes(lw, nc)) return LRAMM_E_WORKSPACE;
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
  w.gate = reinterpret_cast<uint32_t*>(p);
  w.prog = w.gate + kProgWord;
  p += 32;
  w.cm1 = reinterpret_cast<uint32_t*>(p);
  w.nchunks = nc;
  w.rows_per_chunk = rpc;
  const int lt = (int)l;
  // pass 1 on Y (columns at or past l are never read): Q1 = Y L1^-T, written
  // into Q (columns lw .. ldq-1 zero), with its column maxima when asked
  // (sliced copies that the second pass merges; one pass writes the
  // caller's maxima directly)
  const int zero_to = (int)ldq;
  uint32_t* cm1 = colmax ? (passes == 1 ? colmax : w.cm1) : nullptr;
  const int cm_stride = passes == 1 ? 0 : lw;
  // an odd block count leaves X's last row block to the solve, when its LDS
  // fits and the 32-row solve (faster than the last-block one) does not
  const int Tn1 = lw / NB;
  const bool solve_last = (Tn1 % 2 == 1) && ts_solve_last_lds(lw) <= 160 * 1024 && !ts_two_halves(rows, lw);
  const double* Ltri = solve_last ? w.L : nullptr;
  const double* Dlast = solve_last ? w.Dinv + (size_t)(Tn1 - 1) * NB * NB : nullptr;
  // one pass: the solve's Q is final, and it can write Q's bf16 codes too
  TsCodes tc{};
  if (passes == 1 && qcodes && ytype == LRAMM_F32 && round_up(l, (int64_t)64) >= lw) {
    tc.rows = qcodes->rows;
    tc.rpitch = qcodes->rpitch;
    tc.rpe = (int)round_up(l, (int64_t)64);
    tc.rscales = qcodes->rscales;
    tc.cols = qcodes->cols;
    tc.cpitch = qcodes->cpitch;
    tc.cpe = round_up(rows, (int64_t)64);
    tc.cscales = qcodes->cscales;
  }
  if (ytype == LRAMM_F32) {
    LRAMM_TRY(gram<float>(rows, lw, lt, (const float*)Y, ldy, w, 0, s, hook));
    LRAMM_TRY(cholesky_inverse(lw, lt, w, flags, s, hook, solve_last, chain_mode));
    LRAMM_TRY((tsmul<float, false>(rows, lw, lt, (const float*)Y, ldy, w.X, Q, ldq, zero_to, s, hook, cm1, nullptr,
                                   Ltri, Dlast, cm_stride, tc)));
    if (tc.rows) *qcodes->written = true;
  } else if (ytype == LRAMM_F64) {
    LRAMM_TRY(gram<double>(rows, lw, lt, (const double*)Y, ldy, w, 0, s, hook));
    LRAMM_TRY(cholesky_inverse(lw, lt, w, flags, s, hook, solve_last, chain_mode));
    LRAMM_TRY((tsmul<double, false>(rows, lw, lt, (const double*)Y, ldy, w.X, Q, ldq, zero_to, s, hook, cm1,
                                    nullptr, Ltri, Dlast, cm_stride)));
  } else {
    return LRAMM_E_UNSUPPORTED;
  }
  if (passes == 1) return LRAMM_OK;
  // pass 2 on Q1 (in place in Q): expansion of the near-identity factor, or
  // (gated) the full factor; skipped on the device when Q1 is already
  // orthonormal to the second pass's own accuracy (then the expansion kernel
  // hands the first pass's column maxima on)
  LRAMM_TRY(gram<double>(rows, lw, lt, Q, ldq, w, 1, s, hook));
  const int Tn = lw / NB;
  const double tol = 64.0 * (double)lt * 0x1p-53;
  {
    HookScope hs(hook, SUB_CHOL_SERIES);
    hipLaunchKernelGGL(series_kernel, dim3(Tn * (Tn + 1) / 2), dim3(256), 0, s, lw, lt, w.G, w.W, w.L, w.Dinv,
                       w.diag0, tol, flags, w.gate, cm1, colmax);
  }
  LRAMM_HIP(hipGetLastError());
  LRAMM_TRY((tsmul<double, true>(rows, lw, lw, Q, ldq, w.W, Q, ldq, zero_to, s, hook, colmax, w.gate)));
  return LRAMM_OK;
}

}  // namespace lramm
