// Quantisers of the LRAMM hot path (paper Sec. 3.1: symmetric linear
// quantiser, eqs. Quantization / get_lambda / Dequantization) for gfx950.
//
// Two layouts:
//   rows  -- each row of X is one vector; one wavefront owns a row, reads it
//            once for the absmax (wavefront max reduction) and again (from
//            L2) to write the codes; K-contiguous output.
//   cols  -- each column of X is one vector and the codes are written
//            transposed (cols x K).  Pass 1 reduces column maxima with
//            atomicMax on the absmax bit patterns (order independent, hence
//            deterministic); pass 2 quantises 64 x 64 tiles and transposes
//            them through LDS so that both the FP reads and the code writes
//            are coalesced; pass 3 turns the maxima into scales.
// HBM bound: bytes = FP input read (x2 for columns) + code bytes written.
#include "common.hpp"

namespace lramm {

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

lramm_status fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return LRAMM_OK;
  int blocks = (int)(ceil_div(n, 256) < 1024 ? ceil_div(n, 256) : 1024);
  hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks), dim3(256), 0, s, p, v, n);
  LRAMM_HIP(hipGetLastError());
  return LRAMM_OK;
}

// ------------------------------------------------------------------ codes --

// 4 consecutive elements (4-element aligned) as FP32, no bounds test.
template <typename T>
__device__ __forceinline__ void load4_full(const T* p, float v[4]) {
  if constexpr (sizeof(T) == 4) {
    float4 f = *reinterpret_cast<const float4*>(p);
    v[0] = f.x; v[1] = f.y; v[2] = f.z; v[3] = f.w;
  } else if constexpr (sizeof(T) == 2) {
    uint2 u = *reinterpret_cast<const uint2*>(p);
    v[0] = __uint_as_float(u.x << 16);
    v[1] = __uint_as_float(u.x & 0xffff0000u);
    v[2] = __uint_as_float(u.y << 16);
    v[3] = __uint_as_float(u.y & 0xffff0000u);
  } else {
    double4 d = *reinterpret_cast<const double4*>(p);
    v[0] = (float)d.x; v[1] = (float)d.y; v[2] = (float)d.z; v[3] = (float)d.w;
  }
}

template <typename T>
__device__ __forceinline__ void load4(const T* row, int64_t c0, int64_t cols, bool vec, float v[4], bool live[4]) {
  if (vec && c0 + 3 < cols) {
    load4_full<T>(row + c0, v);
#pragma unroll
    for (int j = 0; j < 4; ++j) live[j] = true;
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      live[j] = (c0 + j) < cols;
      v[j] = live[j] ? load_as_f32<T>(row + c0 + j) : 0.0f;
    }
  }
}

// ------------------------------------------------------------ row kernel --

template <typename T, int FMT>
__global__ __launch_bounds__(256) void quant_rows_kernel(int64_t rows, int64_t cols, const T* __restrict__ X,
                                                         int64_t ldx, uint8_t* __restrict__ Xq, int64_t pitch,
                                                         int64_t pelems, float* __restrict__ scales,
                                                         uint32_t* flags, int vec, uint32_t* zero,
                                                             int64_t zero_words) {
  // a buffer of zero_words words cleared on the way (saves the caller a launch)
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < zero_words; e += (int64_t)gridDim.x * 256) zero[e] = 0u;
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  const T* xr = X + row * ldx;
  uint8_t* qr = Xq + row * pitch;
  const float qmax = FMT == LRAMM_INT8 ? 127.0f : (FMT == LRAMM_INT4 ? 7.0f : 448.0f);

  float lam = 1.0f;
  if constexpr (FMT != LRAMM_BF16F) {
    unsigned amax = 0;
    for (int64_t c0 = (int64_t)lane * 4; c0 < cols; c0 += 256) {
      float v[4];
      bool live[4];
      load4<T>(xr, c0, cols, vec != 0, v, live);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (live[j]) amax = max(amax, abs_bits(v[j]));
    }
    unsigned mb = wave_max_u32(amax);             // bit order == value order for |x|
    float m = __uint_as_float(mb);
    if (mb >= 0x7f800000u) {
      if (lane == 0 && flags) atomicOr(flags, LRAMM_FLAG_NONFINITE);
    }
    QParams qp = qparams(m, qmax);
    lam = qp.lam;
    if (lane == 0) scales[row] = qp.d;
  } else {
    if (lane == 0) scales[row] = 1.0f;
  }

  for (int64_t c0 = (int64_t)lane * 4; c0 < pelems; c0 += 256) {
    float v[4];
    bool live[4];
    load4<T>(xr, c0, cols, vec != 0, v, live);
    if constexpr (FMT != LRAMM_BF16F) {
      if (lam == 0.0f) {
#pragma unroll
        for (int j = 0; j < 4; ++j) live[j] = false;
      }
    }
    encode4<FMT>(qr, c0, v, live, lam);
  }
}

// --------------------------------------------------------- column kernels --

// Column maxima of a band of rows: each lane owns 4 consecutive columns (a
// wavefront spans 256), the 4 wavefronts take every 4th row; away from the
// right edge the loads carry no test and 8 rows are in flight per wavefront.
// The band's maxima meet in LDS and go out with one atomicMax per column.
constexpr int kColmaxRows = 128;   // rows per column-max workgroup

// With rmax_bits, the maxima of the rows' 256-column pieces go to the rows'
// words by atomicMax as well (both maxima from one read of X).
template <typename T>
__global__ __launch_bounds__(256) void colmax_kernel(int64_t rows, int64_t cols, const T* __restrict__ X,
                                                     int64_t ldx, uint32_t* __restrict__ amax_bits,
                                                     int64_t rows_per_block, int vec,
                                                     uint32_t* __restrict__ rmax_bits = nullptr) {
  __shared__ unsigned sm[4][256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t cb = (int64_t)blockIdx.x * 256;
  const int64_t c0 = cb + 4 * lane;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < rows ? r0 + rows_per_block : rows;
  unsigned m[4] = {0u, 0u, 0u, 0u};
  int64_t r = r0 + w;
  auto row_max = [&](int64_t row, const float v[4]) {
    if (!rmax_bits) return;
    unsigned x = max(max(abs_bits(v[0]), abs_bits(v[1])), max(abs_bits(v[2]), abs_bits(v[3])));
    x = wave_max_u32(x);
    if (lane == 0 && x) atomicMax(rmax_bits + row, x);
  };
  if (vec && cb + 256 <= cols) {
    for (; r + 28 < r1; r += 32) {
      float v[8][4];
#pragma unroll
      for (int i = 0; i < 8; ++i) load4_full<T>(X + (r + 4 * i) * ldx + c0, v[i]);
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) m[j] = max(m[j], abs_bits(v[i][j]));
#pragma unroll
      for (int i = 0; i < 8; ++i) row_max(r + 4 * i, v[i]);
    }
  }
  for (; r < r1; r += 4) {
    float v[4];
    bool live[4];
    load4<T>(X + r * ldx, c0, cols, vec != 0, v, live);   // zero past cols
#pragma unroll
    for (int j = 0; j < 4; ++j) m[j] = max(m[j], abs_bits(v[j]));
    row_max(r, v);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) sm[w][4 * lane + j] = m[j];
  __syncthreads();
  const int t = threadIdx.x;
  const unsigned mx = max(max(sm[0][t], sm[1][t]), max(sm[2][t], sm[3][t]));
  if (cb + t < cols && mx) atomicMax(amax_bits + cb + t, mx);
}

// Quantise a 64 (K) x 64 (cols) tile and write it transposed.
// With Rq, the tile's row codes (row scales from rmax_bits) are written
// too, untransposed: one read of X gives both code matrices.  Rows of Rq
// hold rpitch bytes; tiles past cols (grid.x may extend over the row
// padding) write zero row codes and no column codes.
template <typename T, int FMT>
__global__ __launch_bounds__(256) void quant_cols_t_kernel(int64_t rows, int64_t cols, const T* __restrict__ X,
                                                           int64_t ldx, const uint32_t* __restrict__ amax_bits,
                                                           uint8_t* __restrict__ Xq, int64_t pitch,
                                                           float* __restrict__ scales_out, uint32_t* flags,
                                                           int vec, uint8_t* __restrict__ Rq = nullptr,
                                                           int64_t rpitch = 0,
                                                           const uint32_t* __restrict__ rmax_bits = nullptr,
                                                           float* __restrict__ rscales = nullptr) {
  // codes of the tile, transposed: sT[col][k]; 2 bytes per code for bf16
  __shared__ uint16_t sT[64][66];
  const int t = threadIdx.x;
  const int64_t col0 = (int64_t)blockIdx.x * 64;
  const int64_t k0 = (int64_t)blockIdx.y * 64;
  const float qmax = FMT == LRAMM_INT8 ? 127.0f : (FMT == LRAMM_INT4 ? 7.0f : 448.0f);
  // the first row of tiles also writes the scales (when the maxima live in a
  // separate buffer) and reports non-finite columns
  if (scales_out && blockIdx.y == 0 && t < 64 && col0 + t < cols) {
    if constexpr (FMT == LRAMM_BF16F) {
      scales_out[col0 + t] = 1.0f;
    } else {
      const uint32_t mb = amax_bits[col0 + t];
      scales_out[col0 + t] = qparams(__uint_as_float(mb), qmax).d;
      if (mb >= 0x7f800000u && flags) atomicOr(flags, LRAMM_FLAG_NONFINITE);
    }
  }
  if (Rq && blockIdx.x == 0 && t < 64 && k0 + t < rows) {
    if constexpr (FMT == LRAMM_BF16F) {
      rscales[k0 + t] = 1.0f;
    } else {
      const uint32_t mb = rmax_bits[k0 + t];
      rscales[k0 + t] = qparams(__uint_as_float(mb), qmax).d;
      if (mb >= 0x7f800000u && flags) atomicOr(flags, LRAMM_FLAG_NONFINITE);
    }
  }
  // reads: lane owns 4 consecutive columns (16 lanes span the tile's 64),
  // rows sub, sub + 16, sub + 32, sub + 48
  const int cg = t & 15, sub = t >> 4;
  const int64_t c4 = col0 + 4 * cg;
  float lam[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    lam[j] = 0.0f;
    if (c4 + j < cols) {
      if constexpr (FMT == LRAMM_BF16F) lam[j] = 1.0f;
      else lam[j] = qparams(__uint_as_float(amax_bits[c4 + j]), qmax).lam;
    }
  }
  float v[4][4];
  if (vec && k0 + 64 <= rows && col0 + 64 <= cols) {
#pragma unroll
    for (int i = 0; i < 4; ++i) load4_full<T>(X + (k0 + sub + 16 * i) * ldx + c4, v[i]);
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t r = k0 + sub + 16 * i;
      bool live[4];
      if (r < rows && c4 < cols) {
        load4<T>(X + r * ldx, c4, cols, vec != 0, v[i], live);
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) v[i][j] = 0.0f;
      }
    }
  }
  if (Rq) {
    // row codes of rows k0 + sub + 16 i, columns c4 .. c4 + 3 (zero past cols)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t r = k0 + sub + 16 * i;
      if (r >= rows) continue;
      float rl = 1.0f;
      if constexpr (FMT != LRAMM_BF16F) rl = qparams(__uint_as_float(rmax_bits[r]), qmax).lam;
      bool live[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) live[j] = c4 + j < cols && (FMT == LRAMM_BF16F || rl != 0.0f);
      encode4<FMT>(Rq + r * rpitch, c4, v[i], live, rl);
    }
  }
  if (col0 >= cols) return;   // a tile of row padding only
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      // rows past the end and columns with a zero lambda give code 0
      const float x = v[i][j];
      uint16_t code = 0;
      if (lam[j] != 0.0f) {
        if constexpr (FMT == LRAMM_INT8) {
          code = (uint16_t)(qcode(x, lam[j], qmax) & 0xff);
        } else if constexpr (FMT == LRAMM_INT4) {
          code = (uint16_t)(qcode(x, lam[j], qmax) & 0xf);
        } else if constexpr (FMT == LRAMM_FP8) {
          code = (uint16_t)e4m3_bits(__fmul_rn(x, lam[j]));
        } else {
          code = bf16_bits(x);
        }
      }
      sT[4 * cg + j][sub + 16 * i] = code;
    }
  __syncthreads();
  // write: output row = column of X, 64 elements of K starting at k0
  const int orow = t >> 2;           // 0..63
  const int part = t & 3;            // quarter of the 64-element chunk
  int64_t oc = (int64_t)blockIdx.x * 64 + orow;
  if (oc >= cols) return;
  uint8_t* dst = Xq + oc * pitch;
  if constexpr (FMT == LRAMM_INT8 || FMT == LRAMM_FP8) {
    uint32_t w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int kk = part * 16 + q * 4;
      w[q] = (uint32_t)sT[orow][kk] | ((uint32_t)sT[orow][kk + 1] << 8) | ((uint32_t)sT[orow][kk + 2] << 16) |
             ((uint32_t)sT[orow][kk + 3] << 24);
    }
    *reinterpret_cast<uint4*>(dst + k0 + part * 16) = make_uint4(w[0], w[1], w[2], w[3]);
  } else if constexpr (FMT == LRAMM_INT4) {
    uint32_t w[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      int kk = part * 16 + q * 8;
      uint32_t x = 0;
#pragma unroll
      for (int j = 0; j < 8; ++j) x |= ((uint32_t)sT[orow][kk + j]) << (4 * j);
      w[q] = x;
    }
    *reinterpret_cast<uint2*>(dst + k0 / 2 + part * 8) = make_uint2(w[0], w[1]);
  } else {
    uint32_t w[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      int kk = part * 16 + 2 * q;
      w[q] = (uint32_t)sT[orow][kk] | ((uint32_t)sT[orow][kk + 1] << 16);
    }
    uint4* d4 = reinterpret_cast<uint4*>(dst + 2 * k0 + part * 32);
    d4[0] = make_uint4(w[0], w[1], w[2], w[3]);
    d4[1] = make_uint4(w[4], w[5], w[6], w[7]);
  }
}

// The K-slice sum of a product (slices [nsplit][rows][cols], FP32) written
// once as C (rows x cols, ldc) and once as bf16 codes of C's columns,
// transposed: codes row c holds column c of C (pitch bytes, zero past rows),
// with unit scales.  The sums are formed in split order from zero, as the
// plain slice sum forms them, so C and the codes are those of the sum-then-
// quantise passes to the bit, with one read of the slices instead of three
// passes.  Tiles of 64 (rows) x 64 (cols), as in quant_cols_t_kernel.
__global__ __launch_bounds__(256) void bf16_cols_from_parts_kernel(int64_t rows, int64_t cols,
                                                                   const float* __restrict__ parts, int nsplit,
                                                                   float* __restrict__ C, int64_t ldc,
                                                                   uint8_t* __restrict__ Xq, int64_t pitch,
                                                                   float* __restrict__ scales, int cvec) {
  __shared__ uint16_t sT[64][66];
  const int t = threadIdx.x;
  const int64_t col0 = (int64_t)blockIdx.x * 64;
  const int64_t k0 = (int64_t)blockIdx.y * 64;
  const int64_t pstride = rows * cols;
  if (blockIdx.y == 0 && t < 64 && col0 + t < cols) scales[col0 + t] = 1.0f;
  const int cg = t & 15, sub = t >> 4;
  const int64_t c4 = col0 + 4 * cg;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t r = k0 + sub + 16 * i;
    float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (r < rows && c4 < cols) {
      const int64_t e0 = r * cols + c4;
      if ((cols & 3) == 0) {
        // a whole quad inside the row: 16-byte loads of each slice
        for (int k = 0; k < nsplit; ++k) {
          const float4 x = *reinterpret_cast<const float4*>(parts + k * pstride + e0);
          v[0] = __fadd_rn(v[0], x.x);
          v[1] = __fadd_rn(v[1], x.y);
          v[2] = __fadd_rn(v[2], x.z);
          v[3] = __fadd_rn(v[3], x.w);
        }
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (c4 + j < cols)
            for (int k = 0; k < nsplit; ++k) v[j] = __fadd_rn(v[j], parts[k * pstride + e0 + j]);
      }
      float* cr = C + r * ldc;
      if (cvec && c4 + 3 < cols) {
        *reinterpret_cast<float4*>(cr + c4) = make_float4(v[0], v[1], v[2], v[3]);
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (c4 + j < cols) cr[c4 + j] = v[j];
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
      sT[4 * cg + j][sub + 16 * i] = (r < rows && c4 + j < cols) ? bf16_bits(v[j]) : (uint16_t)0;
  }
  __syncthreads();
  // write: output row = column of C, 64 elements of K starting at k0
  const int orow = t >> 2;
  const int part = t & 3;
  const int64_t oc = col0 + orow;
  if (oc >= cols) return;
  uint32_t w[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int kk = part * 16 + 2 * q;
    w[q] = (uint32_t)sT[orow][kk] | ((uint32_t)sT[orow][kk + 1] << 16);
  }
  uint4* d4 = reinterpret_cast<uint4*>(Xq + oc * pitch + 2 * k0 + part * 32);
  d4[0] = make_uint4(w[0], w[1], w[2], w[3]);
  d4[1] = make_uint4(w[4], w[5], w[6], w[7]);
}

lramm_status launch_bf16_cols_from_parts(int64_t rows, int64_t cols, const float* parts, int nsplit, float* C,
                                         int64_t ldc, uint8_t* Xq, int64_t pitch, float* scales, hipStream_t s) {
  if (rows == 0 || cols == 0) return LRAMM_OK;
  const int64_t pe = pitch_elems(pitch, LRAMM_BF16F);
  if (pe < rows || pe % 64 != 0) return LRAMM_E_INVALID;
  const int cvec = (ldc % 4 == 0) && ((uintptr_t)C % 16 == 0) ? 1 : 0;
  const dim3 g((unsigned)ceil_div(cols, (int64_t)64), (unsigned)(pe / 64));
  hipLaunchKernelGGL(bf16_cols_from_parts_kernel, g, dim3(256), 0, s, rows, cols, parts, nsplit, C, ldc, Xq, pitch,
                     scales, cvec);
  LRAMM_HIP(hipGetLastError());
  return LRAMM_OK;
}

template <int FMT>
__global__ void col_scales_kernel(int64_t cols, float* scales, uint32_t* flags) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  if constexpr (FMT == LRAMM_BF16F) {
    scales[c] = 1.0f;
  } else {
    uint32_t b = __float_as_uint(scales[c]);
    if (b >= 0x7f800000u && flags) atomicOr(flags, LRAMM_FLAG_NONFINITE);
    const float qmax = FMT == LRAMM_INT8 ? 127.0f : (FMT == LRAMM_INT4 ? 7.0f : 448.0f);
    scales[c] = qparams(__uint_as_float(b), qmax).d;
  }
}
// Row vectors held in registers: one read of the row (all loads issued
// together), the wavefront maximum, then the codes from the registers.  NV
// groups of 4 elements per lane cover 256 NV elements of the padded row.
template <typename T, int FMT, int NV>
__global__ __launch_bounds__(256) void quant_rows_reg_kernel(int64_t rows, int64_t cols, const T* __restrict__ X,
                                                             int64_t ldx, uint8_t* __restrict__ Xq, int64_t pitch,
                                                             int64_t pelems, float* __restrict__ scales,
                                                             uint32_t* flags, int vec, uint32_t* zero,
                                                             int64_t zero_words) {
  // a buffer of zero_words words cleared on the way (saves the caller a launch)
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < zero_words; e += (int64_t)gridDim.x * 256) zero[e] = 0u;
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  const T* xr = X + row * ldx;
  uint8_t* qr = Xq + row * pitch;
  const float qmax = FMT == LRAMM_INT8 ? 127.0f : (FMT == LRAMM_INT4 ? 7.0f : 448.0f);
  float v[NV][4];
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    bool live[4];
    load4<T>(xr, (int64_t)(c * 64 + lane) * 4, cols, vec != 0, v[c], live);
  }
  float lam = 1.0f;
  if constexpr (FMT != LRAMM_BF16F) {
    unsigned amax = 0;
#pragma unroll
    for (int c = 0; c < NV; ++c)
#pragma unroll
      for (int j = 0; j < 4; ++j) amax = max(amax, abs_bits(v[c][j]));   // zero past cols
    unsigned mb = wave_max_u32(amax);             // bit order == value order for |x|
    if (mb >= 0x7f800000u) {
      if (lane == 0 && flags) atomicOr(flags, LRAMM_FLAG_NONFINITE);
    }
    QParams qp = qparams(__uint_as_float(mb), qmax);
    lam = qp.lam;
    if (lane == 0) scales[row] = qp.d;
  } else {
    if (lane == 0) scales[row] = 1.0f;
  }
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    const int64_t c0 = (int64_t)(c * 64 + lane) * 4;
    if (c0 < pelems) {
      bool live[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) live[j] = c0 + j < cols && (FMT == LRAMM_BF16F || lam != 0.0f);
      encode4<FMT>(qr, c0, v[c], live, lam);
    }
  }
}

// bf16 codes of a row-major matrix are the rounded values themselves (no
// maxima, every scale 1): 8 elements of one row per thread over the padded
// row, so that the grid covers every row with full wavefronts however few the
// rows are; zero past cols.  A buffer of zero_words words is cleared on the
// way, as in the row quantisers.
template <typename T>
__global__ __launch_bounds__(256) void bf16_rows_kernel(int64_t rows, int64_t cols, const T* __restrict__ X,
                                                        int64_t ldx, uint8_t* __restrict__ Xq, int64_t pitch,
                                                        int64_t pelems, float* __restrict__ scales, int vec,
                                                        uint32_t* zero, int64_t zero_words) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < zero_words; e += (int64_t)gridDim.x * 256) zero[e] = 0u;
  // 32-bit index arithmetic (the host checks that rows * pelems / 8 fits)
  const uint32_t per_row = (uint32_t)(pelems / 8);
  const uint32_t idx = blockIdx.x * 256u + threadIdx.x;
  if ((uint64_t)idx >= (uint64_t)rows * per_row) return;
  const uint32_t rw = idx / per_row;
  const int64_t row = rw;
  const int64_t c0 = (int64_t)(idx - rw * per_row) * 8;
  const T* xr = X + row * ldx;
  uint8_t* qr = Xq + row * pitch;
  float v[2][4];
  bool live[2][4];
  load4<T>(xr, c0, cols, vec != 0, v[0], live[0]);
  load4<T>(xr, c0 + 4, cols, vec != 0, v[1], live[1]);
  encode4<LRAMM_BF16F>(qr, c0, v[0], live[0], 1.0f);
  encode4<LRAMM_BF16F>(qr, c0 + 4, v[1], live[1], 1.0f);
  if (c0 == 0) scales[row] = 1.0f;
}

// ---------------------------------------------------------------- launch --

template <typename T, int FMT>
static lramm_status quantize_typed(int64_t rows, int64_t cols, const T* X, int64_t ldx, int transpose, uint8_t* Xq,
                                   int64_t pitch, float* scales, uint32_t* flags, hipStream_t s, uint32_t* amax_ws,
                                   bool amax_ready, uint32_t* zero, int64_t zero_words) {
  if (!transpose) {
    if (rows == 0) return zero_words > 0 ? fill_u32(zero, 0u, zero_words, s) : LRAMM_OK;
    int64_t pe = pitch_elems(pitch, FMT);
    bool vec = ((uintptr_t)X % (4 * sizeof(T)) == 0) && (ldx % 4 == 0);
    dim3 grid((unsigned)ceil_div(rows, 4));
    const int v = vec ? 1 : 0;
    // FP64 rows (Q for G2) stay on the register kernel: 7.5 against 8.9 us
    // for 8192 x 416
    if constexpr (FMT == LRAMM_BF16F && sizeof(T) <= 4) {
      if (rows * (pe / 8) < ((int64_t)1 << 31)) {
        const int64_t threads = rows * (pe / 8);
        hipLaunchKernelGGL((bf16_rows_kernel<T>), dim3((unsigned)ceil_div(threads, (int64_t)256)), dim3(256), 0, s,
                           rows, cols, X, ldx, Xq, pitch, pe, scales, v, zero, zero_words);
        LRAMM_HIP(hipGetLastError());
        return LRAMM_OK;
      }
    }
    const int64_t groups = ceil_div(pe, (int64_t)256);   // 4-element groups per lane
#define ROWS_REG(NV)                                                                                            \
  hipLaunchKernelGGL((quant_rows_reg_kernel<T, FMT, NV>), grid, dim3(256), 0, s, rows, cols, X, ldx, Xq, pitch, pe, \
                     scales, flags, v, zero, zero_words)
    if (groups <= 1) ROWS_REG(1);
    else if (groups <= 2) ROWS_REG(2);
    else if (groups <= 4) ROWS_REG(4);
    else if (groups <= 8) ROWS_REG(8);
    else if (groups <= 16) ROWS_REG(16);
    else if (groups <= 32 && sizeof(T) <= 4) ROWS_REG(32);
    else
      hipLaunchKernelGGL((quant_rows_kernel<T, FMT>), grid, dim3(256), 0, s, rows, cols, X, ldx, Xq, pitch, pe,
                         scales, flags, v, zero, zero_words);
#undef ROWS_REG
    LRAMM_HIP(hipGetLastError());
    return LRAMM_OK;
  }
  // column vectors, transposed output: cols x pitch
  if (zero_words > 0) LRAMM_TRY(fill_u32(zero, 0u, zero_words, s));
  if (cols == 0) return LRAMM_OK;
  const int cvec = ((uintptr_t)X % (4 * sizeof(T)) == 0) && (ldx % 4 == 0) ? 1 : 0;
  if (amax_ws) {
    // maxima in a caller-zeroed buffer (or already there): no fill, and the
    // quantise pass writes the scales itself
    if (FMT != LRAMM_BF16F && rows > 0 && !amax_ready) {
      dim3 g1((unsigned)ceil_div(cols, 256), (unsigned)ceil_div(rows, (int64_t)kColmaxRows));
      hipLaunchKernelGGL((colmax_kernel<T>), g1, dim3(256), 0, s, rows, cols, X, ldx, amax_ws, (int64_t)kColmaxRows,
                         cvec);
      LRAMM_HIP(hipGetLastError());
    }
    int64_t pe = pitch_elems(pitch, FMT);
    dim3 g2((unsigned)ceil_div(cols, 64), (unsigned)(pe / 64));
    hipLaunchKernelGGL((quant_cols_t_kernel<T, FMT>), g2, dim3(256), 0, s, rows, cols, X, ldx, amax_ws, Xq, pitch,
                       scales, flags, cvec);
    LRAMM_HIP(hipGetLastError());
    return LRAMM_OK;
  }
  if constexpr (FMT == LRAMM_BF16F) {
    // no maxima: the transposing pass writes the codes and the unit scales
    int64_t pe = pitch_elems(pitch, FMT);
    dim3 g2((unsigned)ceil_div(cols, 64), (unsigned)(pe / 64));
    hipLaunchKernelGGL((quant_cols_t_kernel<T, FMT>), g2, dim3(256), 0, s, rows, cols, X, ldx,
                       (const uint32_t*)nullptr, Xq, pitch, scales, flags, cvec);
    LRAMM_HIP(hipGetLastError());
    return LRAMM_OK;
  }
  uint32_t* amax = reinterpret_cast<uint32_t*>(scales);
  LRAMM_TRY(fill_u32(amax, 0u, cols, s));
  if (FMT != LRAMM_BF16F && rows > 0) {
    dim3 g1((unsigned)ceil_div(cols, 256), (unsigned)ceil_div(rows, (int64_t)kColmaxRows));
    hipLaunchKernelGGL((colmax_kernel<T>), g1, dim3(256), 0, s, rows, cols, X, ldx, amax, (int64_t)kColmaxRows, cvec);
    LRAMM_HIP(hipGetLastError());
  }
  int64_t pe = pitch_elems(pitch, FMT);
  dim3 g2((unsigned)ceil_div(cols, 64), (unsigned)(pe / 64));
  hipLaunchKernelGGL((quant_cols_t_kernel<T, FMT>), g2, dim3(256), 0, s, rows, cols, X, ldx, amax, Xq, pitch,
                     (float*)nullptr, (uint32_t*)nullptr, cvec);
  LRAMM_HIP(hipGetLastError());
  hipLaunchKernelGGL((col_scales_kernel<FMT>), dim3((unsigned)ceil_div(cols, 256)), dim3(256), 0, s, cols, scales,
                     flags);
  LRAMM_HIP(hipGetLastError());
  return LRAMM_OK;
}

// Both code matrices of X from two reads: the row and column maxima
// (skipped for bf16), then the row codes (rows x rpitch) and the transposed
// column codes (cols x cpitch).  rmax / cmax: caller-zeroed rows / cols words.
template <typename T, int FMT>
static lramm_status quantize_both_typed(int64_t rows, int64_t cols, const T* X, int64_t ldx, uint8_t* Rq,
                                        int64_t rpitch, float* rscales, uint8_t* Cq, int64_t cpitch,
                                        float* cscales, uint32_t* rmax, uint32_t* cmax, uint32_t* flags,
                                        hipStream_t s) {
  if (rows == 0 || cols == 0) return LRAMM_OK;
  const int cvec = ((uintptr_t)X % (4 * sizeof(T)) == 0) && (ldx % 4 == 0) ? 1 : 0;
  if (FMT != LRAMM_BF16F) {
    dim3 g1((unsigned)ceil_div(cols, 256), (unsigned)ceil_div(rows, (int64_t)kColmaxRows));
    hipLaunchKernelGGL((colmax_kernel<T>), g1, dim3(256), 0, s, rows, cols, X, ldx, cmax, (int64_t)kColmaxRows,
                       cvec, rmax);
    LRAMM_HIP(hipGetLastError());
  }
  const int64_t pe_c = pitch_elems(cpitch, FMT), pe_r = pitch_elems(rpitch, FMT);
  const int64_t tx = ceil_div(pe_r > cols ? pe_r : cols, (int64_t)64);
  dim3 g2((unsigned)tx, (unsigned)(pe_c / 64));
  hipLaunchKernelGGL((quant_cols_t_kernel<T, FMT>), g2, dim3(256), 0, s, rows, cols, X, ldx, cmax, Cq, cpitch,
                     cscales, flags, cvec, Rq, rpitch, rmax, rscales);
  LRAMM_HIP(hipGetLastError());
  return LRAMM_OK;
}

template <typename T>
static lramm_status quantize_both_fmt(int64_t rows, int64_t cols, const T* X, int64_t ldx, int fmt, uint8_t* Rq,
                                      int64_t rpitch, float* rscales, uint8_t* Cq, int64_t cpitch, float* cscales,
                                      uint32_t* rmax, uint32_t* cmax, uint32_t* flags, hipStream_t s) {
  switch (fmt) {
    case LRAMM_INT8: return quantize_both_typed<T, LRAMM_INT8>(rows, cols, X, ldx, Rq, rpitch, rscales, Cq, cpitch, cscales, rmax, cmax, flags, s);
    case LRAMM_INT4: return quantize_both_typed<T, LRAMM_INT4>(rows, cols, X, ldx, Rq, rpitch, rscales, Cq, cpitch, cscales, rmax, cmax, flags, s);
    case LRAMM_FP8: return quantize_both_typed<T, LRAMM_FP8>(rows, cols, X, ldx, Rq, rpitch, rscales, Cq, cpitch, cscales, rmax, cmax, flags, s);
    case LRAMM_BF16F: return quantize_both_typed<T, LRAMM_BF16F>(rows, cols, X, ldx, Rq, rpitch, rscales, Cq, cpitch, cscales, rmax, cmax, flags, s);
    default: return LRAMM_E_INVALID;
  }
}

template <typename T>
static lramm_status quantize_fmt(int64_t rows, int64_t cols, const T* X, int64_t ldx, int fmt, int transpose,
                                 uint8_t* Xq, int64_t pitch, float* scales, uint32_t* flags, hipStream_t s,
                                 uint32_t* amax_ws, bool amax_ready, uint32_t* zero, int64_t zero_words) {
  switch (fmt) {
    case LRAMM_INT8: return quantize_typed<T, LRAMM_INT8>(rows, cols, X, ldx, transpose, Xq, pitch, scales, flags, s, amax_ws, amax_ready, zero, zero_words);
    case LRAMM_INT4: return quantize_typed<T, LRAMM_INT4>(rows, cols, X, ldx, transpose, Xq, pitch, scales, flags, s, amax_ws, amax_ready, zero, zero_words);
    case LRAMM_FP8: return quantize_typed<T, LRAMM_FP8>(rows, cols, X, ldx, transpose, Xq, pitch, scales, flags, s, amax_ws, amax_ready, zero, zero_words);
    case LRAMM_BF16F: return quantize_typed<T, LRAMM_BF16F>(rows, cols, X, ldx, transpose, Xq, pitch, scales, flags, s, amax_ws, amax_ready, zero, zero_words);
    default: return LRAMM_E_INVALID;
  }
}

lramm_status launch_quantize(int64_t rows, int64_t cols, const void* X, int64_t ldx, int xtype, int fmt,
                             int transpose, void* Xq, int64_t pitch, float* scales, uint32_t* flags,
                             hipStream_t s, uint32_t* amax_ws, bool amax_ready, uint32_t* zero,
                             int64_t zero_words) {
  uint8_t* q = reinterpret_cast<uint8_t*>(Xq);
  switch (xtype) {
    case LRAMM_F32:
      return quantize_fmt<float>(rows, cols, (const float*)X, ldx, fmt, transpose, q, pitch, scales, flags, s, amax_ws, amax_ready, zero, zero_words);
    case LRAMM_BF16:
      return quantize_fmt<uint16_t>(rows, cols, (const uint16_t*)X, ldx, fmt, transpose, q, pitch, scales, flags, s, amax_ws, amax_ready, zero, zero_words);
    case LRAMM_F64:
      return quantize_fmt<double>(rows, cols, (const double*)X, ldx, fmt, transpose, q, pitch, scales, flags, s, amax_ws, amax_ready, zero, zero_words);
    default:
      return LRAMM_E_INVALID;
  }
}

}  // namespace lramm

namespace lramm {

lramm_status launch_quantize_both(int64_t rows, int64_t cols, const void* X, int64_t ldx, int xtype, int fmt,
                                  void* Rq, int64_t rpitch, float* rscales, void* Cq, int64_t cpitch,
                                  float* cscales, uint32_t* rmax, uint32_t* cmax, uint32_t* flags, hipStream_t s) {
  uint8_t* rq = reinterpret_cast<uint8_t*>(Rq);
  uint8_t* cq = reinterpret_cast<uint8_t*>(Cq);
  switch (xtype) {
    case LRAMM_F32:
      return quantize_both_fmt<float>(rows, cols, (const float*)X, ldx, fmt, rq, rpitch, rscales, cq, cpitch, cscales, rmax, cmax, flags, s);
    case LRAMM_BF16:
      return quantize_both_fmt<uint16_t>(rows, cols, (const uint16_t*)X, ldx, fmt, rq, rpitch, rscales, cq, cpitch, cscales, rmax, cmax, flags, s);
    case LRAMM_F64:
      return quantize_both_fmt<double>(rows, cols, (const double*)X, ldx, fmt, rq, rpitch, rscales, cq, cpitch, cscales, rmax, cmax, flags, s);
    default:
      return LRAMM_E_INVALID;
  }
}

}  // namespace lramm
