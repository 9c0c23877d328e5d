// Quantised NT-GEMM of the LRAMM hot path on gfx950 MFMA (paper Sec. 3.1,
// Alg. 2: integer GEMM of the quantised operands, then dequantisation and
// the alpha/beta update):
//
//   C[M x N] = epi( L[M x K] . R[N x K]^T ),  both operands K-contiguous.
//
// Tiling: 256 threads = 4 wavefronts in a 2 x 2 grid; a block tile is
// BM x BN, each wavefront owns (BM/2) x (BN/2) as (BM/64) x (BN/64) tiles of
// the 32 x 32 MFMA.  K advances in stages of 128 bytes of the widened operand
// (128 int8 / int4 / fp8 elements, 64 bf16 elements), double-buffered in LDS with a
// 16-byte row pad (144-byte pitch) so the 16-byte MFMA operand reads of 8
// consecutive rows fall in distinct banks; bytes past the padded K read as
// zero.  Packed int4 rows are read as 64 bytes per stage and widened to int8
// on the way into LDS (no int4 MFMA on CDNA4), so the MFMA loop is the int8
// one.  fp8 (OCP e4m3) runs on the 32 x 32 x 64 f8f6f4 MFMA with unit block
// scales, 32 bytes of K per lane.  The epilogue stages the accumulators in
// LDS and writes 4 consecutive outputs per thread (16-byte stores), applying
// the dequantisation there.
//
// MFMA operand layout (v_mfma_*_32x32x*): lane l supplies row (l % 32) of its
// operand and a 16-byte (fp8: 32-byte) slice of K chosen by l / 32; both operands use the
// same slice mapping, so the K order inside a 32-byte chunk does not matter.
// Result layout: lane l, accumulator r holds row 8(r/4) + 4(l/32) + r%4,
// column l % 32 of the 32 x 32 tile.
//
// Integer accumulation is exact and split-K partials are summed as integers
// in a fixed order, so the result is bit-reproducible for any split.
#include <type_traits>

#include "common.hpp"

namespace lramm {

enum { KIND_I8 = 0, KIND_I4 = 1, KIND_BF16 = 2, KIND_F8 = 3 };

// integer accumulators (exact); otherwise FP32 accumulators
template <int KIND>
constexpr bool kIntAcc = KIND == KIND_I8 || KIND == KIND_I4;
// per-row / per-column dequantisation factors (all but bf16)
template <int KIND>
constexpr bool kScaled = KIND != KIND_BF16;
// K bytes one MFMA consumes: 32 for the 32x32x32 int8 and 32x32x16 bf16
// forms, 64 for the 32x32x64 fp8 form
template <int KIND>
constexpr int kChunk = KIND == KIND_F8 ? 64 : 32;

struct GemmArgs {
  int M, N;
  int nst;                 // K stages of 128 widened bytes
  int st_per_split;        // stages per split-K slice
  int kw;                  // widened K bytes (multiple of 64); bytes past it read as zero
  const uint8_t* L;
  int64_t ldl;             // bytes
  const uint8_t* R;
  int64_t ldr;             // bytes
  const float* dL;
  const float* dR;
  float alpha, beta;
  void* C;
  int64_t ldc;             // elements
  int ctype;
  int c_vec;               // C rows 16-byte aligned (vector stores)
  int col_first;           // dequantise by dR before dL (the output is a transposed product)
  int32_t* acc_out;
  int64_t ld_acc;
  int32_t* part;           // split-K partials [split][M][N] (int32 or float bits)
  int tiles_m, tiles_n;
  int group_m;             // rows of tiles per group of the tile order (0: plain band order)
  int K;                   // K elements (rows of a K-major operand)
};

// Tile of workgroup blockIdx: consecutive workgroup ids go round robin over
// the 8 XCDs, so each XCD first gets a contiguous band of the tile order;
// inside the band, groups of GM rows of tiles are walked column by column, so
// that the workgroups resident at once on one XCD cover a compact block of
// tiles and share their operand panels in that XCD's L2.
__device__ __forceinline__ void tile_order(int bid, int tiles_m, int tiles_n, int gm, int& tm, int& tn) {
  const int ntiles = tiles_m * tiles_n;
  if ((ntiles & 7) == 0) bid = (bid & 7) * (ntiles >> 3) + (bid >> 3);
  if (gm <= 0) {
    const bool m_fast = tiles_m < tiles_n;
    tm = m_fast ? bid % tiles_m : bid / tiles_n;
    tn = m_fast ? bid / tiles_m : bid % tiles_n;
    return;
  }
  const int per_group = gm * tiles_n;
  const int group = bid / per_group;
  const int first_m = group * gm;
  const int gsize = tiles_m - first_m < gm ? tiles_m - first_m : gm;
  const int in = bid - group * per_group;
  tm = first_m + in % gsize;
  tn = in / gsize;
}

constexpr int kStage = 128;                 // widened bytes of K per stage
// stages of K in flight in registers: as deep as the register file allows
// at two workgroups per CU (the LDS limit of the 128-row tiles)
template <int BM, int BN, int KIND>
constexpr int kPrefetchOf = BM * BN >= 128 * 128 ? (KIND == KIND_F8 ? 1 : 2) : (KIND == KIND_F8 ? 2 : 3);
constexpr int kBufferWord3 = 0x00020000;    // buffer resource word 3 (raw byte buffer) on gfx9-family parts
constexpr int kLdsPitch = kStage + 16;      // LDS row pitch (16-byte pad: conflict-free 16 B reads)

template <int KIND>
struct Acc;
template <>
struct Acc<KIND_I8> { typedef v16i T; };
template <>
struct Acc<KIND_I4> { typedef v16i T; };
template <>
struct Acc<KIND_BF16> { typedef v16f T; };
template <>
struct Acc<KIND_F8> { typedef v16f T; };

// One lane's operand fragment: 16 bytes, or 32 for fp8.
template <int KIND>
struct Frag {
  uint4 x[kChunk<KIND> / 32];
};

// Sign-extend the 8 nibbles of w to 8 bytes in element order
// (byte j of w holds element 2j in its low and 2j+1 in its high nibble).
__device__ __forceinline__ uint2 widen_int4(uint32_t w) {
  uint32_t lo = w & 0x0f0f0f0fu;
  uint32_t hi = (w >> 4) & 0x0f0f0f0fu;
  lo |= ((lo >> 3) & 0x01010101u) * 0xf0u;
  hi |= ((hi >> 3) & 0x01010101u) * 0xf0u;
  uint2 o;
  o.x = (lo & 0xffu) | ((hi & 0xffu) << 8) | ((lo & 0xff00u) << 8) | ((hi & 0xff00u) << 16);
  o.y = ((lo >> 16) & 0xffu) | (((hi >> 16) & 0xffu) << 8) | ((lo >> 8) & 0xff0000u) | (hi & 0xff000000u);
  return o;
}

// Global -> registers for one operand tile of ROWS rows at stage st.
//   int8 / bf16: a row holds 8 vectors of 16 B per stage;
//   int4: 4 vectors of 16 B (packed), each widened to 32 B in LDS.
// Loads are buffer loads: the operand base lives in a scalar resource, each
// lane keeps one 32-bit byte offset per vector (its row and its place in the
// stage, fixed for the kernel) and the stage offset is a scalar, so prefetching
// several stages costs no extra address registers.  The lane's place in the
// stage (vector c) is the same for all of its vectors, since 256 lanes cover
// whole rows.
template <int ROWS, int KIND>
struct TileLoader {
  static constexpr int kVecPerRow = KIND == KIND_I4 ? 4 : 8;
  static constexpr int kWPerVec = KIND == KIND_I4 ? 32 : 16;   // widened bytes per global vector
  static constexpr int kVecs = ROWS * kVecPerRow;
  static constexpr int kPerThread = (kVecs + 255) / 256;
  static constexpr int kStageBytes = KIND == KIND_I4 ? kStage / 2 : kStage;   // global bytes per stage
  uint4 r[kPerThread];
  uint32_t m;   // all ones, or zero when the stage's vector lies past the padded K

  // Per-lane offsets: row part (clamped row: results of rows past the end
  // are discarded) and the vector's byte offset inside a stage.
  struct Offsets {
    int row[kPerThread];
    int vec;      // global bytes
    int wvec;     // widened bytes
  };
  static __device__ __forceinline__ Offsets offsets(int64_t ld, int row0, int rows_total, int tid) {
    Offsets o;
    const int c = tid % kVecPerRow;
    o.vec = c * 16;
    o.wvec = c * kWPerVec;
#pragma unroll
    for (int i = 0; i < kPerThread; ++i) {
      const int v = tid + 256 * i;
      int gr = row0 + v / kVecPerRow;
      gr = gr < rows_total ? gr : rows_total - 1;
      o.row[i] = (int)((int64_t)gr * ld);
    }
    return o;
  }

  // MASK: the stage may reach past the padded K (only the last one can);
  // those vectors are loaded from the stage's start in the row (in bounds)
  // and zeroed when stored to LDS, so that nothing waits for the loaded data
  // before the store that needs it anyway.  Both forms are straight-line code.
  template <bool MASK>
  __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t rs, const Offsets& o, int st, int64_t kw64, int tid) {
    const int kw = (int)kw64;
    const int so = st * kStageBytes;
    m = 0xffffffffu;
    int vec = o.vec;
    if constexpr (MASK) {
      const bool in = st * kStage + o.wvec < kw;
      m = in ? 0xffffffffu : 0u;
      vec = in ? vec : 0;
      __asm__("" : "+v"(m));   // opaque: the and-with-mask must not become a branch around the load
    }
#pragma unroll
    for (int i = 0; i < kPerThread; ++i) {
      const int v = tid + 256 * i;
      if (kVecs % 256 == 0 || v < kVecs) {
        typedef unsigned int v4u __attribute__((ext_vector_type(4)));
        const v4u x = __builtin_amdgcn_raw_buffer_load_b128(rs, o.row[i] + vec, so, 0);
        r[i] = make_uint4(x[0], x[1], x[2], x[3]);
      }
    }
  }

  __device__ __forceinline__ void store(uint8_t* lds, int tid) const {
#pragma unroll
    for (int i = 0; i < kPerThread; ++i) {
      const int v = tid + 256 * i;
      if (kVecs % 256 == 0 || v < kVecs) {
        const int row = v / kVecPerRow;
        const int c = v % kVecPerRow;
        const uint4 x = make_uint4(r[i].x & m, r[i].y & m, r[i].z & m, r[i].w & m);
        if constexpr (KIND == KIND_I4) {
          uint2 a = widen_int4(x.x), b = widen_int4(x.y);
          uint2 cc = widen_int4(x.z), d = widen_int4(x.w);
          uint4* dst = reinterpret_cast<uint4*>(lds + row * kLdsPitch + c * 32);
          dst[0] = make_uint4(a.x, a.y, b.x, b.y);
          dst[1] = make_uint4(cc.x, cc.y, d.x, d.y);
        } else {
          *reinterpret_cast<uint4*>(lds + row * kLdsPitch + c * 16) = x;
        }
      }
    }
  }
};

// Global -> registers -> LDS for a bf16 operand stored K-major (K rows of
// the operand's M / N elements, ld bytes apart): the LDS tile has the same
// K-contiguous layout as TileLoader's.  Each of the 256 threads takes a block
// of KR K rows x 8 elements (KR = 4 for 128-row tiles, 2 for 64; K block
// t % (64 / KR), element block t / (64 / KR)), loads it as KR 16-byte
// vectors, transposes it in registers and writes each element row's KR K
// values with one 2 KR-byte LDS store.  Rows past K (and elements past the
// operand) are outside the buffer resource and read as zero.
template <int ROWS>
struct TileLoaderKM {
  static constexpr int KR = ROWS == 128 ? 4 : 2;
  static constexpr int KB = 64 / KR;   // K blocks per 64-row stage
  static_assert(KB * (ROWS / 8) == 256, "one block per thread");
  uint4 r[KR];
  struct Offsets {
    int off;   // bytes: first K row of the block x ld + first element x 2
    int kb, mb;
  };
  static __device__ __forceinline__ Offsets offsets(int64_t ld, int row0, int rows_total, int tid) {
    (void)rows_total;
    Offsets o;
    o.kb = tid % KB;
    o.mb = tid / KB;
    o.off = (int)((int64_t)(KR * o.kb) * ld + (int64_t)(row0 + 8 * o.mb) * 2);
    return o;
  }
  template <bool MASK>
  __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t rs, const Offsets& o, int st, int64_t ld, int tid) {
    (void)tid;
    const int so = (int)((int64_t)st * 64 * ld);
#pragma unroll
    for (int i = 0; i < KR; ++i) {
      typedef unsigned int v4u __attribute__((ext_vector_type(4)));
      const v4u x = __builtin_amdgcn_raw_buffer_load_b128(rs, o.off + (int)(i * ld), so, 0);
      r[i] = make_uint4(x[0], x[1], x[2], x[3]);
    }
  }
  __device__ __forceinline__ void store(uint8_t* lds, const Offsets& o) const {
    uint32_t w[KR][4];
#pragma unroll
    for (int i = 0; i < KR; ++i) w[i][0] = r[i].x, w[i][1] = r[i].y, w[i][2] = r[i].z, w[i][3] = r[i].w;
    uint8_t* base = lds + 8 * o.mb * kLdsPitch + 2 * KR * o.kb;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      // elements 2q (low halves) and 2q + 1 (high halves) of the KR K rows
      if constexpr (KR == 4) {
        const uint2 e0 = make_uint2(__byte_perm(w[0][q], w[1][q], 0x5410), __byte_perm(w[2][q], w[3][q], 0x5410));
        const uint2 e1 = make_uint2(__byte_perm(w[0][q], w[1][q], 0x7632), __byte_perm(w[2][q], w[3][q], 0x7632));
        *reinterpret_cast<uint2*>(base + (2 * q) * kLdsPitch) = e0;
        *reinterpret_cast<uint2*>(base + (2 * q + 1) * kLdsPitch) = e1;
      } else {
        *reinterpret_cast<uint32_t*>(base + (2 * q) * kLdsPitch) = __byte_perm(w[0][q], w[1][q], 0x5410);
        *reinterpret_cast<uint32_t*>(base + (2 * q + 1) * kLdsPitch) = __byte_perm(w[0][q], w[1][q], 0x7632);
      }
    }
  }
};


template <int KIND>
__device__ __forceinline__ Frag<KIND> load_frag(const uint8_t* p) {
  Frag<KIND> f;
#pragma unroll
  for (int i = 0; i < kChunk<KIND> / 32; ++i) f.x[i] = *reinterpret_cast<const uint4*>(p + 16 * i);
  return f;
}

// fp8 operands: format code 0 (OCP e4m3) for both; the block scales are
// E8M0 127, i.e. 2^0, so the instruction is the plain fp8 product.
constexpr int kFmtE4M3 = 0, kScaleOne = 127;

template <int KIND>
__device__ __forceinline__ void mfma_32x32(typename Acc<KIND>::T& acc, const Frag<KIND>& a, const Frag<KIND>& b) {
  if constexpr (KIND == KIND_BF16) {
    v8bf av = __builtin_bit_cast(v8bf, a.x[0]);
    v8bf bv = __builtin_bit_cast(v8bf, b.x[0]);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
  } else if constexpr (KIND == KIND_F8) {
    v8i av = __builtin_bit_cast(v8i, a);
    v8i bv = __builtin_bit_cast(v8i, b);
    acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, acc, kFmtE4M3, kFmtE4M3, 0, kScaleOne, 0,
                                                           kScaleOne);
  } else {
    v4i av = __builtin_bit_cast(v4i, a.x[0]);
    v4i bv = __builtin_bit_cast(v4i, b.x[0]);
    acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(av, bv, acc, 0, 0, 0);
  }
}

__device__ __forceinline__ float load_cin(const void* C, int64_t idx, int ctype) {
  return ctype == LRAMM_F32 ? reinterpret_cast<const float*>(C)[idx]
                            : bf16_to_float(reinterpret_cast<const uint16_t*>(C)[idx]);
}

// Dequantising epilogue of one element: c = fl32(fl32(fl32(acc) * d_i) * d_j)
// with d_i the row factor of the left operand of the product and d_j the
// column factor of the right one; out = fl32(alpha c) [+ fl32(beta Cin)].
// When the kernel computes a transposed product (C^T = R L^T), the paper's
// row factor is the kernel's column factor dR, so col_first swaps the order.
// bf16 operands have no scales.
template <bool SCALED>
__device__ __forceinline__ float epi_value(float accf, float dl, float dr, int col_first, float alpha, float beta,
                                           float cin) {
  float c = accf;
  if (SCALED) {
    const float f1 = col_first ? dr : dl;
    const float f2 = col_first ? dl : dr;
    c = __fmul_rn(__fmul_rn(c, f1), f2);
  }
  c = __fmul_rn(alpha, c);
  if (beta != 0.0f) c = __fadd_rn(c, __fmul_rn(beta, cin));
  return c;
}

// Write 4 finished outputs at columns gn..gn+3 of row gm (FP32 or BF16 C).
__device__ __forceinline__ void store_out4(const GemmArgs& a, int gm, int gn, const float out[4]) {
  const int64_t base = (int64_t)gm * a.ldc + gn;
  const bool full = gn + 3 < a.N;
  if (a.ctype == LRAMM_F32) {
    float* C = reinterpret_cast<float*>(a.C) + base;
    if (full && a.c_vec) {
      *reinterpret_cast<float4*>(C) = make_float4(out[0], out[1], out[2], out[3]);
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (gn + q < a.N) C[q] = out[q];
    }
  } else {
    uint16_t* C = reinterpret_cast<uint16_t*>(a.C) + base;
    if (full && a.c_vec) {
      uint2 w;
      w.x = (uint32_t)bf16_bits(out[0]) | ((uint32_t)bf16_bits(out[1]) << 16);
      w.y = (uint32_t)bf16_bits(out[2]) | ((uint32_t)bf16_bits(out[3]) << 16);
      *reinterpret_cast<uint2*>(C) = w;
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (gn + q < a.N) C[q] = bf16_bits(out[q]);
    }
  }
}

// Store phase for 4 consecutive columns gn..gn+3 of row gm: raw accumulator
// bits v (int32 for integer kinds, float bits otherwise).
template <int KIND, bool SPLIT>
__device__ __forceinline__ void store4(const GemmArgs& a, int split, int gm, int gn, const int32_t v[4]) {
  if constexpr (SPLIT) {
    int32_t* dst = a.part + ((int64_t)split * a.M + gm) * a.N + gn;
    if (gn + 3 < a.N && (a.N & 3) == 0) {
      *reinterpret_cast<int4*>(dst) = make_int4(v[0], v[1], v[2], v[3]);
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (gn + q < a.N) dst[q] = v[q];
    }
    return;
  }
  if constexpr (kIntAcc<KIND>) {
    if (a.acc_out) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (gn + q < a.N) a.acc_out[(int64_t)gm * a.ld_acc + gn + q] = v[q];
    }
  }
  constexpr bool SCALED = kScaled<KIND>;
  const float dl = SCALED ? a.dL[gm] : 1.0f;
  float out[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int n = gn + q < a.N ? gn + q : a.N - 1;
    // v_cvt_f32_i32 rounds to nearest even
    const float accf = kIntAcc<KIND> ? (float)v[q] : __int_as_float(v[q]);
    const float dr = SCALED ? a.dR[n] : 1.0f;
    const float cin = a.beta != 0.0f ? load_cin(a.C, (int64_t)gm * a.ldc + n, a.ctype) : 0.0f;
    out[q] = epi_value<SCALED>(accf, dl, dr, a.col_first, a.alpha, a.beta, cin);
  }
  store_out4(a, gm, gn, out);
}

// Final store of 4 consecutive columns gn..gn+3 of row gm with the
// dequantisation factors already at hand (scaled kinds, no split).
template <int KIND>
__device__ __forceinline__ void store4_scaled(const GemmArgs& a, int gm, int gn, const int32_t v[4], float dl,
                                              const float dr[4]) {
  if constexpr (kIntAcc<KIND>) {
    if (a.acc_out) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (gn + q < a.N) a.acc_out[(int64_t)gm * a.ld_acc + gn + q] = v[q];
    }
  }
  float out[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int n = gn + q < a.N ? gn + q : a.N - 1;
    const float accf = kIntAcc<KIND> ? (float)v[q] : __int_as_float(v[q]);
    const float cin = a.beta != 0.0f ? load_cin(a.C, (int64_t)gm * a.ldc + n, a.ctype) : 0.0f;
    out[q] = epi_value<true>(accf, dl, dr[q], a.col_first, a.alpha, a.beta, cin);
  }
  store_out4(a, gm, gn, out);
}

// One output element from registers (big-tile epilogue).
template <int KIND, bool SPLIT>
__device__ __forceinline__ void store1(const GemmArgs& a, int split, int gm, int gn, int32_t v, float dr) {
  if constexpr (SPLIT) {
    a.part[((int64_t)split * a.M + gm) * a.N + gn] = v;
    return;
  }
  if constexpr (kIntAcc<KIND>) {
    if (a.acc_out) a.acc_out[(int64_t)gm * a.ld_acc + gn] = v;
  }
  constexpr bool SCALED = kScaled<KIND>;
  const float dl = SCALED ? a.dL[gm] : 1.0f;
  const float accf = kIntAcc<KIND> ? (float)v : __int_as_float(v);
  const int64_t idx = (int64_t)gm * a.ldc + gn;
  const float cin = a.beta != 0.0f ? load_cin(a.C, idx, a.ctype) : 0.0f;
  const float out = epi_value<SCALED>(accf, dl, dr, a.col_first, a.alpha, a.beta, cin);
  if (a.ctype == LRAMM_F32) reinterpret_cast<float*>(a.C)[idx] = out;
  else reinterpret_cast<uint16_t*>(a.C)[idx] = bf16_bits(out);
}

// KM: bit 0 the left operand, bit 1 the right one is a bf16 matrix stored
// K-major (TileLoaderKM) instead of K-contiguous codes.
// OCC: more workgroups per CU for short K, where the pipeline's start and
// the epilogue weigh most: one LDS stage buffer (two barriers per stage),
// one stage of register prefetch, and the epilogue staged in two row halves,
// so that LDS (36 KiB per workgroup) and registers (at most 168) admit three
// or four workgroups per CU instead of two.  8192 x 8192 x 416 bf16: 94
// against 121 us; with K = 8192 it loses (115 against 108 us).
template <int BM, int BN, int KIND, bool SPLIT, int KM = 0, bool OCC = false>
__global__ __launch_bounds__(256, OCC ? 3 : 2) void gemm_nt_kernel(GemmArgs a) {
  static_assert(KM == 0 || KIND == KIND_BF16, "K-major operands are bf16");
  constexpr bool LKM = (KM & 1) != 0, RKM = (KM & 2) != 0;
  using LoaderL = typename std::conditional<LKM, TileLoaderKM<BM>, TileLoader<BM, KIND>>::type;
  using LoaderR = typename std::conditional<RKM, TileLoaderKM<BN>, TileLoader<BN, KIND>>::type;
  constexpr int RM = BM / 64;   // 32x32 MFMA tiles per wave along M
  constexpr int kPrefetch = OCC ? 1 : kPrefetchOf<BM, BN, KIND>;
  constexpr int RN = BN / 64;
  constexpr int NB = OCC ? 1 : 2;                       // LDS stage buffers
  constexpr int kABytes = NB * BM * kLdsPitch, kBBytes = NB * BN * kLdsPitch;
  constexpr int kCPitch = BN + 4;                       // floats per staged output row
  constexpr int kPasses = OCC ? 2 : 1;                  // epilogue passes over row slices
  constexpr int kERows = BM / kPasses;
  constexpr int kLds = (kABytes + kBBytes) > kERows * kCPitch * 4 ? (kABytes + kBBytes) : kERows * kCPitch * 4;
  __shared__ __attribute__((aligned(16))) uint8_t smem[kLds];
  uint8_t* sA = smem;
  uint8_t* sB = smem + kABytes;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // XCD-aware tile order: consecutive workgroup ids land on different XCDs
  // (round robin over 8); remap so that each XCD walks a contiguous band of
  // tiles and shares operand rows in its own L2.  Within the band the short
  // side's tile index varies fastest, so that the workgroups reading one tile
  // of the long (larger) operand sit in the same XCD.
  int tm, tn;
  tile_order(blockIdx.x, a.tiles_m, a.tiles_n, a.group_m, tm, tn);
  const int row0 = tm * BM, col0 = tn * BN;
  const int split = blockIdx.y;
  const int st0 = split * a.st_per_split;
  int st1 = st0 + a.st_per_split;
  st1 = st1 < a.nst ? st1 : a.nst;

  typename Acc<KIND>::T acc[RM][RN];
#pragma unroll
  for (int i = 0; i < RM; ++i)
#pragma unroll
    for (int j = 0; j < RN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0;

  // Register prefetch kPrefetch stages deep: stage x sits in slot
  // (x - st0) % kPrefetch from its load until it is written to LDS (double
  // buffer) one iteration before its MFMAs, so every global load has about
  // kPrefetch stages of MFMA work to arrive.
  LoaderL la[kPrefetch];
  LoaderR lb[kPrefetch];
  // operand resources: base and byte extent (rows x pitch, below 2^31; a
  // K-major operand has K rows)
  const __amdgpu_buffer_rsrc_t rsL = __builtin_amdgcn_make_buffer_rsrc(
      (void*)a.L, (short)0, (int)((int64_t)(LKM ? a.K : a.M) * a.ldl), kBufferWord3);
  const __amdgpu_buffer_rsrc_t rsR = __builtin_amdgcn_make_buffer_rsrc(
      (void*)a.R, (short)0, (int)((int64_t)(RKM ? a.K : a.N) * a.ldr), kBufferWord3);
  const typename LoaderL::Offsets oa = LoaderL::offsets(a.ldl, row0, a.M, tid);
  const typename LoaderR::Offsets ob = LoaderR::offsets(a.ldr, col0, a.N, tid);
  // the loaders' last argument: padded K bytes (K-contiguous) or the row
  // stride (K-major)
  const int64_t xl = LKM ? a.ldl : (int64_t)a.kw, xr = RKM ? a.ldr : (int64_t)a.kw;
  const int full = a.kw / kStage;          // stages that lie wholly inside the padded K
  // prologue: the first kPrefetch stages (a short slice repeats its last
  // stage; those copies are never stored)
  if (st0 < st1) {
#pragma unroll
    for (int u = 0; u < kPrefetch; ++u) {
      const int st = st0 + u < st1 ? st0 + u : st1 - 1;
      la[u].template load<true>(rsL, oa, st, xl, tid);
      lb[u].template load<true>(rsR, ob, st, xr, tid);
    }
  }
  auto store_l = [&](const LoaderL& ld, uint8_t* dst) {
    if constexpr (LKM) ld.store(dst, oa);
    else ld.store(dst, tid);
  };
  auto store_r = [&](const LoaderR& ld, uint8_t* dst) {
    if constexpr (RKM) ld.store(dst, ob);
    else ld.store(dst, tid);
  };
  if (st0 < st1) {
    store_l(la[0], sA);
    store_r(lb[0], sB);
  }
  __syncthreads();

  const int arow = wm * (BM / 2) + (lane & 31);
  const int brow = wn * (BN / 2) + (lane & 31);
  constexpr int CH = kChunk<KIND>;
  const int kofs = (lane >> 5) * (CH / 2);

  // one stage: refill slot u (if asked), MFMAs on LDS buffer (st - st0) & 1,
  // then the next stage's slot into the other buffer (single buffer: into
  // the same one, once every wavefront has read it)
  // refill 0: none; 2: stage st + kPrefetch, which may reach past the padded
  // K (clamped to the slice: a repeat of its last stage is never stored)
  auto stage = [&](const int u, const int st, const int refill) {
    const int nx = st + kPrefetch < st1 ? st + kPrefetch : st1 - 1;
    if (refill == 2) {
      la[u].template load<true>(rsL, oa, nx, xl, tid);
      lb[u].template load<true>(rsR, ob, nx, xr, tid);
    }
    const int buf = NB == 1 ? 0 : (st - st0) & 1;
    const uint8_t* A = sA + buf * BM * kLdsPitch;
    const uint8_t* B = sB + buf * BN * kLdsPitch;
#pragma unroll
    for (int c = 0; c < kStage / CH; ++c) {
      Frag<KIND> av[RM], bv[RN];
#pragma unroll
      for (int i = 0; i < RM; ++i) av[i] = load_frag<KIND>(A + (arow + 32 * i) * kLdsPitch + c * CH + kofs);
#pragma unroll
      for (int j = 0; j < RN; ++j) bv[j] = load_frag<KIND>(B + (brow + 32 * j) * kLdsPitch + c * CH + kofs);
#pragma unroll
      for (int i = 0; i < RM; ++i)
#pragma unroll
        for (int j = 0; j < RN; ++j) mfma_32x32<KIND>(acc[i][j], av[i], bv[j]);
    }
    if (st + 1 < st1) {
      if constexpr (NB == 1) __syncthreads();
      const int un = (u + 1) % kPrefetch;
      store_l(la[un], sA + (NB == 1 ? 0 : buf ^ 1) * BM * kLdsPitch);
      store_r(lb[un], sB + (NB == 1 ? 0 : buf ^ 1) * BN * kLdsPitch);
    }
    __syncthreads();
  };

  // whole groups of kPrefetch stages: every refill is issued (clamped to
  // the slice, masked past the padded K), so the loop body is straight-line
  // code and each LDS store waits only for its own stage's loads; then the
  // last stages, with nothing left to load
  int sb = st0;
  for (; sb + kPrefetch <= st1; sb += kPrefetch) {
#pragma unroll
    for (int u = 0; u < kPrefetch; ++u) stage(u, sb + u, 2);
  }
#pragma unroll
  for (int u = 0; u < kPrefetch; ++u)
    if (sb + u < st1) stage(u, sb + u, 0);

  // ---- epilogue: stage raw accumulators in LDS, then coalesced 4-wide stores
  // (kPasses slices of kERows rows; in slice h the wavefronts holding its
  // rows stage them)
  int32_t* sC = reinterpret_cast<int32_t*>(smem);
  constexpr int kQuads = kERows * BN / 4;
  constexpr int kIters = kQuads / 256;
  static_assert(256 % (BN / 4) == 0, "a thread's quads share their columns");
  static_assert(kPasses == 1 || kERows == BM / 2, "a slice is one wavefront row");
  // a thread's quads all sit in columns cq..cq+3 and in rows rq + (256 / (BN / 4)) it
  const int cq = (tid % (BN / 4)) * 4, rq = tid / (BN / 4);
  const int gn = col0 + cq;
#pragma unroll
  for (int h = 0; h < kPasses; ++h) {
    const int rbase = h * kERows;
    if (h > 0) __syncthreads();   // the previous slice has been read
    if (kPasses == 1 || wm == h) {
#pragma unroll
      for (int i = 0; i < RM; ++i)
#pragma unroll
        for (int j = 0; j < RN; ++j) {
          const int cc = wn * (BN / 2) + 32 * j + (lane & 31);
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int rr = wm * (BM / 2) + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3) - rbase;
            int32_t bits;
            if constexpr (kIntAcc<KIND>) bits = acc[i][j][r];
            else bits = __float_as_int(acc[i][j][r]);
            sC[rr * kCPitch + cc] = bits;
          }
        }
    }
    __syncthreads();
    if constexpr (SPLIT || !kScaled<KIND>) {
#pragma unroll 4
      for (int it = 0; it < kIters; ++it) {
        const int rr = rq + (256 / (BN / 4)) * it;
        const int gm = row0 + rbase + rr;
        if (gm < a.M && gn < a.N) {
          const int4 w = *reinterpret_cast<const int4*>(sC + rr * kCPitch + cq);
          const int32_t v[4] = {w.x, w.y, w.z, w.w};
          store4<KIND, SPLIT>(a, split, gm, gn, v);
        }
      }
    } else {
      // dequantisation factors gathered once, all loads issued together
      float dr[4], dl[kIters];
#pragma unroll
      for (int q = 0; q < 4; ++q) dr[q] = a.dR[gn + q < a.N ? gn + q : a.N - 1];
#pragma unroll
      for (int it = 0; it < kIters; ++it) {
        const int gm = row0 + rbase + rq + (256 / (BN / 4)) * it;
        dl[it] = a.dL[gm < a.M ? gm : a.M - 1];
      }
#pragma unroll 4
      for (int it = 0; it < kIters; ++it) {
        const int rr = rq + (256 / (BN / 4)) * it;
        const int gm = row0 + rbase + rr;
        if (gm < a.M && gn < a.N) {
          const int4 w = *reinterpret_cast<const int4*>(sC + rr * kCPitch + cq);
          const int32_t v[4] = {w.x, w.y, w.z, w.w};
          store4_scaled<KIND>(a, gm, gn, v, dl[it], dr);
        }
      }
    }
  }
}

// ------------------------------------------------------- big-tile kernel --
// 256 x 256 (or BM x BN) block tile, 4 wavefronts in a 2 x 2 grid, each
// owning (BM/2) x (BN/2) as (BM/64) x (BN/64) tiles of the 32 x 32 MFMA.  K
// advances in stages of 64 bytes; four stages live in LDS (one __shared__
// array per stage and operand, so that the compiler's wait for a stage's
// direct-to-LDS loads does not wait for the later stages as well) and the
// loads of stage s + 3 are issued right after the barrier that opens stage s.
// Loads go straight from global memory to LDS (buffer loads with the lds
// modifier): each wavefront instruction fills one 1 KB block of 16 rows, lane
// t writing bytes 16 t .. 16 t + 15 of it.  Used for int8 and bf16.  Rows are 64 bytes; the 16-byte
// granule g of row r sits at granule g ^ ((r >> 1) & 3), so that the MFMA
// operand reads (16 bytes from each of 8 consecutive rows per group of lanes)
// fall in distinct banks; the loads fetch the granule each lane's slot holds.
constexpr int kBigK = 64;          // K bytes per stage
constexpr int kBigStages = 4;      // stages resident in LDS

__device__ __forceinline__ int big_swz(int row, int g) { return row * kBigK + ((g ^ ((row >> 1) & 3)) << 4); }

#define LDS_PTR(p) ((__attribute__((address_space(3))) void*)(p))

template <int ROWS>
struct BigLoader {
  static constexpr int kInst = ROWS / 64;   // 1 KB blocks per wavefront per stage
  int voff[kInst];
  __device__ __forceinline__ void init(int64_t ld, int row0, int rows_total, int wave, int lane) {
#pragma unroll
    for (int i = 0; i < kInst; ++i) {
      const int row = (wave + 4 * i) * 16 + (lane >> 2);
      const int g = (lane & 3) ^ ((row >> 1) & 3);
      int gr = row0 + row;
      gr = gr < rows_total ? gr : rows_total - 1;
      voff[i] = (int)((int64_t)gr * ld) + g * 16;
    }
  }
  __device__ __forceinline__ void issue(__amdgpu_buffer_rsrc_t rs, uint8_t* lds, int st, int wave) const {
#pragma unroll
    for (int i = 0; i < kInst; ++i)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, LDS_PTR(lds + (wave + 4 * i) * 1024), 16, voff[i], st * kBigK, 0,
                                               0);
  }
};

// Operand fragments of one MFMA step (chunk c of a stage): RM tiles of the
// left operand and RN of the right one.  bf16 / int8: two 32-byte chunks per
// 64-byte stage, lanes 0-31 taking granule 2c and lanes 32-63 granule
// 2c + 1; fp8: one 64-byte chunk, lanes 0-31 granules 0, 1 and lanes 32-63
// granules 2, 3.
template <int KIND>
constexpr int kBigChunks = KIND == KIND_F8 ? 1 : 2;

template <int KIND, int RM, int RN>
struct BigFrags {
  Frag<KIND> a[RM], b[RN];
  __device__ __forceinline__ void load(const uint8_t* A, const uint8_t* B, int arow, int brow, int half, int c) {
    if constexpr (KIND == KIND_F8) {
#pragma unroll
      for (int i = 0; i < RM; ++i) {
        a[i].x[0] = *reinterpret_cast<const uint4*>(A + big_swz(arow + 32 * i, 2 * half));
        a[i].x[1] = *reinterpret_cast<const uint4*>(A + big_swz(arow + 32 * i, 2 * half + 1));
      }
#pragma unroll
      for (int j = 0; j < RN; ++j) {
        b[j].x[0] = *reinterpret_cast<const uint4*>(B + big_swz(brow + 32 * j, 2 * half));
        b[j].x[1] = *reinterpret_cast<const uint4*>(B + big_swz(brow + 32 * j, 2 * half + 1));
      }
    } else {
#pragma unroll
      for (int i = 0; i < RM; ++i) a[i].x[0] = *reinterpret_cast<const uint4*>(A + big_swz(arow + 32 * i, 2 * c + half));
#pragma unroll
      for (int j = 0; j < RN; ++j) b[j].x[0] = *reinterpret_cast<const uint4*>(B + big_swz(brow + 32 * j, 2 * c + half));
    }
  }
  __device__ __forceinline__ void mma(typename Acc<KIND>::T (&acc)[RM][RN]) const {
#pragma unroll
    for (int i = 0; i < RM; ++i)
#pragma unroll
      for (int j = 0; j < RN; ++j) mfma_32x32<KIND>(acc[i][j], a[i], b[j]);
  }
};

// wait until at most N of this wavefront's direct-to-LDS loads are in flight
template <int N>
__device__ __forceinline__ void big_vmwait() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  if constexpr (N == 0) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  else if constexpr (N == 4) asm volatile("s_waitcnt vmcnt(4)" ::: "memory");
  else if constexpr (N == 6) asm volatile("s_waitcnt vmcnt(6)" ::: "memory");
  else if constexpr (N == 8) asm volatile("s_waitcnt vmcnt(8)" ::: "memory");
  else if constexpr (N == 12) asm volatile("s_waitcnt vmcnt(12)" ::: "memory");
  else if constexpr (N == 16) asm volatile("s_waitcnt vmcnt(16)" ::: "memory");
  else static_assert(N == 0, "unsupported count");
}

// all wavefronts: their loads of the stage are in LDS and their reads of the
// previous stage are done
template <int PER_STAGE>
__device__ __forceinline__ void big_stage_barrier(int later) {
  if (later >= 2) big_vmwait<2 * PER_STAGE>();
  else if (later == 1) big_vmwait<PER_STAGE>();
  else big_vmwait<0>();
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

template <int BM, int BN, int KIND, bool SPLIT>
__global__ __launch_bounds__(256, 1) void gemm_big_kernel(GemmArgs a) {
  constexpr int RM = BM / 64, RN = BN / 64;
  constexpr int PER_STAGE = BM / 64 + BN / 64;   // load instructions per wavefront per stage
  __shared__ __attribute__((aligned(16))) uint8_t sA0[BM * kBigK];
  __shared__ __attribute__((aligned(16))) uint8_t sA1[BM * kBigK];
  __shared__ __attribute__((aligned(16))) uint8_t sA2[BM * kBigK];
  __shared__ __attribute__((aligned(16))) uint8_t sA3[BM * kBigK];
  __shared__ __attribute__((aligned(16))) uint8_t sB0[BN * kBigK];
  __shared__ __attribute__((aligned(16))) uint8_t sB1[BN * kBigK];
  __shared__ __attribute__((aligned(16))) uint8_t sB2[BN * kBigK];
  __shared__ __attribute__((aligned(16))) uint8_t sB3[BN * kBigK];
  uint8_t* const sA[kBigStages] = {sA0, sA1, sA2, sA3};
  uint8_t* const sB[kBigStages] = {sB0, sB1, sB2, sB3};

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  int tm, tn;
  tile_order(blockIdx.x, a.tiles_m, a.tiles_n, a.group_m, tm, tn);
  const int row0 = tm * BM, col0 = tn * BN;
  const int split = blockIdx.y;
  const int st0 = split * a.st_per_split;
  int st1 = st0 + a.st_per_split;
  st1 = st1 < a.nst ? st1 : a.nst;
  const int nst = st1 > st0 ? st1 - st0 : 0;

  typename Acc<KIND>::T acc[RM][RN];
#pragma unroll
  for (int i = 0; i < RM; ++i)
#pragma unroll
    for (int j = 0; j < RN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0;

  const __amdgpu_buffer_rsrc_t rsL =
      __builtin_amdgcn_make_buffer_rsrc((void*)a.L, (short)0, (int)((int64_t)a.M * a.ldl), kBufferWord3);
  const __amdgpu_buffer_rsrc_t rsR =
      __builtin_amdgcn_make_buffer_rsrc((void*)a.R, (short)0, (int)((int64_t)a.N * a.ldr), kBufferWord3);
  BigLoader<BM> la;
  BigLoader<BN> lb;
  la.init(a.ldl, row0, a.M, wave, lane);
  lb.init(a.ldr, col0, a.N, wave, lane);

  // prologue: stages 0 .. 2 in flight, stage 0 resident, its first
  // fragments loaded
  const int arow = wm * (BM / 2) + (lane & 31);
  const int brow = wn * (BN / 2) + (lane & 31);
  const int half = lane >> 5;
#pragma unroll
  for (int u = 0; u < kBigStages - 1; ++u)
    if (u < nst) {
      la.issue(rsL, sA[u], st0 + u, wave);
      lb.issue(rsR, sB[u], st0 + u, wave);
    }
  constexpr int NC = kBigChunks<KIND>;
  BigFrags<KIND, RM, RN> fr[2];
  if (nst > 0) {
    big_stage_barrier<PER_STAGE>(nst - 1);
    if (kBigStages - 1 < nst) {
      la.issue(rsL, sA[kBigStages - 1], st0 + kBigStages - 1, wave);
      lb.issue(rsR, sB[kBigStages - 1], st0 + kBigStages - 1, wave);
    }
    fr[0].load(sA[0], sB[0], arow, brow, half, 0);
  }
  // Stage s, chunk c: the fragments of the next step are read while this
  // step's MFMAs run.  Before the last chunk of stage s the wavefronts meet
  // at the barrier that opens stage s + 1 (its loads are in LDS, every read of
  // stage s is done), and the loads of stage s + 4 go into stage s's buffer.
  for (int sb = 0; sb < nst; sb += kBigStages) {
#pragma unroll
    for (int u = 0; u < kBigStages; ++u) {
      const int s = sb + u;
      if (s < nst) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const int cur = c & 1;   // NC is 1 or 2: chunk parity selects the register set
          if (c + 1 < NC) {
            fr[cur ^ 1].load(sA[u], sB[u], arow, brow, half, c + 1);
            fr[cur].mma(acc);
          } else {
            // last chunk of stage s: open stage s + 1 first
            if (s + 1 < nst) {
              big_stage_barrier<PER_STAGE>(nst - 2 - s);
              if (s + kBigStages < nst) {
                la.issue(rsL, sA[u], st0 + s + kBigStages, wave);
                lb.issue(rsR, sB[u], st0 + s + kBigStages, wave);
              }
              fr[cur ^ 1].load(sA[(u + 1) % kBigStages], sB[(u + 1) % kBigStages], arow, brow, half, 0);
            }
            fr[cur].mma(acc);
          }
        }
        if constexpr (NC == 1) {
          // fp8: one chunk per stage; the next stage's fragments went to the
          // other register set
          BigFrags<KIND, RM, RN> t = fr[0];
          fr[0] = fr[1];
          fr[1] = t;
        }
      }
    }
  }

  // epilogue: each lane stores its accumulators (32 consecutive columns of a
  // row per half-wavefront)
#pragma unroll
  for (int j = 0; j < RN; ++j) {
    const int gn = col0 + wn * (BN / 2) + 32 * j + (lane & 31);
    const int nc = gn < a.N ? gn : a.N - 1;
    const float dr = (!SPLIT && kScaled<KIND>) ? a.dR[nc] : 1.0f;
#pragma unroll
    for (int i = 0; i < RM; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int gm = row0 + wm * (BM / 2) + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (gm < a.M && gn < a.N) {
          int32_t bits;
          if constexpr (kIntAcc<KIND>) bits = acc[i][j][r];
          else bits = __float_as_int(acc[i][j][r]);
          store1<KIND, SPLIT>(a, split, gm, gn, bits, dr);
        }
      }
  }
}

// explicit instantiations (the launch sits behind if constexpr; without them
// the host stubs of some instantiations were not emitted)
template __global__ void gemm_big_kernel<256, 256, KIND_I8, false>(GemmArgs);
template __global__ void gemm_big_kernel<256, 256, KIND_BF16, false>(GemmArgs);

// The split-K sum of a bf16 product whose epilogue is the identity (alpha
// 1, beta 0, FP32 output, no scales), which also writes the sums' bf16 codes
// as the bf16 row quantiser would from C: row r of the codes (pe elements,
// zero past N) and its unit scale.  The sums are formed in split order, as
// in the plain sum below, so C is the same to the bit; the codes save that
// quantiser's read of C.  One thread per 4 columns of the padded rows.
__global__ __launch_bounds__(256) void splitk_reduce_bf16_codes_kernel(GemmArgs a, int nsplit,
                                                                       uint16_t* __restrict__ codes, int64_t cpitch,
                                                                       int pe, float* __restrict__ cscales) {
  const int64_t total = (int64_t)a.M * a.N;
  const uint32_t per_row = (uint32_t)pe / 4;
  const uint32_t idx = blockIdx.x * 256u + threadIdx.x;
  if ((uint64_t)idx >= (uint64_t)a.M * per_row) return;
  const uint32_t row = idx / per_row;
  const int c0 = (int)(idx - row * per_row) * 4;
  const int64_t e0 = (int64_t)row * a.N + c0;
  float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  if ((a.N & 3) == 0 && c0 < a.N) {
    // a whole quad inside the row: 16-byte loads of each slice
    const int4* p4 = reinterpret_cast<const int4*>(a.part + e0);
    const int64_t stride4 = total / 4;
    for (int k = 0; k < nsplit; ++k) {
      const int4 x = p4[(int64_t)k * stride4];
      v[0] = __fadd_rn(v[0], __int_as_float(x.x));
      v[1] = __fadd_rn(v[1], __int_as_float(x.y));
      v[2] = __fadd_rn(v[2], __int_as_float(x.z));
      v[3] = __fadd_rn(v[3], __int_as_float(x.w));
    }
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (c0 + j < a.N)
        for (int k = 0; k < nsplit; ++k) v[j] = __fadd_rn(v[j], __int_as_float(a.part[(int64_t)k * total + e0 + j]));
  }
  float* C = reinterpret_cast<float*>(a.C) + (int64_t)row * a.ldc;
  if (a.c_vec && c0 + 3 < a.N) {
    *reinterpret_cast<float4*>(C + c0) = make_float4(v[0], v[1], v[2], v[3]);
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (c0 + j < a.N) C[c0 + j] = v[j];
  }
  uint32_t h[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) h[j] = c0 + j < a.N ? (uint32_t)bf16_bits(v[j]) : 0u;
  *reinterpret_cast<uint2*>(codes + (int64_t)row * cpitch + c0) = make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
  if (c0 == 0) cscales[row] = 1.0f;
}

// Sum the split-K partials in split order and apply the epilogue.
template <int KIND>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(GemmArgs a, int nsplit) {
  const int64_t total = (int64_t)a.M * a.N;
  const int64_t q = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
  if (q >= total) return;
  const int gm = (int)(q / a.N), gn = (int)(q % a.N);
  int32_t v[4];
  const bool vec = (a.N & 3) == 0;
  if (vec) {
    // whole quad inside a row: 16-byte loads, several slices in flight
    const int4* p4 = reinterpret_cast<const int4*>(a.part + q);
    const int64_t stride4 = total / 4;
    if (kIntAcc<KIND>) {
      int4 acc = make_int4(0, 0, 0, 0);
#pragma unroll 4
      for (int k = 0; k < nsplit; ++k) {
        const int4 x = p4[(int64_t)k * stride4];
        acc.x += x.x; acc.y += x.y; acc.z += x.z; acc.w += x.w;
      }
      v[0] = acc.x; v[1] = acc.y; v[2] = acc.z; v[3] = acc.w;
    } else {
      float f[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 4
      for (int k = 0; k < nsplit; ++k) {
        const int4 x = p4[(int64_t)k * stride4];
        f[0] = __fadd_rn(f[0], __int_as_float(x.x));
        f[1] = __fadd_rn(f[1], __int_as_float(x.y));
        f[2] = __fadd_rn(f[2], __int_as_float(x.z));
        f[3] = __fadd_rn(f[3], __int_as_float(x.w));
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = __float_as_int(f[j]);
    }
    store4<KIND, false>(a, 0, gm, gn, v);
    return;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (kIntAcc<KIND>) {
      int32_t s = 0;
      if (q + j < total)
        for (int k = 0; k < nsplit; ++k) s += a.part[(int64_t)k * total + q + j];
      v[j] = s;
    } else {
      float s = 0.0f;
      if (q + j < total)
        for (int k = 0; k < nsplit; ++k) s = __fadd_rn(s, __int_as_float(a.part[(int64_t)k * total + q + j]));
      v[j] = __float_as_int(s);
    }
  }
  // a quad that may cross a row end: store element by element
  for (int j = 0; j < 4 && q + j < total; ++j) {
    const int m2 = (int)((q + j) / a.N), n2 = (int)((q + j) % a.N);
    int32_t one[4] = {v[j], 0, 0, 0};
    GemmArgs b = a;
    b.N = n2 + 1;   // limit the store to one column
    store4<KIND, false>(b, 0, m2, n2, one);
  }
}

// ------------------------------------------------------------------ host --

static int kind_of(int fmt) {
  switch (fmt) {
    case LRAMM_INT8: return KIND_I8;
    case LRAMM_INT4: return KIND_I4;
    case LRAMM_BF16F: return KIND_BF16;
    case LRAMM_FP8: return KIND_F8;
    default: return -1;
  }
}

struct Plan {
  int bm, bn, split, st_per_split, nst, kw, tiles_m, tiles_n;
  bool big;    // the 256 x 256 kernel (64-byte K stages)
  bool occ;    // the 128 x 128 kernel at three or four workgroups per CU (short K)
  int group;   // rows of tiles per group of the tile order
};

// The 256 x 256 kernel pays off for long K and at least one full round of
// tiles: measured at 8192^3, bf16 1.13 against 1.26 ms (38 % of peak); it
// loses for short K (8192 x 8192 x 448: 210 against 113 us) and for grids
// that leave CUs idle.  Not for int4, whose codes are widened on the way to
// LDS.
static bool use_big(int64_t M, int64_t N, int kw, int fmt) {
  if (fmt == LRAMM_INT4 || fmt == LRAMM_FP8) return false;   // fp8 fragments would spill at 4 x 4 tiles
  if (kw < 32 * kBigK) return false;
  return ceil_div(M, 256) * ceil_div(N, 256) >= 256;
}

static Plan plan_gemm(int64_t M, int64_t N, int64_t K, int fmt, bool allow_split, bool allow_big = true) {
  Plan p;
  p.occ = false;
  const int64_t esz = fmt == LRAMM_BF16F ? 2 : 1;     // widened bytes per element
  p.kw = (int)round_up(K * esz > 0 ? K * esz : 1, 64);
  p.big = allow_big && use_big(M, N, p.kw, fmt);
  if (p.big) {
    p.bm = p.bn = 256;
    p.tiles_m = (int)ceil_div(M, 256);
    p.tiles_n = (int)ceil_div(N, 256);
    p.nst = p.kw / kBigK;
    p.split = 1;
    p.st_per_split = p.nst;
    p.group = 8;   // 8 x 4 tiles per XCD round: 1.13 ms against 1.85 ms in band order at 8192^3
    return p;
  }
  // groups of 4 rows of tiles: 8192^3 bf16 1.26 against 1.52 ms, 8192 x 8192 x 448 113 against 135 us
  p.group = 4;
  p.nst = (int)ceil_div(p.kw, kStage);
  p.bm = M >= 128 ? 128 : 64;
  p.bn = N >= 128 ? 128 : 64;
  // prefer the 64-high M tile when it wastes noticeably less of a short M
  if (p.bm == 128 && (round_up(M, 128) - M) * 4 > M && (round_up(M, 64) - M) < (round_up(M, 128) - M)) p.bm = 64;
  // prefer the 64-wide N tile when it wastes noticeably less of a skinny N
  if (p.bn == 128 && (round_up(N, 128) - N) * 4 > N && (round_up(N, 64) - N) < (round_up(N, 128) - N)) p.bn = 64;
  // a 128 x 64 (64 x 128) grid that leaves CUs idle runs as 64 x 64 tiles:
  // twice the workgroups outweigh the lower operand reuse (4096 x 272 x 4096:
  // 20 us against 21 us, 320 against 160 tiles)
  if (p.bm != p.bn && ceil_div(M, p.bm) * ceil_div(N, p.bn) < 256) p.bm = p.bn = 64;
  p.tiles_m = (int)ceil_div(M, p.bm);
  p.tiles_n = (int)ceil_div(N, p.bn);
  const int tiles = p.tiles_m * p.tiles_n;
  p.split = 1;
  if (allow_split && tiles >= 128 && tiles <= 256 && p.nst >= 64) {
    // one round of at most one workgroup per CU over a long K (l x n
    // products with K = 8192): two K slices give every CU two workgroups
    // (416 x 8192 x 8192 bf16: 108 against 122 us, partial sums included)
    p.split = 2;
  } else if (allow_split && tiles < 128) {
    // too few tiles to occupy half of the 256 CUs and a long K: split K as
    // far as one round of 512 workgroups allows, each slice keeping at least
    // 4 stages; the partials are summed in a second pass.  From 128 tiles on
    // one workgroup per tile is faster: the partial sums' traffic and the
    // extra launch cost more than the idle CUs (measured at 160 tiles,
    // K = 4096: 21 us unsplit against 23 us split in three)
    for (int sp = 2; sp <= 16; ++sp)
      if (tiles * sp <= 512 && p.nst / sp >= 4) p.split = sp;
  }
  p.st_per_split = (int)ceil_div(p.nst, p.split);
  p.split = (int)ceil_div(p.nst, p.st_per_split);
  // bf16 K-contiguous codes (allow_big: no K-major operand), 128 x 128
  // tiles, at most 16 stages and at least two workgroups per CU to place
  p.occ = allow_big && fmt == LRAMM_BF16F && p.bm == 128 && p.bn == 128 && p.split == 1 && p.nst <= 16 &&
          tiles >= 512;
  return p;
}

size_t gemm_nt_workspace(int64_t M, int64_t N, int64_t K, int fmt) {
  Plan p = plan_gemm(M, N, K, fmt, true);
  return p.split > 1 ? (size_t)p.split * M * N * sizeof(int32_t) : 0;
}

template <int BM, int BN, int KIND, int KM = 0>
static void launch_tile(const GemmArgs& a, int split, hipStream_t s) {
  dim3 grid(a.tiles_m * a.tiles_n, split);
  if (split > 1)
    hipLaunchKernelGGL((gemm_nt_kernel<BM, BN, KIND, true, KM>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((gemm_nt_kernel<BM, BN, KIND, false, KM>), grid, dim3(256), 0, s, a);
}

template <int BM, int BN>
static void launch_tile_km(const GemmArgs& a, int split, int km, hipStream_t s) {
  if (km == 1) launch_tile<BM, BN, KIND_BF16, 1>(a, split, s);
  else if (km == 2) launch_tile<BM, BN, KIND_BF16, 2>(a, split, s);
  else launch_tile<BM, BN, KIND_BF16, 3>(a, split, s);
}

static void launch_km(const GemmArgs& a, const Plan& p, int km, hipStream_t s) {
  if (p.bm == 128 && p.bn == 128) launch_tile_km<128, 128>(a, p.split, km, s);
  else if (p.bm == 128) launch_tile_km<128, 64>(a, p.split, km, s);
  else if (p.bn == 128) launch_tile_km<64, 128>(a, p.split, km, s);
  else launch_tile_km<64, 64>(a, p.split, km, s);
}

template <int KIND>
static void launch_kind(const GemmArgs& a, const Plan& p, hipStream_t s) {
  if constexpr (KIND == KIND_I8 || KIND == KIND_BF16) {
    if (p.big) {
      hipLaunchKernelGGL((gemm_big_kernel<256, 256, KIND, false>), dim3(a.tiles_m * a.tiles_n), dim3(256), 0, s, a);
      return;
    }
  }
  if constexpr (KIND == KIND_BF16) {
    if (p.occ) {
      hipLaunchKernelGGL((gemm_nt_kernel<128, 128, KIND_BF16, false, 0, true>), dim3(a.tiles_m * a.tiles_n),
                         dim3(256), 0, s, a);
      return;
    }
  }
  if (p.bm == 128 && p.bn == 128) launch_tile<128, 128, KIND>(a, p.split, s);
  else if (p.bm == 128) launch_tile<128, 64, KIND>(a, p.split, s);
  else if (p.bn == 128) launch_tile<64, 128, KIND>(a, p.split, s);
  else launch_tile<64, 64, KIND>(a, p.split, s);
}

lramm_status launch_gemm_nt(int64_t M, int64_t N, int64_t K, int fmt, const void* Lq, int64_t ldl,
                            const float* dL, const void* Rq, int64_t ldr, const float* dR, float alpha,
                            float beta, void* C, int64_t ldc, int ctype, int32_t* acc_out, int64_t ld_acc,
                            void* ws, size_t ws_bytes, hipStream_t s, bool col_first, int km, const CodesOut* codes) {
  if (codes) *codes->written = false;
  int kind = kind_of(fmt);
  if (kind < 0) return LRAMM_E_UNSUPPORTED;
  if (km != 0 && (kind != KIND_BF16 || (km & ~3))) return LRAMM_E_UNSUPPORTED;
  if (M == 0 || N == 0) return LRAMM_OK;
  // the tile loads address each operand with 32-bit byte offsets
  if (((km & 1) ? K : M) * ldl >= (int64_t)1 << 31 || ((km & 2) ? K : N) * ldr >= (int64_t)1 << 31)
    return LRAMM_E_UNSUPPORTED;
  size_t need = gemm_nt_workspace(M, N, K, fmt);
  bool can_split = ws != nullptr && need > 0 && ws_bytes >= need;
  Plan p = plan_gemm(M, N, K, fmt, can_split, km == 0);
  GemmArgs a;
  a.M = (int)M;
  a.N = (int)N;
  a.nst = p.nst;
  a.st_per_split = p.st_per_split;
  a.L = (const uint8_t*)Lq;
  a.ldl = ldl;
  a.R = (const uint8_t*)Rq;
  a.ldr = ldr;
  a.dL = dL;
  a.dR = dR;
  a.alpha = alpha;
  a.beta = beta;
  a.C = C;
  a.ldc = ldc;
  a.ctype = ctype;
  a.acc_out = acc_out;
  a.ld_acc = ld_acc;
  a.part = (int32_t*)ws;
  a.tiles_m = p.tiles_m;
  a.tiles_n = p.tiles_n;
  a.kw = p.kw;
  a.col_first = col_first ? 1 : 0;
  a.group_m = p.group;
  a.c_vec = (ldc % 4 == 0) && ((uintptr_t)C % (ctype == LRAMM_F32 ? 16 : 8) == 0);
  a.K = (int)K;
  if (K == 0) p.nst = a.nst = 0;
  if (km) {
    launch_km(a, p, km, s);
    LRAMM_HIP(hipGetLastError());
  } else switch (kind) {
    case KIND_I8: launch_kind<KIND_I8>(a, p, s); break;
    case KIND_I4: launch_kind<KIND_I4>(a, p, s); break;
    case KIND_F8: launch_kind<KIND_F8>(a, p, s); break;
    default: launch_kind<KIND_BF16>(a, p, s); break;
  }
  LRAMM_HIP(hipGetLastError());
  if (p.split > 1 && codes && codes->transposed && kind == KIND_BF16 && alpha == 1.0f && beta == 0.0f &&
      ctype == LRAMM_F32 && !acc_out && codes->pe >= M && codes->pe % 64 == 0) {
    // the slice sum and the transposed codes of C's columns in one pass
    LRAMM_TRY(launch_bf16_cols_from_parts(M, N, reinterpret_cast<const float*>(a.part), p.split,
                                          reinterpret_cast<float*>(C), ldc, reinterpret_cast<uint8_t*>(codes->codes),
                                          2 * codes->pitch, codes->scales, s));
    *codes->written = true;
    return LRAMM_OK;
  }
  if (p.split > 1 && codes && !codes->transposed && kind == KIND_BF16 && alpha == 1.0f && beta == 0.0f &&
      ctype == LRAMM_F32 && !acc_out && codes->pe >= N && codes->pe % 4 == 0 &&
      M * (codes->pe / 4) < ((int64_t)1 << 31)) {
    const int64_t threads = M * (codes->pe / 4);
    hipLaunchKernelGGL(splitk_reduce_bf16_codes_kernel, dim3((unsigned)ceil_div(threads, (int64_t)256)), dim3(256), 0,
                       s, a, p.split, codes->codes, codes->pitch, (int)codes->pe, codes->scales);
    LRAMM_HIP(hipGetLastError());
    *codes->written = true;
    return LRAMM_OK;
  }
  if (p.split > 1) {
    int64_t quads = ceil_div(M * N, 4);
    const dim3 g((unsigned)ceil_div(quads, 256));
    switch (kind) {
      case KIND_I8: hipLaunchKernelGGL(splitk_reduce_kernel<KIND_I8>, g, dim3(256), 0, s, a, p.split); break;
      case KIND_I4: hipLaunchKernelGGL(splitk_reduce_kernel<KIND_I4>, g, dim3(256), 0, s, a, p.split); break;
      case KIND_F8: hipLaunchKernelGGL(splitk_reduce_kernel<KIND_F8>, g, dim3(256), 0, s, a, p.split); break;
      default: hipLaunchKernelGGL(splitk_reduce_kernel<KIND_BF16>, g, dim3(256), 0, s, a, p.split); break;
    }
    LRAMM_HIP(hipGetLastError());
  }
  return LRAMM_OK;
}

}  // namespace lramm
