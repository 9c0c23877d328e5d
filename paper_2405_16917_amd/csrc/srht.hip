// Structured test matrix of the range finder: the subsampled randomised
// Hadamard transform (Halko, Martinsson & Tropp 2011, Sec. 4.6; the paper's
// O(mn log r) RSVD cost, Sec. 2.2).  With k' the smallest power of two >= k,
//   Y = A Omega = (A_pad D H)[:, S] / sqrt(l),
// A_pad = A with k' - k zero columns, D = diag(d_i) random signs, H the
// unnormalised k' x k' Sylvester-Hadamard matrix and S a uniformly random set
// of l coordinates in increasing order.  d_i and S come from Philox4x32-10
// with key (seed mod 2^32, seed >> 32): d_i = -1 when bit 0 of word x0 at
// counter (i, 0, 1, 0) is set, and S = the indices of the l smallest pairs
// (x0 at counter (i, 0, 2, 0), i).
//
// srht_keys_kernel: one thread per index of [0, k') draws its key and its
// sign (the two Philox words are the costly part, so they are spread over
// k' / 256 workgroups); the keys go to a scratch array, the signs to a bit
// mask (bit i of word i / 32 set for d_i = -1) from each wavefront's ballot.
// srht_samples_kernel: one workgroup of 1024 threads reads the keys, finds
// the l-th smallest by a radix select (8 bits per pass), and takes every key
// below it and the first of the keys equal to it in index order.
// srht_kernel: one workgroup per row of A; each thread holds EPT consecutive
// elements of the signed row in registers and applies the butterflies of
// the low log2(EPT) index bits there, then the remaining bits in rounds of
// at most min(log2(EPT), 4) bits through LDS (each thread loading the 2^w
// elements that differ only in the round's bits); the l sampled outputs, scaled by
// fl32(1 / sqrt(l)), form row i of Y.  When l is small against k' the last
// round is formed only along the sampled outputs' paths.  The work is
// O(k' log k') additions per row and one pass over A.
#include <math.h>

#include "common.hpp"

namespace lramm {

constexpr int kSrhtMaxK = 32768;
constexpr int kSelThreads = 1024;

int64_t srht_padded(int64_t k) {
  int64_t kp = 1;
  while (kp < k) kp *= 2;
  return kp;
}

__device__ __forceinline__ uint32_t srht_word(uint64_t seed, uint32_t i, uint32_t stream) {
  uint32_t w[4] = {i, 0u, stream, 0u};
  philox4x32_10(w, (uint32_t)seed, (uint32_t)(seed >> 32));
  return w[0];
}

// Inclusive prefix sum over the workgroup (kSelThreads values): a shuffle
// scan inside each wavefront, then the wavefront totals; every thread gets
// the sum up to and including itself.
__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t a = (uint32_t)__shfl_up((int)v, o, 64);
    if (lane >= o) v += a;
  }
  return v;
}

__device__ __forceinline__ uint32_t block_scan_incl(uint32_t v, uint32_t* wsum) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const uint32_t incl = wave_scan_incl(v);
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  uint32_t off = 0;
  for (int u = 0; u < w; ++u) off += wsum[u];
  __syncthreads();
  return incl + off;
}

__global__ __launch_bounds__(256) void srht_keys_kernel(uint64_t seed, int kp, uint32_t* __restrict__ keys,
                                                        uint32_t* __restrict__ sign_bits, uint32_t* zero,
                                                        int64_t zero_words) {
  // a buffer of zero_words words cleared on the way (saves the caller a launch)
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < zero_words; e += (int64_t)gridDim.x * 256) zero[e] = 0u;
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63;
  uint32_t neg = 0;
  if (i < kp) {
    keys[i] = srht_word(seed, (uint32_t)i, 2u);
    neg = srht_word(seed, (uint32_t)i, 1u) & 1u;
  }
  // every lane takes part in the ballot; lanes 0 and 1 store the wavefront's
  // two words (only the first when k' < 64 leaves the second out of range)
  const uint64_t mask = __ballot(neg != 0);
  const int base = i - lane;
  if (lane < 2 && base + 32 * lane < kp) sign_bits[(base >> 5) + lane] = (uint32_t)(mask >> (32 * lane));
}

// C = the keys per thread, max(1, k' / 1024).
template <int C>
__global__ __launch_bounds__(kSelThreads) void srht_samples_kernel(int kp, int l, const uint32_t* __restrict__ keys,
                                                                 int32_t* __restrict__ S) {
  __shared__ uint32_t hist[256];
  __shared__ uint32_t wsum[kSelThreads / 64];
  __shared__ uint32_t s_prefix, s_rank;
  const int t = threadIdx.x, lane = t & 63;
  if (t == 0) {
    s_prefix = 0;
    s_rank = (uint32_t)l;   // 1-based rank of the threshold key
  }
  // this thread's indices: [t C, t C + C) of [0, kp) (live marks the ones
  // in range: all of them unless k' < 1024)
  constexpr int c = C;
  uint32_t u[C];
  uint32_t live = 0;
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const int i = t * c + j;
    const bool in = i < kp;
    u[j] = in ? keys[i] : 0xffffffffu;
    if (in) live |= 1u << j;
  }
  __syncthreads();
  // radix select of the l-th smallest key: digits of 8 bits from the top
  for (int shift = 24; shift >= 0; shift -= 8) {
    if (t < 256) hist[t] = 0;
    __syncthreads();
    const uint32_t pre = s_prefix;
    const uint32_t hi_mask = shift == 24 ? 0u : (0xffffffffu << (shift + 8));
#pragma unroll
    for (int j = 0; j < C; ++j)
      if (((live >> j) & 1u) && (u[j] & hi_mask) == pre) atomicAdd(&hist[(u[j] >> shift) & 255u], 1u);
    __syncthreads();
    if (t < 64) {
      // wavefront 0: lane j holds bins 4j .. 4j + 3
      uint32_t h[4], sum = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) sum += (h[q] = hist[4 * lane + q]);
      const uint32_t rank = s_rank;
      uint32_t cum = wave_scan_incl(sum) - sum;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (cum < rank && cum + h[q] >= rank) {
          s_prefix = pre | ((uint32_t)(4 * lane + q) << shift);
          s_rank = rank - cum;
        }
        cum += h[q];
      }
    }
    __syncthreads();
  }
  // the threshold key T and how many of the keys equal to T are taken (the
  // first ones in index order): s_rank of them
  const uint32_t T = s_prefix, take_eq = s_rank;
  uint32_t nlt = 0, neq = 0;
#pragma unroll
  for (int j = 0; j < C; ++j)
    if ((live >> j) & 1u) {
      nlt += u[j] < T ? 1u : 0u;
      neq += u[j] == T ? 1u : 0u;
    }
  const uint32_t eq_before = block_scan_incl(neq, wsum) - neq;
  uint32_t eq_seen = eq_before, kept = 0;
#pragma unroll
  for (int j = 0; j < C; ++j)
    if (((live >> j) & 1u) && u[j] == T) {
      if (eq_seen < take_eq) ++kept;
      ++eq_seen;
    }
  const uint32_t mine = nlt + kept;
  uint32_t pos = block_scan_incl(mine, wsum) - mine;
  eq_seen = eq_before;
#pragma unroll
  for (int j = 0; j < C; ++j) {
    if (!((live >> j) & 1u)) continue;
    bool sel = u[j] < T;
    if (u[j] == T) {
      sel = eq_seen < take_eq;
      ++eq_seen;
    }
    if (sel) {
      if (pos < (uint32_t)l) S[pos] = t * c + j;
      ++pos;
    }
  }
}

template <typename T>
__device__ __forceinline__ float srht_load(const T* p);
template <>
__device__ __forceinline__ float srht_load<float>(const float* p) { return *p; }
template <>
__device__ __forceinline__ float srht_load<uint16_t>(const uint16_t* p) { return bf16_to_float(*p); }

// EPT consecutive elements at p (16-byte aligned, all in range) as floats.
template <typename T, int EPT>
__device__ __forceinline__ void srht_load_vec(const T* p, float x[EPT]) {
  if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int j = 0; j < EPT; j += 4) {
      const float4 f = *reinterpret_cast<const float4*>(p + j);
      x[j] = f.x, x[j + 1] = f.y, x[j + 2] = f.z, x[j + 3] = f.w;
    }
  } else {
#pragma unroll
    for (int j = 0; j < EPT; j += 8) {
      const uint4 u = *reinterpret_cast<const uint4*>(p + j);
      const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        x[j + 2 * q] = __uint_as_float(w[q] << 16);
        x[j + 2 * q + 1] = __uint_as_float(w[q] & 0xffff0000u);
      }
    }
  }
}

__device__ __forceinline__ int lds_at(int i) { return i + (i >> 5); }

// Elements per thread for k' = 2^P: 32 from k' = 8192 on (256 .. 1024
// threads), else k' / 256 (at least 2).
constexpr int srht_ept(int P) { return P >= 13 ? 32 : P == 12 ? 16 : P == 11 ? 8 : P == 10 ? 4 : 2; }

// P = log2 k' is a template parameter, so every LDS round below is
// straight-line code: its index bits, element counts and (for rounds above
// bit 5) its LDS strides are constants.
template <typename T, int P>
__global__ __launch_bounds__(1024) void srht_kernel(int64_t k, int l, const T* __restrict__ A, int64_t lda,
                                                    const uint32_t* __restrict__ sign_bits,
                                                    const int32_t* __restrict__ S, float scale, float* __restrict__ Y,
                                                    int64_t ldy) {
  extern __shared__ float buf[];
  constexpr int kp = 1 << P;
  constexpr int EPT = srht_ept(P);
  constexpr int E = EPT == 2 ? 1 : EPT == 4 ? 2 : EPT == 8 ? 3 : EPT == 16 ? 4 : 5;
  static_assert((1 << E) == EPT, "EPT is a power of two in 2 .. 32");
  constexpr int RW = E < 4 ? E : 4;   // index bits per LDS round (at most 16 registers)
  constexpr int RN = 1 << RW;
  constexpr int nt = kp / EPT;
  const int t = threadIdx.x;
  const int64_t row = blockIdx.x;
  const T* a = A + row * lda;
  const int i0 = t * EPT;
  float x[EPT];
  constexpr int kVec = sizeof(T) == 4 ? 4 : 8;
  bool vec = false;
  if constexpr (EPT >= kVec) vec = i0 + EPT <= k && ((uintptr_t)(a + i0) % 16) == 0;
  if (vec) {
    if constexpr (EPT >= kVec) srht_load_vec<T, EPT>(a + i0, x);
  } else {
#pragma unroll
    for (int j = 0; j < EPT; ++j) x[j] = (i0 + j < k) ? srht_load<T>(a + i0 + j) : 0.0f;
  }
  // signs: EPT consecutive bits (whole words from 32 on)
#pragma unroll
  for (int j0 = 0; j0 < EPT; j0 += 32) {
    const uint32_t sw = sign_bits[(i0 + j0) >> 5] >> ((i0 + j0) & 31);
#pragma unroll
    for (int j = j0; j < (j0 + 32 < EPT ? j0 + 32 : EPT); ++j)
      if ((sw >> (j - j0)) & 1u) x[j] = -x[j];
  }
  // butterflies of the low E index bits, in registers
#pragma unroll
  for (int s = 1; s < EPT; s <<= 1)
#pragma unroll
    for (int j = 0; j < EPT; ++j)
      if (!(j & s)) {
        const float u = x[j], w = x[j + s];
        x[j] = u + w;
        x[j + s] = u - w;
      }
  // LDS holds element i at i + i / 32: the 32-element runs of consecutive
  // threads then start in different banks
#pragma unroll
  for (int j = 0; j < EPT; ++j) buf[lds_at(i0 + j)] = x[j];
  __syncthreads();
  // the remaining bits [E, P) in rounds of w <= RW bits.  Only l of the k'
  // outputs are kept, so when they are few the last round (bits [BL, P)) is
  // left to the output loop, which forms just the entries that a kept output
  // depends on (2^WL - 1 of the round's additions per output instead of WL
  // per element): every value it forms is the same sum, in the same order,
  // as in the full round
  constexpr int NR = (P - E + RW - 1) / RW;   // LDS rounds (none when P == E)
  constexpr int BL = E + (NR > 0 ? (NR - 1) * RW : 0);
  constexpr int WL = P - BL;
  const bool prune = NR > 0 && (int64_t)l * ((1 << WL) - 1) < (int64_t)kp * WL;
#pragma unroll
  for (int b = E; b < P; b += RW) {
    if (b == BL && prune) break;
    const int w = (P - b) < RW ? (P - b) : RW;
    const int n = 1 << w;
    const int groups = EPT >> w;
#pragma unroll
    for (int g = 0; g < groups; ++g) {
      const int o = g * nt + t;
      const int base = (o & ((1 << b) - 1)) | ((o >> b) << (b + w));
      // from bit 5 on, element base + (v << b) sits at lds_at(base) plus v
      // times a constant stride
      const int a0 = lds_at(base);
      float y[RN];
#pragma unroll
      for (int v = 0; v < RN; ++v)
        if (v < n) y[v] = buf[b >= 5 ? a0 + v * ((1 << b) + (1 << (b - 5))) : lds_at(base + (v << b))];
#pragma unroll
      for (int s = 1; s < RN; s <<= 1)
#pragma unroll
        for (int v = 0; v < RN; ++v)
          if (s < n && v < n && !(v & s)) {
            const float u = y[v], z = y[v + s];
            y[v] = u + z;
            y[v + s] = u - z;
          }
#pragma unroll
      for (int v = 0; v < RN; ++v)
        if (v < n) buf[b >= 5 ? a0 + v * ((1 << b) + (1 << (b - 5))) : lds_at(base + (v << b))] = y[v];
    }
    __syncthreads();
  }
  float* yr = Y + row * ldy;
  if constexpr (NR > 0) {
    if (prune) {
      constexpr int NL = 1 << WL;
      for (int j = t; j < l; j += nt) {
        const int idx = S[j] & (kp - 1);
        const int base = idx & ((1 << BL) - 1);
        const uint32_t h = (uint32_t)idx >> BL;   // the output's bits in the round
        float y[NL];
#pragma unroll
        for (int v = 0; v < NL; ++v) {
          if constexpr (BL >= 5) y[v] = buf[lds_at(base) + v * ((1 << BL) + (1 << (BL - 5)))];
          else y[v] = buf[lds_at(base + (v << BL))];
        }
        // bit s of the round: of the pair (u, z) the output needs u + z when
        // bit s of h is clear and u - z = u + (-z) when it is set; the value
        // for the entry whose lower round bits match h's stays in slot v
#pragma unroll
        for (int sb = 1; sb < NL; sb <<= 1) {
          const uint32_t flip = (h & (uint32_t)sb) ? 0x80000000u : 0u;
#pragma unroll
          for (int v = 0; v < NL; v += 2 * sb) y[v] = y[v] + __uint_as_float(__float_as_uint(y[v + sb]) ^ flip);
        }
        yr[j] = __fmul_rn(y[0], scale);
      }
      return;
    }
  }
  for (int j = t; j < l; j += nt) yr[j] = __fmul_rn(buf[lds_at(S[j] & (kp - 1))], scale);
}

lramm_status launch_srht_samples(uint64_t seed, int64_t k, int64_t l, int32_t* S, uint32_t* sign_bits,
                                 uint32_t* keys, hipStream_t s, uint32_t* zero, int64_t zero_words) {
  const int64_t kp = srht_padded(k);
  if (k < 2 || kp > kSrhtMaxK) return LRAMM_E_UNSUPPORTED;
  if (l < 1 || l > kp) return LRAMM_E_RANK;
  hipLaunchKernelGGL(srht_keys_kernel, dim3((unsigned)ceil_div(kp, (int64_t)256)), dim3(256), 0, s, seed, (int)kp,
                     keys, sign_bits, zero, zero ? zero_words : (int64_t)0);
  LRAMM_HIP(hipGetLastError());
  const int c = kp >= kSelThreads ? (int)(kp / kSelThreads) : 1;
#define SAMPLES(C) \
  hipLaunchKernelGGL(srht_samples_kernel<C>, dim3(1), dim3(kSelThreads), 0, s, (int)kp, (int)l, keys, S)
  switch (c) {
    case 1: SAMPLES(1); break;
    case 2: SAMPLES(2); break;
    case 4: SAMPLES(4); break;
    case 8: SAMPLES(8); break;
    case 16: SAMPLES(16); break;
    default: SAMPLES(32); break;
  }
#undef SAMPLES
  LRAMM_HIP(hipGetLastError());
  return LRAMM_OK;
}

template <typename T, int P>
static lramm_status launch_srht_t(int64_t m, int64_t k, int l, const T* A, int64_t lda, const uint32_t* sign_bits,
                                  const int32_t* S, float scale, float* Y, int64_t ldy, hipStream_t s) {
  constexpr int kp = 1 << P;
  constexpr int nt = kp / srht_ept(P);
  const size_t shm = (size_t)(kp + kp / 32 + 1) * sizeof(float);
  static bool attr_set = false;
  if (!attr_set) {   // rows up to 132 KiB in LDS
    LRAMM_HIP(hipFuncSetAttribute((const void*)srht_kernel<T, P>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)((kSrhtMaxK + kSrhtMaxK / 32 + 1) * sizeof(float))));
    attr_set = true;
  }
  hipLaunchKernelGGL((srht_kernel<T, P>), dim3((unsigned)m), dim3(nt), shm, s, k, l, A, lda, sign_bits, S, scale, Y,
                     ldy);
  LRAMM_HIP(hipGetLastError());
  return LRAMM_OK;
}

template <typename T>
static lramm_status launch_srht_type(int64_t m, int64_t k, int kp, int l, const T* A, int64_t lda,
                                     const uint32_t* sign_bits, const int32_t* S, float scale, float* Y, int64_t ldy,
                                     hipStream_t s) {
  switch (kp) {
#define SRHT_P(P) \
  case 1 << P: return launch_srht_t<T, P>(m, k, l, A, lda, sign_bits, S, scale, Y, ldy, s);
    SRHT_P(1) SRHT_P(2) SRHT_P(3) SRHT_P(4) SRHT_P(5) SRHT_P(6) SRHT_P(7) SRHT_P(8)
    SRHT_P(9) SRHT_P(10) SRHT_P(11) SRHT_P(12) SRHT_P(13) SRHT_P(14) SRHT_P(15)
#undef SRHT_P
    default: return LRAMM_E_UNSUPPORTED;
  }
}

lramm_status launch_srht(int64_t m, int64_t k, int64_t l, const void* A, int64_t lda, int a_type,
                         const uint32_t* sign_bits, const int32_t* S, float* Y, int64_t ldy, hipStream_t s) {
  const int64_t kp = srht_padded(k);
  if (kp > kSrhtMaxK) return LRAMM_E_UNSUPPORTED;
  if (l < 1 || l > kp) return LRAMM_E_RANK;
  if (kp < 2) return LRAMM_E_UNSUPPORTED;   // k = 1: nothing to transform
  if (m == 0) return LRAMM_OK;
  const float scale = (float)(1.0 / sqrt((double)l));
  if (a_type == LRAMM_F32)
    return launch_srht_type<float>(m, k, (int)kp, (int)l, (const float*)A, lda, sign_bits, S, scale, Y, ldy, s);
  if (a_type == LRAMM_BF16)
    return launch_srht_type<uint16_t>(m, k, (int)kp, (int)l, (const uint16_t*)A, lda, sign_bits, S, scale, Y, ldy,
                                      s);
  return LRAMM_E_UNSUPPORTED;
}

}  // namespace lramm
