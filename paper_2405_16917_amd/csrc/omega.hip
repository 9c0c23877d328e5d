// Gaussian test matrix of the range finder (paper Sec. 2.2: Gaussian
// sampling) from the counter-based generator Philox4x32-10 (Salmon, Moraes,
// Dror, Shaw, SC 2011), so that every element is a pure function of
// (seed, index) and no generator state is kept.
//
// Element Omega[i][j] of the k x l matrix is written to OmegaT[j][i]; its
// index e = j*k + i selects counter c = e >> 2 and word e & 3, and the words
// (x0, x1), (x2, x3) become normals by Box-Muller in FP64, rounded once to
// binary32.  Rows j in [l, lrows) of OmegaT are written as zeros.
#include <algorithm>

#include "common.hpp"

namespace lramm {

// Words (x0, x1), (x2, x3) of one Philox output -> four normals in FP64:
// u1 = (x0 + 1) 2^-32, u2 = x1 2^-32, r = sqrt(-2 ln u1), t = 2 pi u2,
// (r cos t, r sin t), and the same for (x2, x3).
__device__ __forceinline__ void box_muller(const uint32_t w[4], double z[4]) {
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const double u1 = ((double)w[2 * p] + 1.0) * 0x1p-32;
    const double u2 = (double)w[2 * p + 1] * 0x1p-32;
    const double rr = sqrt(-2.0 * log(u1));
    const double t = 2.0 * 3.141592653589793 * u2;
    double sn, cs;
    sincos(t, &sn, &cs);
    z[2 * p] = rr * cs;
    z[2 * p + 1] = rr * sn;
  }
}

__global__ __launch_bounds__(256) void omega_kernel(uint64_t seed, int64_t k, int64_t l, int64_t lrows,
                                                    float* __restrict__ OmegaT, int64_t ldo) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;   // one Philox call per thread
  const int64_t total = k * l;
  const int64_t e0 = c * 4;
  if (e0 >= lrows * k) return;
  uint32_t w[4] = {(uint32_t)c, (uint32_t)((uint64_t)c >> 32), 0u, 0u};
  philox4x32_10(w, (uint32_t)seed, (uint32_t)(seed >> 32));
  double z[4];
  box_muller(w, z);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    int64_t e = e0 + q;
    if (e >= lrows * k) break;
    int64_t j = e / k, i = e % k;
    OmegaT[j * ldo + i] = e < total ? (float)z[q] : 0.0f;
  }
}

// Omega generated and quantised in one pass: workgroup j forms row j of
// Omega^T (the k values of column j of Omega, binary32 as lramm_omega writes
// them) in LDS, reduces its absmax and writes its codes and scale by the row
// rule of the quantiser (zero past k up to the pitch).  The FP32 Omega^T is
// not stored.
template <int FMT>
__global__ __launch_bounds__(256) void omega_quant_kernel(uint64_t seed, int64_t k, uint8_t* __restrict__ Oq,
                                                          int64_t pitch, int64_t pelems, float* __restrict__ scales) {
  extern __shared__ float orow[];
  __shared__ unsigned wmax[4];
  const int tid = threadIdx.x, lane = tid & 63;
  const int64_t j = blockIdx.x;
  const int64_t e_lo = j * k, e_hi = e_lo + k;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  unsigned amax = 0;
  for (int64_t c = (e_lo >> 2) + tid; c <= ((e_hi - 1) >> 2); c += 256) {
    uint32_t w[4] = {(uint32_t)c, (uint32_t)((uint64_t)c >> 32), 0u, 0u};
    philox4x32_10(w, k0, k1);
    double z[4];
    box_muller(w, z);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t e = 4 * c + q;
      if (e >= e_lo && e < e_hi) {
        const float v = (float)z[q];
        orow[e - e_lo] = v;
        amax = max(amax, abs_bits(v));
      }
    }
  }
  float lam = 1.0f;
  if constexpr (FMT != LRAMM_BF16F) {
    amax = wave_max_u32(amax);
    if (lane == 0) wmax[tid >> 6] = amax;
  }
  __syncthreads();
  if constexpr (FMT != LRAMM_BF16F) {
    const unsigned mb = max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3]));
    const float qmax = FMT == LRAMM_INT8 ? 127.0f : (FMT == LRAMM_INT4 ? 7.0f : 448.0f);
    const QParams qp = qparams(__uint_as_float(mb), qmax);
    lam = qp.lam;
    if (tid == 0) scales[j] = qp.d;
  } else {
    if (tid == 0) scales[j] = 1.0f;
  }
  uint8_t* qr = Oq + j * pitch;
  for (int64_t c0 = (int64_t)tid * 4; c0 < pelems; c0 += 1024) {
    float v[4];
    bool live[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      live[q] = c0 + q < k && (FMT == LRAMM_BF16F || lam != 0.0f);   // lambda 0 (amax 0): codes 0
      v[q] = c0 + q < k ? orow[c0 + q] : 0.0f;
    }
    encode4<FMT>(qr, c0, v, live, lam);
  }
}

// bf16 codes need no absmax: one Philox call per thread, each of its four
// normals written straight to its place in row j of Omega^T as bf16 of the
// binary32 value.  Workgroups with blockIdx.y == 1 zero the codes past k up
// to the pitch.
__global__ __launch_bounds__(256) void omega_bf16_kernel(uint64_t seed, int64_t k, int64_t l,
                                                         uint16_t* __restrict__ Oq, int64_t ldq, int64_t pelems,
                                                         float* __restrict__ scales) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (blockIdx.y == 1) {
    const int64_t padw = pelems - k;
    if (t < l * padw) Oq[(t / padw) * ldq + k + t % padw] = 0;
    if (t < l) scales[t] = 1.0f;
    return;
  }
  const int64_t total = k * l;
  if (4 * t >= total) return;
  uint32_t w[4] = {(uint32_t)t, (uint32_t)((uint64_t)t >> 32), 0u, 0u};
  philox4x32_10(w, (uint32_t)seed, (uint32_t)(seed >> 32));
  double z[4];
  box_muller(w, z);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t e = 4 * t + q;
    if (e < total) Oq[(e / k) * ldq + e % k] = bf16_bits((float)z[q]);
  }
}

int64_t omega_quant_max_k() { return (int64_t)(128 * 1024) / 4; }

lramm_status launch_omega_quant(uint64_t seed, int64_t k, int64_t l, int fmt, uint8_t* Oq, int64_t pitch,
                                float* scales, hipStream_t s) {
  // bf16: fully parallel; other formats: one workgroup per row (absmax first)
  if (k == 0 || l == 0) return LRAMM_OK;
  const int64_t pe = pitch_elems(pitch, fmt);
  if (fmt == LRAMM_BF16F) {
    const int64_t work = std::max(ceil_div(k * l, 4), std::max(l * (pe - k), l));
    const dim3 grid((unsigned)ceil_div(work, 256), 2);
    hipLaunchKernelGGL(omega_bf16_kernel, grid, dim3(256), 0, s, seed, k, l, reinterpret_cast<uint16_t*>(Oq), pitch / 2,
                       pe, scales);
    LRAMM_HIP(hipGetLastError());
    return LRAMM_OK;
  }
  if (k > omega_quant_max_k()) return LRAMM_E_UNSUPPORTED;
  const size_t shm = (size_t)k * sizeof(float);
  static bool attr_set = false;
  if (!attr_set) {   // row of up to 128 KiB in LDS
    const size_t mx = (size_t)omega_quant_max_k() * sizeof(float);
    LRAMM_HIP(hipFuncSetAttribute((const void*)omega_quant_kernel<LRAMM_INT8>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)mx));
    LRAMM_HIP(hipFuncSetAttribute((const void*)omega_quant_kernel<LRAMM_INT4>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)mx));
    LRAMM_HIP(hipFuncSetAttribute((const void*)omega_quant_kernel<LRAMM_FP8>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)mx));
    LRAMM_HIP(hipFuncSetAttribute((const void*)omega_quant_kernel<LRAMM_BF16F>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)mx));
    attr_set = true;
  }
  const dim3 grid((unsigned)l);
  switch (fmt) {
    case LRAMM_INT8:
      hipLaunchKernelGGL(omega_quant_kernel<LRAMM_INT8>, grid, dim3(256), shm, s, seed, k, Oq, pitch, pe, scales);
      break;
    case LRAMM_INT4:
      hipLaunchKernelGGL(omega_quant_kernel<LRAMM_INT4>, grid, dim3(256), shm, s, seed, k, Oq, pitch, pe, scales);
      break;
    case LRAMM_FP8:
      hipLaunchKernelGGL(omega_quant_kernel<LRAMM_FP8>, grid, dim3(256), shm, s, seed, k, Oq, pitch, pe, scales);
      break;
    case LRAMM_BF16F:
      hipLaunchKernelGGL(omega_quant_kernel<LRAMM_BF16F>, grid, dim3(256), shm, s, seed, k, Oq, pitch, pe, scales);
      break;
    default: return LRAMM_E_INVALID;
  }
  LRAMM_HIP(hipGetLastError());
  return LRAMM_OK;
}

lramm_status launch_omega(uint64_t seed, int64_t k, int64_t l, int64_t lrows, float* OmegaT, int64_t ldo,
                          hipStream_t s) {
  int64_t calls = ceil_div(lrows * k, 4);
  if (calls == 0) return LRAMM_OK;
  hipLaunchKernelGGL(omega_kernel, dim3((unsigned)ceil_div(calls, 256)), dim3(256), 0, s, seed, k, l, lrows, OmegaT,
                     ldo);
  LRAMM_HIP(hipGetLastError());
  return LRAMM_OK;
}

}  // namespace lramm
