// Gaussian test matrix of the range finder (paper Sec. 2.2: Gaussian
// sampling) from the counter-based generator Philox4x32-10 (Salmon, Moraes,
// Dror, Shaw, SC 2011), so that every element is a pure function of
// (seed, index) and no generator state is kept.
//
// Element Omega[i][j] of the k x l matrix is written to OmegaT[j][i]; its
// index e = j*k + i selects counter c = e >> 2 and word e & 3, and the words
// (x0, x1), (x2, x3) become normals by Box-Muller in FP64, rounded once to
// binary32.  Rows j in [l, lrows) of OmegaT are written as zeros.
#include "common.hpp"

namespace lramm {

__device__ __forceinline__ void philox_round(uint32_t& x0, uint32_t& x1, uint32_t& x2, uint32_t& x3, uint32_t k0,
                                             uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  uint32_t hi0 = __umulhi(M0, x0), lo0 = M0 * x0;
  uint32_t hi1 = __umulhi(M1, x2), lo1 = M1 * x2;
  uint32_t n0 = hi1 ^ x1 ^ k0, n2 = hi0 ^ x3 ^ k1;
  x0 = n0;
  x1 = lo1;
  x2 = n2;
  x3 = lo0;
}

__device__ __forceinline__ void philox4x32_10(uint32_t ctr[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    philox_round(ctr[0], ctr[1], ctr[2], ctr[3], k0, k1);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
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
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    double u1 = ((double)w[2 * p] + 1.0) * 0x1p-32;
    double u2 = (double)w[2 * p + 1] * 0x1p-32;
    double rr = sqrt(-2.0 * log(u1));
    double t = 2.0 * 3.141592653589793 * u2;
    z[2 * p] = rr * cos(t);
    z[2 * p + 1] = rr * sin(t);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    int64_t e = e0 + q;
    if (e >= lrows * k) break;
    int64_t j = e / k, i = e % k;
    OmegaT[j * ldo + i] = e < total ? (float)z[q] : 0.0f;
  }
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
