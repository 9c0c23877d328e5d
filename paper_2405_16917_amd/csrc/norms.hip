// Squared Frobenius norms for the a-posteriori error estimate of the range
// finder: for Q with orthonormal columns, ||A - Q Q^T A||_F^2 =
// ||A||_F^2 - ||Q^T A||_F^2, and Q^T A is the projection the forward forms
// anyway (paper Alg. 1, B = Q* A; Sec. 3.3 measures the error of the rank-r
// approximation in the Frobenius norm).
//
// Deterministic: each workgroup sums a fixed band of rows in FP64 (every
// thread its own elements in order, then a fixed tree in LDS) into its slot
// of a partials array, and one workgroup adds the partials in index order.
#include "common.hpp"

namespace lramm {

constexpr int kNormParts = 1024;   // partial sums (workgroups) at most

template <typename T>
__global__ __launch_bounds__(256) void sumsq_partial_kernel(int64_t rows, int64_t cols, const T* __restrict__ X,
                                                            int64_t ldx, int64_t rows_per_block,
                                                            double* __restrict__ part) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < rows ? r0 + rows_per_block : rows;
  double acc = 0.0;
  for (int64_t r = r0; r < r1; ++r) {
    const T* xr = X + r * ldx;
    for (int64_t c = t; c < cols; c += 256) {
      const double x = (double)load_as_f32<T>(xr + c);
      acc = fma(x, x, acc);
    }
  }
  red[t] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) red[t] += red[t + o];
    __syncthreads();
  }
  if (t == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(64) void sum_parts_kernel(int n, const double* __restrict__ part, double* out) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += part[i];
  *out = s;
}

lramm_status launch_sumsq(int64_t rows, int64_t cols, const void* X, int64_t ldx, int xtype, double* part,
                          double* out, hipStream_t s) {
  if (rows <= 0 || cols <= 0) {
    hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(64), 0, s, 0, part, out);
    LRAMM_HIP(hipGetLastError());
    return LRAMM_OK;
  }
  const int64_t rpb = ceil_div(rows, (int64_t)kNormParts);
  const int nb = (int)ceil_div(rows, rpb);
  switch (xtype) {
    case LRAMM_F32:
      hipLaunchKernelGGL(sumsq_partial_kernel<float>, dim3(nb), dim3(256), 0, s, rows, cols, (const float*)X, ldx,
                         rpb, part);
      break;
    case LRAMM_BF16:
      hipLaunchKernelGGL(sumsq_partial_kernel<uint16_t>, dim3(nb), dim3(256), 0, s, rows, cols,
                         (const uint16_t*)X, ldx, rpb, part);
      break;
    default: return LRAMM_E_INVALID;
  }
  LRAMM_HIP(hipGetLastError());
  hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(64), 0, s, nb, part, out);
  LRAMM_HIP(hipGetLastError());
  return LRAMM_OK;
}

int sumsq_parts_max() { return kNormParts; }

}  // namespace lramm
