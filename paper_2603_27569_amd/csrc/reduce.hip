// Sum of the per-row losses in a fixed order (one workgroup, strided partial
// sums then a tree in LDS), so the total is bitwise reproducible.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stockfft {

__global__ __launch_bounds__(1024) void k_sum_rows(const float* __restrict__ rows,
                                                   float* __restrict__ total, int64_t count) {
  __shared__ float part[1024];
  const int t = threadIdx.x;
  float acc = 0.f;
  for (int64_t i = t; i < count; i += 1024) acc += rows[i];
  part[t] = acc;
  __syncthreads();
#pragma unroll
  for (int w = 512; w > 0; w >>= 1) {
    if (t < w) part[t] += part[t + w];
    __syncthreads();
  }
  if (t == 0) total[0] = part[0];
}

hipError_t launch_sum_rows(const float* rows, float* total, int64_t count, hipStream_t s) {
  k_sum_rows<<<dim3(1), dim3(1024), 0, s>>>(rows, total, count);
  return hipGetLastError();
}

}  // namespace stockfft
