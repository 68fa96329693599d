// Small utility kernels of the C ABI.
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace lm {

// any non-finite value in [0, n) sets *flag
__global__ void k_nonfinite(const double* __restrict__ a, size_t n, int* flag) {
  int bad = 0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double v = a[i];
    if (!(v == v) || v - v != 0.0) bad = 1;
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

// one RK4 step done: advance the batched runs' step counters
__global__ void k_batch_tick(long long* counters, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) counters[i] += 1;
}

void launch_batch_tick(hipStream_t st, long long* counters, int n) {
  if (n > 0) hipLaunchKernelGGL(k_batch_tick, dim3((n + 255) / 256), dim3(256), 0, st, counters, n);
}

void launch_nonfinite(RunView& r, const double* a, size_t n, int* flag) {
  hipLaunchKernelGGL(k_nonfinite, dim3(256), dim3(256), 0, r.stream, a, n, flag);
}

}  // namespace lm
