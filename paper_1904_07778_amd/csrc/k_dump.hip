// Dump kernel: copy accumulators out for any number of arrays in one launch
// (a null source writes zeros: the same kernel clears accumulators).  A
// kernel rather than copies and memsets: one launch for all arrays, and it
// may be recorded into a captured graph.
#include "kernels.hpp"

namespace xeng {
namespace {

__global__ __launch_bounds__(256) void dump_kernel(DumpParams d) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int k = 0; k < d.count; ++k) {
    const int2* __restrict__ src = d.acc[k];
    int2* __restrict__ dst = d.dst[k];
    const int64_t n = d.n[k];
    if (src) {
      for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) dst[i] = src[i];
    } else {
      for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) dst[i] = int2{0, 0};
    }
  }
}

}  // namespace

hipError_t dump_launch(int grid, hipStream_t s, const DumpParams& d) {
  hipLaunchKernelGGL(dump_kernel, dim3(grid), dim3(256), 0, s, d);
  return hipGetLastError();
}

}  // namespace xeng
