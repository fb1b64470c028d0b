// The persistent batch kernel (batch.hpp): all supported N in one function.
#include "batch.hpp"

namespace xeng {
namespace batch {
namespace {

__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(1))) void kernel(Params) {
  // The parameters are read in place from the kernel-argument segment (the
  // only explicit argument, at offset 0): indexed by a run-time array number,
  // a by-value copy would be moved into registers or scratch.
  const Params& p = *(const Params*)__builtin_amdgcn_kernarg_segment_ptr();
  __shared__ __attribute__((aligned(1024))) uint8_t lds[lds_bytes()];
  __shared__ int item_slot;
  const int home = blockIdx.x % QUEUES;

  // items of array k in queue x
  auto count = [&](int k, int x) {
    const int g = p.ngroups[k];
    return (range_begin(g, x + 1) - range_begin(g, x)) * p.nchunks[k];
  };

  for (int d = 0; d < QUEUES;) {
    const int x = (home + d) % QUEUES;
    if (threadIdx.x == 0) item_slot = atomicAdd(&p.counters[x], 1);
    __syncthreads();
    int q = item_slot;
    __syncthreads();  // every wave has read the slot before it is written again
    int k = 0;
    for (; k < p.n_arrays; ++k) {
      const int c = count(k, x);
      if (q < c) break;
      q -= c;
    }
    if (k == p.n_arrays) {  // queue x is exhausted: move on to the next one
      ++d;
      continue;
    }
    k = __builtin_amdgcn_readfirstlane(k);
    q = __builtin_amdgcn_readfirstlane(q);
    const int g0 = range_begin(p.ngroups[k], x);
    const int ng = range_begin(p.ngroups[k], x + 1) - g0;
    const Args a = p.arr[k];
    // An opaque copy of the thread index per item: everything the item body
    // derives from it stays inside the loop, instead of being hoisted out for
    // all twelve launch shapes at once (which would not fit the registers).
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    run_if<16>(a.N, a, lds, g0 + q % ng, q / ng, tid);
    __syncthreads();  // the item's last LDS reads are done before the next item's loads land
  }

  // The last workgroup out clears the counters for the next launch.
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const int done = atomicAdd(&p.counters[QUEUES], 1);
    if (done == (int)gridDim.x - 1) {
      for (int x = 0; x <= QUEUES; ++x) atomicExch(&p.counters[x], 0);
    }
  }
}


}  // namespace

hipError_t launch(int grid, hipStream_t s, const Params& p) {
  hipLaunchKernelGGL(kernel, dim3(grid), dim3(THREADS), 0, s, p);
  return hipGetLastError();
}

const void* kernel_function() { return reinterpret_cast<const void*>(&kernel); }

}  // namespace batch
}  // namespace xeng
