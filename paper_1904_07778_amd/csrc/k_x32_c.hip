// Instantiations of the 32-row-tile ring kernel (xcorr32.hpp) for N = 144, 160, 176, 192.
// (One translation unit per four N so that they compile in parallel.)
#include "kernels.hpp"
#include "xcorr32.hpp"

namespace xeng {
namespace x32 {
namespace {

template <int N>
hipError_t launch(dim3 grid, hipStream_t s, const Args& a) {
  constexpr int CPW = cpw_for(N), S = stages_for(N);
  hipLaunchKernelGGL((kernel<N, CPW, S>), grid, dim3(Shape<N, CPW, S>::THREADS), 0, s, a);
  return hipGetLastError();
}

template <int N>
constexpr KernelInfo info() {
  constexpr int CPW = cpw_for(N), S = stages_for(N);
  using C = Shape<N, CPW, S>;
  return KernelInfo{C::NT, C::W, CPW, S, C::THREADS, C::LDS_BYTES, MAX_T_PER_WG, 0, 32, &launch<N>};
}

constexpr int kN[4] = {144, 160, 176, 192};
const KernelInfo kTable[4] = {info<144>(), info<160>(), info<176>(), info<192>()};

}  // namespace
}  // namespace x32

const KernelInfo* x32_kernel_c(int n) {
  for (int i = 0; i < 4; ++i)
    if (x32::kN[i] == n) return &x32::kTable[i];
  return nullptr;
}

}  // namespace xeng
