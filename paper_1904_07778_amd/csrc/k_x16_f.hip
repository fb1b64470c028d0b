// Instantiations of the 16-row-tile ring kernel (xcorr16.hpp) for N = 256.
// (Several translation units so that they compile in parallel.)
#include "kernels.hpp"
#include "xcorr16.hpp"

namespace xeng {
namespace x16 {
namespace {

template <int N>
hipError_t launch(dim3 grid, hipStream_t s, const Args& a) {
  constexpr int CPW = cpw_for(N), S = stages_for(N, KPS_DEFAULT);
  hipLaunchKernelGGL((kernel<N, CPW, S, KPS_DEFAULT>), grid, dim3(Shape<N, CPW, S, KPS_DEFAULT>::THREADS), 0, s,
                     a);
  return hipGetLastError();
}

template <int N>
constexpr KernelInfo info() {
  constexpr int CPW = cpw_for(N), S = stages_for(N, KPS_DEFAULT);
  using C = Shape<N, CPW, S, KPS_DEFAULT>;
  return KernelInfo{C::NT, C::W, CPW, S, C::THREADS, C::LDS_BYTES, MAX_T_PER_WG, MAX_ROW_BYTES, TILE_ROWS,
                    &launch<N>};
}

constexpr int kN[1] = {256};
const KernelInfo kTable[1] = {info<256>()};

}  // namespace
}  // namespace x16

const KernelInfo* x16_kernel_f(int n) {
  for (int i = 0; i < 1; ++i)
    if (x16::kN[i] == n) return &x16::kTable[i];
  return nullptr;
}

}  // namespace xeng
