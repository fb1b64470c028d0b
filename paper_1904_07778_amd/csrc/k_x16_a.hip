// Instantiations of the 16-row-tile ring kernel (xcorr16.hpp) for N = 16, 32, 48, 64, 80, 96, 112.
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

constexpr int kN[7] = {16, 32, 48, 64, 80, 96, 112};
const KernelInfo kTable[7] = {info<16>(), info<32>(), info<48>(), info<64>(), info<80>(), info<96>(), info<112>()};

}  // namespace
}  // namespace x16

const KernelInfo* x16_kernel_a(int n) {
  for (int i = 0; i < 7; ++i)
    if (x16::kN[i] == n) return &x16::kTable[i];
  return nullptr;
}

}  // namespace xeng
