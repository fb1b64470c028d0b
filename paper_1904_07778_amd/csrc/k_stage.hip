// Instantiations of the staging kernel (xcorr.hpp), one per 16-row tile count.
#include <array>
#include <utility>

#include "kernels.hpp"

namespace xeng {
namespace {

template <int NT>
struct StageShape {
  static constexpr int W = waves_for(NT);
  static constexpr int CPW = W >= 4 ? 1 : 4 / W;
};

template <int NT>
hipError_t launch_stage(dim3 grid, hipStream_t s, const Args& a) {
  using SH = StageShape<NT>;
  using C = Cfg<NT, SH::W, SH::CPW>;
  hipLaunchKernelGGL((xcorr_kernel<NT, SH::W, SH::CPW>), grid, dim3(C::THREADS), 0, s, a);
  return hipGetLastError();
}

template <int NT>
constexpr KernelInfo stage_info() {
  using SH = StageShape<NT>;
  using C = Cfg<NT, SH::W, SH::CPW>;
  return KernelInfo{NT, SH::W, SH::CPW, 2, C::THREADS, C::LDS_BYTES, XENG_MAX_T_PER_WG_STAGE, 0, 16,
                    &launch_stage<NT>};
}

template <size_t... I>
constexpr auto make_table(std::index_sequence<I...>) {
  return std::array<KernelInfo, sizeof...(I)>{stage_info<(int)I + 1>()...};
}

const auto kTable = make_table(std::make_index_sequence<16>{});

}  // namespace

const KernelInfo* stage_kernel(int nt) { return (nt >= 1 && nt <= 16) ? &kTable[nt - 1] : nullptr; }

}  // namespace xeng
