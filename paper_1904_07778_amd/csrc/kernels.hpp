// kernels.hpp - the table of compiled X-engine kernels seen by the host code.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xcorr.hpp"

namespace xeng {

using LaunchFn = hipError_t (*)(dim3 grid, hipStream_t s, const Args& a);

struct KernelInfo {
  int nt, w, cpw, stages, threads, lds_bytes;
  int64_t max_t_per_wg;  // longest time range one workgroup may integrate
  int64_t max_row_bytes; // largest time row F*N the kernel addresses (0: any)
  int tile_rows;         // rows of its tiles: 16 or 32
  LaunchFn launch;
};

// Staging kernel (any N), by 16-row tile count nt = ceil(N/16), 1..16.
const KernelInfo* stage_kernel(int nt);
// 32-row-tile ring kernel, N a multiple of 16 up to 256 (one function per
// translation unit; x32_kernel asks each).
const KernelInfo* x32_kernel_a(int n);
const KernelInfo* x32_kernel_b(int n);
const KernelInfo* x32_kernel_c(int n);
const KernelInfo* x32_kernel_d(int n);
inline const KernelInfo* x32_kernel(int n) {
  const KernelInfo* k = x32_kernel_a(n);
  if (!k) k = x32_kernel_b(n);
  if (!k) k = x32_kernel_c(n);
  if (!k) k = x32_kernel_d(n);
  return k;
}
// 16-row-tile ring kernel on v_mfma_i32_16x16x64_i8, N a multiple of 16 up
// to 256 (several translation units; x16_kernel asks each).
const KernelInfo* x16_kernel_a(int n);
const KernelInfo* x16_kernel_b(int n);
const KernelInfo* x16_kernel_c(int n);
const KernelInfo* x16_kernel_d(int n);
const KernelInfo* x16_kernel_e(int n);
const KernelInfo* x16_kernel_f(int n);
inline const KernelInfo* x16_kernel(int n) {
  const KernelInfo* k = x16_kernel_a(n);
  if (!k) k = x16_kernel_b(n);
  if (!k) k = x16_kernel_c(n);
  if (!k) k = x16_kernel_d(n);
  if (!k) k = x16_kernel_e(n);
  if (!k) k = x16_kernel_f(n);
  return k;
}

// Copy n[k] int2 values (re, im) from acc[k] to dst[k] for k < count; a
// null acc[k] writes zeros.  Pointers are 8-byte aligned device memory.
constexpr int DUMP_MAX = 24;
struct DumpParams {
  const int2* acc[DUMP_MAX];
  int2* dst[DUMP_MAX];
  int64_t n[DUMP_MAX];
  int count;
};
hipError_t dump_launch(int grid, hipStream_t s, const DumpParams& d);

}  // namespace xeng
