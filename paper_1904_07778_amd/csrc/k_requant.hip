// k_requant.hip - equaliser / 4-bit requantiser of the F stage (paper
// Sec. 2.1), the step that produces the X-engine's input, and the gain
// update that closes the loop from the X-engine's autocorrelations (Eq. 3);
// C entry points xeng_requantize and xeng_eq_update (include/xeng.h).
//
// Per complex sample: the PFB output word holds an 18-bit two's-complement
// real part in bits 35..18 and imaginary part in bits 17..0 (fix_18_17).
// Each part is multiplied by the channel's scale factor g (unsigned
// fix_18_7, the low 18 bits of its word); the fix_36_24 product is rounded
// half to even at the fix_4_3 least significant bit (product bit 21) and
// saturated to -7 .. 7 (1.001b .. 0.111b); the two 4-bit codes are packed
// into one byte, real part in the high nibble.
//
// Exact in 32-bit integer arithmetic: with g = 512 gh + gl (9 bits each),
//     P = d g = 2^21 (A >> 12) + R,   A = d gh,  R = 512 (A & 4095) + d gl,
// where |A|, |d gl| < 2^26 (24-bit multiplies) and |R| < 2^27, so
// floor(P / 2^21) = (A >> 12) + (R >> 21) and P mod 2^21 = R & (2^21 - 1).
//
// Memory: the kernel streams T*F*N*8 bytes in and T*F*N bytes out, once
// (HBM-bound).  Each thread walks down ROWS time rows (rows are F*N samples
// apart), keeping its gains in registers.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/xeng.h"

namespace xeng {
namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

constexpr int THREADS = 256;
constexpr int ROWS = 16;  // time rows per thread

__device__ __forceinline__ int sext18(uint32_t x) { return ((int)(x << 14)) >> 14; }

__device__ __forceinline__ int code(int d, int g) {
  const int A = __mul24(d, g >> 9);
  const int R = ((A & 4095) << 9) + __mul24(d, g & 511);
  const int base = (A >> 12) + (R >> 21);
  const int rem = R & 0x1FFFFF;
  const int up = (rem > 0x100000 || (rem == 0x100000 && (base & 1))) ? 1 : 0;
  return min(7, max(-7, base + up));
}

__device__ __forceinline__ uint32_t byte_of(uint64_t w, int g) {
  const uint32_t lo = (uint32_t)w, hi = (uint32_t)(w >> 32);
  const int re = sext18((lo >> 18) | (hi << 14));
  const int im = sext18(lo);
  return ((uint32_t)(code(re, g) & 15) << 4) | (uint32_t)(code(im, g) & 15);
}

// Fast path: F*N even, words 16-byte, gains 8-byte, output 2-byte aligned.
// A wave owns 512 consecutive samples of a row (256 pairs) and walks down
// ROWS rows with the 8 gains of each lane in registers.  Per instruction the
// 64 lanes load 64 consecutive 16-byte pairs (1 KB) and store 64 consecutive
// 2-byte pairs (128 bytes): fully coalesced.
__global__ __launch_bounds__(THREADS) void requant8(const uint64_t* __restrict__ w,
                                                    const uint32_t* __restrict__ gains,
                                                    uint8_t* __restrict__ out, int64_t T, int64_t fn2) {
  const int lane = threadIdx.x & 63;
  const int64_t chunk = (int64_t)blockIdx.x * (THREADS / 64) + (threadIdx.x >> 6);  // 256 pairs each
  const int64_t t0 = (int64_t)blockIdx.y * ROWS;
  const int64_t t1 = min(T, t0 + ROWS);
  int64_t pr[4];
  bool ok[4];
  int g[8];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    pr[k] = chunk * 256 + k * 64 + lane;  // pair index in the row
    ok[k] = pr[k] < fn2;
    const u32x2 gg = ok[k] ? reinterpret_cast<const u32x2*>(gains)[pr[k]] : u32x2{0u, 0u};
    g[2 * k] = gg[0] & 0x3FFFF;
    g[2 * k + 1] = gg[1] & 0x3FFFF;
  }
  for (int64_t t = t0; t < t1; ++t) {
    const u32x4* src = reinterpret_cast<const u32x4*>(w) + t * fn2;
    uint16_t* dst = reinterpret_cast<uint16_t*>(out) + t * fn2;
    u32x4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (ok[k]) v[k] = __builtin_nontemporal_load(src + pr[k]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (ok[k]) {
        const uint64_t w0 = ((uint64_t)v[k][1] << 32) | v[k][0];
        const uint64_t w1 = ((uint64_t)v[k][3] << 32) | v[k][2];
        const uint32_t b = byte_of(w0, g[2 * k]) | (byte_of(w1, g[2 * k + 1]) << 8);
        __builtin_nontemporal_store((uint16_t)b, dst + pr[k]);
      }
    }
  }
}

// General path: any F*N and alignment (8-byte words, 4-byte gains).
__global__ __launch_bounds__(THREADS) void requant1(const uint64_t* __restrict__ w,
                                                    const uint32_t* __restrict__ gains,
                                                    uint8_t* __restrict__ out, int64_t T, int64_t fn) {
  const int64_t x = (int64_t)blockIdx.x * THREADS + threadIdx.x;
  if (x >= fn) return;
  const int64_t t0 = (int64_t)blockIdx.y * ROWS;
  const int64_t t1 = min(T, t0 + ROWS);
  const int g = gains[x] & 0x3FFFF;
  for (int64_t t = t0; t < t1; ++t) out[t * fn + x] = (uint8_t)byte_of(w[t * fn + x], g);
}

// Gain update from the autocorrelations (Eq. 3): one thread per (channel,
// input).  G' = round(G t sqrt(2 T / P)), t = tx / 16, halves up, decided
// exactly: a double-precision estimate k is moved until
//     (2k - 1)^2 256 P <= 8 G^2 tx^2 T < (2k + 1)^2 256 P
// holds, comparing 128-bit integer products.
__global__ __launch_bounds__(THREADS) void eq_update(const int32_t* __restrict__ vis, int64_t nbl,
                                                     int64_t T, const uint32_t* __restrict__ gin,
                                                     uint32_t* __restrict__ gout, int F, int N, int tx) {
  const int64_t idx = (int64_t)blockIdx.x * THREADS + threadIdx.x;
  if (idx >= (int64_t)F * N) return;
  const int f = (int)(idx / N), i = (int)(idx % N);
  const int64_t P = vis[((int64_t)f * nbl + (int64_t)i * (i + 1) / 2 + i) * 2];
  const uint32_t word = gin[idx];
  if (P <= 0) {
    gout[idx] = word;
    return;
  }
  const uint64_t G = word & 0x3FFFFu;
  const unsigned __int128 rhs = (unsigned __int128)(8ull * G * G * (uint64_t)tx * (uint64_t)tx) * (uint64_t)T;
  const uint64_t p256 = 256ull * (uint64_t)P;
  auto lhs = [&](int64_t odd) {  // odd^2 * 256 P  (odd < 2^36, so < 2^111)
    return (unsigned __int128)(uint64_t)odd * (uint64_t)odd * p256;
  };
  // |k - x| < 1e-4 for every admissible input (x < 2^35, a few roundings of
  // relative size 2^-53), so each correction takes at most one step; the
  // bound on the loops only guarantees that every lane finishes.
  const double xd = (double)G * tx * sqrt(2.0 * (double)T / (double)P) / 16.0;
  int64_t k = (int64_t)floor(xd + 0.5);
  if (k < 0) k = 0;
  for (int it = 0; it < 4 && k > 0 && lhs(2 * k - 1) > rhs; ++it) --k;
  for (int it = 0; it < 4 && lhs(2 * k + 1) <= rhs; ++it) ++k;
  gout[idx] = (uint32_t)min<int64_t>(max<int64_t>(k, 1), (1 << 18) - 1);
}

}  // namespace
}  // namespace xeng

extern "C" int xeng_eq_update(const int32_t* d_vis, int64_t n_integrated, const uint32_t* d_gains_in,
                              uint32_t* d_gains_out, int32_t n_chans, int32_t n_inputs,
                              int32_t target_rms_x16, void* hip_stream) {
  if (!d_vis || !d_gains_in || !d_gains_out || n_integrated < 1 || n_integrated > XENG_MAX_INTEGRATION ||
      n_chans < 1 || n_inputs < 1 || n_inputs > XENG_MAX_INPUTS || target_rms_x16 < 1 ||
      target_rms_x16 > 255)
    return XENG_EINVAL;
  const int64_t n = (int64_t)n_chans * n_inputs;
  const int64_t blocks = (n + xeng::THREADS - 1) / xeng::THREADS;
  if (blocks > 2147483647LL) return XENG_EINVAL;
  const int64_t nbl = (int64_t)n_inputs * (n_inputs + 1) / 2;
  hipLaunchKernelGGL(xeng::eq_update, dim3((unsigned)blocks), dim3(xeng::THREADS), 0,
                     reinterpret_cast<hipStream_t>(hip_stream), d_vis, nbl, n_integrated, d_gains_in,
                     d_gains_out, n_chans, n_inputs, target_rms_x16);
  return hipGetLastError() == hipSuccess ? XENG_OK : XENG_EDEVICE;
}

extern "C" int xeng_requantize(const uint64_t* d_words, const uint32_t* d_gains, uint8_t* d_out,
                               int64_t n_time, int32_t n_chans, int32_t n_inputs, void* hip_stream) {
  if (!d_words || !d_gains || !d_out || n_time < 0 || n_chans < 1 || n_inputs < 1) return XENG_EINVAL;
  if ((reinterpret_cast<uintptr_t>(d_words) & 7u) || (reinterpret_cast<uintptr_t>(d_gains) & 3u))
    return XENG_EINVAL;
  if (n_time == 0) return XENG_OK;
  const int64_t fn = (int64_t)n_chans * n_inputs;
  const int64_t ty = (n_time + xeng::ROWS - 1) / xeng::ROWS;
  if (ty > 2147483647LL) return XENG_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  const bool fast = fn % 2 == 0 && (reinterpret_cast<uintptr_t>(d_words) & 15u) == 0 &&
                    (reinterpret_cast<uintptr_t>(d_out) & 1u) == 0 &&
                    (reinterpret_cast<uintptr_t>(d_gains) & 7u) == 0;
  const int64_t cols = fast ? fn / 2 : fn;                      // pairs, or samples
  const int64_t per_wg = fast ? 256 * (xeng::THREADS / 64) : xeng::THREADS;
  const int64_t gx = (cols + per_wg - 1) / per_wg;
  if (gx > 2147483647LL) return XENG_EINVAL;
  const dim3 grid((unsigned)gx, (unsigned)ty);
  if (fast)
    hipLaunchKernelGGL(xeng::requant8, grid, dim3(xeng::THREADS), 0, s, d_words, d_gains, d_out, n_time, cols);
  else
    hipLaunchKernelGGL(xeng::requant1, grid, dim3(xeng::THREADS), 0, s, d_words, d_gains, d_out, n_time, cols);
  return hipGetLastError() == hipSuccess ? XENG_OK : XENG_EDEVICE;
}
