// k_ingest.hip - packet ingest and corner turn on the X side (paper
// Sec. 2.3 and Sec. 2.1), with its C entry point xeng_ingest
// (include/xeng.h).
//
// A packet is an 8-byte application header (6-byte big-endian counter MCNT,
// 1 byte Fid = sending board, 1 byte Xid = destination band) followed by 8
// time samples x C channels x 32 inputs of its board, one byte per complex
// sample, [time, channel, input].  The X-engine wants [time, channel, input]
// over all boards: each packet is one 8 x C x 32 tile of the block
// [8 M][C][32 B] the node integrates.
//
// Two passes: (1) one thread per packet parses its header and records the
// packet number in the (time block, board) slot of an index table (the
// later packet of a duplicate pair wins: atomic max); (2) one workgroup per
// time block writes its rows in consecutive 8-byte words, each taken from
// its board's packet, or zeros where no packet arrived (a lost packet; zero
// samples add nothing to a correlation).  Every output byte is written
// once and every payload byte read once.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/xeng.h"

namespace xeng {
namespace {

constexpr int TIMES = 8;
constexpr int BOARD_INPUTS = 32;

__global__ __launch_bounds__(256) void fill_index(int32_t* idx, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) idx[i] = -1;
}

__global__ __launch_bounds__(256) void index_packets(const uint8_t* __restrict__ pk, int64_t n_packets,
                                                     int64_t stride, uint64_t mcnt0, int64_t n_blocks,
                                                     int n_boards, int xid, int32_t* __restrict__ idx) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= n_packets) return;
  const uint64_t h = *reinterpret_cast<const uint64_t*>(pk + p * stride);
  uint64_t mcnt = 0;
#pragma unroll
  for (int k = 0; k < 6; ++k) mcnt = (mcnt << 8) | ((h >> (8 * k)) & 0xFF);
  const int fid = (int)((h >> 48) & 0xFF), x = (int)((h >> 56) & 0xFF);
  if (x != xid || fid >= n_boards || mcnt < mcnt0 || mcnt - mcnt0 >= (uint64_t)n_blocks) return;
  atomicMax(&idx[(int64_t)(mcnt - mcnt0) * n_boards + fid], (int32_t)p);
}

// One workgroup per time block writes its 8 x C output rows of N bytes in
// 8-byte words; word (b, w) of a row comes from board b's packet.  With a
// multiple of four boards, the words go in tiles of 4 rows x 4 boards x 4
// words per wave: each wave then reads one whole 128-byte line of each of
// four packets (4 consecutive rows of 32 bytes) and writes 128 contiguous
// bytes of each of the 4 rows.
__global__ __launch_bounds__(256) void scatter(const uint8_t* __restrict__ pk, int64_t stride,
                                               const int32_t* __restrict__ idx, int n_boards, int n_chans,
                                               uint8_t* __restrict__ out) {
  const int64_t m = blockIdx.x;
  __shared__ const uint64_t* src[XENG_MAX_INPUTS / BOARD_INPUTS];
  if (threadIdx.x < n_boards) {
    const int p = idx[m * n_boards + threadIdx.x];
    src[threadIdx.x] = p < 0 ? nullptr : reinterpret_cast<const uint64_t*>(pk + (int64_t)p * stride + 8);
  }
  __syncthreads();
  const int row_words = n_boards * 4;                      // N / 8
  const int words = TIMES * n_chans * row_words;
  uint64_t* dst = reinterpret_cast<uint64_t*>(out) + m * words;
  if (n_boards % 4 == 0) {
    // q -> (4-row group, 4-board group, row, board, word), word fastest
    const int groups = n_boards / 4;
    for (int q = threadIdx.x; q < words; q += 256) {
      const int j = q & 63, tile = q >> 6;
      const int row = (tile / groups) * 4 + (j >> 4);      // rows 8C is a multiple of 4
      const int b = (tile % groups) * 4 + ((j >> 2) & 3), w = j & 3;
      const uint64_t* s = src[b];
      dst[(int64_t)row * row_words + b * 4 + w] = s ? s[4 * row + w] : 0ull;
    }
  } else {
    for (int q = threadIdx.x; q < words; q += 256) {
      const int row = q / row_words, wr = q % row_words;   // row = t * C + ch
      const int b = wr >> 2, w = wr & 3;
      const uint64_t* s = src[b];
      dst[q] = s ? s[4 * row + w] : 0ull;
    }
  }
}

}  // namespace
}  // namespace xeng

extern "C" int xeng_ingest(const uint8_t* d_packets, int64_t n_packets, int32_t packet_stride,
                           int64_t mcnt0, int32_t n_blocks, int32_t n_boards, int32_t n_chans, int32_t xid,
                           int32_t* d_index, uint8_t* d_out, void* hip_stream) {
  const int64_t pay = (int64_t)xeng::TIMES * n_chans * xeng::BOARD_INPUTS;
  if (!d_index || !d_out || n_packets < 0 || n_packets > 2147483647LL || (n_packets > 0 && !d_packets) ||
      n_blocks < 1 || n_boards < 1 || n_boards * xeng::BOARD_INPUTS > XENG_MAX_INPUTS || n_chans < 1 ||
      xid < 0 || xid > 255 || mcnt0 < 0 || mcnt0 >= (1LL << 48) || packet_stride < 8 + pay ||
      packet_stride % 8 != 0 || (reinterpret_cast<uintptr_t>(d_packets) & 7u) ||
      (reinterpret_cast<uintptr_t>(d_out) & 7u) || (reinterpret_cast<uintptr_t>(d_index) & 3u) ||
      n_blocks > 65535)
    return XENG_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  const int64_t slots = (int64_t)n_blocks * n_boards;
  hipLaunchKernelGGL(xeng::fill_index, dim3((unsigned)((slots + 255) / 256)), dim3(256), 0, s, d_index, slots);
  if (n_packets > 0)
    hipLaunchKernelGGL(xeng::index_packets, dim3((unsigned)((n_packets + 255) / 256)), dim3(256), 0, s,
                       d_packets, n_packets, (int64_t)packet_stride, (uint64_t)mcnt0, (int64_t)n_blocks,
                       n_boards, xid, d_index);
  hipLaunchKernelGGL(xeng::scatter, dim3((unsigned)n_blocks), dim3(256), 0, s, d_packets,
                     (int64_t)packet_stride, d_index, n_boards, n_chans, d_out);
  return hipGetLastError() == hipSuccess ? XENG_OK : XENG_EDEVICE;
}
