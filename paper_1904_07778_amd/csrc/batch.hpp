// batch.hpp - one persistent launch over the X-engine work of many arrays.
//
// The paper gives each GPU of an X node a band of channels (Sec. 2, Sec. 2.2)
// and runs one kernel per band.  Here many independent arrays, of uneven
// input counts, channel counts and integration lengths, share one GPU: their
// work is cut into items (array, channel group, time chunk) and a single
// persistent grid of one workgroup per compute unit pulls items from work
// queues until all are done.  Every item runs the same per-wave body as the
// plain launch of the 16-row-tile kernel (x16::wave_main) with the launch
// shape compiled for its N, so the sums are bit-identical to the plain
// engine's.
//
// Queues.  There is one queue per XCD (workgroup w runs on XCD w % 8).  Each
// array's channel groups are cut into 8 contiguous ranges, one per queue;
// inside a queue the items of one array are taken channel group fastest,
// so the workgroups of one XCD work on neighbouring channels at the same
// time and share the 128-byte lines that straddle two channels in its L2.
// Arrays are listed in the order the host chose (longest items first).  A
// workgroup whose queue is empty takes items from the next queues in turn.
//
// Counters.  counters[0..7] are the queue heads and counters[8] counts the
// workgroups that have finished; all are zero before a launch.  The last
// workgroup to finish resets them, with device-scope atomics, so the next
// launch (for instance the next replay of a captured graph) finds them zero
// without any memset.
#pragma once
#include "xcorr16.hpp"

namespace xeng {
namespace batch {

constexpr int MAX_ARRAYS = 24;   // arrays per launch (kernel-argument space)
constexpr int QUEUES = NUM_XCD;
constexpr int THREADS = 256;     // four waves: the shape of every N <= 192 kernel
constexpr int MAX_N = 192;

// N that the batch kernel is built for: multiples of 16 up to 192.
constexpr bool supports(int n) { return n >= 16 && n <= MAX_N && n % 16 == 0; }

struct Params {
  Args arr[MAX_ARRAYS];          // per array: voltages, accumulator, T, F, N, t_chunk, mode
  int32_t ngroups[MAX_ARRAYS];   // channel groups (ceil(F / CPW))
  int32_t nchunks[MAX_ARRAYS];   // time chunks
  int32_t n_arrays;
  int32_t* counters;             // [QUEUES + 1], zero between launches
};

// Channel groups [begin, end) of queue x for an array with g groups.
__host__ __device__ inline int range_begin(int g, int x) { return (int)((int64_t)g * x / QUEUES); }

// LDS of the largest launch shape among the supported N.
template <int N = 16>
constexpr int lds_bytes() {
  if constexpr (N > MAX_N) {
    return 0;
  } else {
    constexpr int own =
        x16::Shape<N, x16::cpw_for(N), x16::stages_for(N, x16::KPS_DEFAULT), x16::KPS_DEFAULT>::LDS_BYTES;
    constexpr int rest = lds_bytes<N + 16>();
    return own > rest ? own : rest;
  }
}

template <int N>
__device__ __forceinline__ void run_if(int n, const Args& a, uint8_t* lds, int group, int tchunk, int tid) {
  if constexpr (N <= MAX_N) {
    if (n == N)
      x16::run_item<N, x16::KPS_DEFAULT>(a, lds, group, tchunk, tid);
    else
      run_if<N + 16>(n, a, lds, group, tchunk, tid);
  }
}

// The persistent kernel (k_batch.hip) and its host-side launch.
hipError_t launch(int grid, hipStream_t s, const Params& p);
const void* kernel_function();

}  // namespace batch
}  // namespace xeng
