// xcorr.hpp - gfx950 X-engine kernel: 4+4-bit complex voltages -> int32
// visibilities of every input pair (lower triangle, autos included).
//
// What one launch computes (paper Sec. 2 and Sec. 2.2): for each channel f of
// the grid and each pair 0 <= j <= i < N,
//     acc[f][i(i+1)/2 + j] += sum_t x_i(t,f) conj(x_j(t,f))
// over the time range of the launch, exactly, in int32.
//
// How.  With x = a + jb,  Re = sum(a_i a_j + b_i b_j),  Im = sum(b_i a_j - a_i b_j).
// Put the samples of input i over a block of 32 times into the int8 row
//     P_i = [a_i(t..) | b_i(t..)]                   (64 bytes = K of one MFMA)
// and its rotated copy
//     Q_i = [b_i(t..) | -a_i(t..)].
// Then Re_ij = P_i . P_j and Im_ij = Q_i . P_j, so each 16x16 tile pair (I, J),
// I >= J, of the lower triangle is two v_mfma_i32_16x16x64_i8 per 32 samples,
// exact in int32 (|Re|, |Im| <= 128 per sample).
//
// Data flow per workgroup (CPW channels, one time range):
//   HBM  uint8 [T][F][N]   rows of CPW*N contiguous bytes per time sample
//    |  staging threads: dword loads of 4 inputs x 8 times, 4x4 byte transposes
//    |  (v_perm), nibble unpack to sign-extended int8 re, im and -re
//   LDS  PA[c][g][i] 16 B = {re t0..3, re t4..7, im t0..3, im t4..7}
//        NA[c][g][i]  8 B = {-re t0..3, -re t4..7}      (g = 8-sample group)
//    |  double buffered, one barrier per 32-sample step
//   waves: ds_read_b128 of the 16-row fragments, MFMA into register tiles
//   epilogue: add the tiles into the HBM-resident accumulator: plain stores
//   right after a dump, read-modify-write when one workgroup owns the
//   channel, atomics when the time range is split over several workgroups.
//
// Work split inside a channel: see PairPlan below.  Each wave keeps all of its
// accumulators in registers for the whole time range.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xeng {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v2i __attribute__((ext_vector_type(2)));
typedef int v6i __attribute__((ext_vector_type(6)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int KS = 32;  // time samples per MFMA K step (64 int8 = 32 x (re, im))
// The staging kernel sums exact int8 products (|Re|, |Im| <= 128 per sample),
// so any range up to the library's integration limit fits int32.
constexpr int64_t XENG_MAX_T_PER_WG_STAGE = 16777215;

// Work split inside a channel: the NT(NT+1)/2 tile pairs (I, J), J <= I, of
// the lower triangle, taken in row-major order, are cut into W contiguous runs
// whose lengths differ by at most one; wave w of the channel owns run w as a
// list of row segments (I, J0..J1).
constexpr int PAIRS_PER_WAVE = 20;  // 160 accumulator registers per wave

template <int NT, int W>
struct PairPlan {
  int nseg[W];          // rows touched by wave w
  int segI[W][NT];      // tile row of each segment
  int segJ0[W][NT];     // first tile column
  int segJ1[W][NT];     // last tile column (inclusive)
  int npairs[W];
  int maxrow[W];
  constexpr PairPlan() : nseg(), segI(), segJ0(), segJ1(), npairs(), maxrow() {
    const int total = NT * (NT + 1) / 2;
    for (int w = 0; w < W; ++w) {
      const int b = w * total / W, e = (w + 1) * total / W;
      npairs[w] = e - b;
      maxrow[w] = -1;
      int p = 0;
      for (int I = 0; I < NT; ++I) {
        for (int J = 0; J <= I; ++J, ++p) {
          if (p < b || p >= e) continue;
          if (nseg[w] > 0 && segI[w][nseg[w] - 1] == I) {
            segJ1[w][nseg[w] - 1] = J;
          } else {
            segI[w][nseg[w]] = I;
            segJ0[w][nseg[w]] = J;
            segJ1[w][nseg[w]] = J;
            ++nseg[w];
          }
          maxrow[w] = I;
        }
      }
    }
  }
};

// Waves per channel that keep every wave within PAIRS_PER_WAVE tile pairs.
constexpr int waves_for(int nt) { return (nt * (nt + 1) / 2 + PAIRS_PER_WAVE - 1) / PAIRS_PER_WAVE; }

template <int NT, int W, int CPW>
struct Cfg {
  static constexpr int NPAD = NT * 16;
  static constexpr int NQ = NPAD / 4;               // 4-input groups per channel
  static constexpr int WAVES = W * CPW;
  static constexpr int THREADS = 64 * WAVES;
  static constexpr int UNITS = 4 * CPW * NQ;        // (g, c, q) staging units per step
  static constexpr int UPT = (UNITS + THREADS - 1) / THREADS;
  static constexpr int PA_BYTES = CPW * 4 * NPAD * 16;
  static constexpr int NA_BYTES = CPW * 4 * NPAD * 8;
  static constexpr int BUF_BYTES = PA_BYTES + NA_BYTES;
  static constexpr int LDS_BYTES = 2 * BUF_BYTES;
};

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
  return __builtin_amdgcn_perm(hi, lo, sel);
}

// 4x4 byte transpose: byte c of d_r is x[r][c]; byte r of e_c becomes x[r][c].
__device__ __forceinline__ void transpose4x4(uint32_t d0, uint32_t d1, uint32_t d2, uint32_t d3,
                                             uint32_t& e0, uint32_t& e1, uint32_t& e2,
                                             uint32_t& e3) {
  const uint32_t t0 = perm(d1, d0, 0x05010400u);  // x00 x10 x01 x11
  const uint32_t t1 = perm(d1, d0, 0x07030602u);  // x02 x12 x03 x13
  const uint32_t t2 = perm(d3, d2, 0x05010400u);  // x20 x30 x21 x31
  const uint32_t t3 = perm(d3, d2, 0x07030602u);  // x22 x32 x23 x33
  e0 = perm(t2, t0, 0x05040100u);                 // x00 x10 x20 x30
  e1 = perm(t2, t0, 0x07060302u);                 // x01 x11 x21 x31
  e2 = perm(t3, t1, 0x05040100u);                 // x02 x12 x22 x32
  e3 = perm(t3, t1, 0x07060302u);                 // x03 x13 x23 x33
}

// Four packed samples -> sign-extended int8 re, im and -re, byte-parallel.
// With h = code ^ 8 = value + 8 in [0, 15]:
//   value  = (h + 120) ^ 128   (h + 120 < 256, so no carry leaves a byte)
//   -value = (136 - h) ^ 128   (136 - h >= 0, so no borrow leaves a byte)
// The all-zero byte (padding) gives re = im = -re = 0.
__device__ __forceinline__ void unpack4(uint32_t w, uint32_t& re, uint32_t& im, uint32_t& nre) {
  const uint32_t x = w ^ 0x88888888u;
  const uint32_t h = (x >> 4) & 0x0F0F0F0Fu;
  const uint32_t l = x & 0x0F0F0F0Fu;
  re = (h + 0x78787878u) ^ 0x80808080u;
  im = (l + 0x78787878u) ^ 0x80808080u;
  nre = (0x88888888u - h) ^ 0x80808080u;
}

__device__ __forceinline__ uint32_t load_group(const uint8_t* p, int navail, bool aligned) {
  if (aligned) return __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(p));
  uint32_t w = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (k < navail) w |= (uint32_t)p[k] << (8 * k);
  return w;
}

// Channel group of a workgroup.  Workgroups are dealt round-robin to the
// eight XCDs (each with its own L2); this bijection on [0, groups) gives each
// XCD a contiguous band of channel groups, so neighbouring channels, whose
// rows share 128-byte lines in HBM, are fetched through the same L2.
constexpr int NUM_XCD = 8;
__device__ __forceinline__ int xcd_group(int b, int groups) {
  const int q = groups / NUM_XCD, r = groups % NUM_XCD;
  const int x = b % NUM_XCD, k = b / NUM_XCD;
  return x * q + (x < r ? x : r) + k;
}

// Wait states between the last MFMAs and the epilogue, whose accumulator
// reads are inline asm (v_accvgpr_read) and so not covered by the compiler's
// hazard handling: a VALU read of a 16-pass MFMA result needs 19 (an 8-pass
// one 11); this gives 32.  Without it the first reads of the last-written
// tiles can see values from before the final MFMA.
__device__ __forceinline__ void mfma_drain() {
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7\n\ts_nop 7" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
}

struct Args {
  const uint8_t* v;  // [T][F][N]
  int32_t* acc;      // [F][nbl][2]
  int64_t T;         // samples in this call
  int F, N;
  int64_t t_chunk;   // samples per workgroup along time (multiple of KS)
  int mode;          // EpiMode
};

// How a launch leaves its sums in the accumulator.
enum EpiMode : int {
  EPI_STORE = 0,   // accumulator known to be zero: plain stores
  EPI_ADD = 1,     // one workgroup per channel: read-modify-write
  EPI_ATOMIC = 2   // time range split over workgroups: atomic adds
};

// Add one wave's register tiles into the accumulator of channel f.  MFMA
// result layout (16x16): lane holds column n = lane & 15 of rows
// 4*(lane >> 4) + v, v = 0..3.  Within a tile row, the 16 columns of one
// output row are 16 consecutive baselines, so each store instruction writes
// four 128-byte runs.  The tiles live in AGPRs; each value is moved to a
// VGPR right where it is used (v_accvgpr_read), which keeps the compiler from
// copying every tile out of the AGPRs at once when the main loop ends.
template <int NT, int W, int WC, int MODE, int NP>
__device__ __forceinline__ void epilogue(const Args& a, int f, int lane, const v4i (&accR)[NP],
                                         const v4i (&accI)[NP]) {
  constexpr PairPlan<NT, W> plan{};
  constexpr int NS = plan.nseg[WC];
  const int nbl = a.N * (a.N + 1) / 2;
  int32_t* accf = a.acc + (int64_t)f * nbl * 2;
  const int n = lane & 15;
  const int m0 = 4 * (lane >> 4);
  int idx = 0;
#pragma unroll
  for (int sg = 0; sg < NS; ++sg) {
    const int I = plan.segI[WC][sg];
    const int J0 = plan.segJ0[WC][sg], J1 = plan.segJ1[WC][sg];
#pragma unroll
    for (int vv = 0; vv < 4; ++vv) {
      const int i = 16 * I + m0 + vv;
      if (i >= a.N) continue;
      int32_t* rowp = accf + (i * (i + 1) / 2) * 2;
      // read-modify-write: the row's prior values first (distinct baselines),
      // then the sums, one memory round trip per row segment
      v2i prev[NT];
      if (MODE == EPI_ADD) {
#pragma unroll
        for (int J = J0; J <= J1; ++J) {
          const int j = 16 * J + n;
          if (J == I && j > i) continue;
          prev[J - J0] = *reinterpret_cast<const v2i*>(rowp + 2 * j);
        }
      }
#pragma unroll
      for (int J = J0; J <= J1; ++J) {
        const int j = 16 * J + n;
        if (J == I && j > i) continue;
        int32_t* dst = rowp + 2 * j;
        int re, im;
        asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(re) : "a"(accR[idx + J - J0][vv]));
        asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(im) : "a"(accI[idx + J - J0][vv]));
        if (MODE == EPI_ATOMIC) {
          atomicAdd(dst, re);
          atomicAdd(dst + 1, im);
        } else if (MODE == EPI_ADD) {
          *reinterpret_cast<v2i*>(dst) = prev[J - J0] + v2i{re, im};
        } else {
          *reinterpret_cast<v2i*>(dst) = v2i{re, im};
        }
      }
    }
    idx += J1 - J0 + 1;
  }
}

template <int NT, int W, int CPW, int WC>
__device__ __forceinline__ void wave_main(const Args& a, uint8_t* lds) {
  using C = Cfg<NT, W, CPW>;
  constexpr PairPlan<NT, W> plan{};
  constexpr int NP = plan.npairs[WC];
  constexpr int NS = plan.nseg[WC];
  constexpr int NJ = plan.maxrow[WC] + 1;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int c = (tid >> 6) / W;               // channel slot of this wave
  const int r = lane & 15, g = lane >> 4;     // fragment row, 8-sample group
  const int f0 = xcd_group(blockIdx.x, gridDim.x) * CPW;
  const int64_t t_begin = (int64_t)blockIdx.y * a.t_chunk;
  const int64_t t_end = min(a.T, t_begin + a.t_chunk);
  if (t_end <= t_begin) return;  // uniform over the workgroup
  const int nsteps = (int)((t_end - t_begin + KS - 1) / KS);
  const bool aligned = (a.N & 3) == 0;
  const int64_t row_stride = (int64_t)a.F * a.N;

  v4i accR[NP], accI[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    accR[p] = v4i{0, 0, 0, 0};
    accI[p] = v4i{0, 0, 0, 0};
  }

  uint32_t pre[C::UPT][8];

  auto load_step = [&](int s) {
    const int64_t tb = t_begin + (int64_t)s * KS;
#pragma unroll
    for (int k = 0; k < C::UPT; ++k) {
      const int u = tid + k * C::THREADS;
      const int q = u % C::NQ;
      const int cu = (u / C::NQ) % CPW;
      const int gu = u / (C::NQ * CPW);
      const int f = f0 + cu;
      const int i0 = 4 * q;
      const bool ok = (u < C::UNITS) && (f < a.F) && (i0 < a.N);
      const uint8_t* base = a.v + (int64_t)f * a.N + i0;
#pragma unroll
      for (int rr = 0; rr < 8; ++rr) {
        const int64_t t = tb + 8 * gu + rr;
        pre[k][rr] = (ok && t < t_end) ? load_group(base + t * row_stride, a.N - i0, aligned) : 0u;
      }
    }
  };

  auto store_step = [&](int buf) {
    uint8_t* pa = lds + buf * C::BUF_BYTES;
    uint8_t* na = pa + C::PA_BYTES;
#pragma unroll
    for (int k = 0; k < C::UPT; ++k) {
      const int u = tid + k * C::THREADS;
      if (u >= C::UNITS) continue;
      const int q = u % C::NQ;
      const int cu = (u / C::NQ) % CPW;
      const int gu = u / (C::NQ * CPW);
      uint32_t e[8];
      transpose4x4(pre[k][0], pre[k][1], pre[k][2], pre[k][3], e[0], e[1], e[2], e[3]);
      transpose4x4(pre[k][4], pre[k][5], pre[k][6], pre[k][7], e[4], e[5], e[6], e[7]);
      const int row0 = (cu * 4 + gu) * C::NPAD + 4 * q;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        uint32_t re0, im0, nre0, re1, im1, nre1;
        unpack4(e[m], re0, im0, nre0);
        unpack4(e[4 + m], re1, im1, nre1);
        *reinterpret_cast<v4i*>(pa + (row0 + m) * 16) = v4i{(int)re0, (int)re1, (int)im0, (int)im1};
        *reinterpret_cast<v2i*>(na + (row0 + m) * 8) = v2i{(int)nre0, (int)nre1};
      }
    }
  };

  auto compute = [&](int buf) {
    const uint8_t* pa = lds + buf * C::BUF_BYTES;
    const uint8_t* na = pa + C::PA_BYTES;
    const int frag0 = (c * 4 + g) * C::NPAD + r;
    v4i p[NJ];
#pragma unroll
    for (int J = 0; J < NJ; ++J) p[J] = *reinterpret_cast<const v4i*>(pa + (frag0 + 16 * J) * 16);
    int idx = 0;
#pragma unroll
    for (int sg = 0; sg < NS; ++sg) {
      const int I = plan.segI[WC][sg];
      const v2i n = *reinterpret_cast<const v2i*>(na + (frag0 + 16 * I) * 8);
      const v4i q = v4i{p[I][2], p[I][3], n[0], n[1]};
#pragma unroll
      for (int J = plan.segJ0[WC][sg]; J <= plan.segJ1[WC][sg]; ++J) {
        accR[idx] = __builtin_amdgcn_mfma_i32_16x16x64_i8(p[I], p[J], accR[idx], 0, 0, 0);
        accI[idx] = __builtin_amdgcn_mfma_i32_16x16x64_i8(q, p[J], accI[idx], 0, 0, 0);
        ++idx;
      }
    }
  };

  load_step(0);
  store_step(0);
  __syncthreads();
  for (int s = 0; s < nsteps; ++s) {
    const int buf = s & 1;
    const bool more = s + 1 < nsteps;
    if (more) load_step(s + 1);
    compute(buf);
    if (more) store_step(buf ^ 1);
    __syncthreads();
  }
  mfma_drain();

  const int f = f0 + c;
  if (f >= a.F) return;
  if (a.mode == EPI_ATOMIC)
    epilogue<NT, W, WC, EPI_ATOMIC>(a, f, lane, accR, accI);
  else if (a.mode == EPI_ADD)
    epilogue<NT, W, WC, EPI_ADD>(a, f, lane, accR, accI);
  else
    epilogue<NT, W, WC, EPI_STORE>(a, f, lane, accR, accI);
}

template <int NT, int W, int CPW, int WC>
__device__ __forceinline__ void dispatch_wave(int wc, const Args& a, uint8_t* lds) {
  if constexpr (WC < W) {
    if (wc == WC)
      wave_main<NT, W, CPW, WC>(a, lds);
    else
      dispatch_wave<NT, W, CPW, WC + 1>(wc, a, lds);
  }
}

template <int NT, int W, int CPW>
__global__ __launch_bounds__((Cfg<NT, W, CPW>::THREADS)) void xcorr_kernel(Args a) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[Cfg<NT, W, CPW>::LDS_BYTES];
  const int wc = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) % W;
  dispatch_wave<NT, W, CPW, 0>(wc, a, lds);
}

}  // namespace xeng
