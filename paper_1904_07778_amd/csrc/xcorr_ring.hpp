// xcorr_ring.hpp - gfx950 X-engine kernel for N a multiple of 16.
//
// Result (paper Sec. 2 and Sec. 2.2): for each channel f of the grid and each
// pair 0 <= j <= i < N, the exact int32 sum over the launch's time range of
// x_i(t,f) conj(x_j(t,f)), added into acc[f][i(i+1)/2 + j].
//
// 1. Raw packed bytes go from HBM straight into an LDS ring of S stages
//    (global_load_lds_dwordx4: no registers, many bytes in flight).  A stage
//    holds 64 time samples x CPW channels x N inputs as they sit in HBM
//    ([t][c*N + i]), with the 16-byte chunks of time row t rotated by 2t so
//    the transposed reads below spread over the LDS banks.
//
// 2. Each wave pulls its MFMA fragments with ds_read_b64_tr_b8: in every
//    16-lane group, the 16 lanes' 8-byte reads form an 8 x 16 byte block that
//    comes back transposed, so lane r of group g receives input 16J + r at the
//    8 times 8g .. 8g+7 - the layout of one v_mfma_i32_16x16x64_i8 operand
//    (K = 4 groups x (8 re, 8 im)).
//
// 3. Unpack, scaled by 16 (no sign extension):
//        re16 = w & 0xF0F0F0F0          (16 re per byte, exact int8)
//        im16 = (w << 4) & 0xF0F0F0F0   (16 im per byte)
//    P_J = [re16 | im16] is the B operand of every tile pair and the A
//    operand of the real part; the imaginary part uses
//        Q_I = [im16 | ~re16]   (~x = -x - 1: carry-free, and unlike -x it
//                                cannot overflow int8 at x = -128)
//    so that, summed over the time range,
//        Re'_ij = 256 Re_ij,   Im'_ij = 256 Im_ij - 16 S_j,   S_j = sum_t im_j.
//    Im_jj = 0 gives Im'_jj = -16 S_j: each column's bias is its own diagonal
//    element.  The epilogue forms Re = Re' >> 8 and Im = (Im' - Im'_jj) >> 8,
//    both exact.  |Re'|, |Im'| <= 32896 per sample, so a workgroup integrates
//    at most RING_MAX_T_PER_WG = 32768 samples (the host splits longer ranges).
//
// 4. Work split (PairPlan): the NT(NT+1)/2 tile pairs of the lower triangle,
//    in row-major order, are cut into W contiguous runs whose lengths differ
//    by at most one; wave w of a channel owns run w.  With at most 20 pairs
//    (160 accumulator registers) a wave fits in 256 registers, so two waves
//    share each SIMD and one wave's unpacking overlaps the other's MFMAs.
#pragma once
#include "xcorr.hpp"

namespace xeng {

constexpr int RING_T = 64;                // time samples per ring stage
constexpr int RING_MAX_T_PER_WG = 32768;  // int32 headroom of the x256 sums
template <int NT, int W, int CPW, int S>
struct RingCfg {
  static constexpr int N = NT * 16;
  static constexpr int RP = CPW * N;                 // bytes per time row
  static constexpr int RPC = RP / 16;                // 16-byte chunks per row
  static constexpr int STAGE_BYTES = RING_T * RP;
  static constexpr int LOADS = STAGE_BYTES / 1024;   // wave-wide 1 KB loads per stage (= CPW*NT)
  static constexpr int WAVES = W * CPW;
  static constexpr int THREADS = 64 * WAVES;
  static constexpr int LPW_MAX = (LOADS + WAVES - 1) / WAVES;
  static constexpr int LPW_MIN = LOADS / WAVES;
  static constexpr int DIAG_BYTES = CPW * N * 4;
  static constexpr int LDS_BYTES = S * STAGE_BYTES > DIAG_BYTES ? S * STAGE_BYTES : DIAG_BYTES;
  static_assert(LOADS * 1024 == STAGE_BYTES, "stage must be whole 1 KB loads");
  static_assert(S >= 2, "ring needs two stages");
};

// s_waitcnt vmcnt(n), other counters untouched (gfx9 encoding).
template <int n>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(n >= 0 && n < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((n & 0xF) | ((n >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// Wait until at most `ahead` later stages of this wave's loads are in flight.
template <int LPW>
__device__ __forceinline__ void wait_stage(int ahead) {
  if (ahead >= 3) wait_vmcnt<3 * LPW < 63 ? 3 * LPW : 63>();
  else if (ahead == 2) wait_vmcnt<2 * LPW>();
  else if (ahead == 1) wait_vmcnt<LPW>();
  else wait_vmcnt<0>();
}

// One wave-wide 1 KB load: lane i copies 16 bytes from gptr to LDS byte
// address lds_base + 16 i (global_load_lds_dwordx4, base in M0).  Written as
// asm so the compiler does not treat every later LDS read as dependent on it
// (it would wait for all loads in flight); the ring waits for each stage
// explicitly with s_waitcnt vmcnt + barrier instead.  No register is written.
// M0 is otherwise unused by this code (checked in the generated assembly), so
// declaring it clobbered is safe here.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__device__ __forceinline__ void lds_dma16(const uint8_t* gptr, uint32_t lds_base) {
  asm volatile(
      "s_mov_b32 m0, %1\n\t"
      "global_load_lds_dwordx4 %0, off"
      :
      : "v"(gptr), "s"(lds_base)
      : "memory", "m0");
}
#pragma clang diagnostic pop

__device__ __forceinline__ uint32_t lds_addr(const void* p) {
  return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void*)p;
}

// Mask keeping the first n (clamped to 0..4) bytes of a dword.
__device__ __forceinline__ uint32_t byte_mask(int n) {
  return n >= 4 ? 0xFFFFFFFFu : (n <= 0 ? 0u : ((1u << (8 * n)) - 1u));
}

// Add one wave's tiles into the accumulator of channel f, undoing the x16
// operand scaling (>> 8) and the ~re bias of the imaginary part (subtract the
// column's Im' diagonal, dcol[j]).  Result layout and modes as in xcorr.hpp.
template <int NT, int W, int WC, int MODE, int NP>
__device__ __forceinline__ void ring_epilogue(const Args& a, int f, int lane, const v4i (&accR)[NP],
                                              const v4i (&accI)[NP], const int32_t* dcol) {
  constexpr PairPlan<NT, W> plan{};
  constexpr int NS = plan.nseg[WC];
  constexpr int N = NT * 16;
  constexpr int nbl = N * (N + 1) / 2;
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
      int32_t* rowp = accf + (i * (i + 1) / 2) * 2;
#pragma unroll
      for (int J = J0; J <= J1; ++J) {
        const int j = 16 * J + n;
        if (J == I && j > i) continue;
        int32_t* dst = rowp + 2 * j;
        int re, im;
        asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(re) : "a"(accR[idx + J - J0][vv]));
        asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(im) : "a"(accI[idx + J - J0][vv]));
        re >>= 8;
        im = (im - dcol[j]) >> 8;
        if (MODE == EPI_ATOMIC) {
          atomicAdd(dst, re);
          atomicAdd(dst + 1, im);
        } else if (MODE == EPI_ADD) {
          const v2i old = *reinterpret_cast<const v2i*>(dst);
          *reinterpret_cast<v2i*>(dst) = v2i{old[0] + re, old[1] + im};
        } else {
          *reinterpret_cast<v2i*>(dst) = v2i{re, im};
        }
      }
    }
    idx += J1 - J0 + 1;
  }
}

template <int NT, int W, int CPW, int S, int WC>
__device__ __forceinline__ void ring_wave_main(const Args& a, uint8_t* lds) {
  using C = RingCfg<NT, W, CPW, S>;
  constexpr PairPlan<NT, W> plan{};
  constexpr int NP = plan.npairs[WC];
  constexpr int NS = plan.nseg[WC];
  constexpr int NJ = plan.maxrow[WC] + 1;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c = wave / W;
  const int f0 = blockIdx.x * CPW;
  const int64_t t_begin = (int64_t)blockIdx.y * a.t_chunk;
  const int64_t t_end = min(a.T, t_begin + a.t_chunk);
  if (t_end <= t_begin) return;  // uniform over the workgroup
  const int nt = (int)(t_end - t_begin);
  const int nstages = (nt + RING_T - 1) / RING_T;
  const int64_t row_stride = (int64_t)a.F * C::N;  // bytes between time rows in HBM
  const int nch_valid = min(CPW, a.F - f0);        // the last group may be short of channels

  // ---- producer: wave-wide 1 KB loads q = wave, wave + WAVES, ...
  const int my_loads = (C::LOADS - wave + C::WAVES - 1) / C::WAVES;
  // per-load source offset within a stage and LDS slot, fixed for the whole launch
  int64_t src_off[C::LPW_MAX];
  int src_t[C::LPW_MAX];
#pragma unroll
  for (int k = 0; k < C::LPW_MAX; ++k) {
    const int q = wave + k * C::WAVES;
    const int pos = (q < C::LOADS ? q : 0) * 64 + lane;  // LDS chunk this lane fills
    const int t = pos / C::RPC;                          // time row within the stage
    const int kp = pos % C::RPC;                         // rotated chunk position
    int kl = (kp - 2 * t) % C::RPC;                      // logical chunk stored there
    if (kl < 0) kl += C::RPC;
    int ch = kl / NT;                                    // channel slot of that chunk
    const int kc = kl % NT;                              // 16-input group within the channel
    if (ch >= nch_valid) ch = nch_valid - 1;             // past F: any valid bytes, dropped later
    src_t[k] = t;
    src_off[k] = (int64_t)(f0 + ch) * C::N + 16 * kc;
  }
  auto issue_stage = [&](int st) {
    uint8_t* dst = lds + (st % S) * C::STAGE_BYTES;
    const int64_t tb = t_begin + (int64_t)st * RING_T;
#pragma unroll
    for (int k = 0; k < C::LPW_MAX; ++k) {
      const int q = wave + k * C::WAVES;
      if (q < C::LOADS) {
        int64_t tt = tb + src_t[k];
        if (tt >= t_end) tt = t_end - 1;  // tail rows: valid bytes, zeroed by the reader
        lds_dma16(a.v + tt * row_stride + src_off[k],
                  __builtin_amdgcn_readfirstlane(lds_addr(dst + q * 1024)));
      }
    }
  };

  // ---- consumer
  v4i accR[NP], accI[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    accR[p] = v4i{0, 0, 0, 0};
    accI[p] = v4i{0, 0, 0, 0};
  }
  const int r = lane & 15, g = lane >> 4;
  // lane (g, r) of a tr8 read points at time row 8g + r/2, input half 8(r&1)
  const int tr_row = 8 * g + (r >> 1);
  const int tr_half = 8 * (r & 1);

#pragma unroll
  for (int st = 0; st < S - 1; ++st)
    if (st < nstages) issue_stage(st);

  for (int st = 0; st < nstages; ++st) {
    const int ahead = min(S - 2, nstages - 1 - st);  // later stages already issued
    if (my_loads == C::LPW_MAX)
      wait_stage<C::LPW_MAX>(ahead);
    else
      wait_stage<C::LPW_MIN>(ahead);
    __syncthreads();  // stage st landed for every wave; slot of st-1 free
    if (st + S - 1 < nstages) issue_stage(st + S - 1);

    const uint8_t* stage = lds + (st % S) * C::STAGE_BYTES;
    const int valid_t = min(RING_T, nt - st * RING_T);
#pragma unroll 1
    for (int ks = 0; ks < RING_T / KS; ++ks) {
      const int trow = ks * KS + tr_row;
      const uint8_t* rowp = stage + trow * C::RP + tr_half;
      const int nvalid = valid_t - (ks * KS + 8 * g);  // valid samples of this lane's 8
      v4i p[NJ];
#pragma unroll
      for (int J = 0; J < NJ; ++J) {
        int kp = c * NT + J + 2 * trow;
        kp %= C::RPC;
        const v2i w = __builtin_amdgcn_ds_read_tr8_b64_v2i32(
            (__attribute__((address_space(3))) v2i*)(rowp + kp * 16));
        uint32_t w0 = (uint32_t)w[0], w1 = (uint32_t)w[1];
        if (nvalid < 8) {
          w0 &= byte_mask(nvalid);
          w1 &= byte_mask(nvalid - 4);
        }
        p[J] = v4i{(int)(w0 & 0xF0F0F0F0u), (int)(w1 & 0xF0F0F0F0u),
                   (int)((w0 << 4) & 0xF0F0F0F0u), (int)((w1 << 4) & 0xF0F0F0F0u)};
      }
      int idx = 0;
#pragma unroll
      for (int sg = 0; sg < NS; ++sg) {
        const int I = plan.segI[WC][sg];
        const v4i q = v4i{p[I][2], p[I][3], ~p[I][0], ~p[I][1]};
#pragma unroll
        for (int J = plan.segJ0[WC][sg]; J <= plan.segJ1[WC][sg]; ++J) {
          accR[idx] = __builtin_amdgcn_mfma_i32_16x16x64_i8(p[I], p[J], accR[idx], 0, 0, 0);
          accI[idx] = __builtin_amdgcn_mfma_i32_16x16x64_i8(q, p[J], accI[idx], 0, 0, 0);
          ++idx;
        }
      }
    }
  }

  // ---- epilogue: publish each column's Im' diagonal through LDS, then add
  __syncthreads();  // the ring is no longer read
  int32_t* diag = reinterpret_cast<int32_t*>(lds);  // [CPW][N]
  {
    const int n = lane & 15, m0 = 4 * (lane >> 4);
    int idx = 0;
#pragma unroll
    for (int sg = 0; sg < NS; ++sg) {
      const int I = plan.segI[WC][sg];
      const int J1 = plan.segJ1[WC][sg];
      idx += J1 - plan.segJ0[WC][sg];
      if (J1 == I) {
#pragma unroll
        for (int vv = 0; vv < 4; ++vv) {
          if (m0 + vv == n) {
            int d;
            asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(d) : "a"(accI[idx][vv]));
            diag[c * C::N + 16 * I + n] = d;
          }
        }
      }
      ++idx;
    }
  }
  __syncthreads();
  const int f = f0 + c;
  if (f >= a.F) return;
  const int32_t* dcol = diag + c * C::N;
  if (a.mode == EPI_ATOMIC)
    ring_epilogue<NT, W, WC, EPI_ATOMIC>(a, f, lane, accR, accI, dcol);
  else if (a.mode == EPI_ADD)
    ring_epilogue<NT, W, WC, EPI_ADD>(a, f, lane, accR, accI, dcol);
  else
    ring_epilogue<NT, W, WC, EPI_STORE>(a, f, lane, accR, accI, dcol);
}

template <int NT, int W, int CPW, int S, int WC>
__device__ __forceinline__ void ring_dispatch(int wc, const Args& a, uint8_t* lds) {
  if constexpr (WC < W) {
    if (wc == WC)
      ring_wave_main<NT, W, CPW, S, WC>(a, lds);
    else
      ring_dispatch<NT, W, CPW, S, WC + 1>(wc, a, lds);
  }
}

// Launch shape per tile count: W waves per channel (PairPlan), CPW channels
// per workgroup (about 8 waves per workgroup), S ring stages (about 96 KB of
// LDS, of which S-1 stages are in flight).
constexpr int ring_cpw(int nt) {
  const int w = waves_for(nt);
  return w >= 8 ? 1 : (8 / w > 8 ? 8 : 8 / w);
}
constexpr int ring_stages(int nt) {
  const int stage = RING_T * 16 * nt * ring_cpw(nt);
  const int s = (96 * 1024) / stage;
  return s < 3 ? 3 : (s > 6 ? 6 : s);
}

template <int NT, int W, int CPW, int S>
__global__ __launch_bounds__((RingCfg<NT, W, CPW, S>::THREADS))
__attribute__((amdgpu_waves_per_eu(2))) void xcorr_ring_kernel(Args a) {
  __shared__ __attribute__((aligned(1024))) uint8_t lds[RingCfg<NT, W, CPW, S>::LDS_BYTES];
  const int wc = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) % W;
  ring_dispatch<NT, W, CPW, S, 0>(wc, a, lds);
}

}  // namespace xeng
