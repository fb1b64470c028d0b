// xcorr32.hpp - gfx950 X-engine kernel for N a multiple of 16 (32-row tiles).
//
// Result (paper Sec. 2 and Sec. 2.2): for each channel f of the grid and each
// pair 0 <= j <= i < N, the exact int32 sum over the launch's time range of
// x_i(t,f) conj(x_j(t,f)), added into acc[f][i(i+1)/2 + j].
//
// 1. HBM -> LDS ring.  Raw packed bytes go straight into an LDS ring of S
//    stages with global_load_lds_dwordx4 (no registers; S-1 stages in
//    flight).  A stage holds 64 time samples; its time row t holds the CPW*N
//    bytes of the workgroup's channels ([c*N + i], as in HBM) in 16-byte
//    chunks at a pitch of RPP chunks, RPP odd, so that 16 consecutive rows
//    start on 16 different 16-byte bank groups (the spare chunk of a row is
//    filled with a duplicate of its first chunk, which costs no HBM traffic).
//
// 2. Fragments.  ds_read_b64_tr_b8 transposes, in every 16-lane group, the
//    8 x 16 byte block formed by the lanes' 8-byte reads.  Lane l of a wave
//    reads time row 16h + 8(l/32) + ((l%16)/2), bytes 32J + 16((l/16)%2) +
//    8(l%2) of its channel, and receives input 32J + (l%32) at the 8 times
//    16h + 8(l/32) .. +7: one operand of v_mfma_i32_32x32x32_i8 (row l%32,
//    K group l/32) for K-half h (16 samples) of a 32-sample step.
//
// 3. Unpack, scaled by 16 (no sign extension):
//        re16 = w & 0xF0F0F0F0,   im16 = (w << 4) & 0xF0F0F0F0
//    P = [re16 | im16] is the B operand of every product and the A operand
//    of the real part; the imaginary part uses Q = [im16 | ~re16] (~x = -x-1,
//    carry-free, and never overflows int8).  Summed over time:
//        Re'_ij = 256 Re_ij,   Im'_ij = 256 Im_ij - 16 S_j,   S_j = sum_t im_j
//    and Im_jj = 0 gives Im'_jj = -16 S_j, so the epilogue forms
//        Re = Re' >> 8,   Im = (Im' - Im'_jj) >> 8   exactly.
//    |Re'|, |Im'| <= 32896 per sample: a workgroup integrates at most
//    MAX_T_PER_WG = 32768 samples (the host splits longer ranges).
//
// 4. Work split (UnitPlan).  A unit is the real or the imaginary product of
//    one 32 x 32 tile pair (I, J), J <= I: 16 accumulator registers.  The
//    NT(NT+1) units of a channel, in row-major order (I, then J, Re then
//    Im), are cut into W contiguous runs; the runs one unit longer go to the
//    first waves.  A workgroup has four waves, one per SIMD, each with up to
//    11 units (176 accumulator registers); the next K-step's reads and
//    unpacking are independent of the current step's MFMAs, so one wave
//    keeps its SIMD's matrix core busy.  (For N > 192 eight waves of at
//    most 9 units share the four SIMDs.)
#pragma once
#include <type_traits>

#include "xcorr.hpp"

namespace xeng {
namespace x32 {

constexpr int STAGE_T = 64;           // time samples per ring stage
constexpr int MAX_T_PER_WG = 32768;   // int32 headroom of the x256 sums
constexpr int MAX_UNITS_PER_WAVE = 11;

template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    sfor<B + 1, E>(f);
  }
}

// 32-row tiles of an N-input channel and the launch shape for them.
constexpr int tiles(int n) { return (n + 31) / 32; }
constexpr int units(int nt) { return nt * (nt + 1); }
constexpr int waves_per_channel(int nt) {
  return units(nt) <= MAX_UNITS_PER_WAVE ? 1
       : units(nt) <= 2 * MAX_UNITS_PER_WAVE ? 2
       : units(nt) <= 4 * MAX_UNITS_PER_WAVE ? 4 : 8;
}
// Up to four waves per channel: one workgroup of four waves, one wave per
// SIMD (up to 176 accumulator registers each).  Eight waves per channel
// (N > 192): two waves per SIMD, at most 9 units (144 registers) each.
constexpr int waves_per_wg(int nt) { return waves_per_channel(nt) <= 4 ? 4 : 8; }

template <int NT, int W>
struct UnitPlan {
  static constexpr int U = units(NT);
  static constexpr int MAXU = (U + W - 1) / W;
  int nu[W];
  int uI[W][MAXU];
  int uJ[W][MAXU];
  int uIm[W][MAXU];
  bool needP[W][NT];   // tile read as an operand
  bool needQ[W][NT];   // tile used as the row of an imaginary product
  constexpr UnitPlan() : nu(), uI(), uJ(), uIm(), needP(), needQ() {
    const int q = U / W, rem = U % W;
    int u = 0, w = 0, k = 0;
    for (int I = 0; I < NT; ++I)
      for (int J = 0; J <= I; ++J)
        for (int part = 0; part < 2; ++part) {
          while (k == q + (w < rem ? 1 : 0)) {  // this wave's run is full
            ++w;
            k = 0;
          }
          uI[w][k] = I;
          uJ[w][k] = J;
          uIm[w][k] = part;
          needP[w][I] = needP[w][J] = true;
          if (part) needQ[w][I] = true;
          ++k;
          nu[w] = k;
          ++u;
        }
  }
};

template <int N, int CPW, int S>
struct Shape {
  static constexpr int NT = tiles(N);
  static constexpr int W = waves_per_channel(NT);
  static constexpr int THREADS = 64 * W * CPW;
  static constexpr int RPC = CPW * N / 16;            // 16-byte chunks of data per time row
  static constexpr int RPP = RPC | 1;                 // odd row pitch in chunks
  static constexpr int STAGE_BYTES = STAGE_T * RPP * 16;
  static constexpr int LOADS = STAGE_BYTES / 1024;    // wave-wide 1 KB loads per stage (= RPP)
  static constexpr int WAVES = W * CPW;
  static constexpr int LPW_MAX = (LOADS + WAVES - 1) / WAVES;
  static constexpr int LPW_MIN = LOADS / WAVES;
  static constexpr int DIAG_BYTES = CPW * NT * 32 * 4;
  static constexpr int LDS_BYTES = S * STAGE_BYTES > DIAG_BYTES ? S * STAGE_BYTES : DIAG_BYTES;
  static_assert(N % 16 == 0, "N must be a multiple of 16");
  static_assert(LOADS * 1024 == STAGE_BYTES, "a stage is whole 1 KB loads");
  static_assert(S >= 2 && (S - 2) * LPW_MAX < 64, "ring depth");
};

// Launch shape per N: W waves per channel, CPW channels per workgroup, and
// as many ring stages as fit 128 KB (3 to 8).
constexpr int cpw_for(int n) { return waves_per_wg(tiles(n)) / waves_per_channel(tiles(n)); }
constexpr int stages_for(int n) {
  const int stage = STAGE_T * ((cpw_for(n) * n / 16) | 1) * 16;
  const int s = (128 * 1024) / stage;
  return s < 3 ? 3 : (s > 8 ? 8 : s);
}

template <int n>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(n >= 0 && n < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((n & 0xF) | ((n >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// One wave-wide 1 KB load: lane i copies 16 bytes from gptr to LDS byte
// address lds_base + 16 i (global_load_lds_dwordx4, base in M0).  Written as
// asm so the compiler does not make every later LDS read wait for all loads
// in flight; the ring waits for each stage with s_waitcnt vmcnt + barrier.
// No register is written.  M0 is otherwise unused by this code (checked in
// the generated assembly), so clobbering it is safe.
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

__device__ __forceinline__ uint32_t byte_mask(int n) {
  return n >= 4 ? 0xFFFFFFFFu : (n <= 0 ? 0u : ((1u << (8 * n)) - 1u));
}

__device__ __forceinline__ v16i mfma32(v4i a, v4i b, v16i c) {
  return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
}


// Add one wave's tiles into the accumulator of channel f.  32x32 result
// layout: lane l, register v hold row 8(v/4) + 4(l/32) + v%4, column l%32;
// the 32 lanes of a half-wave write 32 consecutive baselines of one row.
template <int N, int W, int WC, int MODE, int NU>
__device__ __forceinline__ void epilogue(const Args& a, int f, int lane, const v16i (&acc)[NU],
                                         const int32_t* dcol) {
  constexpr int NT = tiles(N);
  constexpr UnitPlan<NT, W> plan{};
  constexpr int nbl = N * (N + 1) / 2;
  int32_t* accf = a.acc + (int64_t)f * nbl * 2;
  const int n = lane & 31;
  const int mb = 4 * (lane >> 5);
  // calls body(u, v, pair, im, dst, bias) for every site (unit u, register
  // v) this lane holds among units [U0, U1); bias: the diagonal value D_j
  // for the imaginary part
  auto sites = [&](auto U0, auto U1, auto body) {
    sfor<decltype(U0)::value, decltype(U1)::value>([&](auto u) {
      constexpr int I = plan.uI[WC][u], J = plan.uJ[WC][u], IM = plan.uIm[WC][u];
      // the real and imaginary units of one tile pair, held by this wave one
      // after the other: written together, one 8-byte (re, im) per baseline
      constexpr bool PAIR = !IM && u + 1 < NU && plan.uI[WC][u + 1 < NU ? u + 1 : u] == I &&
                            plan.uJ[WC][u + 1 < NU ? u + 1 : u] == J && plan.uIm[WC][u + 1 < NU ? u + 1 : u];
      constexpr bool DONE = IM && u > 0 && plan.uI[WC][u > 0 ? u - 1 : 0] == I &&
                            plan.uJ[WC][u > 0 ? u - 1 : 0] == J && !plan.uIm[WC][u > 0 ? u - 1 : 0];
      if constexpr (!DONE) {
        const int j = 32 * J + n;
        const int32_t bias = (IM || PAIR) ? dcol[j] : 0;
        sfor<0, 16>([&](auto v) {
          const int i = 32 * I + 8 * (v / 4) + mb + (v % 4);
          if ((N % 32 == 0 || i < N) && (J < I || j <= i))
            body(u, v, std::integral_constant<bool, PAIR>{}, std::integral_constant<int, IM>{},
                 accf + (i * (i + 1) / 2 + j) * 2, bias);
        });
      }
    });
  };
  // this site's (re, im) or single value, with the imaginary bias removed
  auto value = [&](auto u, auto v, auto pair, int32_t bias) {
    int x;
    asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(x) : "a"(acc[u][(int)v]));
    if constexpr (pair.value) {
      constexpr int u1 = u + 1 < NU ? u + 1 : u;
      int y;
      asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(y) : "a"(acc[u1][(int)v]));
      return v2i{x >> 8, (y - bias) >> 8};
    } else {
      return v2i{(x - bias) >> 8, 0};
    }
  };
  using I0 = std::integral_constant<int, 0>;
  using IN = std::integral_constant<int, NU>;
  if constexpr (MODE == EPI_ADD) {
    // Read-modify-write.  A wave's sites are distinct baselines, so the prior
    // values of a chunk of units are all loaded before any of the chunk's
    // sums is stored: one memory round trip per chunk instead of one per
    // site (the compiler cannot prove the sites distinct and would otherwise
    // wait for each load in turn).
    constexpr int CH = 1;
    sfor<0, (NU + CH - 1) / CH>([&](auto c) {
      constexpr int u0 = decltype(c)::value * CH, u1 = u0 + CH < NU ? u0 + CH : NU;
      using U0 = std::integral_constant<int, u0>;
      using U1 = std::integral_constant<int, u1>;
      v2i prev[CH][16];
      sites(U0{}, U1{}, [&](auto u, auto v, auto pair, auto im, int32_t* dst, int) {
        if constexpr (pair.value)
          prev[u - u0][v] = *reinterpret_cast<const v2i*>(dst);
        else
          prev[u - u0][v][0] = dst[im.value];
      });
      sites(U0{}, U1{}, [&](auto u, auto v, auto pair, auto im, int32_t* dst, int32_t bias) {
        const v2i r = value(u, v, pair, bias);
        if constexpr (pair.value)
          *reinterpret_cast<v2i*>(dst) = prev[u - u0][v] + r;
        else
          dst[im.value] = prev[u - u0][v][0] + r[0];
      });
    });
  } else {
    sites(I0{}, IN{}, [&](auto u, auto v, auto pair, auto im, int32_t* dst, int32_t bias) {
      const v2i r = value(u, v, pair, bias);
      if constexpr (pair.value) {
        if constexpr (MODE == EPI_ATOMIC) {
          atomicAdd(dst, r[0]);
          atomicAdd(dst + 1, r[1]);
        } else {
          *reinterpret_cast<v2i*>(dst) = r;
        }
      } else if constexpr (MODE == EPI_ATOMIC) {
        atomicAdd(dst + im.value, r[0]);
      } else {
        dst[im.value] = r[0];
      }
    });
  }
}

// One work item: channel group `group` (channels CPW*group ..) over time
// chunk `tchunk` (samples tchunk*t_chunk ..) of the call described by a.
// tid is threadIdx.x (passed in so that a persistent caller can keep the
// per-lane set-up from being hoisted out of its item loop).
template <int N, int CPW, int S, int WC>
__device__ __forceinline__ void wave_main(const Args& a, uint8_t* lds, int group, int tchunk, int tid) {
  using C = Shape<N, CPW, S>;
  constexpr int NT = C::NT, W = C::W;
  constexpr UnitPlan<NT, W> plan{};
  constexpr int NU = plan.nu[WC];

  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c = wave / W;
  const int f0 = group * CPW;
  const int64_t t_begin = (int64_t)tchunk * a.t_chunk;
  const int64_t t_end = min(a.T, t_begin + a.t_chunk);
  if (t_end <= t_begin) return;  // uniform over the workgroup
  const int nt = (int)(t_end - t_begin);
  const int nstages = (nt + STAGE_T - 1) / STAGE_T;
  const int64_t row_stride = (int64_t)a.F * N;
  const int nch_valid = min(CPW, a.F - f0);  // the last group may be short of channels

  // ---- producer: wave-wide loads q = wave, wave + WAVES, ... of every stage.
  // Each lane keeps the source address of its 16 bytes in stage 0 (time row
  // src_t of the stage); stage st moves it by min(64 st, nt - 1 - src_t) rows,
  // which clamps the rows past the end of the range to the last valid row
  // (zeroed later by the reader) with one min and one multiply-add per load.
  const int my_loads = (C::LOADS - wave + C::WAVES - 1) / C::WAVES;
  // with one channel per workgroup the wave index is WC and known here
  const bool extra_load = CPW == 1 ? (WC + C::LPW_MIN * C::WAVES < C::LOADS)
                                   : (wave + C::LPW_MIN * C::WAVES < C::LOADS);
  const uint8_t* src[C::LPW_MAX];
  int src_last[C::LPW_MAX];  // nt - 1 - src_t: the largest row offset this lane may take
#pragma unroll
  for (int k = 0; k < C::LPW_MAX; ++k) {
    const int q = wave + k * C::WAVES;
    const int slot = (q < C::LOADS ? q : 0) * 64 + lane;  // 16-byte LDS slot this lane fills
    const int t = slot / C::RPP;                          // time row
    int p = slot % C::RPP;                                // chunk within the row
    if (p >= C::RPC) p = 0;                               // pitch padding: duplicate chunk 0
    int ch = p / (N / 16);
    const int kc = p % (N / 16);
    if (ch >= nch_valid) ch = nch_valid - 1;              // channels past F: dropped later
    src_last[k] = nt - 1 - t;
    src[k] = a.v + (t_begin + t) * row_stride + (int64_t)(f0 + ch) * N + 16 * kc;
  }
  const uint32_t ring_base = __builtin_amdgcn_readfirstlane(lds_addr(lds));
  // Addresses of the loads of stage st (computed ahead of their issue).
  const int rs32 = (int)row_stride;  // F N < 2^31 (checked by the host)
  auto stage_src = [&](int st, const uint8_t* (&g)[C::LPW_MAX]) {
#pragma unroll
    for (int k = 0; k < C::LPW_MAX; ++k)
      g[k] = src[k] + (int64_t)min(st * STAGE_T, src_last[k]) * (int64_t)rs32;
  };
  auto issue_loads = [&](int st, const uint8_t* const (&g)[C::LPW_MAX]) {
    const uint32_t base = ring_base + (uint32_t)((st % S) * C::STAGE_BYTES);
#pragma unroll
    for (int k = 0; k < C::LPW_MAX; ++k)
      if (k < C::LPW_MIN || extra_load) lds_dma16(g[k], base + (wave + k * C::WAVES) * 1024);
  };
  auto issue_stage = [&](int st) {
    const uint8_t* g[C::LPW_MAX];
    stage_src(st, g);
    issue_loads(st, g);
  };

  // ---- consumer
  v16i acc[NU];
  sfor<0, NU>([&](auto u) { acc[u] = v16i{}; });
  const int G = lane >> 4;
  // per-lane part of the transposed-read address within a stage
  const int lane_off = (8 * (lane >> 5) + ((lane & 15) >> 1)) * C::RPP * 16 + 16 * (G & 1) + 8 * (lane & 1);
  // lanes reading the empty upper half of a last, half-filled tile: they read
  // the lower half instead (always inside the row) and zero the result
  const bool upper_pad = (N % 32 == 16) && (G & 1);
  const int pad_back = upper_pad ? 16 : 0;

#pragma unroll
  for (int st = 0; st < S - 1; ++st)
    if (st < nstages) issue_stage(st);

  // Wait for stage st (all waves' loads), then refill the slot of stage
  // st-1, which every wave has finished reading: fragments are read one
  // K-step ahead, so by this barrier the reads of stage st-1 are all done.
  // In a last, partial stage the rows past the end hold duplicates of the
  // last valid row; they are zeroed here so the readers need no masks.
  auto enter_stage = [&](int st) {
    // S-2 later stages are in flight in steady state; near the end wait for all
    if (st + S - 2 < nstages) {
      if (my_loads == C::LPW_MAX)
        wait_vmcnt<(S - 2) * C::LPW_MAX>();
      else
        wait_vmcnt<(S - 2) * C::LPW_MIN>();
    } else {
      wait_vmcnt<0>();
    }
    __syncthreads();
    const int valid_t = nt - st * STAGE_T;
    if (valid_t < STAGE_T) {
      uint8_t* slot = lds + (st % S) * C::STAGE_BYTES;
      for (int i = valid_t * C::RPP + tid; i < STAGE_T * C::RPP; i += C::THREADS)
        *reinterpret_cast<v4i*>(slot + 16 * i) = v4i{0, 0, 0, 0};
      __syncthreads();
    }
  };

  // Transposed reads of the raw bytes of K-step ks of stage st (tile X, K-half h).
  auto read_step = [&](int st, int ks, v2i (&raw)[NT][2]) {
    const uint8_t* stage = lds + (st % S) * C::STAGE_BYTES + lane_off;
    sfor<0, NT>([&](auto X) {
      if constexpr (plan.needP[WC][X]) {
        sfor<0, 2>([&](auto h) {
          const uint8_t* p = stage + ((ks * 32 + 16 * h) * C::RPP + c * (N / 16) + 2 * X) * 16 -
                             (X == NT - 1 ? pad_back : 0);
          raw[X][h] = __builtin_amdgcn_ds_read_tr8_b64_v2i32((__attribute__((address_space(3))) v2i*)p);
        });
      }
    });
  };
  // Three-deep software pipeline over K-steps k (two per stage).  Block k
  // issues the transposed reads of step k+2, unpacks step k+1 (read one
  // block earlier, so already in registers) and runs step k's MFMAs; the
  // three parts are independent and the scheduling groups interleave the
  // unpack VALU with the MFMAs.  A block runs as two halves (K-half h = 0,
  // then 1: its unpack and its MFMAs); the ring loads of a later stage are
  // issued between the halves of one block of the stage, with their
  // addresses computed in the first half, so that their issue overlaps
  // running MFMAs instead of the stage barrier.  The stage entry (waits,
  // barrier) sits between blocks and the last stage is peeled off.  Samples
  // past the end of the range are zero (enter_stage), so whole K-steps are
  // run.
  static_assert(STAGE_T == 64, "two K-steps per stage");
  constexpr int NTILE = [] {
    int n = 0;
    for (int x = 0; x < NT; ++x) n += plan.needP[WC][x] ? 1 : 0;
    return n;
  }();
  constexpr int NREAD = 2 * NTILE;
  constexpr int NQ = [] {
    int n = 0;
    for (int x = 0; x < NT; ++x) n += plan.needQ[WC][x] ? 1 : 0;
    return n;
  }();
  // VALU slots per MFMA in a half block: 6 (+2) unpack operations per tile,
  // and the load addresses
  constexpr int VPH = (3 * NREAD + 2 * NQ + 2 * C::LPW_MAX + NU - 1) / NU + 1;
  // scheduling groups of one half block: (the reads,) then MFMA / VALU pairs
  auto interleave_half = [&](auto with_reads) {
    if constexpr (with_reads.value) __builtin_amdgcn_sched_group_barrier(0x100, NREAD, 0);
    sfor<0, NU>([&](auto) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x002, VPH, 0);
    });
  };
  // Unpack the raw bytes of K-half h into MFMA operands, x16 scaled: six
  // registers [re16 | im16 | ~re16] per tile, so that P = elements 0..3 and
  // Q = elements 2..5 are both register windows of one tuple (no copies);
  // tiles that are never the row of an imaginary product skip ~re16.
  auto unpack_h = [&](auto h, const v2i (&raw)[NT][2], v6i (&P)[NT][2]) {
    sfor<0, NT>([&](auto X) {
      if constexpr (plan.needP[WC][X]) {
        uint32_t w0 = (uint32_t)raw[X][h][0], w1 = (uint32_t)raw[X][h][1];
        if constexpr (N % 32 == 16 && X == NT - 1) {
          if (upper_pad) w0 = w1 = 0u;
        }
        const int r0 = (int)(w0 & 0xF0F0F0F0u), r1 = (int)(w1 & 0xF0F0F0F0u);
        const v4i p = v4i{r0, r1, (int)((w0 << 4) & 0xF0F0F0F0u), (int)((w1 << 4) & 0xF0F0F0F0u)};
        if constexpr (plan.needQ[WC][X])
          P[X][h] = __builtin_shufflevector(p, v4i{~r0, ~r1, 0, 0}, 0, 1, 2, 3, 4, 5);
        else
          P[X][h] = __builtin_shufflevector(p, p, 0, 1, 2, 3, -1, -1);
      }
    });
  };
  auto mfma_h = [&](auto h, const v6i (&P)[NT][2]) {
    sfor<0, NU>([&](auto u) {
      constexpr int I = plan.uI[WC][u], J = plan.uJ[WC][u];
      const v4i b = __builtin_shufflevector(P[J][h], P[J][h], 0, 1, 2, 3);
      if constexpr (plan.uIm[WC][u]) {
        acc[u] = mfma32(__builtin_shufflevector(P[I][h], P[I][h], 2, 3, 4, 5), b, acc[u]);
      } else {
        acc[u] = mfma32(__builtin_shufflevector(P[I][h], P[I][h], 0, 1, 2, 3), b, acc[u]);
      }
    });
  };
  // One block: reads of (st_rd, ks_rd), unpack of raw_up into P_up, MFMAs on
  // P_mm; with `loads` the loads of stage load_st go out mid-block.
  auto block = [&](auto loads, int st_rd, int ks_rd, v2i (&raw_rd)[NT][2], const v2i (&raw_up)[NT][2],
                   v6i (&P_up)[NT][2], const v6i (&P_mm)[NT][2], int load_st) {
    read_step(st_rd, ks_rd, raw_rd);
    const uint8_t* g[C::LPW_MAX];
    if constexpr (loads.value) stage_src(load_st, g);
    unpack_h(std::integral_constant<int, 0>{}, raw_up, P_up);
    mfma_h(std::integral_constant<int, 0>{}, P_mm);
    interleave_half(std::true_type{});
    if constexpr (loads.value) {
      __builtin_amdgcn_sched_barrier(0);
      issue_loads(load_st, g);
      __builtin_amdgcn_sched_barrier(0);
    }
    unpack_h(std::integral_constant<int, 1>{}, raw_up, P_up);
    mfma_h(std::integral_constant<int, 1>{}, P_mm);
    interleave_half(std::false_type{});
  };
  v6i P0[NT][2], P1[NT][2];
  v2i rawE[NT][2], rawO[NT][2];  // raw bytes of the even / odd K-step of a stage
  enter_stage(0);
  if (S - 1 < nstages) issue_stage(S - 1);
  read_step(0, 0, rawE);
  read_step(0, 1, rawO);
  unpack_h(std::integral_constant<int, 0>{}, rawE, P0);
  unpack_h(std::integral_constant<int, 1>{}, rawE, P0);
  int st = 0;
  for (; st + S < nstages; ++st) {  // stage st + S is still to be loaded
    enter_stage(st + 1);
    block(std::true_type{}, st + 1, 0, rawE, rawO, P1, P0, st + S);  // the loads go out here
    block(std::false_type{}, st + 1, 1, rawO, rawE, P0, P1, st + S);
  }
  for (; st + 1 < nstages; ++st) {
    enter_stage(st + 1);
    block(std::false_type{}, st + 1, 0, rawE, rawO, P1, P0, 0);
    block(std::false_type{}, st + 1, 1, rawO, rawE, P0, P1, 0);
  }
  unpack_h(std::integral_constant<int, 0>{}, rawO, P1);
  mfma_h(std::integral_constant<int, 0>{}, P0);
  interleave_half(std::false_type{});
  unpack_h(std::integral_constant<int, 1>{}, rawO, P1);
  mfma_h(std::integral_constant<int, 1>{}, P0);
  interleave_half(std::false_type{});
  mfma_h(std::integral_constant<int, 0>{}, P1);
  mfma_h(std::integral_constant<int, 1>{}, P1);
  mfma_drain();

  // ---- epilogue: publish each column's Im' diagonal through LDS, then add
  __syncthreads();  // the ring is no longer read
  int32_t* diag = reinterpret_cast<int32_t*>(lds);  // [CPW][NT * 32]
  sfor<0, NU>([&](auto u) {
    constexpr int I = plan.uI[WC][u], J = plan.uJ[WC][u];
    if constexpr (plan.uIm[WC][u] && I == J) {
      // diagonal element (n, n) sits in the lanes with l/32 == (n%8)/4, register
      // v = 4(n/8) + n%4
      const int n = lane & 31;
      if ((lane >> 5) == ((n & 7) >> 2)) {
        sfor<0, 16>([&](auto v) {
          if (v == 4 * (n >> 3) + (n & 3)) {
            int d;
            asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(d) : "a"(acc[u][(int)v]));
            diag[c * NT * 32 + 32 * I + n] = d;
          }
        });
      }
    }
  });
  __syncthreads();
  const int f = f0 + c;
  if (f >= a.F) return;
  const int32_t* dcol = diag + c * NT * 32;
  if (a.mode == EPI_ATOMIC)
    x32::epilogue<N, W, WC, EPI_ATOMIC>(a, f, lane, acc, dcol);
  else if (a.mode == EPI_ADD)
    x32::epilogue<N, W, WC, EPI_ADD>(a, f, lane, acc, dcol);
  else
    x32::epilogue<N, W, WC, EPI_STORE>(a, f, lane, acc, dcol);
}

template <int N, int CPW, int S, int WC>
__device__ __forceinline__ void dispatch(int wc, const Args& a, uint8_t* lds, int group, int tchunk,
                                         int tid) {
  if constexpr (WC < Shape<N, CPW, S>::W) {
    if (wc == WC)
      x32::wave_main<N, CPW, S, WC>(a, lds, group, tchunk, tid);
    else
      x32::dispatch<N, CPW, S, WC + 1>(wc, a, lds, group, tchunk, tid);
  }
}

// One work item of an N-input array with the launch shape built for N.
template <int N>
__device__ __forceinline__ void run_item(const Args& a, uint8_t* lds, int group, int tchunk, int tid) {
  constexpr int CPW = cpw_for(N), S = stages_for(N);
  const int wc = __builtin_amdgcn_readfirstlane(tid >> 6) % Shape<N, CPW, S>::W;
  x32::dispatch<N, CPW, S, 0>(wc, a, lds, group, tchunk, tid);
}

template <int N, int CPW, int S>
__global__ __launch_bounds__((Shape<N, CPW, S>::THREADS))
__attribute__((amdgpu_waves_per_eu(Shape<N, CPW, S>::WAVES / 4))) void kernel(Args a) {
  __shared__ __attribute__((aligned(1024))) uint8_t lds[Shape<N, CPW, S>::LDS_BYTES];
  const int wc = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) % Shape<N, CPW, S>::W;
  x32::dispatch<N, CPW, S, 0>(wc, a, lds, xcd_group(blockIdx.x, gridDim.x), blockIdx.y, threadIdx.x);
}

}  // namespace x32
}  // namespace xeng
