// xcorr16.hpp - gfx950 X-engine kernel on 16-row tiles (v_mfma_i32_16x16x64_i8),
// N a multiple of 16 up to 256.
//
// Result (paper Sec. 2 and Sec. 2.2): for each channel f of the grid and each
// pair 0 <= j <= i < N, the exact int32 sum over the launch's time range of
// x_i(t,f) conj(x_j(t,f)), added into acc[f][i(i+1)/2 + j].
//
// 1. HBM -> LDS ring.  Raw packed bytes go straight into an LDS ring of S
//    stages of 64 time samples with buffer loads into LDS (no registers).  A
//    stage's time row t holds the CPW*N bytes of the workgroup's channels in
//    16-byte chunks at an odd pitch of RPP chunks.  Each lane keeps a 32-bit
//    offset per load; the stage's base address and its valid byte count sit
//    in a buffer resource built per stage in scalar registers, so rows past
//    the end of the time range read as zero without touching memory and the
//    loads need no per-lane address arithmetic (64 F N < 2^32, checked by
//    the host).  With one channel per workgroup only the two waves with the
//    least unpack work issue loads (3% faster at N=192 than all four).
//
// 2. Fragments.  ds_read_b64_tr_b8 transposes, in every 16-lane group, the
//    8 x 16 byte block of the group's 8-byte reads.  Lane l reads time row
//    32k + 8(l/16) + (l%16)/2, bytes 16X + 8(l%2) of its channel, and receives
//    input 16X + l%16 at the 8 times 32k + 8(l/16) .. +7: the operand of
//    v_mfma_i32_16x16x64_i8 for tile X (row l%16, K group l/16) at the
//    32-sample step k.
//
// 3. Unpack, scaled by 16 (no sign extension), as in the 32-row kernel:
//        re16 = w & 0xF0F0F0F0,   im16 = (w << 4) & 0xF0F0F0F0
//    P = [re16 | im16] and Q = [im16 | ~re16] (~x = -x-1) are the two 4-register
//    windows of one 6-register tuple [re16 | im16 | ~re16].  Summed over time
//        P_i . P_j = 256 Re_ij
//        Q_i . P_j = 256 Im_ij - 16 S_j      (row form)
//        P_i . Q_j = -256 Im_ij - 16 S_i     (column form)
//    with S_n = sum_t im_n.  Both forms give -16 S_n at i = j = n (Im_nn = 0),
//    so with D_n the diagonal value the epilogue forms
//        Re = P.P >> 8,  Im = (Q.P - D_j) >> 8  or  (D_i - P.Q) >> 8,
//    exactly.  |sums| <= 32896 per sample: a workgroup integrates at most
//    MAX_T_PER_WG = 32768 samples (the host splits longer ranges).
//
// 4. Work split (Plan16).  A unit is the real or the imaginary product of
//    one 16 x 16 tile pair (I, J), J <= I: 4 accumulator registers.  With
//    h = NT/2 the units are ordered: the upper-left triangle (tiles < h) row
//    by row, the rectangle of rows >= h and columns < h column by column from
//    the last column, then the lower-right triangle row by row, and cut into
//    W contiguous runs, one per wave.  Each run then touches few tiles (N=192:
//    6, 9, 9 and 6 of the 12, 39 units each), and the unpack work per wave
//    is per tile touched.  Each wave puts its imaginary products in the row
//    or the column form, whichever needs the negated copy of fewer tiles.
//    Compared with 32-row tiles, 16-row tiles halve the work wasted above the
//    diagonal, and the 16x16x64 product keeps the shader clock higher under
//    a full load of the matrix cores.
#pragma once
#include <type_traits>

#include "xcorr.hpp"

namespace xeng {
namespace x16 {

constexpr int MAX_T_PER_WG = 32768;   // int32 headroom of the x256 sums
constexpr int KPS_DEFAULT = 2;        // 32-sample steps per ring stage (64 samples)
constexpr int TILE_ROWS = 16;
// A stage's per-lane offsets and its buffer-resource byte count are 32-bit:
// the kernel needs 32 KPS F N < 2^32 bytes.
constexpr int64_t MAX_ROW_BYTES = ((int64_t)1 << 32) / (32 * KPS_DEFAULT) - 1;
constexpr int MAX_UNITS_PER_WAVE = 60;

template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    sfor<B + 1, E>(f);
  }
}

constexpr int tiles(int n) { return n / 16; }
constexpr int units(int nt) { return nt * (nt + 1); }
// Waves per channel: 1 up to 60 units, else 2 up to 120, else 4; N = 128 (72
// units) takes 4 waves of 18, one channel per workgroup (0.259 against 0.285
// ms at F = 1024, T = 8192 with two waves of 36; N = 144 and 160 measured
// the same either way).
constexpr int waves_per_channel(int nt) {
  return units(nt) <= MAX_UNITS_PER_WAVE ? 1 : nt == 8 ? 4 : units(nt) <= 2 * MAX_UNITS_PER_WAVE ? 2 : 4;
}
// With four waves per channel a wave may hold up to 68 units (N = 256: 272
// accumulator registers, the 256 AGPRs and 16 VGPRs of its 512 at one wave
// per SIMD); the choice of 1, 2 or 4 waves per channel keeps the 60 limit.
constexpr int MAX_UNITS_PER_WAVE_4 = 68;
constexpr bool supported(int n) { return n % 16 == 0 && n >= 16 && units(tiles(n)) <= 4 * MAX_UNITS_PER_WAVE_4; }

template <int NT, int W>
struct Plan16 {
  static constexpr int U = units(NT);
  static constexpr int MAXU = (U + W - 1) / W;
  int nu[W];
  int uI[W][MAXU];
  int uJ[W][MAXU];
  int uIm[W][MAXU];
  bool qcol[W];        // imaginary products of wave w in the column form P_I . Q_J
  bool needP[W][NT];   // tile read as an operand
  bool needQ[W][NT];   // tile whose negated copy ~re16 is used
  int ntile[W];        // tiles wave w unpacks per step
  int lrank[W];        // with four waves per channel: rank among the two loader waves, or -1
  constexpr Plan16() : nu(), uI(), uJ(), uIm(), qcol(), needP(), needQ(), ntile(), lrank() {
    int oI[U] = {}, oJ[U] = {}, oM[U] = {};
    int n = 0;
    const int h = NT / 2;
    auto put = [&](int I, int J) {
      oI[n] = I, oJ[n] = J, oM[n] = 0, ++n;
      oI[n] = I, oJ[n] = J, oM[n] = 1, ++n;
    };
    for (int I = 0; I < h; ++I)
      for (int J = 0; J <= I; ++J) put(I, J);
    for (int J = h - 1; J >= 0; --J)
      for (int I = h; I < NT; ++I) put(I, J);
    for (int I = h; I < NT; ++I)
      for (int J = h; J <= I; ++J) put(I, J);
    const int q = U / W, rem = U % W;
    int k = 0;
    for (int w = 0; w < W; ++w) {
      nu[w] = q + (w < rem ? 1 : 0);
      bool rowt[NT] = {}, colt[NT] = {};
      int nrow = 0, ncol = 0;
      for (int u = 0; u < nu[w]; ++u, ++k) {
        uI[w][u] = oI[k];
        uJ[w][u] = oJ[k];
        uIm[w][u] = oM[k];
        needP[w][oI[k]] = needP[w][oJ[k]] = true;
        if (oM[k]) {
          if (!rowt[oI[k]]) rowt[oI[k]] = true, ++nrow;
          if (!colt[oJ[k]]) colt[oJ[k]] = true, ++ncol;
        }
      }
      qcol[w] = ncol < nrow;
      for (int x = 0; x < NT; ++x) needQ[w][x] = qcol[w] ? colt[x] : rowt[x];
      for (int x = 0; x < NT; ++x) ntile[w] += needP[w][x] ? 1 : 0;
    }
    // The two waves that unpack the fewest tiles issue the ring loads (their
    // MFMA count is the same, their VALU work the smallest).
    for (int w = 0; w < W; ++w) lrank[w] = -1;
    if (W == 4) {
      for (int r = 0; r < 2; ++r) {
        int best = -1;
        for (int w = 0; w < W; ++w)
          if (lrank[w] < 0 && (best < 0 || ntile[w] < ntile[best])) best = w;
        lrank[best] = r;
      }
    }
  }
};

template <int N, int CPW, int S, int KPS>
struct Shape {
  static constexpr int STAGE_T = 32 * KPS;            // time samples per ring stage (KPS 32-sample steps)
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
  static constexpr int DIAG_BYTES = CPW * N * 4;
  static constexpr int LDS_BYTES = S * STAGE_BYTES > DIAG_BYTES ? S * STAGE_BYTES : DIAG_BYTES;
  static_assert(supported(N), "N must be a multiple of 16 up to 256");
  static_assert(LOADS * 1024 == STAGE_BYTES, "a stage is whole 1 KB loads");
  static_assert(S >= 3 && (S - 2) * (CPW == 1 ? (LOADS + 1) / 2 : LPW_MAX) < 64, "ring depth");
  static_assert(KPS >= 2 && KPS % 2 == 0, "an even number of steps per stage");
  static_assert(WAVES == 4, "four waves per workgroup");
};

// Launch shape per N: W waves per channel, 4/W channels per workgroup,
// stages of KPS steps, and as many ring stages as fit 128 KB (3 to 8).
constexpr int cpw_for(int n) { return 4 / waves_per_channel(tiles(n)); }
constexpr int stages_for(int n, int kps) {
  const int stage = 32 * kps * ((cpw_for(n) * n / 16) | 1) * 16;
  const int s = (128 * 1024) / stage;
  return s < 3 ? 3 : (s > 8 ? 8 : s);
}

template <int n>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(n >= 0 && n < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((n & 0xF) | ((n >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// One wave-wide 1 KB buffer load into LDS: lane i copies the 16 bytes at
// rsrc.base + voff to LDS byte address lds_base + 16 i; offsets at or past
// rsrc.num_records read as zero without touching memory.  Written as asm so
// the compiler does not make every later LDS read wait for all loads in
// flight (the ring waits for each stage with s_waitcnt vmcnt + barrier).
// No register is written; M0 is otherwise unused by this code.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__device__ __forceinline__ void buf_dma16(v4i rsrc, uint32_t voff, uint32_t lds_base) {
  asm volatile(
      "s_mov_b32 m0, %2\n\t"
      "buffer_load_dwordx4 %0, %1, 0 offen lds"
      :
      : "v"(voff), "s"(rsrc), "s"(lds_base)
      : "memory", "m0");
}
#pragma clang diagnostic pop

__device__ __forceinline__ uint32_t lds_addr(const void* p) {
  return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void*)p;
}

__device__ __forceinline__ v4i mfma16(v4i a, v4i b, v4i c) {
  return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
}

// Sum v (0..3) of unit tile t (inline asm, so the epilogue's wait states
// before it are explicit: mfma_drain).
__device__ __forceinline__ int32_t acc_read(const v4i& t, int v) {
  int x;
  asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(x) : "a"(t[v]));
  return x;
}

// Add one wave's tiles into the accumulator of channel f.  16x16 result
// layout: lane l, register v hold row 4(l/16) + v, column l%16; the 16 lanes
// of a group write 16 consecutive baselines of one row.  drow: the diagonal
// values D_n of this channel (LDS).
template <int N, int W, int WC, int MODE, int NU>
__device__ __forceinline__ void epilogue(const Args& a, int f, int lane, const v4i (&acc)[NU],
                                         const int32_t* drow) {
  constexpr int NT = tiles(N);
  constexpr Plan16<NT, W> plan{};
  constexpr bool QC = plan.qcol[WC];
  constexpr int nbl = N * (N + 1) / 2;
  int32_t* accf = a.acc + (int64_t)f * nbl * 2;
  const int n = lane & 15;
  const int mb = 4 * (lane >> 4);
  if constexpr (MODE == EPI_ADD) {
    // Read-modify-write.  A wave's sites are distinct baselines, so the prior
    // values of a chunk of units are all loaded before any of the chunk's
    // sums is stored: one memory round trip per chunk instead of one per
    // site (the compiler cannot prove the sites distinct, and otherwise waits
    // for each load in turn; N=192: 0.51 against 0.58 ms per launch).
    constexpr int CH = 16;
    sfor<0, (NU + CH - 1) / CH>([&](auto c) {
      constexpr int u0 = decltype(c)::value * CH, u1 = u0 + CH < NU ? u0 + CH : NU;
      v2i prev[CH][4];
      // calls body(pair, im, dst, j, un) for site (u, v) when this lane holds one
      auto site = [&](auto u, auto v, auto body) {
        constexpr int I = plan.uI[WC][u], J = plan.uJ[WC][u], IM = plan.uIm[WC][u];
        constexpr int un = u + 1 < NU ? u + 1 : u, up = u > 0 ? u - 1 : 0;
        constexpr bool PAIR = !IM && u + 1 < NU && plan.uI[WC][un] == I && plan.uJ[WC][un] == J &&
                              plan.uIm[WC][un];
        constexpr bool DONE = IM && u > 0 && plan.uI[WC][up] == I && plan.uJ[WC][up] == J && !plan.uIm[WC][up];
        if constexpr (!DONE) {
          const int j = 16 * J + n;
          const int i = 16 * I + mb + v;
          if (J < I || j <= i)
            body(std::integral_constant<bool, PAIR>{}, std::integral_constant<int, IM>{},
                 accf + (i * (i + 1) / 2 + j) * 2, j, un);
        }
      };
      sfor<u0, u1>([&](auto u) {
        sfor<0, 4>([&](auto v) {
          site(u, v, [&](auto pair, auto im, int32_t* dst, int, int) {
            if constexpr (pair.value)
              prev[u - u0][v] = *reinterpret_cast<const v2i*>(dst);
            else
              prev[u - u0][v][0] = dst[im.value];
          });
        });
      });
      sfor<u0, u1>([&](auto u) {
        constexpr int I = plan.uI[WC][u];
        sfor<0, 4>([&](auto v) {
          site(u, v, [&](auto pair, auto im, int32_t* dst, int j, int un) {
            auto im_of = [&](int32_t x) {
              if constexpr (QC)
                return (drow[16 * I + mb + (int)v] - x) >> 8;
              else
                return (x - drow[j]) >> 8;
            };
            const int32_t x = acc_read(acc[u], v);
            if constexpr (pair.value) {
              const int32_t y = acc_read(acc[un], v);
              *reinterpret_cast<v2i*>(dst) = prev[u - u0][v] + v2i{x >> 8, im_of(y)};
            } else {
              dst[im.value] = prev[u - u0][v][0] + (im.value ? im_of(x) : x >> 8);
            }
          });
        });
      });
    });
    return;
  }
  sfor<0, NU>([&](auto u) {
    constexpr int I = plan.uI[WC][u], J = plan.uJ[WC][u], IM = plan.uIm[WC][u];
    constexpr int un = u + 1 < NU ? u + 1 : u, up = u > 0 ? u - 1 : 0;
    // the real and imaginary units of one tile pair held by this wave one
    // after the other are written together, one 8-byte (re, im) per baseline
    constexpr bool PAIR = !IM && u + 1 < NU && plan.uI[WC][un] == I && plan.uJ[WC][un] == J &&
                          plan.uIm[WC][un];
    constexpr bool DONE = IM && u > 0 && plan.uI[WC][up] == I && plan.uJ[WC][up] == J && !plan.uIm[WC][up];
    if constexpr (!DONE) {
      const int j = 16 * J + n;
      int32_t dj = 0;
      v4i di = v4i{0, 0, 0, 0};
      if constexpr (IM || PAIR) {
        if constexpr (QC)
          di = *reinterpret_cast<const v4i*>(drow + 16 * I + mb);
        else
          dj = drow[j];
      }
      sfor<0, 4>([&](auto v) {
        const int i = 16 * I + mb + v;
        if (J < I || j <= i) {
          int32_t* dst = accf + (i * (i + 1) / 2 + j) * 2;
          auto im_of = [&](int32_t x) { return QC ? (di[(int)v] - x) >> 8 : (x - dj) >> 8; };
          const int32_t x = acc_read(acc[u], v);
          if constexpr (PAIR) {
            const int32_t y = acc_read(acc[un], v);
            const v2i re_im = v2i{x >> 8, im_of(y)};
            v2i* d2 = reinterpret_cast<v2i*>(dst);
            if constexpr (MODE == EPI_ATOMIC) {
              atomicAdd(dst, re_im[0]);
              atomicAdd(dst + 1, re_im[1]);
            } else {
              *d2 = re_im;
            }
          } else {
            const int32_t r = IM ? im_of(x) : x >> 8;
            if constexpr (MODE == EPI_ATOMIC)
              atomicAdd(dst + IM, r);
            else
              dst[IM] = r;
          }
        }
      });
    }
  });
}

// One work item: channel group `group` (channels CPW*group ..) over time
// chunk `tchunk` (samples tchunk*t_chunk ..) of the call described by a.
// tid is threadIdx.x (passed in so that a persistent caller can keep the
// per-lane set-up from being hoisted out of its item loop).
template <int N, int CPW, int S, int KPS, int WC>
__device__ __forceinline__ void wave_main(const Args& a, uint8_t* lds, int group, int tchunk, int tid) {
  using C = Shape<N, CPW, S, KPS>;
  constexpr int STAGE_T = C::STAGE_T;
  constexpr int NT = C::NT, W = C::W;
  constexpr Plan16<NT, W> plan{};
  constexpr int NU = plan.nu[WC];
  constexpr bool QC = plan.qcol[WC];

  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c = wave / W;
  const int f0 = group * CPW;
  const int64_t t_begin = (int64_t)tchunk * a.t_chunk;
  const int64_t t_end = min(a.T, t_begin + a.t_chunk);
  if (t_end <= t_begin) return;  // uniform over the workgroup
  const int nt = (int)(t_end - t_begin);
  const int nstages = (nt + STAGE_T - 1) / STAGE_T;
  const uint32_t rs32 = (uint32_t)((int64_t)a.F * N);  // one time row; 64 F N < 2^32
  const int nch_valid = min(CPW, a.F - f0);             // the last group may be short of channels

  // ---- producer: the wave-wide 1 KB loads q = 0 .. LOADS-1 of every stage.
  // With one channel per workgroup the two waves with the least unpack work
  // issue them all (q = rank, rank + 2, ...; compile-time counts); with
  // several channels per workgroup every wave issues q = wave, wave + 4, ...
  constexpr bool ONE = CPW == 1;
  constexpr int NLW = ONE ? 2 : C::WAVES;                 // loader waves
  constexpr int LR = ONE ? plan.lrank[WC] : 0;            // this wave's rank (one channel)
  constexpr int LW = ONE ? (LR < 0 ? 0 : (C::LOADS - LR + NLW - 1) / NLW) : 0;
  constexpr int LMAX = ONE ? (C::LOADS + NLW - 1) / NLW : C::LPW_MAX;
  const int rank = ONE ? LR : wave;
  const int my_loads = ONE ? LW : (C::LOADS - wave + C::WAVES - 1) / C::WAVES;
  uint32_t voff[LMAX];
#pragma unroll
  for (int k = 0; k < LMAX; ++k) {
    const int q = (rank < 0 ? 0 : rank) + k * NLW;
    const int slot = (q < C::LOADS ? q : 0) * 64 + lane;  // 16-byte LDS slot this lane fills
    const int t = slot / C::RPP;                          // time row
    int p = slot % C::RPP;                                // chunk within the row
    if (p >= C::RPC) p = 0;                               // pitch padding: duplicate chunk 0
    int ch = p / (N / 16);
    const int kc = p % (N / 16);
    if (ch >= nch_valid) ch = nch_valid - 1;              // channels past F: dropped later
    voff[k] = (uint32_t)t * rs32 + (uint32_t)((f0 + ch) * N + 16 * kc);
  }
  const uint32_t ring_base = __builtin_amdgcn_readfirstlane(lds_addr(lds));
  const uint64_t vbase = (uint64_t)(uintptr_t)a.v + (uint64_t)t_begin * rs32;
  // Stages past the last are issued too, with no valid bytes: every stage
  // then counts the same loads per wave (uniform vmcnt waits) and the loop
  // needs no tail.  Their zeros land in slots that are no longer read, and
  // the epilogue waits for them before it reuses LDS.
  auto issue_stage = [&](int st) {
    const uint64_t b = vbase + (uint64_t)(st * STAGE_T) * rs32;
    // rows of this stage inside the range, clamped to [0, STAGE_T] in scalar
    // registers (a clamp in C becomes a vector med3 and a readfirstlane)
    int rows;
    asm("s_max_i32 %0, %1, 0\n\ts_min_i32 %0, %0, %2"
        : "=s"(rows)
        : "s"(__builtin_amdgcn_readfirstlane(nt - st * STAGE_T)), "s"(STAGE_T));
    v4i rsrc;
    rsrc[0] = __builtin_amdgcn_readfirstlane((int)(uint32_t)b);
    rsrc[1] = __builtin_amdgcn_readfirstlane((int)((uint32_t)(b >> 32) & 0xFFFFu));
    rsrc[2] = __builtin_amdgcn_readfirstlane((int)((uint32_t)rows * rs32));
    rsrc[3] = 0x00020000;  // raw buffer, 32-bit data format
    const uint32_t base = ring_base + (uint32_t)((st % S) * C::STAGE_BYTES);
#pragma unroll
    for (int k = 0; k < LMAX; ++k) {
      if constexpr (ONE) {
        if (k < LW) buf_dma16(rsrc, voff[k], base + (LR + k * NLW) * 1024);
      } else if (k < my_loads) {
        buf_dma16(rsrc, voff[k], base + (wave + k * C::WAVES) * 1024);
      }
    }
  };

  // ---- consumer
  v4i acc[NU];
  sfor<0, NU>([&](auto u) { acc[u] = v4i{0, 0, 0, 0}; });
  // per-lane part of the transposed-read address within a stage
  const int lane_off = (8 * (lane >> 4) + ((lane & 15) >> 1)) * C::RPP * 16 + 8 * (lane & 1);

#pragma unroll
  for (int st = 0; st < S - 1; ++st) issue_stage(st);

  // Wait for stage st (all waves' loads), then the slot of stage st-1 may be
  // refilled: fragments are read one step ahead, and every wave's reads of
  // stage st-1 have completed by this barrier.  In a last, partial stage the
  // rows past the end are zeroed here so the readers need no masks.
  auto enter_stage = [&](int st) {
    // the S-2 stages after st stay in flight
    if constexpr (ONE)
      wait_vmcnt<(S - 2) * LW>();
    else if (my_loads == C::LPW_MAX)
      wait_vmcnt<(S - 2) * C::LPW_MAX>();
    else
      wait_vmcnt<(S - 2) * C::LPW_MIN>();
    __syncthreads();
    const int valid_t = nt - st * STAGE_T;
    if (valid_t < STAGE_T) {
      uint8_t* slot = lds + (st % S) * C::STAGE_BYTES;
      for (int i = valid_t * C::RPP + tid; i < STAGE_T * C::RPP; i += C::THREADS)
        *reinterpret_cast<v4i*>(slot + 16 * i) = v4i{0, 0, 0, 0};
      __syncthreads();
    }
  };

  // Transposed reads of the raw bytes of step ks (0 .. KPS-1) of stage st.
  auto read_step = [&](int st, int ks, v2i (&raw)[NT]) {
    const uint8_t* stage = lds + (st % S) * C::STAGE_BYTES + lane_off;
    sfor<0, NT>([&](auto X) {
      if constexpr (plan.needP[WC][X]) {
        const uint8_t* p = stage + ((ks * 32) * C::RPP + c * (N / 16) + X) * 16;
        raw[X] = __builtin_amdgcn_ds_read_tr8_b64_v2i32((__attribute__((address_space(3))) v2i*)p);
      }
    });
  };
  constexpr int NTILE = [] {
    int n = 0;
    for (int x = 0; x < NT; ++x) n += plan.needP[WC][x] ? 1 : 0;
    return n;
  }();
  constexpr int NQ = [] {
    int n = 0;
    for (int x = 0; x < NT; ++x) n += plan.needQ[WC][x] ? 1 : 0;
    return n;
  }();
  // Unpack raw bytes into MFMA operands, x16 scaled: six registers
  // [re16 | im16 | ~re16] per tile, so that P = elements 0..3 and Q =
  // elements 2..5 are both register windows of one tuple (no copies); tiles
  // whose negated copy is never used skip ~re16.
  auto unpack = [&](const v2i (&raw)[NT], v6i (&P)[NT], auto xlo, auto xhi) {
    sfor<decltype(xlo)::value, decltype(xhi)::value>([&](auto X) {
      if constexpr (plan.needP[WC][X]) {
        const uint32_t w0 = (uint32_t)raw[X][0], w1 = (uint32_t)raw[X][1];
        const int r0 = (int)(w0 & 0xF0F0F0F0u), r1 = (int)(w1 & 0xF0F0F0F0u);
        const v4i p = v4i{r0, r1, (int)((w0 << 4) & 0xF0F0F0F0u), (int)((w1 << 4) & 0xF0F0F0F0u)};
        if constexpr (plan.needQ[WC][X]) {
          P[X] = __builtin_shufflevector(p, v4i{~r0, ~r1, 0, 0}, 0, 1, 2, 3, 4, 5);
          // one definition of the whole tuple, so that the compiler keeps it
          // in six consecutive registers (both windows are then sub-tuples;
          // otherwise it splits the parts and copies im16 for every Q use)
          asm("" : "+v"(P[X]));
        } else {
          P[X] = __builtin_shufflevector(p, p, 0, 1, 2, 3, -1, -1);
        }
      }
    });
  };
  auto mfma_step = [&](const v6i (&P)[NT], auto lo, auto hi) {
    sfor<decltype(lo)::value, decltype(hi)::value>([&](auto u) {
      constexpr int I = plan.uI[WC][u], J = plan.uJ[WC][u];
      const v4i pi = __builtin_shufflevector(P[I], P[I], 0, 1, 2, 3);
      const v4i pj = __builtin_shufflevector(P[J], P[J], 0, 1, 2, 3);
      if constexpr (!plan.uIm[WC][u])
        acc[u] = mfma16(pi, pj, acc[u]);
      else if constexpr (QC)
        acc[u] = mfma16(pi, __builtin_shufflevector(P[J], P[J], 2, 3, 4, 5), acc[u]);
      else
        acc[u] = mfma16(__builtin_shufflevector(P[I], P[I], 2, 3, 4, 5), pj, acc[u]);
    });
  };
  // Scheduling groups of a block: MFMAs interleaved with the transposed
  // reads (first) and the unpack VALU.
  constexpr int NREAD = NTILE;
  constexpr int NVALU = 6 * NTILE + 2 * NQ;
  constexpr int UH = NU / 2;  // the ring loads go out after this many MFMAs
  auto interleave = [&](auto lo, auto hi, auto nv) {
    sfor<decltype(lo)::value, decltype(hi)::value>([&](auto u) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      if constexpr (u < NREAD) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x002, decltype(nv)::value, 0);
    });
  };
  constexpr int VPM = (NVALU + NU - 1) / NU;
  // the unpack of a block with loads is split at tile XM: half the tiles
  // before the loads, half after
  constexpr int XM = [] {
    int n = 0, x = 0;
    for (; x < NT && 2 * n < NTILE; ++x) n += plan.needP[WC][x] ? 1 : 0;
    return x;
  }();
  using I0 = std::integral_constant<int, 0>;
  using IH = std::integral_constant<int, UH>;
  using IN = std::integral_constant<int, NU>;
  using IV = std::integral_constant<int, VPM>;
  using X0 = std::integral_constant<int, 0>;
  using XH = std::integral_constant<int, XM>;
  using XN = std::integral_constant<int, NT>;
  // One block (one 32-sample step): the reads of step (st_rd, ks_rd), the
  // unpack of raw_up into P_up and the MFMAs on P_mm, interleaved; with
  // `loads` the ring loads of stage load_st go out after the first UH MFMAs.
  auto block = [&](auto loads, int st_rd, int ks_rd, v2i (&raw_rd)[NT], const v2i (&raw_up)[NT],
                   v6i (&P_up)[NT], const v6i (&P_mm)[NT], int load_st) {
    read_step(st_rd, ks_rd, raw_rd);
    if constexpr (loads.value) {
      unpack(raw_up, P_up, X0{}, XH{});
      mfma_step(P_mm, I0{}, IH{});
      interleave(I0{}, IH{}, IV{});
      __builtin_amdgcn_sched_barrier(0);
      issue_stage(load_st);
      __builtin_amdgcn_sched_barrier(0);
      unpack(raw_up, P_up, XH{}, XN{});
      mfma_step(P_mm, IH{}, IN{});
      interleave(IH{}, IN{}, IV{});
    } else {
      unpack(raw_up, P_up, X0{}, XN{});
      mfma_step(P_mm, I0{}, IN{});
      interleave(I0{}, IN{}, IV{});
    }
  };
  // Step k of the pipeline: reads of step k+2, unpack of step k+1, MFMAs of
  // step k; even steps use rawE / P0 for their data, odd steps rawO / P1.
  // The reads of stage st+1 start at step KPS-2 of stage st: the stage entry
  // (waits and barrier) comes right before it, and the slot of stage st,
  // whose reads are complete by that barrier, is refilled from the stage's
  // last block.
  v6i P0[NT], P1[NT];
  v2i rawE[NT], rawO[NT];  // raw bytes of the even / odd steps
  auto step = [&](auto ks, auto with_reads, int st) {
    constexpr int K = decltype(ks)::value;
    constexpr int KR = (K + 2) % KPS;          // step of the reads within its stage
    const int st_rd = st + (K + 2) / KPS;
    constexpr bool LOADS = K == KPS - 1;   // (measured: 0.6% faster than in the stage's first block)
    if constexpr (!with_reads.value) {
      if constexpr (K % 2 == 0) {
        unpack(rawO, P1, X0{}, XN{});
        mfma_step(P0, I0{}, IN{});
        interleave(I0{}, IN{}, IV{});
      } else {
        mfma_step(P1, I0{}, IN{});
      }
    } else if constexpr (K % 2 == 0) {
      block(std::integral_constant<bool, LOADS>{}, st_rd, KR, rawE, rawO, P1, P0, st + S);
    } else {
      block(std::integral_constant<bool, LOADS>{}, st_rd, KR, rawO, rawE, P0, P1, st + S);
    }
  };
  enter_stage(0);
  issue_stage(S - 1);
  read_step(0, 0, rawE);
  read_step(0, 1, rawO);
  unpack(rawE, P0, X0{}, XN{});
  for (int st = 0; st + 1 < nstages; ++st) {
    sfor<0, KPS>([&](auto ks) {
      if constexpr (decltype(ks)::value == KPS - 2) enter_stage(st + 1);
      step(ks, std::true_type{}, st);
    });
  }
  // the last stage: no reads of a further stage
  {
    const int st = nstages - 1;
    sfor<0, KPS - 2>([&](auto ks) { step(ks, std::true_type{}, st); });
    step(std::integral_constant<int, KPS - 2>{}, std::false_type{}, st);
    step(std::integral_constant<int, KPS - 1>{}, std::false_type{}, st);
  }
  mfma_drain();

  // ---- epilogue: publish each input's diagonal value D_n through LDS, then add.
  // The loads of the stages past the last (empty, but they still write zeros
  // into their ring slots) must have landed before LDS is reused: wait for
  // all of this wave's loads, then for every wave.
  wait_vmcnt<0>();
  __syncthreads();  // the ring is no longer read or written
  int32_t* diag = reinterpret_cast<int32_t*>(lds);  // [CPW][N]
  sfor<0, NU>([&](auto u) {
    constexpr int I = plan.uI[WC][u], J = plan.uJ[WC][u];
    if constexpr (plan.uIm[WC][u] && I == J) {
      // element (n, n) sits in lane 16(n/4) + n, register n%4
      const int n = lane & 15;
      if ((lane >> 4) == (n >> 2)) {
        sfor<0, 4>([&](auto v) {
          if (v == (n & 3)) diag[c * N + 16 * I + n] = acc_read(acc[u], v);
        });
      }
    }
  });
  __syncthreads();
  const int f = f0 + c;
  if (f >= a.F) return;
  const int32_t* drow = diag + c * N;
  if (a.mode == EPI_ATOMIC)
    x16::epilogue<N, W, WC, EPI_ATOMIC>(a, f, lane, acc, drow);
  else if (a.mode == EPI_ADD)
    x16::epilogue<N, W, WC, EPI_ADD>(a, f, lane, acc, drow);
  else
    x16::epilogue<N, W, WC, EPI_STORE>(a, f, lane, acc, drow);
}

template <int N, int CPW, int S, int KPS, int WC>
__device__ __forceinline__ void dispatch(int wc, const Args& a, uint8_t* lds, int group, int tchunk,
                                         int tid) {
  if constexpr (WC < Shape<N, CPW, S, KPS>::W) {
    if (wc == WC)
      x16::wave_main<N, CPW, S, KPS, WC>(a, lds, group, tchunk, tid);
    else
      x16::dispatch<N, CPW, S, KPS, WC + 1>(wc, a, lds, group, tchunk, tid);
  }
}

// One work item of an N-input array with the launch shape built for N.
template <int N, int KPS>
__device__ __forceinline__ void run_item(const Args& a, uint8_t* lds, int group, int tchunk, int tid) {
  constexpr int CPW = cpw_for(N), S = stages_for(N, KPS);
  const int wc = __builtin_amdgcn_readfirstlane(tid >> 6) % Shape<N, CPW, S, KPS>::W;
  x16::dispatch<N, CPW, S, KPS, 0>(wc, a, lds, group, tchunk, tid);
}

template <int N, int CPW, int S, int KPS>
__global__ __launch_bounds__((Shape<N, CPW, S, KPS>::THREADS))
__attribute__((amdgpu_waves_per_eu(1))) void kernel(Args a) {
  __shared__ __attribute__((aligned(1024))) uint8_t lds[Shape<N, CPW, S, KPS>::LDS_BYTES];
  const int wc = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) % Shape<N, CPW, S, KPS>::W;
  x16::dispatch<N, CPW, S, KPS, 0>(wc, a, lds, xcd_group(blockIdx.x, gridDim.x), blockIdx.y, threadIdx.x);
}

}  // namespace x16
}  // namespace xeng
