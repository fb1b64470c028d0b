// k_chan.hip - F-stage channeliser (paper Sec. 2.1, Eq. 1-2) and its C
// entry points (include/xeng.h).
//
// Per spectrum s and input pair (2q, 2q + 1):
//  1. polyphase FIR: v[n] = sum_{p<4} h[pL + n] x[sL + pL + n] for both
//     inputs (L = 2F real samples per spectrum, h the Hamming-windowed sinc
//     prototype), packed as y[n] = v_2q[n] + j v_2q+1[n] (Eq. 1);
//  2. Stockham FFT of y, L points, natural order out;
//  3. Eq. 2: X_2q[k] = (Y[k] + conj Y[-k]) / 2, X_2q+1[k] = (Y[k] -
//     conj Y[-k]) / 2j, k < F, written to out[s][k][2q .. 2q + 1] (the
//     [time, channel, input] order of the X side).
// Two kernels: for F = 256, 512, 1024 a register-resident one (radix-8
// passes, runs of spectra per workgroup, below); for other F one workgroup
// per (spectrum, pair) with the points in LDS (radix-4 passes and one
// radix-2 pass when log2 L is odd).  Float32 arithmetic; the tables (h and
// the twiddles e^{-2 pi i t / L}) are computed in double and rounded once.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "../../include/xeng.h"

namespace xeng {
namespace {

constexpr int TAPS = 4;
constexpr int THREADS = 256;
constexpr int MAX_L = 2048;

__global__ __launch_bounds__(THREADS) void chan_tables(float* tab, int L) {
  const int i = blockIdx.x * THREADS + threadIdx.x;
  const int PL = TAPS * L;
  if (i < PL) {
    const double w = 0.54 - 0.46 * cos(2.0 * M_PI * i / (PL - 1));
    const double xs = (i - PL / 2.0) / L;
    const double sinc = xs == 0.0 ? 1.0 : sinpi(xs) / (M_PI * xs);
    tab[i] = (float)(w * sinc);
  } else if (i < PL + L / 2) {
    const int t = i - PL;
    double sn, cs;
    sincospi(2.0 * t / L, &sn, &cs);
    tab[PL + 2 * t] = (float)cs;
    tab[PL + 2 * t + 1] = (float)(-sn);
  }
}

// G input pairs of one spectrum per workgroup.  G = 1 measured fastest (more
// workgroups per CU; G = 4, with 64 contiguous output bytes per channel, was
// slower at one workgroup per CU).  Stockham FFT (natural order, ping-pong
// between two LDS buffers of G L points): radix-4 iterations, plus one
// radix-2 iteration when log2 L is odd; the butterflies run in registers.
constexpr int G_MAX = 1;
constexpr int CTHREADS = 256;

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// e^{-2 pi i t / L} for 0 <= t < L from the half table
__device__ __forceinline__ float2 twiddle(const float2* tw, int t, int L) {
  const float2 w = tw[t & (L / 2 - 1)];
  return t < L / 2 ? w : make_float2(-w.x, -w.y);
}

__global__ __launch_bounds__(CTHREADS) void channelise(const int8_t* __restrict__ adc, int64_t n_samples,
                                                       int n_inputs, int L, int log2L, int G,
                                                       const float* __restrict__ tab, float2* __restrict__ out) {
  extern __shared__ float2 lds[];  // [2][G][L]
  float2* buf0 = lds;
  float2* buf1 = lds + G * L;
  // Work item w = (spectrum, pair group), pair group fastest.  Workgroups are
  // dealt to the 8 XCDs in turn; each XCD takes a contiguous range of w, so
  // the pairs of one spectrum, whose outputs interleave in the same 128-byte
  // lines of [spectrum][channel][input], are written through one L2.
  const int64_t total = (int64_t)gridDim.x * gridDim.y;
  const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
  const int64_t xq = total / 8, xr = total % 8, xcd = b % 8;
  const int64_t w = xcd * xq + (xcd < xr ? xcd : xr) + b / 8;
  const int q0 = (int)(w % gridDim.x) * G;   // first pair
  const int64_t s = w / gridDim.x;
  const int F = L / 2;
  const float* h = tab;
  const float2* tw = reinterpret_cast<const float2*>(tab + TAPS * L);

  // 1. polyphase FIR of every pair, 8 consecutive samples per thread-step
  const int steps = G * (L / 8);
  for (int u = threadIdx.x; u < steps; u += CTHREADS) {
    const int g = u / (L / 8), n0 = 8 * (u % (L / 8));
    const int8_t* x0 = adc + (int64_t)(2 * (q0 + g)) * n_samples + s * L + n0;
    const int8_t* x1 = x0 + n_samples;
    float a[8] = {}, b[8] = {};
#pragma unroll
    for (int p = 0; p < TAPS; ++p) {
      const uint2 u0 = *reinterpret_cast<const uint2*>(x0 + p * L);
      const uint2 u1 = *reinterpret_cast<const uint2*>(x1 + p * L);
      const float4 h0 = *reinterpret_cast<const float4*>(h + p * L + n0);
      const float4 h1 = *reinterpret_cast<const float4*>(h + p * L + n0 + 4);
      const float hv[8] = {h0.x, h0.y, h0.z, h0.w, h1.x, h1.y, h1.z, h1.w};
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int8_t s0 = (int8_t)(((k < 4 ? u0.x : u0.y) >> (8 * (k & 3))) & 0xFF);
        const int8_t s1 = (int8_t)(((k < 4 ? u1.x : u1.y) >> (8 * (k & 3))) & 0xFF);
        a[k] = fmaf(hv[k], (float)s0, a[k]);
        b[k] = fmaf(hv[k], (float)s1, b[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) buf0[g * L + n0 + k] = make_float2(a[k], b[k]);
  }
  __syncthreads();

  // 2. Stockham iterations: sub-transform size Ns -> R Ns
  float2* src = buf0;
  float2* dst = buf1;
  int Ns = 1;
  if (log2L & 1) {  // one radix-2 iteration
    for (int u = threadIdx.x; u < G * (L / 2); u += CTHREADS) {
      const int g = u / (L / 2), j = u % (L / 2);
      const float2 v0 = src[g * L + j], v1 = src[g * L + j + L / 2];
      dst[g * L + 2 * j] = make_float2(v0.x + v1.x, v0.y + v1.y);
      dst[g * L + 2 * j + 1] = make_float2(v0.x - v1.x, v0.y - v1.y);
    }
    Ns = 2;
    float2* t = src;
    src = dst;
    dst = t;
    __syncthreads();
  }
  for (; Ns < L; Ns <<= 2) {  // radix-4 iterations
    const int q = L / 4;
    for (int u = threadIdx.x; u < G * q; u += CTHREADS) {
      const int g = u / q, j = u % q;
      const float2* sg = src + g * L;
      const int k = j & (Ns - 1);
      const int t = k * (L / (4 * Ns));  // angle step of this butterfly, in units of 2 pi / L
      const float2 v0 = sg[j];
      const float2 v1 = cmul(sg[j + q], twiddle(tw, t, L));
      const float2 v2 = cmul(sg[j + 2 * q], twiddle(tw, 2 * t, L));
      const float2 v3 = cmul(sg[j + 3 * q], twiddle(tw, 3 * t, L));
      const float2 t0 = make_float2(v0.x + v2.x, v0.y + v2.y), t1 = make_float2(v0.x - v2.x, v0.y - v2.y);
      const float2 t2 = make_float2(v1.x + v3.x, v1.y + v3.y);
      const float2 t3 = make_float2(v1.y - v3.y, v3.x - v1.x);  // -i (v1 - v3)
      float2* dg = dst + g * L + ((j - k) << 2) + k;
      dg[0] = make_float2(t0.x + t2.x, t0.y + t2.y);
      dg[Ns] = make_float2(t1.x + t3.x, t1.y + t3.y);
      dg[2 * Ns] = make_float2(t0.x - t2.x, t0.y - t2.y);
      dg[3 * Ns] = make_float2(t1.x - t3.x, t1.y - t3.y);
    }
    float2* tmp = src;
    src = dst;
    dst = tmp;
    __syncthreads();
  }

  // 3. Eq. 2 split.  Lane (k, g): the pairs of one channel are consecutive
  //    lanes -> 16 G contiguous bytes per channel
  float4* o = reinterpret_cast<float4*>(out + (s * F) * (int64_t)n_inputs + 2 * q0);
  for (int u = threadIdx.x; u < G * F; u += CTHREADS) {
    const int k = u / G, g = u % G;
    const float2 yk = src[g * L + k], ym = src[g * L + ((L - k) & (L - 1))];
    const float2 x1 = make_float2(0.5f * (yk.x + ym.x), 0.5f * (yk.y - ym.y));
    const float dr = yk.x - ym.x, di = yk.y + ym.y;   // Y[k] - conj(Y[-k])
    o[(int64_t)k * (n_inputs / 2) + g] = make_float4(x1.x, x1.y, 0.5f * di, -0.5f * dr);
  }
}

// ---------------------------------------------------------------------------
// Register-resident form for L = 512, 1024, 2048 (F = 256, 512, 1024; the
// paper's FFT lengths are 512 and 1024 complex points).  A workgroup takes
// P input pairs (2 when the pair count is even, else 1), L / 8 threads per
// pair, and a run of consecutive spectra:
//  - thread t of a pair owns the points n = t + m L/8 (m < 8) of every
//    stage, which are the inputs of its first radix-8 butterfly; its 32
//    filter taps h[pL + n] and its twiddles stay in registers for the run;
//  - the four input blocks a spectrum's filter reads slide along the run:
//    each block of each stream is loaded once per run (one byte per point,
//    64 consecutive bytes per wave and point), converted once, and kept in
//    registers while the four spectra that use it are formed; the next
//    block's loads are issued a spectrum ahead;
//  - Stockham FFT: three radix-8 passes and, for L = 1024 / 2048, one
//    radix-2 / radix-4 pass, butterflies in registers; between passes the
//    points go through LDS (two buffers per pair, one barrier per exchange),
//    with an address swizzle per exchange chosen so that neither the writes
//    nor the reads of that exchange have bank conflicts;
//  - Eq. 2 reads Y[k] and Y[L - k] from LDS; neighbouring lanes take the P
//    pairs of one channel, so each store writes 16 P contiguous bytes.
// The output is [spectrum][channel][input]: a pair owns 16 bytes of each
// 1536-byte channel row at N = 192, and the cost of the run is in those
// scattered stores.  Short runs (8 spectra) keep the workgroups that share
// a 128-byte line close in time, so that the line is completed in L2 before
// it is written back; each XCD takes a contiguous range of work items (pair
// group fastest).
// ---------------------------------------------------------------------------

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// 4-point forward DFT in place
__device__ __forceinline__ void dft4(float2& x0, float2& x1, float2& x2, float2& x3) {
  const float2 s02 = cadd(x0, x2), d02 = csub(x0, x2);
  const float2 s13 = cadd(x1, x3);
  const float2 d13 = make_float2(x1.y - x3.y, x3.x - x1.x);  // -i (x1 - x3)
  x0 = cadd(s02, s13);
  x2 = csub(s02, s13);
  x1 = cadd(d02, d13);
  x3 = csub(d02, d13);
}

// 8-point forward DFT in place, natural order: X[2r] = DFT4(a_n + a_n+4)[r],
// X[2r+1] = DFT4((a_n - a_n+4) e^{-2 pi i n / 8})[r]
__device__ __forceinline__ void dft8(float2 (&a)[8]) {
  constexpr float R = 0.70710678118654752440f;
  float2 e0 = cadd(a[0], a[4]), e1 = cadd(a[1], a[5]), e2 = cadd(a[2], a[6]), e3 = cadd(a[3], a[7]);
  float2 o0 = csub(a[0], a[4]), o1 = csub(a[1], a[5]), o2 = csub(a[2], a[6]), o3 = csub(a[3], a[7]);
  o1 = make_float2((o1.x + o1.y) * R, (o1.y - o1.x) * R);      // x (1 - i) / sqrt 2
  o2 = make_float2(o2.y, -o2.x);                               // x (-i)
  o3 = make_float2((o3.y - o3.x) * R, -(o3.x + o3.y) * R);     // x (-1 - i) / sqrt 2
  dft4(e0, e1, e2, e3);
  dft4(o0, o1, o2, o3);
  a[0] = e0; a[2] = e1; a[4] = e2; a[6] = e3;
  a[1] = o0; a[3] = o1; a[5] = o2; a[7] = o3;
}

// LDS address swizzles, one per exchange (bijections on [0, L); the second
// pads one entry per 32)
struct SwzA { __device__ int operator()(int i) const { return i ^ ((i >> 3) & 31); } };
struct SwzB { __device__ int operator()(int i) const { return i + (i >> 5); } };
struct SwzY { __device__ int operator()(int i) const { return i ^ ((i >> 2) & 1); } };

constexpr int REG_CHUNK = 8;   // spectra per workgroup run

template <int L, int P>
__global__ __launch_bounds__(P * L / 8) void channelise_reg(const int8_t* __restrict__ adc, int64_t n_samples,
                                                         int n_inputs, int n_spec, int chunk,
                                                         const float* __restrict__ tab,
                                                         float4* __restrict__ out) {
  constexpr int TH = L / 8, F = L / 2, RL = L / 512;     // RL: radix of the last pass (1: none)
  constexpr int EX = RL > 1 ? 4 : 3;                      // LDS exchanges per spectrum
  constexpr int BUF = L + L / 32 + 8;
  __shared__ float2 lds_all[2][P][BUF];
  const int pp = threadIdx.x / TH;
  const int t = threadIdx.x % TH;
  const int pairs = n_inputs / 2;
  const int groups = pairs / P;
  // work item (pair group fastest): each XCD takes a contiguous range
  const int64_t total = gridDim.x, b = blockIdx.x;
  const int64_t xq = total / 8, xr = total % 8, xcd = b % 8;
  const int64_t w = xcd * xq + (xcd < xr ? xcd : xr) + b / 8;
  const int qg = (int)(w % groups);
  const int q = qg * P + pp;
  const int s0 = (int)(w / groups) * chunk;
  const int s1 = min(n_spec, s0 + chunk);
  const float2* tw = reinterpret_cast<const float2*>(tab + 4 * L);

  float hr[4][8];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int m = 0; m < 8; ++m) hr[p][m] = tab[p * L + t + m * TH];
  float2 w2[8], w3[8], wl[8];
#pragma unroll
  for (int m = 1; m < 8; ++m) {
    w2[m] = twiddle(tw, (m * (t & 7) * (L / 64)) & (L - 1), L);     // pass 2: Ns = 8
    w3[m] = twiddle(tw, (m * (t & 63) * (L / 512)) & (L - 1), L);   // pass 3: Ns = 64
  }
  if constexpr (RL == 4) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int m = 1; m < 4; ++m) wl[4 * i + m] = twiddle(tw, (m * (t + i * TH)) & (L - 1), L);
  } else if constexpr (RL == 2) {
#pragma unroll
    for (int i = 0; i < 4; ++i) wl[i] = twiddle(tw, t + i * TH, L);
  }

  const int8_t* xs[2] = {adc + (int64_t)(2 * q) * n_samples + t, adc + (int64_t)(2 * q + 1) * n_samples + t};
  float xw[4][2][8];   // window slot (block - s0) mod 4, stream, point
  int inc[2][8];       // loads of the next block
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int m = 0; m < 8; ++m) xw[b][c][m] = (float)xs[c][(int64_t)(s0 + b) * L + m * TH];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int m = 0; m < 8; ++m) inc[c][m] = xs[c][(int64_t)(s0 + 3) * L + m * TH];

  auto exchange_write = [&](int buf, auto swz, const float2 (&a)[8], auto index) {
#pragma unroll
    for (int m = 0; m < 8; ++m) lds_all[buf][pp][swz(index(m))] = a[m];
  };
  auto exchange_read = [&](int buf, auto swz, float2 (&a)[8]) {
#pragma unroll
    for (int m = 0; m < 8; ++m) a[m] = lds_all[buf][pp][swz(t + m * TH)];
  };
  auto twiddled_dft8 = [&](float2 (&a)[8], const float2 (&wv)[8]) {
#pragma unroll
    for (int m = 1; m < 8; ++m) a[m] = cmul(a[m], wv[m]);
    dft8(a);
  };

  auto spectrum = [&](auto U_, int s) {
    constexpr int U = decltype(U_)::value;
    constexpr int E0 = (U * EX) & 1;                    // buffer of this spectrum's first exchange
    // block s + 3 has arrived; issue block s + 4 for the next spectrum
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int m = 0; m < 8; ++m) xw[(U + 3) & 3][c][m] = (float)inc[c][m];
    if (s + 1 < s1) {
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int m = 0; m < 8; ++m) inc[c][m] = xs[c][(int64_t)(s + 4) * L + m * TH];
    }
    // Eq. 1 after the polyphase filter: y = v_2q + j v_2q+1
    float2 a[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      float v0 = hr[0][m] * xw[U & 3][0][m], v1 = hr[0][m] * xw[U & 3][1][m];
#pragma unroll
      for (int p = 1; p < 4; ++p) {
        v0 = fmaf(hr[p][m], xw[(U + p) & 3][0][m], v0);
        v1 = fmaf(hr[p][m], xw[(U + p) & 3][1][m], v1);
      }
      a[m] = make_float2(v0, v1);
    }
    // pass 1 (Ns = 1): outputs to 8 t + m
    dft8(a);
    exchange_write(E0, SwzA{}, a, [&](int m) { return 8 * t + m; });
    __syncthreads();
    exchange_read(E0, SwzA{}, a);
    // pass 2 (Ns = 8)
    twiddled_dft8(a, w2);
    exchange_write(E0 ^ 1, SwzA{}, a, [&](int m) { return 8 * (t & ~7) + (t & 7) + 8 * m; });
    __syncthreads();
    exchange_read(E0 ^ 1, SwzA{}, a);
    // pass 3 (Ns = 64)
    twiddled_dft8(a, w3);
    int ybuf;
    if constexpr (RL == 1) {           // Y in natural order
      exchange_write(E0, SwzY{}, a, [&](int m) { return 8 * (t & ~63) + (t & 63) + 64 * m; });
      ybuf = E0;
    } else {
      exchange_write(E0, SwzB{}, a, [&](int m) { return 8 * (t & ~63) + (t & 63) + 64 * m; });
      __syncthreads();
      exchange_read(E0, SwzB{}, a);
      // last pass (Ns = L / RL): butterfly j = t + i L/8 reads points j + m L/RL
      if constexpr (RL == 4) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          float2 b0 = a[i], b1 = cmul(a[i + 2], wl[4 * i + 1]), b2 = cmul(a[i + 4], wl[4 * i + 2]),
                 b3 = cmul(a[i + 6], wl[4 * i + 3]);
          dft4(b0, b1, b2, b3);
          a[i] = b0; a[i + 2] = b1; a[i + 4] = b2; a[i + 6] = b3;
        }
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float2 b = cmul(a[i + 4], wl[i]);
          const float2 u = a[i];
          a[i] = cadd(u, b);
          a[i + 4] = csub(u, b);
        }
      }
      exchange_write(E0 ^ 1, SwzY{}, a, [&](int m) { return t + m * TH; });
      ybuf = E0 ^ 1;
    }
    __syncthreads();
    // Eq. 2 split: lane u takes pair u % P of channel u / P (+ r L/8), so
    // the P pairs of a channel are written by neighbouring lanes
    float4* o = out + ((int64_t)s * F) * pairs + qg * P;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int u = threadIdx.x;
      const int p2 = u % P;
      const int k = u / P + r * TH;
      const float2 yk = lds_all[ybuf][p2][SwzY{}(k)], ym = lds_all[ybuf][p2][SwzY{}((L - k) & (L - 1))];
      const float dr = yk.x - ym.x, di = yk.y + ym.y;   // Y[k] - conj(Y[-k])
      o[(int64_t)k * pairs + p2] = make_float4(0.5f * (yk.x + ym.x), 0.5f * (yk.y - ym.y), 0.5f * di, -0.5f * dr);
    }
  };

  for (int s = s0; s < s1; s += 4) {
    spectrum(std::integral_constant<int, 0>{}, s);
    if (s + 1 >= s1) break;
    spectrum(std::integral_constant<int, 1>{}, s + 1);
    if (s + 2 >= s1) break;
    spectrum(std::integral_constant<int, 2>{}, s + 2);
    if (s + 3 >= s1) break;
    spectrum(std::integral_constant<int, 3>{}, s + 3);
  }
}

int log2_exact(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return (1 << l) == v ? l : -1;
}

}  // namespace
}  // namespace xeng

extern "C" int64_t xeng_channelise_spectra(int64_t n_samples, int32_t n_chans) {
  if (n_samples < 0 || n_chans < 1) return -1;
  const int64_t L = 2LL * n_chans;
  const int64_t s = n_samples / L - xeng::TAPS + 1;
  return s > 0 ? s : 0;
}

extern "C" int64_t xeng_channelise_table_floats(int32_t n_chans) {
  if (n_chans < 1) return -1;
  return (int64_t)xeng::TAPS * 2 * n_chans + 2 * n_chans;  // h[4L] + L/2 complex twiddles
}

namespace xeng {
namespace {

int channelise_impl(const int8_t* d_adc, int64_t n_samples, int32_t n_inputs, int32_t n_chans, float* d_out,
                    float* d_tables, void* hip_stream) {
  const int L = 2 * n_chans;
  const int log2L = xeng::log2_exact(L);
  if (!d_adc || !d_tables || n_inputs < 2 || n_inputs % 2 || n_chans < 8 || L > xeng::MAX_L ||
      log2L < 0 || n_samples < 0 || n_samples % 8 || (reinterpret_cast<uintptr_t>(d_adc) & 7u) ||
      (reinterpret_cast<uintptr_t>(d_out) & 15u) || (reinterpret_cast<uintptr_t>(d_tables) & 15u))
    return XENG_EINVAL;
  const int64_t S = xeng_channelise_spectra(n_samples, n_chans);
  if (S > 0 && !d_out) return XENG_EINVAL;  // (no spectra: d_out is not touched and may be null)
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const int tab_n = xeng::TAPS * L + L / 2;
  hipLaunchKernelGGL(xeng::chan_tables, dim3((tab_n + xeng::THREADS - 1) / xeng::THREADS), dim3(xeng::THREADS),
                     0, st, d_tables, L);
  if (S > 0) {
    if (S > 2147483647LL) return XENG_EINVAL;
    const int pairs = n_inputs / 2;
    if (L >= 512) {
      // two pairs per workgroup when the pair count allows, runs of
      // REG_CHUNK spectra
      const int P = pairs % 2 == 0 ? 2 : 1;
      const int64_t wgs = (int64_t)(pairs / P) * ((S + xeng::REG_CHUNK - 1) / xeng::REG_CHUNK);
      if (wgs > 2147483647LL) return XENG_EINVAL;
      const dim3 grid((unsigned)wgs), block((unsigned)(P * L / 8));
      auto out4 = reinterpret_cast<float4*>(d_out);
      const int chunk = xeng::REG_CHUNK;
#define XENG_CHAN_REG(LL, PP)                                                                                 \
  hipLaunchKernelGGL((xeng::channelise_reg<LL, PP>), grid, block, 0, st, d_adc, n_samples, n_inputs, (int)S, \
                     chunk, d_tables, out4)
      if (L == 512) {
        if (P == 2) XENG_CHAN_REG(512, 2); else XENG_CHAN_REG(512, 1);
      } else if (L == 1024) {
        if (P == 2) XENG_CHAN_REG(1024, 2); else XENG_CHAN_REG(1024, 1);
      } else {
        if (P == 2) XENG_CHAN_REG(2048, 2); else XENG_CHAN_REG(2048, 1);
      }
#undef XENG_CHAN_REG
      return hipGetLastError() == hipSuccess ? XENG_OK : XENG_EDEVICE;
    }
    int G = xeng::G_MAX;
    while (pairs % G) G >>= 1;
    const size_t lds = (size_t)2 * G * L * sizeof(float2);  // up to 128 KB
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&xeng::channelise),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
      return XENG_EDEVICE;
    hipLaunchKernelGGL(xeng::channelise, dim3((unsigned)(pairs / G), (unsigned)S), dim3(xeng::CTHREADS),
                       lds, st, d_adc, n_samples, n_inputs, L, log2L, G, d_tables,
                       reinterpret_cast<float2*>(d_out));
  }
  return hipGetLastError() == hipSuccess ? XENG_OK : XENG_EDEVICE;
}

// Table scratch of the allocation-free entry point: one array per GPU, for
// the largest spectrum (F = 1024: 4 * 2F + 2F floats), held until the
// process ends.  In host code `scratch` only names the symbol; its device
// address, per device, comes from hipGetSymbolAddress on the first call made
// with that device current.
constexpr int SCRATCH_FLOATS = TAPS * MAX_L + MAX_L;
static __device__ __align__(256) float scratch[SCRATCH_FLOATS];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mutex;
float* scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on the current device (null on failure).
float* scratch_on_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(scratch_mutex);
  if (!scratch_ptr[dev]) {
    float* ptr = nullptr;
    if (hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return nullptr;
    }
    scratch_ptr[dev] = ptr;
  }
  return scratch_ptr[dev];
}

}  // namespace
}  // namespace xeng

extern "C" int xeng_channelise(const int8_t* d_adc, int64_t n_samples, int32_t n_inputs, int32_t n_chans,
                               float* d_out, float* d_tables, void* hip_stream) {
  return xeng::channelise_impl(d_adc, n_samples, n_inputs, n_chans, d_out, d_tables, hip_stream);
}

extern "C" int xeng_channelise_noalloc(const int8_t* d_adc, int64_t n_samples, int32_t n_inputs,
                                       int32_t n_chans, float* d_out, void* hip_stream) {
  if (n_chans < 1 || xeng_channelise_table_floats(n_chans) > xeng::SCRATCH_FLOATS) return XENG_EINVAL;
  float* tables = xeng::scratch_on_current_device();
  if (!tables) return XENG_EDEVICE;
  return xeng::channelise_impl(d_adc, n_samples, n_inputs, n_chans, d_out, tables, hip_stream);
}
