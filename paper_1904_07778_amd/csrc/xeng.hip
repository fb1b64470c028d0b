// xeng.hip - host side of the X-engine C ABI (declared in include/xeng.h).
//
// A plan holds, per array, the HBM-resident int32 accumulator [F][nbl][2],
// the number of samples integrated since the last dump, and the kernel
// configuration chosen for its N.  xeng_correlate validates, applies the
// overflow guard and launches; xeng_dump copies the accumulator out and
// clears it on the plan's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/xeng.h"
#include "kernels.hpp"

namespace {

using xeng::KernelInfo;

struct ArrayState {
  xeng_array_desc d{};
  int32_t* acc = nullptr;
  size_t acc_bytes = 0;
  int64_t n_integrated = 0;
  bool clean = true;  // accumulator is all zero (no launch since the last clear)
  const KernelInfo* k = nullptr;
};

}  // namespace

struct xeng_plan_s {
  int device = 0;
  int n_cu = 256;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool dead = false;
  std::vector<ArrayState> arrays;
  std::string err;
};

namespace {

int fail(xeng_plan_t* p, int status, const char* fmt, ...) {
  if (p) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    p->err = buf;
    if (status == XENG_EDEVICE) p->dead = true;
  }
  return status;
}

int hip_fail(xeng_plan_t* p, hipError_t e, const char* what) {
  return fail(p, XENG_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool aligned16(const void* ptr) { return (reinterpret_cast<uintptr_t>(ptr) & 15u) == 0; }

int64_t nbl_of(int32_t n) { return (int64_t)n * (n + 1) / 2; }

// Grid for one call: channel groups x time splits.  Time is split only when
// the channel groups alone leave the GPU short of workgroups.
void grid_for(const xeng_plan_t* p, const ArrayState& s, int64_t T, dim3& grid, int64_t& t_chunk,
              int& mode) {
  const int ngroups = (s.d.n_chans + s.k->cpw - 1) / s.k->cpw;
  const int64_t target = 2LL * p->n_cu;
  int64_t ts = (target + ngroups - 1) / ngroups;
  ts = std::max<int64_t>(1, std::min<int64_t>(ts, T / 256));
  ts = std::max<int64_t>(ts, (T + s.k->max_t_per_wg - 1) / s.k->max_t_per_wg);
  t_chunk = (T + ts - 1) / ts;
  t_chunk = (t_chunk + xeng::KS - 1) / xeng::KS * xeng::KS;
  ts = (T + t_chunk - 1) / t_chunk;
  grid = dim3((unsigned)ngroups, (unsigned)ts, 1);
  mode = ts > 1 ? xeng::EPI_ATOMIC : (s.clean ? xeng::EPI_STORE : xeng::EPI_ADD);
}

}  // namespace

extern "C" {

int64_t xeng_nbaselines(int32_t n) { return n < 0 ? -1 : nbl_of(n); }

int64_t xeng_baseline_index(int32_t i, int32_t j) {
  if (i < 0 || j < 0 || j > i) return -1;
  return (int64_t)i * (i + 1) / 2 + j;
}

const char* xeng_strerror(int status) {
  switch (status) {
    case XENG_OK: return "ok";
    case XENG_EINVAL: return "invalid argument";
    case XENG_ENOMEM: return "out of memory";
    case XENG_EOVERFLOW: return "integration would overflow int32";
    case XENG_EDEVICE: return "HIP device error";
    case XENG_ESTATE: return "plan unusable after an earlier device error";
    default: return "unknown status";
  }
}

const char* xeng_last_error(const xeng_plan_t* p) { return p ? p->err.c_str() : ""; }

int64_t xeng_integrated(const xeng_plan_t* p, int32_t array) {
  if (!p || array < 0 || array >= (int32_t)p->arrays.size()) return -1;
  return p->arrays[array].n_integrated;
}

int xeng_plan(xeng_plan_t** out, const xeng_array_desc* arrays, int32_t n_arrays, uint32_t flags,
              void* hip_stream) {
  if (!out || !arrays || n_arrays < 1 || flags != 0) return XENG_EINVAL;
  *out = nullptr;
  for (int32_t a = 0; a < n_arrays; ++a) {
    const xeng_array_desc& d = arrays[a];
    if (d.n_inputs < 1 || d.n_inputs > XENG_MAX_INPUTS || d.n_chans < 1 ||
        d.max_time_per_call < 1 || d.max_time_per_call > XENG_MAX_INTEGRATION)
      return XENG_EINVAL;
  }
  xeng_plan_t* p = new (std::nothrow) xeng_plan_t();
  if (!p) return XENG_ENOMEM;
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    delete p;
    return XENG_EDEVICE;
  }
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p->device) == hipSuccess &&
      ncu > 0)
    p->n_cu = ncu;
  if (hip_stream) {
    p->stream = reinterpret_cast<hipStream_t>(hip_stream);
  } else {
    e = hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete p;
      return XENG_EDEVICE;
    }
    p->own_stream = true;
  }
  p->arrays.resize(n_arrays);
  for (int32_t a = 0; a < n_arrays; ++a) {
    ArrayState& s = p->arrays[a];
    s.d = arrays[a];
    const int nt = (s.d.n_inputs + 15) / 16;
    s.k = (s.d.n_inputs % 16 == 0) ? xeng::x32_kernel(s.d.n_inputs) : xeng::stage_kernel(nt);
    s.acc_bytes = (size_t)s.d.n_chans * nbl_of(s.d.n_inputs) * 2 * sizeof(int32_t);
    e = hipMalloc(&s.acc, s.acc_bytes);
    if (e != hipSuccess) {
      xeng_destroy(p);
      return e == hipErrorOutOfMemory ? XENG_ENOMEM : XENG_EDEVICE;
    }
    e = hipMemsetAsync(s.acc, 0, s.acc_bytes, p->stream);
    if (e != hipSuccess) {
      xeng_destroy(p);
      return XENG_EDEVICE;
    }
  }
  *out = p;
  return XENG_OK;
}

int xeng_correlate(xeng_plan_t* p, const uint8_t* const* d_voltages, const int64_t* n_time) {
  if (!p || !n_time) return XENG_EINVAL;
  if (p->dead) return XENG_ESTATE;
  const int32_t na = (int32_t)p->arrays.size();
  for (int32_t a = 0; a < na; ++a) {
    const ArrayState& s = p->arrays[a];
    const int64_t T = n_time[a];
    if (T < 0 || T > s.d.max_time_per_call)
      return fail(p, XENG_EINVAL, "array %d: n_time %lld outside [0, %lld]", a, (long long)T,
                  (long long)s.d.max_time_per_call);
    if (T > 0 && (!d_voltages || !d_voltages[a] || !aligned16(d_voltages[a])))
      return fail(p, XENG_EINVAL, "array %d: voltage pointer null or not 16-byte aligned", a);
    if (s.n_integrated + T > XENG_MAX_INTEGRATION)
      return fail(p, XENG_EOVERFLOW, "array %d: %lld + %lld samples exceed %lld", a,
                  (long long)s.n_integrated, (long long)T, (long long)XENG_MAX_INTEGRATION);
  }
  for (int32_t a = 0; a < na; ++a) {
    ArrayState& s = p->arrays[a];
    const int64_t T = n_time[a];
    if (T == 0) continue;
    xeng::Args args{};
    args.v = d_voltages[a];
    args.acc = s.acc;
    args.T = T;
    args.F = s.d.n_chans;
    args.N = s.d.n_inputs;
    dim3 grid;
    grid_for(p, s, T, grid, args.t_chunk, args.mode);
    hipError_t e = s.k->launch(grid, p->stream, args);
    if (e != hipSuccess) return hip_fail(p, e, "kernel launch");
    s.n_integrated += T;
    s.clean = false;
  }
  return XENG_OK;
}

int xeng_dump(xeng_plan_t* p, int32_t array, int32_t* const* dst, uint32_t flags,
              int64_t* n_integrated) {
  if (!p || !dst) return XENG_EINVAL;
  if (p->dead) return XENG_ESTATE;
  if (flags & ~(uint32_t)(XENG_DUMP_KEEP | XENG_DUMP_TO_HOST)) return XENG_EINVAL;
  const int32_t na = (int32_t)p->arrays.size();
  if (array < -1 || array >= na) return fail(p, XENG_EINVAL, "array index %d out of range", array);
  const int32_t a0 = array < 0 ? 0 : array, a1 = array < 0 ? na : array + 1;
  for (int32_t a = a0; a < a1; ++a)
    if (!dst[a - a0]) return fail(p, XENG_EINVAL, "dump destination %d is null", a - a0);
  const bool to_host = (flags & XENG_DUMP_TO_HOST) != 0;
  for (int32_t a = a0; a < a1; ++a) {
    ArrayState& s = p->arrays[a];
    hipError_t e = hipMemcpyAsync(dst[a - a0], s.acc, s.acc_bytes,
                                  to_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                                  p->stream);
    if (e != hipSuccess) return hip_fail(p, e, "dump copy");
    if (n_integrated) n_integrated[a - a0] = s.n_integrated;
    if (!(flags & XENG_DUMP_KEEP)) {
      e = hipMemsetAsync(s.acc, 0, s.acc_bytes, p->stream);
      if (e != hipSuccess) return hip_fail(p, e, "dump clear");
      s.n_integrated = 0;
      s.clean = true;
    }
  }
  if (to_host) {
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(p, e, "dump synchronize");
  }
  return XENG_OK;
}

void xeng_destroy(xeng_plan_t* p) {
  if (!p) return;
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  for (ArrayState& s : p->arrays)
    if (s.acc) (void)hipFree(s.acc);
  if (p->own_stream && p->stream) (void)hipStreamDestroy(p->stream);
  delete p;
}

}  // extern "C"
