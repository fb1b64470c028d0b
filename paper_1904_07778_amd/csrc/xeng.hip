// xeng.hip - host side of the X-engine C ABI (declared in include/xeng.h).
//
// A plan holds, per array slot, the HBM-resident int32 accumulator
// [F][nbl][2], the number of samples integrated since the last dump, and the
// kernel configuration chosen for its N.  xeng_correlate validates, applies
// the overflow guard and launches: one launch per array in a plain plan, one
// captured graph around the persistent batch kernel in a batched plan.
// xeng_dump copies the accumulators out and clears them on the plan's
// stream.  Slots can be attached and detached between calls (admission in a
// serving loop).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/xeng.h"
#include "batch.hpp"
#include "kernels.hpp"

namespace {

using xeng::KernelInfo;

struct ArrayState {
  xeng_array_desc d{};
  bool active = false;  // slot holds an array (attached, not detached)
  int32_t* acc = nullptr;
  size_t acc_bytes = 0;
  int64_t n_integrated = 0;
  bool clean = true;   // integration is empty (no launch since the last dump or clear)
  bool zeroed = true;  // accumulator memory holds zeros (a dump does not clear it:
                       // the next launch overwrites it with plain stores, or
                       // zeroes it first when it must add atomically)
  const KernelInfo* k = nullptr;  // kernel of the plain launch
  int split = 1;                  // plain launch: aim for split * n_cu workgroups
  bool own_launch = false;        // batched plan: a plain launch of its own inside the
                                  // graph instead of items of the persistent launch
};

// ---- tuning cache: the launch shapes the autotuner picked, by GPU
// architecture, plan kind, N and the power-of-two buckets of F and T, for the
// whole process (xeng_tune_cache_save / _load write and read it as text).
enum KernelKind { KIND_X16 = 0, KIND_X32 = 1, KIND_STAGE = 2 };

const KernelInfo* kernel_of(int kind, int32_t n) {
  switch (kind) {
    case KIND_X16: return xeng::x16_kernel(n);
    case KIND_X32: return xeng::x32_kernel(n);
    case KIND_STAGE: return xeng::stage_kernel((n + 15) / 16);
    default: return nullptr;
  }
}

int kind_of(const KernelInfo* k, int32_t n) {
  if (k == xeng::x16_kernel(n)) return KIND_X16;
  if (k == xeng::x32_kernel(n)) return KIND_X32;
  return KIND_STAGE;
}

int bucket(int64_t v) {  // ceil(log2 v)
  int b = 0;
  while (((int64_t)1 << b) < v && b < 62) ++b;
  return b;
}

struct TuneKey {
  std::string arch;
  int batched, n, fb, tb;
  bool operator<(const TuneKey& o) const {
    return std::tie(arch, batched, n, fb, tb) < std::tie(o.arch, o.batched, o.n, o.fb, o.tb);
  }
};
struct TuneVal {
  int kind, split, own;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;

}  // namespace

struct xeng_plan_s {
  int device = 0;
  int n_cu = 256;
  std::string arch;       // gcnArchName of the device (tuning-cache key)
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool dead = false;
  bool batched = false;   // calls go through the persistent batch launch
  int batch_split = 2;    // batch: about batch_split items per workgroup
  std::vector<ArrayState> arrays;
  int32_t* counters = nullptr;  // batch queue heads, zero between launches
  // Ring of instantiated graphs of batched calls, each with the event of its
  // last launch (a graph is updated only once that launch has completed).
  static constexpr int GRAPH_RING = 4;
  hipGraphExec_t exec[GRAPH_RING] = {};
  hipEvent_t done[GRAPH_RING] = {};
  int next_graph = 0;
  xeng_stats_t stats{};   // counters since the plan was made
  bool trace = false;     // XENG_TRACE set: one stderr line per launch
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
  const int64_t target = (int64_t)s.split * p->n_cu;
  int64_t ts = (target + ngroups - 1) / ngroups;
  ts = std::max<int64_t>(1, std::min<int64_t>(ts, T / 256));
  ts = std::max<int64_t>(ts, (T + s.k->max_t_per_wg - 1) / s.k->max_t_per_wg);
  t_chunk = (T + ts - 1) / ts;
  t_chunk = (t_chunk + xeng::KS - 1) / xeng::KS * xeng::KS;
  ts = (T + t_chunk - 1) / t_chunk;
  grid = dim3((unsigned)ngroups, (unsigned)ts, 1);
  mode = ts > 1 ? xeng::EPI_ATOMIC : (s.clean ? xeng::EPI_STORE : xeng::EPI_ADD);
}


bool valid_desc(const xeng_array_desc& d) {
  return d.n_inputs >= 1 && d.n_inputs <= XENG_MAX_INPUTS && d.n_chans >= 1 &&
         (int64_t)d.n_chans * d.n_inputs <= INT32_MAX &&  // one time row indexes in 32 bits
         d.max_time_per_call >= 1 && d.max_time_per_call <= XENG_MAX_INTEGRATION;
}

bool kernel_fits(const KernelInfo* k, const xeng_array_desc& d) {
  return k && (k->max_row_bytes == 0 || (int64_t)d.n_chans * d.n_inputs <= k->max_row_bytes);
}

// Default kernel for an array: the 16-row-tile ring kernel when N is a
// multiple of 16 it is built for (and its time rows fit its 32-bit offsets),
// else the 32-row-tile ring kernel when N is a multiple of 16, else the
// staging kernel of 16-row tiles.
const KernelInfo* default_kernel(const xeng_array_desc& d) {
  const int32_t n = d.n_inputs;
  if (n % 16 == 0) {
    const KernelInfo* k = xeng::x16_kernel(n);
    if (kernel_fits(k, d)) return k;
    k = xeng::x32_kernel(n);
    if (k) return k;
  }
  return xeng::stage_kernel((n + 15) / 16);
}

// The cached choice for an array of this plan, if the autotuner has made one.
void apply_cached(const xeng_plan_t* p, ArrayState& s, int64_t T) {
  const TuneKey key{p->arch, p->batched ? 1 : 0, s.d.n_inputs, bucket(s.d.n_chans), bucket(T)};
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tune.find(key);
  if (it == g_tune.end()) return;
  const KernelInfo* k = kernel_of(it->second.kind, s.d.n_inputs);
  if (!kernel_fits(k, s.d)) return;
  s.k = k;
  s.split = it->second.split;
  s.own_launch = p->batched && it->second.own;
}

// The batched plan's own choice (items per workgroup) is kept under N = 0,
// keyed by the base-2 bucket of the plan's array count.
TuneKey plan_key(const xeng_plan_t* p, int32_t n_arrays) { return TuneKey{p->arch, 1, 0, 0, bucket(n_arrays)}; }

void apply_cached_plan(xeng_plan_t* p, int32_t n_arrays) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tune.find(plan_key(p, n_arrays));
  if (it != g_tune.end()) p->batch_split = it->second.split;
}

void record_choice(const xeng_plan_t* p, const ArrayState& s, int64_t T) {
  const TuneKey key{p->arch, p->batched ? 1 : 0, s.d.n_inputs, bucket(s.d.n_chans), bucket(T)};
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune[key] = TuneVal{kind_of(s.k, s.d.n_inputs), s.split, s.own_launch ? 1 : 0};
}

// Untuned time split: two workgroups per CU where the kernel's LDS lets
// several share a CU (the staging kernel, the ring kernel at N = 16), one
// where its ring fills most of the CU's LDS: a second workgroup could not
// run beside the first, and aiming for it only splits time into atomic adds
// and a zeroing pass (45-60% slower at N = 48..112, F = 1024).
int default_split(const KernelInfo* k) { return k->lds_bytes <= 64 * 1024 ? 2 : 1; }

int init_slot(xeng_plan_t* p, ArrayState& s, const xeng_array_desc& d) {
  s = ArrayState{};
  s.d = d;
  s.k = default_kernel(d);
  s.split = default_split(s.k);
  apply_cached(p, s, d.max_time_per_call);
  s.acc_bytes = (size_t)d.n_chans * nbl_of(d.n_inputs) * 2 * sizeof(int32_t);
  hipError_t e = hipMalloc(&s.acc, s.acc_bytes);
  if (e != hipSuccess) {
    s.acc = nullptr;
    return e == hipErrorOutOfMemory ? fail(p, XENG_ENOMEM, "accumulator of %zu bytes", s.acc_bytes)
                                    : hip_fail(p, e, "accumulator allocation");
  }
  e = hipMemsetAsync(s.acc, 0, s.acc_bytes, p->stream);
  if (e != hipSuccess) return hip_fail(p, e, "accumulator clear");
  s.active = true;
  return XENG_OK;
}

// Zero the accumulators of the given arrays with one kernel launch (the dump
// kernel with a null source), so the launch may be recorded into a graph.
int zero_fill(xeng_plan_t* p, const std::vector<ArrayState*>& arrays) {
  xeng::DumpParams dp{};
  int64_t most = 0;
  auto flush = [&]() -> int {
    if (dp.count == 0) return XENG_OK;
    const int64_t blocks = std::min<int64_t>((most + 1023) / 1024, 8LL * p->n_cu);
    hipError_t e = xeng::dump_launch((int)std::max<int64_t>(1, blocks), p->stream, dp);
    dp.count = 0;
    most = 0;
    return e == hipSuccess ? XENG_OK : hip_fail(p, e, "accumulator clear");
  };
  for (ArrayState* s : arrays) {
    dp.acc[dp.count] = nullptr;
    dp.dst[dp.count] = reinterpret_cast<int2*>(s->acc);
    dp.n[dp.count] = (int64_t)(s->acc_bytes / sizeof(int2));
    most = std::max(most, dp.n[dp.count]);
    s->zeroed = true;
    if (++dp.count == xeng::DUMP_MAX) {
      const int st = flush();
      if (st != XENG_OK) return st;
    }
  }
  return flush();
}

xeng::Args base_args(const ArrayState& s, const uint8_t* v, int64_t T) {
  xeng::Args a{};
  a.v = v;
  a.acc = s.acc;
  a.T = T;
  a.F = s.d.n_chans;
  a.N = s.d.n_inputs;
  return a;
}

int launch_plain(xeng_plan_t* p, ArrayState& s, const uint8_t* v, int64_t T) {
  xeng::Args args = base_args(s, v, T);
  dim3 grid;
  grid_for(p, s, T, grid, args.t_chunk, args.mode);
  ++p->stats.launches;
  if (p->trace)
    fprintf(stderr, "xeng: plan %p plain launch N=%d F=%d T=%lld grid=%ux%u threads=%d mode=%d\n", (void*)p,
            args.N, args.F, (long long)T, grid.x, grid.y, s.k->threads, args.mode);
  if (args.mode == xeng::EPI_ATOMIC && s.clean && !s.zeroed) {
    const int st = zero_fill(p, {&s});
    if (st != XENG_OK) return st;
  }
  hipError_t e = s.k->launch(grid, p->stream, args);
  return e == hipSuccess ? XENG_OK : hip_fail(p, e, "kernel launch");
}

// Batched call.  Arrays whose N the batch kernel covers become items of one
// persistent launch (several when there are more than batch::MAX_ARRAYS);
// the rest get their plain launch.  Per array the time range is cut into
// chunks so that the items come to about batch_split per workgroup, from a
// cost model of the kernel (the larger of its MFMA cycles and its HBM bytes
// per sample, plus a fixed start-up cost per item); arrays are queued longest
// item first.
constexpr double ITEM_START_CYCLES = 4000.0;  // ring fill and epilogue of one item
constexpr double HBM_BYTES_PER_CYCLE = 13.0;  // 8 TB/s over 256 CUs at 2.4 GHz

double cycles_per_sample(const KernelInfo* k, int32_t n) {
  // units (real or imaginary product of one tile pair) per channel; a 32-row
  // unit takes 32 MFMA cycles per 16 samples, a 16-row unit 16 cycles per 32
  // samples; a workgroup's four SIMDs share its CPW channels' units
  const int nt = (n + k->tile_rows - 1) / k->tile_rows;
  const double per_unit = k->tile_rows == 32 ? 2.0 : 0.5;
  const double mfma = (double)nt * (nt + 1) * per_unit * k->cpw / 4.0;
  const double hbm = (double)k->cpw * n / HBM_BYTES_PER_CYCLE;
  return mfma > hbm ? mfma : hbm;
}

struct BatchEntry {
  int32_t a;
  int32_t ngroups, nchunks;
  int64_t t_chunk;
  double item_cycles;
};

int record_batched(xeng_plan_t* p, const uint8_t* const* v, const int64_t* n_time) {
  std::vector<BatchEntry> items;
  std::vector<int32_t> others;
  double total = 0;
  for (int32_t a = 0; a < (int32_t)p->arrays.size(); ++a) {
    const ArrayState& s = p->arrays[a];
    if (!s.active || n_time[a] == 0) continue;
    if (s.own_launch || !xeng::batch::supports(s.d.n_inputs) || s.k != xeng::x16_kernel(s.d.n_inputs)) {
      others.push_back(a);
      continue;
    }
    BatchEntry b{};
    b.a = a;
    b.ngroups = (s.d.n_chans + s.k->cpw - 1) / s.k->cpw;
    total += (double)b.ngroups * (n_time[a] * cycles_per_sample(s.k, s.d.n_inputs) + ITEM_START_CYCLES);
    items.push_back(b);
  }
  const double target = total / ((double)std::max(1, p->batch_split) * p->n_cu);
  for (BatchEntry& b : items) {
    const ArrayState& s = p->arrays[b.a];
    const int64_t T = n_time[b.a];
    const double full = T * cycles_per_sample(s.k, s.d.n_inputs);
    int64_t nc = (int64_t)std::ceil(full / std::max(target, 1.0));
    nc = std::max<int64_t>(1, std::min<int64_t>(nc, T / 256));
    nc = std::max<int64_t>(nc, (T + s.k->max_t_per_wg - 1) / s.k->max_t_per_wg);
    int64_t tc = (T + nc - 1) / nc;
    tc = (tc + xeng::KS - 1) / xeng::KS * xeng::KS;
    b.t_chunk = tc;
    b.nchunks = (int32_t)((T + tc - 1) / tc);
    b.item_cycles = tc * cycles_per_sample(s.k, s.d.n_inputs) + ITEM_START_CYCLES;
  }
  std::stable_sort(items.begin(), items.end(),
                   [](const BatchEntry& x, const BatchEntry& y) { return x.item_cycles > y.item_cycles; });
  // arrays that start an integration with atomic adds need zeroed memory
  std::vector<ArrayState*> to_zero;
  for (const BatchEntry& b : items) {
    ArrayState& s = p->arrays[b.a];
    if (b.nchunks > 1 && s.clean && !s.zeroed) to_zero.push_back(&s);
  }
  if (!to_zero.empty()) {
    const int st = zero_fill(p, to_zero);
    if (st != XENG_OK) return st;
  }
  for (size_t first = 0; first < items.size(); first += xeng::batch::MAX_ARRAYS) {
    xeng::batch::Params bp{};
    bp.counters = p->counters;
    int64_t n_items = 0;
    const size_t last = std::min(items.size(), first + xeng::batch::MAX_ARRAYS);
    for (size_t i = first; i < last; ++i) {
      const BatchEntry& b = items[i];
      const ArrayState& s = p->arrays[b.a];
      const int k = bp.n_arrays++;
      bp.arr[k] = base_args(s, v[b.a], n_time[b.a]);
      bp.arr[k].t_chunk = b.t_chunk;
      bp.arr[k].mode = b.nchunks > 1 ? xeng::EPI_ATOMIC : (s.clean ? xeng::EPI_STORE : xeng::EPI_ADD);
      bp.ngroups[k] = b.ngroups;
      bp.nchunks[k] = b.nchunks;
      n_items += (int64_t)b.ngroups * b.nchunks;
    }
    const int grid = (int)std::min<int64_t>(p->n_cu, n_items);
    ++p->stats.launches;
    if (p->trace)
      fprintf(stderr, "xeng: plan %p batch launch arrays=%d items=%lld grid=%d\n", (void*)p, bp.n_arrays,
              (long long)n_items, grid);
    hipError_t e = xeng::batch::launch(grid, p->stream, bp);
    if (e != hipSuccess) return hip_fail(p, e, "batch kernel launch");
  }
  for (int32_t a : others) {
    const int st = launch_plain(p, p->arrays[a], v[a], n_time[a]);
    if (st != XENG_OK) return st;
  }
  return XENG_OK;
}

// Record the batched call into a graph on the plan's stream (stream capture),
// then launch it.  Instantiated graphs are kept in a ring and updated in place
// for later calls (hipGraphExecUpdate; a fresh instantiation if the update is
// refused); a graph is updated only after its previous launch has completed,
// so a launch in flight never sees new parameters.
int run_batched(xeng_plan_t* p, const uint8_t* const* v, const int64_t* n_time) {
  bool any = false;
  for (int32_t a = 0; a < (int32_t)p->arrays.size(); ++a) any = any || (p->arrays[a].active && n_time[a] > 0);
  if (!any) return XENG_OK;  // nothing to launch
  const int slot = p->next_graph;
  p->next_graph = (slot + 1) % xeng_plan_s::GRAPH_RING;
  hipError_t e;
  if (!p->done[slot]) {
    e = hipEventCreateWithFlags(&p->done[slot], hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(p, e, "graph event");
  } else {
    e = hipEventSynchronize(p->done[slot]);
    if (e != hipSuccess) return hip_fail(p, e, "graph event wait");
  }
  e = hipStreamBeginCapture(p->stream, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return hip_fail(p, e, "begin capture");
  const int st = record_batched(p, v, n_time);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(p->stream, &graph);
  if (st != XENG_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return hip_fail(p, e, "end capture");
  if (p->exec[slot]) {
    hipGraphNode_t err_node = nullptr;
    hipGraphExecUpdateResult res;
    if (hipGraphExecUpdate(p->exec[slot], graph, &err_node, &res) != hipSuccess ||
        res != hipGraphExecUpdateSuccess) {
      (void)hipGetLastError();
      (void)hipGraphExecDestroy(p->exec[slot]);
      p->exec[slot] = nullptr;
    }
  }
  if (!p->exec[slot]) {
    e = hipGraphInstantiate(&p->exec[slot], graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      p->exec[slot] = nullptr;
      (void)hipGraphDestroy(graph);
      return hip_fail(p, e, "graph instantiate");
    }
  }
  (void)hipGraphDestroy(graph);
  e = hipGraphLaunch(p->exec[slot], p->stream);
  if (e != hipSuccess) return hip_fail(p, e, "graph launch");
  e = hipEventRecord(p->done[slot], p->stream);
  if (e != hipSuccess) return hip_fail(p, e, "graph event record");
  return XENG_OK;
}

int zero_accumulators(xeng_plan_t* p) {
  for (ArrayState& s : p->arrays) {
    if (!s.active) continue;
    hipError_t e = hipMemsetAsync(s.acc, 0, s.acc_bytes, p->stream);
    if (e != hipSuccess) return hip_fail(p, e, "accumulator clear");
    s.clean = s.zeroed = true;
    s.n_integrated = 0;
  }
  return XENG_OK;
}

int validate_call(xeng_plan_t* p, const uint8_t* const* d_voltages, const int64_t* n_time) {
  for (int32_t a = 0; a < (int32_t)p->arrays.size(); ++a) {
    const ArrayState& s = p->arrays[a];
    const int64_t T = n_time[a];
    if (!s.active) {
      if (T != 0) return fail(p, XENG_EINVAL, "slot %d holds no array but n_time is %lld", a, (long long)T);
      continue;
    }
    if (T < 0 || T > s.d.max_time_per_call)
      return fail(p, XENG_EINVAL, "array %d: n_time %lld outside [0, %lld]", a, (long long)T,
                  (long long)s.d.max_time_per_call);
    if (T > 0 && (!d_voltages || !d_voltages[a] || !aligned16(d_voltages[a])))
      return fail(p, XENG_EINVAL, "array %d: voltage pointer null or not 16-byte aligned", a);
    if (s.n_integrated + T > XENG_MAX_INTEGRATION)
      return fail(p, XENG_EOVERFLOW, "array %d: %lld + %lld samples exceed %lld", a,
                  (long long)s.n_integrated, (long long)T, (long long)XENG_MAX_INTEGRATION);
  }
  return XENG_OK;
}

int correlate_unchecked(xeng_plan_t* p, const uint8_t* const* d_voltages, const int64_t* n_time) {
  if (p->batched) {
    const int st = run_batched(p, d_voltages, n_time);
    if (st != XENG_OK) return st;
  } else {
    for (int32_t a = 0; a < (int32_t)p->arrays.size(); ++a) {
      if (!p->arrays[a].active || n_time[a] == 0) continue;
      const int st = launch_plain(p, p->arrays[a], d_voltages[a], n_time[a]);
      if (st != XENG_OK) return st;
    }
  }
  ++p->stats.calls;
  for (int32_t a = 0; a < (int32_t)p->arrays.size(); ++a) {
    ArrayState& s = p->arrays[a];
    if (!s.active || n_time[a] == 0) continue;
    s.n_integrated += n_time[a];
    s.clean = s.zeroed = false;
    p->stats.samples += n_time[a];
    p->stats.cmacs += n_time[a] * (int64_t)s.d.n_chans * nbl_of(s.d.n_inputs);
    p->stats.bytes_in += n_time[a] * (int64_t)s.d.n_chans * s.d.n_inputs;
  }
  return XENG_OK;
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
  if (!p || array < 0 || array >= (int32_t)p->arrays.size() || !p->arrays[array].active) return -1;
  return p->arrays[array].n_integrated;
}

int32_t xeng_slots(const xeng_plan_t* p) { return p ? (int32_t)p->arrays.size() : -1; }

int64_t xeng_accumulator_bytes(int32_t n_inputs, int32_t n_chans) {
  if (n_inputs < 1 || n_chans < 1) return -1;
  return (int64_t)n_chans * nbl_of(n_inputs) * 2 * (int64_t)sizeof(int32_t);
}

int xeng_plan(xeng_plan_t** out, const xeng_array_desc* arrays, int32_t n_arrays, uint32_t flags,
              void* hip_stream) {
  if (!out || n_arrays < 0 || (n_arrays > 0 && !arrays) || (flags & ~(uint32_t)XENG_PLAN_BATCH))
    return XENG_EINVAL;
  if (n_arrays == 0 && !(flags & XENG_PLAN_BATCH)) return XENG_EINVAL;
  *out = nullptr;
  for (int32_t a = 0; a < n_arrays; ++a)
    if (!valid_desc(arrays[a])) return XENG_EINVAL;
  xeng_plan_t* p = new (std::nothrow) xeng_plan_t();
  if (!p) return XENG_ENOMEM;
  p->batched = n_arrays > 1 || (flags & XENG_PLAN_BATCH);
  {
    const char* t = getenv("XENG_TRACE");
    p->trace = t && *t && strcmp(t, "0") != 0;
  }
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    delete p;
    return XENG_EDEVICE;
  }
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p->device) == hipSuccess &&
      ncu > 0)
    p->n_cu = ncu;
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) {
      p->arch = prop.gcnArchName;
      const size_t colon = p->arch.find(':');
      if (colon != std::string::npos) p->arch.resize(colon);
    }
  }
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
  if (p->batched) {
    const size_t cbytes = (xeng::batch::QUEUES + 1) * sizeof(int32_t);
    e = hipMalloc(&p->counters, cbytes);
    if (e == hipSuccess) e = hipMemsetAsync(p->counters, 0, cbytes, p->stream);
    if (e != hipSuccess) {
      xeng_destroy(p);
      return e == hipErrorOutOfMemory ? XENG_ENOMEM : XENG_EDEVICE;
    }
  }
  p->arrays.resize(n_arrays);
  for (int32_t a = 0; a < n_arrays; ++a) {
    const int st = init_slot(p, p->arrays[a], arrays[a]);
    if (st != XENG_OK) {
      xeng_destroy(p);
      return st;
    }
  }
  if (p->batched) apply_cached_plan(p, n_arrays);
  *out = p;
  return XENG_OK;
}

int xeng_attach(xeng_plan_t* p, const xeng_array_desc* d, int32_t* index) {
  if (!p || !d || !index) return XENG_EINVAL;
  if (p->dead) return XENG_ESTATE;
  if (!p->batched) return fail(p, XENG_EINVAL, "attach needs a batched plan");
  if (!valid_desc(*d)) return fail(p, XENG_EINVAL, "bad array descriptor");
  int32_t slot = 0;
  while (slot < (int32_t)p->arrays.size() && p->arrays[slot].active) ++slot;
  if (slot == (int32_t)p->arrays.size()) p->arrays.emplace_back();
  const int st = init_slot(p, p->arrays[slot], *d);
  if (st != XENG_OK) {
    if (p->arrays[slot].acc) (void)hipFree(p->arrays[slot].acc);
    p->arrays[slot] = ArrayState{};
    return st;
  }
  *index = slot;
  return XENG_OK;
}

int xeng_detach(xeng_plan_t* p, int32_t index) {
  if (!p) return XENG_EINVAL;
  if (p->dead) return XENG_ESTATE;
  if (index < 0 || index >= (int32_t)p->arrays.size() || !p->arrays[index].active)
    return fail(p, XENG_EINVAL, "slot %d holds no array", index);
  hipError_t e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return hip_fail(p, e, "detach synchronize");
  e = hipFree(p->arrays[index].acc);
  p->arrays[index] = ArrayState{};
  if (e != hipSuccess) return hip_fail(p, e, "accumulator free");
  return XENG_OK;
}

int xeng_correlate(xeng_plan_t* p, const uint8_t* const* d_voltages, const int64_t* n_time) {
  if (!p || !n_time) return XENG_EINVAL;
  if (p->dead) return XENG_ESTATE;
  const int st = validate_call(p, d_voltages, n_time);
  if (st != XENG_OK) return st;
  return correlate_unchecked(p, d_voltages, n_time);
}

int xeng_correlate_dump(xeng_plan_t* p, const uint8_t* const* d_voltages, const int64_t* n_time,
                        int32_t* const* d_dst, int64_t* n_integrated) {
  if (!p || !n_time || !d_dst) return XENG_EINVAL;
  if (p->dead) return XENG_ESTATE;
  int st = validate_call(p, d_voltages, n_time);
  if (st != XENG_OK) return st;
  const int32_t na = (int32_t)p->arrays.size();
  for (int32_t a = 0; a < na; ++a) {
    if (!p->arrays[a].active || !d_dst[a]) continue;
    if ((reinterpret_cast<uintptr_t>(d_dst[a]) & 7u) != 0)
      return fail(p, XENG_EINVAL, "array %d: destination not 8-byte aligned", a);
    hipPointerAttribute_t attr{};
    if (hipPointerGetAttributes(&attr, d_dst[a]) != hipSuccess || attr.type != hipMemoryTypeDevice) {
      (void)hipGetLastError();
      return fail(p, XENG_EINVAL, "array %d: destination is not device memory", a);
    }
  }
  // Arrays dumped without new samples: a plain dump each.
  for (int32_t a = 0; a < na; ++a) {
    if (!p->arrays[a].active || !d_dst[a] || n_time[a] != 0) continue;
    int32_t* dst[1] = {d_dst[a]};
    st = xeng_dump(p, a, dst, 0, n_integrated ? n_integrated + a : nullptr);
    if (st != XENG_OK) return st;
  }
  // The others integrate straight into their destination: an empty
  // integration starts there from nothing (plain stores, or atomic adds into
  // zeroed memory); earlier samples are copied over first and added to.
  struct Saved {
    int32_t a;
    int32_t* acc;
    bool clean, zeroed;
    int64_t n;
  };
  std::vector<Saved> redirected;
  xeng::DumpParams dp{};
  int64_t most = 0;
  auto flush = [&]() -> int {
    if (dp.count == 0) return XENG_OK;
    const int64_t blocks = std::min<int64_t>((most + 1023) / 1024, 8LL * p->n_cu);
    hipError_t e = xeng::dump_launch((int)std::max<int64_t>(1, blocks), p->stream, dp);
    dp.count = 0;
    most = 0;
    return e == hipSuccess ? XENG_OK : hip_fail(p, e, "carry-over copy");
  };
  for (int32_t a = 0; a < na; ++a) {
    ArrayState& s = p->arrays[a];
    if (!s.active || !d_dst[a] || n_time[a] == 0) continue;
    redirected.push_back(Saved{a, s.acc, s.clean, s.zeroed, s.n_integrated});
    if (!s.clean) {
      dp.acc[dp.count] = reinterpret_cast<const int2*>(s.acc);
      dp.dst[dp.count] = reinterpret_cast<int2*>(d_dst[a]);
      dp.n[dp.count] = (int64_t)(s.acc_bytes / sizeof(int2));
      most = std::max(most, dp.n[dp.count]);
      if (++dp.count == xeng::DUMP_MAX) {
        st = flush();
        if (st != XENG_OK) return st;
      }
    }
  }
  st = flush();
  if (st != XENG_OK) return st;
  for (const Saved& r : redirected) {
    ArrayState& s = p->arrays[r.a];
    s.acc = d_dst[r.a];
    s.zeroed = false;  // clean (empty) destinations hold unknown values
  }
  st = correlate_unchecked(p, d_voltages, n_time);
  for (const Saved& r : redirected) {
    ArrayState& s = p->arrays[r.a];
    s.acc = r.acc;
    if (st != XENG_OK) {
      s.clean = r.clean;
      s.zeroed = r.zeroed;
      s.n_integrated = r.n;
      continue;
    }
    if (n_integrated) n_integrated[r.a] = r.n + n_time[r.a];
    ++p->stats.dumps;
    p->stats.bytes_out += (int64_t)s.acc_bytes;
    // the integration restarts; an accumulator that was empty was not written
    s.n_integrated = 0;
    s.clean = true;
    s.zeroed = r.clean && r.zeroed;
  }
  return st;
}

int xeng_autotune(xeng_plan_t* p, const uint8_t* const* d_voltages, const int64_t* n_time,
                  int32_t reps, float* best_ms) {
  if (!p || !n_time || reps < 1) return XENG_EINVAL;
  if (p->dead) return XENG_ESTATE;
  for (const ArrayState& s : p->arrays)
    if (s.active && s.n_integrated != 0)
      return fail(p, XENG_EINVAL, "autotune needs every accumulator freshly dumped");
  int st = validate_call(p, d_voltages, n_time);
  if (st != XENG_OK) return st;

  hipEvent_t t0, t1;
  if (hipEventCreate(&t0) != hipSuccess) return fail(p, XENG_EDEVICE, "event");
  if (hipEventCreate(&t1) != hipSuccess) {
    (void)hipEventDestroy(t0);
    return fail(p, XENG_EDEVICE, "event");
  }
  // one trial: reps calls from clean accumulators, timed on the stream
  auto trial = [&](float& ms) -> int {
    int r = zero_accumulators(p);
    if (r != XENG_OK) return r;
    r = correlate_unchecked(p, d_voltages, n_time);  // warm-up (also builds the graph)
    if (r != XENG_OK) return r;
    if (hipEventRecord(t0, p->stream) != hipSuccess) return fail(p, XENG_EDEVICE, "event record");
    // (the sums of these calls are thrown away, so the overflow guard is not applied)
    for (int i = 0; i < reps && r == XENG_OK; ++i) r = correlate_unchecked(p, d_voltages, n_time);
    if (r != XENG_OK) return r;
    if (hipEventRecord(t1, p->stream) != hipSuccess || hipEventSynchronize(t1) != hipSuccess)
      return fail(p, XENG_EDEVICE, "event wait");
    return hipEventElapsedTime(&ms, t0, t1) == hipSuccess ? XENG_OK : fail(p, XENG_EDEVICE, "timing");
  };

  float best = 0;
  if (p->batched) {
    // work-item granularity of the persistent launch
    const int cand[] = {1, 2, 4, 8};
    int pick = p->batch_split;
    for (int i = 0; i < 4 && st == XENG_OK; ++i) {
      p->batch_split = cand[i];
      float ms = 0;
      st = trial(ms);
      if (st == XENG_OK && (best == 0 || ms < best)) {
        best = ms;
        pick = cand[i];
      }
    }
    p->batch_split = pick;
    // Per array, largest work first: items of the persistent launch (16-row
    // tiles), or a plain launch of its own inside the same graph with the
    // tile shape and time split that suit it best; kept when the whole call
    // gets faster by more than 1%.
    std::vector<int32_t> order;
    for (int32_t a = 0; a < (int32_t)p->arrays.size(); ++a)
      if (p->arrays[a].active && n_time[a] > 0) order.push_back(a);
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
      const ArrayState &sx = p->arrays[x], &sy = p->arrays[y];
      return n_time[x] * sx.d.n_chans * nbl_of(sx.d.n_inputs) > n_time[y] * sy.d.n_chans * nbl_of(sy.d.n_inputs);
    });
    for (int32_t a : order) {
      if (st != XENG_OK) break;
      ArrayState& s = p->arrays[a];
      const ArrayState keep = s;
      ArrayState choice = s;
      for (int kind : {KIND_X16, KIND_X32, KIND_STAGE}) {
        const KernelInfo* k = kernel_of(kind, s.d.n_inputs);
        if (!kernel_fits(k, s.d) || (kind != KIND_STAGE && s.d.n_inputs % 16 != 0)) continue;
        for (int split : {1, 2}) {
          s.k = k;
          s.split = split;
          s.own_launch = true;
          float ms = 0;
          st = trial(ms);
          if (st != XENG_OK) break;
          if (ms < 0.99f * best) {
            best = ms;
            choice = s;
          }
        }
        if (st != XENG_OK) break;
      }
      const bool own = choice.own_launch;
      s = keep;
      if (own) {
        s.k = choice.k;
        s.split = choice.split;
        s.own_launch = true;
      }
    }
    for (int32_t a : order) record_choice(p, p->arrays[a], n_time[a]);
    {
      std::lock_guard<std::mutex> lock(g_tune_mu);
      g_tune[plan_key(p, (int32_t)p->arrays.size())] = TuneVal{KIND_X16, p->batch_split, 0};
    }
  } else {
    // per array: tile shape (32-row tiles of the ring kernel or 16-row tiles
    // of the staging kernel) and workgroups per CU of the time split
    for (ArrayState& s : p->arrays) {
      if (!s.active) continue;
      std::vector<const KernelInfo*> kernels;
      if (s.d.n_inputs % 16 == 0) {
        if (kernel_fits(xeng::x16_kernel(s.d.n_inputs), s.d)) kernels.push_back(xeng::x16_kernel(s.d.n_inputs));
        kernels.push_back(xeng::x32_kernel(s.d.n_inputs));
      }
      kernels.push_back(xeng::stage_kernel((s.d.n_inputs + 15) / 16));
      const KernelInfo* pick_k = s.k;
      int pick_split = s.split;
      float arr_best = 0;
      for (const KernelInfo* k : kernels) {
        if (!k) continue;
        for (int split : {1, 2, 4}) {
          s.k = k;
          s.split = split;
          float ms = 0;
          st = trial(ms);
          if (st != XENG_OK) break;
          if (arr_best == 0 || ms < arr_best) {
            arr_best = ms;
            pick_k = k;
            pick_split = split;
          }
        }
        if (st != XENG_OK) break;
      }
      s.k = pick_k;
      s.split = pick_split;
      best += arr_best;
      if (st != XENG_OK) break;
      if (n_time[&s - &p->arrays[0]] > 0) record_choice(p, s, n_time[&s - &p->arrays[0]]);
    }
  }
  const int z = zero_accumulators(p);
  if (st == XENG_OK) st = z;
  if (st == XENG_OK && hipStreamSynchronize(p->stream) != hipSuccess) st = fail(p, XENG_EDEVICE, "sync");
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (st == XENG_OK && best_ms) *best_ms = best / (float)reps;
  return st;
}

int xeng_tune_cache_save(const char* path) {
  if (!path) return XENG_EINVAL;
  FILE* f = fopen(path, "w");
  if (!f) return XENG_EINVAL;
  fprintf(f, "# xeng tuning cache: arch batched N log2F log2T kernel(0=16-row,1=32-row,2=staging) split own\n");
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    for (const auto& kv : g_tune)
      fprintf(f, "%s %d %d %d %d %d %d %d\n", kv.first.arch.c_str(), kv.first.batched, kv.first.n, kv.first.fb,
              kv.first.tb, kv.second.kind, kv.second.split, kv.second.own);
  }
  return fclose(f) == 0 ? XENG_OK : XENG_EINVAL;
}

int xeng_tune_cache_load(const char* path) {
  if (!path) return XENG_EINVAL;
  FILE* f = fopen(path, "r");
  if (!f) return XENG_EINVAL;
  char line[512];
  int st = XENG_OK;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  while (fgets(line, sizeof line, f)) {
    if (line[0] == '#' || line[0] == '\n') continue;
    char arch[128];
    int b, n, fb, tb, kind, split, own;
    if (sscanf(line, "%127s %d %d %d %d %d %d %d", arch, &b, &n, &fb, &tb, &kind, &split, &own) != 8 ||
        n < 0 || n > XENG_MAX_INPUTS || (n == 0 && !b) || kind < KIND_X16 || kind > KIND_STAGE || split < 1 ||
        split > 64) {
      st = XENG_EINVAL;  // malformed line: skipped, reported
      continue;
    }
    g_tune[TuneKey{arch, b ? 1 : 0, n, fb, tb}] = TuneVal{kind, split, own ? 1 : 0};
  }
  fclose(f);
  return st;
}

int xeng_tune_cache_clear(void) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune.clear();
  return XENG_OK;
}

int xeng_dump(xeng_plan_t* p, int32_t array, int32_t* const* dst, uint32_t flags,
              int64_t* n_integrated) {
  if (!p || !dst) return XENG_EINVAL;
  if (p->dead) return XENG_ESTATE;
  if (flags & ~(uint32_t)(XENG_DUMP_KEEP | XENG_DUMP_TO_HOST)) return XENG_EINVAL;
  const int32_t na = (int32_t)p->arrays.size();
  if (array < -1 || array >= na) return fail(p, XENG_EINVAL, "array index %d out of range", array);
  if (array >= 0 && !p->arrays[array].active) return fail(p, XENG_EINVAL, "slot %d holds no array", array);
  const int32_t a0 = array < 0 ? 0 : array, a1 = array < 0 ? na : array + 1;
  for (int32_t a = a0; a < a1; ++a)
    if (p->arrays[a].active && !dst[a - a0])
      return fail(p, XENG_EINVAL, "dump destination %d is null", a - a0);
  const bool to_host = (flags & XENG_DUMP_TO_HOST) != 0;
  const bool keep = (flags & XENG_DUMP_KEEP) != 0;
  // An empty integration whose memory still holds an earlier dump's sums
  // (clean, not zeroed) is dumped as zeros.  Without KEEP the accumulator is
  // not cleared here: it is marked empty, and the next launch overwrites it.
  xeng::DumpParams dp{};
  int64_t most = 0;
  auto flush = [&]() -> int {
    if (dp.count == 0) return XENG_OK;
    const int64_t blocks = std::min<int64_t>((most + 1023) / 1024, 8LL * p->n_cu);
    hipError_t e = xeng::dump_launch((int)std::max<int64_t>(1, blocks), p->stream, dp);
    dp.count = 0;
    most = 0;
    return e == hipSuccess ? XENG_OK : hip_fail(p, e, "dump kernel");
  };
  for (int32_t a = a0; a < a1; ++a) {
    ArrayState& s = p->arrays[a];
    if (!s.active) continue;
    int32_t* d = dst[a - a0];
    const bool stale = s.clean && !s.zeroed;
    if (!to_host && (reinterpret_cast<uintptr_t>(d) & 7u) == 0) {
      // device destination: one dump kernel copies every array
      dp.acc[dp.count] = stale ? nullptr : reinterpret_cast<const int2*>(s.acc);
      dp.dst[dp.count] = reinterpret_cast<int2*>(d);
      dp.n[dp.count] = (int64_t)(s.acc_bytes / sizeof(int2));
      most = std::max(most, dp.n[dp.count]);
      if (++dp.count == xeng::DUMP_MAX) {
        const int st = flush();
        if (st != XENG_OK) return st;
      }
    } else {
      if (stale) {
        const int st = zero_fill(p, {&s});
        if (st != XENG_OK) return st;
      }
      hipError_t e = hipMemcpyAsync(d, s.acc, s.acc_bytes,
                                    to_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, p->stream);
      if (e != hipSuccess) return hip_fail(p, e, "dump copy");
    }
    if (n_integrated) n_integrated[a - a0] = s.n_integrated;
    ++p->stats.dumps;
    p->stats.bytes_out += (int64_t)s.acc_bytes;
    if (!keep) {
      s.n_integrated = 0;
      s.clean = true;
    }
  }
  const int st = flush();
  if (st != XENG_OK) return st;
  if (to_host) {
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(p, e, "dump synchronize");
  }
  return XENG_OK;
}

int xeng_stats(const xeng_plan_t* p, xeng_stats_t* out) {
  if (!p || !out) return XENG_EINVAL;
  *out = p->stats;
  return XENG_OK;
}

int xeng_load_acc(xeng_plan_t* p, int32_t array, const int32_t* src, int64_t n_integrated) {
  if (!p || !src) return XENG_EINVAL;
  if (p->dead) return XENG_ESTATE;
  if (array < 0 || array >= (int32_t)p->arrays.size() || !p->arrays[array].active)
    return fail(p, XENG_EINVAL, "slot %d holds no array", array);
  if (n_integrated < 0 || n_integrated > XENG_MAX_INTEGRATION)
    return fail(p, XENG_EINVAL, "n_integrated %lld outside [0, %lld]", (long long)n_integrated,
                (long long)XENG_MAX_INTEGRATION);
  ArrayState& s = p->arrays[array];
  hipError_t e = hipMemcpyAsync(s.acc, src, s.acc_bytes, hipMemcpyDefault, p->stream);
  if (e != hipSuccess) return hip_fail(p, e, "accumulator load");
  s.n_integrated = n_integrated;
  s.clean = false;   // the next launch adds to the loaded sums
  s.zeroed = false;
  return XENG_OK;
}

void xeng_destroy(xeng_plan_t* p) {
  if (!p) return;
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  for (int i = 0; i < xeng_plan_s::GRAPH_RING; ++i) {
    if (p->exec[i]) (void)hipGraphExecDestroy(p->exec[i]);
    if (p->done[i]) (void)hipEventDestroy(p->done[i]);
  }
  for (ArrayState& s : p->arrays)
    if (s.acc) (void)hipFree(s.acc);
  if (p->counters) (void)hipFree(p->counters);
  if (p->own_stream && p->stream) (void)hipStreamDestroy(p->stream);
  delete p;
}

}  // extern "C"
