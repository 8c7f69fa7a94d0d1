// C ABI of libsnn: argument checks, device memory, and the orchestration of
// Algorithm 1 (snn_index) and Algorithm 2 (snn_query / snn_query_self) as a
// chain of kernels on the caller's stream with a single host read-back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "query_plan.h"
#include "snn_internal.h"
#include "snn_testing.h"

namespace snn {

void launch_self_qnorm(const float* ynorm, int64_t n, double* out, hipStream_t s);

namespace {
thread_local std::string g_err;
}

void fail(snn_status code, const std::string& msg) { throw Error(code, msg); }

// SNN_FAULT_INJECT=n (tests): the n-th checked HIP result of an entry
// point's call reads as a failure (the call itself was made), so that every
// error path can be driven from the host; set per call by DeviceScope.
thread_local long t_fault_countdown = 0;

void check_hip(hipError_t e, const char* what, const char* file, int line) {
  char buf[512];
  if (t_fault_countdown > 0 && --t_fault_countdown == 0) {
    std::snprintf(buf, sizeof(buf), "injected HIP failure (SNN_FAULT_INJECT) in %s at %s:%d", what, file, line);
    throw Error(SNN_EDEVICE, buf);
  }
  if (e == hipSuccess) return;
  std::snprintf(buf, sizeof(buf), "HIP error %d (%s) in %s at %s:%d", (int)e, hipGetErrorString(e), what, file,
                line);
  throw Error(e == hipErrorOutOfMemory ? SNN_ENOMEM : SNN_EDEVICE, buf);
}

void* DeviceArena::alloc(size_t bytes) {
  if (bytes == 0) bytes = 256;
  void* p = nullptr;
  if (dev_.alloc) {
    p = dev_.alloc(dev_.ctx, bytes);
    if (!p) fail(SNN_ENOMEM, "device allocator returned NULL for " + std::to_string(bytes) + " bytes");
  } else {
    hipError_t e = hipMalloc(&p, bytes);
    if (e == hipErrorOutOfMemory) {
      (void)hipGetLastError();
      fail(SNN_ENOMEM, "hipMalloc failed for " + std::to_string(bytes) + " bytes");
    }
    SNN_HIP(e);
  }
  return p;
}

void DeviceArena::release(void* p) {
  if (!p) return;
  if (dev_.free)
    dev_.free(dev_.ctx, p);
  else
    (void)hipFree(p);
}

void Buffer::ensure(DeviceArena& a, size_t need) {
  if (need <= bytes && ptr) return;
  reset(a);
  ptr = a.alloc(need);
  bytes = need;
  log_line(3, "workspace buffer of %zu bytes", need);
}

void Buffer::reset(DeviceArena& a) {
  if (ptr && !view) a.release(ptr);
  ptr = nullptr;
  bytes = 0;
  view = false;
}

const DeviceInfo& device_info(int device) {
  static std::mutex mu;
  static std::vector<DeviceInfo> cache;
  static std::vector<bool> have;
  std::lock_guard<std::mutex> lk(mu);
  if ((int)cache.size() <= device) {
    cache.resize(device + 1);
    have.resize(device + 1, false);
  }
  if (!have[device]) {
    int cus = 0;
    SNN_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
    cache[device].cus = cus > 0 ? cus : 1;
    cache[device].xcds = cus >= 64 ? 8 : 1;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
      cache[device].lds_bytes = lds;
    else
      (void)hipGetLastError();
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
      cache[device].clock_khz = khz;
    else
      (void)hipGetLastError();
    have[device] = true;
  }
  return cache[device];
}

// Select the device of `dev` for the duration of a call, check it is gfx950.
DeviceScope::DeviceScope(int device) {
  {
    const char* f = std::getenv("SNN_FAULT_INJECT");
    t_fault_countdown = f && *f ? std::atol(f) : 0;
  }
  // device count and architecture are checked once per process and device
  // (every call passes through here; each HIP query costs the host time on
  // the call's critical path)
  static std::atomic<int> count{-1};
  static std::atomic<int> ok[64];
  int c = count.load(std::memory_order_acquire);
  if (c < 0) {
    hipError_t e = hipGetDeviceCount(&c);
    if (e != hipSuccess || c <= 0) {
      (void)hipGetLastError();
      fail(SNN_EDEVICE, "no HIP device available");
    }
    count.store(c, std::memory_order_release);
  }
  if (device < 0 || device >= c) fail(SNN_EINVAL, "device ordinal out of range");
  if (device >= 64) fail(SNN_ENOTSUP, "device ordinals above 63 are not supported");
  int v = ok[device].load(std::memory_order_acquire);  // 0 unknown, 1 gfx950, 2 other
  if (v == 0) {
    hipDeviceProp_t p;
    SNN_HIP(hipGetDeviceProperties(&p, device));
    v = std::strncmp(p.gcnArchName, "gfx950", 6) == 0 ? 1 : 2;
    ok[device].store(v, std::memory_order_release);
  }
  if (v != 1) fail(SNN_EDEVICE, "device is not gfx950 (this library is built for MI355X only)");
  int cur = -1;
  SNN_HIP(hipGetDevice(&cur));
  if (cur != device) {
    SNN_HIP(hipSetDevice(device));
    prev = cur;
  }
}

DeviceScope::~DeviceScope() {
  if (prev >= 0) (void)hipSetDevice(prev);
}

void set_last_error(const std::string& msg) { g_err = msg; }

void* pinned_host(size_t bytes) {
  thread_local void* p = nullptr;
  thread_local size_t cap = 0;
  if (bytes > cap) {
    // (a call that failed between its copies and their wait can leave one
    // in flight into the old block)
    if (p) {
      (void)hipDeviceSynchronize();
      (void)hipHostFree(p);
    }
    p = nullptr;
    cap = 0;
    const size_t want = std::max<size_t>(bytes, 64 * 1024);
    SNN_HIP(hipHostMalloc(&p, want, hipHostMallocDefault));
    cap = want;
  }
  return p;
}

static int env_int(const char* name) {
  const char* v = std::getenv(name);
  return v && *v ? std::atoi(v) : 0;
}

int log_level() { return std::min(3, std::max(0, env_int("SNN_LOG"))); }

bool profile_on() { return env_int("SNN_PROFILE") != 0; }

void log_line(int level, const char* fmt, ...) {
  if (level > log_level()) return;
  char buf[640];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  std::fprintf(stderr, "[snn] %s\n", buf);
}

void report_failure(snn_status code, const std::string& msg) {
  set_last_error(msg);
  static const char* const names[] = {"OK", "EINVAL", "ENOMEM", "EDEVICE", "EOVERFLOW", "ENOTSUP"};
  const int k = -(int)code;
  log_line(1, "failed: SNN_%s: %s", k >= 0 && k <= 5 ? names[k] : "?", msg.c_str());
}

namespace {

constexpr double kU64 = 1.1102230246251565e-16;  // 2^-53

double gamma64(int k) { return k * kU64 / (1.0 - k * kU64); }

// Control block read back once per query.
struct Ctl {
  unsigned long long counters[kMaxXcd];
  unsigned long long survivors;
  unsigned long long pairs_window;
  unsigned long long list_counts[8];
  unsigned long long row_max;
  unsigned long long executed;
  unsigned long long accepted;  // neighbour entries (clustering mode)
  unsigned long long nnz;       // neighbour entries (lists mode)
  unsigned long long screen_mark[2];  // device clock marks of the screen launch (QueryDev::stamps)
  unsigned long long call_mark[2];    // device clock at the call's first kernel and after its last
  int bad;
  int scan_err;  // a look-back scan's wait did not end (not expected)
};

struct HostCtl {
  Ctl ctl;
  int64_t nnz;
};

// Device time of the call from its clock marks.
double call_ms_of(const Ctl& c, const DeviceInfo& di) {
  if (di.clock_khz <= 0 || c.call_mark[1] < c.call_mark[0]) return 0.0;
  return (double)(c.call_mark[1] - c.call_mark[0]) / di.clock_khz;
}

// Duration of the screen launch from its clock marks (0 without a launch).
double screen_ms_of(const Ctl& c, const DeviceInfo& di) {
  const unsigned long long t0 = ~c.screen_mark[0], t1 = c.screen_mark[1];
  if (c.screen_mark[1] == 0 || t1 < t0 || di.clock_khz <= 0) return 0.0;
  return (double)(t1 - t0) / di.clock_khz;
}


}  // namespace

// ------------------------------------------------------------------------ query
static void build_fp32_operands(Index& ix) {
  if (ix.vcand_built) return;
  ix.vcand.ensure(ix.arena, sizeof(float) * mfma32_operand_floats(ix.n, ix.d) + 256);
  launch_mfma32_operands(ix.ys.as<float>(), ix.n, ix.d, ix.vcand.as<float>(), ix.arena.stream());
  ix.vcand_built = true;
}

// The screen a query runs.  Each matrix-core screen passes every pair whose
// decomposed distance is within about band = 2 c_rep Y^2 of R^2 (Y = max
// ||y||), so the pairs re-decided in float64 grow with band / R^2.  One
// 16-bit product per coordinate is cheapest on the matrix cores, and fp16
// (scaled rows) has a band 8x narrower than bf16 at the same rate; the bf16
// hi/lo split costs three products and narrows the band by ~2^8 more; the fp32
// screen (d <= 16) has an essentially empty band at a quarter of the rate.
struct ScreenPlan {
  snn_precision prec;  // FP64, MIXED (bf16), FP16 or FP32
  int kind;            // OperandKind of a matrix-core screen
  int terms() const { return kind == kOpBf16x3 ? 3 : ((prec == SNN_PREC_MIXED || prec == SNN_PREC_FP16) ? 1 : 0); }
};

// AUTO takes fp16 while its band is at most this fraction of R^2 (measured
// on the n = 1e6, d = 16 mixture against the bf16 hi/lo screen; see the
// design notes)
constexpr double kF16AutoBand = 1.0;

int operand_ka(int kind, int d) { return (((kind == kOpBf16x3 ? 3 : 1) * d + 15) / 16) * 16; }

static ScreenPlan plan_screen(const Index& ix, const snn_options& o, double R2) {
  const int d = ix.d;
  const double Y = ix.max_norm;
  auto fits = [&](int kind) { return operand_ka(kind, d) <= 16 * mixed_max_slices() && screen_in_range(kind, Y); };
  auto band = [&](int kind) { return R2 > 0 ? 2.0 * mixed_c_rep(kind) * Y * Y / R2 : INFINITY; };
  const bool fp32_ok = d <= mfma32_max_d() && screen_in_range(kOpF32, Y);
  ScreenPlan p{o.precision, kOpBf16};
  snn_precision want = o.precision;
  if (want == SNN_PREC_AUTO && o.mixed_terms != 0) want = SNN_PREC_MIXED;  // bf16 terms asked for
  switch (want) {
    case SNN_PREC_FP64:
      return p;
    case SNN_PREC_MIXED: {
      int t = o.mixed_terms;
      if (t == 0) t = ((fits(kOpBf16) && band(kOpBf16) <= 0.1) || !fits(kOpBf16x3)) ? 1 : 3;
      p.prec = SNN_PREC_MIXED;
      p.kind = t == 3 ? kOpBf16x3 : kOpBf16;
      if (!fits(p.kind))
        fail(SNN_ENOTSUP, "bf16 screen: packed operand rows longer than 128 values or data too large for fp32 "
                          "(lower d, use terms = 1, or FP64)");
      return p;
    }
    case SNN_PREC_FP16:
      p.kind = kOpF16;
      if (!fits(kOpF16)) fail(SNN_ENOTSUP, "fp16 screen: d > 128 or data too large to scale into fp16 (use FP64)");
      return p;
    case SNN_PREC_FP32:
      p.kind = kOpF32;
      if (!fp32_ok) fail(SNN_ENOTSUP, "fp32 screen supports d <= 16 and data within fp32 range");
      return p;
    default:
      break;
  }
  if (fits(kOpF16) && band(kOpF16) <= kF16AutoBand) return ScreenPlan{SNN_PREC_FP16, kOpF16};
  if (fits(kOpBf16x3) && band(kOpBf16x3) <= 0.5) return ScreenPlan{SNN_PREC_MIXED, kOpBf16x3};
  if (fp32_ok) return ScreenPlan{SNN_PREC_FP32, kOpF32};
  if (fits(kOpF16) && band(kOpF16) <= 2.0) return ScreenPlan{SNN_PREC_FP16, kOpF16};
  return ScreenPlan{SNN_PREC_FP64, kOpBf16};
}

// The grid over the sorted scores that confines the window searches,
// built once per set of rows.
static const int32_t* window_cells(Index& ix) {
  if (!ix.wcells_built) {
    ix.wcells_n = window_table_cells(ix.n);
    ix.wcells.ensure(ix.arena, sizeof(int32_t) * (ix.wcells_n + 1) + 256);
    launch_window_table(ix.key.as<double>(), (int)ix.n, ix.wcells_n, ix.wcells.as<int32_t>(), ix.arena.stream());
    ix.wcells_built = true;
  }
  return ix.wcells.as<int32_t>();
}

// Operands and start values of a 16-bit screen for one query call: for
// out-of-sample queries the request in *op that the gather into score order
// carries out; for a self-query the bound its own start-value pass takes
// (*self_bound).
static MixedDev prepare_mixed(Index& ix, int kind, double R2, bool self, uint16_t* qop, float* cthr,
                              QueryOperands* op, MixedBound* self_bound) {
  MixedOperands& mo = ix.mixed[mixed_slot(kind)];
  const MixedBound mb = mixed_bound(kind, mo.ka, ix.d, R2, ix.max_norm);
  MixedDev mx{};
  mx.KA = mo.ka;
  mx.KB = mo.kb;
  mx.f16 = kind == kOpF16;
  mx.cop = mo.cand.as<uint16_t>();
  mx.h = kind == kOpF16 ? mo.hs.as<float>() : ix.h.as<float>();
  mx.cthr = cthr;
  if (self) {
    mx.qop = mo.qself.as<uint16_t>();
    *self_bound = mb;
  } else {
    mx.qop = qop;
    op->mode = kQOp16;
    op->kind = kind;
    op->e = mo.e;
    op->KA = mo.ka;
    op->b = mb;
    op->qop = qop;
    op->cthr = cthr;
  }
  return mx;
}

// Query rows and start values of the fp32 screen for one query call (as
// prepare_mixed).
static void prepare_fp32(Index& ix, double R2, bool self, float* vq, QueryOperands* op, MixedBound* self_bound) {
  // K = d rounded up to the two coordinates of one fp32 matrix instruction
  const MixedBound vb = mixed_bound(kOpF32, 2 * ((ix.d + 1) / 2), ix.d, R2, ix.max_norm);
  if (self) {
    *self_bound = vb;
  } else {
    op->mode = kQOp32;
    op->DV = mfma32_query_floats(ix.d);
    op->b = vb;
    op->vq = vq;
  }
}

// The control block read back through the index's pinned host copy: a
// copy into pageable memory holds the host until the stream drains and then
// needs a further staging copy, one into pinned memory is an ordinary
// asynchronous copy that the call's synchronisation completes.
static Ctl* pinned_ctl(Index& ix) {
  if (!ix.host_ctl) SNN_HIP(hipHostMalloc(&ix.host_ctl, sizeof(Ctl), hipHostMallocDefault));
  return static_cast<Ctl*>(ix.host_ctl);
}

static uint64_t bits_of(double x) {
  uint64_t u;
  std::memcpy(&u, &x, sizeof u);
  return u;
}

// The graph slot of a call with key k: the slot that saw k before (its use
// count raised), else the least recently used slot, emptied and given k.
static QueryGraph* query_graph(Index& ix, const GraphKey& k) {
  const uint64_t now = ++ix.qgraph_clock;
  for (QueryGraph& g : ix.qgraphs)
    if (g.uses > 0 && std::memcmp(g.key.v, k.v, sizeof k.v) == 0) {
      ++g.uses;
      g.stamp = now;
      return &g;
    }
  QueryGraph* v = &ix.qgraphs[0];
  for (QueryGraph& g : ix.qgraphs)
    if (g.stamp < v->stamp) v = &g;
  destroy_query_graph(*v);
  v->key = k;
  v->uses = 1;
  v->stamp = now;
  return v;
}

// Runs body's launches on the index's stream: by replaying *g when it holds
// a graph, else by capturing them into *g and replaying that when capture
// is set, else directly.  An instantiation the runtime refuses falls back to
// the direct launches.
template <typename F>
static void run_captured(Index& ix, hipGraphExec_t* g, bool capture, F&& body) {
  hipStream_t s = ix.arena.stream();
  if (g && *g) {
    SNN_HIP(hipGraphLaunch(*g, s));
    return;
  }
  if (!g || !capture) {
    body();
    return;
  }
  // (checked only when it fails: an injected failure after a begun capture
  // would leave the stream capturing)
  const hipError_t eb = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (eb != hipSuccess) check_hip(eb, "hipStreamBeginCapture", __FILE__, __LINE__);
  hipGraph_t graph = nullptr;
  try {
    body();
  } catch (...) {
    (void)hipStreamEndCapture(s, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    throw;
  }
  {
    const hipError_t ee = hipStreamEndCapture(s, &graph);
    if (ee != hipSuccess) check_hip(ee, "hipStreamEndCapture", __FILE__, __LINE__);
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    log_line(3, "graph instantiation refused (%d): launching directly", (int)e);
    body();
    return;
  }
  log_line(3, "captured a repeated call's launches into a graph");
  *g = exec;
  SNN_HIP(hipGraphLaunch(exec, s));
}

// Clustering request: the self-query's accepted pairs go to DBSCAN instead
// of being assembled into neighbour lists.
struct DbscanReq {
  int32_t min_samples;
  int32_t* labels;     // device, n (original order)
  uint8_t* core;       // device, n or nullptr
  int64_t nclusters;   // out
};

// Stage times of a profiled call from its events: ev[0] call start,
// ev[4] queries in score order, ev[5] windows and tile plan done, ev[1] /
// ev[2] screen start / end (of the last attempt), ev[6] recheck done,
// ev[end] call end.
static void stage_times(hipEvent_t* ev, int end, snn_stats* st) {
  const int from[SNN_STAGES] = {0, 4, 1, 2, 6};
  const int to[SNN_STAGES] = {4, 5, 2, 6, end};
  for (int k = 0; k < SNN_STAGES; ++k) {
    float t = 0;
    SNN_HIP(hipEventElapsedTime(&t, ev[from[k]], ev[to[k]]));
    st->stage_ms[k] = t;
  }
}

static const char* screen_name(snn_precision p, int terms) {
  switch (p) {
    case SNN_PREC_FP16:
      return "fp16";
    case SNN_PREC_FP32:
      return "fp32";
    case SNN_PREC_MIXED:
      return terms == 1 ? "bf16" : "bf16x3";
    default:
      return "fp64";
  }
}

// One SNN_LOG=2 line per query.
static void log_query(const Index& ix, int64_t m, double R, bool self, snn_precision prec, int terms,
                      unsigned long long window, unsigned long long survivors, int64_t result, const snn_stats* st,
                      const QueryGraph* qg, const char* result_name) {
  if (log_level() < 2) return;
  char times[200] = "";
  if (st) {
    int k = std::snprintf(times, sizeof(times), ", device %.3f ms (screen %.3f)", st->total_ms, st->screen_ms);
    if (st->stage_ms[0] >= 0)
      std::snprintf(times + k, sizeof(times) - k, ", stages %.3f / %.3f / %.3f / %.3f / %.3f ms", st->stage_ms[0],
                    st->stage_ms[1], st->stage_ms[2], st->stage_ms[3], st->stage_ms[4]);
  }
  log_line(2, "%s n=%lld d=%d m=%lld R=%.17g screen=%s window pairs=%llu survivors=%llu %s=%lld%s%s",
           self ? "self-query" : "query", (long long)ix.n, ix.d, (long long)m, R, screen_name(prec, terms), window,
           survivors, result_name, (long long)result, qg && qg->uses > 2 ? " (graph replay)" : "", times);
}

static void run_query(Index& ix, const void* Q, int64_t m, double R, bool self, const snn_options* opts,
                      snn_csr* out, snn_stats* st, DbscanReq* db = nullptr) {
  if (db && !self) fail(SNN_EINVAL, "clustering needs an all-points self-query");
  if (!std::isfinite(R) || R < 0) fail(SNN_EINVAL, "R must be finite and >= 0");
  if (m < 0) fail(SNN_EINVAL, "m must be >= 0");
  if (m >= (int64_t)INT32_MAX) fail(SNN_EINVAL, "m must be < 2^31 - 1");
  if (!self && m > 0 && !Q) fail(SNN_EINVAL, "Q is NULL");
  if (!db) {
    if (!out) fail(SNN_EINVAL, "out is NULL");
    if (!out->row_ptr) fail(SNN_EINVAL, "out->row_ptr is NULL");
    if (out->nnz_cap < 0) fail(SNN_EINVAL, "nnz_cap must be >= 0");
    if (out->nnz_cap > 0 && (!out->col || !out->dist)) fail(SNN_EINVAL, "out->col / out->dist is NULL");
  }
  snn_options o{};
  o.precision = SNN_PREC_AUTO;
  if (opts) o = *opts;
  if (o.precision != SNN_PREC_FP64 && o.precision != SNN_PREC_MIXED && o.precision != SNN_PREC_AUTO &&
      o.precision != SNN_PREC_FP32 && o.precision != SNN_PREC_FP16)
    fail(SNN_EINVAL, "unknown precision");
  if (o.mixed_terms != 0 && o.mixed_terms != 1 && o.mixed_terms != 3) fail(SNN_EINVAL, "mixed_terms must be 0, 1 or 3");
  if (o.tile_q < 0 || o.tile_c < 0) fail(SNN_EINVAL, "tile sizes must be >= 0");
  if (o.tile_q % 64 != 0) fail(SNN_EINVAL, "tile_q must be a multiple of 64");
  if (o.full_self_scan != 0 && o.full_self_scan != 1) fail(SNN_EINVAL, "full_self_scan must be 0 or 1");
  if (o.metric != SNN_METRIC_L2 && o.metric != SNN_METRIC_L1 && o.metric != SNN_METRIC_ANGULAR &&
      o.metric != SNN_METRIC_COSINE)
    fail(SNN_EINVAL, "unknown metric");
  if (o.metric == SNN_METRIC_ANGULAR && R > M_PI) fail(SNN_EINVAL, "angular radius must be at most pi");

  DeviceScope scope(ix.arena.dev().device);
  hipStream_t s = ix.arena.stream();
  const DeviceInfo& di = device_info(ix.arena.dev().device);
  const int d = ix.d;
  const int64_t n = ix.n;
  // L1: every point with M(p, q) <= R has S(p, q) <= fl(Rs*Rs) for the
  // widened radius Rs = R (1 + 8 gamma_{d+2}): the exact 1-norm is at most
  // M (1 + 2 gamma_{d+1}), the 2-norm at most the 1-norm, and S at most the
  // exact squared 2-norm times (1 + gamma_{d+2}).  The window and the screen
  // use Rs, the recheck decides by M <= R.
  //
  // Angular and cosine searches of unit rows compare S with the squared
  // chord T = fl(2 - 2 cos a) or fl(2 c) (Section 2) instead of fl(R*R); the
  // window and the screen take Rs = sqrt(T) rounded up, so Rs^2 >= T.
  double Rs = R, R2 = R * R;
  if (o.metric == SNN_METRIC_L1) {
    Rs = R * (1.0 + 8.0 * gamma64(d + 2));
    R2 = Rs * Rs;
  } else if (o.metric == SNN_METRIC_ANGULAR || o.metric == SNN_METRIC_COSINE) {
    R2 = o.metric == SNN_METRIC_ANGULAR ? 2.0 - 2.0 * std::cos(R) : 2.0 * R;
    if (!std::isfinite(R2)) fail(SNN_EINVAL, "cosine radius too large");
    Rs = std::nextafter(std::sqrt(R2), INFINITY);
  }

  // ---- precision plan
  const ScreenPlan sp = plan_screen(ix, o, R2);
  const snn_precision prec = sp.prec;
  const bool mix16 = prec == SNN_PREC_MIXED || prec == SNN_PREC_FP16;  // 16-bit operand screens
  const double Y = ix.max_norm;
  int T_fixed = 0;
  if (mix16) T_fixed = 4 * mixed_queries_per_wave(operand_ka(sp.kind, d), sp.kind == kOpF16);
  if (prec == SNN_PREC_FP32) T_fixed = mfma32_queries_per_tile();
  if (T_fixed && o.tile_q && o.tile_q != T_fixed)
    fail(SNN_EINVAL, "tile_q must be " + std::to_string(T_fixed) + " for this screen and dimension");
  const int T = T_fixed ? T_fixed : (o.tile_q ? o.tile_q : 64);
  // candidates per work unit: 8192 for the matrix-core screens (measured best
  // against 2048-16384 with 256-query tiles), 1024 for the float64 screen
  const int ntiles = (int)std::max<int64_t>(1, (m + T - 1) / T);
  int CH = o.tile_c ? o.tile_c : (prec == SNN_PREC_FP64 ? 1024 : 8192);
  if (!o.tile_c) {
    // a small call: shorter units until every CU can get a few (uniform2d,
    // 1e3 queries over 1e4 points: 6 units of 8192 candidates kept 6
    // workgroups busy for the whole screen)
    const int64_t want = 4LL * di.cus;
    const int floor_ch = prec == SNN_PREC_FP64 ? 128 : 256;
    while (CH > floor_ch && (int64_t)ntiles * ((n + CH - 1) / CH) < want) CH /= 2;
  }
  if (prec != SNN_PREC_FP64 && CH % 32 != 0) fail(SNN_EINVAL, "matrix-core screens: tile_c must be a multiple of 32");
  if (mix16) build_mixed_operands(ix, sp.kind);
  if (prec == SNN_PREC_FP32) build_fp32_operands(ix);
  // the float64 rows: read by the fp64 screen, and as the query rows of a
  // self-query's recheck; filled before any capture (a replay never needs it)
  if (prec == SNN_PREC_FP64 || self) build_rows64(ix);

  // stats: the device clock marks the call's start (its first kernel) and
  // end (a mark kernel after the last one), and the screen's workgroups
  // mark the screen's; events (each costs the host microseconds on the
  // critical path) only for a profiled call, at the call's start and end
  // and between its stages (kept on the index)
  hipEvent_t* ev = ix.ev;
  const bool prof = st && profile_on();
  const bool marks = st && di.clock_khz > 0;
  if (st) {
    if (prof || !marks)
      for (int i = 0; i < (prof ? 7 : 4); ++i)
        if (!ev[i]) SNN_HIP(hipEventCreate(&ev[i]));
    for (double& t : st->stage_ms) t = -1;
    if (prof || !marks) SNN_HIP(hipEventRecord(ev[0], s));
  }
  auto mark = [&](int i) {
    if (prof) SNN_HIP(hipEventRecord(ev[i], s));
  };

  // ---- workspace
  const int nbuckets = query_buckets(m);
  Carver probe(nullptr);
  auto plan_query = [&](Carver& c) {
    struct P {
      uint32_t* ukey;
      uint32_t* val;
      uint32_t* hist;
      double* qa_in;
      double* qn_in;
      double* q64;
      int32_t* qorig;
      double* qa;
      double* qn;
      int32_t* lo;
      int32_t* hi;
      int32_t* tlo;
      int32_t* thi;
      int32_t* units;
      int64_t* unit_off;
      int32_t* gbase;
      unsigned long long* wpart;
      char* scan_scratch;
      Ctl* ctl;
      unsigned long long* lb_buckets;  // look-back scan states (zeroed with ctl)
      unsigned long long* lb_rows;     // (two: slot-order and caller-order rows)
      int ctl_words;                   // words zeroed at the call's start
      int32_t* row_cnt;                // per query slot
      int64_t* rp_s;                   // slot-order row offsets
      int32_t* cnt_o;                  // per caller row
      int32_t* lists;
      uint16_t* qop;
      float* cthr;
      float* vq;
    } p;
    const size_t mq = self ? 1 : (size_t)m;
    p.ukey = c.take<uint32_t>(mq);  // bucket of each query
    p.val = c.take<uint32_t>(mq);   // slot of each query in its bucket
    p.hist = c.take<uint32_t>(self ? 1 : nbuckets);
    p.qa_in = c.take<double>(mq);
    p.qn_in = c.take<double>(mq);
    // float64 copies of out-of-sample queries in score order: only the
    // float64 screen reads them (the recheck of the others reads the
    // caller's rows through qorig)
    p.q64 = prec == SNN_PREC_FP64 ? c.take<double>(mq * ix.dp) : nullptr;
    p.qorig = c.take<int32_t>(mq);
    p.qa = c.take<double>(mq);
    p.qn = c.take<double>(std::max<size_t>(m, 1));
    p.lo = nullptr;
    p.hi = nullptr;
    p.tlo = c.take<int32_t>(ntiles);
    p.thi = c.take<int32_t>(ntiles);
    p.units = c.take<int32_t>(ntiles);
    p.unit_off = c.take<int64_t>(ntiles + 1);
    p.gbase = c.take<int32_t>(ntiles);
    p.wpart = c.take<unsigned long long>(kWindowMaxBlocks);
    p.scan_scratch = c.take<char>(std::max({scan_scratch_bytes(ntiles), scan_scratch_bytes(std::max<int64_t>(m, 1)),
                                            scan_scratch_bytes(nbuckets)}));
    {
      const size_t wc = sizeof(Ctl) / 8, wb = lookback_words(nbuckets), wr = lookback_words(m);
      unsigned long long* region = c.take<unsigned long long>(wc + wb + 2 * wr);
      p.ctl = reinterpret_cast<Ctl*>(region);
      p.lb_buckets = region + wc;
      p.lb_rows = region + wc + wb;
      p.ctl_words = (int)(wc + wb + 2 * wr);
    }
    p.row_cnt = c.take<int32_t>(std::max<int64_t>(m, 1));
    p.rp_s = c.take<int64_t>(m + 1);
    p.cnt_o = c.take<int32_t>(std::max<int64_t>(m, 1));
    p.lists =c.take<int32_t>((size_t)row_sort_lists() * std::max<int64_t>(m, 1));
    p.qop = c.take<uint16_t>(mix16 && !self ? (size_t)m * operand_ka(sp.kind, d) : 1);
    p.cthr = c.take<float>(mix16 ? std::max<int64_t>(m, 1) : 1);
    p.vq = c.take<float>(prec == SNN_PREC_FP32 ? (size_t)std::max<int64_t>(m, 1) * mfma32_query_floats(d) : 1);
    return p;
  };
  plan_query(probe);
  ix.ws[0].ensure(ix.arena, probe.off + 256);
  Carver carve(ix.ws[0].ptr);
  auto P = plan_query(carve);

  // ---- host values of every launch of the call
  // screen operands and start values: built by the gather for out-of-sample
  // queries, by their own pass for self-queries
  QueryOperands qop{};
  MixedDev mx{};
  MixedBound self_bound{};
  if (mix16) mx = prepare_mixed(ix, sp.kind, R2, self, P.qop, P.cthr, &qop, &self_bound);
  if (prec == SNN_PREC_FP32) prepare_fp32(ix, R2, self, P.vq, &qop, &self_bound);
  const double* q64 = self ? ix.p64.as<double>() : P.q64;  // NULL: the recheck reads Q
  const int32_t* qorig = self ? ix.perm.as<int32_t>() : P.qorig;
  const double* qa = self ? ix.key.as<double>() : P.qa;
  const double* qn = P.qn;

  // W_q = R ||v|| (1 + 4 gamma_{d+3}) + key_eps + eps_q, eps_q = c ||y_q||
  const double u32 = std::ldexp(1.0, -24);
  const double w_base = Rs * ix.vnorm * (1.0 + 4.0 * gamma64(d + 3)) + ix.key_eps;
  const double eps_scale = 1.01 * (u32 + gamma64(d + 2)) * (1.0 + u32) * ix.vnorm;
  // self-queries scan each unordered pair once (S is exactly symmetric)
  const int sym = (self && !o.full_self_scan) ? 1 : 0;
  const int32_t* cells = window_cells(ix);  // built on the index's first query
  // query slots per wavefront (stats): the matrix-core screens evaluate
  // whole 32-query blocks, the float64 screen one query at a time
  const int qpw = mix16                   ? mixed_queries_per_wave(operand_ka(sp.kind, d), sp.kind == kOpF16)
                  : prec == SNN_PREC_FP32 ? mfma32_queries_per_tile() / 4
                                          : 1;
  // chunk-major work order inside groups of G score-adjacent tiles (L2 reuse)
  const int G = prec == SNN_PREC_FP64 ? 16 : 8;
  const int ngroups = (ntiles + G - 1) / G;

  QueryDev qd{};
  qd.G = G;
  qd.ngroups = ngroups;
  qd.units = P.units;
  qd.m = m;
  qd.d = d;
  qd.dp = ix.dp;
  qd.T = T;
  qd.CH = CH;
  qd.ntiles = ntiles;
  qd.R2 = R2;
  qd.metric = o.metric;
  qd.R1 = R;
  qd.q64 = q64;
  qd.qsrc = Q;
  qd.qorig = qorig;
  qd.p64 = ix.p64.as<double>();
  qd.perm = ix.perm.as<int32_t>();
  qd.tlo = P.tlo;
  qd.thi = P.thi;
  qd.group_off = P.unit_off;
  qd.gbase = P.gbase;
  qd.counters = P.ctl->counters;
  qd.nxcd = di.xcds;
  qd.sym = sym;
  // the screen's duration from clock marks its workgroups leave (no events
  // around the launch, which would cost the host a few microseconds each)
  qd.stamps = st && di.clock_khz > 0 ? P.ctl->screen_mark : nullptr;

  // survivors: capacity remembered on the index, grown on overflow
  // bytes per survivor: the pair, and per result row, column, distance, slot
  // (clustering: the pair and one accepted mark)
  const int per = db ? 1 : (sym ? 2 : 1);
  const size_t per_bytes = db ? 12 : 8 + 16 * (size_t)per;
  long long cap = std::max<long long>(1 << 16, (long long)(ix.ws[1].bytes / per_bytes));
  HostCtl hc{};
  Ctl* hctl = pinned_ctl(ix);
  // the mark kernel after the call's last kernel (the end of the post
  // sequence, or after the work that follows the read-back), read back
  auto end_mark = [&](bool read_back) {
    if (!marks) return;
    launch_clock_mark(&P.ctl->call_mark[1], s);
    if (read_back) {
      SNN_HIP(hipMemcpyAsync(&hctl->call_mark[1], &P.ctl->call_mark[1], 8, hipMemcpyDeviceToHost, s));
      SNN_HIP(hipStreamSynchronize(s));
      hc.ctl.call_mark[1] = hctl->call_mark[1];
    }
  };
  // device time of the call; later: work was enqueued after the read-back
  auto call_end_ms = [&](bool later) -> double {
    if (marks && !prof) {
      if (later) end_mark(true);
      return call_ms_of(hc.ctl, di);
    }
    if (later) SNN_HIP(hipEventRecord(ev[3], s));
    SNN_HIP(hipEventSynchronize(ev[3]));
    float b = 0;
    SNN_HIP(hipEventElapsedTime(&b, ev[0], ev[3]));
    return b;
  };
  Survivors sv{};
  uint64_t* stage_key = nullptr;  // neighbour keys in slot-order rows
  RowMove mv{};                   // their move to the caller's rows
  // The survivor list and the staging rows are carved before any launch, so
  // that every launch of the call is fixed by the values above.  The rows of
  // up to 16 neighbours are assembled before the sizes are read back, so the
  // device does not wait for the host in between: the staging rows hold
  // every neighbour this attempt can produce (cap x per), the scatter does
  // nothing when the survivor list overflowed, and the moves write nothing
  // when the rows exceed the caller's capacity (the host then retries or
  // reports it).
  auto carve_survivors = [&]() {
    // five arrays, each padded to 256 bytes by the carver
    const size_t need = (size_t)cap * per_bytes + 2048;
    ix.ws[1].ensure(ix.arena, need);
    cap = (long long)((ix.ws[1].bytes - 2048) / per_bytes);
    Carver sc(ix.ws[1].ptr);
    sv = Survivors{};
    sv.per = per;
    sv.pairs = sc.take<int2>(cap);
    sv.res_q = sc.take<int32_t>(cap * per);
    sv.res_key = db ? nullptr : sc.take<uint64_t>(cap * per);
    sv.res_slot = db ? nullptr : sc.take<int32_t>(cap * per);
    sv.cap = cap;
    sv.count = &P.ctl->survivors;
    qd.sink.out = sv.pairs;
    qd.sink.counter = sv.count;
    qd.sink.cap = cap;
    if (!db) {
      const size_t stage_n = (size_t)cap * per;
      ix.ws[3].ensure(ix.arena, stage_n * 8 + 512);
      Carver gc(ix.ws[3].ptr);
      stage_key = gc.take<uint64_t>(stage_n);
      mv = RowMove{P.rp_s, stage_key, qorig, out->row_ptr, out->col, out->dist, &P.ctl->nnz,
                   (unsigned long long)out->nnz_cap};
    }
  };
  carve_survivors();
  const int per_cu = mix16                   ? mixed_blocks_per_cu(mx.KA, mx.KB, mx.f16 != 0)
                     : prec == SNN_PREC_FP32 ? mfma32_blocks_per_cu(d)
                                             : fp64_blocks_per_cu(ix.dp);
  // persistent workgroups: enough to fill the chip, but no more than the
  // work units the tile plan can make (each tile has at most ceil(n / CH) + 1
  // chunks); a small query then does not dispatch thousands of idle ones
  const int64_t units_max = (int64_t)ntiles * ((n + CH - 1) / CH + 1);
  const int grid = (int)std::max<int64_t>(
      di.xcds, std::min<int64_t>((di.cus * per_cu / di.xcds) * di.xcds, (units_max + di.xcds - 1) / di.xcds * di.xcds));

  // ---- the launches before the screen: queries into score order, their
  // operands, windows and the tile plan
  const bool sort_queries = !self && m > 0;
  auto enqueue_pre = [&]() {
    launch_query_init(reinterpret_cast<unsigned long long*>(P.ctl), P.ctl_words, P.row_cnt, m,
                      sort_queries ? P.hist : nullptr, nbuckets, P.tlo, P.thi, ntiles, s,
                      marks ? (int)(offsetof(Ctl, call_mark) / 8) : -1);
    if (self && mix16) launch_mixed_qprep_self(ix.ys.as<float>(), ix.n, ix.d, self_bound, P.cthr, s);
    if (self && prec == SNN_PREC_FP32) launch_mfma32_qprep_self(ix.ys.as<float>(), ix.n, ix.d, self_bound, P.vq, s);
    if (sort_queries) {
      // queries into score order by a counting sort on a uniform score grid
      launch_query_keys(ix.dtype, Q, m, d, ix.mu.as<double>(), ix.v.as<double>(), ix.key.as<double>(), (int)n,
                        nbuckets, P.ukey, P.val, P.hist, P.qa_in, P.qn_in, &P.ctl->bad, P.lb_buckets,
                        &P.ctl->scan_err, s);
      launch_query_gather(ix.dtype, Q, m, d, ix.dp, P.ukey, P.val, P.hist, P.qa_in, P.qn_in, P.q64, P.qorig, P.qa,
                          P.qn, ix.mu.as<double>(), qop, s);
    }
    if (self) launch_self_qnorm(ix.ynorm.as<float>(), n, P.qn, s);
    mark(4);
    TilePlanArgs plan{};
    plan.tlo = P.tlo;
    plan.thi = P.thi;
    plan.ntiles = ntiles;
    plan.CH = CH;
    plan.align = prec == SNN_PREC_FP64 ? 1 : 32;
    plan.sym_T = sym ? T : 0;
    plan.units = P.units;
    plan.G = G;
    plan.unit_off = P.unit_off;
    plan.gbase = P.gbase;
    plan.T = T;
    plan.m = m;
    plan.qpw = qpw;
    plan.executed = st ? &P.ctl->executed : nullptr;
    plan.wpart = P.wpart;
    plan.nwpart = window_blocks(m);
    plan.pairs_window = &P.ctl->pairs_window;
    launch_windows_plan(ix.key.as<double>(), (int)n, cells, ix.wcells_n, qa, qn, m, w_base, eps_scale, T, sym, P.lo,
                        P.hi, plan, s);
    mark(5);
  };
  // ---- the screen
  auto enqueue_screen = [&]() {
    if (m <= 0) return;
    if (mix16)
      launch_cand_mfma(qd, mx, grid, s);
    else if (prec == SNN_PREC_FP32)
      launch_cand_mfma32(qd, Mfma32Dev{P.vq, mfma32_query_floats(d), d, ix.vcand.as<float>(), ix.h.as<float>()}, grid,
                         s);
    else
      launch_cand_fp64(qd, grid, s);
  };
  // ---- the launches after the screen: recheck, row offsets, the
  // neighbours into their rows and the rows of up to 16 neighbours sorted
  // into the caller's rows (longer rows follow the read-back)
  auto enqueue_post = [&]() {
    // grid of the survivor passes from the list's capacity (a grid-stride
    // loop: few workgroups for the short lists of sparse outputs, where the
    // dispatch of thousands of idle ones would dominate)
    const int sgrid = (int)std::min<long long>(16LL * di.cus, std::max<long long>(2LL * di.cus, cap / 2048));
    launch_recheck(qd, sv, ix.dtype, ix.po.ptr, self, P.row_cnt, sgrid, s);
    mark(6);
    // slot-order row offsets (where the neighbours are assembled) with the
    // counts in the caller's order, the longest row, the total and the rows
    // by length class; then the caller's row offsets
    launch_rows_scan(P.row_cnt, m, P.rp_s, P.lb_rows, &P.ctl->scan_err,
                     RowsExtra{qorig, P.cnt_o, &P.ctl->row_max, &P.ctl->nnz, P.lists, P.ctl->list_counts}, s);
    // the caller-order scan and the scatter in one launch for short survivor
    // lists (one launch fewer); for long ones (dense outputs) apart, as the
    // scan's registers and LDS would hold down the scatter's occupancy
    // (blobs3d: 4.7 ms fused against 3.9 + 0.1 ms)
    if (cap <= (1LL << 20)) {
      launch_rows_scan_scatter(P.cnt_o, m, out->row_ptr, P.lb_rows + lookback_words(m), &P.ctl->scan_err, sv,
                               P.rp_s, stage_key, sgrid, s);
    } else {
      launch_rows_scan(P.cnt_o, m, out->row_ptr, P.lb_rows + lookback_words(m), &P.ctl->scan_err, RowsExtra{}, s);
      launch_scatter(sv, P.rp_s, stage_key, sgrid, s);
    }
    launch_row_sort_short(mv, P.lists, P.ctl->list_counts, s);
    end_mark(false);
  };

  // A call repeated with the same inputs, outputs and workspace (a serving
  // loop) replays the launch sequences before and after the screen from
  // graphs captured on its second occurrence: one launch each instead of
  // about fifteen.
  QueryGraph* qg = nullptr;
  if (!db && s && !prof) {  // (the null stream cannot be captured)
    GraphKey gk{};
    const uint64_t fields[] = {reinterpret_cast<uint64_t>(Q), (uint64_t)m, bits_of(R), (uint64_t)self,
                               (uint64_t)o.precision, (uint64_t)o.mixed_terms, (uint64_t)o.tile_q,
                               (uint64_t)o.tile_c, (uint64_t)o.full_self_scan, (uint64_t)o.metric,
                               reinterpret_cast<uint64_t>(out->row_ptr), reinterpret_cast<uint64_t>(out->col),
                               reinterpret_cast<uint64_t>(out->dist), (uint64_t)out->nnz_cap, st ? 1ull : 0ull,
                               ix.epoch, reinterpret_cast<uint64_t>(ix.ws[0].ptr), (uint64_t)ix.ws[0].bytes,
                               reinterpret_cast<uint64_t>(ix.ws[1].ptr), (uint64_t)ix.ws[1].bytes,
                               reinterpret_cast<uint64_t>(ix.ws[3].ptr), (uint64_t)ix.ws[3].bytes, (uint64_t)cap,
                               reinterpret_cast<uint64_t>(s)};
    static_assert(sizeof(fields) <= sizeof(gk.v), "graph key too long");
    std::memcpy(gk.v, fields, sizeof(fields));
    qg = query_graph(ix, gk);
  }
  run_captured(ix, qg ? &qg->pre : nullptr, qg && qg->uses > 1, enqueue_pre);

  for (int attempt = 0;; ++attempt) {
    if (attempt > 0) {
      carve_survivors();
      launch_fill_u64(P.ctl->counters, kMaxXcd, 0ull, s);
      launch_fill_u64(&P.ctl->survivors, 1, 0ull, s);
      launch_fill_u64(&P.ctl->accepted, 1, 0ull, s);
      launch_fill_u64(P.ctl->list_counts, 8, 0ull, s);
      launch_fill_u64(&P.ctl->row_max, 1, 0ull, s);
      launch_fill_u64(P.ctl->screen_mark, 2, 0ull, s);
      launch_fill_u64(P.lb_rows, 2 * (int64_t)lookback_words(m), 0ull, s);
      launch_fill_i32(P.row_cnt, m, 0, s);
    }
    mark(1);
    enqueue_screen();
    mark(2);
    if (db) {
      launch_recheck_edges(qd, sv, ix.dtype, ix.po.ptr, P.row_cnt, &P.ctl->accepted, di.cus * 16, s);
      mark(6);
      SNN_HIP(hipMemcpyAsync(hctl, P.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
      SNN_HIP(hipStreamSynchronize(s));
      hc.ctl = *hctl;
      if ((long long)hc.ctl.survivors <= cap) {
        ix.ws[3].ensure(ix.arena, dbscan_work_bytes(n));
        db->nclusters = dbscan_from_survivors(sv, n, P.row_cnt, ix.perm.as<int32_t>(), db->min_samples,
                                              ix.ws[3].ptr, db->labels, db->core, di.cus * 16, s);
        if (st) {
          st->pairs_window = (int64_t)hc.ctl.pairs_window;
          st->flops_window = 2.0 * d * (double)hc.ctl.pairs_window;
          st->pairs_recheck = (int64_t)hc.ctl.survivors;
          st->nnz = (int64_t)hc.ctl.accepted;
          st->precision_used = prec;
          st->terms_used = sp.terms();
        }
        break;
      }
      log_line(3, "survivor list of %lld overflowed (%llu survivors): screening again", cap, hc.ctl.survivors);
      cap = (long long)(hc.ctl.survivors * 5 / 4) + 1024;
      ix.ws[1].reset(ix.arena);
      continue;
    }
    // (a retry's larger survivor list is not the captured call's)
    run_captured(ix, qg && attempt == 0 ? &qg->post : nullptr, qg && qg->uses > 1, enqueue_post);
    SNN_HIP(hipMemcpyAsync(hctl, P.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    // the call's end unless longer rows follow the read-back
    if (prof || (st && !marks)) SNN_HIP(hipEventRecord(ev[3], s));
    SNN_HIP(hipStreamSynchronize(s));
    hc.ctl = *hctl;
    hc.nnz = (int64_t)hc.ctl.nnz;
    if (hc.ctl.bad) fail(SNN_EINVAL, "Q contains NaN or Inf");
    if (hc.ctl.scan_err) fail(SNN_EDEVICE, "a single-pass scan did not complete");
    if ((long long)hc.ctl.survivors <= cap) {
      out->nnz = hc.nnz;
      if (st) {
        st->pairs_window = (int64_t)hc.ctl.pairs_window;
        st->flops_window = 2.0 * d * (double)hc.ctl.pairs_window;
        st->pairs_recheck = (int64_t)hc.ctl.survivors;
        st->nnz = hc.nnz;
        st->precision_used = prec;
        st->terms_used = sp.terms();
      }
      if (hc.nnz > out->nnz_cap) {
        char buf[160];
        std::snprintf(buf, sizeof(buf), "CSR capacity %lld < %lld neighbours", (long long)out->nnz_cap,
                      (long long)hc.nnz);
        throw Error(SNN_EOVERFLOW, buf);
      }
      break;
    }
    log_line(3, "survivor list of %lld overflowed (%llu survivors): screening again", cap, hc.ctl.survivors);
    cap = (long long)(hc.ctl.survivors * 5 / 4) + 1024;
    ix.ws[1].reset(ix.arena);
  }

  if (db) {
    if (st) {
      // (the clustering ran after the read-back)
      st->total_ms = call_end_ms(true);
      st->screen_ms = screen_ms_of(hc.ctl, di);
      st->pairs_executed = (int64_t)hc.ctl.executed;
      // (the clustering after the read-back is the assembly stage)
      if (prof) stage_times(ev, 3, st);
    }
    log_query(ix, m, R, self, prec, sp.terms(), hc.ctl.pairs_window, hc.ctl.survivors, (int64_t)hc.ctl.accepted, st,
              qg, "clusters");
    return;
  }

  // ---- rows: ids ascending, moved to the caller's row order
  int32_t* tmp_col = nullptr;
  float* tmp_dist = nullptr;
  if (hc.ctl.row_max > 4096) {
    ix.ws[2].ensure(ix.arena, (size_t)hc.nnz * 8 + 512);
    Carver tc(ix.ws[2].ptr);
    tmp_col = tc.take<int32_t>(hc.nnz);
    tmp_dist = tc.take<float>(hc.nnz);
  }
  launch_row_sort_tail(mv, m, (int64_t)hc.ctl.row_max, P.lists, P.ctl->list_counts, tmp_col, tmp_dist, s);

  if (st) {
    // longer rows were sorted after the read-back
    st->total_ms = call_end_ms(hc.ctl.row_max > 16);
    st->screen_ms = screen_ms_of(hc.ctl, di);
    st->pairs_executed = (int64_t)hc.ctl.executed;
    if (prof) stage_times(ev, 3, st);
  }
  log_query(ix, m, R, self, prec, sp.terms(), hc.ctl.pairs_window, hc.ctl.survivors, hc.nnz, st, qg, "nnz");
}

// ------------------------------------------------------------------------ test support
// The screen a query would run, and the sizes of its operand rows.
static ScreenPlan debug_plan(const Index& ix, double R, const snn_options* opts, snn_screen_layout* lay) {
  if (!std::isfinite(R) || R < 0) fail(SNN_EINVAL, "R must be finite and >= 0");
  snn_options o{};
  o.precision = SNN_PREC_AUTO;
  if (opts) o = *opts;
  if (o.metric != SNN_METRIC_L2) fail(SNN_EINVAL, "screen values are dumped for the Euclidean metric");
  if (o.mixed_terms != 0 && o.mixed_terms != 1 && o.mixed_terms != 3) fail(SNN_EINVAL, "mixed_terms must be 0, 1 or 3");
  const ScreenPlan sp = plan_screen(ix, o, R * R);
  if (sp.prec == SNN_PREC_FP64) fail(SNN_EINVAL, "the float64 path has no screen values");
  const int d = ix.d;
  lay->precision = sp.prec;
  lay->terms = sp.terms();
  if (sp.prec == SNN_PREC_FP32) {
    lay->ka = mfma32_query_floats(d);
    lay->kb = d;
    lay->chain = 2 * ((d + 1) / 2);
    lay->scale_exp = 0;
  } else {
    lay->ka = operand_ka(sp.kind, d);
    lay->kb = (sp.kind == kOpBf16x3 && d % 16 == 0) ? 2 * d : lay->ka;
    lay->chain = lay->ka;
    lay->scale_exp = sp.kind == kOpF16 ? f16_scale_exp(ix.max_norm) : 0;
  }
  return sp;
}

static void debug_screen(Index& ix, const void* Q, int64_t m, double R, const snn_options* opts, float* D, float* H,
                         float* C, void* A, void* B, snn_screen_layout* lay) {
  const ScreenPlan sp = debug_plan(ix, R, opts, lay);
  if (m < 1 || m >= (int64_t)INT32_MAX) fail(SNN_EINVAL, "m must be in [1, 2^31 - 1)");
  if (!Q || !D || !H || !C || !A || !B) fail(SNN_EINVAL, "NULL buffer");
  DeviceScope scope(ix.arena.dev().device);
  hipStream_t s = ix.arena.stream();
  const int d = ix.d;
  const int64_t n = ix.n;
  const double R2 = R * R;
  const bool mix16 = sp.prec != SNN_PREC_FP32;
  if (mix16)
    build_mixed_operands(ix, sp.kind);
  else
    build_fp32_operands(ix);
  // the queries in score order, as a query call sorts them
  const int nb = query_buckets(m);
  auto plan = [&](Carver& c) {
    struct P {
      unsigned long long* ctl;
      uint32_t *ukey, *val, *hist;
      double *qa_in, *qn_in, *q64, *qa, *qn;
      int32_t *qorig, *row_cnt;
      uint16_t* qop;
      float *cthr, *vq;
    } p;
    // ints: bad, scan error; then the bucket scan's look-back state
    p.ctl = c.take<unsigned long long>(1 + lookback_words(nb));
    p.ukey = c.take<uint32_t>(m);
    p.val = c.take<uint32_t>(m);
    p.hist = c.take<uint32_t>(nb);
    p.qa_in = c.take<double>(m);
    p.qn_in = c.take<double>(m);
    p.q64 = c.take<double>((size_t)m * ix.dp);
    p.qa = c.take<double>(m);
    p.qn = c.take<double>(m);
    p.qorig = c.take<int32_t>(m);
    p.row_cnt = c.take<int32_t>(m);
    p.qop = c.take<uint16_t>(mix16 ? (size_t)m * lay->ka : 1);
    p.cthr = c.take<float>(m);
    p.vq = c.take<float>(mix16 ? 1 : (size_t)m * lay->ka);
    return p;
  };
  Carver probe(nullptr);
  plan(probe);
  ScopedAlloc mem(ix.arena, probe.off + 256);
  Carver carve(mem.get());
  auto P = plan(carve);
  launch_query_init(P.ctl, (int)(1 + lookback_words(nb)), P.row_cnt, m, P.hist, nb, nullptr, nullptr, 0, s);
  QueryOperands qop{};
  MixedDev mx{};
  MixedBound unused{};
  if (mix16)
    mx = prepare_mixed(ix, sp.kind, R2, false, P.qop, P.cthr, &qop, &unused);
  else
    prepare_fp32(ix, R2, false, P.vq, &qop, &unused);
  launch_query_keys(ix.dtype, Q, m, d, ix.mu.as<double>(), ix.v.as<double>(), ix.key.as<double>(), (int)n, nb, P.ukey,
                    P.val, P.hist, P.qa_in, P.qn_in, reinterpret_cast<int*>(P.ctl), P.ctl + 1,
                    reinterpret_cast<int*>(P.ctl) + 1, s);
  launch_query_gather(ix.dtype, Q, m, d, ix.dp, P.ukey, P.val, P.hist, P.qa_in, P.qn_in, P.q64, P.qorig, P.qa, P.qn,
                      ix.mu.as<double>(), qop, s);
  if (mix16) {
    launch_dump_mixed(mx, m, n, P.qorig, D, s);
    SNN_HIP(hipMemcpyAsync(H, mx.h, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
    launch_dump_rows_f32(P.cthr, m, 1, P.qorig, C, s);
    launch_dump_rows_u16(P.qop, m, lay->ka, P.qorig, static_cast<uint16_t*>(A), s);
    launch_dump_cand16(mx.cop, n, lay->kb, static_cast<uint16_t*>(B), s);
  } else {
    const Mfma32Dev x{P.vq, lay->ka, d, ix.vcand.as<float>(), ix.h.as<float>()};
    launch_dump_mfma32(x, m, n, P.qorig, D, s);
    SNN_HIP(hipMemcpyAsync(H, ix.h.ptr, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
    launch_dump_rows_f32(P.vq, m, lay->ka, P.qorig, static_cast<float*>(A), s);
    SNN_HIP(hipMemcpy2DAsync(C, sizeof(float), static_cast<float*>(A) + d, sizeof(float) * lay->ka, sizeof(float), m,
                             hipMemcpyDeviceToDevice, s));
    SNN_HIP(hipMemcpyAsync(B, ix.ys.ptr, sizeof(float) * n * d, hipMemcpyDeviceToDevice, s));
  }
  int flags[2] = {0, 0};  // NaN/Inf flag, scan error
  SNN_HIP(hipMemcpyAsync(flags, P.ctl, sizeof(flags), hipMemcpyDeviceToHost, s));
  SNN_HIP(hipStreamSynchronize(s));
  if (flags[0]) fail(SNN_EINVAL, "Q contains NaN or Inf");
  if (flags[1]) fail(SNN_EDEVICE, "a single-pass scan did not complete");
}

}  // namespace snn

using namespace snn;

struct snn_index_s : Index {
  explicit snn_index_s(const snn_device& d) : Index(d) {}
};

static void free_index(snn_index_s* ix) {
  if (!ix) return;
  DeviceArena& a = ix->arena;
  Buffer* bufs[] = {&ix->mu,    &ix->v,  &ix->key,   &ix->perm,           &ix->po,   &ix->p64,
                    &ix->ys,    &ix->h,  &ix->ynorm, &ix->stats_host_dev, &ix->rows};
  for (Buffer* b : bufs) b->reset(a);
  for (auto& mo : ix->mixed) {
    mo.cand.reset(a);
    mo.qself.reset(a);
    mo.hs.reset(a);
  }
  ix->vcand.reset(a);
  ix->wcells.reset(a);
  for (hipEvent_t& e : ix->ev)
    if (e) (void)hipEventDestroy(e);
  for (QueryGraph& g : ix->qgraphs) destroy_query_graph(g);
  if (ix->host_ctl) (void)hipHostFree(ix->host_ctl);
  for (auto& w : ix->ws) w.reset(a);
  delete ix;
}

extern "C" {

snn_status snn_index(const snn_device* dev, const void* X, int64_t n, int32_t d, snn_dtype dtype,
                     snn_index_t* out) {
  return guard([&] {
    if (!dev || !out) fail(SNN_EINVAL, "dev / out is NULL");
    *out = nullptr;
    if (!X) fail(SNN_EINVAL, "X is NULL");
    if (n < 1 || n >= (int64_t)INT32_MAX) fail(SNN_EINVAL, "n must be in [1, 2^31 - 1)");
    if (d < 1 || d > 1024) fail(SNN_EINVAL, "d must be in [1, 1024]");
    if (dtype != SNN_F32 && dtype != SNN_F64) fail(SNN_EINVAL, "unknown dtype");
    if ((dev->alloc == nullptr) != (dev->free == nullptr)) fail(SNN_EINVAL, "alloc and free must both be set");
    DeviceScope scope(dev->device);
    snn_index_s* ix = new snn_index_s(*dev);
    ix->n = n;
    ix->d = d;
    ix->dp = ((d + 3) / 4) * 4;
    ix->dtype = dtype;
    try {
      build_index(*ix, X);
    } catch (...) {
      free_index(ix);
      throw;
    }
    *out = ix;
  });
}

snn_status snn_query(snn_index_t idx, const void* Q, int64_t m, double R, const snn_options* opts, snn_csr* out,
                     snn_stats* st) {
  return guard([&] {
    if (!idx) fail(SNN_EINVAL, "index is NULL");
    run_query(*idx, Q, m, R, false, opts, out, st);
  });
}

snn_status snn_query_self(snn_index_t idx, double R, const snn_options* opts, snn_csr* out, snn_stats* st) {
  return guard([&] {
    if (!idx) fail(SNN_EINVAL, "index is NULL");
    run_query(*idx, nullptr, idx->n, R, true, opts, out, st);
  });
}

snn_status snn_dbscan_index(snn_index_t idx, double eps, int32_t min_samples, const snn_options* opts,
                            int32_t* labels, uint8_t* core, int64_t* nclusters, snn_stats* st) {
  return guard([&] {
    if (!idx) fail(SNN_EINVAL, "index is NULL");
    if (min_samples < 1) fail(SNN_EINVAL, "min_samples must be >= 1");
    if (idx->n > 0 && !labels) fail(SNN_EINVAL, "labels is NULL");
    DbscanReq db{min_samples, labels, core, 0};
    run_query(*idx, nullptr, idx->n, eps, true, opts, nullptr, st, &db);
    if (nclusters) *nclusters = db.nclusters;
  });
}

snn_status snn_index_insert(snn_index_t idx, const void* X, int64_t k) {
  return guard([&] {
    if (!idx) fail(SNN_EINVAL, "index is NULL");
    if (k < 0) fail(SNN_EINVAL, "k must be >= 0");
    if (k > 0 && !X) fail(SNN_EINVAL, "X is NULL");
    if (idx->n + k >= (int64_t)INT32_MAX) fail(SNN_EINVAL, "n + k must be < 2^31 - 1");
    DeviceScope scope(idx->arena.dev().device);
    insert_points(*idx, X, k);
  });
}

snn_status snn_index_get_view(snn_index_t idx, snn_index_view* view) {
  return guard([&] {
    if (!idx || !view) fail(SNN_EINVAL, "NULL argument");
    view->n = idx->n;
    view->d = idx->d;
    view->dtype = idx->dtype;
    view->mu = idx->mu.as<double>();
    view->v = idx->v.as<double>();
    view->key = idx->key.as<double>();
    view->perm = idx->perm.as<int32_t>();
    view->max_norm = idx->max_norm;
    view->key_eps = idx->key_eps;
    view->power_iters = idx->power_iters;
  });
}

void snn_index_free(snn_index_t idx) {
  if (!idx) return;
  try {
    DeviceScope scope(idx->arena.dev().device);
    (void)hipStreamSynchronize(idx->arena.stream());
    free_index(idx);
  } catch (...) {
    free_index(idx);
  }
}

snn_status snn_sort_pairs_u32(const snn_device* dev, uint32_t* keys, uint32_t* vals, int64_t n, int begin_bit,
                              int end_bit) {
  return guard([&] {
    if (!dev) fail(SNN_EINVAL, "dev is NULL");
    if (n < 0) fail(SNN_EINVAL, "n must be >= 0");
    if (n > 0 && (!keys || !vals)) fail(SNN_EINVAL, "keys / vals is NULL");
    if (begin_bit < 0 || end_bit > 32 || begin_bit >= end_bit) fail(SNN_EINVAL, "bad bit range");
    if ((dev->alloc == nullptr) != (dev->free == nullptr)) fail(SNN_EINVAL, "alloc and free must both be set");
    DeviceScope scope(dev->device);
    DeviceArena a(*dev);
    radix_sort_pairs(a, keys, vals, n, begin_bit, end_bit, a.stream());
  });
}

snn_status snn_debug_screen_layout(snn_index_t idx, double R, const snn_options* opts, snn_screen_layout* layout) {
  return guard([&] {
    if (!idx || !layout) fail(SNN_EINVAL, "NULL argument");
    debug_plan(*idx, R, opts, layout);
  });
}

snn_status snn_debug_screen(snn_index_t idx, const void* Q, int64_t m, double R, const snn_options* opts, float* D,
                            float* H, float* C, void* A, void* B, snn_screen_layout* layout) {
  return guard([&] {
    if (!idx || !layout) fail(SNN_EINVAL, "NULL argument");
    debug_screen(*idx, Q, m, R, opts, D, H, C, A, B, layout);
  });
}

const char* snn_last_error(void) { return g_err.c_str(); }

const char* snn_version(void) { return "snn-mi355x 0.1"; }

}  // extern "C"
