// Host-side internals of libsnn: error plumbing, device memory, the index
// object and the launchers each kernel file provides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "snn.h"

namespace snn {

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
  snn_status code;
  Error(snn_status c, const std::string& msg) : std::runtime_error(msg), code(c) {}
};

[[noreturn]] void fail(snn_status code, const std::string& msg);
void check_hip(hipError_t e, const char* what, const char* file, int line);
#define SNN_HIP(call) ::snn::check_hip((call), #call, __FILE__, __LINE__)
#define SNN_LAUNCH_CHECK() ::snn::check_hip(hipGetLastError(), "kernel launch", __FILE__, __LINE__)

// Page-locked host memory of at least `bytes` for small read-backs, one
// block per host thread, kept until the process ends (a copy into pageable
// memory is staged by the runtime and costs the call microseconds).
void* pinned_host(size_t bytes);

// thread-local message returned by snn_last_error()
void set_last_error(const std::string& msg);
// set_last_error plus, with SNN_LOG >= 1, a line on stderr
void report_failure(snn_status code, const std::string& msg);

// SNN_LOG level, 0..3 (read from the environment at every call)
int log_level();
// "[snn] <text>" on stderr when level <= log_level()
void log_line(int level, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
// SNN_PROFILE set to a non-zero integer: per-stage device times in snn_stats
bool profile_on();

// Runs f, turning every exception into a status code (nothing crosses the C ABI).
template <class F>
snn_status guard(F&& f) {
  try {
    f();
    set_last_error("");
    return SNN_OK;
  } catch (const Error& e) {
    report_failure(e.code, e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    report_failure(SNN_ENOMEM, "host allocation failed");
    return SNN_ENOMEM;
  } catch (const std::exception& e) {
    report_failure(SNN_EDEVICE, e.what());
    return SNN_EDEVICE;
  } catch (...) {
    report_failure(SNN_EDEVICE, "unknown error");
    return SNN_EDEVICE;
  }
}

// Selects a device for the duration of a call and checks that it is gfx950.
struct DeviceScope {
  int prev = -1;
  explicit DeviceScope(int device);
  ~DeviceScope();
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Carves 256-byte aligned sub-arrays out of one buffer (base nullptr: sizing pass).
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <typename T>
  T* take(size_t count) {
    T* p = reinterpret_cast<T*>(base + off);
    off += align256(sizeof(T) * (count > 0 ? count : 1));
    return p;
  }
};

// ---------------------------------------------------------------- memory
// Device allocations through snn_device.alloc (or hipMalloc).  Freed with
// the matching free; all frees happen after the stream work using the
// buffer has been enqueued, which is safe for stream-ordered allocators and
// for hipFree (which synchronises).
class DeviceArena {
 public:
  explicit DeviceArena(const snn_device& d) : dev_(d) {}
  void* alloc(size_t bytes);
  void release(void* p);
  const snn_device& dev() const { return dev_; }
  hipStream_t stream() const { return (hipStream_t)dev_.stream; }

 private:
  snn_device dev_;
};

// A device allocation for the duration of one call: released when the scope
// ends, also when an error is thrown part way (the release is stream-ordered
// for the caller's allocator and synchronous for hipFree, so work already
// enqueued on the buffer is not cut short).
class ScopedAlloc {
 public:
  ScopedAlloc(DeviceArena& a, size_t bytes) : a_(a), p_(a.alloc(bytes)) {}
  ~ScopedAlloc() { a_.release(p_); }
  ScopedAlloc(const ScopedAlloc&) = delete;
  ScopedAlloc& operator=(const ScopedAlloc&) = delete;
  void* get() const { return p_; }

 private:
  DeviceArena& a_;
  void* p_;
};

// A grow-only device buffer owned by an arena.
struct Buffer {
  void* ptr = nullptr;
  size_t bytes = 0;
  bool view = false;  // a range of another buffer: reset forgets it, frees nothing
  template <typename T>
  T* as() const {
    return reinterpret_cast<T*>(ptr);
  }
  void ensure(DeviceArena& a, size_t need);
  void reset(DeviceArena& a);
};

// ---------------------------------------------------------------- device info
struct DeviceInfo {
  int cus = 256;       // compute units
  int xcds = 8;        // accelerator complex dies (separate L2 each)
  int lds_bytes = 64 * 1024;  // LDS one workgroup may use (queried)
  double clock_khz = 0;       // rate of the device's constant clock (wall_clock64), 0 if unknown
};
const DeviceInfo& device_info(int device);

// ---------------------------------------------------------------- index
// Everything lives in sorted (score) order unless noted.
struct MixedOperands {
  bool built = false;  // operands of the current rows
  int ka = 0;          // query operand row length in 16-bit values (multiple of 16)
  int kb = 0;          // candidate row length: ka, or 2 ka / 3 when the rows are [hi | lo]
  int e = 0;           // fp16: operands are fp16(2^e y)
  Buffer cand;         // (n + 32) x kb: candidate operand rows, zero padding rows
  Buffer qself;        // n x ka: query operand rows for self-queries
  Buffer hs;           // fp16: n + 32 floats, h scaled by 2^(2e) (rounded down), padding +inf
};
// Slot of an operand kind (OperandKind of query_plan.h: bf16, bf16 hi/lo, fp16) in Index::mixed.
inline int mixed_slot(int kind) { return kind == 3 ? 1 : (kind == 4 ? 2 : 0); }

// Launch sequences of a repeated query call captured as graphs (runtime.hip):
// the key holds every value the launches depend on.
struct GraphKey {
  uint64_t v[32];
};
struct QueryGraph {
  GraphKey key{};
  hipGraphExec_t pre = nullptr;   // query order, operands, windows, tile plan
  hipGraphExec_t post = nullptr;  // recheck to the rows of up to 16 neighbours
  int uses = 0;                   // calls with this key since the slot was taken
  uint64_t stamp = 0;             // last use (least recently used slot is reused)
};
inline void destroy_query_graph(QueryGraph& g) {
  if (g.pre) (void)hipGraphExecDestroy(g.pre);
  if (g.post) (void)hipGraphExecDestroy(g.post);
  g = QueryGraph{};
}

struct Index {
  explicit Index(const snn_device& d) : arena(d) {}
  DeviceArena arena;
  int64_t n = 0;
  int d = 0;
  int dp = 4;  // padded float64 row stride (multiple of 4)
  snn_dtype dtype = SNN_F32;

  Buffer mu;    // d doubles
  Buffer v;     // d doubles (unit)
  Buffer key;   // n doubles: fl32(score) in ascending order
  Buffer perm;  // n int32: sorted position -> original id
  Buffer po;    // n x d input dtype: original rows, sorted
  Buffer p64;   // n x dp doubles: original rows, sorted, zero-padded (filled on the first fp64 screen: p64_ready)
  Buffer ys;    // n x d floats: fl32(p - mu), sorted
  Buffer h;     // n + 32 floats: ||ys||^2 / 2 rounded to nearest, sorted; padding +inf
  Buffer ynorm; // n floats: ||ys|| rounded up, sorted
  MixedOperands mixed[3];  // bf16 one term, bf16 hi/lo, fp16 (mixed_slot)
  Buffer vcand;            // fp32 screen candidate operand blocks (k_cand_mfma32)
  bool vcand_built = false;
  bool p64_ready = false;  // p64 holds the rows (only the fp64 screen reads them)
  Buffer wcells;           // window_table_cells(n) + 1 int32: grid cells of the sorted scores
  int wcells_n = 0;
  bool wcells_built = false;

  double max_norm = 0;  // max ||ys_i|| (float64, rounded up)
  double vnorm = 1;     // ||v|| (float64, rounded up)
  double key_eps = 0;   // bound on |key_i - v.(p_i - mu)|
  int power_iters = 0;

  uint64_t epoch = 0;   // raised by every change of the indexed rows

  // one allocation holding key, perm, po, p64, ys, h and ynorm as views
  // (each allocation may cross into the caller's allocator)
  Buffer rows;

  // per-call workspace (grow-only)
  Buffer ws[16];
  QueryGraph qgraphs[4];
  uint64_t qgraph_clock = 0;
  // stats timing (created on first use): call start, screen start and end,
  // call end, then the stage boundaries of a profiled call
  hipEvent_t ev[8] = {};
  Buffer stats_host_dev;  // small device block read back at the end of a query
  void* host_ctl = nullptr;  // pinned host copy of a query's control block (hipHostMalloc)
};

// ---------------------------------------------------------------- launchers
// (each defined in the kernel file named in the comment)

// k_sort.hip
void radix_sort_pairs(DeviceArena& a, uint32_t* keys, uint32_t* vals, int64_t n, int begin_bit, int end_bit,
                      hipStream_t s);
size_t radix_sort_ws_bytes(int64_t n);
// kres/vres: leave the result where the last pass wrote it and return those
// pointers (no copy back into keys/vals).  err: a device int, nonzero after
// the work if a look-back wait ran out (then the order is wrong); the caller
// must read it back; without it the sort uses the scan that needs no check.
void radix_sort_pairs_ws(uint32_t* keys, uint32_t* vals, int64_t n, int begin_bit, int end_bit, void* ws,
                         hipStream_t s, uint32_t** kres = nullptr, uint32_t** vres = nullptr, int* err = nullptr);
size_t scan_scratch_bytes(int64_t n);
// Exclusive scan of int32 counts into int64 offsets (out has n+1 entries,
// out[n] = total).  scratch: scan_scratch_bytes(n).
void exclusive_scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, void* scratch, hipStream_t s);
void exclusive_scan_u32(uint32_t* data, int64_t n, void* scratch, hipStream_t s);
// Single-pass exclusive scans (decoupled look-back, one launch): state holds
// lookback_words(n) 64-bit words that must be zero before the launch; *err
// is set if a wait for an earlier tile did not end (not expected).
size_t lookback_words(int64_t n);
void lookback_scan_u32(uint32_t* data, int64_t n, unsigned long long* state, int* err, hipStream_t s);

// k_index.hip
void build_index(Index& ix, const void* X);
// screen operands of one OperandKind (bf16, bf16 hi/lo or fp16) for the current rows
void build_mixed_operands(Index& ix, int kind);
// fills ix.p64 from the sorted rows ix.po on the index's stream, once per index version
void build_rows64(Index& ix);
// appends k rows (ids n .. n+k-1) with the index's mu and v: merged into the
// key order, bounds updated, screen operands marked for rebuilding
void insert_points(Index& ix, const void* X, int64_t k);

// k_query.hip / k_cand_*.hip / k_csr.hip are driven from runtime.hip through
// the declarations in query_plan.h.

}  // namespace snn
