// The batching form: many independent instances (data, queries, radius) run
// as one captured HIP graph of batched kernels, with the candidate screen of
// every instance in one persistent launch.  Tile shapes (candidates per work
// unit, tiles per work group) come from a small autotuner that times the
// captured query graph on the batch itself.
//
// A plan fixes the instance sizes; the data in the caller's buffers and the
// output arrays may change between runs (the output table is uploaded before
// each run, the data are read by the graph).  Per-instance screen operand
// terms (1 or 3 bf16 terms per coordinate) are chosen once, at creation, from
// the width of each instance's rounding band relative to R^2; any choice keeps
// the result exact.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "batch_plan.h"
#include "snn_internal.h"

namespace snn {

namespace {

constexpr int kChunkRows = 4096;  // rows per chunk of the centring / Gram passes
constexpr int kPowerIters = 100;

int pad16(int x) { return (x + 15) / 16 * 16; }
int64_t ceil32(int64_t x) { return (x + 31) / 32 * 32; }
int bits_for(int count) {
  int b = 1;
  while ((1 << b) < count) ++b;
  return b;
}

struct TuneCache {
  std::mutex mu;
  std::map<std::string, std::pair<int, int>> mem;
};
TuneCache& tune_cache() {
  static TuneCache c;
  return c;
}

}  // namespace

// Read-back of one run.
struct RunResult {
  BatchCtl ctl{};
  std::vector<int64_t> nnz;
  int64_t total = 0;
  float graph_ms = 0, screen_ms = -1;
  float stage_ms[SNN_STAGES] = {-1, -1, -1, -1, -1};
};

struct BatchPlan {
  explicit BatchPlan(const snn_device& d) : arena(d) {}
  DeviceArena arena;
  hipStream_t cap_stream = nullptr;  // private stream used for capture only
  snn_dtype dtype = SNN_F32;
  int count = 0;
  std::vector<snn_instance> src;
  std::vector<BatchInst> inst;
  std::vector<int64_t> in_off, qin_off;
  std::vector<int32_t> tile_inst, chunk_inst;
  std::vector<int64_t> chunk_r0, chunk_r1;
  int64_t N = 0, M = 0, NR = 0, MS = 0, P64 = 0, Q64 = 0, GRAM = 0;
  int ntiles = 0, nchunks = 0, dmax = 1, vec_total = 0, ibits = 1;
  int KA = 16, T = 512, CH = 4096, G = 8, max_terms = 1;
  int NK32 = 0, D32 = 0, DV32 = 0;  // fp32 screen row shape (NK32 = 0: no fp32 instance)
  int n16 = 0;                      // instances on the 16-bit screen
  int screen_grid = 0, screen_grid32 = 0;
  int64_t sv_cap = 0, stage_cap = 0;

  // device memory
  Buffer tables;  // inst, offsets, tile / chunk tables, outs
  Buffer index;   // index pass arrays
  Buffer query;   // query pass arrays
  Buffer surv;    // survivors
  Buffer stage;   // CSR staging + merge temporaries

  // carved pointers
  BatchInst* d_inst = nullptr;
  BatchDyn* d_dyn = nullptr;
  int64_t *d_in_off = nullptr, *d_qin_off = nullptr;
  int32_t *d_tile_inst = nullptr, *d_chunk_inst = nullptr;
  int64_t *d_chunk_r0 = nullptr, *d_chunk_r1 = nullptr;
  BatchOut* d_outs = nullptr;
  double *mu = nullptr, *v = nullptr, *C = nullptr, *part1 = nullptr, *part2 = nullptr;
  uint32_t *ukey = nullptr, *val = nullptr, *ikey = nullptr, *idx = nullptr;
  void* sort_ws = nullptr;
  double *key = nullptr, *p64 = nullptr;
  int32_t* perm = nullptr;
  float* h = nullptr;
  uint16_t* cop = nullptr;
  float* cop32 = nullptr;
  uint32_t *qkey = nullptr, *qval = nullptr, *qikey = nullptr, *qidx = nullptr;
  double *qa_in = nullptr, *qn_in = nullptr, *q64 = nullptr, *qa = nullptr, *qn = nullptr;
  int32_t* qorig = nullptr;
  uint16_t* qop = nullptr;
  float* cthr = nullptr;
  float* vq32 = nullptr;
  int32_t *tlo = nullptr, *thi = nullptr, *units = nullptr;
  int64_t* group_off = nullptr;
  int32_t* gbase = nullptr;
  // the fp32 screen's tile windows and work units (its own tile plan)
  int32_t *tlo32 = nullptr, *thi32 = nullptr, *units32 = nullptr;
  int64_t* group_off32 = nullptr;
  int32_t* gbase32 = nullptr;
  void* scan_ws = nullptr;
  BatchCtl* ctl = nullptr;
  int32_t* row_cnt = nullptr;  // per query slot
  int32_t* cnt_o = nullptr;    // per output row
  int64_t* rp_s = nullptr;     // slot-order row offsets
  int64_t* rp_sg = nullptr;    // the same, zero when the staging arrays overflowed
  int64_t *row_ptr = nullptr, *nnz_base = nullptr, *nnz = nullptr;  // output order
  int32_t* lists = nullptr;
  Survivors sv{};
  uint64_t* key_s = nullptr;                     // neighbour keys in slot-order rows
  int32_t *col_o = nullptr, *tmp_col = nullptr;  // output order, merges
  float *dist_o = nullptr, *tmp_dist = nullptr;

  // graphs: index pass, query pass, both
  hipGraphExec_t g_index = nullptr, g_query = nullptr, g_all = nullptr;
  bool f16 = false;           // the 16-bit screen on fp16 operands (every instance), else bf16
  bool screen_timed = false;  // device clock stamps bracket the screen in the query graph
  bool profiled = false;      // ... and every stage of the query pass (SNN_PROFILE at creation)
  double clock_khz = 0;       // frequency of that clock
  float last_tune_ms = 0;
  RunResult last;  // read-back of the latest query pass

  BatchDev dev() const {
    BatchDev b{};
    b.inst = d_inst;
    b.dyn = d_dyn;
    b.in_off = d_in_off;
    b.qin_off = d_qin_off;
    b.tile_inst = d_tile_inst;
    b.count = count;
    b.T = T;
    b.KA = KA;
    b.ntiles = ntiles;
    b.NK32 = NK32;
    b.D32 = D32;
    b.DV32 = DV32;
    b.cop32 = cop32;
    b.vq32 = vq32;
    b.N = N;
    b.M = M;
    b.NR = NR;
    b.MS = MS;
    return b;
  }
};

namespace {

void destroy_graphs(BatchPlan& p) {
  for (hipGraphExec_t* g : {&p.g_index, &p.g_query, &p.g_all}) {
    if (*g) (void)hipGraphExecDestroy(*g);
    *g = nullptr;
  }
}

// ---- layout ------------------------------------------------------------------
void plan_layout(BatchPlan& p) {
  const int I = p.count;
  p.in_off.assign(I + 1, 0);
  p.qin_off.assign(I + 1, 0);
  p.tile_inst.clear();
  p.chunk_inst.clear();
  p.chunk_r0.clear();
  p.chunk_r1.clear();
  int64_t row = 0, p64o = 0, slot = 0, q64o = 0, gram = 0;
  int vec = 0, tiles = 0;
  p.dmax = 1;
  for (int i = 0; i < I; ++i) {
    BatchInst& b = p.inst[i];
    p.dmax = std::max(p.dmax, b.d);
    b.in_off = p.in_off[i];
    p.in_off[i + 1] = p.in_off[i] + b.n;
    b.qin_off = p.qin_off[i];
    p.qin_off[i + 1] = p.qin_off[i] + b.m;
    b.row_base = row;
    row += ceil32(b.n);
    b.p64_off = p64o;
    p64o += ceil32(b.n) * b.dp;
    b.ntiles = (int)((b.m + p.T - 1) / p.T);
    b.tile_base = tiles;
    b.slot_base = (int64_t)tiles * p.T;
    b.q64_off = q64o;
    q64o += (int64_t)b.ntiles * p.T * b.dp;
    for (int t = 0; t < b.ntiles; ++t) p.tile_inst.push_back(i);
    tiles += b.ntiles;
    b.gram_off = gram;
    gram += (int64_t)b.d * b.d;
    b.vec_off = vec;
    vec += b.d;
    b.chunk_base = (int)p.chunk_inst.size();
    for (int64_t r = 0; r < b.n; r += kChunkRows) {
      p.chunk_inst.push_back(i);
      p.chunk_r0.push_back(r);
      p.chunk_r1.push_back(std::min<int64_t>(b.n, r + kChunkRows));
    }
    b.nchunks = (int)p.chunk_inst.size() - b.chunk_base;
  }
  p.N = p.in_off[I];
  p.M = p.qin_off[I];
  p.NR = row;
  p.P64 = p64o;
  p.Q64 = q64o;
  p.GRAM = gram;
  p.vec_total = vec;
  p.ntiles = tiles;
  p.MS = (int64_t)tiles * p.T;
  p.nchunks = (int)p.chunk_inst.size();
  p.ibits = bits_for(I);
  if (p.NR >= (int64_t)INT32_MAX || p.MS >= (int64_t)INT32_MAX)
    fail(SNN_EINVAL, "batch too large: more than 2^31 rows or query slots in total");
}

// ---- device memory -------------------------------------------------------------
void alloc_tables(BatchPlan& p) {
  auto carve = [&](Carver& c) {
    p.d_inst = c.take<BatchInst>(p.count);
    p.d_dyn = c.take<BatchDyn>(p.count);
    p.d_in_off = c.take<int64_t>(p.count + 1);
    p.d_qin_off = c.take<int64_t>(p.count + 1);
    p.d_tile_inst = c.take<int32_t>(std::max(p.ntiles, 1));
    p.d_chunk_inst = c.take<int32_t>(p.nchunks);
    p.d_chunk_r0 = c.take<int64_t>(p.nchunks);
    p.d_chunk_r1 = c.take<int64_t>(p.nchunks);
    p.d_outs = c.take<BatchOut>(p.count);
  };
  Carver probe(nullptr);
  carve(probe);
  p.tables.ensure(p.arena, probe.off + 256);
  Carver c(p.tables.ptr);
  carve(c);
  hipStream_t s = p.arena.stream();
  SNN_HIP(hipMemcpyAsync(p.d_inst, p.inst.data(), sizeof(BatchInst) * p.count, hipMemcpyHostToDevice, s));
  SNN_HIP(hipMemcpyAsync(p.d_in_off, p.in_off.data(), sizeof(int64_t) * (p.count + 1), hipMemcpyHostToDevice, s));
  SNN_HIP(hipMemcpyAsync(p.d_qin_off, p.qin_off.data(), sizeof(int64_t) * (p.count + 1), hipMemcpyHostToDevice, s));
  if (p.ntiles)
    SNN_HIP(hipMemcpyAsync(p.d_tile_inst, p.tile_inst.data(), sizeof(int32_t) * p.ntiles, hipMemcpyHostToDevice, s));
  SNN_HIP(hipMemcpyAsync(p.d_chunk_inst, p.chunk_inst.data(), sizeof(int32_t) * p.nchunks, hipMemcpyHostToDevice, s));
  SNN_HIP(hipMemcpyAsync(p.d_chunk_r0, p.chunk_r0.data(), sizeof(int64_t) * p.nchunks, hipMemcpyHostToDevice, s));
  SNN_HIP(hipMemcpyAsync(p.d_chunk_r1, p.chunk_r1.data(), sizeof(int64_t) * p.nchunks, hipMemcpyHostToDevice, s));
  SNN_HIP(hipStreamSynchronize(s));
}

void alloc_index(BatchPlan& p, bool with_operands) {
  auto carve = [&](Carver& c) {
    p.mu = c.take<double>(p.vec_total);
    p.v = c.take<double>(p.vec_total);
    p.C = c.take<double>(p.GRAM);
    p.part1 = c.take<double>((size_t)p.nchunks * kBatchMaxD);
    p.part2 = c.take<double>((size_t)p.nchunks * p.dmax * p.dmax);
    p.ukey = c.take<uint32_t>(p.N);
    p.val = c.take<uint32_t>(p.N);
    p.ikey = c.take<uint32_t>(p.N);
    p.idx = c.take<uint32_t>(p.N);
    p.sort_ws = c.take<char>(radix_sort_ws_bytes(std::max(p.N, p.M)));
    p.key = c.take<double>(p.NR);
    p.perm = c.take<int32_t>(p.NR);
    p.p64 = nullptr;  // (the recheck reads the caller's rows)
    p.h = c.take<float>(p.NR);
    p.cop = c.take<uint16_t>(with_operands ? (size_t)p.NR * p.KA : 1);
    p.cop32 = c.take<float>(with_operands && p.NK32 ? (size_t)p.NR * p.D32 : 1);
  };
  Carver probe(nullptr);
  carve(probe);
  p.index.ensure(p.arena, probe.off + 256);
  Carver c(p.index.ptr);
  carve(c);
}

void alloc_query(BatchPlan& p) {
  const int64_t M = std::max<int64_t>(p.M, 1), MS = std::max<int64_t>(p.MS, 1);
  const int nt = std::max(p.ntiles, 1);
  auto carve = [&](Carver& c) {
    p.qkey = c.take<uint32_t>(M);
    p.qval = c.take<uint32_t>(M);
    p.qikey = c.take<uint32_t>(M);
    p.qidx = c.take<uint32_t>(M);
    p.qa_in = c.take<double>(M);
    p.qn_in = c.take<double>(M);
    p.q64 = nullptr;
    p.qa = c.take<double>(MS);
    p.qn = c.take<double>(MS);
    p.qorig = c.take<int32_t>(MS);
    p.qop = c.take<uint16_t>((size_t)MS * p.KA);
    p.cthr = c.take<float>(MS);
    p.vq32 = c.take<float>(p.NK32 ? (size_t)MS * p.DV32 : 1);
    p.tlo = c.take<int32_t>(nt);
    p.thi = c.take<int32_t>(nt);
    p.units = c.take<int32_t>(nt);
    p.group_off = c.take<int64_t>(nt + 1);
    p.gbase = c.take<int32_t>(nt);
    const int nt32 = p.NK32 ? nt : 1;
    p.tlo32 = c.take<int32_t>(nt32);
    p.thi32 = c.take<int32_t>(nt32);
    p.units32 = c.take<int32_t>(nt32);
    p.group_off32 = c.take<int64_t>(nt32 + 1);
    p.gbase32 = c.take<int32_t>(nt32);
    p.scan_ws = c.take<char>(std::max(scan_scratch_bytes(nt + 1), scan_scratch_bytes(MS + 1)));
    p.ctl = c.take<BatchCtl>(1);
    p.row_cnt = c.take<int32_t>(MS);
    p.rp_s = c.take<int64_t>(MS + 1);
    p.rp_sg = c.take<int64_t>(MS + 1);
    p.cnt_o = c.take<int32_t>(M);
    p.row_ptr = c.take<int64_t>(M + 1);
    p.nnz_base = c.take<int64_t>(p.count + 1);
    p.nnz = c.take<int64_t>(p.count);
    p.lists = c.take<int32_t>((size_t)row_sort_lists() * MS);
  };
  Carver probe(nullptr);
  carve(probe);
  p.query.ensure(p.arena, probe.off + 256);
  Carver c(p.query.ptr);
  carve(c);
}

void alloc_survivors(BatchPlan& p, int64_t cap) {
  p.surv.reset(p.arena);
  auto carve = [&](Carver& c) {
    p.sv.pairs = c.take<int2>(cap);
    p.sv.res_q = c.take<int32_t>(cap);
    p.sv.res_key = c.take<uint64_t>(cap);
    p.sv.res_slot = c.take<int32_t>(cap);
  };
  Carver probe(nullptr);
  carve(probe);
  p.surv.ensure(p.arena, probe.off + 256);
  Carver c(p.surv.ptr);
  carve(c);
  p.sv.cap = cap;
  p.sv.per = 1;
  p.sv.count = &p.ctl->survivors;
  p.sv_cap = cap;
}

void alloc_stage(BatchPlan& p, int64_t cap) {
  p.stage.reset(p.arena);
  cap = std::max<int64_t>(cap, 1);
  auto carve = [&](Carver& c) {
    p.key_s = c.take<uint64_t>(cap);
    p.col_o = c.take<int32_t>(cap);
    p.dist_o = c.take<float>(cap);
    p.tmp_col = c.take<int32_t>(cap);
    p.tmp_dist = c.take<float>(cap);
  };
  Carver probe(nullptr);
  carve(probe);
  p.stage.ensure(p.arena, probe.off + 256);
  Carver c(p.stage.ptr);
  carve(c);
  p.stage_cap = cap;
}

// ---- the two passes as kernel sequences (eager or captured) -----------------------
void enqueue_index(BatchPlan& p, hipStream_t s, bool full) {
  const BatchDev b = p.dev();
  launch_fill_u64(reinterpret_cast<unsigned long long*>(p.d_dyn), (int64_t)p.count * sizeof(BatchDyn) / 8, 0ull, s);
  batch_colsum(p.dtype, b, p.nchunks, p.d_chunk_inst, p.d_chunk_r0, p.d_chunk_r1, p.part1, p.mu, s);
  batch_gram(p.dtype, b, p.nchunks, p.dmax, p.d_chunk_inst, p.d_chunk_r0, p.d_chunk_r1, p.mu, p.part2, p.C, s);
  batch_power(b, p.C, kPowerIters, p.v, s);
  batch_project(p.dtype, b, p.mu, p.v, p.ukey, p.val, s);
  if (!full) return;  // sizing pre-pass: only the norms are needed
  radix_sort_pairs_ws(p.ukey, p.val, p.N, 0, 32, p.sort_ws, s);
  batch_inst_keys(p.d_in_off, p.count, p.val, p.N, p.ikey, p.idx, s);
  radix_sort_pairs_ws(p.ikey, p.idx, p.N, 0, p.ibits, p.sort_ws, s);
  batch_finalize(b, s);
  batch_gather(p.dtype, b, p.mu, p.ukey, p.val, p.ikey, p.idx, p.key, p.perm, p.p64, p.h, p.cop, s);
  batch_pad_rows(b, p.h, p.perm, p.cop, s);
}

void enqueue_query(BatchPlan& p, hipStream_t s, bool timed) {
  const BatchDev b = p.dev();
  const DeviceInfo& di = device_info(p.arena.dev().device);
  launch_query_init(reinterpret_cast<unsigned long long*>(p.ctl), (int)(sizeof(BatchCtl) / 8), p.row_cnt,
                    p.M ? p.MS : 0, nullptr, 0, p.tlo, p.thi, p.M ? p.ntiles : 0, s);
  if (p.M == 0) {
    batch_zero_i64(p.row_ptr, 1, s);
    batch_outputs(b, p.d_outs, p.row_ptr, p.col_o, p.dist_o, p.stage_cap, p.nnz_base, p.nnz, s);
    return;
  }
  const bool prof = timed && p.profiled;
  if (prof) batch_stamp(&p.ctl->stamp[0], s);
  batch_query_keys(p.dtype, b, p.mu, p.v, p.qkey, p.qval, p.qa_in, p.qn_in, p.ctl, s);
  radix_sort_pairs_ws(p.qkey, p.qval, p.M, 0, 32, p.sort_ws, s);
  batch_inst_keys(p.d_qin_off, p.count, p.qval, p.M, p.qikey, p.qidx, s);
  radix_sort_pairs_ws(p.qikey, p.qidx, p.M, 0, p.ibits, p.sort_ws, s);
  batch_query_pad(b, p.qorig, p.qa, p.qn, p.qop, p.cthr, s);
  batch_query_gather(p.dtype, b, p.mu, p.qval, p.qikey, p.qidx, p.qa_in, p.qn_in, p.q64, p.qorig, p.qa, p.qn, p.qop,
                     p.cthr, s);
  if (prof) batch_stamp(&p.ctl->stamp[1], s);
  batch_windows(b, p.key, p.qa, p.qn, p.qorig, p.tlo, p.thi, p.ctl, s);
  const int ngroups = (p.ntiles + p.G - 1) / p.G;
  // instances on the fp32 screen get a tile plan of their own (the tiles of
  // the other screen empty in each plan), so each screen's persistent launch
  // takes only its own work units
  if (p.NK32) batch_split_tiles(b, p.tlo, p.thi, p.tlo32, p.thi32, s);
  launch_tile_plan(p.tlo, p.thi, p.ntiles, p.CH, 32, 0, p.units, p.G, p.group_off, p.gbase, p.T, p.MS, 1, nullptr,
                   nullptr, 0, nullptr, s);
  batch_executed(b, p.tlo, p.thi, p.T / 4, p.ctl, s);
  if (p.NK32) {
    launch_tile_plan(p.tlo32, p.thi32, p.ntiles, p.CH, 32, 0, p.units32, p.G, p.group_off32, p.gbase32, p.T, p.MS, 1,
                     nullptr, nullptr, 0, nullptr, s);
    batch_executed(b, p.tlo32, p.thi32, p.T / 4, p.ctl, s);
  }

  QueryDev qd{};
  qd.m = p.MS;
  qd.T = p.T;
  qd.CH = p.CH;
  qd.ntiles = p.ntiles;
  qd.G = p.G;
  qd.ngroups = ngroups;
  qd.tlo = p.tlo;
  qd.thi = p.thi;
  qd.units = p.units;
  qd.group_off = p.group_off;
  qd.gbase = p.gbase;
  qd.counters = p.ctl->counters;
  qd.nxcd = di.xcds;
  qd.sink.out = p.sv.pairs;
  qd.sink.counter = p.sv.count;
  qd.sink.cap = p.sv.cap;
  MixedDev mx{};
  mx.qop = p.qop;
  mx.cthr = p.cthr;
  mx.cop = p.cop;
  mx.h = p.h;
  mx.KA = p.KA;
  mx.KB = p.KA;
  mx.f16 = p.f16 ? 1 : 0;
  if (timed) batch_stamp(&p.ctl->stamp[2], s);
  if (p.n16) launch_cand_mfma(qd, mx, p.screen_grid, s);
  if (p.NK32) {
    QueryDev q32 = qd;
    q32.tlo = p.tlo32;
    q32.thi = p.thi32;
    q32.units = p.units32;
    q32.group_off = p.group_off32;
    q32.gbase = p.gbase32;
    q32.counters = p.ctl->counters32;
    launch_cand_mfma32_batch(q32, Mfma32Dev{p.vq32, p.DV32, p.D32, p.cop32, p.h}, p.screen_grid32, s);
  }
  if (timed) batch_stamp(&p.ctl->stamp[3], s);

  // neighbours are assembled in slot order (a tile's rows are contiguous),
  // then each row is sorted on its way to its output row
  batch_recheck(p.dtype, b, p.sv, p.qorig, p.perm, p.row_cnt, di.cus * 16, s);
  if (prof) batch_stamp(&p.ctl->stamp[4], s);
  exclusive_scan_i32_to_i64(p.row_cnt, p.rp_s, p.MS, p.scan_ws, s);
  launch_perm_counts(p.rp_s, p.MS, p.qorig, p.cnt_o, s);
  exclusive_scan_i32_to_i64(p.cnt_o, p.row_ptr, p.M, p.scan_ws, s);
  batch_scatter(p.sv, p.rp_s, p.MS, p.key_s, p.stage_cap, di.cus * 16, s);
  batch_rowptr_guard(p.rp_s, p.MS, p.stage_cap, p.rp_sg, s);
  const RowMove mv{p.rp_sg, p.key_s, p.qorig, p.row_ptr, p.col_o, p.dist_o};
  launch_row_sort_move(mv, p.MS, INT64_MAX, p.lists, p.ctl->list_counts, p.tmp_col, p.tmp_dist, s);
  batch_outputs(b, p.d_outs, p.row_ptr, p.col_o, p.dist_o, p.stage_cap, p.nnz_base, p.nnz, s);
  if (prof) batch_stamp(&p.ctl->stamp[5], s);
}

template <class F>
hipGraphExec_t capture(BatchPlan& p, F&& body) {
  hipStream_t s = p.cap_stream;
  // (begin and end of a capture are checked only when they fail: an injected
  // failure would leave the stream capturing or the graph unowned)
  const hipError_t eb = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (eb != hipSuccess) check_hip(eb, "hipStreamBeginCapture", __FILE__, __LINE__);
  hipGraph_t graph = nullptr;
  try {
    body(s);
  } catch (...) {
    (void)hipStreamEndCapture(s, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    throw;
  }
  {
    const hipError_t ee = hipStreamEndCapture(s, &graph);
    if (ee != hipSuccess) check_hip(ee, "hipStreamEndCapture", __FILE__, __LINE__);
  }
  hipGraphExec_t exec = nullptr;
  hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  SNN_HIP(e);
  return exec;
}

void build_graphs(BatchPlan& p) {
  destroy_graphs(p);
  p.g_index = capture(p, [&](hipStream_t s) { enqueue_index(p, s, true); });
  p.g_query = capture(p, [&](hipStream_t s) { enqueue_query(p, s, true); });
  p.g_all = capture(p, [&](hipStream_t s) {
    enqueue_index(p, s, true);
    enqueue_query(p, s, false);
  });
}

void upload_outputs(BatchPlan& p, std::vector<BatchOut>& host) {
  host.resize(p.count);
  for (int i = 0; i < p.count; ++i) {
    const snn_csr* o = p.src[i].out;
    if (!o || !o->row_ptr) fail(SNN_EINVAL, "instance " + std::to_string(i) + ": out / out->row_ptr is NULL");
    if (o->nnz_cap < 0) fail(SNN_EINVAL, "instance " + std::to_string(i) + ": nnz_cap < 0");
    if (o->nnz_cap > 0 && (!o->col || !o->dist))
      fail(SNN_EINVAL, "instance " + std::to_string(i) + ": out->col / out->dist is NULL");
    host[i] = BatchOut{o->row_ptr, o->col, o->dist, o->nnz_cap};
  }
  SNN_HIP(hipMemcpyAsync(p.d_outs, host.data(), sizeof(BatchOut) * p.count, hipMemcpyHostToDevice,
                         p.arena.stream()));
}

// One launch of a graph (or of both passes) plus the read-back; grows the
// survivor list or the staging arrays and runs the query pass again when
// either overflowed.
RunResult run_graphs(BatchPlan& p, bool do_index, bool do_query) {
  hipStream_t s = p.arena.stream();
  std::vector<BatchOut> outs;
  upload_outputs(p, outs);
  RunResult rr;
  rr.nnz.assign(p.count, 0);
  hipEvent_t e0, e1;
  SNN_HIP(hipEventCreate(&e0));
  SNN_HIP(hipEventCreate(&e1));
  struct EvGuard {
    hipEvent_t a, b;
    ~EvGuard() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } eg{e0, e1};
  bool index_pending = do_index;
  for (int attempt = 0; attempt < 8; ++attempt) {
    SNN_HIP(hipEventRecord(e0, s));
    if (index_pending && do_query)
      SNN_HIP(hipGraphLaunch(p.g_all, s));
    else if (index_pending)
      SNN_HIP(hipGraphLaunch(p.g_index, s));
    else if (do_query)
      SNN_HIP(hipGraphLaunch(p.g_query, s));
    SNN_HIP(hipEventRecord(e1, s));
    index_pending = false;
    // one read-back into page-locked memory (pageable copies are staged)
    const size_t o_ctl = align256(sizeof(BatchDyn) * p.count), o_nnz = o_ctl + align256(sizeof(BatchCtl)),
                 o_tot = o_nnz + align256(sizeof(int64_t) * p.count);
    char* hb = static_cast<char*>(pinned_host(o_tot + sizeof(int64_t)));
    SNN_HIP(hipMemcpyAsync(hb, p.d_dyn, sizeof(BatchDyn) * p.count, hipMemcpyDeviceToHost, s));
    SNN_HIP(hipMemcpyAsync(hb + o_ctl, p.ctl, sizeof(BatchCtl), hipMemcpyDeviceToHost, s));
    SNN_HIP(hipMemcpyAsync(hb + o_nnz, p.nnz, sizeof(int64_t) * p.count, hipMemcpyDeviceToHost, s));
    SNN_HIP(hipMemcpyAsync(hb + o_tot, p.nnz_base + p.count, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SNN_HIP(hipStreamSynchronize(s));
    std::vector<BatchDyn> dyn(p.count);
    std::memcpy(dyn.data(), hb, sizeof(BatchDyn) * p.count);
    std::memcpy(&rr.ctl, hb + o_ctl, sizeof(BatchCtl));
    std::memcpy(rr.nnz.data(), hb + o_nnz, sizeof(int64_t) * p.count);
    std::memcpy(&rr.total, hb + o_tot, sizeof(int64_t));
    SNN_HIP(hipEventElapsedTime(&rr.graph_ms, e0, e1));
    for (int i = 0; i < p.count; ++i)
      if (dyn[i].bad) fail(SNN_EINVAL, "instance " + std::to_string(i) + ": X contains NaN or Inf");
    if (!do_query) return rr;
    if (rr.ctl.qbad) fail(SNN_EINVAL, "some Q contains NaN or Inf");
    const bool sv_over = (int64_t)rr.ctl.survivors > p.sv_cap;
    const bool st_over = !sv_over && rr.total > p.stage_cap;
    if (!sv_over && !st_over) {
      rr.screen_ms = -1;
      const unsigned long long* t = rr.ctl.stamp;
      if (!do_index && p.M > 0 && p.clock_khz > 0 && t[3] > t[2])
        rr.screen_ms = (float)((double)(t[3] - t[2]) / p.clock_khz);
      if (!do_index && p.M > 0 && p.profiled)
        for (int k = 0; k < SNN_STAGES; ++k)
          rr.stage_ms[k] = t[k + 1] >= t[k] ? (float)((double)(t[k + 1] - t[k]) / p.clock_khz) : -1.0f;
      p.last = rr;
      return rr;
    }
    log_line(3, "batch: %s overflowed (%llu survivors, %lld neighbours): growing and running the query pass again",
             sv_over ? "survivor list" : "staging arrays", rr.ctl.survivors, (long long)rr.total);
    if (sv_over) alloc_survivors(p, (int64_t)rr.ctl.survivors * 5 / 4 + 4096);
    if (st_over) alloc_stage(p, rr.total * 5 / 4 + 4096);
    build_graphs(p);
  }
  fail(SNN_EDEVICE, "batch: survivor / staging sizes did not settle");
}

// ---- autotuner ---------------------------------------------------------------------
std::string tune_key(const BatchPlan& p) {
  // the shape of the work: operand width, tile size, instance mix and totals
  std::map<std::pair<int, int>, int> mix;
  for (const BatchInst& b : p.inst) mix[{b.d, b.terms}]++;
  std::ostringstream k;
  k << "gfx950 KA=" << p.KA << (p.f16 ? " f16" : "") << " T=" << p.T << " I=" << p.count << " logN=" << (int)std::log2((double)p.N + 1)
    << " logM=" << (int)std::log2((double)p.M + 1);
  for (auto& e : mix) k << " d" << e.first.first << "t" << e.first.second << "x" << e.second;
  return k.str();
}

bool cache_lookup(const std::string& key, const char* path, int& CH, int& G) {
  TuneCache& tc = tune_cache();
  std::lock_guard<std::mutex> lk(tc.mu);
  auto it = tc.mem.find(key);
  if (it != tc.mem.end()) {
    CH = it->second.first;
    G = it->second.second;
    return true;
  }
  if (!path || !*path) return false;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    const size_t tab = line.find('\t');
    if (tab == std::string::npos || line.substr(0, tab) != key) continue;
    int a = 0, b = 0;
    if (std::sscanf(line.c_str() + tab + 1, "%d %d", &a, &b) == 2 && a > 0 && b > 0) {
      tc.mem[key] = {a, b};
      CH = a;
      G = b;
      return true;
    }
  }
  return false;
}

void cache_store(const std::string& key, const char* path, int CH, int G) {
  TuneCache& tc = tune_cache();
  std::lock_guard<std::mutex> lk(tc.mu);
  tc.mem[key] = {CH, G};
  if (!path || !*path) return;
  std::ofstream f(path, std::ios::app);
  if (f) f << key << '\t' << CH << ' ' << G << '\n';
}

// Times the captured query pass for every candidate (CH, G) on this batch
// and keeps the fastest; each candidate runs once to warm up, then the
// minimum of three timed launches counts.
void autotune(BatchPlan& p, const char* cache_path) {
  const std::string key = tune_key(p);
  int CH = 0, G = 0;
  if (cache_lookup(key, cache_path, CH, G)) {
    p.CH = CH;
    p.G = G;
    return;
  }
  hipStream_t s = p.arena.stream();
  float best = INFINITY;
  int bCH = p.CH, bG = p.G;
  for (int ch : {1024, 2048, 4096, 8192}) {
    for (int g : {4, 8, 16}) {
      p.CH = ch;
      p.G = g;
      build_graphs(p);
      run_graphs(p, false, true);  // warm-up, and settles buffer sizes
      float t = INFINITY;
      for (int r = 0; r < 3; ++r) {
        hipEvent_t a, b;
        SNN_HIP(hipEventCreate(&a));
        SNN_HIP(hipEventCreate(&b));
        SNN_HIP(hipEventRecord(a, s));
        SNN_HIP(hipGraphLaunch(p.g_query, s));
        SNN_HIP(hipEventRecord(b, s));
        SNN_HIP(hipEventSynchronize(b));
        float ms = 0;
        SNN_HIP(hipEventElapsedTime(&ms, a, b));
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        t = std::min(t, ms);
      }
      if (t < best) {
        best = t;
        bCH = ch;
        bG = g;
      }
    }
  }
  p.CH = bCH;
  p.G = bG;
  p.last_tune_ms = best;
  cache_store(key, cache_path, bCH, bG);
}

void free_plan(BatchPlan* p) {
  if (!p) return;
  destroy_graphs(*p);
  for (Buffer* b : {&p->tables, &p->index, &p->query, &p->surv, &p->stage}) b->reset(p->arena);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  delete p;
}

void fill_stats(const BatchPlan& p, const RunResult& rr, snn_stats* st) {
  if (!st) return;
  st->pairs_window = (int64_t)rr.ctl.pairs_window;
  st->pairs_executed = (int64_t)rr.ctl.executed;
  st->pairs_recheck = (int64_t)rr.ctl.survivors;
  st->nnz = rr.total;
  st->precision_used = p.f16 ? SNN_PREC_FP16 : SNN_PREC_MIXED;
  st->terms_used = p.max_terms;
  st->screen_ms = rr.screen_ms;
  st->total_ms = rr.graph_ms;
  st->flops_window = (double)rr.ctl.flops;
  for (int k = 0; k < SNN_STAGES; ++k) st->stage_ms[k] = rr.stage_ms[k];
}

void finish_outputs(BatchPlan& p, const RunResult& rr) {
  int over = -1;
  for (int i = 0; i < p.count; ++i) {
    p.src[i].out->nnz = rr.nnz[i];
    if (rr.nnz[i] > p.src[i].out->nnz_cap && over < 0) over = i;
  }
  if (over >= 0) {
    char buf[200];
    std::snprintf(buf, sizeof(buf), "instance %d: CSR capacity %lld < %lld neighbours (see each out->nnz)", over,
                  (long long)p.src[over].out->nnz_cap, (long long)rr.nnz[over]);
    throw Error(SNN_EOVERFLOW, buf);
  }
}

}  // namespace

BatchPlan* create_batch(const snn_device& devc, snn_dtype dtype, const snn_instance* in, int32_t count,
                        const snn_batch_options* opts) {
  if (count < 1 || count > 65536) fail(SNN_EINVAL, "count must be in [1, 65536]");
  if (!in) fail(SNN_EINVAL, "instances is NULL");
  if (dtype != SNN_F32 && dtype != SNN_F64) fail(SNN_EINVAL, "unknown dtype");
  snn_batch_options o{};
  if (opts) o = *opts;
  if (o.mixed_terms != 0 && o.mixed_terms != 1 && o.mixed_terms != 3) fail(SNN_EINVAL, "mixed_terms must be 0, 1 or 3");
  if (o.tile_c < 0 || o.tile_c % 32 != 0) fail(SNN_EINVAL, "tile_c must be a non-negative multiple of 32");
  if (o.tile_g < 0) fail(SNN_EINVAL, "tile_g must be >= 0");
  for (int i = 0; i < count; ++i) {
    const snn_instance& x = in[i];
    const std::string w = "instance " + std::to_string(i) + ": ";
    if (!x.X) fail(SNN_EINVAL, w + "X is NULL");
    if (x.n < 1 || x.n >= (int64_t)INT32_MAX) fail(SNN_EINVAL, w + "n must be in [1, 2^31 - 1)");
    if (x.d < 1 || x.d > kBatchMaxD) fail(SNN_EINVAL, w + "d must be in [1, 128] in a batch");
    if (!std::isfinite(x.R) || x.R < 0) fail(SNN_EINVAL, w + "R must be finite and >= 0");
    if (x.m < 0 || x.m >= (int64_t)INT32_MAX) fail(SNN_EINVAL, w + "m must be in [0, 2^31 - 1)");
    if (!x.Q && x.m != 0 && x.m != x.n) fail(SNN_EINVAL, w + "Q NULL needs m = n (self-query) or m = 0");
    if (!x.out) fail(SNN_EINVAL, w + "out is NULL");
  }
  if ((devc.alloc == nullptr) != (devc.free == nullptr)) fail(SNN_EINVAL, "alloc and free must both be set");
  DeviceScope scope(devc.device);

  BatchPlan* pp = new BatchPlan(devc);
  try {
    BatchPlan& p = *pp;
    p.dtype = dtype;
    p.count = count;
    p.src.assign(in, in + count);
    p.inst.resize(count);
    for (int i = 0; i < count; ++i) {
      BatchInst& b = p.inst[i];
      std::memset(&b, 0, sizeof(b));
      b.X = in[i].X;
      b.Q = in[i].Q ? in[i].Q : in[i].X;
      b.n = in[i].n;
      b.m = in[i].m;
      b.d = in[i].d;
      b.dp = (b.d + 1) / 2 * 2;
      b.terms = 1;
      b.R = in[i].R;
      b.R2 = in[i].R * in[i].R;
    }
    SNN_HIP(hipStreamCreateWithFlags(&p.cap_stream, hipStreamNonBlocking));
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, devc.device) != hipSuccess) {
      (void)hipGetLastError();
      khz = 0;
    }
    p.clock_khz = khz;
    p.screen_timed = khz > 0;
    p.profiled = p.screen_timed && profile_on();

    // pre-pass: centring, direction and norms decide the operand terms
    p.T = 512;
    plan_layout(p);
    alloc_tables(p);
    alloc_index(p, false);
    hipStream_t s = p.arena.stream();
    enqueue_index(p, s, false);
    std::vector<BatchDyn> dyn(count);
    SNN_HIP(hipMemcpyAsync(dyn.data(), p.d_dyn, sizeof(BatchDyn) * count, hipMemcpyDeviceToHost, s));
    SNN_HIP(hipStreamSynchronize(s));
    int KA = 16;
    p.max_terms = 1;
    p.NK32 = 0;
    p.n16 = 0;
    bool all_f16 = o.mixed_terms == 0;
    for (int i = 0; i < count; ++i) {
      if (dyn[i].bad) fail(SNN_EINVAL, "instance " + std::to_string(i) + ": X contains NaN or Inf");
      BatchInst& b = p.inst[i];
      int t = o.mixed_terms;
      if (t == 0) {
        // relative bands 2 c_rep Y^2 / R^2 of one and three bf16 terms (the
        // single-instance policy): one term while its band is <= 0.1 R^2,
        // three while theirs is <= 0.5 R^2, else the fp32 screen for d <= 16
        const double Y = std::sqrt(dyn[i].maxnorm2);
        auto band = [&](int kind) { return b.R2 > 0 ? 2.0 * mixed_c_rep(kind) * Y * Y / b.R2 : INFINITY; };
        // (the bound's Y, rounded up as the index pass rounds it)
        const double Yup = Y * (1.0 + 4.0 * (b.d + 2) * 1.1102230246251565e-16);
        if (!(screen_in_range(kOpF16, Yup) && b.d <= kBatchMaxD && band(kOpF16) <= 1.0)) all_f16 = false;
        if (band(kOpBf16) <= 0.1 || 3 * b.d > kBatchMaxD)
          t = 1;
        else if (band(kOpBf16x3) <= 0.5 || b.d > mfma32_max_d() || !screen_in_range(kOpF32, Y))
          t = 3;
        else
          t = 0;
      }
      if (t == 3 && 3 * b.d > kBatchMaxD) fail(SNN_ENOTSUP, "instance " + std::to_string(i) + ": 3 terms need d <= 42");
      b.terms = t;
      if (t == 0) {
        p.NK32 = std::max(p.NK32, (b.d + 1) / 2);
      } else {
        ++p.n16;
        p.max_terms = std::max(p.max_terms, t);
        KA = std::max(KA, pad16(t * b.d));
      }
    }
    // fp16 operands for every instance when each one's fp16 band is at most
    // R^2 (the single-instance policy), its rows scale into fp16, and the
    // shared operand row gets shorter: one product per coordinate where bf16
    // needs three.  The 16-bit screen of a launch has one operand type and
    // one row length for all instances, so the choice is made for the whole
    // batch; with the same row length the three bf16 terms keep a narrower
    // band (batch256: 10.7e6 against 8.3e6 survivors at the same screen time).
    int KA16 = 16;
    for (const BatchInst& b : p.inst) KA16 = std::max(KA16, pad16(b.d));
    p.f16 = all_f16 && count > 0 && KA16 < KA;
    if (p.f16) {
      p.NK32 = 0;
      p.n16 = count;
      p.max_terms = 1;
      KA = KA16;
      for (BatchInst& b : p.inst) b.terms = kOpF16;
    }
    p.D32 = 2 * p.NK32;
    p.DV32 = p.NK32 ? mfma32_query_floats(p.D32) : 0;
    p.KA = KA;
    p.T = 4 * mixed_queries_per_wave(KA, p.f16);
    if (p.NK32 && p.T != mfma32_batch_queries_per_tile())
      fail(SNN_EDEVICE, "internal: the fp32 and 16-bit screens need one tile size");
    p.CH = o.tile_c ? o.tile_c : 4096;
    p.G = o.tile_g ? o.tile_g : 8;
    plan_layout(p);
    p.index.reset(p.arena);
    p.tables.reset(p.arena);
    alloc_tables(p);
    alloc_index(p, true);
    alloc_query(p);
    int64_t caps = 0;
    for (int i = 0; i < count; ++i) caps += std::max<int64_t>(0, in[i].out->nnz_cap);
    alloc_survivors(p, std::max<int64_t>(1 << 20, 2 * p.M + caps));
    alloc_stage(p, std::max<int64_t>(1 << 16, caps));
    const DeviceInfo& di = device_info(devc.device);
    const int per_cu = mixed_blocks_per_cu(p.KA, p.KA, p.f16);
    p.screen_grid = std::max(di.xcds, (di.cus * per_cu / di.xcds) * di.xcds);
    if (p.NK32) {
      const int per_cu32 = mfma32_batch_blocks_per_cu(p.D32);
      p.screen_grid32 = std::max(di.xcds, (di.cus * per_cu32 / di.xcds) * di.xcds);
    }
    build_graphs(p);
    // first run: builds the index and sizes the survivor / staging arrays
    run_graphs(p, true, true);
    if (o.autotune && p.M > 0 && !o.tile_c && !o.tile_g) {
      // the options' cache file, else the environment's SNN_TUNE_CACHE
      autotune(p, o.tune_cache ? o.tune_cache : std::getenv("SNN_TUNE_CACHE"));
      build_graphs(p);
    }
    return pp;
  } catch (...) {
    free_plan(pp);
    throw;
  }
}

}  // namespace snn

using namespace snn;

extern "C" {

snn_status snn_batch_create(const snn_device* dev, snn_dtype dtype, const snn_instance* instances, int32_t count,
                            const snn_batch_options* opts, snn_batch_t* out) {
  return guard([&] {
    if (!dev || !out) fail(SNN_EINVAL, "dev / out is NULL");
    *out = nullptr;
    *out = reinterpret_cast<snn_batch_t>(create_batch(*dev, dtype, instances, count, opts));
  });
}

snn_status snn_batch_run(snn_batch_t b, int32_t what, snn_stats* st) {
  return guard([&] {
    if (!b) fail(SNN_EINVAL, "batch is NULL");
    if (what & ~(SNN_BATCH_INDEX | SNN_BATCH_QUERY) || what == 0) fail(SNN_EINVAL, "bad pass selection");
    BatchPlan& p = *reinterpret_cast<BatchPlan*>(b);
    DeviceScope scope(p.arena.dev().device);
    const bool q = (what & SNN_BATCH_QUERY) != 0;
    RunResult rr = run_graphs(p, (what & SNN_BATCH_INDEX) != 0, q);
    if (q) {
      fill_stats(p, rr, st);
      log_line(2, "batch run: %d instances, %lld queries, window pairs=%llu survivors=%llu nnz=%lld, graph %.3f ms "
                  "(screen %.3f)", p.count, (long long)p.M, rr.ctl.pairs_window, rr.ctl.survivors,
               (long long)rr.total, rr.graph_ms, rr.screen_ms);
      finish_outputs(p, rr);
    } else if (st) {
      std::memset(st, 0, sizeof(*st));
      st->total_ms = rr.graph_ms;
      st->screen_ms = -1;
      for (double& t : st->stage_ms) t = -1;
    }
  });
}

snn_status snn_batch_info(snn_batch_t b, snn_batch_info_t* info) {
  return guard([&] {
    if (!b || !info) fail(SNN_EINVAL, "NULL argument");
    const BatchPlan& p = *reinterpret_cast<BatchPlan*>(b);
    info->tile_q = p.T;
    info->tile_c = p.CH;
    info->tile_g = p.G;
    info->operand_k = p.KA;
    info->graph_timed_screen = p.screen_timed ? 1 : 0;
    info->tuned_query_ms = p.last_tune_ms;
    info->fp32_instances = p.count - p.n16;
    info->fp32_k = p.D32;
  });
}

void snn_batch_free(snn_batch_t b) {
  if (!b) return;
  BatchPlan* p = reinterpret_cast<BatchPlan*>(b);
  try {
    DeviceScope scope(p->arena.dev().device);
    (void)hipStreamSynchronize(p->arena.stream());
    free_plan(p);
  } catch (...) {
    free_plan(p);
  }
}

snn_status snn_query_batch(const snn_device* dev, snn_dtype dtype, const snn_instance* instances, int32_t count,
                           const snn_batch_options* opts, snn_stats* st) {
  snn_batch_t b = nullptr;
  snn_status r = snn_batch_create(dev, dtype, instances, count, opts, &b);
  if (r != SNN_OK) return r;
  // creation already ran both passes (the latest query pass wrote the outputs)
  r = guard([&] {
    BatchPlan& p = *reinterpret_cast<BatchPlan*>(b);
    fill_stats(p, p.last, st);
    finish_outputs(p, p.last);
  });
  snn_batch_free(b);
  return r;
}

}  // extern "C"
