// Shared description of one query call (Algorithm 2 over many queries):
// the queries in score order, their candidate windows, the query tiles and
// the work units the candidate-screen kernels consume.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "device_common.h"
#include "snn.h"

namespace snn {

constexpr int kMaxXcd = 8;

// Tile t holds score-ordered queries [t*T, min((t+1)*T, m)) and the union
// window [tlo[t], thi[t]), cut into chunks of at most CH candidates.
//
// Work units are ordered chunk-major inside groups of G consecutive tiles:
// unit u of group g (group_off[g] <= u < group_off[g+1]) is chunk
// k = l / Gg of tile t = g*G + l % Gg, with l = u - group_off[g] and Gg the
// tiles in the group.  Score-adjacent tiles have nearly the same window, so
// the units that run at the same time on one XCD read the same candidate
// rows from its L2.  Two kinds of group:
//  * long windows (gbase[g] >= 0): chunk k is the absolute range
//    [B*CH, (B+1)*CH), B = gbase[g] + k, clipped to the tile's window, so
//    all tiles of the group read it at the same addresses; the group
//    reserves its chunk span x Gg units;
//  * short windows (gbase[g] = -1): chunk k is [tlo + k*CH, tlo + (k+1)*CH)
//    clipped to the window (units[t] chunks), which does not cut a short
//    window in two; the group reserves (max units[t]) x Gg units.
// A unit whose chunk misses its tile's window is empty.
struct QueryDev {
  int64_t m;
  int d;
  int dp;  // padded row stride of q64 / p64 (multiple of 4, zero-filled)
  int T;   // queries per tile (multiple of 64)
  int CH;  // candidates per work unit
  int ntiles;
  int G;        // tiles per group
  int ngroups;
  double R2;  // fl64(R*R) of the screen radius
  int metric; // snn_metric of the recheck
  double R1;  // the L1 radius (metric L1; R2 then belongs to the widened L2 radius)
  const double* q64;     // m x dp: query rows in float64, score order (the float64 screen and self-queries)
  const void* qsrc;      // the caller's query rows (input dtype), read by the recheck when q64 is NULL
  const int32_t* qorig;  // m: score-order position -> caller's query row
  const double* p64;     // n x dp: data rows in float64, score order
  const int32_t* perm;   // n: score-order position -> original data row
  const int32_t* tlo;    // ntiles
  const int32_t* thi;    // ntiles
  const int32_t* units;          // ntiles
  const int64_t* group_off;      // ngroups + 1
  const int32_t* gbase;          // ngroups: first absolute chunk, or -1
  unsigned long long* counters;  // kMaxXcd work counters (zeroed per call)
  int nxcd;
  // Symmetric self-query: query position s is data position s, tiles scan
  // candidates from their own first row on, and a pair (s, j) with j >= s is
  // decided once and reported in both rows (S is exactly symmetric).
  int sym;
  PairSink sink;
  // device clock marks of the launch, or NULL: [0] the complement of the
  // earliest workgroup start (zero is then the neutral value of atomicMax),
  // [1] the latest workgroup end
  unsigned long long* stamps;
};

__device__ __forceinline__ int uniform_i32(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uniform_i64(int64_t x) {
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(x & 0xffffffffu));
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Clock marks of a screen launch (thread 0 of each workgroup, at its start
// and after its last work unit).
__device__ __forceinline__ void mark_begin(const QueryDev& q) {
  if (q.stamps && threadIdx.x == 0) atomicMax(&q.stamps[0], ~(unsigned long long)wall_clock64());
}
__device__ __forceinline__ void mark_end(const QueryDev& q) {
  if (q.stamps && threadIdx.x == 0) atomicMax(&q.stamps[1], (unsigned long long)wall_clock64());
}

// Next work unit for a block on XCD `xcd`: each XCD owns a contiguous range
// of units (so blocks sharing an L2 work on neighbouring tiles); when its
// range is exhausted the block steals from the other ranges.  -1 when done.
__device__ __forceinline__ int64_t next_unit(const QueryDev& q, int xcd) {
  const int64_t total = q.group_off[q.ngroups];
  for (int k = 0; k < q.nxcd; ++k) {
    const int x = (xcd + k) % q.nxcd;
    const int64_t beg = total * x / q.nxcd, end = total * (x + 1) / q.nxcd;
    if (beg >= end) continue;
    const unsigned long long c = atomicAdd(&q.counters[x], 1ull);
    if (beg + (int64_t)c < end) return beg + (int64_t)c;
  }
  return -1;
}

// Tile and candidate range [j0, j1) of unit u; false for an empty unit.
// Results are wavefront-uniform.
__device__ __forceinline__ bool decode_unit(const QueryDev& q, int64_t u, int& tile, int64_t& j0, int64_t& j1) {
  int lo = 0, hi = q.ngroups - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (q.group_off[mid] <= u)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int gg = min(q.G, q.ntiles - lo * q.G);
  const int64_t l = u - q.group_off[lo];
  const int64_t k = uniform_i64(l / gg);
  const int gb = uniform_i32(q.gbase[lo]);
  tile = uniform_i32(lo * q.G + (int)(l % gg));
  if (gb < 0) {
    if (k >= q.units[tile]) return false;
    j0 = uniform_i64((int64_t)q.tlo[tile] + k * q.CH);
    j1 = uniform_i64(min((int64_t)q.thi[tile], j0 + q.CH));
  } else {
    const int64_t B = gb + k;
    j0 = uniform_i64(max((int64_t)q.tlo[tile], B * q.CH));
    j1 = uniform_i64(min((int64_t)q.thi[tile], (B + 1) * q.CH));
  }
  return j0 < j1;
}

// ---------------------------------------------------------------- launchers
int query_buckets(int64_t m);
// keys, buckets and slots of the queries, then hist (K counts, zero
// beforehand) turned into bucket offsets (scan_state: lookback_words(K)
// zero words)
void launch_query_keys(snn_dtype dt, const void* Q, int64_t m, int d, const double* mu, const double* v,
                       const double* key, int n, int K, uint32_t* bucket, uint32_t* slot, uint32_t* hist,
                       double* qalpha, double* qnorm, int* bad, unsigned long long* scan_state, int* scan_err,
                       hipStream_t s);
struct QueryOperands;
// queries into score order (bucket offsets boff), with the screen's query
// operands and start values (op.mode: none, 16-bit rows + C_q, fp32 rows)
void launch_query_gather(snn_dtype dt, const void* Q, int64_t m, int d, int dp, const uint32_t* bucket,
                         const uint32_t* slot, const uint32_t* boff, const double* qalpha_in, const double* qnorm_in,
                         double* q64, int32_t* qorig, double* qalpha, double* qnorm, const double* mu,
                         const QueryOperands& op, hipStream_t s);
// start of every cell of a uniform grid over the sorted scores (cells + 1 entries)
int window_table_cells(int64_t n);
void launch_window_table(const double* key, int n, int C, int32_t* start, hipStream_t s);
// align: tile windows are widened outward to multiples of `align` rows (the
// mixed screen reads 32-row blocks); extra candidates never change results.
// sym: symmetric self-query (counts only candidates j >= s, tiles start at
// their first row; see QueryDev::sym)
// k_window writes one partial window-pair count per workgroup (wpart, at
// most kWindowMaxBlocks of them: window_blocks(m)); k_tile_plan sums them
constexpr int kWindowMaxBlocks = 2048;
int window_blocks(int64_t m);
// Arguments of the tile plan (k_tile_plan): per-tile windows widened to
// `align`, work units of CH
// candidates, groups of G tiles with their unit offsets and absolute chunk
// bases, the executed-pair count and the window-pair total.
struct TilePlanArgs {
  int32_t* tlo;
  int32_t* thi;
  int ntiles;
  int CH;
  int align;
  int sym_T;  // T for a symmetric self-query, else 0
  int32_t* units;
  int G;
  int64_t* unit_off;
  int32_t* gbase;
  int T;
  int64_t m;
  int qpw;
  unsigned long long* executed;
  const unsigned long long* wpart;
  int nwpart;
  unsigned long long* pairs_window;
};
// k_window (m > 0) followed by the tile plan
void launch_windows_plan(const double* key, int n, const int32_t* cells, int C, const double* qalpha,
                         const double* qnorm, int64_t m, double w_base, double eps_scale, int T, int sym, int32_t* lo,
                         int32_t* hi, const TilePlanArgs& plan, hipStream_t s);
// one launch: zero ctl_words control words, row_cnt (m) and hist (nb, may be
// NULL), and empty tile windows (tlo = INT_MAX, thi = INT_MIN)
// mark_word >= 0: that word of ctl takes the device clock (wall_clock64)
// instead of zero
void launch_query_init(unsigned long long* ctl, int ctl_words, int32_t* row_cnt, int64_t m, uint32_t* hist, int nb,
                       int32_t* tlo, int32_t* thi, int ntiles, hipStream_t s, int mark_word = -1);
// *out = the device clock (wall_clock64) when the stream reaches it
void launch_clock_mark(unsigned long long* out, hipStream_t s);
// one single-workgroup launch after the windows: tile windows clamped and
// aligned, units per tile, G x max units per group of G tiles scanned into
// unit_off (ngroups + 1 entries), evaluated pairs added to *executed
// (nullable; qpw query slots per wavefront)
// wpart / nwpart / pairs_window: the window-pair partials of k_window and
// their total (NULL / 0 / NULL when there are none)
void launch_tile_plan(int32_t* tlo, int32_t* thi, int ntiles, int CH, int align, int sym, int32_t* units, int G,
                      int64_t* unit_off, int32_t* gbase, int T, int64_t m, int qpw, unsigned long long* executed,
                      const unsigned long long* wpart, int nwpart, unsigned long long* pairs_window,
                      hipStream_t s);


// k_cand_fp64.hip: plain float64 screen (every window pair, normative rule)
void launch_cand_fp64(const QueryDev& q, int grid, hipStream_t s);
int fp64_blocks_per_cu(int dp);

// k_cand_mfma.hip: mixed-precision screen on the matrix cores
struct MixedDev {
  const uint16_t* qop;  // m x KA 16-bit operands: query operand rows (score order)
  const float* cthr;    // m: per-query accumulator start C_q (scaled units)
  const uint16_t* cop;  // (n + 32) x KB 16-bit operands: candidate operand rows (score order)
  const float* h;       // n + 32: the candidates' half squared norms in the accumulator's units, padding +inf
  int KA;               // query operand row length = product chain length
  int KB;               // candidate row length: KA, or 2 KA / 3 for the split layout
  int f16;              // 1: fp16 operands (v_mfma_f32_32x32x16_f16), 0: bf16
};

// Operand encodings of the matrix-core screens.
enum OperandKind {
  kOpF32 = 0,     // the fp32 centred rows themselves
  kOpBf16 = 1,    // one bf16 value per coordinate
  kOpBf16x3 = 3,  // bf16 hi/lo split, three products hi*hi + hi*lo + lo*hi
  kOpF16 = 4      // one fp16 value per coordinate of the rows scaled by 2^e
};

struct MixedBound {
  double r2p_half;  // R2' / 2
  double sqrt_r2p;  // sqrt(R2'), rounded up
  double u32p;      // 1.01 u32
  double Y;         // max_j ||y_j||
  double c_rep;     // representation error coefficient of the operands
  double sub;       // (1 + u) sqrt(K) delta: operands below the normal range, times (||y_q|| + Y)
  double sub2;      // K delta^2
  double g_acc;     // 2 gamma32_{K+1}
  double e_h;       // rounding of h_j to fp32
  double g64;       // gamma64_{d+1}: relative error of h_q in float64
  double scale2;    // s^2 = 2^(2e): accumulator units (fp16 operands), else 1
};

// Representation error coefficient of the screen operands:
// bf16 (u_b = 2^-8): |y - bf16(y)| <= u_b |y|, so the product of two rounded
//   operands differs from y_q . y_j by at most u_b (2 + u_b) |y_q||y_j|;
// bf16 hi/lo: hi + lo leaves u_b^2 |y| and the dropped lo*lo product adds
//   u_b^2, giving u_b^2 (3 + 3 u_b);
// fp16 (u_h = 2^-11) of the rows scaled by a power of two: u_h (2 + u_h);
// fp32: the operands are the rows themselves.
__host__ __device__ inline double mixed_c_rep(int kind) {
  const double ub = 0.00390625, uh = 0.00048828125;
  switch (kind) {
    case kOpF32: return 0.0;
    case kOpBf16: return 1.01 * ub * (2.0 + ub);
    case kOpF16: return 1.01 * uh * (2.0 + uh);
    default: return 1.01 * ub * ub * (3.0 + 3.0 * ub);
  }
}

// fp16 operands hold s y with s = 2^e chosen so that every |s y_k| <= s Y <=
// 2^15 (fp16's largest finite value is 65504); 0 when Y = 0.
__host__ __device__ inline int f16_scale_exp(double Y) {
  if (!(Y > 0)) return 0;
  int ex = 0;
  frexp(Y, &ex);  // Y < 2^ex
  int e = 15 - ex;
  return e < -60 ? -60 : (e > 60 ? 60 : e);
}
// Whether a screen's fp32 arithmetic holds every value it forms for rows of
// norm at most Y: squared norms below 2^120 (bf16 / fp32 operands), scaled
// fp16 rows below 2^15.
__host__ __device__ inline bool screen_in_range(int kind, double Y) {
  if (kind == kOpF16) return ldexp(Y, f16_scale_exp(Y)) <= 32768.0;
  return Y <= ldexp(1.0, 60);
}

// Constants of the screen start value for one index and radius (the terms
// of C_q derived in k_cand_mfma.hip).  K: the product chain length.
__host__ __device__ inline MixedBound mixed_bound(int kind, int K, int d, double R2, double Y) {
  const double u32 = 5.9604644775390625e-08, u64 = 1.1102230246251565e-16;
  const double ga = (K + 1) * u32 / (1.0 - (K + 1) * u32);
  const double gr = (d + 2) * u64 / (1.0 - (d + 2) * u64);
  const double gh = (d + 1) * u64 / (1.0 - (d + 1) * u64);
  MixedBound b;
  const double r2p = R2 * (1.0 + 2.0 * gr);
  b.r2p_half = 0.5 * r2p;
  b.sqrt_r2p = sqrt(r2p) * (1.0 + 1e-15);
  b.u32p = 1.01 * u32;
  b.Y = Y;
  b.c_rep = mixed_c_rep(kind);
  // delta: the largest error of an operand below the normal range, whether
  // the conversion keeps it subnormal or the matrix core reads it as zero:
  // fp16's smallest normal 2^-14 in the scaled units (2^-14 / s unscaled),
  // else bf16's / fp32's 2^-126.
  const int e = kind == kOpF16 ? f16_scale_exp(Y) : 0;
  const double delta = kind == kOpF16 ? ldexp(1.0, -14 - e) : ldexp(1.0, -126);
  const double terms = kind == kOpBf16x3 ? 3.0 : 1.0;  // operand values per coordinate
  b.sub = 1.01 * (1.0 + 0.00390625) * terms * sqrt((double)K) * delta;
  b.sub2 = 1.01 * terms * K * delta * delta;
  b.g_acc = 2.0 * ga;
  b.e_h = 1.01 * u32 * Y * Y * 0.5;
  b.g64 = gh;
  b.scale2 = ldexp(1.0, 2 * e);
  return b;
}

__device__ __forceinline__ float round_up_f32(double c) {
  float f = (float)c;
  if ((double)f < c) f = nextafterf(f, INFINITY);
  return f;
}

// Accumulator start C_q of a screen (see k_cand_mfma.hip): every pair with
// S(p_j, q) <= fl(R*R) satisfies (screen value) >= (the candidate's h in
// accumulator units).  hq = ||y_q||^2/2 and nq >= ||y_q|| in float64.
__device__ __forceinline__ float screen_threshold(const MixedBound& b, double hq, double nq) {
  const double eta = b.u32p * (b.Y + nq);
  const double hlo = hq * (1.0 - b.g64);
  const double e_sub = b.sub * (nq + b.Y) + b.sub2;
  double c0 = b.r2p_half - hlo + eta * b.sqrt_r2p + 0.5 * eta * eta + b.c_rep * b.Y * nq + e_sub + b.e_h;
  c0 += 8.0 * 1.1102230246251565e-16 * (b.r2p_half + hq + b.Y * nq) + 1e-30;
  const double e_acc = b.g_acc * (1.02 * b.Y * nq + e_sub + fabs(c0)) * 1.01;
  return round_up_f32((c0 + e_acc) * b.scale2);
}
// Query operands built while the queries are gathered into score order.
enum { kQOpNone = 0, kQOp16 = 1, kQOp32 = 2 };
struct QueryOperands {
  int mode = kQOpNone;
  int kind = kOpBf16;  // 16-bit rows: OperandKind
  int e = 0;           // fp16 scale exponent
  int KA = 0;          // 16-bit row length
  int DV = 0;          // fp32 row stride
  MixedBound b{};
  uint16_t* qop = nullptr;
  float* cthr = nullptr;
  float* vq = nullptr;
};

int mixed_max_slices();
int mixed_queries_per_wave(int KA, bool f16);  // 32 x query blocks per wavefront
int mixed_blocks_per_cu(int KA, int KB, bool f16);
// operand row length (16-bit values) of an OperandKind at dimension d
int operand_ka(int kind, int d);
void launch_mixed_qprep_self(const float* ys, int64_t n, int d, const MixedBound& b, float* cthr, hipStream_t s);
void launch_cand_mfma(const QueryDev& q, const MixedDev& x, int grid, hipStream_t s);

// k_cand_mfma.hip: fp32 matrix-core screen for d <= 16
struct Mfma32Dev {
  const float* vq;   // m x DV: query rows [y, C_q, 0 ...] (score order)
  int DV;
  int d;
  const float* cop;  // candidate operand blocks (see k_cand_mfma32)
  const float* h;    // n + 64: fl32(||y_j||^2 / 2), padding +inf
};
int mfma32_max_d();
int mfma32_query_floats(int d);  // stride of a query row [y, C_q, 0 ...]
int mfma32_queries_per_tile();
int64_t mfma32_operand_floats(int64_t n, int d);
int mfma32_blocks_per_cu(int d);
void launch_mfma32_operands(const float* ys, int64_t n, int d, float* cop, hipStream_t s);
void launch_mfma32_qprep_self(const float* ys, int64_t n, int d, const MixedBound& b, float* vq, hipStream_t s);
void launch_cand_mfma32(const QueryDev& q, const Mfma32Dev& x, int grid, hipStream_t s);
// the same screen with two query blocks per wavefront (tiles of
// mfma32_batch_queries_per_tile() = 256 slots), for the batch
int mfma32_batch_queries_per_tile();
int mfma32_batch_blocks_per_cu(int d);
void launch_cand_mfma32_batch(const QueryDev& q, const Mfma32Dev& x, int grid, hipStream_t s);

// Test support (k_cand_mfma.hip): every pair's screen value of a small query,
// D[qorig[q] n + j] (q < m score-order queries, j < n score-order
// candidates), with the operand loads and product chains of the screens; and
// the operands in plain row-major form.
void launch_dump_mixed(const MixedDev& x, int64_t m, int64_t n, const int32_t* qorig, float* D, hipStream_t s);
void launch_dump_mfma32(const Mfma32Dev& x, int64_t m, int64_t n, const int32_t* qorig, float* D, hipStream_t s);
void launch_dump_cand16(const uint16_t* cop, int64_t n, int KB, uint16_t* out, hipStream_t s);
void launch_dump_rows_u16(const uint16_t* in, int64_t m, int W, const int32_t* qorig, uint16_t* out, hipStream_t s);
void launch_dump_rows_f32(const float* in, int64_t m, int W, const int32_t* qorig, float* out, hipStream_t s);

// k_csr.hip
struct Survivors {
  int2* pairs;                 // (query score position, data score position)
  unsigned long long* count;   // may exceed cap (then pairs were dropped)
  long long cap;
  int per;                     // results per pair: 1, or 2 for a symmetric self-query
  int32_t* res_q;              // per * cap: row (query slot) or -1
  uint64_t* res_key;           // per * cap: neighbour key (id << 32 | distance bits)
  int32_t* res_slot;           // per * cap: position within the row
};
// neighbour key: ordering keys orders by id (ids are unique within a row)
__host__ __device__ __forceinline__ uint64_t neighbour_key(int32_t id, float dist) {
  return ((uint64_t)(uint32_t)id << 32) | (uint64_t)__builtin_bit_cast(uint32_t, dist);
}
// po: the index's data rows in the input dtype, score order (n x d);
// row_cnt: counts of the slot-order rows (m, zero beforehand)
void launch_recheck(const QueryDev& q, const Survivors& sv, snn_dtype dt, const void* po, bool self,
                    int32_t* row_cnt, int grid, hipStream_t s);
// Optional outputs of launch_rows_scan (each may be NULL): counts in the
// destination order cnt_dst[map[r]] = cnt[r], the longest row (atomic max),
// the total, and the rows by length class (lists: row_sort_lists() x m,
// list_counts zero beforehand; lists NULL: none).
struct RowsExtra {
  const int32_t* map;
  int32_t* cnt_dst;
  unsigned long long* row_max;
  unsigned long long* total;
  int32_t* lists;
  unsigned long long* list_counts;
};
// row_ptr (m + 1) from the counts in one launch; state: lookback_words(m)
// zero words
// launch_rows_scan without extras and launch_scatter as one launch
void launch_rows_scan_scatter(const int32_t* cnt, int64_t m, int64_t* row_ptr, unsigned long long* state, int* err,
                              const Survivors& sv, const int64_t* rp_s, uint64_t* keys, int scatter_grid,
                              hipStream_t s);
void launch_rows_scan(const int32_t* cnt, int64_t m, int64_t* row_ptr, unsigned long long* state, int* err,
                      const RowsExtra& ex, hipStream_t s);
// keys into slot-order rows at row_ptr[row] + slot
// (does nothing when the survivor list overflowed: *sv.count > sv.cap)
void launch_scatter(const Survivors& sv, const int64_t* row_ptr, uint64_t* keys, int grid, hipStream_t s);
// self-queries for clustering: row counts of both points of every accepted
// pair, res_q[i] = query slot of survivor i if accepted else -1 (one entry
// per survivor), *accepted += neighbour entries
void launch_recheck_edges(const QueryDev& q, const Survivors& sv, snn_dtype dt, const void* po, int32_t* row_cnt,
                          unsigned long long* accepted, int grid, hipStream_t s);

// dbscan.hip: clustering of a self-query's accepted pairs (slot space =
// score order; perm maps a slot to its original id).  work: dbscan_work_bytes(n).
size_t dbscan_work_bytes(int64_t n);
// labels / core: original order (core nullable); returns the cluster count
// (synchronises the stream)
int64_t dbscan_from_survivors(const Survivors& sv, int64_t n, const int32_t* row_cnt, const int32_t* perm,
                              int min_samples, void* work, int32_t* labels, uint8_t* core, int grid, hipStream_t s);
// Source row r of a CSR of neighbour keys goes, sorted by id, to
// destination row map[r] (row r when map is NULL) of the caller's CSR.
struct RowMove {
  const int64_t* src_rp;
  const uint64_t* src_key;
  const int32_t* map;  // source row -> destination row (< 0: empty padding row), or NULL
  const int64_t* dst_rp;
  int32_t* dst_col;
  float* dst_dist;
  // optional guard for moves enqueued before the host has checked the
  // sizes: nothing is written unless *total <= cap (total NULL: no guard)
  const unsigned long long* total;
  unsigned long long cap;
};
// lists: row_sort_lists() x m int32, list_counts: 8 counters, tmp_col /
// tmp_dist: destination nnz entries (may be NULL when no row exceeds 4096)
int row_sort_lists();
// max_len: an upper bound on the row lengths when the host knows one (the
// kernels of longer length classes are not launched), else INT64_MAX
void launch_row_sort_move(const RowMove& mv, int64_t m, int64_t max_len, int32_t* lists,
                          unsigned long long* list_counts, int32_t* tmp_col, float* tmp_dist, hipStream_t s);
// The same in two parts: the head (class lists and rows of up to 16 entries)
// needs no host-side size, so it can be enqueued before the sizes are read
// back; the tail launches the longer classes up to max_len.
void launch_row_sort_head(const RowMove& mv, int64_t m, int32_t* lists, unsigned long long* list_counts,
                          hipStream_t s);
void launch_row_sort_tail(const RowMove& mv, int64_t m, int64_t max_len, int32_t* lists,
                          unsigned long long* list_counts, int32_t* tmp_col, float* tmp_dist, hipStream_t s);
// cnt_dst[map[r]] = length of source row r
void launch_perm_counts(const int64_t* src_rp, int64_t m, const int32_t* map, int32_t* cnt_dst, hipStream_t s);
// the same, plus *row_max = max row length (atomic max; zero beforehand) and
// *total = src_rp[m]
void launch_perm_counts_stats(const int64_t* src_rp, int64_t m, const int32_t* map, int32_t* cnt_dst,
                              unsigned long long* row_max, unsigned long long* total, hipStream_t s);
// the same pass also appending every row to the list of its length class
// (lists / list_counts as for launch_row_sort_head, counts zero beforehand)
void launch_rows_stats(const int64_t* src_rp, int64_t m, const int32_t* map, int32_t* cnt_dst,
                       unsigned long long* row_max, unsigned long long* total, int32_t* lists,
                       unsigned long long* list_counts, hipStream_t s);
// rows of at most 16 entries of classified lists, moved sorted
void launch_row_sort_short(const RowMove& mv, int32_t* lists, unsigned long long* list_counts, hipStream_t s);
void launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s);
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);

}  // namespace snn
