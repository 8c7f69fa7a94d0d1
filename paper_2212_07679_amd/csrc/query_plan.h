// Shared description of one query call (Algorithm 2 over many queries):
// the queries in score order, their candidate windows, the query tiles and
// the work units the candidate-screen kernels consume.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"
#include "snn.h"

namespace snn {

constexpr int kMaxXcd = 8;

// Work unit u covers tile t = the tile with unit_off[t] <= u < unit_off[t+1]
// and candidates [tlo[t] + c*CH, min(tlo[t] + (c+1)*CH, thi[t])) with
// c = u - unit_off[t].  Tile t holds sorted queries [t*T, min((t+1)*T, m)).
struct QueryDev {
  int64_t m;
  int d;
  int dp;  // padded row stride of q64 / p64 (multiple of 4, zero-filled)
  int T;   // queries per tile (multiple of 64)
  int CH;  // candidates per work unit
  int ntiles;
  double R2;  // fl64(R*R)
  const double* q64;     // m x dp: query rows in float64, score order
  const int32_t* qorig;  // m: score-order position -> caller's query row
  const double* p64;     // n x dp: data rows in float64, score order
  const int32_t* perm;   // n: score-order position -> original data row
  const int32_t* tlo;    // ntiles
  const int32_t* thi;    // ntiles
  const int64_t* unit_off;       // ntiles + 1
  unsigned long long* counters;  // kMaxXcd work counters (zeroed per call)
  int nxcd;
  PairSink sink;
};

__device__ __forceinline__ int uniform_i32(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uniform_i64(int64_t x) {
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(x & 0xffffffffu));
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Next work unit for a block on XCD `xcd`: each XCD owns a contiguous range
// of units (so blocks sharing an L2 work on neighbouring tiles); when its
// range is exhausted the block steals from the other ranges.  -1 when done.
__device__ __forceinline__ int64_t next_unit(const QueryDev& q, int xcd) {
  const int64_t total = q.unit_off[q.ntiles];
  for (int k = 0; k < q.nxcd; ++k) {
    const int x = (xcd + k) % q.nxcd;
    const int64_t beg = total * x / q.nxcd, end = total * (x + 1) / q.nxcd;
    if (beg >= end) continue;
    const unsigned long long c = atomicAdd(&q.counters[x], 1ull);
    if (beg + (int64_t)c < end) return beg + (int64_t)c;
  }
  return -1;
}

// tile of unit u (binary search over unit_off)
__device__ __forceinline__ int unit_tile(const QueryDev& q, int64_t u) {
  int lo = 0, hi = q.ntiles - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (q.unit_off[mid] <= u)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------- launchers
void launch_query_keys(snn_dtype dt, const void* Q, int64_t m, int d, const double* mu, const double* v,
                       uint32_t* ukey, uint32_t* val, double* qalpha, double* qnorm, int* bad, hipStream_t s);
void launch_query_gather(snn_dtype dt, const void* Q, int64_t m, int d, int dp, const uint32_t* qperm,
                         const double* qalpha_in, const double* qnorm_in, double* q64, int32_t* qorig,
                         double* qalpha, double* qnorm, hipStream_t s);
void launch_windows(const double* key, int n, const double* qalpha, const double* qnorm, int64_t m, double w_base,
                    double eps_scale, int T, int CH, int ntiles, int32_t* lo, int32_t* hi, int32_t* tlo,
                    int32_t* thi, int32_t* units, unsigned long long* pairs_window, hipStream_t s);

// k_cand_fp64.hip: plain float64 screen (every window pair, normative rule)
void launch_cand_fp64(const QueryDev& q, int grid, hipStream_t s);
int fp64_blocks_per_cu(int dp);

// k_cand_mfma.hip: mixed-precision screen on the matrix cores
struct MixedDev {
  const uint16_t* qop;  // m x KA bf16: query operand rows (score order)
  const float* cthr;    // m: per-query accumulator start C_q
  const uint16_t* cop;  // (n + 32) x KB bf16: candidate operand rows (score order)
  const float* h;       // n + 32: fl32(||y_j||^2 / 2), padding +inf
  int KA;               // query operand row length = product chain length
  int KB;               // candidate row length: KA, or 2 KA / 3 for the split layout
};
struct MixedBound {
  double r2p_half;  // R2' / 2
  double sqrt_r2p;  // sqrt(R2'), rounded up
  double u32p;      // 1.01 u32
  double Y;         // max_j ||y_j||
  double c_rep;     // bf16 representation error coefficient
  double g_acc;     // 2 gamma32_{K+1}
  double e_h;       // rounding of h_j to fp32
  double g64;       // gamma64_{d+1}: relative error of h_q in float64
};
double mixed_c_rep(int terms);
MixedBound mixed_bound(int terms, int KA, int d, double R2, double Y);
int mixed_max_slices();
int mixed_queries_per_wave();
int mixed_blocks_per_cu(int KA, int KB);
void launch_mixed_qprep(const double* q64, int64_t m, int d, int dp, const double* mu, int terms, int KA,
                        const MixedBound& b, uint16_t* qop, float* cthr, hipStream_t s);
void launch_mixed_qprep_self(const float* ys, int64_t n, int d, const MixedBound& b, float* cthr, hipStream_t s);
void launch_cand_mfma(const QueryDev& q, const MixedDev& x, int grid, hipStream_t s);

// k_csr.hip
struct Survivors {
  int2* pairs;                 // (query score position, data score position)
  unsigned long long* count;   // may exceed cap (then pairs were dropped)
  long long cap;
  int32_t* res_q;              // caller query row or -1
  int32_t* res_id;
  float* res_dist;
  int32_t* res_slot;
};
void launch_recheck(const QueryDev& q, const Survivors& sv, int32_t* row_cnt, int grid, hipStream_t s);
void launch_scatter(const Survivors& sv, const int64_t* row_ptr, int32_t* col, float* dist, int grid,
                    hipStream_t s);
void launch_row_sort(const int64_t* row_ptr, int64_t m, int32_t* col, float* dist, int32_t* lists,
                     unsigned long long* list_counts, int grid, hipStream_t s);
void launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s);
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);

}  // namespace snn
