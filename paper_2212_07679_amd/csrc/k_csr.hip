// From surviving (query, candidate) pairs to CSR neighbour lists.
//
//  k_recheck    every survivor is decided by the normative rule on the
//               original coordinates in float64 (direct form of eq. (ip1),
//               left to right, no fused multiply-add; inclusive compare of
//               Section 3.2).  Neighbours take a slot in their row; rows are
//               query slots (score order).
//  k_rows_scan  row counts -> row offsets in one launch (look-back scan);
//               for the slot-order rows also the counts in the caller's
//               order, the longest row, the total and the rows by length
//               class; again for the caller's row offsets
//  k_scatter    neighbours into their slot-order rows
//  row sort     each row sorted by id on its way to the caller's row order:
//               rows of <= 16 / 32 / 64 entries by lane groups of that size
//               (bitonic across lanes), up to 512 by one wavefront with 2 / 4
//               / 8 entries per lane, longer rows by one workgroup (bitonic in
//               LDS, then merge passes).
#include <hip/hip_runtime.h>

#include <climits>

#include "device_common.h"
#include "query_plan.h"
#include "snn_internal.h"

#pragma clang fp contract(off)

namespace snn {

namespace {
constexpr int kThreads = 256;

// The normative measure of a pair in float64, left to right over the
// coordinates, no fused multiply-add: S = sum fl(t_k * t_k) (L2, compared
// with fl(R*R)) or M = sum |t_k| (L1, compared with R), t_k = fl(p_k - q_k).
template <typename A, typename B>
__device__ __forceinline__ double pair_measure(int metric, const A* __restrict__ p, const B* __restrict__ qv,
                                               int d) {
  double s = 0.0;
  if (metric == SNN_METRIC_L1) {
    for (int k = 0; k < d; ++k) s = s + fabs((double)p[k] - (double)qv[k]);
  } else {
    for (int k = 0; k < d; ++k) {
      const double t = (double)p[k] - (double)qv[k];
      s = s + t * t;
    }
  }
  return s;
}

// Reported distance of an accepted pair from its measure s: the 1-norm (L1),
// the angle 2 asin(sqrt(S) / 2) or the cosine distance S / 2 of unit rows
// (Section 2), else the Euclidean distance sqrt(S); float64, rounded once.
__device__ __forceinline__ float pair_distance(int metric, double s) {
  if (metric == SNN_METRIC_L1) return (float)s;
  if (metric == SNN_METRIC_ANGULAR) return (float)(2.0 * asin(fmin(1.0, 0.5 * sqrt(s))));
  if (metric == SNN_METRIC_COSINE) return (float)(0.5 * s);
  return (float)sqrt(s);
}

// Slot of this lane's entry in row `row` (lanes with `want`): lanes of the
// wavefront that add to the same row share one atomic, taken by the first of
// them.  The screens push the passing pairs one accumulator row at a time,
// so the survivors list holds runs of one query row and a wavefront sees few
// distinct rows (blobs3d: the recheck 5.05 -> 4.31 ms); the grouping costs a
// ballot per distinct row, the atomics stay one instruction.
__device__ __forceinline__ int grouped_slot(bool want, int row, int32_t* __restrict__ row_cnt) {
  const int lane = lane_id();
  const uint64_t lt = (1ull << lane) - 1ull;
  uint64_t todo = __ballot(want);
  int leader = -1, count = 0, rank = 0;
  while (todo) {
    const int l = __builtin_ctzll(todo);
    const int lr = __shfl(row, l, kWave);
    const uint64_t peers = __ballot(want && row == lr) & todo;
    if (lane == l) count = __popcll(peers);
    if ((peers >> lane) & 1ull) {
      leader = l;
      rank = __popcll(peers & lt);
    }
    todo &= ~peers;
  }
  int base = 0;
  if (want && leader == lane) base = atomicAdd(&row_cnt[row], count);
  base = __shfl(base, leader < 0 ? lane : leader, kWave);
  return base + rank;
}

// Data rows are read in the input dtype (their promotion to float64 is
// exact), the query rows of a self-query likewise; out-of-sample query rows
// are the float64 copies in score order, or the caller's rows (input dtype,
// through qorig) when the screen made no such copies.
template <typename T, bool SELF>
__global__ __launch_bounds__(kThreads) void k_recheck(QueryDev q, Survivors sv, const T* __restrict__ po,
                                                     int32_t* __restrict__ row_cnt) {
  const long long cnt = (long long)min((unsigned long long)sv.cap, *sv.count);
  const int d = q.d;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (long long)gridDim.x * blockDim.x) {
    const int2 pr = sv.pairs[i];
    const int64_t r0 = (int64_t)sv.per * i;
    // symmetric self-query: a pair below the diagonal is the mirror of one
    // the other query of the tile decides
    bool keep = !q.sym || pr.y >= pr.x;
    double s = 0.0;
    if (keep) {
      const T* pp = po + (int64_t)pr.y * d;
      if (SELF)
        s = pair_measure(q.metric, pp, po + (int64_t)pr.x * d, d);
      else if (q.q64)
        s = pair_measure(q.metric, pp, q.q64 + (int64_t)pr.x * q.dp, d);
      else
        s = pair_measure(q.metric, pp, static_cast<const T*>(q.qsrc) + (int64_t)q.qorig[pr.x] * d, d);
      keep = q.metric == SNN_METRIC_L1 ? s <= q.R1 : s <= q.R2;
    }
    // rows are query slots (score order): a tile's rows are neighbours in
    // memory, so the counters and the later writes stay cache-local.  The
    // dense outputs are self-queries, whose runs of one row make the grouping
    // pay; the sparse lists of out-of-sample queries mix rows in a wavefront
    // (grouping took the gmm16 recheck from 9.3 to 10 us)
    int slot = 0;
    if (SELF)
      slot = grouped_slot(keep, pr.x, row_cnt);
    else if (keep)
      slot = atomicAdd(&row_cnt[pr.x], 1);
    if (keep) {
      const float dist = pair_distance(q.metric, s);
      sv.res_q[r0] = pr.x;
      sv.res_key[r0] = neighbour_key(q.perm[pr.y], dist);
      sv.res_slot[r0] = slot;
      if (sv.per == 2) {
        if (pr.y != pr.x) {  // the mirrored pair, in the candidate's row (its slot is its position)
          sv.res_q[r0 + 1] = pr.y;
          sv.res_key[r0 + 1] = neighbour_key(q.qorig[pr.x], dist);
          sv.res_slot[r0 + 1] = atomicAdd(&row_cnt[pr.y], 1);
        } else {
          sv.res_q[r0 + 1] = -1;
        }
      }
    } else {
      sv.res_q[r0] = -1;
      if (sv.per == 2) sv.res_q[r0 + 1] = -1;
    }
  }
}

// Self-query survivors for clustering: the same normative decision, but a
// survivor only counts in the rows of both its points (a pair below the
// diagonal of a symmetric scan is the mirror of one decided elsewhere) and
// keeps its query slot in res_q as the "accepted" mark (-1 otherwise); no
// distances, no row slots.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_recheck_edges(QueryDev q, Survivors sv, const T* __restrict__ po,
                                                           int32_t* __restrict__ row_cnt,
                                                           unsigned long long* __restrict__ accepted) {
  const long long cnt = (long long)min((unsigned long long)sv.cap, *sv.count);
  const int d = q.d;
  unsigned long long acc = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (long long)gridDim.x * blockDim.x) {
    const int2 pr = sv.pairs[i];
    bool keep = !q.sym || pr.y >= pr.x;
    if (keep) {
      const double s = pair_measure(q.metric, po + (int64_t)pr.y * d, po + (int64_t)pr.x * d, d);
      keep = q.metric == SNN_METRIC_L1 ? s <= q.R1 : s <= q.R2;
    }
    if (keep) {
      atomicAdd(&row_cnt[pr.x], 1);
      ++acc;
      if (q.sym && pr.y != pr.x) {
        atomicAdd(&row_cnt[pr.y], 1);
        ++acc;
      }
    }
    sv.res_q[i] = keep ? pr.x : -1;
  }
  acc = wave_sum(acc);
  if (lane_id() == 0 && acc) atomicAdd(accepted, acc);
}

__device__ __forceinline__ void scatter_body(const Survivors& sv, const int64_t* __restrict__ row_ptr,
                                             uint64_t* __restrict__ keys, int block, int nblocks) {
  if (*sv.count > (unsigned long long)sv.cap) return;  // overflowed: the host runs the query again
  const long long cnt = (long long)*sv.count * sv.per;
  for (long long i = (long long)block * blockDim.x + threadIdx.x; i < cnt; i += (long long)nblocks * blockDim.x) {
    const int qo = sv.res_q[i];
    if (qo < 0) continue;
    keys[row_ptr[qo] + sv.res_slot[i]] = sv.res_key[i];
  }
}

__global__ __launch_bounds__(kThreads) void k_scatter(Survivors sv, const int64_t* __restrict__ row_ptr,
                                                     uint64_t* __restrict__ keys) {
  scatter_body(sv, row_ptr, keys, blockIdx.x, gridDim.x);
}

// false when the move was enqueued before the host checked the sizes and
// the rows do not fit the destination (then nothing is written)
__device__ __forceinline__ bool rows_fit(const RowMove& mv) { return !mv.total || *mv.total <= mv.cap; }

// Row length classes: 2..16, 17..32, 33..64, 65..128, 129..256, 257..512 and
// longer (kRowClasses lists).
constexpr int kRowClasses = 7;

__device__ __forceinline__ int len_class(int64_t len) {
  if (len <= 0) return -1;
  if (len <= 16) return 0;
  if (len <= 32) return 1;
  if (len <= 64) return 2;
  if (len <= 128) return 3;
  if (len <= 256) return 4;
  if (len <= 512) return 5;
  return 6;
}

__device__ __forceinline__ int row_class(const int64_t* __restrict__ row_ptr, int64_t r) {
  return len_class(row_ptr[r + 1] - row_ptr[r]);
}

// about 4096 rows per workgroup (at most 1024 workgroups): each reserves
// list space with one atomic per class, and atomics on one address serialise
inline int classify_blocks(int64_t m) { return (int)std::min<int64_t>(1024, std::max<int64_t>(1, m / 4096)); }

// Rows by length class, each class appended to its own list.  A block owns a
// contiguous range of rows: it counts its rows per class in LDS, reserves
// each class's space with one global atomic, then writes (so the global
// counters see one atomic per block and class).
__global__ __launch_bounds__(kThreads) void k_row_classify(const int64_t* __restrict__ row_ptr, int64_t m,
                                                          int32_t* __restrict__ lists,
                                                          unsigned long long* __restrict__ counts) {
  __shared__ int cnt[kRowClasses];
  __shared__ unsigned long long base[kRowClasses];
  const int t = threadIdx.x;
  const int64_t per = (m + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * per, r1 = min(m, r0 + per);
  if (t < kRowClasses) cnt[t] = 0;
  __syncthreads();
  for (int64_t r = r0 + t; r < r1; r += kThreads) {
    const int c = row_class(row_ptr, r);
    if (c >= 0) atomicAdd(&cnt[c], 1);
  }
  __syncthreads();
  if (t < kRowClasses) {
    base[t] = cnt[t] ? atomicAdd(&counts[t], (unsigned long long)cnt[t]) : 0ull;
    cnt[t] = 0;
  }
  __syncthreads();
  for (int64_t r = r0 + t; r < r1; r += kThreads) {
    const int c = row_class(row_ptr, r);
    if (c >= 0) lists[(int64_t)c * m + (int64_t)base[c] + atomicAdd(&cnt[c], 1)] = (int32_t)r;
  }
}

// Rows of at most SEG entries, 64 / SEG rows per wavefront: each group of SEG
// lanes holds one row as (id << 32 | dist bits) and runs a bitonic network
// across its lanes (partners at distance < SEG stay inside the group).  Ids
// are unique within a row, so the order is by id alone.  The sorted row is
// written to its destination row.
template <int SEG>
__global__ __launch_bounds__(kThreads) void k_row_sort_seg(RowMove mv, const int32_t* __restrict__ list,
                                                          const unsigned long long* __restrict__ count) {
  if (!rows_fit(mv)) return;
  constexpr int kRows = kWave / SEG;
  const long long nrows = (long long)*count;
  const int lane = lane_id(), sub = lane % SEG, grp = lane / SEG;
  const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const long long nwaves = ((long long)gridDim.x * blockDim.x) / kWave;
  for (long long w = wave; w * kRows < nrows; w += nwaves) {
    const long long k = w * kRows + grp;
    int64_t b = 0, o = 0;
    int len = 0;
    if (k < nrows) {
      const int r = list[k];
      b = mv.src_rp[r];
      len = (int)(mv.src_rp[r + 1] - b);
      o = mv.dst_rp[mv.map ? mv.map[r] : r];
    }
    uint64_t key = sub < len ? mv.src_key[b + sub] : ~0ull;
#pragma unroll
    for (int kk = 2; kk <= SEG; kk <<= 1) {
#pragma unroll
      for (int j = kk >> 1; j > 0; j >>= 1) {
        const uint64_t x = __shfl_xor(key, j, kWave);
        const bool take_min = ((sub & kk) == 0) == ((sub & j) == 0);
        key = take_min ? (x < key ? x : key) : (x > key ? x : key);
      }
    }
    if (sub < len) {
      mv.dst_col[o + sub] = (int32_t)(key >> 32);
      mv.dst_dist[o + sub] = __builtin_bit_cast(float, (uint32_t)(key & 0xffffffffu));
    }
  }
}

// Rows of 65 .. 64 E entries, one wavefront per row, E entries per lane:
// entry i sits in lane i % 64, slot i / 64.  In the bitonic network a partner
// at distance j >= 64 is another slot of the same lane (a register
// compare-exchange), a partner at j < 64 the same slot of lane ^ j (one
// shuffle).
template <int E>
__global__ __launch_bounds__(kThreads) void k_row_sort_reg(RowMove mv, const int32_t* __restrict__ list,
                                                          const unsigned long long* __restrict__ count) {
  if (!rows_fit(mv)) return;
  constexpr int N = kWave * E;
  const long long nrows = (long long)*count;
  const int lane = lane_id();
  const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const long long nwaves = ((long long)gridDim.x * blockDim.x) / kWave;
  for (long long w = wave; w < nrows; w += nwaves) {
    const int r = list[w];
    const int64_t b = mv.src_rp[r];
    const int len = (int)(mv.src_rp[r + 1] - b);
    const int64_t o = mv.dst_rp[mv.map ? mv.map[r] : r];
    uint64_t key[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i = e * kWave + lane;
      key[e] = i < len ? mv.src_key[b + i] : ~0ull;
    }
#pragma unroll
    for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
      for (int j = k >> 1; j > 0; j >>= 1) {
        if (j >= kWave) {
          const int js = j / kWave;
#pragma unroll
          for (int e = 0; e < E; ++e) {
            if (e & js) continue;
            const int i = e * kWave + lane;
            const bool asc = (i & k) == 0;
            const uint64_t x = key[e], y = key[e | js];
            const uint64_t lo = x < y ? x : y, hi = x < y ? y : x;
            key[e] = asc ? lo : hi;
            key[e | js] = asc ? hi : lo;
          }
        } else {
#pragma unroll
          for (int e = 0; e < E; ++e) {
            const int i = e * kWave + lane;
            const uint64_t x = __shfl_xor(key[e], j, kWave);
            const bool take_min = ((i & k) == 0) == ((lane & j) == 0);
            key[e] = take_min ? (x < key[e] ? x : key[e]) : (x > key[e] ? x : key[e]);
          }
        }
      }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i = e * kWave + lane;
      if (i < len) {
        mv.dst_col[o + i] = (int32_t)(key[e] >> 32);
        mv.dst_dist[o + i] = __builtin_bit_cast(float, (uint32_t)(key[e] & 0xffffffffu));
      }
    }
  }
}

constexpr int kBlockSort = 4096;

__device__ __forceinline__ void bitonic_lds(uint64_t* a, int n) {
  for (int k = 2; k <= n; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const uint64_t x = a[i], y = a[ixj];
          const bool up = ((i & k) == 0);
          if ((x > y) == up) {
            a[i] = y;
            a[ixj] = x;
          }
        }
      }
      __syncthreads();
    }
  }
}

// One workgroup per row of more than 512 entries: runs of 4096 are sorted
// in LDS on their way from the source row to the destination row, then runs
// are merged pairwise in the destination (each element finds its rank in the
// partner run by binary search; ids are unique within a row), ping-ponging
// through tmp at the destination offsets (tmp holds the destination nnz).
__global__ __launch_bounds__(kThreads) void k_row_sort_block(RowMove mv, const int32_t* __restrict__ list,
                                                            const unsigned long long* __restrict__ count,
                                                            int32_t* __restrict__ tmp_col,
                                                            float* __restrict__ tmp_dist) {
  __shared__ uint64_t a[kBlockSort];
  if (!rows_fit(mv)) return;  // uniform: before any barrier
  const long long nrows = (long long)*count;
  for (long long w = blockIdx.x; w < nrows; w += gridDim.x) {
    const int r = list[w];
    const int64_t b = mv.src_rp[r];
    const int64_t len = mv.src_rp[r + 1] - b;
    const int64_t o = mv.dst_rp[mv.map ? mv.map[r] : r];
    for (int64_t c0 = 0; c0 < len; c0 += kBlockSort) {
      const int cl = (int)min((int64_t)kBlockSort, len - c0);
      int np2 = 1;
      while (np2 < cl) np2 <<= 1;
      __syncthreads();
      for (int i = threadIdx.x; i < np2; i += blockDim.x)
        a[i] = i < cl ? mv.src_key[b + c0 + i] : ~0ull;
      __syncthreads();
      bitonic_lds(a, np2);
      for (int i = threadIdx.x; i < cl; i += blockDim.x) {
        mv.dst_col[o + c0 + i] = (int32_t)(a[i] >> 32);
        mv.dst_dist[o + c0 + i] = __builtin_bit_cast(float, (uint32_t)(a[i] & 0xffffffffu));
      }
    }
    __syncthreads();
    int32_t *sc = mv.dst_col + o, *dc = tmp_col + o;
    float *sd = mv.dst_dist + o, *dd = tmp_dist + o;
    bool in_tmp = false;
    for (int64_t width = kBlockSort; width < len; width <<= 1) {
      for (int64_t i = threadIdx.x; i < len; i += blockDim.x) {
        const int64_t run = i / width;
        const int64_t rs = run * width;
        const int64_t ps = (run ^ 1) * width;  // partner run start
        const int64_t pair = min(rs, ps);
        const int32_t key = sc[i];
        int64_t rank = 0;
        if (ps < len) {
          int64_t lo = ps, hi = min(ps + width, len);
          while (lo < hi) {
            const int64_t md = (lo + hi) >> 1;
            if (sc[md] < key)
              lo = md + 1;
            else
              hi = md;
          }
          rank = lo - ps;
        }
        const int64_t out = pair + (i - rs) + rank;
        dc[out] = key;
        dd[out] = sd[i];
      }
      __syncthreads();
      int32_t* t1 = sc;
      sc = dc;
      dc = t1;
      float* t2 = sd;
      sd = dd;
      dd = t2;
      in_tmp = !in_tmp;
    }
    if (in_tmp) {
      for (int64_t i = threadIdx.x; i < len; i += blockDim.x) {
        dc[i] = sc[i];
        dd[i] = sd[i];
      }
    }
    __syncthreads();
  }
}

// counts of the destination rows: cnt_dst[map[r]] = length of source row r
// (rows with map < 0 are padding and empty)
__global__ __launch_bounds__(kThreads) void k_perm_counts(const int64_t* __restrict__ src_rp, int64_t m,
                                                         const int32_t* __restrict__ map,
                                                         int32_t* __restrict__ cnt_dst) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x) {
    const int d = map[r];
    if (d >= 0) cnt_dst[d] = (int32_t)(src_rp[r + 1] - src_rp[r]);
  }
}

// k_perm_counts_stats and k_row_classify in one pass: a block owns a
// contiguous range of rows (about 1024), counts its rows per class in LDS and
// reserves each class's list space with one global atomic.
__global__ __launch_bounds__(kThreads) void k_rows_stats(const int64_t* __restrict__ src_rp, int64_t m,
                                                        const int32_t* __restrict__ map, int32_t* __restrict__ cnt_dst,
                                                        unsigned long long* __restrict__ row_max,
                                                        unsigned long long* __restrict__ total,
                                                        int32_t* __restrict__ lists,
                                                        unsigned long long* __restrict__ counts) {
  __shared__ int cnt[kRowClasses];
  __shared__ unsigned long long base[kRowClasses];
  __shared__ int red[kThreads / kWave];
  const int t = threadIdx.x;
  const int64_t per = (m + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * per, r1 = min(m, r0 + per);
  if (t < kRowClasses) cnt[t] = 0;
  __syncthreads();
  int v = 0;
  for (int64_t r = r0 + t; r < r1; r += kThreads) {
    const int len = (int)(src_rp[r + 1] - src_rp[r]);
    const int d = map[r];
    if (d >= 0) cnt_dst[d] = len;
    v = max(v, len);
    const int c = row_class(src_rp, r);
    if (c >= 0) atomicAdd(&cnt[c], 1);
  }
  v = wave_max(v);
  if (lane_id() == 0) red[t / kWave] = v;
  __syncthreads();
  if (t < kRowClasses) {
    base[t] = cnt[t] ? atomicAdd(&counts[t], (unsigned long long)cnt[t]) : 0ull;
    cnt[t] = 0;
  }
  if (t == 0) {
    for (int w = 1; w < kThreads / kWave; ++w) v = max(v, red[w]);
    if (v > 0 && (unsigned long long)v > __hip_atomic_load(row_max, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMax(row_max, (unsigned long long)v);
    if (blockIdx.x == 0) *total = (unsigned long long)src_rp[m];
  }
  __syncthreads();
  for (int64_t r = r0 + t; r < r1; r += kThreads) {
    const int c = row_class(src_rp, r);
    if (c >= 0) lists[(int64_t)c * m + (int64_t)base[c] + atomicAdd(&cnt[c], 1)] = (int32_t)r;
  }
}

// Row offsets from row counts in one launch (look-back scan: row_ptr[r] =
// sum of cnt before r, row_ptr[m] = total) and, when given (RowsExtra), the
// counts in the destination order (cnt_dst[map[r]] = cnt[r]), the longest
// row, the total and the rows by length class (each workgroup reserves its
// class list space with one atomic per class).
__device__ void rows_scan_body(const int32_t* __restrict__ cnt, int64_t m, int64_t* __restrict__ row_ptr,
                               unsigned long long* __restrict__ state, int* __restrict__ err, const RowsExtra& ex) {
  const int32_t* __restrict__ map = ex.map;
  int32_t* __restrict__ cnt_dst = ex.cnt_dst;
  unsigned long long* __restrict__ row_max = ex.row_max;
  unsigned long long* __restrict__ total = ex.total;
  int32_t* __restrict__ lists = ex.lists;
  unsigned long long* __restrict__ list_counts = ex.list_counts;
  __shared__ unsigned long long s_tile;
  __shared__ long long s_wave[kLookbackThreads / kWave];
  __shared__ int s_max[kLookbackThreads / kWave];
  __shared__ long long s_excl;
  __shared__ int s_cls[kRowClasses];
  __shared__ unsigned long long s_base[kRowClasses];
  const int t = threadIdx.x, lane = lane_id(), w = t / kWave;
  if (t == 0) s_tile = atomicAdd(&state[0], 1ull);
  if (t < kRowClasses) s_cls[t] = 0;
  __syncthreads();
  const long long tile = (long long)s_tile;
  const int64_t i0 = tile * kLookbackTile + (int64_t)t * kLookbackItems;
  int v[kLookbackItems];
  long long sum = 0;
  int vmax = 0;
#pragma unroll
  for (int k = 0; k < kLookbackItems; ++k) {
    v[k] = i0 + k < m ? cnt[i0 + k] : 0;
    sum += v[k];
    vmax = max(vmax, v[k]);
    if (lists) {
      const int c = len_class(v[k]);
      if (c >= 0) atomicAdd(&s_cls[c], 1);
    }
    if (map && i0 + k < m) {
      const int r = map[i0 + k];
      if (r >= 0) cnt_dst[r] = v[k];
    }
  }
  long long x = sum;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const long long y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  vmax = wave_max(vmax);
  if (lane == kWave - 1) s_wave[w] = x;
  if (lane == 0) s_max[w] = vmax;
  __syncthreads();
  long long before = 0, tot = 0;
  int bmax = 0;
#pragma unroll
  for (int k = 0; k < kLookbackThreads / kWave; ++k) {
    if (k < w) before += s_wave[k];
    tot += s_wave[k];
    bmax = max(bmax, s_max[k]);
  }
  if (w == 0) {
    unsigned long long excl = 0;
    if (tile == 0) {
      if (lane == 0) lookback_publish(state, 0, 2, (unsigned long long)tot);
    } else {
      if (lane == 0) lookback_publish(state, tile, 1, (unsigned long long)tot);
      excl = lookback_exclusive(state, tile, err);
      if (lane == 0) lookback_publish(state, tile, 2, excl + (unsigned long long)tot);
    }
    if (lane == 0) {
      s_excl = (long long)excl;
      // the maximum only grows: a workgroup that cannot raise it skips the atomic
      if (row_max && bmax > 0 &&
          (unsigned long long)bmax > __hip_atomic_load(row_max, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMax(row_max, (unsigned long long)bmax);
      if ((tile + 1) * kLookbackTile >= m) {  // the last tile: the total
        row_ptr[m] = (int64_t)(excl + (unsigned long long)tot);
        if (total) *total = excl + (unsigned long long)tot;
      }
    }
  } else if (lists && w == 1 && lane < kRowClasses) {
    s_base[lane] = s_cls[lane] ? atomicAdd(&list_counts[lane], (unsigned long long)s_cls[lane]) : 0ull;
    s_cls[lane] = 0;
  }
  __syncthreads();
  long long run = s_excl + before + x - sum;
#pragma unroll
  for (int k = 0; k < kLookbackItems; ++k) {
    if (i0 + k < m) {
      row_ptr[i0 + k] = run;
      const int c = lists ? len_class(v[k]) : -1;
      if (c >= 0) lists[(int64_t)c * m + (int64_t)s_base[c] + atomicAdd(&s_cls[c], 1)] = (int32_t)(i0 + k);
    }
    run += v[k];
  }
}

__global__ __launch_bounds__(kLookbackThreads) void k_rows_scan(const int32_t* __restrict__ cnt, int64_t m,
                                                               int64_t* __restrict__ row_ptr,
                                                               unsigned long long* __restrict__ state,
                                                               int* __restrict__ err, RowsExtra ex) {
  rows_scan_body(cnt, m, row_ptr, state, err, ex);
}

// k_rows_scan (no extras) and k_scatter in one launch: the first nscan
// workgroups scan, the others scatter (the two are independent; the scan's
// tiles are taken in ticket order, so its look-back only ever waits for
// workgroups that are already running).
__global__ __launch_bounds__(kLookbackThreads) void k_rows_scan_scatter(const int32_t* __restrict__ cnt, int64_t m,
                                                                       int64_t* __restrict__ row_ptr,
                                                                       unsigned long long* __restrict__ state,
                                                                       int* __restrict__ err, int nscan,
                                                                       Survivors sv,
                                                                       const int64_t* __restrict__ rp_s,
                                                                       uint64_t* __restrict__ keys) {
  if ((int)blockIdx.x < nscan)
    rows_scan_body(cnt, m, row_ptr, state, err, RowsExtra{});
  else
    scatter_body(sv, rp_s, keys, blockIdx.x - nscan, gridDim.x - nscan);
}

// k_perm_counts plus the longest row and (block 0, thread 0) the total.
__global__ __launch_bounds__(kThreads) void k_perm_counts_stats(const int64_t* __restrict__ src_rp, int64_t m,
                                                               const int32_t* __restrict__ map,
                                                               int32_t* __restrict__ cnt_dst,
                                                               unsigned long long* __restrict__ row_max,
                                                               unsigned long long* __restrict__ total) {
  __shared__ int red[kThreads / kWave];
  int v = 0;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x) {
    const int len = (int)(src_rp[r + 1] - src_rp[r]);
    const int d = map[r];
    if (d >= 0) cnt_dst[d] = len;
    v = max(v, len);
  }
  v = wave_max(v);
  if (lane_id() == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kThreads / kWave; ++w) v = max(v, red[w]);
    // the maximum only grows, so a workgroup that cannot raise it skips the
    // atomic (atomics on one address serialise); a stale read only costs an
    // unneeded atomic
    if (v > 0 && (unsigned long long)v > __hip_atomic_load(row_max, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMax(row_max, (unsigned long long)v);
    if (blockIdx.x == 0) *total = (unsigned long long)src_rp[m];
  }
}

__global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_self_qnorm(const float* __restrict__ ynorm, int64_t n, double* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (double)ynorm[i];
}

int grid_for(int64_t work, int cap) {
  int64_t g = (work + kThreads - 1) / kThreads;
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

void launch_self_qnorm(const float* ynorm, int64_t n, double* out, hipStream_t s) {
  k_self_qnorm<<<grid_for(n, 4096), kThreads, 0, s>>>(ynorm, n, out);
  SNN_LAUNCH_CHECK();
}

void launch_recheck(const QueryDev& q, const Survivors& sv, snn_dtype dt, const void* po, bool self,
                    int32_t* row_cnt, int grid, hipStream_t s) {
  if (dt == SNN_F32) {
    if (self)
      k_recheck<float, true><<<grid, kThreads, 0, s>>>(q, sv, static_cast<const float*>(po), row_cnt);
    else
      k_recheck<float, false><<<grid, kThreads, 0, s>>>(q, sv, static_cast<const float*>(po), row_cnt);
  } else {
    if (self)
      k_recheck<double, true><<<grid, kThreads, 0, s>>>(q, sv, static_cast<const double*>(po), row_cnt);
    else
      k_recheck<double, false><<<grid, kThreads, 0, s>>>(q, sv, static_cast<const double*>(po), row_cnt);
  }
  SNN_LAUNCH_CHECK();
}

void launch_recheck_edges(const QueryDev& q, const Survivors& sv, snn_dtype dt, const void* po, int32_t* row_cnt,
                          unsigned long long* accepted, int grid, hipStream_t s) {
  if (dt == SNN_F32)
    k_recheck_edges<float><<<grid, kThreads, 0, s>>>(q, sv, static_cast<const float*>(po), row_cnt, accepted);
  else
    k_recheck_edges<double><<<grid, kThreads, 0, s>>>(q, sv, static_cast<const double*>(po), row_cnt, accepted);
  SNN_LAUNCH_CHECK();
}

void launch_scatter(const Survivors& sv, const int64_t* row_ptr, uint64_t* keys, int grid, hipStream_t s) {
  k_scatter<<<grid, kThreads, 0, s>>>(sv, row_ptr, keys);
  SNN_LAUNCH_CHECK();
}

// m source rows; lists: row_sort_lists() x m int32 (one list per length
// class); list_counts: 8 counters; tmp_col / tmp_dist: destination nnz
// entries, needed only when a row exceeds 4096.  Fixed grids (the counts stay
// on the device), so the sequence can be captured.
void launch_row_sort_head(const RowMove& mv, int64_t m, int32_t* lists, unsigned long long* list_counts,
                          hipStream_t s) {
  k_fill_u64<<<1, 64, 0, s>>>(list_counts, 8, 0ull);
  SNN_LAUNCH_CHECK();
  if (m <= 0) return;
  k_row_classify<<<classify_blocks(m), kThreads, 0, s>>>(mv.src_rp, m, lists, list_counts);
  SNN_LAUNCH_CHECK();
  k_row_sort_seg<16><<<2048, kThreads, 0, s>>>(mv, lists, list_counts);
  SNN_LAUNCH_CHECK();
}

// classes whose shortest row exceeds max_len are empty and not launched
void launch_row_sort_tail(const RowMove& mv, int64_t m, int64_t max_len, int32_t* lists,
                          unsigned long long* list_counts, int32_t* tmp_col, float* tmp_dist, hipStream_t s) {
  if (m <= 0 || max_len <= 16) return;
  k_row_sort_seg<32><<<2048, kThreads, 0, s>>>(mv, lists + m, list_counts + 1);
  SNN_LAUNCH_CHECK();
  if (max_len > 32) {
    k_row_sort_seg<64><<<2048, kThreads, 0, s>>>(mv, lists + 2 * m, list_counts + 2);
    SNN_LAUNCH_CHECK();
  }
  if (max_len > 64) {
    k_row_sort_reg<2><<<2048, kThreads, 0, s>>>(mv, lists + 3 * m, list_counts + 3);
    SNN_LAUNCH_CHECK();
  }
  if (max_len > 128) {
    k_row_sort_reg<4><<<2048, kThreads, 0, s>>>(mv, lists + 4 * m, list_counts + 4);
    SNN_LAUNCH_CHECK();
  }
  if (max_len > 256) {
    k_row_sort_reg<8><<<2048, kThreads, 0, s>>>(mv, lists + 5 * m, list_counts + 5);
    SNN_LAUNCH_CHECK();
  }
  if (max_len > 512) {
    k_row_sort_block<<<512, kThreads, 0, s>>>(mv, lists + 6 * m, list_counts + 6, tmp_col, tmp_dist);
    SNN_LAUNCH_CHECK();
  }
}

void launch_row_sort_move(const RowMove& mv, int64_t m, int64_t max_len, int32_t* lists,
                          unsigned long long* list_counts, int32_t* tmp_col, float* tmp_dist, hipStream_t s) {
  k_fill_u64<<<1, 64, 0, s>>>(list_counts, 8, 0ull);
  SNN_LAUNCH_CHECK();
  if (m <= 0 || max_len <= 0) return;
  k_row_classify<<<classify_blocks(m), kThreads, 0, s>>>(mv.src_rp, m, lists, list_counts);
  SNN_LAUNCH_CHECK();
  k_row_sort_seg<16><<<2048, kThreads, 0, s>>>(mv, lists, list_counts);
  SNN_LAUNCH_CHECK();
  launch_row_sort_tail(mv, m, max_len, lists, list_counts, tmp_col, tmp_dist, s);
}

void launch_perm_counts(const int64_t* src_rp, int64_t m, const int32_t* map, int32_t* cnt_dst, hipStream_t s) {
  if (m <= 0) return;
  k_perm_counts<<<grid_for(m, 4096), kThreads, 0, s>>>(src_rp, m, map, cnt_dst);
  SNN_LAUNCH_CHECK();
}

void launch_rows_stats(const int64_t* src_rp, int64_t m, const int32_t* map, int32_t* cnt_dst,
                       unsigned long long* row_max, unsigned long long* total, int32_t* lists,
                       unsigned long long* list_counts, hipStream_t s) {
  const int blocks = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (m + 1023) / 1024));
  k_rows_stats<<<blocks, kThreads, 0, s>>>(src_rp, m, map, cnt_dst, row_max, total, lists, list_counts);
  SNN_LAUNCH_CHECK();
}

void launch_rows_scan(const int32_t* cnt, int64_t m, int64_t* row_ptr, unsigned long long* state, int* err,
                      const RowsExtra& ex, hipStream_t s) {
  const int blocks = (int)std::max<int64_t>(1, (m + kLookbackTile - 1) / kLookbackTile);
  k_rows_scan<<<blocks, kLookbackThreads, 0, s>>>(cnt, m, row_ptr, state, err, ex);
  SNN_LAUNCH_CHECK();
}

void launch_rows_scan_scatter(const int32_t* cnt, int64_t m, int64_t* row_ptr, unsigned long long* state, int* err,
                              const Survivors& sv, const int64_t* rp_s, uint64_t* keys, int scatter_grid,
                              hipStream_t s) {
  const int nscan = (int)std::max<int64_t>(1, (m + kLookbackTile - 1) / kLookbackTile);
  k_rows_scan_scatter<<<nscan + scatter_grid, kLookbackThreads, 0, s>>>(cnt, m, row_ptr, state, err, nscan, sv, rp_s,
                                                                        keys);
  SNN_LAUNCH_CHECK();
}

void launch_row_sort_short(const RowMove& mv, int32_t* lists, unsigned long long* list_counts, hipStream_t s) {
  k_row_sort_seg<16><<<2048, kThreads, 0, s>>>(mv, lists, list_counts);
  SNN_LAUNCH_CHECK();
}

void launch_perm_counts_stats(const int64_t* src_rp, int64_t m, const int32_t* map, int32_t* cnt_dst,
                              unsigned long long* row_max, unsigned long long* total, hipStream_t s) {
  k_perm_counts_stats<<<grid_for(m, 4096), kThreads, 0, s>>>(src_rp, m, map, cnt_dst, row_max, total);
  SNN_LAUNCH_CHECK();
}

int row_sort_lists() { return kRowClasses; }

void launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s) {
  if (n <= 0) return;
  k_fill_u64<<<grid_for(n, 4096), kThreads, 0, s>>>(p, n, v);
  SNN_LAUNCH_CHECK();
}

void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return;
  k_fill_i32<<<grid_for(n, 4096), kThreads, 0, s>>>(p, n, v);
  SNN_LAUNCH_CHECK();
}

}  // namespace snn
