// DBSCAN on the neighbour lists of an all-points self-query (Section 6.4
// runs DBSCAN with SNN as its radius search, eps = R).
//
// With row i of the lists = N(i) (ids j with S(p_j, p_i) <= fl(eps^2), i
// included, membership symmetric):
//   core(i)   <=> |N(i)| >= min_samples
//   clusters   = connected components of the core points under "j in N(i)",
//                numbered 0, 1, ... in order of their smallest core id
//   label(i)   = its cluster for a core point; for a non-core point the
//                smallest cluster number among the core points of N(i);
//                -1 (noise) when there is none.
// These are the labels of the classic DBSCAN that visits points in index
// order and grows each cluster through core points.
//
// GPU form: a lock-free union-find over the core-core pairs.  Every root
// is the smallest id of its tree (a root is only ever hooked under a
// smaller root, by compare-and-swap), so after the hooking pass each
// component's root is its smallest core id; ranking the roots by an
// exclusive scan numbers the clusters in the required order.  Parent links
// only ever decrease, so path halving (a node re-pointed to its
// grandparent) keeps a valid forest under races.  The links are read with
// device-scope atomic loads: the hooking pass runs on every XCD, and a
// stale copy of a root in one XCD's L2 would make a retry loop spin.
//
// Passes: validate the lists (ids in range, rows non-decreasing), init
// (core flags, parent = self), hook (one wavefront per row, pairs j > i
// with both ends core), compress (parent = root), root ranks (scan),
// labels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "device_common.h"
#include "query_plan.h"
#include "snn_internal.h"

namespace snn {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ int uf_load(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void uf_store(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x with path halving.
__device__ int32_t uf_find(int32_t* parent, int32_t x) {
  for (;;) {
    const int32_t p = uf_load(parent + x);
    if (p == x) return x;
    const int32_t gp = uf_load(parent + p);
    if (gp == p) return p;
    uf_store(parent + x, gp);
    x = gp;
  }
}

// Joins the trees of a and b, hooking the larger root under the smaller.
__device__ void uf_union(int32_t* parent, int32_t a, int32_t b) {
  for (;;) {
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a == b) return;
    if (a < b) {
      const int32_t t = a;
      a = b;
      b = t;
    }
    int32_t expected = a;
    if (__hip_atomic_compare_exchange_strong(parent + a, &expected, b, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT))
      return;
  }
}

__global__ __launch_bounds__(kThreads) void k_db_validate(const int64_t* __restrict__ row_ptr,
                                                          const int32_t* __restrict__ col, int64_t n, int64_t nnz,
                                                          int* __restrict__ bad) {
  int b = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    if (row_ptr[i] > row_ptr[i + 1]) b = 1;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride) {
    const int32_t j = col[e];
    if (j < 0 || (int64_t)j >= n) b = 1;
  }
  if (__ballot(b) && lane_id() == 0) atomicOr(bad, 1);
}

__global__ __launch_bounds__(kThreads) void k_db_init(const int64_t* __restrict__ row_ptr, int64_t n,
                                                      int min_samples, uint8_t* __restrict__ core,
                                                      int32_t* __restrict__ parent) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    core[i] = (row_ptr[i + 1] - row_ptr[i]) >= (int64_t)min_samples ? 1 : 0;
    parent[i] = (int32_t)i;
  }
}

// One wavefront per row; the lanes walk the row 64 entries at a time.
__global__ __launch_bounds__(kThreads) void k_db_hook(const int64_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ col, int64_t n,
                                                      const uint8_t* __restrict__ core, int32_t* parent) {
  const int lane = lane_id();
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
  for (int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; i < n; i += waves) {
    if (!core[i]) continue;
    const int64_t e0 = row_ptr[i], e1 = row_ptr[i + 1];
    for (int64_t e = e0 + lane; e < e1; e += kWave) {
      const int32_t j = col[e];
      if ((int64_t)j > i && core[j]) uf_union(parent, (int32_t)i, j);
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_db_roots(int64_t n, const uint8_t* __restrict__ core,
                                                       int32_t* parent, int32_t* __restrict__ is_root) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    int32_t r = 0;
    if (core[i]) {
      const int32_t root = uf_find(parent, (int32_t)i);
      uf_store(parent + i, root);
      r = root == (int32_t)i ? 1 : 0;
    }
    is_root[i] = r;
  }
}

__global__ __launch_bounds__(kThreads) void k_db_label(const int64_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ col, int64_t n,
                                                       const uint8_t* __restrict__ core,
                                                       const int32_t* __restrict__ parent,
                                                       const int64_t* __restrict__ rank, int32_t* __restrict__ labels) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    int64_t lab = -1;
    if (core[i]) {
      lab = rank[parent[i]];
    } else {
      for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
        const int32_t j = col[e];
        if (core[j]) {
          const int64_t r = rank[parent[j]];
          if (lab < 0 || r < lab) lab = r;
        }
      }
    }
    labels[i] = (int32_t)lab;
  }
}

// ---- clustering straight from a self-query's accepted pairs ---------------
// Nodes are index slots (score order), so the pairs of a point lie close to
// it and the links stay cache-local; roots are ordered by original id
// (ord = perm) so that each component's root is its smallest original core
// id, as the numbering requires.
__device__ void uf_union_ord(int32_t* parent, const int32_t* __restrict__ ord, int32_t a, int32_t b) {
  for (;;) {
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a == b) return;
    if (ord[a] < ord[b]) {
      const int32_t t = a;
      a = b;
      b = t;
    }
    int32_t expected = a;
    if (__hip_atomic_compare_exchange_strong(parent + a, &expected, b, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT))
      return;
  }
}

__global__ __launch_bounds__(kThreads) void k_dbe_init(int64_t n, const int32_t* __restrict__ row_cnt,
                                                       int min_samples, uint8_t* __restrict__ core_s,
                                                       int32_t* __restrict__ parent, int32_t* __restrict__ flag) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    core_s[i] = row_cnt[i] >= min_samples ? 1 : 0;
    parent[i] = (int32_t)i;
    flag[i] = 0;
  }
}

// The survivors come in score order, so neighbouring entries belong to the
// same few growing components: each wavefront takes its own contiguous
// slice of the list, so that the pairs in flight at any moment are spread
// over the whole point set (and over many roots) while every wavefront still
// reads its slice coalesced.
__global__ __launch_bounds__(kThreads) void k_dbe_hook(Survivors sv, const uint8_t* __restrict__ core_s,
                                                       int32_t* parent, const int32_t* __restrict__ perm) {
  const long long cnt = (long long)min((unsigned long long)sv.cap, *sv.count);
  const long long nw = (long long)gridDim.x * (blockDim.x / kWave);
  const long long w = (long long)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const long long per = (cnt + nw - 1) / nw;
  const long long k1 = min(cnt, (w + 1) * per);
  for (long long k = w * per + lane_id(); k < k1; k += kWave) {
    if (sv.res_q[k] < 0) continue;
    const int2 pr = sv.pairs[k];
    if (pr.x != pr.y && core_s[pr.x] && core_s[pr.y]) uf_union_ord(parent, perm, pr.x, pr.y);
  }
}

// Roots flagged at their original id: the scan of the flags numbers the
// clusters by smallest original core id.
__global__ __launch_bounds__(kThreads) void k_dbe_roots(int64_t n, const uint8_t* __restrict__ core_s,
                                                        int32_t* parent, const int32_t* __restrict__ perm,
                                                        int32_t* __restrict__ flag) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (!core_s[i]) continue;
    const int32_t root = uf_find(parent, (int32_t)i);
    uf_store(parent + i, root);
    if (root == (int32_t)i) flag[perm[i]] = 1;
  }
}

// Core points take their cluster; the others start at INT_MAX (lowered by
// k_dbe_border, noise if it stays).
__global__ __launch_bounds__(kThreads) void k_dbe_core_labels(int64_t n, const uint8_t* __restrict__ core_s,
                                                              const int32_t* __restrict__ parent,
                                                              const int32_t* __restrict__ perm,
                                                              const int64_t* __restrict__ rank,
                                                              int32_t* __restrict__ labels, uint8_t* __restrict__ core) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t o = perm[i];
    const bool c = core_s[i] != 0;
    labels[o] = c ? (int32_t)rank[perm[parent[i]]] : INT_MAX;
    if (core) core[o] = c ? 1 : 0;
  }
}

__global__ __launch_bounds__(kThreads) void k_dbe_border(Survivors sv, const uint8_t* __restrict__ core_s,
                                                         const int32_t* __restrict__ perm, int32_t* labels) {
  const long long cnt = (long long)min((unsigned long long)sv.cap, *sv.count);
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < cnt;
       k += (long long)gridDim.x * blockDim.x) {
    if (sv.res_q[k] < 0) continue;
    const int2 pr = sv.pairs[k];
    const bool cx = core_s[pr.x] != 0, cy = core_s[pr.y] != 0;
    if (cx == cy) continue;
    const int32_t c = cx ? pr.x : pr.y, b = cx ? pr.y : pr.x;
    atomicMin(&labels[perm[b]], labels[perm[c]]);
  }
}

__global__ __launch_bounds__(kThreads) void k_dbe_noise(int64_t n, int32_t* __restrict__ labels) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (labels[i] == INT_MAX) labels[i] = -1;
}

int grid_for(int64_t work, int cap) {
  int64_t g = (work + kThreads - 1) / kThreads;
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

size_t dbscan_work_bytes(int64_t n) {
  Carver c(nullptr);
  c.take<int32_t>(n);      // parent
  c.take<int32_t>(n);      // flag
  c.take<int64_t>(n + 1);  // rank
  c.take<uint8_t>(n);      // core flags, slot order
  c.take<char>(scan_scratch_bytes(std::max<int64_t>(n, 1)));
  return c.off + 256;
}

int64_t dbscan_from_survivors(const Survivors& sv, int64_t n, const int32_t* row_cnt, const int32_t* perm,
                              int min_samples, void* work, int32_t* labels, uint8_t* core, int grid, hipStream_t s) {
  if (n == 0) return 0;
  Carver c(work);
  int32_t* parent = c.take<int32_t>(n);
  int32_t* flag = c.take<int32_t>(n);
  int64_t* rank = c.take<int64_t>(n + 1);
  uint8_t* core_s = c.take<uint8_t>(n);
  char* scratch = c.take<char>(scan_scratch_bytes(std::max<int64_t>(n, 1)));
  const int g = grid_for(n, grid);
  k_dbe_init<<<g, kThreads, 0, s>>>(n, row_cnt, min_samples, core_s, parent, flag);
  SNN_LAUNCH_CHECK();
  k_dbe_hook<<<grid, kThreads, 0, s>>>(sv, core_s, parent, perm);
  SNN_LAUNCH_CHECK();
  k_dbe_roots<<<g, kThreads, 0, s>>>(n, core_s, parent, perm, flag);
  SNN_LAUNCH_CHECK();
  exclusive_scan_i32_to_i64(flag, rank, n, scratch, s);
  k_dbe_core_labels<<<g, kThreads, 0, s>>>(n, core_s, parent, perm, rank, labels, core);
  SNN_LAUNCH_CHECK();
  k_dbe_border<<<grid, kThreads, 0, s>>>(sv, core_s, perm, labels);
  SNN_LAUNCH_CHECK();
  k_dbe_noise<<<g, kThreads, 0, s>>>(n, labels);
  SNN_LAUNCH_CHECK();
  int64_t total = 0;
  SNN_HIP(hipMemcpyAsync(&total, rank + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  SNN_HIP(hipStreamSynchronize(s));
  return total;
}

}  // namespace snn

using namespace snn;

extern "C" {

snn_status snn_dbscan(const snn_device* dev, int64_t n, const int64_t* row_ptr, const int32_t* col,
                      int32_t min_samples, int32_t* labels, uint8_t* core, int64_t* nclusters) {
  return guard([&] {
    if (!dev) fail(SNN_EINVAL, "dev is NULL");
    if (n < 0) fail(SNN_EINVAL, "n must be >= 0");
    if (n >= (int64_t)INT32_MAX) fail(SNN_EINVAL, "n must be < 2^31 - 1");
    if (min_samples < 1) fail(SNN_EINVAL, "min_samples must be >= 1");
    if (!row_ptr) fail(SNN_EINVAL, "row_ptr is NULL");
    if (n > 0 && !labels) fail(SNN_EINVAL, "labels is NULL");
    if ((dev->alloc == nullptr) != (dev->free == nullptr)) fail(SNN_EINVAL, "alloc and free must both be set");
    DeviceScope scope(dev->device);
    DeviceArena a(*dev);
    hipStream_t s = a.stream();
    const DeviceInfo& di = device_info(dev->device);

    int64_t ends[2] = {0, 0};
    SNN_HIP(hipMemcpyAsync(&ends[0], row_ptr, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SNN_HIP(hipMemcpyAsync(&ends[1], row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SNN_HIP(hipStreamSynchronize(s));
    const int64_t nnz = ends[1];
    if (ends[0] != 0 || nnz < 0) fail(SNN_EINVAL, "row_ptr must start at 0 and end at nnz >= 0");
    if (nnz > 0 && !col) fail(SNN_EINVAL, "col is NULL");
    if (n == 0) {
      if (nclusters) *nclusters = 0;
      return;
    }

    Carver sz(nullptr);
    sz.take<int32_t>(n);                       // parent
    sz.take<int32_t>(n);                       // is_root
    sz.take<int64_t>(n + 1);                   // rank
    sz.take<uint8_t>(core ? 1 : n);            // core flags when the caller passes none
    sz.take<char>(scan_scratch_bytes(n));
    sz.take<int>(1);                           // bad flag
    ScopedAlloc scratch_mem(a, sz.off);
    Carver c(scratch_mem.get());
    int32_t* parent = c.take<int32_t>(n);
    int32_t* is_root = c.take<int32_t>(n);
    int64_t* rank = c.take<int64_t>(n + 1);
    uint8_t* own_core = c.take<uint8_t>(core ? 1 : n);
    char* scratch = c.take<char>(scan_scratch_bytes(n));
    int* bad = c.take<int>(1);
    if (!core) core = own_core;

    const int grid = grid_for(std::max(n, nnz), di.cus * 16);
    launch_fill_i32(bad, 1, 0, s);
    k_db_validate<<<grid, kThreads, 0, s>>>(row_ptr, col, n, nnz, bad);
    SNN_LAUNCH_CHECK();
    int hbad = 0;
    SNN_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    SNN_HIP(hipStreamSynchronize(s));
    if (hbad) fail(SNN_EINVAL, "neighbour lists: row_ptr decreasing or an id outside [0, n)");

    k_db_init<<<grid_for(n, di.cus * 16), kThreads, 0, s>>>(row_ptr, n, min_samples, core, parent);
    SNN_LAUNCH_CHECK();
    k_db_hook<<<(int)std::min<int64_t>((n + kThreads / kWave - 1) / (kThreads / kWave), di.cus * 16), kThreads, 0,
                s>>>(row_ptr, col, n, core, parent);
    SNN_LAUNCH_CHECK();
    k_db_roots<<<grid_for(n, di.cus * 16), kThreads, 0, s>>>(n, core, parent, is_root);
    SNN_LAUNCH_CHECK();
    exclusive_scan_i32_to_i64(is_root, rank, n, scratch, s);
    k_db_label<<<grid_for(n, di.cus * 16), kThreads, 0, s>>>(row_ptr, col, n, core, parent, rank, labels);
    SNN_LAUNCH_CHECK();
    int64_t total = 0;
    SNN_HIP(hipMemcpyAsync(&total, rank + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SNN_HIP(hipStreamSynchronize(s));
    if (nclusters) *nclusters = total;
  });
}

}  // extern "C"
