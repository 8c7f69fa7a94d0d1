// Query preparation and windows (Algorithm 2, steps 2-4, Section 3.2).
//
//  k_query_keys    x_q = q - mu, alpha_q = x_q . v (float64), ||fl32(x_q)||,
//                  and a bucket of alpha_q on a uniform grid over the range of
//                  the index scores; each query takes a slot in its bucket
//  (scan)          bucket offsets
//  k_query_gather  query rows in float64, in bucket (score) order, so that a
//                  tile of consecutive queries shares one union window (the
//                  gemm over the union of candidate sets, Section 4).  Any
//                  query order gives the same result; score order only keeps
//                  the union windows tight.
//  k_window        J_q = [lo_q, hi_q) by binary search on the sorted keys,
//                  with the half-width widened outward by a rigorous bound on
//                  the score rounding (eq. (lower) is exact only for exact
//                  scores); per-tile union windows
//  k_tile_units    work units per tile
#include <hip/hip_runtime.h>

#include <climits>

#include "device_common.h"
#include "query_plan.h"
#include "snn_internal.h"

namespace snn {

namespace {
constexpr int kThreads = 256;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_query_keys(const T* __restrict__ Q, int64_t m, int d,
                                                        const double* __restrict__ mu, const double* __restrict__ v,
                                                        const double* __restrict__ key, int n, int K,
                                                        uint32_t* __restrict__ bucket, uint32_t* __restrict__ slot,
                                                        uint32_t* __restrict__ hist, double* __restrict__ qalpha,
                                                        double* __restrict__ qnorm, int* __restrict__ bad) {
  const double amin = key[0], amax = key[n - 1];
  const double scale = amax > amin ? (double)K / (amax - amin) : 0.0;
  int badloc = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const T* q = Q + i * d;
    double a = 0.0, nn = 0.0;
    for (int k = 0; k < d; ++k) {
      double qk = (double)q[k];
      if (!isfinite(qk)) badloc = 1;
      double x = qk - mu[k];
      a += x * v[k];
      double y = (double)(float)x;
      nn += y * y;
    }
    const double t = (a - amin) * scale;
    const int b = (t >= 0.0) ? (t < (double)K ? (int)t : K - 1) : 0;
    bucket[i] = (uint32_t)b;
    slot[i] = atomicAdd(&hist[b], 1u);
    qalpha[i] = a;
    qnorm[i] = sqrt(nn);
  }
  if (badloc) atomicOr(bad, 1);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_query_gather(const T* __restrict__ Q, int64_t m, int d, int dp,
                                                          const uint32_t* __restrict__ bucket,
                                                          const uint32_t* __restrict__ slot,
                                                          const uint32_t* __restrict__ boff,
                                                          const double* __restrict__ qalpha_in,
                                                          const double* __restrict__ qnorm_in,
                                                          double* __restrict__ q64, int32_t* __restrict__ qorig,
                                                          double* __restrict__ qalpha, double* __restrict__ qnorm) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m * dp; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / dp;
    const int k = (int)(e % dp);
    const int64_t s = (int64_t)boff[bucket[i]] + slot[i];
    q64[s * dp + k] = k < d ? (double)Q[i * d + k] : 0.0;
    if (k == 0) {
      qorig[s] = (int32_t)i;
      qalpha[s] = qalpha_in[i];
      qnorm[s] = qnorm_in[i];
    }
  }
}

// W_q = (R ||v|| (1 + 4 gamma_{d+3}) + key_eps + eps_q) (1 + 8u) with
// eps_q = eps_scale * ||y_q||; the bounds are then rounded outward.  The
// lower and upper binary searches run interleaved (independent loads).
// Requires T % 64 == 0 so that a wavefront never straddles two tiles.
__global__ __launch_bounds__(kThreads) void k_window(const double* __restrict__ key, int n,
                                                    const double* __restrict__ qalpha,
                                                    const double* __restrict__ qnorm, int64_t m, double w_base,
                                                    double eps_scale, int T, int sym, int32_t* __restrict__ lo_out,
                                                    int32_t* __restrict__ hi_out, int32_t* __restrict__ tlo,
                                                    int32_t* __restrict__ thi,
                                                    unsigned long long* __restrict__ pairs_window) {
  const double u = 1.1102230246251565e-16;
  __shared__ unsigned long long red[kThreads / kWave];
  unsigned long long acc = 0;  // this lane's window sizes over the grid-stride loop
  for (int64_t s0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x / kWave) * kWave; s0 < m;
       s0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = s0 + lane_id();
    int lo = INT_MAX, hi = INT_MIN;
    if (s < m) {
      const double W = (w_base + eps_scale * qnorm[s]) * (1.0 + 8.0 * u);
      const double a = qalpha[s];
      const double lv = nextafter(a - W, -INFINITY);
      const double hv = nextafter(a + W, INFINITY);
      // lo: first index with key >= lv;  hi: first index with key > hv
      int l0 = 0, l1 = n, h0 = 0, h1 = n;
      while (l0 < l1 || h0 < h1) {
        const int lm = (l0 + l1) >> 1, hm = (h0 + h1) >> 1;
        const double kl = key[min(lm, n - 1)], kh = key[min(hm, n - 1)];
        if (l0 < l1) {
          if (kl < lv)
            l0 = lm + 1;
          else
            l1 = lm;
        }
        if (h0 < h1) {
          if (kh <= hv)
            h0 = hm + 1;
          else
            h1 = hm;
        }
      }
      lo = l0;
      hi = h0;
      if (lo_out) {
        lo_out[s] = lo;
        hi_out[s] = hi;
      }
      if (hi > lo) {
        // symmetric self-query: only the candidates at or after s are scanned
        const int from = sym ? max(lo, (int)s) : lo;
        if (hi > from) acc += (unsigned long long)(hi - from);
      } else {  // empty window: neutral for the tile union
        lo = INT_MAX;
        hi = INT_MIN;
      }
    }
    const int wlo = wave_min(lo), whi = wave_max(hi);
    if (lane_id() == 0 && wlo != INT_MAX) {
      const int tile = (int)(s0 / T);
      atomicMin(&tlo[tile], wlo);
      atomicMax(&thi[tile], whi);
    }
  }
  // one counter atomic per block (same-address atomics serialise)
  const unsigned long long wc = wave_sum(acc);
  if (lane_id() == 0) red[threadIdx.x / kWave] = wc;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long c = 0;
    for (int w = 0; w < kThreads / kWave; ++w) c += red[w];
    if (c) atomicAdd(pairs_window, c);
  }
}

__global__ void k_tile_init(int32_t* __restrict__ tlo, int32_t* __restrict__ thi, int ntiles) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < ntiles; t += gridDim.x * blockDim.x) {
    tlo[t] = INT_MAX;
    thi[t] = INT_MIN;
  }
}

__global__ void k_tile_units(int32_t* __restrict__ tlo, int32_t* __restrict__ thi, int ntiles, int CH, int align,
                             int sym_T, int32_t* __restrict__ units) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < ntiles; t += gridDim.x * blockDim.x) {
    int a = tlo[t], b = thi[t];
    if (sym_T > 0 && a != INT_MAX) a = max(a, t * sym_T);  // symmetric self-query: from the tile's first row
    if (a == INT_MAX || b <= a) {
      tlo[t] = 0;
      thi[t] = 0;
      units[t] = 0;
    } else {
      a -= a % align;
      b = (int)((((int64_t)b + align - 1) / align) * align);
      tlo[t] = a;
      thi[t] = b;
      units[t] = (int32_t)(((int64_t)b - a + CH - 1) / CH);
    }
  }
}

__global__ void k_group_units(const int32_t* __restrict__ units, int ntiles, int G, int32_t* __restrict__ gunits) {
  const int ngroups = (ntiles + G - 1) / G;
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < ngroups; g += gridDim.x * blockDim.x) {
    const int t0 = g * G, t1 = min(ntiles, t0 + G);
    int mx = 0;
    for (int t = t0; t < t1; ++t) mx = max(mx, units[t]);
    gunits[g] = mx * (t1 - t0);
  }
}

// Pairs the screen evaluates: wavefronts (of qpw query slots) with at least
// one real query, times their slots, times the tile's scanned window.
__global__ void k_executed(const int32_t* __restrict__ tlo, const int32_t* __restrict__ thi, int ntiles, int T,
                           int64_t m, int qpw, unsigned long long* __restrict__ out) {
  unsigned long long e = 0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < ntiles; t += gridDim.x * blockDim.x) {
    const int64_t valid = min((int64_t)T, max((int64_t)0, m - (int64_t)t * T));
    const int64_t waves = (valid + qpw - 1) / qpw;
    e += (unsigned long long)(waves * qpw) * (unsigned long long)max(0, thi[t] - tlo[t]);
  }
  e = wave_sum(e);
  if (lane_id() == 0 && e) atomicAdd(out, e);
}

// ---------------------------------------------------------------- launchers
namespace {
int grid_for(int64_t work, int cap) {
  int64_t g = (work + kThreads - 1) / kThreads;
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}
}  // namespace

void launch_tile_init(int32_t* tlo, int32_t* thi, int ntiles, hipStream_t s) {
  k_tile_init<<<grid_for(ntiles, 1024), kThreads, 0, s>>>(tlo, thi, ntiles);
  SNN_LAUNCH_CHECK();
}

void launch_tile_units(int32_t* tlo, int32_t* thi, int ntiles, int CH, int align, int32_t* units, hipStream_t s) {
  k_tile_units<<<grid_for(ntiles, 1024), kThreads, 0, s>>>(tlo, thi, ntiles, CH, align, 0, units);
  SNN_LAUNCH_CHECK();
}

void launch_executed(const int32_t* tlo, const int32_t* thi, int ntiles, int T, int64_t m, int qpw,
                     unsigned long long* out, hipStream_t s) {
  k_executed<<<grid_for(ntiles, 64), kThreads, 0, s>>>(tlo, thi, ntiles, T, m, qpw, out);
  SNN_LAUNCH_CHECK();
}

void launch_group_units(const int32_t* units, int ntiles, int G, int32_t* gunits, hipStream_t s) {
  k_group_units<<<grid_for((ntiles + G - 1) / G, 1024), kThreads, 0, s>>>(units, ntiles, G, gunits);
  SNN_LAUNCH_CHECK();
}

int query_buckets(int64_t m) {
  int K = 256;
  while (K < 65536 && K < m) K <<= 1;
  return K;
}

void launch_query_keys(snn_dtype dt, const void* Q, int64_t m, int d, const double* mu, const double* v,
                       const double* key, int n, int K, uint32_t* bucket, uint32_t* slot, uint32_t* hist,
                       double* qalpha, double* qnorm, int* bad, hipStream_t s) {
  const int g = grid_for(m, 8192);
  if (dt == SNN_F32)
    k_query_keys<float><<<g, kThreads, 0, s>>>((const float*)Q, m, d, mu, v, key, n, K, bucket, slot, hist, qalpha,
                                               qnorm, bad);
  else
    k_query_keys<double><<<g, kThreads, 0, s>>>((const double*)Q, m, d, mu, v, key, n, K, bucket, slot, hist,
                                                qalpha, qnorm, bad);
  SNN_LAUNCH_CHECK();
}

void launch_query_gather(snn_dtype dt, const void* Q, int64_t m, int d, int dp, const uint32_t* bucket,
                         const uint32_t* slot, const uint32_t* boff, const double* qalpha_in, const double* qnorm_in,
                         double* q64, int32_t* qorig, double* qalpha, double* qnorm, hipStream_t s) {
  const int g = grid_for(m * dp, 16384);
  if (dt == SNN_F32)
    k_query_gather<float><<<g, kThreads, 0, s>>>((const float*)Q, m, d, dp, bucket, slot, boff, qalpha_in, qnorm_in,
                                                 q64, qorig, qalpha, qnorm);
  else
    k_query_gather<double><<<g, kThreads, 0, s>>>((const double*)Q, m, d, dp, bucket, slot, boff, qalpha_in,
                                                  qnorm_in, q64, qorig, qalpha, qnorm);
  SNN_LAUNCH_CHECK();
}

void launch_windows(const double* key, int n, const double* qalpha, const double* qnorm, int64_t m, double w_base,
                    double eps_scale, int T, int CH, int align, int ntiles, int sym, int32_t* lo, int32_t* hi,
                    int32_t* tlo, int32_t* thi, int32_t* units, unsigned long long* pairs_window, hipStream_t s) {
  k_tile_init<<<grid_for(ntiles, 1024), kThreads, 0, s>>>(tlo, thi, ntiles);
  SNN_LAUNCH_CHECK();
  if (m > 0) {
    k_window<<<grid_for(m, 2048), kThreads, 0, s>>>(key, n, qalpha, qnorm, m, w_base, eps_scale, T, sym, lo, hi,
                                                    tlo, thi, pairs_window);
    SNN_LAUNCH_CHECK();
  }
  k_tile_units<<<grid_for(ntiles, 1024), kThreads, 0, s>>>(tlo, thi, ntiles, CH, align, sym ? T : 0, units);
  SNN_LAUNCH_CHECK();
}

}  // namespace snn
