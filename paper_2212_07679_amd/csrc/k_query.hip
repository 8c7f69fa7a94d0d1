// Query preparation and windows (Algorithm 2, steps 2-4, Section 3.2).
//
//  k_query_keys    x_q = q - mu, alpha_q = x_q . v (float64), ||fl32(x_q)||,
//                  and a bucket of alpha_q on a uniform grid over the range of
//                  the index scores; each query takes a slot in its bucket
//  (scan)          bucket offsets (one launch, look-back)
//  k_query_gather  query rows in float64, in bucket (score) order, so that a
//                  tile of consecutive queries shares one union window (the
//                  gemm over the union of candidate sets, Section 4), and the
//                  screen's query operands and start values.  Any query
//                  order gives the same result; score order only keeps the
//                  union windows tight.
//  k_window        J_q = [lo_q, hi_q) by binary search on the sorted keys,
//                  with the half-width widened outward by a rigorous bound on
//                  the score rounding (eq. (lower) is exact only for exact
//                  scores), each search confined to one cell of a uniform
//                  grid over the score range (k_window_table); per-tile
//                  union windows
//  k_tile_plan     work units per tile and their offsets (one workgroup)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <type_traits>

#include "device_common.h"
#include "query_plan.h"
#include "snn_internal.h"

namespace snn {

namespace {
constexpr int kThreads = 256;
}

// G lanes per query row (coalesced row reads); the row's partial sums meet
// by shuffles within its G lanes in a fixed order (deterministic; any order
// stays within the float64 bounds the windows and the screen allow for).
template <typename T, int G>
__global__ __launch_bounds__(kThreads) void k_query_keys(const T* __restrict__ Q, int64_t m, int d,
                                                        const double* __restrict__ mu, const double* __restrict__ v,
                                                        const double* __restrict__ key, int n, int K,
                                                        uint32_t* __restrict__ bucket, uint32_t* __restrict__ slot,
                                                        uint32_t* __restrict__ hist, double* __restrict__ qalpha,
                                                        double* __restrict__ qnorm, int* __restrict__ bad) {
  const double amin = key[0], amax = key[n - 1];
  const double scale = amax > amin ? (double)K / (amax - amin) : 0.0;
  const int sub = threadIdx.x % G;
  int badloc = 0;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G; i < m;
       i += ((int64_t)gridDim.x * blockDim.x) / G) {
    const T* q = Q + i * d;
    double a = 0.0, nn = 0.0;
    for (int k = sub; k < d; k += G) {
      const double qk = (double)q[k];
      if (!isfinite(qk)) badloc = 1;
      const double x = qk - mu[k];
      a += x * v[k];
      const double y = (double)(float)x;
      nn += y * y;
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
      a += __shfl_xor(a, off, G);
      nn += __shfl_xor(nn, off, G);
    }
    if (sub == 0) {
      const double t = (a - amin) * scale;
      const int b = (t >= 0.0) ? (t < (double)K ? (int)t : K - 1) : 0;
      bucket[i] = (uint32_t)b;
      slot[i] = atomicAdd(&hist[b], 1u);
      qalpha[i] = a;
      qnorm[i] = sqrt(nn);
    }
  }
  if (badloc) atomicOr(bad, 1);
}

// The same for float rows of d <= 16: four lanes per row, each a run of
// four coordinates (one 16-byte load where the rows are 16-byte aligned).
__global__ __launch_bounds__(kThreads) void k_query_keys4(const float* __restrict__ Q, int64_t m, int d,
                                                         const double* __restrict__ mu,
                                                         const double* __restrict__ v,
                                                         const double* __restrict__ key, int n, int K,
                                                         uint32_t* __restrict__ bucket, uint32_t* __restrict__ slot,
                                                         uint32_t* __restrict__ hist, double* __restrict__ qalpha,
                                                         double* __restrict__ qnorm, int* __restrict__ bad, int vec) {
  const double amin = key[0], amax = key[n - 1];
  const double scale = amax > amin ? (double)K / (amax - amin) : 0.0;
  const int sub = threadIdx.x & 3, k0 = 4 * sub;
  int badloc = 0;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 4; i < m;
       i += ((int64_t)gridDim.x * blockDim.x) / 4) {
    const float* q = Q + i * d;
    float qv[4];
    if (vec && k0 < d) {
      const float4 t = *reinterpret_cast<const float4*>(q + k0);
      qv[0] = t.x, qv[1] = t.y, qv[2] = t.z, qv[3] = t.w;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) qv[j] = k0 + j < d ? q[k0 + j] : 0.f;
    }
    double a = 0.0, nn = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (k0 + j < d) {
        const double qk = (double)qv[j];
        if (!isfinite(qk)) badloc = 1;
        const double x = qk - mu[k0 + j];
        a += x * v[k0 + j];
        const double y = (double)(float)x;
        nn += y * y;
      }
    a += __shfl_xor(a, 1, 4);
    nn += __shfl_xor(nn, 1, 4);
    a += __shfl_xor(a, 2, 4);
    nn += __shfl_xor(nn, 2, 4);
    if (sub == 0) {
      const double t = (a - amin) * scale;
      const int b = (t >= 0.0) ? (t < (double)K ? (int)t : K - 1) : 0;
      bucket[i] = (uint32_t)b;
      slot[i] = atomicAdd(&hist[b], 1u);
      qalpha[i] = a;
      qnorm[i] = sqrt(nn);
    }
  }
  if (badloc) atomicOr(bad, 1);
}

// G lanes per query row: the row's destination slot is read once per group,
// its elements are copied G at a time, and the lanes build the screen's
// operand row and start value from the centred row y = fl32(q - mu)
// (k_cand_mfma.hip): 16-bit rows [bf16(y)], [hi | hi | lo] or [fp16(2^e y)]
// with C_q, or the fp32 row [y, C_q, 0 ...].
template <typename T, int G>
__global__ __launch_bounds__(kThreads) void k_query_gather(const T* __restrict__ Q, int64_t m, int d, int dp,
                                                          const uint32_t* __restrict__ bucket,
                                                          const uint32_t* __restrict__ slot,
                                                          const uint32_t* __restrict__ boff,
                                                          const double* __restrict__ qalpha_in,
                                                          const double* __restrict__ qnorm_in,
                                                          double* __restrict__ q64, int32_t* __restrict__ qorig,
                                                          double* __restrict__ qalpha, double* __restrict__ qnorm,
                                                          const double* __restrict__ mu, QueryOperands op) {
  const int sub = threadIdx.x % G;
  const int terms = op.kind == kOpBf16x3 ? 3 : 1;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G; i < m;
       i += ((int64_t)gridDim.x * blockDim.x) / G) {
    const int64_t s = (int64_t)boff[bucket[i]] + slot[i];
    const T* q = Q + i * d;
    if (q64)
      for (int k = sub; k < dp; k += G) q64[s * dp + k] = k < d ? (double)q[k] : 0.0;
    if (sub == 0) {
      qorig[s] = (int32_t)i;
      qalpha[s] = qalpha_in[i];
      qnorm[s] = qnorm_in[i];
    }
    if (op.mode == kQOpNone) continue;
    double nn = 0.0;
    for (int k = sub; k < d; k += G) {
      const float y = (float)((double)q[k] - mu[k]);
      nn += (double)y * (double)y;
    }
    // any summation order stays within the gamma_{d+1} bound the start value allows for
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) nn += __shfl_xor(nn, off, G);
    const float c = screen_threshold(op.b, 0.5 * nn, sqrt(nn) * (1.0 + 1e-15));
    if (op.mode == kQOp16) {
      uint16_t* o = op.qop + s * op.KA;
      for (int k = sub; k < op.KA; k += G) {
        uint16_t v = 0;
        if (k < terms * d) {
          const int seg = k / d, cc = k % d;
          const float y = (float)((double)q[cc] - mu[cc]);
          if (op.kind == kOpF16) {
            v = __builtin_bit_cast(uint16_t, (_Float16)ldexpf(y, op.e));
          } else {
            const uint16_t hi = f32_to_bf16_rne(y);
            v = (seg == 2) ? f32_to_bf16_rne(y - bf16_to_f32(hi)) : hi;
          }
        }
        o[k] = v;
      }
      if (sub == 0) op.cthr[s] = c;
    } else {
      float* o = op.vq + s * op.DV;
      for (int k = sub; k < op.DV; k += G) o[k] = k < d ? (float)((double)q[k] - mu[k]) : (k == d ? c : 0.f);
    }
  }
}

// The same for float rows of at most 16 values per output row (d <= 16 and
// one operand value per coordinate): four lanes per row, each a run of four
// coordinates read once and written with wide stores (float64 row: 32
// bytes, operand row: 8 bytes per lane).  Results are identical to
// k_query_gather's.
__global__ __launch_bounds__(kThreads) void k_query_gather4(const float* __restrict__ Q, int64_t m, int d, int dp,
                                                           const uint32_t* __restrict__ bucket,
                                                           const uint32_t* __restrict__ slot,
                                                           const uint32_t* __restrict__ boff,
                                                           const double* __restrict__ qalpha_in,
                                                           const double* __restrict__ qnorm_in,
                                                           double* __restrict__ q64, int32_t* __restrict__ qorig,
                                                           double* __restrict__ qalpha, double* __restrict__ qnorm,
                                                           const double* __restrict__ mu, QueryOperands op,
                                                           int vec) {
  const int sub = threadIdx.x & 3, k0 = 4 * sub;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 4; i < m;
       i += ((int64_t)gridDim.x * blockDim.x) / 4) {
    const int64_t s = (int64_t)boff[bucket[i]] + slot[i];
    const float* q = Q + i * d;
    float qv[4];
    if (vec && k0 < d) {  // rows 16-byte aligned
      const float4 t = *reinterpret_cast<const float4*>(q + k0);
      qv[0] = t.x, qv[1] = t.y, qv[2] = t.z, qv[3] = t.w;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) qv[j] = k0 + j < d ? q[k0 + j] : 0.f;
    }
    if (q64 && k0 < dp) {  // dp is a multiple of 4
      double2* o = reinterpret_cast<double2*>(q64 + s * dp + k0);
      o[0] = make_double2((double)qv[0], (double)qv[1]);
      o[1] = make_double2((double)qv[2], (double)qv[3]);
    }
    if (sub == 0) {
      qorig[s] = (int32_t)i;
      qalpha[s] = qalpha_in[i];
      qnorm[s] = qnorm_in[i];
    }
    if (op.mode == kQOpNone) continue;
    float y[4];
    double nn = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      y[j] = k0 + j < d ? (float)((double)qv[j] - mu[k0 + j]) : 0.f;
      nn += (double)y[j] * (double)y[j];
    }
    // any summation order stays within the gamma_{d+1} bound the start value allows for
    nn += __shfl_xor(nn, 1, 4);
    nn += __shfl_xor(nn, 2, 4);
    const float c = screen_threshold(op.b, 0.5 * nn, sqrt(nn) * (1.0 + 1e-15));
    if (k0 < op.KA) {  // KA is a multiple of 16
      uint16_t v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        v[j] = op.kind == kOpF16 ? __builtin_bit_cast(uint16_t, (_Float16)ldexpf(y[j], op.e)) : f32_to_bf16_rne(y[j]);
      *reinterpret_cast<uint2*>(op.qop + s * op.KA + k0) =
          make_uint2((uint32_t)v[0] | ((uint32_t)v[1] << 16), (uint32_t)v[2] | ((uint32_t)v[3] << 16));
    }
    if (sub == 0) op.cthr[s] = c;
  }
}

// Start of every cell of a uniform grid over the score range: start[c] is
// the first sorted position whose key lies in cell c or beyond (start[C] =
// n).  The cell of a score x is floor((x - key[0]) * C / (key[n-1] -
// key[0])) clamped to [0, C - 1], monotone in x, so every key below a score
// x's cell is below x and every key beyond it above: a search for x stays
// within [start[cell(x)], start[cell(x) + 1]].
__device__ __forceinline__ int score_cell(double x, double amin, double scale, int C) {
  const double t = (x - amin) * scale;
  return t >= 0.0 ? (t < (double)C ? (int)t : C - 1) : 0;
}

__global__ __launch_bounds__(kThreads) void k_window_table(const double* __restrict__ key, int n, int C,
                                                          int32_t* __restrict__ start) {
  const double amin = key[0], amax = key[n - 1];
  const double scale = amax > amin ? (double)C / (amax - amin) : 0.0;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    const int cj = score_cell(key[j], amin, scale, C);
    const int cp = j > 0 ? score_cell(key[j - 1], amin, scale, C) : -1;
    for (int c = cp + 1; c <= cj; ++c) start[c] = j;
    if (j == n - 1)
      for (int c = cj + 1; c <= C; ++c) start[c] = n;
  }
}

// W_q = (R ||v|| (1 + 4 gamma_{d+3}) + key_eps + eps_q) (1 + 8u) with
// eps_q = eps_scale * ||y_q||; the bounds are then rounded outward.  The
// lower and upper binary searches run interleaved (independent loads).
// Requires T % 64 == 0 so that a wavefront never straddles two tiles.
__global__ __launch_bounds__(kThreads) void k_window(const double* __restrict__ key, int n,
                                                    const int32_t* __restrict__ cells, int C,
                                                    const double* __restrict__ qalpha,
                                                    const double* __restrict__ qnorm, int64_t m, double w_base,
                                                    double eps_scale, int T, int sym, int32_t* __restrict__ lo_out,
                                                    int32_t* __restrict__ hi_out, int32_t* __restrict__ tlo,
                                                    int32_t* __restrict__ thi,
                                                    unsigned long long* __restrict__ wpart) {
  const double u = 1.1102230246251565e-16;
  const double amin = key[0], amax = key[n - 1];
  const double scale = amax > amin ? (double)C / (amax - amin) : 0.0;
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
      // lo: first index with key >= lv;  hi: first index with key > hv,
      // each within the grid cell of its bound
      const int cl = score_cell(lv, amin, scale, C), ch = score_cell(hv, amin, scale, C);
      int l0 = cells[cl], l1 = cells[cl + 1], h0 = cells[ch], h1 = cells[ch + 1];
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
  // one partial count per workgroup, summed by k_tile_plan (atomics on a
  // single address serialise)
  const unsigned long long wc = wave_sum(acc);
  if (lane_id() == 0) red[threadIdx.x / kWave] = wc;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long c = 0;
    for (int w = 0; w < kThreads / kWave; ++w) c += red[w];
    wpart[blockIdx.x] = c;
  }
}

// Per-call initialisation in one launch: the control words, the per-slot
// row counters, the bucket histogram of the query sort and the tile windows
// (empty: tlo = INT_MAX, thi = INT_MIN, lowered / raised by k_window).
__global__ __launch_bounds__(kThreads) void k_query_init(unsigned long long* __restrict__ ctl, int ctl_words,
                                                        int32_t* __restrict__ row_cnt, int64_t m,
                                                        uint32_t* __restrict__ hist, int nb,
                                                        int32_t* __restrict__ tlo, int32_t* __restrict__ thi,
                                                        int ntiles, int mark_word) {
  const int64_t top = max(max((int64_t)ctl_words, m), (int64_t)max(nb, ntiles));
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < top; i += (int64_t)gridDim.x * blockDim.x) {
    // (the word mark_word of the control block takes the device clock: the
    // start of the call)
    if (i < ctl_words) ctl[i] = i == mark_word ? (unsigned long long)wall_clock64() : 0ull;
    if (i < m) row_cnt[i] = 0;
    if (hist && i < nb) hist[i] = 0u;
    if (i < ntiles) {
      tlo[i] = INT_MAX;
      thi[i] = INT_MIN;
    }
  }
}

// The tile plan in one single-workgroup launch (the tile count is small
// next to the work): clamp and align every tile window (symmetric
// self-queries start a tile at its own first row), count its work units,
// add the evaluated pairs (stats), reserve G x max units per group of G
// tiles, and scan the groups into unit offsets (unit_off[ngroups] = total).
constexpr int kAbsChunks = 8;

__device__ void tile_plan_body(const TilePlanArgs& pa) {
  int32_t* __restrict__ tlo = pa.tlo;
  int32_t* __restrict__ thi = pa.thi;
  int32_t* __restrict__ units = pa.units;
  int64_t* __restrict__ unit_off = pa.unit_off;
  int32_t* __restrict__ gbase = pa.gbase;
  unsigned long long* __restrict__ executed = pa.executed;
  const unsigned long long* __restrict__ wpart = pa.wpart;
  unsigned long long* __restrict__ pairs_window = pa.pairs_window;
  const int ntiles = pa.ntiles, CH = pa.CH, align = pa.align, sym_T = pa.sym_T, G = pa.G, T = pa.T, qpw = pa.qpw;
  const int nwpart = pa.nwpart;
  const int64_t m = pa.m;
  __shared__ int64_t carry;
  __shared__ int64_t wsum[1024 / kWave];  // (any workgroup of up to 1024 threads)
  if (pairs_window) {  // the window-pair total from the per-workgroup partials
    __shared__ unsigned long long pw_s[1024 / kWave];
    unsigned long long pw = 0;
    for (int b = threadIdx.x; b < nwpart; b += blockDim.x) pw += wpart[b];
    pw = wave_sum(pw);
    if (lane_id() == 0) pw_s[threadIdx.x / kWave] = pw;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long t = 0;
      for (int w = 0; w < (int)(blockDim.x / kWave); ++w) t += pw_s[w];
      *pairs_window = t;
    }
  }
  unsigned long long e = 0;
  for (int t = threadIdx.x; t < ntiles; t += blockDim.x) {
    int a = tlo[t], b = thi[t];
    if (sym_T > 0 && a != INT_MAX) a = max(a, t * sym_T);
    int u = 0;
    if (a == INT_MAX || b <= a) {
      a = 0;
      b = 0;
    } else {
      a -= a % align;
      b = (int)((((int64_t)b + align - 1) / align) * align);
      u = (int)(((int64_t)b - a + CH - 1) / CH);
    }
    tlo[t] = a;
    thi[t] = b;
    units[t] = u;
    if (executed) {
      const int64_t valid = min((int64_t)T, max((int64_t)0, m - (int64_t)t * T));
      e += (unsigned long long)(((valid + qpw - 1) / qpw) * qpw) * (unsigned long long)(b - a);
    }
  }
  if (executed) {
    e = wave_sum(e);
    if (lane_id() == 0 && e) atomicAdd(executed, e);
  }
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const int ngroups = (ntiles + G - 1) / G;
  const int lane = lane_id(), w = threadIdx.x / kWave;
  for (int g0 = 0; g0 < ngroups; g0 += blockDim.x) {
    const int g = g0 + threadIdx.x;
    int64_t v = 0;
    if (g < ngroups) {
      const int t0 = g * G, t1 = min(ntiles, t0 + G);
      // absolute chunks when the windows average at least kAbsChunks
      // chunks (then the chunks cut at window ends cost little)
      int b0 = INT_MAX, b1 = 0, mx = 0, nt = 0;
      int64_t len = 0;
      for (int t = t0; t < t1; ++t)
        if (units[t] > 0) {
          b0 = min(b0, tlo[t] / CH);
          b1 = max(b1, (thi[t] - 1) / CH + 1);
          mx = max(mx, units[t]);
          len += thi[t] - tlo[t];
          ++nt;
        }
      if (nt > 0 && len >= (int64_t)kAbsChunks * CH * nt) {
        gbase[g] = b0;
        v = (int64_t)(b1 - b0) * (t1 - t0);
      } else {
        gbase[g] = -1;
        v = (int64_t)mx * (t1 - t0);
      }
    }
    // exclusive scan of v over the block, offset by the running carry
    int64_t x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int64_t y = __shfl_up(x, o, kWave);
      if (lane >= o) x += y;
    }
    if (lane == kWave - 1) wsum[w] = x;
    __syncthreads();
    int64_t pre = carry, tot = 0;
    for (int k = 0; k < (int)(blockDim.x / kWave); ++k) {
      if (k < w) pre += wsum[k];
      tot += wsum[k];
    }
    if (g < ngroups) unit_off[g] = pre + x - v;
    __syncthreads();
    if (threadIdx.x == 0) carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) unit_off[ngroups] = carry;
}

__global__ __launch_bounds__(1024) void k_tile_plan(TilePlanArgs pa) { tile_plan_body(pa); }

// ---------------------------------------------------------------- launchers
namespace {
int grid_for(int64_t work, int cap) {
  int64_t g = (work + kThreads - 1) / kThreads;
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}
}  // namespace

// about as many buckets as queries, at most 65536: the key pass takes each
// query's slot with an atomic on its bucket's count, and atomics on one
// cache line serialise (measured on 1e5 clustered queries: 11 us with 65536
// buckets, 27 us with 4096)
int query_buckets(int64_t m) {
  int K = 256;
  while (K < 65536 && K < m) K <<= 1;
  return K;
}

namespace {
// lanes per query row: enough to read a short row in one step, at most 16
int query_row_lanes(int width) { return width <= 4 ? 4 : (width <= 8 ? 8 : 16); }

template <typename T, int G>
void query_keys_t(const T* Q, int64_t m, int d, const double* mu, const double* v, const double* key, int n, int K,
                  uint32_t* bucket, uint32_t* slot, uint32_t* hist, double* qalpha, double* qnorm, int* bad,
                  hipStream_t s) {
  k_query_keys<T, G><<<grid_for(m * G, 8192), kThreads, 0, s>>>(Q, m, d, mu, v, key, n, K, bucket, slot, hist,
                                                                qalpha, qnorm, bad);
}

template <typename T>
void query_keys_d(const T* Q, int64_t m, int d, const double* mu, const double* v, const double* key, int n, int K,
                  uint32_t* bucket, uint32_t* slot, uint32_t* hist, double* qalpha, double* qnorm, int* bad,
                  hipStream_t s) {
  if (std::is_same<T, float>::value && d <= 16) {
    const int vec = d % 4 == 0 && reinterpret_cast<uintptr_t>(Q) % 16 == 0;
    k_query_keys4<<<grid_for(m * 4, 8192), kThreads, 0, s>>>(reinterpret_cast<const float*>(Q), m, d, mu, v, key, n,
                                                            K, bucket, slot, hist, qalpha, qnorm, bad, vec);
    return;
  }
  switch (query_row_lanes(d)) {
    case 4: query_keys_t<T, 4>(Q, m, d, mu, v, key, n, K, bucket, slot, hist, qalpha, qnorm, bad, s); break;
    case 8: query_keys_t<T, 8>(Q, m, d, mu, v, key, n, K, bucket, slot, hist, qalpha, qnorm, bad, s); break;
    default: query_keys_t<T, 16>(Q, m, d, mu, v, key, n, K, bucket, slot, hist, qalpha, qnorm, bad, s); break;
  }
}

}  // namespace

void launch_query_keys(snn_dtype dt, const void* Q, int64_t m, int d, const double* mu, const double* v,
                       const double* key, int n, int K, uint32_t* bucket, uint32_t* slot, uint32_t* hist,
                       double* qalpha, double* qnorm, int* bad, unsigned long long* scan_state, int* scan_err,
                       hipStream_t s) {
  if (dt == SNN_F32)
    query_keys_d<float>((const float*)Q, m, d, mu, v, key, n, K, bucket, slot, hist, qalpha, qnorm, bad, s);
  else
    query_keys_d<double>((const double*)Q, m, d, mu, v, key, n, K, bucket, slot, hist, qalpha, qnorm, bad, s);
  SNN_LAUNCH_CHECK();
  lookback_scan_u32(hist, K, scan_state, scan_err, s);
}

namespace {
template <typename T>
void query_gather_d(const T* Q, int64_t m, int d, int dp, const uint32_t* bucket, const uint32_t* slot,
                    const uint32_t* boff, const double* qalpha_in, const double* qnorm_in, double* q64, int32_t* qorig,
                    double* qalpha, double* qnorm, const double* mu, const QueryOperands& op, hipStream_t s) {
  const int width = std::max(dp, op.mode == kQOp16 ? op.KA : (op.mode == kQOp32 ? op.DV : 0));
  if (std::is_same<T, float>::value && width <= 16 &&
      (op.mode == kQOpNone || (op.mode == kQOp16 && op.kind != kOpBf16x3))) {
    const int vec = d % 4 == 0 && reinterpret_cast<uintptr_t>(Q) % 16 == 0;
    k_query_gather4<<<grid_for(m * 4, 8192), kThreads, 0, s>>>(reinterpret_cast<const float*>(Q), m, d, dp, bucket,
                                                              slot, boff, qalpha_in, qnorm_in, q64, qorig, qalpha,
                                                              qnorm, mu, op, vec);
    return;
  }
  const int G = query_row_lanes(width);
  const int g = grid_for(m * G, 8192);
  if (G == 4)
    k_query_gather<T, 4><<<g, kThreads, 0, s>>>(Q, m, d, dp, bucket, slot, boff, qalpha_in, qnorm_in, q64, qorig,
                                                qalpha, qnorm, mu, op);
  else if (G == 8)
    k_query_gather<T, 8><<<g, kThreads, 0, s>>>(Q, m, d, dp, bucket, slot, boff, qalpha_in, qnorm_in, q64, qorig,
                                                qalpha, qnorm, mu, op);
  else
    k_query_gather<T, 16><<<g, kThreads, 0, s>>>(Q, m, d, dp, bucket, slot, boff, qalpha_in, qnorm_in, q64, qorig,
                                                 qalpha, qnorm, mu, op);
}

}  // namespace

void launch_query_gather(snn_dtype dt, const void* Q, int64_t m, int d, int dp, const uint32_t* bucket,
                         const uint32_t* slot, const uint32_t* boff, const double* qalpha_in, const double* qnorm_in,
                         double* q64, int32_t* qorig, double* qalpha, double* qnorm, const double* mu,
                         const QueryOperands& op, hipStream_t s) {
  if (dt == SNN_F32)
    query_gather_d<float>((const float*)Q, m, d, dp, bucket, slot, boff, qalpha_in, qnorm_in, q64, qorig, qalpha,
                          qnorm, mu, op, s);
  else
    query_gather_d<double>((const double*)Q, m, d, dp, bucket, slot, boff, qalpha_in, qnorm_in, q64, qorig, qalpha,
                           qnorm, mu, op, s);
  SNN_LAUNCH_CHECK();
}

int window_table_cells(int64_t n) { return (int)std::max<int64_t>(1, n / 8); }

void launch_window_table(const double* key, int n, int C, int32_t* start, hipStream_t s) {
  k_window_table<<<grid_for(n, 8192), kThreads, 0, s>>>(key, n, C, start);
  SNN_LAUNCH_CHECK();
}

void launch_query_init(unsigned long long* ctl, int ctl_words, int32_t* row_cnt, int64_t m, uint32_t* hist, int nb,
                       int32_t* tlo, int32_t* thi, int ntiles, hipStream_t s, int mark_word) {
  const int64_t top = std::max(std::max((int64_t)ctl_words, m), (int64_t)std::max(nb, ntiles));
  k_query_init<<<grid_for(top, 4096), kThreads, 0, s>>>(ctl, ctl_words, row_cnt, m, hist, nb, tlo, thi, ntiles,
                                                        mark_word);
  SNN_LAUNCH_CHECK();
}

__global__ void k_clock_mark(unsigned long long* out) {
  if (threadIdx.x == 0) *out = (unsigned long long)wall_clock64();
}

void launch_clock_mark(unsigned long long* out, hipStream_t s) {
  k_clock_mark<<<1, 64, 0, s>>>(out);
  SNN_LAUNCH_CHECK();
}

int window_blocks(int64_t m) { return m > 0 ? grid_for(m, kWindowMaxBlocks) : 0; }

void launch_windows_plan(const double* key, int n, const int32_t* cells, int C, const double* qalpha,
                         const double* qnorm, int64_t m, double w_base, double eps_scale, int T, int sym, int32_t* lo,
                         int32_t* hi, const TilePlanArgs& plan, hipStream_t s) {
  // (The plan run by the last k_window workgroup to finish, found with a
  // ticket, gave no shorter call: with device-scope fences it took 20 us
  // longer, as such a fence writes back the XCD's whole L2, and with
  // device-scope loads and workgroup fences it was no faster.)
  TilePlanArgs pa = plan;
  pa.nwpart = window_blocks(m);
  if (m > 0) {
    k_window<<<pa.nwpart, kThreads, 0, s>>>(key, n, cells, C, qalpha, qnorm, m, w_base, eps_scale, T, sym, lo, hi,
                                            plan.tlo, plan.thi, const_cast<unsigned long long*>(plan.wpart));
    SNN_LAUNCH_CHECK();
  }
  k_tile_plan<<<1, 1024, 0, s>>>(pa);
  SNN_LAUNCH_CHECK();
}

void launch_tile_plan(int32_t* tlo, int32_t* thi, int ntiles, int CH, int align, int sym, int32_t* units, int G,
                      int64_t* unit_off, int32_t* gbase, int T, int64_t m, int qpw, unsigned long long* executed,
                      const unsigned long long* wpart, int nwpart, unsigned long long* pairs_window,
                      hipStream_t s) {
  const TilePlanArgs pa{tlo, thi, ntiles, CH, align, sym ? T : 0, units, G, unit_off, gbase, T, m, qpw, executed,
                        wpart, nwpart, pairs_window};
  k_tile_plan<<<1, 1024, 0, s>>>(pa);
  SNN_LAUNCH_CHECK();
}

}  // namespace snn
