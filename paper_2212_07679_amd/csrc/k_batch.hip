// Batched index construction and query preparation for many independent
// instances (the batching form).  Each kernel covers every instance at once;
// instance data is found through the descriptor table (batch_plan.h), so one
// launch serves instances of any mix of n, m, d and R.
//
// Index (Algorithm 1, Section 3.1, per instance):
//   kb_colsum / kb_colsum_final   column means in float64 over row chunks
//   kb_gram / kb_gram_final       centred Gram matrix C = X^T X
//   kb_power                      power iteration for the top eigenvector
//                                 (any unit direction keeps the result exact,
//                                 eq. (lower); only window sizes depend on it)
//   kb_project                    keys fl32(x . v), max ||fl32(x)||^2
//   (radix sort by key, then by instance: stable, so each instance ends up
//    contiguous and in score order)
//   kb_finalize                   window widths and screen constants
//   kb_gather / kb_pad_rows       rows in score order: float64 originals,
//                                 h = ||y||^2 / 2, bf16 screen operands
// Queries (Algorithm 2, Section 3.2):
//   kb_query_keys, (sort), kb_query_gather / kb_query_pad, kb_window
// Survivors of the candidate screen:
//   kb_recheck (normative float64 rule), kb_scatter, kb_outputs_*.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>

#include "batch_plan.h"
#include "device_common.h"
#include "snn_internal.h"

#pragma clang fp contract(off)

namespace snn {

namespace {

constexpr int kThreads = 256;
constexpr double kU64 = 1.1102230246251565e-16;
constexpr double kU32 = 5.9604644775390625e-08;

__device__ __forceinline__ double gamma64d(int k) { return k * kU64 / (1.0 - k * kU64); }

// Largest i in [0, count) with off[i] <= x (off: count + 1 non-decreasing entries).
__device__ __forceinline__ int find_seg(const int64_t* __restrict__ off, int count, int64_t x) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= x)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Screen operand value k of a row (see k_operands in k_index.hip for the
// layouts): terms = 1: bf16(y_k); terms = 3: candidates [hi | lo | hi],
// queries [hi | hi | lo], hi = bf16(y), lo = bf16(y - hi).
template <typename T>
__device__ __forceinline__ uint16_t operand_value(int terms, int d, int k, const T* __restrict__ x,
                                                  const double* __restrict__ mu, bool query, int e16) {
  if (terms == kOpF16) {  // fp16 of the row scaled by 2^e16 (exact scaling, one rounding)
    if (k >= d) return 0;
    return __builtin_bit_cast(uint16_t, (_Float16)ldexpf((float)((double)x[k] - mu[k]), e16));
  }
  if (terms == 1) {
    if (k >= d) return 0;
    return f32_to_bf16_rne((float)((double)x[k] - mu[k]));
  }
  if (k >= 3 * d) return 0;
  const int seg = k / d, c = k % d;
  const float y = (float)((double)x[c] - mu[c]);
  const uint16_t hi = f32_to_bf16_rne(y);
  const bool take_lo = query ? seg == 2 : seg == 1;
  return take_lo ? f32_to_bf16_rne(y - bf16_to_f32(hi)) : hi;
}

// lanes per row in the row kernels (gathers of data and query rows)
constexpr int kQG = 16;

// KA bf16 values of one row as 16-byte stores: dst[c8] for c8 < KA / 8, where
// dst(c8) gives the address of the c8-th group of 8 values; groups c8_0,
// c8_0 + c8_step, ... (several lanes may share a row).
template <typename T, typename Dst>
__device__ __forceinline__ void write_operand_row(int terms, int d, int KA, const T* __restrict__ x,
                                                  const double* __restrict__ mu, bool query, int e16, Dst dst,
                                                  int c8_0 = 0, int c8_step = 1) {
  for (int c8 = c8_0; c8 < KA / 8; c8 += c8_step) {
    uint32_t w[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint32_t a = operand_value<T>(terms, d, 8 * c8 + 2 * e, x, mu, query, e16);
      const uint32_t b = operand_value<T>(terms, d, 8 * c8 + 2 * e + 1, x, mu, query, e16);
      w[e] = a | (b << 16);
    }
    *dst(c8) = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

// ---- centring ----------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void kb_colsum(BatchDev b, const int32_t* __restrict__ chunk_inst,
                                                     const int64_t* __restrict__ chunk_r0,
                                                     const int64_t* __restrict__ chunk_r1,
                                                     double* __restrict__ part) {
  __shared__ double red[kThreads];
  const int c = blockIdx.x, t = threadIdx.x;
  const int i = chunk_inst[c];
  const BatchInst in = b.inst[i];
  const int d = in.d;
  const int rpp = kThreads / d;
  const int roff = t / d, col = t % d;
  const T* X = static_cast<const T*>(in.X);
  double s = 0.0;
  int bad = 0;
  if (roff < rpp) {
    for (int64_t r = chunk_r0[c] + roff; r < chunk_r1[c]; r += rpp) {
      const double x = (double)X[r * d + col];
      if (!isfinite(x)) bad = 1;
      s += x;
    }
  }
  red[t] = roff < rpp ? s : 0.0;
  __syncthreads();
  if (t < d) {
    double tot = 0.0;
    for (int k = 0; k < rpp; ++k) tot += red[k * d + t];
    part[(int64_t)c * kBatchMaxD + t] = tot;
  }
  if (bad) atomicOr(&b.dyn[i].bad, 1);
}

__global__ __launch_bounds__(kBatchMaxD) void kb_colsum_final(BatchDev b, const double* __restrict__ part,
                                                             double* __restrict__ mu) {
  const int i = blockIdx.x, t = threadIdx.x;
  const BatchInst in = b.inst[i];
  if (t >= in.d) return;
  double s = 0.0;
  for (int c = 0; c < in.nchunks; ++c) s += part[(int64_t)(in.chunk_base + c) * kBatchMaxD + t];
  mu[in.vec_off + t] = s / (double)in.n;
}

// ---- Gram matrix ---------------------------------------------------------------
constexpr int kGramStage = 4096;  // doubles of centred rows in LDS

// Thread t owns the TS x TS tile of C at rows ta.., columns tb.. (at most
// 256 tiles: TS = 1, 2, 4, 8 for d up to 16, 32, 64, 128), so each pair of
// staged values read from LDS feeds TS^2 / 2 fused multiply-adds.  Entries
// (a, b) and (b, a) see the same products in the same order, so C stays
// exactly symmetric.
template <int TS>
__device__ __forceinline__ void gram_tiles(int d, int rows, const double* __restrict__ stage, double (&acc)[TS][TS]) {
  const int tiles_1d = (d + TS - 1) / TS;
  const int t = threadIdx.x;
  if (t >= tiles_1d * tiles_1d) return;
  const int ta = (t / tiles_1d) * TS, tb = (t % tiles_1d) * TS;
  for (int r = 0; r < rows; ++r) {
    const double* row = stage + r * d;
    double a[TS], b[TS];
#pragma unroll
    for (int k = 0; k < TS; ++k) {
      a[k] = ta + k < d ? row[ta + k] : 0.0;
      b[k] = tb + k < d ? row[tb + k] : 0.0;
    }
#pragma unroll
    for (int x = 0; x < TS; ++x)
#pragma unroll
      for (int y = 0; y < TS; ++y) acc[x][y] = fma(a[x], b[y], acc[x][y]);
  }
}

template <typename T, int TS>
__device__ __forceinline__ void gram_chunk(const T* __restrict__ X, int d, const double* __restrict__ m, int64_t r0,
                                           int64_t r1, double* __restrict__ stage, double* __restrict__ out) {
  double acc[TS][TS];
#pragma unroll
  for (int x = 0; x < TS; ++x)
#pragma unroll
    for (int y = 0; y < TS; ++y) acc[x][y] = 0.0;
  const int rc = kGramStage / d;
  for (int64_t ra = r0; ra < r1; ra += rc) {
    const int rows = (int)min((int64_t)rc, r1 - ra);
    __syncthreads();
    for (int e = threadIdx.x; e < rows * d; e += kThreads) stage[e] = (double)X[ra * d + e] - m[e % d];
    __syncthreads();
    gram_tiles<TS>(d, rows, stage, acc);
  }
  const int tiles_1d = (d + TS - 1) / TS;
  const int t = threadIdx.x;
  if (t >= tiles_1d * tiles_1d) return;
  const int ta = (t / tiles_1d) * TS, tb = (t % tiles_1d) * TS;
#pragma unroll
  for (int x = 0; x < TS; ++x)
#pragma unroll
    for (int y = 0; y < TS; ++y)
      if (ta + x < d && tb + y < d) out[(ta + x) * d + tb + y] = acc[x][y];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void kb_gram(BatchDev b, int ddmax, const int32_t* __restrict__ chunk_inst,
                                                   const int64_t* __restrict__ chunk_r0,
                                                   const int64_t* __restrict__ chunk_r1,
                                                   const double* __restrict__ mu, double* __restrict__ part) {
  __shared__ double stage[kGramStage];
  const int c = blockIdx.x;
  const int i = chunk_inst[c];
  const BatchInst in = b.inst[i];
  const int d = in.d;
  const T* X = static_cast<const T*>(in.X);
  const double* m = mu + in.vec_off;
  double* out = part + (int64_t)c * ddmax;
  if (d <= 16)
    gram_chunk<T, 1>(X, d, m, chunk_r0[c], chunk_r1[c], stage, out);
  else if (d <= 32)
    gram_chunk<T, 2>(X, d, m, chunk_r0[c], chunk_r1[c], stage, out);
  else if (d <= 64)
    gram_chunk<T, 4>(X, d, m, chunk_r0[c], chunk_r1[c], stage, out);
  else
    gram_chunk<T, 8>(X, d, m, chunk_r0[c], chunk_r1[c], stage, out);
}

__global__ __launch_bounds__(kThreads) void kb_gram_final(BatchDev b, int ddmax, const double* __restrict__ part,
                                                         double* __restrict__ C) {
  const int i = blockIdx.x;
  const BatchInst in = b.inst[i];
  const int e = blockIdx.y * kThreads + threadIdx.x;
  if (e >= in.d * in.d) return;
  double s = 0.0;
  for (int c = 0; c < in.nchunks; ++c) s += part[(int64_t)(in.chunk_base + c) * ddmax + e];
  C[in.gram_off + e] = s;
}

// ---- power iteration -------------------------------------------------------------
__device__ __forceinline__ double block_sum256(double x, double* red) {
  x = wave_sum(x);
  __syncthreads();
  if (lane_id() == 0) red[threadIdx.x / kWave] = x;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// One workgroup per instance.  C is staged in LDS when it fits; a row of
// C v is computed by tpr lanes (a power of two) and reduced across them.
// Stops when the Rayleigh quotient changes by at most 1e-10 relative, or
// after max_iter.  Largest-magnitude entry positive; C = 0 gives e_1.
constexpr int kPowerLds = 64 * 64;

__global__ __launch_bounds__(kThreads) void kb_power(BatchDev b, const double* __restrict__ C, int max_iter,
                                                    double* __restrict__ v_out) {
  __shared__ double cs[kPowerLds];
  __shared__ double v[kBatchMaxD], w[kBatchMaxD], red[kThreads / kWave];
  __shared__ int s_stop;
  const int i = blockIdx.x, t = threadIdx.x;
  const BatchInst in = b.inst[i];
  const int d = in.d;
  const double* Cg = C + in.gram_off;
  const bool in_lds = d * d <= kPowerLds;
  for (int e = t; in_lds && e < d * d; e += kThreads) cs[e] = Cg[e];
  const double* Cm = in_lds ? cs : Cg;
  int tpr = 1;
  while (tpr < kWave && tpr * 2 * d <= kThreads) tpr *= 2;
  const int row = t / tpr, sub = t % tpr;
  for (int k = t; k < d; k += kThreads) v[k] = 1.0 + 0.01 * (double)((k * 2654435761u) % 1000u) / 1000.0;
  __syncthreads();
  double nv = sqrt(block_sum256(t < d ? v[t] * v[t] : 0.0, red));
  if (t < d) v[t] /= nv;
  __syncthreads();
  double lambda_prev = -1.0;
  bool zero = false;
  int it = 1;
  for (; it <= max_iter; ++it) {
    double s = 0.0;
    if (row < d)
      for (int j = sub; j < d; j += tpr) s += Cm[row * d + j] * v[j];
    for (int o = tpr / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
    if (row < d && sub == 0) w[row] = s;
    __syncthreads();
    const double lambda = block_sum256(t < d ? w[t] * v[t] : 0.0, red);
    const double nw = sqrt(block_sum256(t < d ? w[t] * w[t] : 0.0, red));
    if (!(nw > 0.0)) {
      zero = true;
      break;
    }
    if (t < d) v[t] = w[t] / nw;
    if (t == 0) s_stop = fabs(lambda - lambda_prev) <= 1e-10 * fabs(lambda) ? 1 : 0;
    __syncthreads();
    if (s_stop) break;
    lambda_prev = lambda;
  }
  __syncthreads();
  if (t == 0) {
    if (zero)
      for (int k = 0; k < d; ++k) v[k] = k == 0 ? 1.0 : 0.0;
    int im = 0;
    double am = -1.0;
    for (int k = 0; k < d; ++k)
      if (fabs(v[k]) > am) {
        am = fabs(v[k]);
        im = k;
      }
    const double sgn = v[im] < 0 ? -1.0 : 1.0;
    double ss = 0.0;
    for (int k = 0; k < d; ++k) ss += v[k] * v[k];
    const double inv = 1.0 / sqrt(ss);
    double vn = 0.0;
    for (int k = 0; k < d; ++k) {
      const double x = sgn * v[k] * inv;
      v_out[in.vec_off + k] = x;
      vn += x * x;
    }
    b.dyn[i].vnorm = sqrt(vn) * (1.0 + 4.0 * (d + 2) * kU64);
    b.dyn[i].iters = it > max_iter ? max_iter : it;
  }
}

// ---- scores --------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void kb_project(BatchDev b, const double* __restrict__ mu,
                                                      const double* __restrict__ v, uint32_t* __restrict__ ukey,
                                                      uint32_t* __restrict__ val) {
  const int lane = lane_id();
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t g0 = (int64_t)blockIdx.x * kThreads + (threadIdx.x / kWave) * kWave; g0 < b.N; g0 += stride) {
    const int64_t g = g0 + lane;
    const bool valid = g < b.N;
    int i = -1;
    double nn = 0.0;
    if (valid) {
      i = find_seg(b.in_off, b.count, g);
      const BatchInst in = b.inst[i];
      const int d = in.d;
      const T* x = static_cast<const T*>(in.X) + (g - in.in_off) * d;
      const double* m = mu + in.vec_off;
      const double* vv = v + in.vec_off;
      double a = 0.0;
      for (int k = 0; k < d; ++k) {
        const double xc = (double)x[k] - m[k];
        a += xc * vv[k];
        const double y = (double)(float)xc;
        nn += y * y;
      }
      ukey[g] = float_to_ordered((float)a);
      val[g] = (uint32_t)g;
    }
    // per-instance maximum: one atomic per wavefront when the wave lies in one instance
    const int i0 = __builtin_amdgcn_readfirstlane(i);
    if (__all(i == i0 || i < 0)) {
      const double mx = wave_max(nn);
      if (lane == 0) atomic_max_nonneg(&b.dyn[i0].maxnorm2, mx);
    } else if (valid) {
      atomic_max_nonneg(&b.dyn[i].maxnorm2, nn);
    }
  }
}

__global__ __launch_bounds__(kThreads) void kb_inst_keys(const int64_t* __restrict__ offsets, int count,
                                                        const uint32_t* __restrict__ vals, int64_t n,
                                                        uint32_t* __restrict__ ikey, uint32_t* __restrict__ idx) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    ikey[t] = (uint32_t)find_seg(offsets, count, (int64_t)vals[t]);
    idx[t] = (uint32_t)t;
  }
}

// Window widths and screen constants of every instance (one thread each):
//   Y       = max ||y|| (1 + 4 (d + 2) u64), y = fl32(p - mu)
//   key_eps = 1.01 (u32 + gamma_{d+2}) (1 + u32) Y ||v||   bounds the key rounding
//   W_q     = R ||v|| (1 + 4 gamma_{d+3}) + key_eps + eps_scale ||y_q||
__global__ void kb_finalize(BatchDev b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= b.count) return;
  const BatchInst in = b.inst[i];
  BatchDyn& dy = b.dyn[i];
  const int d = in.d;
  const double Y = sqrt(dy.maxnorm2) * (1.0 + 4.0 * (d + 2) * kU64);
  dy.Y = Y;
  dy.key_eps = 1.01 * (kU32 + gamma64d(d + 2)) * (1.0 + kU32) * Y * dy.vnorm;
  dy.w_base = in.R * dy.vnorm * (1.0 + 4.0 * gamma64d(d + 3)) + dy.key_eps;
  dy.eps_scale = 1.01 * (kU32 + gamma64d(d + 2)) * (1.0 + kU32) * dy.vnorm;
  // terms 0: the fp32 screen (kOpF32) over D32 coordinates
  dy.mb = mixed_bound(in.terms, in.terms == 0 ? b.D32 : b.KA, d, in.R2, Y);
  dy.e16 = in.terms == kOpF16 ? f16_scale_exp(Y) : 0;
}

// ---- rows into score order ---------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void kb_gather(BatchDev b, const double* __restrict__ mu,
                                                     const uint32_t* __restrict__ ukey,
                                                     const uint32_t* __restrict__ val,
                                                     const uint32_t* __restrict__ ikey,
                                                     const uint32_t* __restrict__ idx, double* __restrict__ key,
                                                     int32_t* __restrict__ perm, double* __restrict__ p64,
                                                     float* __restrict__ h, uint16_t* __restrict__ cop) {
  // kQG lanes per row: the float64 copy and the squared norm G elements at
  // a time (partial sums meet by shuffles in a fixed order; any order stays
  // within the bound the screen allows for), the operand groups shared out
  const int KA = b.KA, sub = threadIdx.x % kQG;
  for (int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kQG; t < b.N;
       t += ((int64_t)gridDim.x * blockDim.x) / kQG) {
    const uint32_t p = idx[t];
    const int i = (int)ikey[t];
    const BatchInst in = b.inst[i];
    const int d = in.d;
    const int64_t r = t - in.in_off;
    const int64_t R = in.row_base + r;
    const int64_t local = (int64_t)val[p] - in.in_off;
    const T* x = static_cast<const T*>(in.X) + local * d;
    const double* m = mu + in.vec_off;
    double nn = 0.0;
    for (int k = sub; k < in.dp; k += kQG) {
      const double xv = k < d ? (double)x[k] : 0.0;
      if (p64) p64[in.p64_off + r * in.dp + k] = xv;
      if (k < d) {
        const float y = (float)(xv - m[k]);
        nn += (double)y * (double)y;
      }
    }
#pragma unroll
    for (int off = kQG / 2; off > 0; off >>= 1) nn += __shfl_xor(nn, off, kQG);
    if (sub == 0) {
      key[R] = (double)ordered_to_float(ukey[p]);
      perm[R] = (int32_t)local;
      float hv = (float)(0.5 * nn);
      if (in.terms == kOpF16) {
        // h in the accumulator's units 2^(2 e16): exact unless it lands below
        // fp32's normal range, then rounded down (the screen passes more)
        const double x2 = ldexp((double)hv, 2 * b.dyn[i].e16);
        hv = (float)x2;
        if ((double)hv > x2) hv = nextafterf(hv, -INFINITY);
      }
      h[R] = hv;
    }
    if (in.terms == 0) {
      // fp32 screen: coordinate k of row R at slice k / 2, lane R % 32 + 32 (k % 2)
      float* blk32 = b.cop32 + (R / 32) * (int64_t)b.NK32 * 64 + (R % 32);
      for (int k = sub; k < b.D32; k += kQG)
        blk32[(k / 2) * 64 + 32 * (k % 2)] = k < d ? (float)((double)x[k] - m[k]) : 0.f;
      continue;
    }
    // candidate operands in the 32-row block layout of the matrix-core screen
    uint16_t* blk = cop + (R / 32) * (int64_t)KA * 32 + (R % 32) * 8;
    write_operand_row<T>(
        in.terms, d, KA, x, m, false, b.dyn[i].e16,
        [&](int c8) { return reinterpret_cast<uint4*>(blk + (int64_t)c8 * 256); }, sub, kQG);
  }
}

__global__ void kb_pad_rows(BatchDev b, float* __restrict__ h, int32_t* __restrict__ perm,
                            uint16_t* __restrict__ cop) {
  const int i = blockIdx.x;
  const BatchInst in = b.inst[i];
  const int64_t rows = (in.n + 31) / 32 * 32;
  const int KA = b.KA;
  for (int64_t r = in.n + threadIdx.x; r < rows; r += blockDim.x) {
    const int64_t R = in.row_base + r;
    h[R] = INFINITY;
    perm[R] = -1;
    if (in.terms == 0) {
      float* blk32 = b.cop32 + (R / 32) * (int64_t)b.NK32 * 64 + (R % 32);
      for (int k = 0; k < b.D32; ++k) blk32[(k / 2) * 64 + 32 * (k % 2)] = 0.f;
      continue;
    }
    uint16_t* blk = cop + (R / 32) * (int64_t)KA * 32 + (R % 32) * 8;
    for (int c8 = 0; c8 < KA / 8; ++c8) *reinterpret_cast<uint4*>(blk + (int64_t)c8 * 256) = make_uint4(0, 0, 0, 0);
  }
}

// ---- queries -----------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void kb_query_keys(BatchDev b, const double* __restrict__ mu,
                                                         const double* __restrict__ v, uint32_t* __restrict__ qkey,
                                                         uint32_t* __restrict__ qval, double* __restrict__ qa_in,
                                                         double* __restrict__ qn_in,
                                                         unsigned long long* __restrict__ qbad) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < b.M; g += (int64_t)gridDim.x * blockDim.x) {
    const int i = find_seg(b.qin_off, b.count, g);
    const BatchInst in = b.inst[i];
    const int d = in.d;
    const T* q = static_cast<const T*>(in.Q) + (g - in.qin_off) * d;
    const double* m = mu + in.vec_off;
    const double* vv = v + in.vec_off;
    double a = 0.0, nn = 0.0;
    int bad = 0;
    for (int k = 0; k < d; ++k) {
      const double qk = (double)q[k];
      if (!isfinite(qk)) bad = 1;
      const double x = qk - m[k];
      a += x * vv[k];
      const double y = (double)(float)x;
      nn += y * y;
    }
    if (bad) atomicOr(qbad, 1ull);
    qkey[g] = float_to_ordered((float)a);
    qval[g] = (uint32_t)g;
    qa_in[g] = a;
    qn_in[g] = sqrt(nn);
  }
}

// Padding slots of every instance: never a window, start value -inf, zero operands.
__global__ __launch_bounds__(kThreads) void kb_query_pad(BatchDev b, int32_t* __restrict__ qorig,
                                                        double* __restrict__ qa, double* __restrict__ qn,
                                                        uint16_t* __restrict__ qop, float* __restrict__ cthr) {
  const int i = blockIdx.x;
  const BatchInst in = b.inst[i];
  const int64_t slots = (int64_t)in.ntiles * b.T;
  const int KA = b.KA;
  for (int64_t r = in.m + threadIdx.x; r < slots; r += blockDim.x) {
    const int64_t s = in.slot_base + r;
    qorig[s] = -1;
    qa[s] = 0.0;
    qn[s] = 0.0;
    cthr[s] = -INFINITY;
    if (in.terms == 0) {  // fp32 query row: zeros, start value -inf
      float* row32 = b.vq32 + s * b.DV32;
      for (int k = 0; k < b.DV32; ++k) row32[k] = k == b.D32 ? -INFINITY : 0.f;
      continue;
    }
    uint4* row = reinterpret_cast<uint4*>(qop + s * KA);
    for (int c8 = 0; c8 < KA / 8; ++c8) row[c8] = make_uint4(0, 0, 0, 0);
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void kb_query_gather(
    BatchDev b, const double* __restrict__ mu, const uint32_t* __restrict__ qval, const uint32_t* __restrict__ qikey,
    const uint32_t* __restrict__ qidx, const double* __restrict__ qa_in, const double* __restrict__ qn_in,
    double* __restrict__ q64, int32_t* __restrict__ qorig, double* __restrict__ qa, double* __restrict__ qn,
    uint16_t* __restrict__ qop, float* __restrict__ cthr) {
  // kQG lanes per query (four queries per wavefront): lanes cover the
  // coordinates and the operand row
  const int KA = b.KA, lane = threadIdx.x % kQG;
  for (int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kQG; t < b.M;
       t += ((int64_t)gridDim.x * blockDim.x) / kQG) {
    const uint32_t p = qidx[t];
    const int i = (int)qikey[t];
    const BatchInst& in = b.inst[i];
    const int d = in.d;
    const int64_t g = (int64_t)qval[p];
    const int64_t r = t - in.qin_off;
    const int64_t s = in.slot_base + r;
    const T* q = static_cast<const T*>(in.Q) + (g - in.qin_off) * d;
    const double* m = mu + in.vec_off;
    double nn = 0.0;
    for (int k = lane; k < in.dp; k += kQG) {
      const double qv = k < d ? (double)q[k] : 0.0;
      if (q64) q64[in.q64_off + r * in.dp + k] = qv;
      if (k < d) {
        const float y = (float)(qv - m[k]);
        nn += (double)y * (double)y;
      }
    }
    // any summation order of the squares stays within the gamma_{d+1} bound
    // the start value allows for
#pragma unroll
    for (int off = kQG / 2; off > 0; off >>= 1) nn += __shfl_xor(nn, off, kQG);
    const float c = screen_threshold(b.dyn[i].mb, 0.5 * nn, sqrt(nn) * (1.0 + 1e-15));
    if (in.terms == 0) {  // fp32 query row [y, 0 .., C_q at D32, 0 ..]
      float* row32 = b.vq32 + s * b.DV32;
      for (int k = lane; k < b.DV32; k += kQG)
        row32[k] = k < d ? (float)((double)q[k] - m[k]) : (k == b.D32 ? c : 0.f);
    } else {
      uint16_t* row = qop + s * KA;
      const int e16 = b.dyn[i].e16;
      for (int k = lane; k < KA; k += kQG) row[k] = operand_value<T>(in.terms, d, k, q, m, true, e16);
    }
    if (lane == 0) {
      qorig[s] = (int32_t)g;
      qa[s] = qa_in[g];
      qn[s] = qn_in[g];
      cthr[s] = c;
    }
  }
}

// lo: first index with key >= lv, hi: first index with key > hv, over the n
// sorted keys (the two binary searches interleaved: independent loads).
__device__ __forceinline__ void window_bounds(const double* __restrict__ key, int n, double lv, double hv, int& lo,
                                              int& hi) {
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
}

// Windows J_q of every query slot by binary search inside its instance's
// rows (half-width widened outward exactly as for one instance), and the
// union window of each tile.  T is a multiple of 64, so a wavefront lies in
// one tile.
__global__ __launch_bounds__(kThreads) void kb_window(BatchDev b, const double* __restrict__ key,
                                                     const double* __restrict__ qa, const double* __restrict__ qn,
                                                     const int32_t* __restrict__ qorig, int32_t* __restrict__ tlo,
                                                     int32_t* __restrict__ thi, BatchCtl* __restrict__ ctl) {
  __shared__ unsigned long long red[2][kThreads / kWave];
  unsigned long long acc_cnt = 0, acc_fl = 0;  // this lane's totals over the grid-stride loop
  for (int64_t s0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x / kWave) * kWave; s0 < b.MS;
       s0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = s0 + lane_id();
    int lo = INT_MAX, hi = INT_MIN;
    // the wavefront's slots share one tile, hence one instance
    const int i = __builtin_amdgcn_readfirstlane(b.tile_inst[s0 / b.T]);
    if (s < b.MS && qorig[s] >= 0) {
      const BatchInst& in = b.inst[i];
      const BatchDyn& dy = b.dyn[i];
      const double W = (dy.w_base + dy.eps_scale * qn[s]) * (1.0 + 8.0 * kU64);
      const double a = qa[s];
      const int base = (int)in.row_base, n = (int)in.n;
      int l0, h0;
      window_bounds(key + base, n, nextafter(a - W, -INFINITY), nextafter(a + W, INFINITY), l0, h0);
      if (h0 > l0) {
        lo = base + l0;
        hi = base + h0;
        acc_cnt += (unsigned long long)(h0 - l0);
        acc_fl += (unsigned long long)(h0 - l0) * 2ull * (unsigned long long)in.d;
      }
    }
    const int wlo = wave_min(lo), whi = wave_max(hi);
    if (lane_id() == 0 && wlo != INT_MAX) {
      const int tile = (int)(s0 / b.T);
      atomicMin(&tlo[tile], wlo);
      atomicMax(&thi[tile], whi);
    }
  }
  // one pair of counter atomics per block (same-address atomics serialise)
  const unsigned long long wc = wave_sum(acc_cnt), wf = wave_sum(acc_fl);
  if (lane_id() == 0) {
    red[0][threadIdx.x / kWave] = wc;
    red[1][threadIdx.x / kWave] = wf;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long c = 0, f = 0;
    for (int w = 0; w < kThreads / kWave; ++w) {
      c += red[0][w];
      f += red[1][w];
    }
    if (c) {
      atomicAdd(&ctl->pairs_window, c);
      atomicAdd(&ctl->flops, f);
    }
  }
}

__global__ __launch_bounds__(kThreads) void kb_split_tiles(BatchDev b, int32_t* __restrict__ tlo,
                                                          int32_t* __restrict__ thi, int32_t* __restrict__ tlo32,
                                                          int32_t* __restrict__ thi32) {
  const int tile = blockIdx.x * blockDim.x + threadIdx.x;
  if (tile >= b.ntiles) return;
  if (b.inst[b.tile_inst[tile]].terms == 0) {
    tlo32[tile] = tlo[tile];
    thi32[tile] = thi[tile];
    tlo[tile] = INT_MAX;
    thi[tile] = INT_MIN;
  } else {
    tlo32[tile] = INT_MAX;
    thi32[tile] = INT_MIN;
  }
}

// Pairs the screen evaluates: wavefronts with at least one real query, times
// their queries, times the tile's (aligned) window.
__global__ __launch_bounds__(kThreads) void kb_executed(BatchDev b, const int32_t* __restrict__ tlo,
                                                       const int32_t* __restrict__ thi, int qpw,
                                                       BatchCtl* __restrict__ ctl) {
  unsigned long long e = 0;
  const int tile = blockIdx.x * blockDim.x + threadIdx.x;
  if (tile < b.ntiles) {
    const BatchInst in = b.inst[b.tile_inst[tile]];
    const int64_t valid = min((int64_t)b.T, max((int64_t)0, in.m - (tile - in.tile_base) * (int64_t)b.T));
    const int64_t waves = (valid + qpw - 1) / qpw;
    e = (unsigned long long)(waves * qpw) * (unsigned long long)max(0, thi[tile] - tlo[tile]);
  }
  e = wave_sum(e);
  if (lane_id() == 0 && e) atomicAdd(&ctl->executed, e);
}

// ---- survivors -> CSR ------------------------------------------------------------------------
// The caller's rows in their dtype (promotion to float64 is exact): the
// data row through perm, the query row through qorig.
template <typename T>
__global__ __launch_bounds__(kThreads) void kb_recheck(BatchDev b, Survivors sv, const int32_t* __restrict__ qorig,
                                                      const int32_t* __restrict__ perm,
                                                      int32_t* __restrict__ row_cnt) {
  const long long cnt = (long long)min((unsigned long long)sv.cap, *sv.count);
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < cnt;
       k += (long long)gridDim.x * blockDim.x) {
    const int2 pr = sv.pairs[k];
    const int i = b.tile_inst[pr.x / b.T];
    const BatchInst& in = b.inst[i];
    const int d = in.d;
    const int pj = perm[pr.y];
    const T* pp = static_cast<const T*>(in.X) + (int64_t)pj * d;
    const T* qp = static_cast<const T*>(in.Q) + ((int64_t)qorig[pr.x] - in.qin_off) * d;
    double s = 0.0;
    for (int c = 0; c < d; ++c) {
      const double t = (double)pp[c] - (double)qp[c];
      s = s + t * t;
    }
    if (s <= in.R2) {
      // rows are query slots: a tile's rows are neighbours in memory
      sv.res_q[k] = pr.x;
      sv.res_key[k] = neighbour_key(pj, (float)sqrt(s));
      sv.res_slot[k] = atomicAdd(&row_cnt[pr.x], 1);
    } else {
      sv.res_q[k] = -1;
    }
  }
}

__global__ __launch_bounds__(kThreads) void kb_scatter(Survivors sv, const int64_t* __restrict__ row_ptr, int64_t M,
                                                      uint64_t* __restrict__ keys, int64_t cap) {
  if (row_ptr[M] > cap) return;  // staging too small: the host grows it and runs again
  const long long cnt = (long long)min((unsigned long long)sv.cap, *sv.count);
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < cnt;
       k += (long long)gridDim.x * blockDim.x) {
    const int o = sv.res_q[k];
    if (o < 0) continue;
    keys[row_ptr[o] + sv.res_slot[k]] = sv.res_key[k];
  }
}

__global__ __launch_bounds__(kThreads) void kb_rowptr_guard(const int64_t* __restrict__ row_ptr, int64_t M,
                                                           int64_t cap, int64_t* __restrict__ out) {
  const bool ok = row_ptr[M] <= cap;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= M; r += (int64_t)gridDim.x * blockDim.x)
    out[r] = ok ? row_ptr[r] : 0;
}

__global__ void kb_inst_nnz(BatchDev b, const int64_t* __restrict__ row_ptr, int64_t* __restrict__ nnz_base,
                            int64_t* __restrict__ nnz) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < b.count) {
    const BatchInst in = b.inst[i];
    const int64_t base = row_ptr[in.qin_off];
    nnz_base[i] = base;
    nnz[i] = row_ptr[in.qin_off + in.m] - base;
  }
  if (i == 0) nnz_base[b.count] = row_ptr[b.M];
}

// row_ptr of every instance (m_i + 1 entries each): entry e of the
// concatenation belongs to the instance with qin_off_i + i <= e.
__global__ __launch_bounds__(kThreads) void kb_out_rowptr(BatchDev b, const BatchOut* __restrict__ outs,
                                                         const int64_t* __restrict__ row_ptr,
                                                         const int64_t* __restrict__ nnz_base) {
  const int64_t total = b.M + b.count;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = b.count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (b.qin_off[mid] + mid <= e)
        lo = mid;
      else
        hi = mid - 1;
    }
    const int64_t r = e - b.qin_off[lo] - lo;
    outs[lo].row_ptr[r] = row_ptr[b.qin_off[lo] + r] - nnz_base[lo];
  }
}

__global__ __launch_bounds__(kThreads) void kb_out_cols(BatchDev b, const BatchOut* __restrict__ outs,
                                                       const int32_t* __restrict__ col, const float* __restrict__ dist,
                                                       int64_t cap, const int64_t* __restrict__ nnz_base,
                                                       const int64_t* __restrict__ nnz) {
  const int64_t total = nnz_base[b.count];
  if (total > cap) return;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < total; p += (int64_t)gridDim.x * blockDim.x) {
    const int i = find_seg(nnz_base, b.count, p);
    if (nnz[i] > outs[i].cap) continue;
    const int64_t o = p - nnz_base[i];
    outs[i].col[o] = col[p];
    outs[i].dist[o] = dist[p];
  }
}

__global__ void kb_fill_f32(float* p, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void kb_stamp(unsigned long long* out) {
  if (threadIdx.x == 0) *out = (unsigned long long)wall_clock64();
}

__global__ void kb_zero_i64(int64_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

unsigned grid_for(int64_t work, int cap) {
  int64_t g = (work + kThreads - 1) / kThreads;
  return (unsigned)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

// ---------------------------------------------------------------- launchers
#define SNN_DT_LAUNCH(K, grid, block, ...)                                                           \
  do {                                                                                               \
    if (dt == SNN_F32)                                                                               \
      K<float><<<(grid), (block), 0, s>>>(__VA_ARGS__);                                              \
    else                                                                                             \
      K<double><<<(grid), (block), 0, s>>>(__VA_ARGS__);                                             \
    SNN_LAUNCH_CHECK();                                                                              \
  } while (0)

void batch_colsum(snn_dtype dt, const BatchDev& b, int nchunks, const int32_t* chunk_inst, const int64_t* chunk_r0,
                  const int64_t* chunk_r1, double* part, double* mu, hipStream_t s) {
  SNN_DT_LAUNCH(kb_colsum, nchunks, kThreads, b, chunk_inst, chunk_r0, chunk_r1, part);
  kb_colsum_final<<<b.count, kBatchMaxD, 0, s>>>(b, part, mu);
  SNN_LAUNCH_CHECK();
}

void batch_gram(snn_dtype dt, const BatchDev& b, int nchunks, int dmax, const int32_t* chunk_inst,
                const int64_t* chunk_r0, const int64_t* chunk_r1, const double* mu, double* part, double* C,
                hipStream_t s) {
  const int ddmax = dmax * dmax;
  SNN_DT_LAUNCH(kb_gram, nchunks, kThreads, b, ddmax, chunk_inst, chunk_r0, chunk_r1, mu, part);
  dim3 g(b.count, (ddmax + kThreads - 1) / kThreads);
  kb_gram_final<<<g, kThreads, 0, s>>>(b, ddmax, part, C);
  SNN_LAUNCH_CHECK();
}

void batch_power(const BatchDev& b, const double* C, int max_iter, double* v, hipStream_t s) {
  kb_power<<<b.count, kThreads, 0, s>>>(b, C, max_iter, v);
  SNN_LAUNCH_CHECK();
}

void batch_project(snn_dtype dt, const BatchDev& b, const double* mu, const double* v, uint32_t* ukey,
                   uint32_t* val, hipStream_t s) {
  SNN_DT_LAUNCH(kb_project, grid_for(b.N, 8192), kThreads, b, mu, v, ukey, val);
}

void batch_inst_keys(const int64_t* offsets, int count, const uint32_t* vals, int64_t n, uint32_t* ikey,
                     uint32_t* idx, hipStream_t s) {
  kb_inst_keys<<<grid_for(n, 8192), kThreads, 0, s>>>(offsets, count, vals, n, ikey, idx);
  SNN_LAUNCH_CHECK();
}

void batch_finalize(const BatchDev& b, hipStream_t s) {
  kb_finalize<<<(b.count + 63) / 64, 64, 0, s>>>(b);
  SNN_LAUNCH_CHECK();
}

void batch_gather(snn_dtype dt, const BatchDev& b, const double* mu, const uint32_t* ukey, const uint32_t* val,
                  const uint32_t* ikey, const uint32_t* idx, double* key, int32_t* perm, double* p64, float* h,
                  uint16_t* cop, hipStream_t s) {
  SNN_DT_LAUNCH(kb_gather, grid_for(b.N * (int64_t)kQG, 65536), kThreads, b, mu, ukey, val, ikey, idx, key, perm, p64,
                h, cop);
}

void batch_pad_rows(const BatchDev& b, float* h, int32_t* perm, uint16_t* cop, hipStream_t s) {
  kb_pad_rows<<<b.count, 32, 0, s>>>(b, h, perm, cop);
  SNN_LAUNCH_CHECK();
}

void batch_query_keys(snn_dtype dt, const BatchDev& b, const double* mu, const double* v, uint32_t* qkey,
                      uint32_t* qval, double* qa_in, double* qn_in, BatchCtl* ctl, hipStream_t s) {
  SNN_DT_LAUNCH(kb_query_keys, grid_for(b.M, 8192), kThreads, b, mu, v, qkey, qval, qa_in, qn_in, &ctl->qbad);
}

void batch_query_pad(const BatchDev& b, int32_t* qorig, double* qa, double* qn, uint16_t* qop, float* cthr,
                     hipStream_t s) {
  kb_query_pad<<<b.count, kThreads, 0, s>>>(b, qorig, qa, qn, qop, cthr);
  SNN_LAUNCH_CHECK();
}

void batch_query_gather(snn_dtype dt, const BatchDev& b, const double* mu, const uint32_t* qval,
                        const uint32_t* qikey, const uint32_t* qidx, const double* qa_in, const double* qn_in,
                        double* q64, int32_t* qorig, double* qa, double* qn, uint16_t* qop, float* cthr,
                        hipStream_t s) {
  SNN_DT_LAUNCH(kb_query_gather, grid_for(b.M * (int64_t)kQG, 16384), kThreads, b, mu, qval, qikey, qidx, qa_in,
                qn_in, q64, qorig, qa, qn, qop, cthr);
}

void batch_windows(const BatchDev& b, const double* key, const double* qa, const double* qn, const int32_t* qorig,
                   int32_t* tlo, int32_t* thi, BatchCtl* ctl, hipStream_t s) {
  kb_window<<<grid_for(b.MS, 1024), kThreads, 0, s>>>(b, key, qa, qn, qorig, tlo, thi, ctl);
  SNN_LAUNCH_CHECK();
}

void batch_split_tiles(const BatchDev& b, int32_t* tlo, int32_t* thi, int32_t* tlo32, int32_t* thi32, hipStream_t s) {
  if (b.ntiles <= 0) return;
  kb_split_tiles<<<(b.ntiles + kThreads - 1) / kThreads, kThreads, 0, s>>>(b, tlo, thi, tlo32, thi32);
  SNN_LAUNCH_CHECK();
}

void batch_executed(const BatchDev& b, const int32_t* tlo, const int32_t* thi, int queries_per_wave, BatchCtl* ctl,
                    hipStream_t s) {
  kb_executed<<<(unsigned)((b.ntiles + kThreads - 1) / kThreads), kThreads, 0, s>>>(b, tlo, thi, queries_per_wave,
                                                                                     ctl);
  SNN_LAUNCH_CHECK();
}

void batch_recheck(snn_dtype dt, const BatchDev& b, const Survivors& sv, const int32_t* qorig,
                   const int32_t* perm, int32_t* row_cnt, int grid, hipStream_t s) {
  SNN_DT_LAUNCH(kb_recheck, grid, kThreads, b, sv, qorig, perm, row_cnt);
  SNN_LAUNCH_CHECK();
}

void batch_scatter(const Survivors& sv, const int64_t* row_ptr, int64_t M, uint64_t* keys, int64_t cap, int grid,
                   hipStream_t s) {
  kb_scatter<<<grid, kThreads, 0, s>>>(sv, row_ptr, M, keys, cap);
  SNN_LAUNCH_CHECK();
}

void batch_rowptr_guard(const int64_t* row_ptr, int64_t M, int64_t cap, int64_t* row_ptr_s, hipStream_t s) {
  kb_rowptr_guard<<<grid_for(M + 1, 4096), kThreads, 0, s>>>(row_ptr, M, cap, row_ptr_s);
  SNN_LAUNCH_CHECK();
}

void batch_outputs(const BatchDev& b, const BatchOut* outs, const int64_t* row_ptr, const int32_t* col,
                   const float* dist, int64_t cap, int64_t* nnz_base, int64_t* nnz, hipStream_t s) {
  kb_inst_nnz<<<(b.count + 63) / 64, 64, 0, s>>>(b, row_ptr, nnz_base, nnz);
  SNN_LAUNCH_CHECK();
  kb_out_rowptr<<<grid_for(b.M + b.count, 4096), kThreads, 0, s>>>(b, outs, row_ptr, nnz_base);
  SNN_LAUNCH_CHECK();
  kb_out_cols<<<2048, kThreads, 0, s>>>(b, outs, col, dist, cap, nnz_base, nnz);
  SNN_LAUNCH_CHECK();
}

void batch_fill_f32(float* p, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return;
  kb_fill_f32<<<grid_for(n, 4096), kThreads, 0, s>>>(p, n, v);
  SNN_LAUNCH_CHECK();
}

void batch_stamp(unsigned long long* out, hipStream_t s) {
  kb_stamp<<<1, 64, 0, s>>>(out);
  SNN_LAUNCH_CHECK();
}

void batch_zero_i64(int64_t* p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  kb_zero_i64<<<grid_for(n, 4096), kThreads, 0, s>>>(p, n);
  SNN_LAUNCH_CHECK();
}

}  // namespace snn
