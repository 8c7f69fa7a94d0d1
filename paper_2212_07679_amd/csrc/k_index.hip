// Index construction (Algorithm 1, Section 3.1) on gfx950.
//
//  step 2  column means          k_colsum_partial + k_colsum_final (float64,
//                                fixed-order reductions: deterministic)
//  step 4  first principal dir.  centred Gram matrix C = X^T X in float64
//                                (register-tiled, LDS-staged rows) and a
//                                power iteration in one workgroup.  The SVD of
//                                eq. (svd) is replaced: any unit direction
//                                keeps the query exact (eq. (lower)); only
//                                the window sizes depend on it.
//  step 5  scores                key_i = fl32(x_i . v), x_i = p_i - mu in float64
//  step 6  sort                  LSD radix sort of order-preserving keys
//  step 7  norms                 h_i = ||y_i||^2 / 2 with y_i = fl32(p_i - mu),
//                                gathered with the rows into score order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <cmath>
#include <cstring>
#include <vector>

#include "device_common.h"
#include "query_plan.h"
#include "snn_internal.h"

namespace snn {

namespace {

constexpr int kThreads = 256;

template <typename T>
__device__ __forceinline__ double ld(const T* p, int64_t i) {
  return (double)p[i];
}

// ---- step 2: column sums ---------------------------------------------------
// Thread layout: cols_per_pass = min(d, 256) consecutive columns, rows_per_pass
// rows at once; each thread owns one column of a fixed row subset.  Partials
// are stored column-major (part[c * nblocks + b]) so that the final pass
// reads each column's partials contiguously.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_colsum_partial(const T* __restrict__ X, int64_t n, int d,
                                                            int64_t rows_per_block, double* __restrict__ part,
                                                            int* __restrict__ bad) {
  __shared__ double red[kThreads];
  const int t = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = min(n, r0 + rows_per_block);
  int badloc = 0;
  for (int c0 = 0; c0 < d; c0 += kThreads) {
    const int cpp = min(d - c0, kThreads);
    const int rpp = kThreads / cpp;
    const int roff = t / cpp, c = c0 + t % cpp;
    double s = 0.0;
    if (roff < rpp) {
      // eight independent loads in flight, added in row order
      int64_t r = r0 + roff;
      for (; r + 7 * rpp < r1; r += 8 * rpp) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = ld(X, (r + u * rpp) * d + c);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (!isfinite(x[u])) badloc = 1;
          s += x[u];
        }
      }
      for (; r < r1; r += rpp) {
        const double x = ld(X, r * d + c);
        if (!isfinite(x)) badloc = 1;
        s += x;
      }
    }
    red[t] = (roff < rpp) ? s : 0.0;
    __syncthreads();
    if (t < cpp) {
      double tot = 0.0;
      for (int k = 0; k < rpp; ++k) tot += red[k * cpp + t];
      part[(int64_t)(c0 + t) * gridDim.x + blockIdx.x] = tot;
    }
    __syncthreads();
  }
  if (badloc) atomicOr(bad, 1);
}

// One wavefront per column: the lanes take the block partials in a fixed
// interleaved order and meet by shuffles (deterministic).
__global__ __launch_bounds__(kWave) void k_colsum_final(const double* __restrict__ part, int nblocks, int d,
                                                       int64_t n, double* __restrict__ mu) {
  const int c = blockIdx.x;
  const double* pc = part + (int64_t)c * nblocks;
  double s = 0.0;
  int b = threadIdx.x;
  for (; b + 7 * kWave < nblocks; b += 8 * kWave) {  // eight loads in flight, added in order
    double x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = pc[b + u * kWave];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += x[u];
  }
  for (; b < nblocks; b += kWave) s += pc[b];
  s = wave_sum(s);
  if (threadIdx.x == 0) mu[c] = s / (double)n;
}

// ---- step 4: centred Gram matrix --------------------------------------------
// Narrow data (d < kGramMfmaMinD, so d * d < 64): thread t owns entry
// (t / d, t % d) of one partial C; rows are staged in LDS, centred in float64.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gram_partial(const T* __restrict__ X, int64_t n, int d,
                                                          const double* __restrict__ mu, int64_t rows_per_block,
                                                          int rows_chunk, double* __restrict__ part) {
  extern __shared__ double stage[];  // rows_chunk x d
  const int t = threadIdx.x;
  const bool active = t < d * d;
  const int ea = active ? t / d : 0, eb = active ? t % d : 0;
  double acc = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = min(n, r0 + rows_per_block);
  for (int64_t rc = r0; rc < r1; rc += rows_chunk) {
    const int rows = (int)min((int64_t)rows_chunk, r1 - rc);
    __syncthreads();
    for (int e = t; e < rows * d; e += kThreads) stage[e] = ld(X, rc * d + e) - mu[e % d];
    __syncthreads();
    if (active)
      for (int r = 0; r < rows; ++r) acc = fma(stage[r * d + ea], stage[r * d + eb], acc);
  }
  if (active) part[(int64_t)blockIdx.x * d * d + t] = acc;
}

// The same partial Gram matrices on the float64 matrix cores
// (v_mfma_f64_16x16x4f64): C is cut into column blocks of BW = 16 TB and
// each wavefront owns one pair of blocks (a, b), a <= b, accumulating
// Y[:, a]^T Y[:, b] over 4 rows per instruction, Y = X - mu in float64.
// Operands go from memory straight into registers (no LDS): lane l loads
// column 16 t + l % 16 of row l / 16 of each 4-row step.  Only entries on or
// above the diagonal are kept and each is written to both halves, so every
// partial (and C) is exactly symmetric.
constexpr int kGramWaves = 4;
// below 8 columns the 16-wide tiles are mostly padding (at d = 3 the
// one-entry-per-thread form above is measured faster)
constexpr int kGramMfmaMinD = 8;
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T, int TB>
__global__ __launch_bounds__(kGramWaves * kWave) void k_gram_mfma(const T* __restrict__ X, int64_t n, int d,
                                                                const double* __restrict__ mu,
                                                                int64_t rows_per_block, int npairs,
                                                                double* __restrict__ part) {
  constexpr int BW = 16 * TB;
  const int wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
  // one pair (d <= 64): every wavefront of the workgroup takes that pair over
  // its own share of the workgroup's rows, and the sums meet in LDS below
  const bool split = npairs == 1;
  const int pair = split ? 0 : blockIdx.y * nw + wv;
  if (pair >= npairs) return;  // never in split mode, the only one with barriers
  const int nbk = (d + BW - 1) / BW;
  int ba = 0, rest = pair;
  while (rest >= nbk - ba) {
    rest -= nbk - ba;
    ++ba;
  }
  const int bb = ba + rest;
  const bool diag = ba == bb;
  const int l = lane_id(), c16 = l % 16, k4 = l / 16;
  int ca[TB], cb[TB];
  double mua[TB], mub[TB];
#pragma unroll
  for (int t = 0; t < TB; ++t) {
    ca[t] = ba * BW + 16 * t + c16;
    cb[t] = bb * BW + 16 * t + c16;
    mua[t] = ca[t] < d ? mu[ca[t]] : 0.0;
    mub[t] = cb[t] < d ? mu[cb[t]] : 0.0;
  }
  f64x4 acc[TB][TB];
#pragma unroll
  for (int i = 0; i < TB; ++i)
#pragma unroll
    for (int j = 0; j < TB; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
  int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  int64_t r1 = min(n, r0 + rows_per_block);
  if (split) {  // contiguous shares of a multiple of 4 rows (the last ones may be empty)
    const int64_t per = ((rows_per_block + nw - 1) / nw + 3) & ~int64_t(3);
    r0 += wv * per;
    r1 = min(r1, r0 + per);
  }
  // raw operands of the next PF steps stay in flight in a register ring
  // (measured: 8 steps for one or two tiles a side, 2 for the 16-tile pairs)
  constexpr int PF = (TB >= 3 ? 2 : 8) / (sizeof(T) == 8 ? 2 : 1);
  T ra[PF][TB], rb[PF][TB];
  auto issue = [&](int64_t step, T* xa, T* xb) {
    const int64_t row = step + k4;
    const bool ok = row < r1;
#pragma unroll
    for (int t = 0; t < TB; ++t) {
      xa[t] = (ok && ca[t] < d) ? X[row * d + ca[t]] : T(0);
      if (!diag) xb[t] = (ok && cb[t] < d) ? X[row * d + cb[t]] : T(0);
    }
  };
#pragma unroll
  for (int q = 0; q < PF; ++q) issue(r0 + 4 * q, ra[q], rb[q]);
  for (int64_t step = r0; step < r1; step += 4 * PF) {
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int64_t row = step + 4 * q + k4;
      double a[TB], b[TB];
#pragma unroll
      for (int t = 0; t < TB; ++t) {  // padding (rows past r1, columns past d) stays exactly zero
        a[t] = (row < r1 && ca[t] < d) ? (double)ra[q][t] - mua[t] : 0.0;
        b[t] = diag ? a[t] : ((row < r1 && cb[t] < d) ? (double)rb[q][t] - mub[t] : 0.0);
      }
      issue(step + 4 * (q + PF), ra[q], rb[q]);
#pragma unroll
      for (int i = 0; i < TB; ++i)
#pragma unroll
        for (int j = 0; j < TB; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
  if (split) {  // wavefronts 1.. add into wavefront 0, one at a time (a fixed order)
    __shared__ f64x4 red[TB * TB][kWave];
    const int l2 = lane_id();
    for (int src = 1; src < nw; ++src) {
      if (wv == src)
#pragma unroll
        for (int i = 0; i < TB; ++i)
#pragma unroll
          for (int j = 0; j < TB; ++j) red[i * TB + j][l2] = acc[i][j];
      __syncthreads();
      if (wv == 0)
#pragma unroll
        for (int i = 0; i < TB; ++i)
#pragma unroll
          for (int j = 0; j < TB; ++j) acc[i][j] += red[i * TB + j][l2];
      __syncthreads();
    }
    if (wv != 0) return;
  }
  // element e of lane l holds D[l / 16 + 4 e][l % 16] of each 16 x 16 tile
  double* out = part + (int64_t)blockIdx.x * d * d;
#pragma unroll
  for (int i = 0; i < TB; ++i)
#pragma unroll
    for (int j = 0; j < TB; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gi = ba * BW + 16 * i + k4 + 4 * e, gj = bb * BW + 16 * j + c16;
        if (gi < d && gj < d && gi <= gj) {
          out[(int64_t)gi * d + gj] = acc[i][j][e];
          out[(int64_t)gj * d + gi] = acc[i][j][e];
        }
      }
}

// Sum of the partial Gram matrices: a workgroup of kGramFinalWaves
// wavefronts takes 64 consecutive entries (one per lane, coalesced); wave w
// adds partials w, w + W, ... in order with eight loads in flight, and the W
// wave sums meet in LDS in wave order.  C[a][b] and C[b][a] have equal
// partials and the same order, so C stays exactly symmetric.
constexpr int kGramFinalWaves = 16;

__global__ __launch_bounds__(kGramFinalWaves * kWave) void k_gram_final(const double* __restrict__ part,
                                                                       int nblocks, int64_t dd,
                                                                       double* __restrict__ C) {
  __shared__ double red[kGramFinalWaves][kWave];
  const int w = threadIdx.x / kWave, l = lane_id();
  const int64_t e = (int64_t)blockIdx.x * kWave + l;
  double s = 0.0;
  if (e < dd) {
    int b = w;
    for (; b + 7 * kGramFinalWaves < nblocks; b += 8 * kGramFinalWaves) {
      double x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = part[(int64_t)(b + u * kGramFinalWaves) * dd + e];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += x[u];
    }
    for (; b < nblocks; b += kGramFinalWaves) s += part[(int64_t)b * dd + e];
  }
  red[w][l] = s;
  __syncthreads();
  if (w == 0 && e < dd) {
    double t = 0.0;
    for (int k = 0; k < kGramFinalWaves; ++k) t += red[k][l];
    C[e] = t;
  }
}

// Power iteration v <- C v / ||C v|| in one workgroup of NT threads (the
// general form, used for d > 128): thread i owns rows i, i + NT, ...; C is
// symmetric, so row i of C v is read down column i (C[j][i], j = 0..d-1),
// one coalesced row of C per j across the threads; v and C v stay in LDS.  Stops when the Rayleigh quotient
// changes by less than 1e-12 relative (it converges at twice the rate of v)
// or after max_iter.  The largest-magnitude entry is made positive; C = 0
// gives e_1.
template <int NT>
__device__ __forceinline__ double group_sum(double x, double* red) {
  x = wave_sum(x);
  if (NT == kWave) return x;
  __syncthreads();
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = x;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < NT / kWave; ++w) s += red[w];
  return s;
}

template <int NT>
__global__ __launch_bounds__(NT) void k_power_iter(const double* __restrict__ C, int d, int max_iter,
                                                  double* __restrict__ v_out, int* __restrict__ iters_out) {
  extern __shared__ double lds[];
  __shared__ double red[NT / kWave];
  const int t = threadIdx.x;
  double* v = lds;      // d
  double* w = lds + d;  // d
  // deterministic start: 1 + small distinct perturbation per coordinate
  double loc = 0.0;
  for (int i = t; i < d; i += NT) {
    const double x = 1.0 + 0.01 * (double)((i * 2654435761u) % 1000u) / 1000.0;
    v[i] = x;
    loc += x * x;
  }
  const double nv = sqrt(group_sum<NT>(loc, red));
  for (int i = t; i < d; i += NT) v[i] /= nv;
  __syncthreads();
  double lambda_prev = -1.0;
  int it = 0;
  bool zero = false;
  for (it = 1; it <= max_iter; ++it) {
    double part = 0.0, nn = 0.0;
    for (int i0 = 0; i0 < d; i0 += NT) {
      const int i = i0 + t;
      double sacc = 0.0;
      if (i < d)
        for (int j = 0; j < d; ++j) sacc += C[(int64_t)j * d + i] * v[j];
      if (i < d) {
        w[i] = sacc;
        part += sacc * v[i];
        nn += sacc * sacc;
      }
    }
    const double lambda = group_sum<NT>(part, red);  // Rayleigh quotient v^T C v
    const double nw = sqrt(group_sum<NT>(nn, red));
    if (!(nw > 0.0)) {
      zero = true;
      break;
    }
    __syncthreads();
    for (int i = t; i < d; i += NT) v[i] = w[i] / nw;
    __syncthreads();
    if (fabs(lambda - lambda_prev) <= 1e-12 * fabs(lambda)) break;
    lambda_prev = lambda;
  }
  __syncthreads();
  if (t == 0) {
    if (zero) {
      for (int i = 0; i < d; ++i) v[i] = (i == 0) ? 1.0 : 0.0;
    }
    int im = 0;
    double am = -1.0;
    for (int i = 0; i < d; ++i)
      if (fabs(v[i]) > am) {
        am = fabs(v[i]);
        im = i;
      }
    double sgn = v[im] < 0 ? -1.0 : 1.0;
    double ss = 0.0;
    for (int i = 0; i < d; ++i) ss += v[i] * v[i];
    double inv = 1.0 / sqrt(ss);
    for (int i = 0; i < d; ++i) v_out[i] = sgn * v[i] * inv;
    *iters_out = it > max_iter ? max_iter : it;
  }
}

// The same iteration for d <= DB <= 64 in one wavefront with no LDS traffic
// or barriers in the loop: lane i holds row i of C (= column i) in registers
// and v_i; v_j reaches every lane by a lane read, and the two sums of a step
// are taken over lane reads in lane order, so every lane holds the same
// value and the stopping test is uniform.
__device__ __forceinline__ double readlane_f64(double x, int lane) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

template <int DB>
__device__ __forceinline__ double lanes_sum(double x) {
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < DB; ++j) s += readlane_f64(x, j);
  return s;
}

constexpr int kPowerSquarings = 10;

template <int DB>
__global__ __launch_bounds__(kWave) void k_power_iter_wave(const double* __restrict__ C, int d, int max_iter,
                                                          double* __restrict__ v_out, int* __restrict__ iters_out) {
  __shared__ double vs[kWave];
  const int i = threadIdx.x;
  double crow[DB];
#pragma unroll
  for (int j = 0; j < DB; ++j) crow[j] = (i < d && j < d) ? C[(int64_t)j * d + i] : 0.0;
  // deterministic start: 1 + small distinct perturbation per coordinate
  double vi = i < d ? 1.0 + 0.01 * (double)((i * 2654435761u) % 1000u) / 1000.0 : 0.0;
  if constexpr (DB <= 16) {
    // d <= 16: the start is first taken through C^(2^kPowerSquarings), built
    // by repeated squaring on the matrix cores (four 16x16x4 fp64 products per
    // square, each square scaled to unit Frobenius norm), so a slow ratio of
    // the two largest eigenvalues costs a few squarings instead of hundreds
    // of iterations; the iteration below still decides convergence on C.
    // Lane l holds M[l % 16][4 kb + l / 16] for kb = 0..3, every entry once,
    // which is both operands of M M since M is symmetric.
    __shared__ double ms[16][17];
    const int c16 = i % 16, k4 = i / 16;
    double op[4];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      const int col = 4 * kb + k4;
      op[kb] = (c16 < d && col < d) ? C[(int64_t)c16 * d + col] : 0.0;
    }
    int done = 0;  // squares written to ms (uniform across lanes)
    // sums of squares by butterfly, lane 0's value taken by all (uniform)
    auto frob2 = [](double x) { return readlane_f64(wave_sum(x), 0); };
    double ss = frob2(op[0] * op[0] + op[1] * op[1] + op[2] * op[2] + op[3] * op[3]);
    if (ss > 0.0 && ss < INFINITY) {
      const double inv0 = 1.0 / sqrt(ss);
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) op[kb] *= inv0;
      for (; done < kPowerSquarings; ++done) {
        f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(op[kb], op[kb], acc, 0, 0, 0);
        ss = frob2(acc[0] * acc[0] + acc[1] * acc[1] + acc[2] * acc[2] + acc[3] * acc[3]);
        if (!(ss > 0.0 && ss < INFINITY)) break;
        const double inv = 1.0 / sqrt(ss);
        __syncthreads();  // the previous square has been read
        // element e of lane l holds the square's entry [l / 16 + 4 e][l % 16]
#pragma unroll
        for (int e = 0; e < 4; ++e) ms[k4 + 4 * e][c16] = acc[e] * inv;
        __syncthreads();
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) op[kb] = ms[c16][4 * kb + k4];
      }
    }
    if (done > 0) {  // start from M x0
      double w = 0.0;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const double xj = readlane_f64(vi, j);
        if (i < d) w += ms[i][j] * xj;
      }
      const double nw = lanes_sum<DB>(w * w);
      if (nw > 0.0 && nw < INFINITY) vi = w;
    }
  }
  vi /= sqrt(lanes_sum<DB>(vi * vi));
  double lambda_prev = -1.0;
  int it = 0;
  bool zero = false;
  for (it = 1; it <= max_iter; ++it) {
    double w = 0.0;
#pragma unroll
    for (int j = 0; j < DB; ++j) w += crow[j] * readlane_f64(vi, j);
    const double lambda = lanes_sum<DB>(w * vi);  // Rayleigh quotient v^T C v
    const double nw = sqrt(lanes_sum<DB>(w * w));
    if (!(nw > 0.0)) {
      zero = true;
      break;
    }
    vi = w / nw;
    if (fabs(lambda - lambda_prev) <= 1e-12 * fabs(lambda)) break;
    lambda_prev = lambda;
  }
  vs[i] = vi;
  __syncthreads();
  if (i == 0) {
    if (zero)
      for (int k = 0; k < d; ++k) vs[k] = (k == 0) ? 1.0 : 0.0;
    int im = 0;
    double am = -1.0;
    for (int k = 0; k < d; ++k)
      if (fabs(vs[k]) > am) {
        am = fabs(vs[k]);
        im = k;
      }
    const double sgn = vs[im] < 0 ? -1.0 : 1.0;
    double ss = 0.0;
    for (int k = 0; k < d; ++k) ss += vs[k] * vs[k];
    const double inv = 1.0 / sqrt(ss);
    for (int k = 0; k < d; ++k) v_out[k] = sgn * vs[k] * inv;
    *iters_out = it > max_iter ? max_iter : it;
  }
}

// d <= kJacobiMaxD: the top eigenvector of C by cyclic Jacobi rotations
// (symmetric Schur rotations, rows and columns of a rotation updated by the
// lanes k < d), which converges in a few sweeps however close the two
// largest eigenvalues are, where the power iteration would need hundreds of
// steps.  A and the accumulated rotations V sit in LDS; the rotation of each
// pair (p, q) is computed by every lane from the same values (uniform).
// Stops when the off-diagonal entries are below 1e-30 of the squared
// Frobenius norm, or after 30 sweeps; v is the column of V of the largest
// diagonal entry, with the same sign convention as the power iteration (C = 0
// gives e_1).  iters_out counts sweeps.
constexpr int kJacobiMaxD = 4;

__global__ __launch_bounds__(kWave) void k_eig_jacobi(const double* __restrict__ C, int d, double* __restrict__ v_out,
                                                     int* __restrict__ iters_out) {
  __shared__ double A[kJacobiMaxD][kJacobiMaxD], V[kJacobiMaxD][kJacobiMaxD];
  const int k = threadIdx.x;
  if (k < d)
    for (int j = 0; j < d; ++j) {
      A[k][j] = C[(int64_t)k * d + j];
      V[k][j] = k == j ? 1.0 : 0.0;
    }
  __syncthreads();
  double fro = 0.0;
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) fro += A[i][j] * A[i][j];
  int sweep = 0;
  for (; sweep < 30; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < d; ++i)
      for (int j = i + 1; j < d; ++j) off += A[i][j] * A[i][j];
    if (!(off > 1e-30 * fro)) break;
    for (int p = 0; p < d; ++p)
      for (int q = p + 1; q < d; ++q) {
        const double apq = A[p][q];
        if (apq == 0.0) continue;
        const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double c = 1.0 / sqrt(1.0 + t * t), sn = t * c;
        __syncthreads();  // every lane has read A[p][q], A[p][p], A[q][q]
        if (k < d) {      // columns p, q of A and V
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - sn * akq;
          A[k][q] = sn * akp + c * akq;
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - sn * vkq;
          V[k][q] = sn * vkp + c * vkq;
        }
        __syncthreads();
        if (k < d) {  // rows p, q of A
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - sn * aqk;
          A[q][k] = sn * apk + c * aqk;
        }
        __syncthreads();
      }
  }
  if (k == 0) {
    int best = 0;
    for (int i = 1; i < d; ++i)
      if (A[i][i] > A[best][best]) best = i;
    double col[kJacobiMaxD];
    for (int i = 0; i < d; ++i) col[i] = fro > 0.0 ? V[i][best] : (i == 0 ? 1.0 : 0.0);
    int im = 0;
    double am = -1.0;
    for (int i = 0; i < d; ++i)
      if (fabs(col[i]) > am) {
        am = fabs(col[i]);
        im = i;
      }
    const double sgn = col[im] < 0 ? -1.0 : 1.0;
    double ss = 0.0;
    for (int i = 0; i < d; ++i) ss += col[i] * col[i];
    const double inv = 1.0 / sqrt(ss);
    for (int i = 0; i < d; ++i) v_out[i] = sgn * col[i] * inv;
    *iters_out = sweep > 0 ? sweep : 1;
  }
}

// Same iteration for 64 < d <= 128 with C resident in LDS (at most 128 KB):
// read once from HBM instead of from L2 on every step.  512 threads = 4 parts
// x 128 row slots; part p sums columns j = p, p + 4, ... of row i (C[j][i],
// conflict-free across a wavefront), the 4 partial sums meet in LDS, and the
// Rayleigh quotient and ||C v||^2 share one reduction.
constexpr int kPiSlots = 128, kPiParts = 4, kPiThreads = kPiSlots * kPiParts;

__global__ __launch_bounds__(kPiThreads) void k_power_iter_lds(const double* __restrict__ Cg, int d, int max_iter,
                                                               double* __restrict__ v_out,
                                                               int* __restrict__ iters_out) {
  extern __shared__ double lds[];
  __shared__ double red[2 * (kPiSlots / kWave)];
  double* v = lds;                 // kPiSlots
  double* wp = v + kPiSlots;       // kPiParts x kPiSlots partial sums
  double* C = wp + kPiThreads;     // d x d
  const int t = threadIdx.x, i = t % kPiSlots, p = t / kPiSlots;
  for (int e = t; e < d * d; e += kPiThreads) C[e] = Cg[e];
  double x = 0.0;
  if (t < d) x = 1.0 + 0.01 * (double)((t * 2654435761u) % 1000u) / 1000.0;
  if (t < kPiSlots) v[t] = x;
  __syncthreads();
  double loc = 0.0;
  for (int k = 0; k < d; ++k) loc += v[k] * v[k];
  __syncthreads();  // every thread has read v before it is overwritten
  if (t < kPiSlots) v[t] = x / sqrt(loc);
  __syncthreads();
  double lambda_prev = -1.0;
  int it = 0;
  bool zero = false;
  for (it = 1; it <= max_iter; ++it) {
    if (i < d) {
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      int j = p;
      for (; j + 3 * kPiParts < d; j += 4 * kPiParts) {
        a0 += C[j * d + i] * v[j];
        a1 += C[(j + kPiParts) * d + i] * v[j + kPiParts];
        a2 += C[(j + 2 * kPiParts) * d + i] * v[j + 2 * kPiParts];
        a3 += C[(j + 3 * kPiParts) * d + i] * v[j + 3 * kPiParts];
      }
      for (; j < d; j += kPiParts) a0 += C[j * d + i] * v[j];
      wp[p * kPiSlots + i] = (a0 + a1) + (a2 + a3);
    }
    __syncthreads();
    double sacc = 0.0, part = 0.0, nn = 0.0;
    if (t < kPiSlots) {  // waves 0 and 1 own the rows
      if (t < d) {
        sacc = (wp[t] + wp[kPiSlots + t]) + (wp[2 * kPiSlots + t] + wp[3 * kPiSlots + t]);
        part = sacc * v[t];
        nn = sacc * sacc;
      }
      part = wave_sum(part);
      nn = wave_sum(nn);
      if (lane_id() == 0) {
        red[2 * (t / kWave)] = part;
        red[2 * (t / kWave) + 1] = nn;
      }
    }
    __syncthreads();
    double lambda = 0.0, n2 = 0.0;
    for (int w = 0; w < kPiSlots / kWave; ++w) {
      lambda += red[2 * w];
      n2 += red[2 * w + 1];
    }
    const double nw = sqrt(n2);
    if (!(nw > 0.0)) {
      zero = true;
      break;
    }
    if (t < kPiSlots) v[t] = sacc / nw;  // every read of v this step is behind the barrier above
    __syncthreads();
    if (fabs(lambda - lambda_prev) <= 1e-12 * fabs(lambda)) break;
    lambda_prev = lambda;
  }
  __syncthreads();
  if (t == 0) {
    if (zero)
      for (int k = 0; k < d; ++k) v[k] = (k == 0) ? 1.0 : 0.0;
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
    for (int k = 0; k < d; ++k) v_out[k] = sgn * v[k] * inv;
    *iters_out = it > max_iter ? max_iter : it;
  }
}

size_t power_iter_lds_bytes(int d) { return sizeof(double) * ((size_t)kPiSlots + kPiThreads + (size_t)d * d); }

// The LDS form needs more than the default 64 KB of dynamic LDS: allowed
// when the device reports enough per workgroup and the limit can be raised.
bool power_iter_lds_ok(const DeviceInfo& di, int d) {
  const size_t need = power_iter_lds_bytes(d);
  if (need + 64 > (size_t)di.lds_bytes) return false;
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_power_iter_lds),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)need) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return true;
}

// ---- step 5: scores ----------------------------------------------------------
// Row kernels: G lanes per row (coalesced row reads), each lane taking
// elements sub, sub + G, ... of the row, NE of them per pass; a group of G
// lanes takes U rows at once (the projection: U = 8 / NE, so about eight
// loads per lane are in flight; the gather, whose row reads are random and
// whose occupancy matters more, U = 1).  The 64 / G groups of a wavefront take
// consecutive rows in each of the U slots, so that one load or store
// instruction covers one contiguous stretch of memory.  The mu and v entries
// a lane needs sit in its registers when a row takes one pass (d <= NE G),
// else in LDS (PM_LDS; d is at most 1024).
// The partial sums of a row meet by shuffles within its G lanes, in a fixed
// order (deterministic); any order stays within the gamma_{d+2} bound of the
// key error.
enum ParamMode { PM_REG, PM_LDS };

template <typename T, int G, int NE, int U, int PM>
__global__ __launch_bounds__(kThreads) void k_project(const T* __restrict__ X, int64_t n, int d,
                                                     const double* __restrict__ mu, const double* __restrict__ v,
                                                     uint32_t* __restrict__ ukey, uint32_t* __restrict__ val,
                                                     double* __restrict__ block_max) {
  extern __shared__ double prm[];  // PM_LDS: mu (d) | v (d), at most 16 KB
  const double* mup = mu;
  const double* vp = v;
  if (PM == PM_LDS) {
    for (int k = threadIdx.x; k < d; k += kThreads) {
      prm[k] = mu[k];
      prm[d + k] = v[k];
    }
    __syncthreads();
    mup = prm;
    vp = prm + d;
  }
  constexpr int GW = kWave / G;  // groups per wavefront
  const int sub = threadIdx.x % G, q = (threadIdx.x % kWave) / G;
  double mur[NE], vr[NE];  // PM_REG: the lane's entries k = sub + j G
#pragma unroll
  for (int j = 0; j < NE; ++j) {
    const int k = sub + j * G;
    mur[j] = (PM == PM_REG && k < d) ? mu[k] : 0.0;
    vr[j] = (PM == PM_REG && k < d) ? v[k] : 0.0;
  }
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  double nmax = 0.0;
  for (int64_t base = wave * U * GW; base < n; base += nwaves * U * GW) {
    const int64_t i0 = base + q;  // rows i0 + u GW
    double a[U], nn[U];
#pragma unroll
    for (int u = 0; u < U; ++u) a[u] = nn[u] = 0.0;
    for (int kc = 0; kc < d; kc += NE * G) {
      T xv[U][NE];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int j = 0; j < NE; ++j) {
          const int k = kc + sub + j * G;
          xv[u][j] = (i0 + u * GW < n && k < d) ? X[(i0 + u * GW) * d + k] : T(0);
        }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int j = 0; j < NE; ++j) {
          const int k = kc + sub + j * G;
          if (k < d) {
            const double x = (double)xv[u][j] - (PM == PM_REG ? mur[j] : mup[k]);
            a[u] += x * (PM == PM_REG ? vr[j] : vp[k]);
            const double y = (double)(float)x;
            nn[u] += y * y;
          }
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int off = G / 2; off > 0; off >>= 1) {
        a[u] += __shfl_xor(a[u], off, G);
        nn[u] += __shfl_xor(nn[u], off, G);
      }
      if (sub == 0 && i0 + u * GW < n) {
        ukey[i0 + u * GW] = float_to_ordered((float)a[u]);
        val[i0 + u * GW] = (uint32_t)(i0 + u * GW);
      }
      nmax = fmax(nmax, nn[u]);
    }
  }
  // one maximum per workgroup, folded by k_max_final (atomics on a single
  // address serialise: thousands of them cost more than the whole pass)
  __shared__ double red[kThreads / kWave];
  nmax = wave_max(nmax);
  if (lane_id() == 0) red[threadIdx.x / kWave] = nmax;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kThreads / kWave; ++w) nmax = fmax(nmax, red[w]);
    block_max[blockIdx.x] = nmax;
  }
}

// The same for float rows of d <= 16: four lanes per row, each a run of
// four coordinates (one 16-byte load where the rows are 16-byte aligned, vec),
// U rows per group of lanes in flight.
template <int U>
__global__ __launch_bounds__(kThreads) void k_project4(const float* __restrict__ X, int64_t n, int d,
                                                      const double* __restrict__ mu, const double* __restrict__ v,
                                                      uint32_t* __restrict__ ukey, uint32_t* __restrict__ val,
                                                      double* __restrict__ block_max, int vec) {
  const int sub = threadIdx.x & 3, k0 = 4 * sub, grp = (threadIdx.x % kWave) >> 2;
  double mur[4], vr[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    mur[j] = k0 + j < d ? mu[k0 + j] : 0.0;
    vr[j] = k0 + j < d ? v[k0 + j] : 0.0;
  }
  constexpr int GW = kWave / 4;  // rows per wavefront and unroll step
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  double nmax = 0.0;
  for (int64_t base = wave * U * GW; base < n; base += nwaves * U * GW) {
    float xv[U][4];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = base + grp + u * GW;
      const float* x = X + i * d;
      if (vec && i < n && k0 < d) {
        const float4 t = *reinterpret_cast<const float4*>(x + k0);
        xv[u][0] = t.x, xv[u][1] = t.y, xv[u][2] = t.z, xv[u][3] = t.w;
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) xv[u][j] = (i < n && k0 + j < d) ? x[k0 + j] : 0.f;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = base + grp + u * GW;
      double a = 0.0, nn = 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (k0 + j < d) {
          const double x = (double)xv[u][j] - mur[j];
          a += x * vr[j];
          const double y = (double)(float)x;
          nn += y * y;
        }
      a += __shfl_xor(a, 1, 4);
      nn += __shfl_xor(nn, 1, 4);
      a += __shfl_xor(a, 2, 4);
      nn += __shfl_xor(nn, 2, 4);
      if (sub == 0 && i < n) {
        ukey[i] = float_to_ordered((float)a);
        val[i] = (uint32_t)i;
      }
      if (i < n) nmax = fmax(nmax, nn);
    }
  }
  __shared__ double red[kThreads / kWave];
  nmax = wave_max(nmax);
  if (lane_id() == 0) red[threadIdx.x / kWave] = nmax;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kThreads / kWave; ++w) nmax = fmax(nmax, red[w]);
    block_max[blockIdx.x] = nmax;
  }
}

// *max_norm = max(*max_norm, block_max[0 .. nblocks)) in one workgroup of
// kMaxFinalThreads, eight loads in flight per thread
constexpr int kMaxFinalThreads = 1024;

__global__ __launch_bounds__(kMaxFinalThreads) void k_max_final(const double* __restrict__ block_max, int nblocks,
                                                                double* __restrict__ max_norm) {
  __shared__ double red[kMaxFinalThreads / kWave];
  double m = 0.0;
  int b = threadIdx.x;
  for (; b + 7 * kMaxFinalThreads < nblocks; b += 8 * kMaxFinalThreads) {
    double x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = block_max[b + u * kMaxFinalThreads];
#pragma unroll
    for (int u = 0; u < 8; ++u) m = fmax(m, x[u]);
  }
  for (; b < nblocks; b += kMaxFinalThreads) m = fmax(m, block_max[b]);
  m = wave_max(m);
  if (lane_id() == 0) red[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 0; w < kMaxFinalThreads / kWave; ++w) m = fmax(m, red[w]);
    *max_norm = fmax(*max_norm, m);
  }
}

// ---- gather into score order -------------------------------------------------
// Same lane layout: a group gathers U consecutive destination rows (random
// source rows of X), G consecutive elements at a time; the squared norm of
// each row meets by shuffles within its G lanes.
template <typename T, int G, int NE, int U, int PM>
__global__ __launch_bounds__(kThreads) void k_gather(const T* __restrict__ X, int64_t n, int d, int dp,
                                                    const double* __restrict__ mu,
                                                    const uint32_t* __restrict__ ukey,
                                                    const uint32_t* __restrict__ val, double* __restrict__ key,
                                                    int32_t* __restrict__ perm, T* __restrict__ po,
                                                    double* __restrict__ p64, float* __restrict__ ys,
                                                    float* __restrict__ h, float* __restrict__ ynorm,
                                                    int64_t id_base) {
  extern __shared__ double prm[];  // PM_LDS: mu (d)
  const double* mup = mu;
  if (PM == PM_LDS) {
    for (int k = threadIdx.x; k < d; k += kThreads) prm[k] = mu[k];
    __syncthreads();
    mup = prm;
  }
  double mur[NE];  // PM_REG: the lane's entries k = sub + j G
#pragma unroll
  for (int j = 0; j < NE; ++j) {
    const int k = threadIdx.x % G + j * G;
    mur[j] = (PM == PM_REG && k < d) ? mu[k] : 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x < 64) h[n + threadIdx.x] = INFINITY;  // padding rows
  constexpr int GW = kWave / G;  // groups per wavefront
  const int sub = threadIdx.x % G, q = (threadIdx.x % kWave) / G;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t base = wave * U * GW; base < n; base += nwaves * U * GW) {
    const int64_t s0 = base + q;  // destination rows s0 + u GW
    uint32_t src[U];
    double nn[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      src[u] = s0 + u * GW < n ? val[s0 + u * GW] : 0u;
      nn[u] = 0.0;
    }
    for (int kc = 0; kc < dp; kc += NE * G) {
      T xv[U][NE];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int j = 0; j < NE; ++j) {
          const int k = kc + sub + j * G;
          xv[u][j] = (s0 + u * GW < n && k < d) ? X[(int64_t)src[u] * d + k] : T(0);
        }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int j = 0; j < NE; ++j) {
          const int64_t s = s0 + u * GW;
          const int k = kc + sub + j * G;
          if (s < n && k < dp) {
            if (k < d) {
              const T x = xv[u][j];
              po[s * d + k] = x;
              if (p64) p64[s * dp + k] = (double)x;
              const float y = (float)((double)x - (PM == PM_REG ? mur[j] : mup[k]));
              ys[s * d + k] = y;
              nn[u] += (double)y * (double)y;
            } else if (p64) {
              p64[s * dp + k] = 0.0;
            }
          }
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t s = s0 + u * GW;
#pragma unroll
      for (int off = G / 2; off > 0; off >>= 1) nn[u] += __shfl_xor(nn[u], off, G);
      if (sub == 0 && s < n) {
        perm[s] = (int32_t)(id_base + src[u]);
        key[s] = (double)ordered_to_float(ukey[s]);
        h[s] = (float)(0.5 * nn[u]);
        // round ||y|| up to float so it bounds the true norm
        float nr = (float)sqrt(nn[u]);
        if ((double)nr < sqrt(nn[u])) nr = nextafterf(nr, INFINITY);
        ynorm[s] = nr;
      }
    }
  }
}

// The same for float rows of d <= 16 (dp <= 16): four lanes per row, each a
// run of four coordinates, U destination rows per group of lanes in flight;
// 16-byte loads and stores where the rows are 16-byte aligned (vec).
template <int U>
__global__ __launch_bounds__(kThreads) void k_gather4(const float* __restrict__ X, int64_t n, int d, int dp,
                                                     const double* __restrict__ mu,
                                                     const uint32_t* __restrict__ ukey,
                                                     const uint32_t* __restrict__ val, double* __restrict__ key,
                                                     int32_t* __restrict__ perm, float* __restrict__ po,
                                                     double* __restrict__ p64, float* __restrict__ ys,
                                                     float* __restrict__ h, float* __restrict__ ynorm,
                                                     int64_t id_base, int vec) {
  const int sub = threadIdx.x & 3, k0 = 4 * sub, grp = (threadIdx.x % kWave) >> 2;
  double mur[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) mur[j] = k0 + j < d ? mu[k0 + j] : 0.0;
  if (blockIdx.x == 0 && threadIdx.x < 64) h[n + threadIdx.x] = INFINITY;  // padding rows
  constexpr int GW = kWave / 4;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t base = wave * U * GW; base < n; base += nwaves * U * GW) {
    uint32_t src[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t s = base + grp + u * GW;
      src[u] = s < n ? val[s] : 0u;
    }
    float xv[U][4];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t s = base + grp + u * GW;
      const float* x = X + (int64_t)src[u] * d;
      if (vec && s < n && k0 < d) {
        const float4 t = *reinterpret_cast<const float4*>(x + k0);
        xv[u][0] = t.x, xv[u][1] = t.y, xv[u][2] = t.z, xv[u][3] = t.w;
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) xv[u][j] = (s < n && k0 + j < d) ? x[k0 + j] : 0.f;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t s = base + grp + u * GW;
      float y[4];
      double nn = 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        y[j] = k0 + j < d ? (float)((double)xv[u][j] - mur[j]) : 0.f;
        nn += (double)y[j] * (double)y[j];
      }
      if (s < n) {
        if (vec) {
          if (k0 < d) {
            *reinterpret_cast<float4*>(po + s * d + k0) = make_float4(xv[u][0], xv[u][1], xv[u][2], xv[u][3]);
            *reinterpret_cast<float4*>(ys + s * d + k0) = make_float4(y[0], y[1], y[2], y[3]);
          }
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (k0 + j < d) {
              po[s * d + k0 + j] = xv[u][j];
              ys[s * d + k0 + j] = y[j];
            }
        }
        if (p64 && k0 < dp) {  // dp is a multiple of 4; the padding columns are zero
          double2* o = reinterpret_cast<double2*>(p64 + s * dp + k0);
          o[0] = make_double2((double)xv[u][0], (double)xv[u][1]);
          o[1] = make_double2((double)xv[u][2], (double)xv[u][3]);
        }
      }
      nn += __shfl_xor(nn, 1, 4);
      nn += __shfl_xor(nn, 2, 4);
      if (sub == 0 && s < n) {
        perm[s] = (int32_t)(id_base + src[u]);
        key[s] = (double)ordered_to_float(ukey[s]);
        h[s] = (float)(0.5 * nn);
        // round ||y|| up to float so it bounds the true norm
        float nr = (float)sqrt(nn);
        if ((double)nr < sqrt(nn)) nr = nextafterf(nr, INFINITY);
        ynorm[s] = nr;
      }
    }
  }
}

int grid_for(int64_t work, int per_block, int cap);

// Lanes per row G of the row kernels (enough to read a short row in one
// step, at most 16) and elements per lane per pass NE (a power of two, at
// most 8; rows wider than 8 G take several passes).  f is called with both as
// integral constants.
template <typename F>
void row_shape(int width, F&& f) {
  using std::integral_constant;
  if (width <= 4)
    f(integral_constant<int, 4>{}, integral_constant<int, 1>{});
  else if (width <= 8)
    f(integral_constant<int, 8>{}, integral_constant<int, 1>{});
  else if (width <= 16)
    f(integral_constant<int, 16>{}, integral_constant<int, 1>{});
  else if (width <= 32)
    f(integral_constant<int, 16>{}, integral_constant<int, 2>{});
  else if (width <= 64)
    f(integral_constant<int, 16>{}, integral_constant<int, 4>{});
  else
    f(integral_constant<int, 16>{}, integral_constant<int, 8>{});
}

// block_max: cap doubles of scratch; *max_norm is raised to the largest
// squared norm of fl32(x - mu) over the rows
template <typename T>
void launch_project(const T* X, int64_t n, int d, const double* mu, const double* v, uint32_t* ukey, uint32_t* val,
                    double* block_max, double* max_norm, int cap, hipStream_t s) {
  int grid = 1;
  if (std::is_same<T, float>::value && d <= 16) {
    constexpr int U = 4;
    const int vec = d % 4 == 0 && reinterpret_cast<uintptr_t>(X) % 16 == 0;
    grid = grid_for((std::max<int64_t>(n, 1) + U - 1) / U * 4, kThreads, cap);
    k_project4<U><<<grid, kThreads, 0, s>>>(reinterpret_cast<const float*>(X), n, d, mu, v, ukey, val, block_max,
                                            vec);
    SNN_LAUNCH_CHECK();
    k_max_final<<<1, kMaxFinalThreads, 0, s>>>(block_max, grid, max_norm);
    SNN_LAUNCH_CHECK();
    return;
  }
  row_shape(d, [&](auto g, auto ne) {
    constexpr int G = decltype(g)::value, NE = decltype(ne)::value, U = NE >= 8 ? 1 : 8 / NE;
    grid = grid_for((std::max<int64_t>(n, 1) + U - 1) / U * G, kThreads, cap);
    if (d <= NE * G)
      k_project<T, G, NE, U, PM_REG><<<grid, kThreads, 0, s>>>(X, n, d, mu, v, ukey, val, block_max);
    else
      k_project<T, G, NE, U, PM_LDS><<<grid, kThreads, 2 * sizeof(double) * d, s>>>(X, n, d, mu, v, ukey, val,
                                                                                   block_max);
  });
  SNN_LAUNCH_CHECK();
  k_max_final<<<1, kMaxFinalThreads, 0, s>>>(block_max, grid, max_norm);
  SNN_LAUNCH_CHECK();
}

template <typename T>
void launch_gather(const T* X, int64_t n, int d, int dp, const double* mu, const uint32_t* ukey, const uint32_t* val,
                   double* key, int32_t* perm, T* po, double* p64, float* ys, float* h, float* ynorm, int64_t id_base,
                   int cap, hipStream_t s) {
  if (std::is_same<T, float>::value && dp <= 16) {
    constexpr int U = 2;
    const int vec = d % 4 == 0 && reinterpret_cast<uintptr_t>(X) % 16 == 0;
    const int grid = grid_for((std::max<int64_t>(n, 1) + U - 1) / U * 4, kThreads, cap);
    k_gather4<U><<<grid, kThreads, 0, s>>>(reinterpret_cast<const float*>(X), n, d, dp, mu, ukey, val, key, perm,
                                           reinterpret_cast<float*>(po), p64, ys, h, ynorm, id_base, vec);
    SNN_LAUNCH_CHECK();
    return;
  }
  row_shape(dp, [&](auto g, auto ne) {
    constexpr int G = decltype(g)::value, NE = decltype(ne)::value;
    const int grid = grid_for(std::max<int64_t>(n, 1) * G, kThreads, cap);
    if (dp <= NE * G)
      k_gather<T, G, NE, 1, PM_REG><<<grid, kThreads, 0, s>>>(X, n, d, dp, mu, ukey, val, key, perm, po, p64, ys, h,
                                                           ynorm, id_base);
    else
      k_gather<T, G, NE, 1, PM_LDS><<<grid, kThreads, sizeof(double) * d, s>>>(X, n, d, dp, mu, ukey, val, key, perm,
                                                                          po, p64, ys, h, ynorm, id_base);
  });
  SNN_LAUNCH_CHECK();
}

// ---- mixed-precision operand rows ---------------------------------------------
// terms = 1: row = [bf16(y_0..y_{d-1}), 0...]                 (ka = pad16(d))
// terms = 3: cand = [hi | lo | hi], query = [hi | hi | lo]     (ka = pad16(3d))
// with hi = bf16(y), lo = bf16(y - hi) (y - hi is exact in float).  When d is
// a multiple of 16 the candidate rows are stored as [hi | lo] (kb = 2d): the
// third segment equals the first and the screen reuses its registers.
//
// Candidate rows are stored in the matrix-core operand order: blocks of 32
// rows, and inside a block [slice s of 16][half h of 8][row r][8 values], so
// that one wavefront load of 16 bytes per lane (lane = 32 h + r) reads 1 KB
// of contiguous memory.  npad (a multiple of 32, at least n + 32) rows are
// stored; rows n .. npad-1 are zero.  Query rows for self-queries stay
// row-major (ka per row).
// Screen operand rows of the sorted centred rows y (see k_cand_mfma.hip):
// kind bf16: bf16(y); bf16 hi/lo: candidates [hi | lo], queries [hi | hi |
// lo] (hi = bf16(y), lo = bf16(y - hi)); fp16: fp16(2^e y).  Candidate rows
// go to 32-row blocks of 16-value slices (half-slice h of row r at
// ((block * nl + slice) * 2 + h) * 256 + r * 8), query rows stay row-major.
// For fp16 the candidates' h is scaled by 2^(2e) and rounded down into hs.
__global__ __launch_bounds__(kThreads) void k_operands(const float* __restrict__ ys, const float* __restrict__ h,
                                                      int64_t n, int64_t npad, int d, int kind, int e, int ka, int kb,
                                                      uint16_t* __restrict__ cand, uint16_t* __restrict__ qself,
                                                      float* __restrict__ hs) {
  // four consecutive columns per thread (ka and kb are multiples of 16, so
  // the four lie in one 8-column group of the candidate layout and both
  // stores are 8-byte aligned)
  const int ka4 = ka / 4;
  const int64_t total = npad * (int64_t)ka4;
  const int nl = kb / 16;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = g / ka4;
    const int k0 = 4 * (int)(g - s * ka4);
    uint16_t cv[4] = {0, 0, 0, 0}, qv[4] = {0, 0, 0, 0};
    if (s < n) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = k0 + u;
        if (kind == kOpF16) {
          if (k < d) cv[u] = qv[u] = __builtin_bit_cast(uint16_t, (_Float16)ldexpf(ys[s * d + k], e));
        } else if (kind == kOpBf16) {
          if (k < d) cv[u] = qv[u] = f32_to_bf16_rne(ys[s * d + k]);
        } else if (k < 3 * d) {
          const int seg = k / d, c = k % d;
          const float y = ys[s * d + c];
          const uint16_t hi = f32_to_bf16_rne(y);
          const uint16_t lo = f32_to_bf16_rne(y - bf16_to_f32(hi));
          cv[u] = (seg == 1) ? lo : hi;
          qv[u] = (seg == 2) ? lo : hi;
        }
      }
    }
    if (k0 < kb) {
      const int64_t blk = s / 32;
      const int r = (int)(s % 32), sl = k0 / 16, hh = (k0 % 16) / 8, c8 = k0 % 8;
      *reinterpret_cast<uint2*>(cand + ((blk * nl + sl) * 2 + hh) * 256 + r * 8 + c8) =
          make_uint2(cv[0] | (uint32_t)cv[1] << 16, cv[2] | (uint32_t)cv[3] << 16);
    }
    if (qself && s < n)
      *reinterpret_cast<uint2*>(qself + s * ka + k0) =
          make_uint2(qv[0] | (uint32_t)qv[1] << 16, qv[2] | (uint32_t)qv[3] << 16);
    if (hs && k0 == 0) {
      float v = INFINITY;
      if (s < n) {
        // the scaling is exact unless it lands below fp32's normal range
        const double x = ldexp((double)h[s], 2 * e);
        v = (float)x;
        if ((double)v > x) v = nextafterf(v, -INFINITY);
      }
      hs[s] = v;
    }
  }
}

int grid_for(int64_t work, int per_block = kThreads, int cap = 8192) {
  int64_t g = (work + per_block - 1) / per_block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

template <typename T>
void build_index_t(Index& ix, const T* X) {
  hipStream_t s = ix.arena.stream();
  const int64_t n = ix.n;
  const int d = ix.d;
  const DeviceInfo& di = device_info(ix.arena.dev().device);

  ix.mu.ensure(ix.arena, sizeof(double) * d);
  ix.v.ensure(ix.arena, sizeof(double) * d);
  {
    Buffer* views[] = {&ix.key, &ix.perm, &ix.po, &ix.p64, &ix.ys, &ix.h, &ix.ynorm};
    const size_t sizes[] = {sizeof(double) * n,         sizeof(int32_t) * n,      sizeof(T) * n * d,
                            sizeof(double) * n * ix.dp, sizeof(float) * n * d,    sizeof(float) * (n + 64),
                            sizeof(float) * n};
    size_t total = 0;
    for (size_t b : sizes) total += align256(b);
    for (Buffer* b : views) b->reset(ix.arena);
    ix.rows.ensure(ix.arena, total);
    char* base = static_cast<char*>(ix.rows.ptr);
    for (int k = 0; k < 7; ++k) {
      views[k]->ptr = base;
      views[k]->bytes = sizes[k];
      views[k]->view = true;
      base += align256(sizes[k]);
    }
  }

  // scratch: partials, flags, Gram, power-iteration work
  // at least 16 elements per thread (4096 per workgroup) keep enough loads
  // in flight; at most 4096 workgroups
  const int g1 = (int)std::min<int64_t>(4096, std::max<int64_t>(1, (n * d + 4095) / 4096));
  const int64_t rpb1 = (n + g1 - 1) / g1;
  int64_t dd = (int64_t)d * d;
  // Gram tiles on the matrix cores: 16 * tb columns a side, npairs tile
  // pairs on or above the diagonal (one pair up to d = 64)
  const int tb = d <= 16 ? 1 : d <= 32 ? 2 : d <= 48 ? 3 : 4;
  const int nbk = (d + 16 * tb - 1) / (16 * tb), npairs = nbk * (nbk + 1) / 2;
  const bool gram_mfma = d >= kGramMfmaMinD;
  const bool gram_split = gram_mfma && npairs == 1;
  // about 512 rows per wavefront and up to 8 wavefronts per CU: with fewer,
  // larger blocks the staging rounds of the rows are latency-bound.  With
  // one pair, kGramWaves wavefronts share a workgroup's rows (one partial
  // Gram matrix per kGramWaves wavefronts for the final sum to read).
  const int64_t rows_wg = gram_split ? 512 * kGramWaves : 512;
  const int64_t max_wg = gram_split ? 8 * (int64_t)di.cus / kGramWaves : 8 * (int64_t)di.cus;
  int g2 = (int)std::min<int64_t>(std::max<int64_t>(1, (n + rows_wg - 1) / rows_wg), max_wg);
  g2 = (int)std::max<int64_t>(1, std::min<int64_t>(g2, (int64_t)(256ll << 20) / (dd * 8)));
  const int64_t rpb2 = (n + g2 - 1) / g2;
  const int rows_chunk = (int)std::max<int64_t>(1, std::min<int64_t>(64, 4096 / d));

  struct Scratch {
    int bad;
    int iters;
    double max_norm;
    int sort_err;
  };
  const size_t off_part1 = 256;
  const size_t off_part2 = off_part1 + ((sizeof(double) * g1 * d + 255) & ~size_t(255));
  const size_t off_C = off_part2 + ((sizeof(double) * g2 * dd + 255) & ~size_t(255));
  const int proj_cap = 4 * di.cus * 8;
  const size_t off_bmax = off_C + ((sizeof(double) * dd + 255) & ~size_t(255));
  const size_t off_keys = off_bmax + ((sizeof(double) * proj_cap + 255) & ~size_t(255));
  const size_t off_sort = off_keys + align256(2 * sizeof(uint32_t) * n);
  const size_t total = off_sort + radix_sort_ws_bytes(n) + 256;
  ScopedAlloc scratch(ix.arena, total);
  char* mem = static_cast<char*>(scratch.get());
  Scratch* sc = reinterpret_cast<Scratch*>(mem);
  double* part1 = reinterpret_cast<double*>(mem + off_part1);
  double* part2 = reinterpret_cast<double*>(mem + off_part2);
  double* C = reinterpret_cast<double*>(mem + off_C);
  double* bmax = reinterpret_cast<double*>(mem + off_bmax);
  uint32_t* ukey = reinterpret_cast<uint32_t*>(mem + off_keys);
  uint32_t* val = ukey + n;

  SNN_HIP(hipMemsetAsync(sc, 0, sizeof(Scratch), s));
  k_colsum_partial<T><<<g1, kThreads, 0, s>>>(X, n, d, rpb1, part1, &sc->bad);
  SNN_LAUNCH_CHECK();
  k_colsum_final<<<d, kWave, 0, s>>>(part1, g1, d, n, ix.mu.as<double>());
  SNN_LAUNCH_CHECK();

  const size_t lds2 = sizeof(double) * rows_chunk * d;
  if (gram_mfma) {
    const int w = gram_split ? kGramWaves : std::min(npairs, kGramWaves);
    const dim3 grid(g2, gram_split ? 1 : (npairs + w - 1) / w);
    const double* mu = ix.mu.as<double>();
    switch (tb) {
      case 1: k_gram_mfma<T, 1><<<grid, w * kWave, 0, s>>>(X, n, d, mu, rpb2, npairs, part2); break;
      case 2: k_gram_mfma<T, 2><<<grid, w * kWave, 0, s>>>(X, n, d, mu, rpb2, npairs, part2); break;
      case 3: k_gram_mfma<T, 3><<<grid, w * kWave, 0, s>>>(X, n, d, mu, rpb2, npairs, part2); break;
      default: k_gram_mfma<T, 4><<<grid, w * kWave, 0, s>>>(X, n, d, mu, rpb2, npairs, part2); break;
    }
  } else {
    k_gram_partial<T><<<g2, kThreads, lds2, s>>>(X, n, d, ix.mu.as<double>(), rpb2, rows_chunk, part2);
  }
  SNN_LAUNCH_CHECK();
  k_gram_final<<<(int)((dd + kWave - 1) / kWave), kGramFinalWaves * kWave, 0, s>>>(part2, g2, dd, C);
  SNN_LAUNCH_CHECK();
  if (d <= kJacobiMaxD)
    k_eig_jacobi<<<1, kWave, 0, s>>>(C, d, ix.v.as<double>(), &sc->iters);
  else if (d <= 8)
    k_power_iter_wave<8><<<1, kWave, 0, s>>>(C, d, 500, ix.v.as<double>(), &sc->iters);
  else if (d <= 16)
    k_power_iter_wave<16><<<1, kWave, 0, s>>>(C, d, 500, ix.v.as<double>(), &sc->iters);
  else if (d <= 32)
    k_power_iter_wave<32><<<1, kWave, 0, s>>>(C, d, 500, ix.v.as<double>(), &sc->iters);
  else if (d <= kWave)
    k_power_iter_wave<64><<<1, kWave, 0, s>>>(C, d, 500, ix.v.as<double>(), &sc->iters);
  else if (d <= kPiSlots && power_iter_lds_ok(di, d))
    k_power_iter_lds<<<1, kPiThreads, power_iter_lds_bytes(d), s>>>(C, d, 500, ix.v.as<double>(), &sc->iters);
  else
    k_power_iter<1024><<<1, 1024, 2 * sizeof(double) * d, s>>>(C, d, 500, ix.v.as<double>(), &sc->iters);
  SNN_LAUNCH_CHECK();
  launch_project<T>(X, n, d, ix.mu.as<double>(), ix.v.as<double>(), ukey, val, bmax, &sc->max_norm, proj_cap, s);
  uint32_t *skey, *sval;  // the sorted pairs, where the last pass left them
  radix_sort_pairs_ws(ukey, val, n, 0, 32, mem + off_sort, s, &skey, &sval, &sc->sort_err);
  T* po = ix.po.as<T>();
  // the float64 rows wait for the first fp64 screen (build_rows64)
  double* p64 = nullptr;
  ix.p64_ready = false;
  launch_gather<T>(X, n, d, ix.dp, ix.mu.as<double>(), skey, sval, ix.key.as<double>(), ix.perm.as<int32_t>(), po, p64,
                   ix.ys.as<float>(), ix.h.as<float>(), ix.ynorm.as<float>(), 0, 4 * di.cus * 8, s);

  // one read-back into page-locked memory: the flags and the direction
  char* hb = static_cast<char*>(pinned_host(256 + sizeof(double) * d));
  SNN_HIP(hipMemcpyAsync(hb, sc, sizeof(Scratch), hipMemcpyDeviceToHost, s));
  SNN_HIP(hipMemcpyAsync(hb + 256, ix.v.ptr, sizeof(double) * d, hipMemcpyDeviceToHost, s));
  SNN_HIP(hipStreamSynchronize(s));
  Scratch hs;
  std::memcpy(&hs, hb, sizeof(Scratch));
  if (hs.bad) fail(SNN_EINVAL, "snn_index: X contains NaN or Inf");
  if (hs.sort_err) fail(SNN_EDEVICE, "snn_index: a scan of the radix sort did not complete");
  const double* vh = reinterpret_cast<const double*>(hb + 256);
  double vn = 0.0;
  for (int k = 0; k < d; ++k) vn += vh[k] * vh[k];
  const double u64 = std::ldexp(1.0, -53), u32 = std::ldexp(1.0, -24);
  ix.vnorm = std::sqrt(vn) * (1.0 + 4.0 * (d + 2) * u64);
  ix.max_norm = std::sqrt(hs.max_norm) * (1.0 + 4.0 * (d + 2) * u64);
  ix.power_iters = hs.iters;
  // |fl32(fl64(x . v)) - (p - mu).v| <= (u32 + gamma64_{d+2}) ||p - mu|| ||v||,
  // and ||p - mu|| <= ||y|| (1 + u32) with y = fl32(p - mu).
  const double g64 = (d + 2) * u64 / (1.0 - (d + 2) * u64);
  ix.key_eps = 1.01 * (u32 + g64) * (1.0 + u32) * ix.max_norm * ix.vnorm;
}

}  // namespace

void build_index(Index& ix, const void* X) {
  if (ix.dtype == SNN_F32)
    build_index_t<float>(ix, static_cast<const float*>(X));
  else
    build_index_t<double>(ix, static_cast<const double*>(X));
}

namespace {
// float64 copy of the sorted rows, zero-padded to dp columns
template <typename T>
__global__ __launch_bounds__(kThreads) void k_rows64(const T* __restrict__ po, int64_t n, int d, int dp,
                                                    double* __restrict__ p64) {
  const int64_t total = n * (int64_t)dp;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = e / dp;
    const int k = (int)(e - s * dp);
    p64[e] = k < d ? (double)po[s * d + k] : 0.0;
  }
}
}  // namespace

void build_rows64(Index& ix) {
  if (ix.p64_ready || ix.n == 0) return;
  const int grid = grid_for(ix.n * (int64_t)ix.dp, kThreads, 4 * device_info(ix.arena.dev().device).cus * 8);
  if (ix.dtype == SNN_F32)
    k_rows64<float><<<grid, kThreads, 0, ix.arena.stream()>>>(ix.po.as<float>(), ix.n, ix.d, ix.dp,
                                                              ix.p64.as<double>());
  else
    k_rows64<double><<<grid, kThreads, 0, ix.arena.stream()>>>(ix.po.as<double>(), ix.n, ix.d, ix.dp,
                                                               ix.p64.as<double>());
  SNN_LAUNCH_CHECK();
  ix.p64_ready = true;
}

// ---- streaming inserts ---------------------------------------------------------
// Merge path: output row t of the merge of A (old rows, na) and B (new
// rows, nb), both sorted by key, comes from A[i] or B[t - i] where i is the
// number of A rows among the first t outputs; equal keys keep A first.
// src[t] = i (from A) or -(t - i) - 1 (from B).
__global__ __launch_bounds__(kThreads) void k_merge_path(const double* __restrict__ ka, int64_t na,
                                                         const double* __restrict__ kb, int64_t nb,
                                                         int64_t* __restrict__ src) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < na + nb;
       t += (int64_t)gridDim.x * blockDim.x) {
    // smallest i in [max(0, t - nb), min(t, na)] with "A[i] comes after B[t - i - 1]"
    int64_t lo = t - nb > 0 ? t - nb : 0, hi = t < na ? t : na;
    while (lo < hi) {
      const int64_t i = (lo + hi) / 2;  // A[i] vs B[t - i - 1]: if A[i] <= B[t-i-1], A[i] is among the first t
      if (ka[i] <= kb[t - i - 1])
        lo = i + 1;
      else
        hi = i;
    }
    // output t is the smaller of A[lo] and B[t - lo] (A first on ties)
    const bool fromA = lo < na && (t - lo >= nb || ka[lo] <= kb[t - lo]);
    src[t] = fromA ? lo : -(t - lo) - 1;
  }
}

// Copies w values per row from A or B into the merged array.
template <typename V>
__global__ __launch_bounds__(kThreads) void k_merge_rows(const V* __restrict__ a, const V* __restrict__ b,
                                                         const int64_t* __restrict__ src, int64_t rows, int w,
                                                         V* __restrict__ out) {
  const int64_t total = rows * w;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = e / w;
    const int c = (int)(e % w);
    const int64_t sidx = src[t];
    out[e] = sidx >= 0 ? a[sidx * w + c] : b[(-sidx - 1) * w + c];
  }
}

template <typename V>
static void merge_rows(const V* a, const V* b, const int64_t* src, int64_t rows, int w, V* out, int cap,
                       hipStream_t s) {
  k_merge_rows<V><<<grid_for(rows * w, kThreads, cap), kThreads, 0, s>>>(a, b, src, rows, w, out);
  SNN_LAUNCH_CHECK();
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_check_finite(const T* __restrict__ X, int64_t total,
                                                           int* __restrict__ bad) {
  int b = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite((double)X[e])) b = 1;
  if (b) atomicOr(bad, 1);
}

__global__ void k_fill_inf(float* __restrict__ p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = INFINITY;
}

template <typename T>
static void insert_points_t(Index& ix, const T* Xn, int64_t k) {
  hipStream_t s = ix.arena.stream();
  const DeviceInfo& di = device_info(ix.arena.dev().device);
  const int d = ix.d, dp = ix.dp;
  const int64_t na = ix.n, nt = na + k;

  // the new rows in key order, with the index's mu and v (scratch)
  struct Scratch {
    int bad;
    int pad;
    double max_norm;
  };
  Carver sz(nullptr);
  sz.take<Scratch>(1);
  sz.take<uint32_t>(k);
  sz.take<uint32_t>(k);
  sz.take<double>(k);                 // key
  sz.take<int32_t>(k);                // perm
  sz.take<T>((size_t)k * d);          // po
  sz.take<float>((size_t)k * d);      // ys
  sz.take<float>(k + 64);             // h
  sz.take<float>(k);                  // ynorm
  sz.take<int64_t>(nt);               // merge sources
  sz.take<double>(4 * di.cus * 8);    // per-workgroup norm maxima
  ScopedAlloc scratch(ix.arena, sz.off);
  Carver c(scratch.get());
  Scratch* sc = c.take<Scratch>(1);
  uint32_t* ukey = c.take<uint32_t>(k);
  uint32_t* val = c.take<uint32_t>(k);
  double* keyb = c.take<double>(k);
  int32_t* permb = c.take<int32_t>(k);
  T* pob = c.take<T>((size_t)k * d);
  float* ysb = c.take<float>((size_t)k * d);
  float* hb = c.take<float>(k + 64);
  float* ynb = c.take<float>(k);
  int64_t* src = c.take<int64_t>(nt);
  double* bmax = c.take<double>(4 * di.cus * 8);

  SNN_HIP(hipMemsetAsync(sc, 0, sizeof(Scratch), s));
  const int cap = 4 * di.cus * 8;
  k_check_finite<T><<<grid_for(k * d, kThreads, cap), kThreads, 0, s>>>(Xn, k * d, &sc->bad);
  SNN_LAUNCH_CHECK();
  launch_project<T>(Xn, k, d, ix.mu.as<double>(), ix.v.as<double>(), ukey, val, bmax, &sc->max_norm, cap, s);
  radix_sort_pairs(ix.arena, ukey, val, k, 0, 32, s);
  launch_gather<T>(Xn, k, d, dp, ix.mu.as<double>(), ukey, val, keyb, permb, pob, nullptr, ysb, hb, ynb, na, cap, s);
  Scratch hs;
  SNN_HIP(hipMemcpyAsync(&hs, sc, sizeof(Scratch), hipMemcpyDeviceToHost, s));
  SNN_HIP(hipStreamSynchronize(s));
  if (hs.bad) fail(SNN_EINVAL, "snn_index_insert: X contains NaN or Inf");

  // merged arrays
  k_merge_path<<<grid_for(nt, kThreads, 4 * di.cus * 8), kThreads, 0, s>>>(ix.key.as<double>(), na, keyb, k, src);
  SNN_LAUNCH_CHECK();
  Buffer key, perm, po, p64, ys, h, ynorm;
  // released at scope end: after the swaps below these hold the old arrays,
  // and on an error part way the new ones
  struct ReleaseAll {
    DeviceArena& a;
    std::initializer_list<Buffer*> bufs;
    ~ReleaseAll() {
      for (Buffer* b : bufs) b->reset(a);
    }
  } release_all{ix.arena, {&key, &perm, &po, &p64, &ys, &h, &ynorm}};
  key.ensure(ix.arena, sizeof(double) * nt);
  perm.ensure(ix.arena, sizeof(int32_t) * nt);
  po.ensure(ix.arena, sizeof(T) * nt * d);
  p64.ensure(ix.arena, sizeof(double) * nt * dp);
  ys.ensure(ix.arena, sizeof(float) * nt * d);
  h.ensure(ix.arena, sizeof(float) * (nt + 64));
  ynorm.ensure(ix.arena, sizeof(float) * nt);
  merge_rows<double>(ix.key.as<double>(), keyb, src, nt, 1, key.as<double>(), cap, s);
  merge_rows<int32_t>(ix.perm.as<int32_t>(), permb, src, nt, 1, perm.as<int32_t>(), cap, s);
  merge_rows<T>(ix.po.as<T>(), pob, src, nt, d, po.as<T>(), cap, s);
  // p64 of the grown index is filled by the next fp64 screen (p64_ready)
  merge_rows<float>(ix.ys.as<float>(), ysb, src, nt, d, ys.as<float>(), cap, s);
  merge_rows<float>(ix.h.as<float>(), hb, src, nt, 1, h.as<float>(), cap, s);
  merge_rows<float>(ix.ynorm.as<float>(), ynb, src, nt, 1, ynorm.as<float>(), cap, s);
  k_fill_inf<<<1, 64, 0, s>>>(h.as<float>() + nt, 64);  // padding rows
  SNN_LAUNCH_CHECK();
  SNN_HIP(hipStreamSynchronize(s));
  std::swap(ix.key, key);
  std::swap(ix.perm, perm);
  std::swap(ix.po, po);
  std::swap(ix.p64, p64);
  std::swap(ix.ys, ys);
  std::swap(ix.h, h);
  std::swap(ix.ynorm, ynorm);
  // the arrays of the build (views into one allocation) are all replaced
  if (key.view) {
    for (Buffer* b : {&key, &perm, &po, &p64, &ys, &h, &ynorm}) b->reset(ix.arena);
    ix.rows.reset(ix.arena);
  }

  // bounds over all points; screen operands are rebuilt on the next query
  const double u64 = std::ldexp(1.0, -53), u32 = std::ldexp(1.0, -24);
  ix.n = nt;
  ix.max_norm = std::max(ix.max_norm, std::sqrt(hs.max_norm) * (1.0 + 4.0 * (d + 2) * u64));
  const double g64 = (d + 2) * u64 / (1.0 - (d + 2) * u64);
  ix.key_eps = 1.01 * (u32 + g64) * (1.0 + u32) * ix.max_norm * ix.vnorm;
  for (auto& mo : ix.mixed) mo.built = false;
  ix.vcand_built = false;
  ix.p64_ready = false;
  ix.wcells_built = false;
  ++ix.epoch;
}

void insert_points(Index& ix, const void* X, int64_t k) {
  if (k == 0) return;
  if (ix.dtype == SNN_F32)
    insert_points_t<float>(ix, static_cast<const float*>(X), k);
  else
    insert_points_t<double>(ix, static_cast<const double*>(X), k);
}

void build_mixed_operands(Index& ix, int kind) {
  MixedOperands& mo = ix.mixed[mixed_slot(kind)];
  if (mo.built) return;
  const int d = ix.d;
  const int ka = kind == kOpBf16x3 ? ((3 * d + 15) / 16) * 16 : ((d + 15) / 16) * 16;
  const int kb = (kind == kOpBf16x3 && d % 16 == 0) ? 2 * d : ka;
  const int e = kind == kOpF16 ? f16_scale_exp(ix.max_norm) : 0;
  const int64_t npad = ((ix.n + 32 + 31) / 32) * 32;
  mo.cand.ensure(ix.arena, sizeof(uint16_t) * npad * kb + 256);
  mo.qself.ensure(ix.arena, sizeof(uint16_t) * ix.n * ka + 256);
  if (kind == kOpF16) mo.hs.ensure(ix.arena, sizeof(float) * npad + 256);
  const DeviceInfo& di = device_info(ix.arena.dev().device);
  k_operands<<<grid_for(npad * (ka / 4), kThreads, 4 * di.cus * 8), kThreads, 0, ix.arena.stream()>>>(
      ix.ys.as<float>(), ix.h.as<float>(), ix.n, npad, d, kind, e, ka, kb, mo.cand.as<uint16_t>(),
      mo.qself.as<uint16_t>(), kind == kOpF16 ? mo.hs.as<float>() : nullptr);
  SNN_LAUNCH_CHECK();
  mo.built = true;
  mo.ka = ka;
  mo.kb = kb;
  mo.e = e;
}

}  // namespace snn
