// Plain float64 candidate screen: every (query, window candidate) pair is
// decided by the normative rule S(p_j, q) <= fl(R*R), with S the direct
// form of eq. (ip1) summed left to right without fused multiply-add
// (Section 4).  This is the exact reference kernel the mixed-precision
// screen is measured against.
//
// Layout: a workgroup takes one work unit (a tile of T score-ordered queries
// x up to CH window candidates).  Each lane holds one candidate row in
// float64 registers; the tile's query rows are read through the constant
// address space with a wavefront-uniform address, i.e. with scalar loads,
// so each query coordinate is one SGPR operand shared by the 64 lanes.
// Rows are zero-padded to DP coordinates: the padded terms add
// (0 - 0)^2 = +0 to a non-negative partial sum, which leaves it unchanged,
// so the loop needs no per-coordinate branch.  Cost per pair: d
// subtractions, d multiplications, d - 1 additions and one compare.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "query_plan.h"
#include "snn_internal.h"

#pragma clang fp contract(off)

namespace snn {

namespace {

constexpr int kThreads = 256;
constexpr int kStage = 2048;

typedef const __attribute__((address_space(4))) double cdouble;

template <int DP>
__global__ __launch_bounds__(kThreads) void k_cand_fp64_reg(QueryDev q) {
  __shared__ PairStage<kStage> st;
  __shared__ long long s_unit;
  stage_init(st);
  mark_begin(q);
  const int xcd = blockIdx.x % q.nxcd;
  for (;;) {
    __syncthreads();
    stage_drain(st, q.sink);
    if (threadIdx.x == 0) s_unit = next_unit(q, xcd);
    __syncthreads();
    const int64_t u = uniform_i64(s_unit);
    if (u < 0) break;
    int tile;
    int64_t j0, j1;
    if (!decode_unit(q, u, tile, j0, j1)) continue;
    const int64_t q0 = (int64_t)tile * q.T;
    const int qn = (int)min((int64_t)q.T, q.m - q0);
    for (int64_t jb = j0; jb < j1; jb += kThreads) {
      const int64_t jr = jb + threadIdx.x;
      const bool valid = jr < j1;
      const int64_t j = valid ? jr : j1 - 1;
      double p[DP];
      const double* pr = q.p64 + j * DP;
#pragma unroll
      for (int k = 0; k < DP; ++k) p[k] = pr[k];
      cdouble* qr = (cdouble*)(q.q64 + q0 * DP);
      for (int sq = 0; sq < qn; ++sq, qr += DP) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < DP; ++k) {
          const double t = p[k] - qr[k];
          s = s + t * t;
        }
        stage_push_wave(st, q.sink, valid && s <= q.R2, (int)(q0 + sq), (int)j);
      }
    }
  }
  stage_flush(st, q.sink);
  mark_end(q);
}

// Large d: the candidate is streamed in chunks of 16 coordinates while the
// partial sums of a group of 16 queries stay in registers, so the
// left-to-right order of each sum is kept.
__global__ __launch_bounds__(kThreads) void k_cand_fp64_big(QueryDev q, int dp) {
  constexpr int QG = 16, KC = 16;
  __shared__ PairStage<kStage> st;
  __shared__ long long s_unit;
  stage_init(st);
  mark_begin(q);
  const int xcd = blockIdx.x % q.nxcd;
  for (;;) {
    __syncthreads();
    stage_drain(st, q.sink);
    if (threadIdx.x == 0) s_unit = next_unit(q, xcd);
    __syncthreads();
    const int64_t u = uniform_i64(s_unit);
    if (u < 0) break;
    int tile;
    int64_t j0, j1;
    if (!decode_unit(q, u, tile, j0, j1)) continue;
    const int64_t q0 = (int64_t)tile * q.T;
    const int qn = (int)min((int64_t)q.T, q.m - q0);
    for (int64_t jb = j0; jb < j1; jb += kThreads) {
      const int64_t jr = jb + threadIdx.x;
      const bool valid = jr < j1;
      const int64_t j = valid ? jr : j1 - 1;
      const double* pr = q.p64 + j * dp;
      for (int g0 = 0; g0 < qn; g0 += QG) {
        double s[QG];
#pragma unroll
        for (int i = 0; i < QG; ++i) s[i] = 0.0;
        for (int k0 = 0; k0 < dp; k0 += KC) {
          double p[KC];
#pragma unroll
          for (int k = 0; k < KC; ++k) p[k] = (k0 + k < dp) ? pr[k0 + k] : 0.0;
#pragma unroll
          for (int i = 0; i < QG; ++i) {
            if (g0 + i < qn) {
              cdouble* qr = (cdouble*)(q.q64 + (q0 + g0 + i) * dp + k0);
#pragma unroll
              for (int k = 0; k < KC; ++k) {
                if (k0 + k < dp) {
                  const double t = p[k] - qr[k];
                  s[i] = s[i] + t * t;
                }
              }
            }
          }
        }
#pragma unroll
        for (int i = 0; i < QG; ++i) {
          if (g0 + i < qn) stage_push_wave(st, q.sink, valid && s[i] <= q.R2, (int)(q0 + g0 + i), (int)j);
        }
      }
    }
  }
  stage_flush(st, q.sink);
  mark_end(q);
}

}  // namespace

int fp64_blocks_per_cu(int dp) {
  int nb = 0;
  hipError_t e;
  switch (dp) {
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_cand_fp64_reg<4>, kThreads, 0); break;
    case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_cand_fp64_reg<8>, kThreads, 0); break;
    case 12: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_cand_fp64_reg<12>, kThreads, 0); break;
    case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_cand_fp64_reg<16>, kThreads, 0); break;
    case 20: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_cand_fp64_reg<20>, kThreads, 0); break;
    case 24: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_cand_fp64_reg<24>, kThreads, 0); break;
    case 28: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_cand_fp64_reg<28>, kThreads, 0); break;
    case 32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_cand_fp64_reg<32>, kThreads, 0); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_cand_fp64_big, kThreads, 0); break;
  }
  if (e != hipSuccess || nb < 1) {
    (void)hipGetLastError();
    nb = 1;
  }
  return nb;
}

void launch_cand_fp64(const QueryDev& q, int grid, hipStream_t s) {
  switch (q.dp) {
    case 4: k_cand_fp64_reg<4><<<grid, kThreads, 0, s>>>(q); break;
    case 8: k_cand_fp64_reg<8><<<grid, kThreads, 0, s>>>(q); break;
    case 12: k_cand_fp64_reg<12><<<grid, kThreads, 0, s>>>(q); break;
    case 16: k_cand_fp64_reg<16><<<grid, kThreads, 0, s>>>(q); break;
    case 20: k_cand_fp64_reg<20><<<grid, kThreads, 0, s>>>(q); break;
    case 24: k_cand_fp64_reg<24><<<grid, kThreads, 0, s>>>(q); break;
    case 28: k_cand_fp64_reg<28><<<grid, kThreads, 0, s>>>(q); break;
    case 32: k_cand_fp64_reg<32><<<grid, kThreads, 0, s>>>(q); break;
    default: k_cand_fp64_big<<<grid, kThreads, 0, s>>>(q, q.dp); break;
  }
  SNN_LAUNCH_CHECK();
}

}  // namespace snn
