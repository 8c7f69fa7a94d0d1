// Small-d fp32 candidate screen on the vector ALUs.
//
// Same decomposition and rigorous pass rule as the matrix-core screen
// (eq. (ip2) of Section 4 with a widened per-query start value, see
// k_cand_mfma.hip), but the operands are the fp32 centred rows themselves,
// so the only screen error is the fp32 rounding of d fused multiply-adds:
// the band around R^2 that goes to the float64 recheck is a few ulps wide.
// For low dimensions (the particle-like d = 3 workload, R = 0.005 in the
// unit cube) a bf16 band would be several times R^2 wide.
//
// Layout: a wavefront owns 64 score-ordered queries, one per lane (y_q and
// C_q in registers); the unit's candidates are read with scalar loads
// (wavefront-uniform addresses), 8 at a time, so each candidate coordinate is
// an SGPR operand of one v_fma_f32 serving 64 pairs.  Per pair: d fused
// multiply-adds and one compare.
//   query row     [y_0 .. y_{d-1}, C_q, 0 ...]   (DV floats, DV = pad4(d + 1))
//   candidate row [y_0 .. y_{d-1}, h_j, 0 ...]   (8 extra rows, h = +inf)
#include <hip/hip_runtime.h>

#include <cmath>

#include "device_common.h"
#include "query_plan.h"
#include "snn_internal.h"

namespace snn {

namespace {

constexpr int kThreads = 256;
// per-wavefront pair stage, flushed when fewer than one batch of pushes would fit
constexpr int kWaveStage = 1024;
constexpr int kBatch = 8;

typedef const __attribute__((address_space(4))) float cfloat;

__global__ __launch_bounds__(kThreads) void k_valu_operands(const float* __restrict__ ys,
                                                           const float* __restrict__ h, int64_t n, int d, int DV,
                                                           float* __restrict__ vc) {
  const int64_t total = (n + kBatch) * DV;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = e / DV;
    const int k = (int)(e % DV);
    float v = 0.f;
    if (k == d)
      v = s < n ? h[s] : INFINITY;
    else if (k < d && s < n)
      v = ys[s * d + k];
    vc[e] = v;
  }
}

__global__ __launch_bounds__(kThreads) void k_valu_qprep(const double* __restrict__ q64, int64_t m, int d, int dp,
                                                        const double* __restrict__ mu, int DV, MixedBound b,
                                                        float* __restrict__ vq) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < m; s += (int64_t)gridDim.x * blockDim.x) {
    float* o = vq + s * DV;
    double nn = 0.0;
    for (int k = 0; k < d; ++k) {
      const float y = (float)(q64[s * dp + k] - mu[k]);
      nn += (double)y * (double)y;
      o[k] = y;
    }
    for (int k = d + 1; k < DV; ++k) o[k] = 0.f;
    o[d] = screen_threshold(b, 0.5 * nn, sqrt(nn) * (1.0 + 1e-15));
  }
}

__global__ __launch_bounds__(kThreads) void k_valu_qprep_self(const float* __restrict__ ys, int64_t n, int d, int DV,
                                                             MixedBound b, float* __restrict__ vq) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x) {
    float* o = vq + s * DV;
    double nn = 0.0;
    for (int k = 0; k < d; ++k) {
      const float y = ys[s * d + k];
      nn += (double)y * (double)y;
      o[k] = y;
    }
    for (int k = d + 1; k < DV; ++k) o[k] = 0.f;
    o[d] = screen_threshold(b, 0.5 * nn, sqrt(nn) * (1.0 + 1e-15));
  }
}

template <int D>
__global__ __launch_bounds__(kThreads) void k_cand_valu(QueryDev q, const float* __restrict__ vq,
                                                       const float* __restrict__ vc) {
  constexpr int DV = ((D + 1 + 3) / 4) * 4;
  __shared__ int2 wstage[kThreads / kWave][kWaveStage];
  __shared__ long long s_unit;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int xcd = blockIdx.x % q.nxcd;
  int2* wbuf = wstage[wave];
  int wcnt = 0;  // wave-uniform fill of wbuf
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_unit = next_unit(q, xcd);
    __syncthreads();
    const int64_t u = uniform_i64(s_unit);
    if (u < 0) break;
    int tile;
    int64_t c;
    if (!decode_unit(q, u, tile, c)) continue;
    const int64_t q0 = (int64_t)tile * q.T + (int64_t)wave * kWave;
    const int64_t j0 = q.tlo[tile] + c * q.CH;
    const int64_t j1 = min(j0 + q.CH, (int64_t)q.thi[tile]);
    if (q0 >= q.m) continue;  // no queries for this wave in the ragged last tile
    const int64_t qi = q0 + lane;
    const bool vqi = qi < q.m;
    const float* qrow = vq + (vqi ? qi : 0) * DV;
    float y[D];
#pragma unroll
    for (int k = 0; k < D; ++k) y[k] = qrow[k];
    const float cq = vqi ? qrow[D] : -INFINITY;
    // Full batches: NB candidate rows (scalar registers) per round, one
    // wave-uniform branch per round; then the ragged tail one row at a time.
    constexpr int NB = (64 / DV) < 1 ? 1 : ((64 / DV) > kBatch ? kBatch : (64 / DV));
    int64_t jb = j0;
    for (; jb + NB <= j1; jb += NB) {
      cfloat* cr = (cfloat*)(vc + jb * DV);
      float cv[NB * DV];
#pragma unroll
      for (int e = 0; e < NB * DV; ++e) cv[e] = cr[e];
      // the compare of each candidate is a lane mask in scalar registers
      uint64_t mk[NB];
      uint64_t any = 0;
#pragma unroll
      for (int cc = 0; cc < NB; ++cc) {
        float acc = cq;
#pragma unroll
        for (int k = 0; k < D; ++k) acc = fmaf(y[k], cv[cc * DV + k], acc);
        mk[cc] = __ballot(acc >= cv[cc * DV + D]);
        any |= mk[cc];
      }
      if (any) {
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) wave_push(wbuf, wcnt, (mk[cc] >> lane) & 1ull, (int)qi, (int)(jb + cc));
        if (wcnt > kWaveStage - NB * kWave) wave_flush(wbuf, wcnt, q.sink);
      }
    }
    for (; jb < j1; ++jb) {
      cfloat* cr = (cfloat*)(vc + jb * DV);
      float acc = cq;
#pragma unroll
      for (int k = 0; k < D; ++k) acc = fmaf(y[k], cr[k], acc);
      wave_push(wbuf, wcnt, acc >= cr[D], (int)qi, (int)jb);
      if (wcnt > kWaveStage - kWave) wave_flush(wbuf, wcnt, q.sink);
    }
  }
  wave_flush(wbuf, wcnt, q.sink);
}

typedef void (*ValuKernel)(QueryDev, const float*, const float*);

ValuKernel pick(int d) {
  switch (d) {
    case 1: return k_cand_valu<1>;
    case 2: return k_cand_valu<2>;
    case 3: return k_cand_valu<3>;
    case 4: return k_cand_valu<4>;
    case 5: return k_cand_valu<5>;
    case 6: return k_cand_valu<6>;
    case 7: return k_cand_valu<7>;
    case 8: return k_cand_valu<8>;
    case 9: return k_cand_valu<9>;
    case 10: return k_cand_valu<10>;
    case 11: return k_cand_valu<11>;
    case 12: return k_cand_valu<12>;
    case 13: return k_cand_valu<13>;
    case 14: return k_cand_valu<14>;
    case 15: return k_cand_valu<15>;
    case 16: return k_cand_valu<16>;
    default: return nullptr;
  }
}

int grid_for(int64_t work, int cap) {
  int64_t g = (work + kThreads - 1) / kThreads;
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

int valu_max_d() { return 16; }
int valu_row_floats(int d) { return ((d + 1 + 3) / 4) * 4; }
int valu_queries_per_tile() { return kThreads; }

int valu_blocks_per_cu(int d) {
  ValuKernel k = pick(d);
  int nb = 0;
  if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kThreads, 0) != hipSuccess || nb < 1) {
    (void)hipGetLastError();
    nb = 1;
  }
  return nb;
}

void launch_valu_operands(const float* ys, const float* h, int64_t n, int d, float* vc, hipStream_t s) {
  const int DV = valu_row_floats(d);
  k_valu_operands<<<grid_for((n + kBatch) * DV, 16384), kThreads, 0, s>>>(ys, h, n, d, DV, vc);
  SNN_LAUNCH_CHECK();
}

void launch_valu_qprep(const double* q64, int64_t m, int d, int dp, const double* mu, const MixedBound& b, float* vq,
                       hipStream_t s) {
  if (m <= 0) return;
  k_valu_qprep<<<grid_for(m, 8192), kThreads, 0, s>>>(q64, m, d, dp, mu, valu_row_floats(d), b, vq);
  SNN_LAUNCH_CHECK();
}

void launch_valu_qprep_self(const float* ys, int64_t n, int d, const MixedBound& b, float* vq, hipStream_t s) {
  k_valu_qprep_self<<<grid_for(n, 8192), kThreads, 0, s>>>(ys, n, d, valu_row_floats(d), b, vq);
  SNN_LAUNCH_CHECK();
}

void launch_cand_valu(const QueryDev& q, const float* vq, const float* vc, int grid, hipStream_t s) {
  ValuKernel k = pick(q.d);
  if (!k) fail(SNN_ENOTSUP, "fp32 vector screen supports d <= 16");
  k<<<grid, kThreads, 0, s>>>(q, vq, vc);
  SNN_LAUNCH_CHECK();
}

}  // namespace snn
