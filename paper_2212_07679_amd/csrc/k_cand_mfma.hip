// Mixed-precision candidate screen on the gfx950 matrix cores (the
// "precision form").
//
// Section 4 rewrites the radius test ||x_j - x_q||^2 <= R^2 as eq. (ip2),
//     xbar_j - x_j^T x_q <= (R^2 - x_q^T x_q) / 2,
// so a block of score-adjacent queries against a block of window candidates
// is one small matrix product (the gemm over the union window).  Here that
// product runs as v_mfma_f32_32x32x16_bf16: bf16 operands, fp32 accumulation.
// The screen never decides a pair by itself: it only REJECTS pairs it can
// prove to be outside the radius, using a rigorous bound on everything the
// bf16/fp32 evaluation can get wrong; every other pair goes to the float64
// recheck (normative rule), so the result is exact.
//
// With y = fl32(p - mu) (centred rows), h_j = ||y_j||^2 / 2 and a per-query
// constant C_q, the screen passes (q, j) iff
//     D = fl_mfma( sum_k a_qk b_jk + C_q )  >=  fl32(h_j),
// where the packed operands satisfy sum_k a_qk b_jk ~ y_q . y_j:
//   bf16, one term:  a = bf16(y_q),              b = bf16(y_j)
//   bf16, 3 terms:   a = [hi_q, hi_q, lo_q],     b = [hi_j, lo_j, hi_j]
//                    hi = bf16(y), lo = bf16(y - hi)   (hi*hi + hi*lo + lo*hi)
//   fp16:            a = fp16(s y_q),            b = fp16(s y_j),  s = 2^e
//                    (v_mfma_f32_32x32x16_f16; the accumulator, C_q and h_j
//                    are then in units scaled by s^2, which is exact)
// C_q is chosen (k_query_gather, k_mixed_qprep_self) so that every pair with S(p_j, q) <= fl(R*R)
// passes:
//   C_q >= R2'/2 - h_q + eta sqrt(R2') + eta^2/2 + e_rep + e_acc + e_h
//   R2'   = fl(R*R) (1 + 2 gamma64_{d+2})   bounds the exact ||p - q||^2
//   eta   = 1.01 u32 (Y + ||y_q||)          centring rounding, Y = max_j ||y_j||
//   e_rep = c_rep Y ||y_q|| + e_sub         operand representation error
//           c_rep = u_b (2 + u_b) (bf16), u_b^2 (3 + 3 u_b) (bf16 x3), u_b = 2^-8,
//                   u_h (2 + u_h) (fp16), u_h = 2^-11
//           e_sub = (1 + u) t sqrt(K) delta (||y_q|| + Y) + t K delta^2: an operand
//                   below the normal range is off by at most delta (its format's
//                   smallest normal, fp16: 2^-14 / s) whether it is kept subnormal
//                   or read as zero (t operand values per coordinate)
//   e_acc = 2 gamma32_{K+1} (1.02 Y ||y_q|| + |C_q|)  fp32 accumulation of the
//           K exact bf16 products and C (factor 2: the accumulation order and
//           rounding inside the matrix core are not specified)
//   e_h   = 1.01 u32 Y^2 / 2                rounding of h_j to fp32
// and rounded up to fp32.
//
// Data layout.  Candidates and queries are rows of KA bf16 (KA a multiple
// of 16) in score order.  A wavefront owns QB blocks of 32 queries (the A
// operand, loaded once per work unit) and sweeps the unit's candidates 32
// at a time (the B operand: lane l loads 16 contiguous bytes of candidate
// l % 32, so a step reads 32 consecutive rows).  The accumulator of the
// 32x32 block starts at C_q (each lane's 16 accumulators belong to 16
// queries and one candidate), so the epilogue is a max over the lane's 16
// values and one compare with h_j; only when some lane passes does the
// wave walk its accumulators and append (query, candidate) pairs.
#include <hip/hip_runtime.h>

#include <cmath>

#include "device_common.h"
#include "query_plan.h"
#include "snn_internal.h"

namespace snn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// The 16-bit operand format of a screen: its vector type and its 32x32x16
// matrix instruction (same operand layout for both).
template <bool F16>
struct Op16;
template <>
struct Op16<false> {
  typedef bf16x8 V;
  static __device__ __forceinline__ f32x16 mfma(V a, V b, const f32x16& c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Op16<true> {
  typedef f16x8 V;
  static __device__ __forceinline__ f32x16 mfma(V a, V b, const f32x16& c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

// fp16 bits of x (round to nearest even, subnormals kept: the kernels run
// with fp16 denormals enabled)
__device__ __forceinline__ uint16_t f32_to_f16_bits(float x) { return __builtin_bit_cast(uint16_t, (_Float16)x); }

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;
// Per-wavefront pair stages (entries): flushed when fewer than one query
// block's worth of pushes (16 x 64) would fit.  The 16-bit screens keep theirs
// small enough for four workgroups (four waves per SIMD) per CU; the fp32
// screen, whose dense outputs push much more, keeps a larger one (measured on
// the n = 1e6, d = 16 set: 0.420 ms with 1264 entries against 0.422 ms with
// 1536 at two steps of prefetch, 0.442 against 0.480 ms at one).
#ifndef SNN_WAVE_STAGE
#define SNN_WAVE_STAGE 1264
#endif
constexpr int kWaveStage16 = SNN_WAVE_STAGE;
constexpr int kWaveStage32 = 1536;
// candidate steps whose operands are in flight ahead of the one being
// screened in the 16-bit screens (same set: 0.422 ms with two or three,
// 0.480 ms with one)
#ifndef SNN_SCREEN_PREFETCH
#define SNN_SCREEN_PREFETCH 2
#endif
constexpr int kPrefetch = SNN_SCREEN_PREFETCH;

// Self-queries: the query rows are the index rows; G lanes read a row
// together and their partial squared norms meet by shuffles (any order stays
// within the gamma_{d+1} bound the start value allows for).
template <int G>
__global__ __launch_bounds__(kThreads) void k_mixed_qprep_self(const float* __restrict__ ys, int64_t n, int d,
                                                              MixedBound b, float* __restrict__ cthr) {
  const int sub = threadIdx.x % G;
  for (int64_t s = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G; s < n;
       s += ((int64_t)gridDim.x * blockDim.x) / G) {
    const float* y = ys + s * d;
    double nn = 0.0;
    for (int k = sub; k < d; k += G) nn += (double)y[k] * (double)y[k];
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) nn += __shfl_xor(nn, off, G);
    if (sub == 0) cthr[s] = screen_threshold(b, 0.5 * nn, sqrt(nn) * (1.0 + 1e-15));
  }
}

__device__ __forceinline__ float max16(const f32x16& a) {
  float m0 = fmaxf(fmaxf(a[0], a[1]), a[2]);
  float m1 = fmaxf(fmaxf(a[3], a[4]), a[5]);
  float m2 = fmaxf(fmaxf(a[6], a[7]), a[8]);
  float m3 = fmaxf(fmaxf(a[9], a[10]), a[11]);
  float m4 = fmaxf(fmaxf(a[12], a[13]), a[14]);
  m0 = fmaxf(fmaxf(m0, m1), m2);
  m3 = fmaxf(fmaxf(m3, m4), a[15]);
  return fmaxf(m0, m3);
}

// max of m and the 16 values of a (eight 3-input maxima)
__device__ __forceinline__ float max16_into(float m, const f32x16& a) {
  float m0 = fmaxf(fmaxf(m, a[0]), a[1]);
  float m1 = fmaxf(fmaxf(a[2], a[3]), a[4]);
  float m2 = fmaxf(fmaxf(a[5], a[6]), a[7]);
  float m3 = fmaxf(fmaxf(a[8], a[9]), a[10]);
  float m4 = fmaxf(fmaxf(a[11], a[12]), a[13]);
  m0 = fmaxf(fmaxf(m0, m1), m2);
  m3 = fmaxf(fmaxf(m3, m4), a[14]);
  return fmaxf(fmaxf(m0, m3), a[15]);
}

// max over the QB blocks of a lane's accumulators
template <int QB>
__device__ __forceinline__ float max_blocks(const f32x16 (&acc)[QB]) {
  float m = max16(acc[0]);
#pragma unroll
  for (int b = 1; b < QB; ++b) m = max16_into(m, acc[b]);
  return m;
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kRsrcWord3 = 0x00020000;  // raw buffer, 32-bit data format

// Operands of step `it` through buffer resources whose base is the unit's
// first 32-row block: the lane offset is fixed and the step offset is a
// scalar, so no per-step vector address arithmetic exists.  Reads past the
// unit (the look-ahead of the last step) are outside num_records and return
// zeros without touching memory.
template <int NL, typename V>
__device__ __forceinline__ void load_cand(V (&B)[NL], __amdgpu_buffer_rsrc_t rc, int voff_c, int it) {
#pragma unroll
  for (int s = 0; s < NL; ++s)  // slices are 1 KB apart in a 32-row block
    B[s] = __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(rc, voff_c, it * (NL * 1024) + s * 1024, 0));
}
__device__ __forceinline__ float load_h(__amdgpu_buffer_rsrc_t rh, int voff_h, int it) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rh, voff_h, it * 128, 0));
}
template <int NL, typename V>
__device__ __forceinline__ void load_step(V (&B)[NL], float& h, __amdgpu_buffer_rsrc_t rc,
                                          __amdgpu_buffer_rsrc_t rh, int voff_c, int voff_h, int it) {
  load_cand<NL>(B, rc, voff_c, it);
  h = load_h(rh, voff_h, it);
}

// The max/compare epilogue of one step: acc[b] is the 32x32 block of query
// block b against the step's 32 candidates (lane l: candidate l % 32;
// accumulator r: query 8 (r / 4) + 4 (l / 32) + r % 4 of the block).
// Two ways of collecting the passing pairs of a block with a passing lane:
// ROWS: one wave-wide compare per accumulator row r (16 scalar masks), and a
//       push for each row with passing lanes (cheaper when a block holds
//       few passes, as with the short fp32 chains);
// else: each lane packs its passing accumulators into a bit mask and the
//       wave pushes one pair per lane per round (cheaper when passes are
//       many, as in dense bf16 outputs: measured on one box, 1.25 vs 1.51 ms
//       for the 256-instance batch, 21 vs 17 ms for the d = 3 particles).
// The common case is one max over all the lane's accumulators and one
// compare; blocks are told apart only when some lane passes.
template <int QB, bool ROWS, int STAGE>
__device__ __forceinline__ void screen_pushes(const f32x16 (&acc)[QB], float hj, int jj, int64_t q0, int half,
                                              int2* wbuf, int& wcnt, const PairSink& sink) {
  uint64_t pm[QB];  // wave masks: lanes with a passing accumulator in block b
#pragma unroll
  for (int b = 0; b < QB; ++b) pm[b] = QB == 1 ? ~0ull : __ballot(max16(acc[b]) >= hj);
  // uncommon: push the passing pairs of each block with a passing lane into
  // the wavefront's LDS stage (at most 16 x 64 per block).  The row base is
  // made opaque per step so that the 16 QB row offsets are not hoisted out of
  // the step loop into registers.
  int qb = (int)q0 + 4 * half;
  asm volatile("" : "+v"(qb));
#pragma unroll
  for (int b = 0; b < QB; ++b) {
    if (!pm[b]) continue;
    if (ROWS) {
#pragma unroll
      for (int r = 0; r < 16; ++r) wave_push(wbuf, wcnt, acc[b][r] >= hj, qb + b * 32 + 8 * (r >> 2) + (r & 3), jj);
    } else {
      uint32_t bits = 0;
#pragma unroll
      for (int r = 0; r < 16; ++r) bits |= (acc[b][r] >= hj ? 1u : 0u) << r;
      while (__ballot(bits != 0)) {
        const bool p = bits != 0;
        const int r = p ? __ffs(bits) - 1 : 0;
        bits &= bits - 1;
        wave_push(wbuf, wcnt, p, qb + b * 32 + 8 * (r >> 2) + (r & 3), jj);
      }
    }
    if (wcnt > STAGE - 16 * kWave) wave_flush(wbuf, wcnt, sink);
  }
}

template <int QB, bool ROWS, int STAGE>
__device__ __forceinline__ void screen_epilogue(const f32x16 (&acc)[QB], float hj, int jj, int64_t q0, int half,
                                                int2* wbuf, int& wcnt, const PairSink& sink) {
  if (!__ballot(max_blocks<QB>(acc) >= hj)) return;
  screen_pushes<QB, ROWS, STAGE>(acc, hj, jj, q0, half, wbuf, wcnt, sink);
}

// The products of one 32-candidate step for QB blocks of 32 queries.
// Operand slice s of the candidate is B[s] for s < NL and B[s - NL] beyond
// (the split layout repeats hi as the third segment).
template <bool F16, int NS, int QB, int NL>
__device__ __forceinline__ void step_products(const typename Op16<F16>::V (&A)[QB][NS], const f32x16 (&Cin)[QB],
                                              const typename Op16<F16>::V (&B)[NL], f32x16 (&acc)[QB]) {
#pragma unroll
  for (int b = 0; b < QB; ++b) acc[b] = Op16<F16>::mfma(A[b][0], B[0], Cin[b]);
#pragma unroll
  for (int s = 1; s < NS; ++s)
#pragma unroll
    for (int b = 0; b < QB; ++b) acc[b] = Op16<F16>::mfma(A[b][s], B[s < NL ? s : s - NL], acc[b]);
}

// One 32-candidate step of a 16-bit screen on operand set (B, h): products,
// the next load into the set (PF steps ahead; reads past the unit return
// zeros), one max over the lane's accumulators and one compare.  Only the
// last step of a unit can have lanes past its span (units are cut at
// multiples of 32 rows except at the end of the index), so only it masks.
// (Loading the block together with h after the compare keeps the compiler's
// load-count waits exact but starts the block's load a compare later: 0.385
// against 0.378 ms on the n = 1e6, d = 16 set.)
template <bool F16, int NS, int QB, int NL, int PF, bool LAST>
__device__ __forceinline__ void mixed_step(const typename Op16<F16>::V (&A)[QB][NS], const f32x16 (&Cin)[QB],
                                           typename Op16<F16>::V (&B)[NL], float& h, __amdgpu_buffer_rsrc_t rc,
                                           __amdgpu_buffer_rsrc_t rh, int voff_c, int voff_h, int it, int span,
                                           int l32, int j0, int64_t q0, int half, int2* wbuf, int& wcnt,
                                           const PairSink& sink) {
  f32x16 acc[QB];
  step_products<F16, NS, QB, NL>(A, Cin, B, acc);
  if (!LAST) load_cand<NL>(B, rc, voff_c, it + PF);
  float hj = h;
  if (LAST && it * 32 + l32 >= span) hj = INFINITY;
  if (__ballot(max_blocks<QB>(acc) >= hj))
    screen_pushes<QB, false, kWaveStage16>(acc, hj, j0 + it * 32 + l32, q0, half, wbuf, wcnt, sink);
  // the set's next h goes into the register the compare just read: the load
  // stays after every use of hj (hoisted above one, it would need a second
  // register and a copy that waits for the load at the end of every step)
  __builtin_amdgcn_sched_barrier(0);
  if (!LAST) h = load_h(rh, voff_h, it + PF);
}

// Query operands of one wavefront: QB blocks of 32 rows of NS slices (lane
// l: row l % 32, 8 values at 8 (l / 32) of each 16-value slice) and the
// blocks' start values in accumulator order; rows past m are zero / -inf.
template <bool F16, int NS, int QB>
__device__ __forceinline__ void load_queries(const MixedDev& x, int64_t m, int64_t q0, int l32, int half,
                                             typename Op16<F16>::V (&A)[QB][NS], f32x16 (&Cin)[QB]) {
  typedef typename Op16<F16>::V V;
#pragma unroll
  for (int b = 0; b < QB; ++b) {
    const int64_t qr = q0 + b * 32 + l32;
    const bool vq = qr < m;
    const V* src = reinterpret_cast<const V*>(x.qop + (vq ? qr : 0) * x.KA + 8 * half);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      V v = src[2 * s];
      if (!vq) v = V{};
      A[b][s] = v;
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t qi = q0 + b * 32 + 8 * (r / 4) + 4 * half + (r % 4);
      Cin[b][r] = qi < m ? x.cthr[qi] : -INFINITY;
    }
  }
}

template <bool F16, int NS, int QB, int NL>
__global__ __launch_bounds__(kThreads) void k_cand_mfma(QueryDev q, MixedDev x) {
  typedef typename Op16<F16>::V V;
  __shared__ int2 wstage[kWaves][kWaveStage16];
  __shared__ long long s_unit;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int l32 = lane & 31, half = lane >> 5;
  const int xcd = blockIdx.x % q.nxcd;
  int2* wbuf = wstage[wave];
  int wcnt = 0;  // wave-uniform fill of wbuf
  mark_begin(q);
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_unit = next_unit(q, xcd);
    __syncthreads();
    const int64_t u = uniform_i64(s_unit);
    if (u < 0) break;
    int tile;
    int64_t j0, j1;
    if (!decode_unit(q, u, tile, j0, j1)) continue;
    const int64_t q0 = (int64_t)tile * q.T + (int64_t)wave * 32 * QB;
    if (q0 >= q.m) continue;  // this wave has no queries in the (ragged) last tile
    // padding query slots (start value -inf) only occur after the real
    // queries of a tile: a wave whose first slot is padding has no work
    if (x.cthr[q0] == -INFINITY) continue;

    V A[QB][NS];
    f32x16 Cin[QB];
    load_queries<F16, NS, QB>(x, q.m, q0, l32, half, A, Cin);

    // Candidate rows j0 + 32*it + l32 (for the split layout a row is
    // [hi | lo] and the third operand slice reuses hi).  j0 is a multiple of
    // 32 (tile windows are aligned), so step `it` is one 32-row block of the
    // operand array and lane l reads 16 bytes at l * 16 of each 1 KB slice.
    // Lanes past j1 are masked by h = +inf.  Two register sets alternate, so
    // the next step's operands load while this step's products run.
    const int span = (int)(j1 - j0);
    const int nsteps = (span + 31) / 32;
    const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(reinterpret_cast<const char*>(x.cop) + (j0 / 32) * (NL * 1024)), (short)0, nsteps * NL * 1024,
        kRsrcWord3);
    const __amdgpu_buffer_rsrc_t rh =
        __builtin_amdgcn_make_buffer_rsrc((void*)(x.h + j0), (short)0, nsteps * 128, kRsrcWord3);
    const int voff_c = lane * 16, voff_h = l32 * 4;
    // kPrefetch register sets of operands rotate: step it uses set it % PF,
    // whose next load (step it + PF) is issued as soon as the step's matrix
    // instructions have read it; the candidate's h is read once the step's
    // compare has used it.
    constexpr int PF = kPrefetch;
    V Bs[PF][NL];
    float hs[PF];
#pragma unroll
    for (int p = 0; p < PF; ++p) load_step<NL>(Bs[p], hs[p], rc, rh, voff_c, voff_h, p);
    const int last = nsteps - 1;
    // whole rounds of PF steps (no exit inside a round, which keeps the
    // compiler's load-count waits at the depth the ring gives), the rest of
    // the steps before the last, then the last step
    int it0 = 0;
    for (; it0 + PF <= last; it0 += PF) {
#pragma unroll
      for (int p = 0; p < PF; ++p)
        mixed_step<F16, NS, QB, NL, PF, false>(A, Cin, Bs[p], hs[p], rc, rh, voff_c, voff_h, it0 + p, span, l32,
                                               (int)j0, q0, half, wbuf, wcnt, q.sink);
    }
#pragma unroll
    for (int p = 0; p < PF - 1; ++p)
      if (it0 + p < last)
        mixed_step<F16, NS, QB, NL, PF, false>(A, Cin, Bs[p], hs[p], rc, rh, voff_c, voff_h, it0 + p, span, l32,
                                               (int)j0, q0, half, wbuf, wcnt, q.sink);
#pragma unroll
    for (int p = 0; p < PF; ++p)
      if (last % PF == p)
        mixed_step<F16, NS, QB, NL, PF, true>(A, Cin, Bs[p], hs[p], rc, rh, voff_c, voff_h, last, span, l32, (int)j0,
                                              q0, half, wbuf, wcnt, q.sink);
  }
  wave_flush(wbuf, wcnt, q.sink);
  mark_end(q);
}

// ---- fp32 operands ------------------------------------------------------------
// The same screen with v_mfma_f32_32x32x2_f32: the operands are the fp32
// centred rows themselves (no representation error, c_rep = 0), so the only
// screen error is the fp32 rounding of the product chain and the band that
// goes to the float64 recheck is a few ulps wide (a bf16 band would be several
// times R^2 wide for low-dimensional particle data), while the compare
// epilogue is amortised over 32 x 32 blocks.  K = 2 NK coordinates (zero padded).
// Candidate operands: blocks of 32 rows, NK slices of two coordinates, a
// slice being 64 floats [k][row], so lane l = 32 k + row reads float l.  The
// query rows are [y, C_q, 0 ...] of stride DV (k_query_gather, k_mfma32_qprep_self).
// Query operands of one wavefront for the fp32 screen: QB blocks of 32 rows,
// lane l holding coordinate 2 s + l / 32 of row l % 32 in slice s, and the
// start values C_q in accumulator order; rows past m are zero / -inf.
template <int NK, int QB>
__device__ __forceinline__ void load_queries32(const Mfma32Dev& x, int64_t m, int64_t q0, int l32, int half,
                                               float (&A)[QB][NK], f32x16 (&Cin)[QB]) {
#pragma unroll
  for (int b = 0; b < QB; ++b) {
    const int64_t qr = q0 + b * 32 + l32;
    const bool vq = qr < m;
    const float* row = x.vq + (vq ? qr : 0) * x.DV;
#pragma unroll
    for (int s = 0; s < NK; ++s) {
      const int k = 2 * s + half;
      A[b][s] = (vq && k < x.d) ? row[k] : 0.f;
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t qi = q0 + b * 32 + 8 * (r / 4) + 4 * half + (r % 4);
      Cin[b][r] = qi < m ? x.vq[qi * x.DV + x.d] : -INFINITY;
    }
  }
}

// The fp32 product chain of one 32-candidate step for QB query blocks.
template <int NK, int QB>
__device__ __forceinline__ void step_products32(const float (&A)[QB][NK], const f32x16 (&Cin)[QB],
                                                const float (&B)[NK], f32x16 (&acc)[QB]) {
#pragma unroll
  for (int b = 0; b < QB; ++b) acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(A[b][0], B[0], Cin[b], 0, 0, 0);
#pragma unroll
  for (int s = 1; s < NK; ++s)
#pragma unroll
    for (int b = 0; b < QB; ++b) acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(A[b][s], B[s], acc[b], 0, 0, 0);
}

template <int NK, int QB>
__global__ __launch_bounds__(kThreads) void k_cand_mfma32(QueryDev q, Mfma32Dev x) {
  __shared__ int2 wstage[kWaves][kWaveStage32];
  __shared__ long long s_unit;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int l32 = lane & 31, half = lane >> 5;
  const int xcd = blockIdx.x % q.nxcd;
  int2* wbuf = wstage[wave];
  int wcnt = 0;  // wave-uniform fill of wbuf
  mark_begin(q);
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_unit = next_unit(q, xcd);
    __syncthreads();
    const int64_t u = uniform_i64(s_unit);
    if (u < 0) break;
    int tile;
    int64_t j0, j1;
    if (!decode_unit(q, u, tile, j0, j1)) continue;
    const int64_t q0 = (int64_t)tile * q.T + (int64_t)wave * 32 * QB;
    if (q0 >= q.m) continue;  // this wave has no queries in the (ragged) last tile

    float A[QB][NK];
    f32x16 Cin[QB];
    load_queries32<NK, QB>(x, q.m, q0, l32, half, A, Cin);

    // Step `it` covers candidates j0 + 32 it + l32 (j0 is a multiple of 32):
    // NK slices of 256 bytes through a buffer resource whose reads past the
    // unit return zeros; lanes past j1 are masked by h = +inf.  Two register
    // sets alternate so the next step's operands load during this step.
    const int span = (int)(j1 - j0);
    const int nsteps = (span + 31) / 32;
    const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(x.cop + (j0 / 32) * (NK * 64)), (short)0, nsteps * NK * 256, kRsrcWord3);
    const __amdgpu_buffer_rsrc_t rh =
        __builtin_amdgcn_make_buffer_rsrc((void*)(x.h + j0), (short)0, nsteps * 128, kRsrcWord3);
    const int voff_c = lane * 4, voff_h = l32 * 4;
    float B0[NK], B1[NK];
    float h0, h1;
    auto load = [&](float (&B)[NK], float& h, int it) {
#pragma unroll
      for (int s = 0; s < NK; ++s)
        B[s] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rc, voff_c, it * (NK * 256) + s * 256, 0));
      h = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rh, voff_h, it * 128, 0));
    };
    auto step = [&](const float (&B)[NK], float hv, int it) {
      const int jr = it * 32 + l32;
      const float hj = jr < span ? hv : INFINITY;
      f32x16 acc[QB];
      step_products32<NK, QB>(A, Cin, B, acc);
      screen_epilogue<QB, true, kWaveStage32>(acc, hj, (int)j0 + jr, q0, half, wbuf, wcnt, q.sink);
    };
    load(B0, h0, 0);
    for (int it = 0; it < nsteps; it += 2) {
      load(B1, h1, it + 1);
      step(B0, h0, it);
      if (it + 1 >= nsteps) break;
      load(B0, h0, it + 2);
      step(B1, h1, it + 1);
    }
  }
  wave_flush(wbuf, wcnt, q.sink);
  mark_end(q);
}

__global__ __launch_bounds__(kThreads) void k_mfma32_operands(const float* __restrict__ ys, int64_t n, int64_t npad,
                                                             int d, int NK, float* __restrict__ cop) {
  const int64_t total = npad * NK * 2;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t blk = e / (NK * 64);
    const int s = (int)((e / 64) % NK), w = (int)(e % 64);
    const int64_t row = blk * 32 + (w % 32);
    const int k = 2 * s + w / 32;
    cop[e] = (row < n && k < d) ? ys[row * d + k] : 0.f;
  }
}

// Query rows of the fp32 screen for a self-query: [y_0 .. y_{d-1}, C_q, 0 ...]
// with stride pad4(d + 1); C_q is the rigorous start value for the fp32
// product chain (out-of-sample queries get theirs in k_query_gather).
__global__ __launch_bounds__(kThreads) void k_mfma32_qprep_self(const float* __restrict__ ys, int64_t n, int d, int DV,
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

// ---- screen values of every pair (test support) ------------------------------
// One wavefront per (32-query block, 32-candidate block) of a small query:
// the operand loads and the product chain of the screens above, with the
// accumulators written out instead of compared.  D[qorig[q] n + j] for
// score-order queries q < m and candidates j < n.
template <bool F16, int NS, int NL>
__global__ __launch_bounds__(kWave) void k_dump_mixed(MixedDev x, int64_t m, int64_t n,
                                                     const int32_t* __restrict__ qorig, float* __restrict__ D) {
  typedef typename Op16<F16>::V V;
  const int lane = threadIdx.x, l32 = lane & 31, half = lane >> 5;
  const int64_t q0 = (int64_t)blockIdx.x * 32, jb = blockIdx.y;
  V A[1][NS];
  f32x16 Cin[1];
  load_queries<F16, NS, 1>(x, m, q0, l32, half, A, Cin);
  V B[NL];
  const char* blk = reinterpret_cast<const char*>(x.cop) + jb * (NL * 1024);
#pragma unroll
  for (int s = 0; s < NL; ++s) B[s] = *reinterpret_cast<const V*>(blk + s * 1024 + lane * 16);
  f32x16 acc[1];
  step_products<F16, NS, 1, NL>(A, Cin, B, acc);
  const int64_t j = jb * 32 + l32;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t qi = q0 + 8 * (r / 4) + 4 * half + (r % 4);
    if (qi < m && j < n) D[(int64_t)qorig[qi] * n + j] = acc[0][r];
  }
}

template <int NK>
__global__ __launch_bounds__(kWave) void k_dump_mfma32(Mfma32Dev x, int64_t m, int64_t n,
                                                      const int32_t* __restrict__ qorig, float* __restrict__ D) {
  const int lane = threadIdx.x, l32 = lane & 31, half = lane >> 5;
  const int64_t q0 = (int64_t)blockIdx.x * 32, jb = blockIdx.y;
  float A[1][NK];
  f32x16 Cin[1];
  load_queries32<NK, 1>(x, m, q0, l32, half, A, Cin);
  float B[NK];
#pragma unroll
  for (int s = 0; s < NK; ++s) B[s] = x.cop[(jb * NK + s) * 64 + lane];
  f32x16 acc[1];
  step_products32<NK, 1>(A, Cin, B, acc);
  const int64_t j = jb * 32 + l32;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t qi = q0 + 8 * (r / 4) + 4 * half + (r % 4);
    if (qi < m && j < n) D[(int64_t)qorig[qi] * n + j] = acc[0][r];
  }
}

// Candidate operand rows out of the 32-row block layout: out[j KB + k], j < n.
__global__ __launch_bounds__(kThreads) void k_dump_cand16(const uint16_t* __restrict__ cop, int64_t n, int KB,
                                                         uint16_t* __restrict__ out) {
  const int nl = KB / 16;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * KB; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / KB;
    const int k = (int)(e % KB);
    out[e] = cop[((j / 32 * nl + k / 16) * 2 + (k % 16) / 8) * 256 + (j % 32) * 8 + k % 8];
  }
}

// Score-order rows of W values into the caller's order: out[qorig[s] W + k].
template <typename T>
__global__ __launch_bounds__(kThreads) void k_dump_rows(const T* __restrict__ in, int64_t m, int W,
                                                       const int32_t* __restrict__ qorig, T* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m * W; e += (int64_t)gridDim.x * blockDim.x)
    out[(int64_t)qorig[e / W] * W + e % W] = in[e];
}

// Query blocks of 32 per wavefront in the fp32 screen: with two product
// slices per chain (d <= 4) four blocks keep the matrix pipe busiest
// (measured on the 5e6-point d = 3 self-query: 30.5 ms per query pass with
// four blocks, 30.6-31.1 with three, 32.3 with two).
constexpr int kQB32 = 4;

typedef void (*Mfma32Kernel)(QueryDev, Mfma32Dev);

// query blocks per wavefront: kQB32 for single queries, 2 in the batch
// (whose tiles of 256 slots are shared with the 16-bit screen)
template <int QB>
Mfma32Kernel pick_kernel32_qb(int d) {
  switch ((d + 1) / 2) {
    case 1: return k_cand_mfma32<1, QB>;
    case 2: return k_cand_mfma32<2, QB>;
    case 3: return k_cand_mfma32<3, QB>;
    case 4: return k_cand_mfma32<4, QB>;
    case 5: return k_cand_mfma32<5, QB>;
    case 6: return k_cand_mfma32<6, QB>;
    case 7: return k_cand_mfma32<7, QB>;
    case 8: return k_cand_mfma32<8, QB>;
    default: return nullptr;
  }
}
Mfma32Kernel pick_kernel32(int d) { return pick_kernel32_qb<kQB32>(d); }
constexpr int kQB32Batch = 2;

typedef void (*MixedKernel)(QueryDev, MixedDev);

// Query blocks of 32 per wavefront.  More blocks share each candidate load
// among more product chains, but also make the tiles (4 wavefronts x QB x
// 32 queries) longer, and with them the union windows of small instances.
// The one-slice fp16 screen has one product per block and step, so its
// candidate loads are the larger share of the work: three blocks there
// (n = 1e6, d = 16 set: 0.379 ms against 0.415 ms with two, 0.374 ms with
// four at 5% more executed pairs and two wavefronts per SIMD).  Two blocks
// elsewhere: two against four measured 1.03-1.05 vs 1.25-1.31 ms for the
// 256-instance batch screen and equal within noise for the d = 16 set in
// three-term bf16; issuing the next step's products before the previous
// step's compare epilogue (two accumulator sets) gained nothing at two
// blocks and lost a wave per SIMD at four.
constexpr int qb_for(bool f16, int ns) { return f16 && ns == 1 ? 3 : 2; }

// (slices per product chain, slices loaded per candidate row); fp16
// operands come one per coordinate only (ns = nl)
MixedKernel pick_kernel(int KA, int KB, bool f16) {
  const int ns = KA / 16, nl = KB / 16;
#define SNN_CASE(NS_, NL_) \
  if (ns == NS_ && nl == NL_) return f16 ? k_cand_mfma<true, NS_, qb_for(true, NS_), NL_> : k_cand_mfma<false, NS_, qb_for(false, NS_), NL_>;
  SNN_CASE(1, 1) SNN_CASE(2, 2) SNN_CASE(3, 3) SNN_CASE(4, 4) SNN_CASE(5, 5) SNN_CASE(6, 6) SNN_CASE(7, 7)
  SNN_CASE(8, 8)
#undef SNN_CASE
#define SNN_CASE(NS_, NL_) \
  if (!f16 && ns == NS_ && nl == NL_) return k_cand_mfma<false, NS_, qb_for(false, NS_), NL_>;
  SNN_CASE(3, 2) SNN_CASE(6, 4)
#undef SNN_CASE
  return nullptr;
}

int grid_for(int64_t work, int cap) {
  int64_t g = (work + kThreads - 1) / kThreads;
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

int mixed_max_slices() { return 8; }
int mixed_queries_per_wave(int KA, bool f16) { return 32 * qb_for(f16, KA / 16); }

int mixed_blocks_per_cu(int KA, int KB, bool f16) {
  MixedKernel k = pick_kernel(KA, KB, f16);
  int nb = 0;
  if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kThreads, 0) != hipSuccess || nb < 1) {
    (void)hipGetLastError();
    nb = 1;
  }
  return nb;
}

void launch_mixed_qprep_self(const float* ys, int64_t n, int d, const MixedBound& b, float* cthr, hipStream_t s) {
  if (d <= 8)
    k_mixed_qprep_self<1><<<grid_for(n, 8192), kThreads, 0, s>>>(ys, n, d, b, cthr);
  else
    k_mixed_qprep_self<16><<<grid_for(n * 16, 8192), kThreads, 0, s>>>(ys, n, d, b, cthr);
  SNN_LAUNCH_CHECK();
}

int mfma32_max_d() { return 16; }
int mfma32_query_floats(int d) { return ((d + 1 + 3) / 4) * 4; }
int mfma32_queries_per_tile() { return 4 * 32 * kQB32; }
int64_t mfma32_operand_floats(int64_t n, int d) { return ((n + 32 + 31) / 32) * 32 * 2 * ((d + 1) / 2); }

int mfma32_blocks_per_cu(int d) {
  Mfma32Kernel k = pick_kernel32(d);
  int nb = 0;
  if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kThreads, 0) != hipSuccess || nb < 1) {
    (void)hipGetLastError();
    nb = 1;
  }
  return nb;
}

void launch_mfma32_operands(const float* ys, int64_t n, int d, float* cop, hipStream_t s) {
  const int64_t npad = ((n + 32 + 31) / 32) * 32;
  k_mfma32_operands<<<grid_for(npad * 2 * ((d + 1) / 2), 16384), kThreads, 0, s>>>(ys, n, npad, d, (d + 1) / 2, cop);
  SNN_LAUNCH_CHECK();
}

void launch_mfma32_qprep_self(const float* ys, int64_t n, int d, const MixedBound& b, float* vq, hipStream_t s) {
  if (n <= 0) return;
  k_mfma32_qprep_self<<<grid_for(n, 8192), kThreads, 0, s>>>(ys, n, d, mfma32_query_floats(d), b, vq);
  SNN_LAUNCH_CHECK();
}

// T must equal mfma32_queries_per_tile(); tile windows aligned to 32 rows.
void launch_cand_mfma32(const QueryDev& q, const Mfma32Dev& x, int grid, hipStream_t s) {
  Mfma32Kernel k = pick_kernel32(x.d);
  if (!k) fail(SNN_ENOTSUP, "fp32 matrix-core screen supports d <= 16");
  k<<<grid, kThreads, 0, s>>>(q, x);
  SNN_LAUNCH_CHECK();
}

int mfma32_batch_queries_per_tile() { return 4 * 32 * kQB32Batch; }
int mfma32_batch_blocks_per_cu(int d) {
  Mfma32Kernel k = pick_kernel32_qb<kQB32Batch>(d);
  int nb = 0;
  if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kThreads, 0) != hipSuccess || nb < 1) {
    (void)hipGetLastError();
    nb = 1;
  }
  return nb;
}
void launch_cand_mfma32_batch(const QueryDev& q, const Mfma32Dev& x, int grid, hipStream_t s) {
  Mfma32Kernel k = pick_kernel32_qb<kQB32Batch>(x.d);
  if (!k) fail(SNN_ENOTSUP, "fp32 matrix-core screen supports d <= 16");
  k<<<grid, kThreads, 0, s>>>(q, x);
  SNN_LAUNCH_CHECK();
}

void launch_dump_mixed(const MixedDev& x, int64_t m, int64_t n, const int32_t* qorig, float* D, hipStream_t s) {
  const dim3 grid((unsigned)((m + 31) / 32), (unsigned)((n + 31) / 32));
  const int ns = x.KA / 16, nl = x.KB / 16;
  if (m <= 0 || n <= 0) return;
#define SNN_CASE(NS_, NL_)                                                                          \
  if (ns == NS_ && nl == NL_) {                                                                     \
    if (x.f16)                                                                                      \
      k_dump_mixed<true, NS_, NL_><<<grid, kWave, 0, s>>>(x, m, n, qorig, D);                        \
    else                                                                                            \
      k_dump_mixed<false, NS_, NL_><<<grid, kWave, 0, s>>>(x, m, n, qorig, D);                       \
    SNN_LAUNCH_CHECK();                                                                             \
    return;                                                                                         \
  }
  SNN_CASE(1, 1) SNN_CASE(2, 2) SNN_CASE(3, 3) SNN_CASE(4, 4) SNN_CASE(5, 5) SNN_CASE(6, 6) SNN_CASE(7, 7)
  SNN_CASE(8, 8) SNN_CASE(3, 2) SNN_CASE(6, 4)
#undef SNN_CASE
  fail(SNN_ENOTSUP, "no screen for this operand layout");
}

void launch_dump_mfma32(const Mfma32Dev& x, int64_t m, int64_t n, const int32_t* qorig, float* D, hipStream_t s) {
  if (m <= 0 || n <= 0) return;
  const dim3 grid((unsigned)((m + 31) / 32), (unsigned)((n + 31) / 32));
  switch ((x.d + 1) / 2) {
#define SNN_CASE(NK_) \
  case NK_: k_dump_mfma32<NK_><<<grid, kWave, 0, s>>>(x, m, n, qorig, D); break;
    SNN_CASE(1) SNN_CASE(2) SNN_CASE(3) SNN_CASE(4) SNN_CASE(5) SNN_CASE(6) SNN_CASE(7) SNN_CASE(8)
#undef SNN_CASE
    default: fail(SNN_ENOTSUP, "fp32 matrix-core screen supports d <= 16");
  }
  SNN_LAUNCH_CHECK();
}

void launch_dump_cand16(const uint16_t* cop, int64_t n, int KB, uint16_t* out, hipStream_t s) {
  if (n <= 0) return;
  k_dump_cand16<<<grid_for(n * KB, 8192), kThreads, 0, s>>>(cop, n, KB, out);
  SNN_LAUNCH_CHECK();
}

void launch_dump_rows_u16(const uint16_t* in, int64_t m, int W, const int32_t* qorig, uint16_t* out, hipStream_t s) {
  if (m <= 0) return;
  k_dump_rows<uint16_t><<<grid_for(m * W, 8192), kThreads, 0, s>>>(in, m, W, qorig, out);
  SNN_LAUNCH_CHECK();
}

void launch_dump_rows_f32(const float* in, int64_t m, int W, const int32_t* qorig, float* out, hipStream_t s) {
  if (m <= 0) return;
  k_dump_rows<float><<<grid_for(m * W, 8192), kThreads, 0, s>>>(in, m, W, qorig, out);
  SNN_LAUNCH_CHECK();
}

// T must equal 4 waves x 32 x QB (QB = 2).
void launch_cand_mfma(const QueryDev& q, const MixedDev& x, int grid, hipStream_t s) {
  MixedKernel k = pick_kernel(x.KA, x.KB, x.f16 != 0);
  if (!k) fail(SNN_ENOTSUP, "16-bit screens support operand rows of at most 128 values");
  k<<<grid, kThreads, 0, s>>>(q, x);
  SNN_LAUNCH_CHECK();
}

}  // namespace snn
