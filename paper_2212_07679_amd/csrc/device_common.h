// Device-side helpers shared by the gfx950 kernels: wavefront reductions,
// order-preserving float keys, bf16 rounding, and an LDS-staged appender for
// (query, candidate) pairs.  gfx950 wavefronts are 64 lanes wide.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace snn {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Order-preserving map float -> uint32: a < b (as floats, -0 < +0) iff
// key(a) < key(b).  NaN never reaches these kernels (inputs are checked).
__host__ __device__ __forceinline__ uint32_t float_to_ordered(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ __forceinline__ float ordered_to_float(uint32_t k) {
  uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
  return __builtin_bit_cast(float, u);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    T w = __shfl_xor(v, o, kWave);
    v = w > v ? w : v;
  }
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    T w = __shfl_xor(v, o, kWave);
    v = w < v ? w : v;
  }
  return v;
}

// Round-to-nearest-even float -> bf16 bits (finite inputs).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(r >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t b) {
  return __builtin_bit_cast(float, (uint32_t)b << 16);
}

// atomicMax on non-negative doubles via their bit patterns (monotone for x >= 0).
__device__ __forceinline__ void atomic_max_nonneg(double* addr, double v) {
  atomicMax(reinterpret_cast<unsigned long long*>(addr),
            (unsigned long long)__builtin_bit_cast(uint64_t, v));
}

// Survivor pairs are written as (query sorted position, candidate sorted
// position).  Each workgroup stages its pairs in LDS and reserves global
// space with one atomic at the end; if the LDS stage is full a pair goes
// straight to global memory.  The global list has capacity `cap`; the
// counter keeps counting past it so the host learns the size needed.
struct PairSink {
  int2* out;
  unsigned long long* counter;
  long long cap;
};

template <int kStage>
struct PairStage {
  int2 buf[kStage];
  int count;
  long long base;
};

template <int kStage>
__device__ __forceinline__ void stage_init(PairStage<kStage>& st) {
  if (threadIdx.x == 0) st.count = 0;
}

// Global-memory accesses through explicitly global pointers: a generic
// (flat) access would count against both the vector-memory and the LDS wait
// counters and force full waits on the loads in flight around it.
typedef __attribute__((address_space(1))) unsigned long long global_u64;

// an int2 (x at the lower address) stored as one little-endian 64-bit word
__device__ __forceinline__ void sink_store(const PairSink& sink, long long g, int2 v) {
  if (g < sink.cap)
    ((global_u64*)sink.out)[g] = ((unsigned long long)(uint32_t)v.y << 32) | (unsigned long long)(uint32_t)v.x;
}
__device__ __forceinline__ unsigned long long sink_reserve(const PairSink& sink, unsigned long long cnt) {
  return __hip_atomic_fetch_add((global_u64*)sink.counter, cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int kStage>
__device__ __forceinline__ void stage_push(PairStage<kStage>& st, const PairSink& sink, int q, int j) {
  int pos = atomicAdd(&st.count, 1);
  if (pos < kStage) {
    st.buf[pos] = make_int2(q, j);
  } else {
    sink_store(sink, (long long)sink_reserve(sink, 1ull), make_int2(q, j));
  }
}

// Wave-aggregated push: every lane with `pred` pushes (q, j).  One LDS
// atomic per wave; the pairs that no longer fit in the stage go straight to
// the global list under one global reservation per wave.
template <int kStage>
__device__ __forceinline__ void stage_push_wave(PairStage<kStage>& st, const PairSink& sink, bool pred, int q,
                                                int j) {
  uint64_t mask = __ballot(pred);
  if (mask == 0) return;
  const int cnt = __popcll(mask);
  const int leader = __ffsll((long long)mask) - 1;
  const int rank = __popcll(mask & ((1ull << lane_id()) - 1ull));
  int base = 0;
  if (lane_id() == leader) base = atomicAdd(&st.count, cnt);
  base = __shfl(base, leader, kWave);
  const int first_over = base > kStage ? base : kStage;
  const int over = base + cnt - first_over;  // pairs past the stage's end
  unsigned long long g = 0;
  if (over > 0) {
    if (lane_id() == leader) g = sink_reserve(sink, (unsigned long long)over);
    g = __shfl(g, leader, kWave);
  }
  if (pred) {
    const int pos = base + rank;
    if (pos < kStage)
      st.buf[pos] = make_int2(q, j);
    else
      sink_store(sink, (long long)g + (pos - first_over), make_int2(q, j));
  }
}

// Per-wavefront staging of pairs in LDS.  The fill count is wave-uniform
// (the caller keeps it in a scalar register), so a push is one ballot, a lane
// rank and an LDS store: no atomics and no cross-lane shuffles.  The caller
// flushes whenever fewer free entries remain than its largest burst of
// pushes, and once at the end; a flush takes one global reservation.
__device__ __forceinline__ void wave_push(int2* buf, int& wcnt, bool p, int q, int j) {
  const uint64_t m = __ballot(p);
  if (!m) return;
  if (p) {
    const int rank =
        (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    buf[wcnt + rank] = make_int2(q, j);
  }
  wcnt += __popcll(m);
}

__device__ __forceinline__ void wave_flush(int2* buf, int& wcnt, const PairSink& sink) {
  if (wcnt == 0) return;
  __builtin_amdgcn_wave_barrier();  // the lanes' LDS stores come before these reads
  unsigned long long base = 0;
  if (lane_id() == 0) base = sink_reserve(sink, (unsigned long long)wcnt);
  base = __shfl(base, 0, kWave);
  for (int i = lane_id(); i < wcnt; i += kWave) sink_store(sink, (long long)base + i, buf[i]);
  __builtin_amdgcn_wave_barrier();  // and these reads before the next pushes
  // this (rare) path drains the wave's memory counters, so that the callers'
  // load waits after it are counted as on the path without a flush
  __builtin_amdgcn_s_waitcnt(0);
  wcnt = 0;
}

// Moves the staged pairs to the global list and empties the stage.  All
// threads of the block call it right after a __syncthreads(), with no push in
// flight; the caller's next barrier orders the reset before new pushes.
template <int kStage>
__device__ __forceinline__ void stage_drain(PairStage<kStage>& st, const PairSink& sink) {
  const int cnt = st.count < kStage ? st.count : kStage;
  if (cnt == 0) return;  // block-uniform: every thread read the same value after the barrier
  if (threadIdx.x == 0) st.base = (long long)sink_reserve(sink, (unsigned long long)cnt);
  __syncthreads();
  const long long base = st.base;
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) sink_store(sink, base + i, st.buf[i]);
  __syncthreads();
  if (threadIdx.x == 0) st.count = 0;
}

// Must be called by all threads of the block after the last push.
template <int kStage>
__device__ __forceinline__ void stage_flush(PairStage<kStage>& st, const PairSink& sink) {
  __syncthreads();
  int cnt = st.count < kStage ? st.count : kStage;
  if (threadIdx.x == 0) {
    st.base = cnt ? (long long)sink_reserve(sink, (unsigned long long)cnt) : 0;
  }
  __syncthreads();
  long long base = st.base;
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) sink_store(sink, base + i, st.buf[i]);
}


// ---- single-pass scans (decoupled look-back)
// A workgroup takes its tile of kLookbackTile elements by a ticket, so every
// tile before it belongs to a workgroup that has already started; it
// publishes its tile total, then adds the totals of the tiles before it,
// one wavefront reading 64 of them at a time, back to the nearest tile that
// has published its inclusive prefix, and publishes its own.  state[0] is
// the ticket, state[1 + t] tile t's word: (flag << 62) | value with flag 0
// (nothing yet), 1 (tile total) or 2 (inclusive prefix); the whole state is
// zero before the launch.  A wait that does not end within kLookbackSpins
// polls sets *err and takes 0, so the kernel still ends (the host then
// reports the error); it cannot happen while every started workgroup
// progresses.
constexpr int kLookbackThreads = 256;
// four items per thread: on 1e5 rows the two row scans took 2.5 us less
// than with eight (more, shorter tiles; the wait for a predecessor is short)
constexpr int kLookbackItems = 4;
constexpr int kLookbackTile = kLookbackThreads * kLookbackItems;
constexpr int kLookbackSpins = 1 << 22;
constexpr unsigned long long kLookbackValue = (1ull << 62) - 1;

__device__ __forceinline__ void lookback_publish(unsigned long long* state, long long t, unsigned long long flag,
                                                 unsigned long long v) {
  __hip_atomic_store(&state[1 + t], (flag << 62) | (v & kLookbackValue), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive prefix of tile t (t > 0), called by one whole wavefront.
__device__ __forceinline__ unsigned long long lookback_exclusive(unsigned long long* state, long long t, int* err) {
  const int lane = lane_id();
  unsigned long long excl = 0;
  long long base = t - 1;
  int spins = 0;
  for (;;) {
    const long long j = base - lane;
    unsigned long long w = 2ull << 62;  // before tile 0: an inclusive prefix of 0
    if (j >= 0) w = __hip_atomic_load(&state[1 + j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long flag = w >> 62;
    const uint64_t pre = __ballot(flag == 2);
    const int p = pre ? __ffsll((long long)pre) - 1 : kWave;  // nearest prefix within the window
    const uint64_t need = p == kWave ? ~0ull : (p == 63 ? ~0ull : ((2ull << p) - 1ull));
    if (__ballot(flag == 0) & need) {  // a tile this window needs has not published yet
      if (++spins > kLookbackSpins) {
        if (lane == 0) *err = 1;
        return 0;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    excl += wave_sum(lane <= p ? (w & kLookbackValue) : 0ull);
    if (p < kWave) return excl;
    base -= kWave;
  }
}

}  // namespace snn
