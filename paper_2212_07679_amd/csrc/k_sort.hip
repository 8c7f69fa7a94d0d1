// LSD radix sort of (uint32 key, uint32 value) pairs and exclusive scans.
//
// Algorithm 1 step 6 sorts the data by score; here the scores are mapped to
// order-preserving uint32 keys and sorted least-significant digit first with
// 8-bit digits.  Each pass: per-block digit histograms (digit-major layout),
// one exclusive scan over them, and a stable scatter in which every block
// ranks its keys with wavefront ballots (64-lane match of equal digits) and
// LDS counters, so equal keys keep their input order.  (11-bit digits, three
// passes for 32 bits, were slower on 1e6 keys: with 2 keys per digit and
// workgroup the scatter's writes hardly coalesce, and the larger LDS
// histograms halve the workgroups.)
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"
#include "snn_internal.h"

namespace snn {

namespace {

constexpr int kSortThreads = 256;
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;

// ITEMS keys per thread, kSortThreads * ITEMS per block.  With lb set the
// kernel also clears the lb_words state words of the look-back scan that
// follows it.
template <int ITEMS>
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint32_t* __restrict__ keys, int64_t n,
                                                            int shift, uint32_t mask, uint32_t* __restrict__ hist,
                                                            int nblocks, unsigned long long* __restrict__ lb,
                                                            int lb_words) {
  __shared__ uint32_t h[kSortThreads / kWave][kRadix];
  const int t = threadIdx.x, w = t / kWave;
  if (lb)
    for (int i = blockIdx.x * kSortThreads + t; i < lb_words; i += gridDim.x * kSortThreads) lb[i] = 0ull;
  for (int i = t; i < (kSortThreads / kWave) * kRadix; i += kSortThreads) (&h[0][0])[i] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortThreads * ITEMS;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    int64_t idx = base + (int64_t)i * kSortThreads + t;
    if (idx < n) atomicAdd(&h[w][(keys[idx] >> shift) & mask], 1u);
  }
  __syncthreads();
  if (t < kRadix) {
    uint32_t s = 0;
#pragma unroll
    for (int ww = 0; ww < kSortThreads / kWave; ++ww) s += h[ww][t];
    hist[(int64_t)t * nblocks + blockIdx.x] = s;
  }
}

template <int ITEMS>
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const uint32_t* __restrict__ kin,
                                                               const uint32_t* __restrict__ vin,
                                                               uint32_t* __restrict__ kout,
                                                               uint32_t* __restrict__ vout, int64_t n, int shift,
                                                               int bits, const uint32_t* __restrict__ hist,
                                                               int nblocks) {
  constexpr int kW = kSortThreads / kWave;
  __shared__ uint32_t s_off[kRadix];       // the block's first output position per digit
  __shared__ uint32_t s_run[kRadix];       // keys of each digit placed in earlier rounds
  __shared__ uint32_t s_wcnt[kW][kRadix];  // this round's count per wavefront and digit (0 where absent)
  const int t = threadIdx.x, w = t / kWave, lane = t % kWave;
  const uint32_t mask = (1u << bits) - 1u;
  if (t < kRadix) {
    s_off[t] = ((uint32_t)t <= mask) ? hist[(int64_t)t * nblocks + blockIdx.x] : 0u;
    s_run[t] = 0;
#pragma unroll
    for (int ww = 0; ww < kW; ++ww) s_wcnt[ww][t] = 0;
  }
  __syncthreads();
  const uint64_t lt = (1ull << lane) - 1ull;
  const int64_t base = (int64_t)blockIdx.x * kSortThreads * ITEMS;
  // every item of the thread is loaded up front (all loads in flight at
  // once), then ranked round by round; round i holds block positions
  // i * kSortThreads + t, so wavefront order within a round and round order
  // are the input order
  uint32_t ks[ITEMS], vs[ITEMS];
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const int64_t idx = base + (int64_t)i * kSortThreads + t;
    ks[i] = idx < n ? kin[idx] : 0u;
    vs[i] = idx < n ? vin[idx] : 0u;
  }
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const int64_t idx = base + (int64_t)i * kSortThreads + t;
    const bool valid = idx < n;
    const uint32_t k = ks[i], v = vs[i];
    const uint32_t dg = valid ? (k >> shift) & mask : 0u;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < bits; ++b) {
      uint64_t mb = __ballot((dg >> b) & 1u);
      peers &= ((dg >> b) & 1u) ? mb : ~mb;
    }
    const uint64_t below = peers & lt;
    const uint32_t rank = (uint32_t)__popcll(below);
    const uint32_t cnt = (uint32_t)__popcll(peers);
    // the lowest lane of each group of equal digits speaks for the group
    const bool leader = valid && below == 0;
    if (leader) s_wcnt[w][dg] = cnt;
    __syncthreads();
    if (valid) {
      uint32_t pos = s_run[dg] + rank;
      for (int ww = 0; ww < w; ++ww) pos += s_wcnt[ww][dg];
      const uint32_t g = s_off[dg] + pos;
      kout[g] = k;
      vout[g] = v;
    }
    __syncthreads();
    // after every read of this round: the group's count moves into the
    // running total and its slot is cleared for the next round (only this
    // wavefront writes that slot, and the next round reads it after the
    // next barrier)
    if (leader) {
      s_wcnt[w][dg] = 0;
      atomicAdd(&s_run[dg], cnt);
    }
  }
}

// ---------------------------------------------------------------- scans
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* lds, T& total) {
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  T x = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  if (lane == kWave - 1) lds[w] = x;
  __syncthreads();
  T pre = 0, tot = 0;
#pragma unroll
  for (int ww = 0; ww < kScanThreads / kWave; ++ww) {
    T s = lds[ww];
    if (ww < w) pre += s;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return pre + x - v;
}

template <typename TI, typename TO>
__global__ __launch_bounds__(kScanThreads) void k_scan_sums(const TI* __restrict__ in, int64_t n,
                                                           TO* __restrict__ sums) {
  __shared__ TO lds[kScanThreads / kWave];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  TO s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    int64_t idx = base + i;
    if (idx < n) s += (TO)in[idx];
  }
  TO total;
  block_exclusive_scan<TO>(s, lds, total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// out[i] = offset of the block + exclusive prefix within the tile; if
// `write_total` the thread owning element n-1 also writes out[n].  The
// block's offset is offsets[block] (scanned block sums), or, with
// `raw_sums`, the sum of offsets[0 .. block) taken here (the block sums
// unscanned: saves the launch that would scan them; at most kScanTile
// blocks).
template <typename TI, typename TO>
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const TI* in, TO* out, int64_t n,
                                                            const TO* __restrict__ offsets, int write_total,
                                                            int raw_sums = 0) {
  __shared__ TO lds[kScanThreads / kWave];
  __shared__ TO block_off;
  if (raw_sums) {
    TO part = 0;
    for (int b = threadIdx.x; b < (int)blockIdx.x; b += kScanThreads) part += offsets[b];
    part = wave_sum(part);
    if (lane_id() == 0) lds[threadIdx.x / kWave] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
      TO t = 0;
      for (int w = 0; w < kScanThreads / kWave; ++w) t += lds[w];
      block_off = t;
    }
    __syncthreads();  // lds is reused by the scan below
  }
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  TI vals[kScanItems];
  TO s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    int64_t idx = base + i;
    vals[i] = idx < n ? in[idx] : (TI)0;
    s += (TO)vals[i];
  }
  TO total;
  TO run = block_exclusive_scan<TO>(s, lds, total) + (raw_sums ? block_off : offsets ? offsets[blockIdx.x] : (TO)0);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    int64_t idx = base + i;
    if (idx < n) {
      out[idx] = run;
      run += (TO)vals[i];
      if (write_total && idx == n - 1) out[n] = run;
    }
  }
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Exclusive scan in one workgroup for short arrays: passes of 1024 x 16
// elements with a running carry (one launch instead of three; in place is
// safe, every thread reads its elements before writing them).  Each pass is
// latency-bound, so it is used for arrays of one pass only (measured: seven
// passes over 1e5 counts took ~70 us, three launches far less).
constexpr int kScan1Threads = 1024;
constexpr int kScan1Items = 16;
constexpr int64_t kScan1Max = (int64_t)kScan1Threads * kScan1Items;

template <typename TI, typename TO>
__global__ __launch_bounds__(kScan1Threads) void k_scan_single(const TI* in, TO* out, int64_t n, int write_total) {
  __shared__ TO wsum[kScan1Threads / kWave];
  __shared__ TO carry_s;
  const int t = threadIdx.x, lane = t % kWave, w = t / kWave;
  if (t == 0) carry_s = 0;
  __syncthreads();
  for (int64_t base = 0; base < n; base += (int64_t)kScan1Threads * kScan1Items) {
    const int64_t i0 = base + (int64_t)t * kScan1Items;
    TI v[kScan1Items];
    TO sum = 0;
#pragma unroll
    for (int i = 0; i < kScan1Items; ++i) {
      v[i] = i0 + i < n ? in[i0 + i] : (TI)0;
      sum += (TO)v[i];
    }
    TO x = sum;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const TO y = __shfl_up(x, o, kWave);
      if (lane >= o) x += y;
    }
    if (lane == kWave - 1) wsum[w] = x;
    __syncthreads();
    TO pre = carry_s, tot = 0;
    for (int k = 0; k < kScan1Threads / kWave; ++k) {
      const TO ws = wsum[k];
      if (k < w) pre += ws;
      tot += ws;
    }
    TO run = pre + x - sum;
#pragma unroll
    for (int i = 0; i < kScan1Items; ++i) {
      if (i0 + i < n) out[i0 + i] = run;
      run += (TO)v[i];
    }
    __syncthreads();
    if (t == 0) carry_s += tot;
    __syncthreads();
  }
  if (write_total && t == 0) out[n] = carry_s;
}

// Recursive exclusive scan; scratch holds the block sums of every level.
template <typename TI, typename TO>
void scan_rec(const TI* in, TO* out, int64_t n, int write_total, TO* scratch, hipStream_t s) {
  if (n <= 0) {
    if (write_total) {
      k_scan_single<TI, TO><<<1, kScan1Threads, 0, s>>>(in, out, 0, 1);  // out[0] = 0, as a kernel
      SNN_LAUNCH_CHECK();
    }
    return;
  }
  const int64_t nb = ceil_div(n, kScanTile);
  if (nb == 1) {
    k_scan_apply<TI, TO><<<1, kScanThreads, 0, s>>>(in, out, n, nullptr, write_total);
    SNN_LAUNCH_CHECK();
    return;
  }
  if (n <= kScan1Max) {
    k_scan_single<TI, TO><<<1, kScan1Threads, 0, s>>>(in, out, n, write_total);
    SNN_LAUNCH_CHECK();
    return;
  }
  TO* sums = scratch;
  k_scan_sums<TI, TO><<<(unsigned)nb, kScanThreads, 0, s>>>(in, n, sums);
  SNN_LAUNCH_CHECK();
  if (nb <= kScanTile) {  // each block adds up the sums before it
    k_scan_apply<TI, TO><<<(unsigned)nb, kScanThreads, 0, s>>>(in, out, n, sums, write_total, 1);
    SNN_LAUNCH_CHECK();
    return;
  }
  scan_rec<TO, TO>(sums, sums, nb, 0, scratch + nb, s);
  k_scan_apply<TI, TO><<<(unsigned)nb, kScanThreads, 0, s>>>(in, out, n, sums, write_total);
  SNN_LAUNCH_CHECK();
}

// In-place exclusive scan of n u32 values in one launch (look-back; state:
// lookback_words(n) zeroed words).
__global__ __launch_bounds__(kLookbackThreads) void k_scan_u32_lookback(uint32_t* __restrict__ data, int64_t n,
                                                                       unsigned long long* __restrict__ state,
                                                                       int* __restrict__ err) {
  __shared__ unsigned long long s_tile;
  __shared__ uint32_t s_wave[kLookbackThreads / kWave];
  __shared__ uint32_t s_excl;
  const int t = threadIdx.x, lane = lane_id(), w = t / kWave;
  if (t == 0) s_tile = atomicAdd(&state[0], 1ull);
  __syncthreads();
  const long long tile = (long long)s_tile;
  const int64_t i0 = tile * kLookbackTile + (int64_t)t * kLookbackItems;
  uint32_t v[kLookbackItems], sum = 0;
#pragma unroll
  for (int k = 0; k < kLookbackItems; ++k) {
    v[k] = i0 + k < n ? data[i0 + k] : 0u;
    sum += v[k];
  }
  uint32_t x = sum;  // inclusive scan of the thread sums within the wavefront
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  if (lane == kWave - 1) s_wave[w] = x;
  __syncthreads();
  uint32_t before = 0, total = 0;
#pragma unroll
  for (int k = 0; k < kLookbackThreads / kWave; ++k) {
    if (k < w) before += s_wave[k];
    total += s_wave[k];
  }
  if (w == 0) {
    unsigned long long excl = 0;
    if (tile == 0) {
      if (lane == 0) lookback_publish(state, 0, 2, total);
    } else {
      if (lane == 0) lookback_publish(state, tile, 1, total);
      excl = lookback_exclusive(state, tile, err);
      if (lane == 0) lookback_publish(state, tile, 2, excl + total);
    }
    if (lane == 0) s_excl = (uint32_t)excl;
  }
  __syncthreads();
  uint32_t run = s_excl + before + x - sum;
#pragma unroll
  for (int k = 0; k < kLookbackItems; ++k) {
    if (i0 + k < n) data[i0 + k] = run;
    run += v[k];
  }
}

}  // namespace

size_t lookback_words(int64_t n) { return 1 + (size_t)std::max<int64_t>(1, ceil_div(n, kLookbackTile)); }

void lookback_scan_u32(uint32_t* data, int64_t n, unsigned long long* state, int* err, hipStream_t s) {
  if (n <= 0) return;
  k_scan_u32_lookback<<<(unsigned)ceil_div(n, kLookbackTile), kLookbackThreads, 0, s>>>(data, n, state, err);
  SNN_LAUNCH_CHECK();
}

size_t scan_scratch_bytes(int64_t n) {
  size_t total = 0;
  int64_t m = n;
  while (m > kScanTile) {
    m = ceil_div(m, kScanTile);
    total += (size_t)m;
  }
  return (total + 64) * sizeof(int64_t);
}

void exclusive_scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, void* scratch, hipStream_t s) {
  scan_rec<int32_t, int64_t>(in, out, n, 1, reinterpret_cast<int64_t*>(scratch), s);
}

void exclusive_scan_u32(uint32_t* data, int64_t n, void* scratch, hipStream_t s) {
  scan_rec<uint32_t, uint32_t>(data, data, n, 0, reinterpret_cast<uint32_t*>(scratch), s);
}

namespace {
// keys per thread of the radix kernels: 8 up to 2^21 keys (more workgroups
// for mid-size sorts), 16 above (measured: 1e6 keys 6% faster with 8,
// 5e6 keys 1% faster with 16)
int sort_items(int64_t n) { return n <= (int64_t(1) << 21) ? 8 : 16; }
int64_t sort_tile(int64_t n) { return (int64_t)kSortThreads * sort_items(n); }

// one 8-bit pass: histograms, their scan, the stable scatter.  With err the
// histograms are scanned in one look-back launch (state words in scratch,
// cleared by the histogram kernel; a wait that runs out sets *err), else
// by the two-launch scan, which needs no error word.
void radix_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout, int64_t n, int shift,
                int bits, uint32_t mask, uint32_t* hist, size_t nhist, int nblocks, void* scratch, int* err,
                hipStream_t s) {
  unsigned long long* lb = err ? static_cast<unsigned long long*>(scratch) : nullptr;
  const int lbw = err ? (int)lookback_words((int64_t)nhist) : 0;
  if (sort_items(n) == 8)
    k_radix_hist<8><<<nblocks, kSortThreads, 0, s>>>(kin, n, shift, mask, hist, nblocks, lb, lbw);
  else
    k_radix_hist<16><<<nblocks, kSortThreads, 0, s>>>(kin, n, shift, mask, hist, nblocks, lb, lbw);
  SNN_LAUNCH_CHECK();
  if (err)
    lookback_scan_u32(hist, (int64_t)nhist, lb, err, s);
  else
    exclusive_scan_u32(hist, (int64_t)nhist, scratch, s);
  if (sort_items(n) == 8)
    k_radix_scatter<8><<<nblocks, kSortThreads, 0, s>>>(kin, vin, kout, vout, n, shift, bits, hist, nblocks);
  else
    k_radix_scatter<16><<<nblocks, kSortThreads, 0, s>>>(kin, vin, kout, vout, n, shift, bits, hist, nblocks);
  SNN_LAUNCH_CHECK();
}

// Workspace: the ping-pong copies, one pass's histograms, and the scan's
// block sums or look-back state, whichever is larger.
size_t ws_bytes(int64_t n, size_t nhist) {
  const size_t aux = std::max(scan_scratch_bytes((int64_t)nhist), sizeof(unsigned long long) * lookback_words((int64_t)nhist));
  return 2 * (size_t)n * sizeof(uint32_t) + nhist * sizeof(uint32_t) + aux + 1024;
}

// All passes from keys/vals through the workspace; kin/vin end up naming
// the buffers that hold the result.
void radix_passes(uint32_t*& kin, uint32_t*& vin, int64_t n, int begin_bit, int end_bit, void* ws, int* err,
                  hipStream_t s) {
  const int nblocks = (int)ceil_div(n, sort_tile(n));
  const size_t nhist = (size_t)nblocks * kRadix;
  uint32_t* k2 = static_cast<uint32_t*>(ws);
  uint32_t* v2 = k2 + n;
  uint32_t* hist = v2 + n;
  void* scratch = reinterpret_cast<void*>((reinterpret_cast<uintptr_t>(hist + nhist) + 255) & ~uintptr_t(255));
  uint32_t *kout = k2, *vout = v2;
  for (int shift = begin_bit; shift < end_bit; shift += kRadixBits) {
    const int bits = std::min(kRadixBits, end_bit - shift);
    const uint32_t mask = (1u << bits) - 1u;
    radix_pass(kin, vin, kout, vout, n, shift, bits, mask, hist, nhist, nblocks, scratch, err, s);
    std::swap(kin, kout);
    std::swap(vin, vout);
  }
}
}  // namespace

void radix_sort_pairs(DeviceArena& a, uint32_t* keys, uint32_t* vals, int64_t n, int begin_bit, int end_bit,
                      hipStream_t s) {
  if (n <= 1 || begin_bit >= end_bit) return;
  if (n > (int64_t)UINT32_MAX / 2) fail(SNN_EINVAL, "radix sort: too many keys");
  ScopedAlloc mem(a, radix_sort_ws_bytes(n));
  uint32_t *kin = keys, *vin = vals;
  radix_passes(kin, vin, n, begin_bit, end_bit, mem.get(), nullptr, s);
  if (kin != keys) {
    SNN_HIP(hipMemcpyAsync(keys, kin, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    SNN_HIP(hipMemcpyAsync(vals, vin, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
  }
}

size_t radix_sort_ws_bytes(int64_t n) {
  const int64_t nblocks = ceil_div(std::max<int64_t>(n, 1), sort_tile(n));
  return ws_bytes(n, (size_t)nblocks * kRadix);
}

namespace {
__global__ void k_copy_pairs(const uint32_t* __restrict__ ks, const uint32_t* __restrict__ vs,
                             uint32_t* __restrict__ kd, uint32_t* __restrict__ vd, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    kd[i] = ks[i];
    vd[i] = vs[i];
  }
}
}  // namespace

// Same sort with caller-provided workspace (radix_sort_ws_bytes(n) bytes) and
// kernels only (no allocation, no copy or memset calls): usable under
// stream capture.  With err (a device word the caller reads back and
// checks) the histogram scans take the one-launch look-back scan.  With kres/vres the sorted pairs are left where the last
// pass wrote them (keys/vals or the start of the workspace) and those
// pointers returned; without, they are copied back into keys/vals.
void radix_sort_pairs_ws(uint32_t* keys, uint32_t* vals, int64_t n, int begin_bit, int end_bit, void* ws,
                         hipStream_t s, uint32_t** kres, uint32_t** vres, int* err) {
  uint32_t *kin = keys, *vin = vals;
  if (n > (int64_t)UINT32_MAX / 2) fail(SNN_EINVAL, "radix sort: too many keys");
  if (n > 1 && begin_bit < end_bit) radix_passes(kin, vin, n, begin_bit, end_bit, ws, err, s);
  if (kres) {
    *kres = kin;
    *vres = vin;
    return;
  }
  if (kin != keys) {
    k_copy_pairs<<<(unsigned)std::min<int64_t>(ceil_div(n, 256), 4096), 256, 0, s>>>(kin, vin, keys, vals, n);
    SNN_LAUNCH_CHECK();
  }
}

}  // namespace snn
