// The allocation-free entry point: the stable LSD radix sort of (key, value)
// pairs (the building block of Algorithm 1, step 6) with its workspace in a
// static device array instead of memory from the caller's allocator.
//
// `scratch` is a file-scope device array: every GPU the library runs on
// holds its own copy from the moment the code object is loaded there until
// the process ends.  In host code its name only stands in for the symbol;
// the device address of a GPU's copy comes from hipGetSymbolAddress, taken
// once per device (with that device current) on the first call there and
// kept, and only that address reaches kernels.  Every call on one GPU shares
// its copy, so calls that overlap on one GPU race.  The sort writes every
// workspace entry it reads (each pass rebuilds its histograms and scan
// sums), so nothing has to start at zero.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "snn_internal.h"

namespace snn {
namespace {
// at most 2^21 pairs: both ping-pong copies (16 MiB), the per-block
// histograms of one pass (1 MiB) and their scan sums
constexpr int64_t kNoAllocMaxPairs = int64_t(1) << 21;
constexpr size_t kScratchBytes = size_t(18) << 20;
}  // namespace

// referenced only through its looked-up address: kept in the code object
static __device__ __align__(256) __attribute__((used)) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of each GPU's copy (null: not looked up yet)

// Address of the current device's copy of `scratch`, looked up once per device.
void* scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) fail(SNN_EINVAL, "device ordinal beyond the static scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    SNN_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) fail(SNN_EDEVICE, "hipGetSymbolAddress returned no address for the static scratch");
    g_scratch_ptr[device] = p;
  }
  return g_scratch_ptr[device];
}

}  // namespace
}  // namespace snn

using namespace snn;

extern "C" snn_status snn_sort_pairs_u32_noalloc(const snn_device* dev, uint32_t* keys, uint32_t* vals, int64_t n,
                                                 int begin_bit, int end_bit) {
  return guard([&] {
    if (!dev) fail(SNN_EINVAL, "dev is NULL");
    if (n < 0) fail(SNN_EINVAL, "n must be >= 0");
    if (n > kNoAllocMaxPairs)
      fail(SNN_EINVAL, "n = " + std::to_string(n) + " exceeds the static scratch of the allocation-free sort (at most " +
                           std::to_string(kNoAllocMaxPairs) + " pairs; use snn_sort_pairs_u32)");
    if (n > 0 && (!keys || !vals)) fail(SNN_EINVAL, "keys / vals is NULL");
    if (begin_bit < 0 || end_bit > 32 || begin_bit >= end_bit) fail(SNN_EINVAL, "bad bit range");
    DeviceScope scope(dev->device);
    void* ws = scratch_address(dev->device);
    if (radix_sort_ws_bytes(n) > kScratchBytes) fail(SNN_EINVAL, "workspace larger than the static scratch");
    radix_sort_pairs_ws(keys, vals, n, begin_bit, end_bit, ws, (hipStream_t)dev->stream);
  });
}
