// Unit-norm rows for angular and cosine neighbours (Section 2): on
// normalised vectors the angle is at most a iff the squared Euclidean
// distance is at most 2 - 2 cos(a), and the cosine distance is half the
// squared Euclidean distance, so both searches are Euclidean searches of the
// normalised rows.
//
// y_k = fl_T(x_k / sqrt(s)), s = the float64 sum, left to right, of x_k^2
// (inputs promoted exactly; sqrt and the quotient correctly rounded in
// float64, then one rounding to the row dtype).  One thread per row keeps
// the summation order; a zero or non-finite row raises a flag.
#include <hip/hip_runtime.h>

#include <cmath>

#include "device_common.h"
#include "query_plan.h"
#include "snn_internal.h"

#pragma clang fp contract(off)

namespace snn {

namespace {

constexpr int kThreads = 256;

template <typename T>
__global__ __launch_bounds__(kThreads) void k_normalize_rows(const T* __restrict__ X, int64_t n, int d,
                                                             T* __restrict__ Y, int* __restrict__ bad) {
  int b = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const T* x = X + i * d;
    double s = 0.0;
    for (int k = 0; k < d; ++k) {
      const double v = (double)x[k];
      s = s + v * v;
    }
    const double nrm = sqrt(s);
    if (!(nrm > 0.0) || !isfinite(nrm)) {
      b = 1;
      continue;
    }
    T* y = Y + i * d;
    for (int k = 0; k < d; ++k) y[k] = (T)((double)x[k] / nrm);
  }
  if (__ballot(b) && lane_id() == 0) atomicOr(bad, 1);
}

int grid_for(int64_t work, int cap) {
  int64_t g = (work + kThreads - 1) / kThreads;
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

}  // namespace snn

using namespace snn;

extern "C" {

snn_status snn_normalize_rows(const snn_device* dev, const void* X, int64_t n, int32_t d, snn_dtype dtype, void* Y) {
  return guard([&] {
    if (!dev) fail(SNN_EINVAL, "dev is NULL");
    if (n < 0) fail(SNN_EINVAL, "n must be >= 0");
    if (d < 1) fail(SNN_EINVAL, "d must be >= 1");
    if (dtype != SNN_F32 && dtype != SNN_F64) fail(SNN_EINVAL, "unknown dtype");
    if (n > 0 && (!X || !Y)) fail(SNN_EINVAL, "X / Y is NULL");
    if ((dev->alloc == nullptr) != (dev->free == nullptr)) fail(SNN_EINVAL, "alloc and free must both be set");
    if (n == 0) return;
    DeviceScope scope(dev->device);
    DeviceArena a(*dev);
    hipStream_t s = a.stream();
    const DeviceInfo& di = device_info(dev->device);
    ScopedAlloc flag(a, 256);
    int* bad = static_cast<int*>(flag.get());
    launch_fill_i32(bad, 1, 0, s);
    const int grid = grid_for(n, di.cus * 16);
    if (dtype == SNN_F32)
      k_normalize_rows<float><<<grid, kThreads, 0, s>>>(static_cast<const float*>(X), n, d, static_cast<float*>(Y),
                                                        bad);
    else
      k_normalize_rows<double><<<grid, kThreads, 0, s>>>(static_cast<const double*>(X), n, d,
                                                         static_cast<double*>(Y), bad);
    SNN_LAUNCH_CHECK();
    int hbad = 0;
    SNN_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    SNN_HIP(hipStreamSynchronize(s));
    if (hbad) fail(SNN_EINVAL, "a row is zero or holds NaN/Inf");
  });
}

}  // extern "C"
