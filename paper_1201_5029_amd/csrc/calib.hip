// Plain device-to-device copy used to calibrate memory counters and to
// report the achievable HBM bandwidth beside the lattice kernels.

#include <cmath>

#include "internal.h"
#include "timing.h"

namespace symlat {
namespace {

// One 16-byte element per lane, one workgroup per 4 KB: the fastest simple
// copy shape measured on MI355X (wider per-lane accesses and grid-stride
// loops are slower).
__global__ __launch_bounds__(kBlock) void copy_kernel(const double2* __restrict__ src,
                                                     double2* __restrict__ dst, size_t count) {
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < count) dst[e] = src[e];
}

}  // namespace
}  // namespace symlat

extern "C" sl_status sl_hbm_copy_bench(size_t bytes, int32_t iters, double* gbs) {
  using namespace symlat;
  if (bytes < 1024 || (bytes % 16) != 0 || iters < 1 || !gbs) return SL_E_INVALID;
  void* a = nullptr;
  void* b = nullptr;
  if (hipMalloc(&a, bytes) != hipSuccess) return SL_E_NOMEM;
  if (hipMalloc(&b, bytes) != hipSuccess) {
    (void)hipFree(a);
    return SL_E_NOMEM;
  }
  hipStream_t s;
  hipEvent_t e0, e1;
  sl_status st = SL_OK;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
    (void)hipFree(a);
    (void)hipFree(b);
    return SL_E_DEVICE;
  }
  (void)timing_event_create(&e0);
  (void)timing_event_create(&e1);
  const size_t count = bytes / 16;
  const unsigned grid = unsigned((count + kBlock - 1) / kBlock);
  (void)hipMemsetAsync(a, 0, bytes, s);
  hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(kBlock), 0, s,
                     static_cast<const double2*>(a), static_cast<double2*>(b), count);
  (void)hipEventRecord(e0, s);
  for (int i = 0; i < iters; ++i)
    hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(kBlock), 0, s,
                       static_cast<const double2*>(a), static_cast<double2*>(b), count);
  (void)hipEventRecord(e1, s);
  if (hipStreamSynchronize(s) != hipSuccess) st = SL_E_DEVICE;
  float ms = 0.0f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  *gbs = 2.0 * double(bytes) * iters / (double(ms) * 1e-3) / 1e9;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(s);
  (void)hipFree(a);
  (void)hipFree(b);
  return st;
}
