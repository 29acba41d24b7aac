// Optional check of results for non-finite values (environment
// LOS_CHECK_FINITE=1): after an entry point has enqueued its work, the output
// array is scanned on the device and the call waits for the count.  Off by
// default: it costs a stream synchronisation per call.
#include <cstdlib>
#include <mutex>

#include "los_internal.hpp"

namespace los {
namespace {

template <typename T>
__global__ __launch_bounds__(256) void count_nonfinite_kernel(const T *p, int64_t n,
                                                              unsigned int *count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  unsigned int c = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    c += isfinite((double)p[i]) ? 0u : 1u;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, c);
}

constexpr int kMaxDev = 64;
std::mutex g_mu;
unsigned int *g_count[kMaxDev] = {};

}  // namespace

bool finite_check_enabled() {
  const char *v = std::getenv("LOS_CHECK_FINITE");
  return v && std::atoi(v) != 0;
}

hipError_t count_nonfinite(const void *p, int64_t n, bool f32, hipStream_t s,
                           unsigned long long *bad) {
  *bad = 0;
  if (n <= 0) return hipSuccess;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDev) return hipErrorInvalidDevice;
  unsigned int *cnt = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_count[dev] && (e = hipMalloc((void **)&g_count[dev], sizeof(unsigned int))) != hipSuccess)
      return e;
    cnt = g_count[dev];
  }
  if ((e = hipMemsetAsync(cnt, 0, sizeof(unsigned int), s)) != hipSuccess) return e;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (f32)
    hipLaunchKernelGGL(count_nonfinite_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                       (const float *)p, n, cnt);
  else
    hipLaunchKernelGGL(count_nonfinite_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                       (const double *)p, n, cnt);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  unsigned int h = 0;
  if ((e = hipMemcpyAsync(&h, cnt, sizeof h, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  *bad = h;
  return hipSuccess;
}

}  // namespace los
