// clock.hip -- tq_clock_mhz: the shader clock measured on the device while
// every compute unit runs a dependent chain of vector instructions.
//
// Each workgroup reads the shader-clock counter (s_memtime) and the
// constant-rate real-time counter (s_memrealtime) before and after the chain;
// the clock is the ratio of the two deltas times the real-time counter's
// frequency.  Reported so that rates quoted against a peak computed at the
// 2.4 GHz data-sheet clock can be read against the clock actually running.
#include <algorithm>
#include <vector>

#include "tq_runtime.h"

namespace {

__global__ __launch_bounds__(256) void clock_probe_kernel(unsigned long long *__restrict__ out, int iters,
                                                          float seed) {
  const unsigned long long t0 = __builtin_amdgcn_s_memtime();
  const unsigned long long r0 = __builtin_amdgcn_s_memrealtime();
  float a = seed + static_cast<float>(threadIdx.x), b = 0.999f;
  for (int i = 0; i < iters; ++i) {
    a = a * b + 0.25f;
    b = b * a + 0.5f;
  }
  const unsigned long long t1 = __builtin_amdgcn_s_memtime();
  const unsigned long long r1 = __builtin_amdgcn_s_memrealtime();
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = t1 - t0;
    out[2 * blockIdx.x + 1] = r1 - r0;
  }
  if (a == b && a == 1234.5f) out[0] = 0;  // keeps the chain
}

}  // namespace

extern "C" int tq_clock_mhz(double *mhz, void *stream) {
  using namespace tqr;
  clear_error();
  if (!mhz) return fail(TQ_ERR_INVALID, "null mhz");
  int dev;
  int rc = current_device(&dev);
  if (rc) return rc;
  DevCtx *ctx;
  if ((rc = device_ctx(dev, &ctx))) return rc;
  int wall_khz = 0;
  hipError_t e = hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev);
  if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute(wall clock rate)");
  if (wall_khz <= 0) return fail(TQ_ERR_DEVICE, "no real-time counter rate");
  const int blocks = 4 * (ctx->num_cu > 0 ? ctx->num_cu : 256);
  unsigned long long *d = nullptr;
  if ((e = dev_malloc(&d, sizeof(unsigned long long) * 2 * blocks)) != hipSuccess)
    return hip_fail(e, "device allocation (clock probe)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<unsigned long long> h(2 * blocks);
  hipLaunchKernelGGL(clock_probe_kernel, dim3(blocks), dim3(256), 0, s, d, 1 << 16, 1.0f);
  e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpyAsync(h.data(), d, sizeof(unsigned long long) * 2 * blocks, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  dev_free(d);
  if (e != hipSuccess) return hip_fail(e, "clock probe");
  std::vector<double> r;
  for (int b = 0; b < blocks; ++b)
    if (h[2 * b + 1] > 0) r.push_back(static_cast<double>(h[2 * b]) / static_cast<double>(h[2 * b + 1]));
  if (r.empty()) return fail(TQ_ERR_DEVICE, "clock probe: no real-time ticks");
  std::sort(r.begin(), r.end());
  *mhz = r[r.size() / 2] * wall_khz / 1000.0;
  return TQ_OK;
}
