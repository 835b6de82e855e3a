// clock.hip -- dqj_measure_engine_clock: the engine clock a device sustains under an FP32
// FMA load (declared in dqj_measure.h). Measurement support only: nothing on the render
// path calls it.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <vector>

#include "dqj_measure.h"
#include "runtime_internal.h"

namespace dqj {
namespace {

constexpr int kWavesPerBlock = 4;
constexpr int kBlocksPerCu = 8;   // 8 waves per SIMD

// Each wave runs `iters` rounds of two dependent FMA chains (16 FMAs each) and writes its
// shader-clock and wall-clock deltas to out[2w], out[2w + 1]. The chains converge to +1
// and -1, so the final test never holds; it keeps them live (a sink word at the end).
__global__ __launch_bounds__(256) void engine_clock_kernel(unsigned long long *__restrict__ out,
                                                           int iters, int nwaves) {
  float a = 1.0f + 1e-7f * (float)threadIdx.x, d = -a;
  const float b = 0.999f;
  const unsigned long long w0 = wall_clock64();
  const unsigned long long c0 = clock64();
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      a = fmaf(a, b, 1e-3f);
      d = fmaf(d, b, -1e-3f);
    }
  }
  const unsigned long long c1 = clock64();
  const unsigned long long w1 = wall_clock64();
  const int wave = (int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  if ((threadIdx.x & 63) == 0 && wave < nwaves) {
    out[2 * wave] = c1 - c0;
    out[2 * wave + 1] = w1 - w0;
  }
  if (a == d) out[2 * nwaves] = 1ull;
}

// Launch with `iters` rounds; returns the summed deltas.
hipError_t run_probe(unsigned long long *dev, int blocks, int nwaves, int iters,
                     std::vector<unsigned long long> &host, unsigned long long &dc,
                     unsigned long long &dw) {
  hipLaunchKernelGGL(engine_clock_kernel, dim3(blocks), dim3(64 * kWavesPerBlock), 0, nullptr, dev,
                     iters, nwaves);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess)
    e = hipMemcpy(host.data(), dev, sizeof(unsigned long long) * 2 * (size_t)nwaves,
                  hipMemcpyDeviceToHost);
  dc = dw = 0;
  if (e == hipSuccess) {
    for (int w = 0; w < nwaves; ++w) {
      dc += host[2 * (size_t)w];
      dw += host[2 * (size_t)w + 1];
    }
  }
  return e;
}

}  // namespace
}  // namespace dqj

using namespace dqj;

extern "C" dqj_status dqj_measure_engine_clock(int32_t device, double seconds, double *mhz) {
  try {
    if (!mhz) return fail(DQJ_E_INVALID, "mhz is NULL");
    if (!(seconds > 0.0 && seconds <= 10.0))
      return fail(DQJ_E_INVALID, "seconds must lie in (0, 10], got %g", seconds);
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= count) return fail(DQJ_E_INVALID, "no device %d", device);
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
      return fail(DQJ_E_UNSUPPORTED, "device %d is '%s', not gfx950", device, prop.gcnArchName);
    int wall_khz = 0;
    e = hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, device);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute(WallClockRate)");
    if (wall_khz <= 0) return fail(DQJ_E_DEVICE, "device %d reports no wall clock rate", device);

    int prev = 0;
    e = hipGetDevice(&prev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    e = hipSetDevice(device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const int blocks = prop.multiProcessorCount * kBlocksPerCu;
    const int nwaves = blocks * kWavesPerBlock;
    unsigned long long *dev = nullptr;
    e = hipMalloc(&dev, sizeof(unsigned long long) * (2 * (size_t)nwaves + 1));
    if (e != hipSuccess) {
      (void)hipSetDevice(prev);
      return fail(DQJ_E_NOMEM, "hipMalloc of the clock probe's buffer failed");
    }
    std::vector<unsigned long long> host(2 * (size_t)nwaves);
    unsigned long long dc = 0, dw = 0;
    // a short launch sets the loop count for the requested length
    const int iters0 = 2000;
    e = run_probe(dev, blocks, nwaves, iters0, host, dc, dw);
    double result = 0.0;
    if (e == hipSuccess && dw > 0) {
      const double per_iter_s = (double)dw / nwaves / (wall_khz * 1e3) / iters0;
      double n = seconds / per_iter_s;
      if (n < iters0) n = iters0;
      if (n > 3e7) n = 3e7;   // about 10 s at the expected rate, whatever the clocks report
      e = run_probe(dev, blocks, nwaves, (int)n, host, dc, dw);
      if (e == hipSuccess && dw > 0) result = (double)dc / (double)dw * (wall_khz * 1e-3);
    }
    (void)hipFree(dev);
    (void)hipSetDevice(prev);
    if (e != hipSuccess) return hip_fail(e, "engine clock probe");
    if (!(result > 0.0)) return fail(DQJ_E_DEVICE, "engine clock probe measured no time");
    *mhz = result;
    return DQJ_OK;
  } catch (const std::bad_alloc &) {
    return fail(DQJ_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(DQJ_E_DEVICE, "unexpected internal error");
  }
}
