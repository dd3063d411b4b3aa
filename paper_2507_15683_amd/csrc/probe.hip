// Issue-rate probe for the VALU roofline: independent chains of FP32 fused
// multiply-adds (no packed forms), timed with events on the given stream.
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace hgsr {

constexpr int kProbeChains = 32;  // FMAs per loop iteration, each on its own accumulator

__global__ __launch_bounds__(256) void valu_probe_kernel(float* out, int iters, float scale) {
  // the multiplier is a per-lane value, as in the kernels the probe stands
  // for (a scalar operand measured a third slower)
  const float w = scale * static_cast<float>(threadIdx.x + 1);
  float a[kProbeChains];
#pragma unroll
  for (int d = 0; d < kProbeChains; ++d) a[d] = static_cast<float>(threadIdx.x + d) * 1e-3f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int d = 0; d < kProbeChains; ++d) a[d] = fmaf(w, a[(d + 1) % kProbeChains], a[d]);
  }
  float t = 0.f;
#pragma unroll
  for (int d = 0; d < kProbeChains; ++d) t += a[d];
  out[blockIdx.x * 256 + threadIdx.x] = t;
}

hipError_t probe_valu_rate(int n_cu, hipStream_t s, double* wave_fma_per_s) {
  const int blocks = 8 * n_cu, iters = 4000;
  float* out = nullptr;
  hipError_t e = hipMalloc(&out, static_cast<size_t>(blocks) * 256 * sizeof(float));
  if (e != hipSuccess) return e;
  hipEvent_t a = nullptr, b = nullptr;
  if ((e = hipEventCreate(&a)) != hipSuccess || (e = hipEventCreate(&b)) != hipSuccess) {
    (void)hipFree(out);
    return e;
  }
  // three launches to bring the clock up, then the best of three timed ones
  for (int w = 0; w < 3; ++w)
    hipLaunchKernelGGL(valu_probe_kernel, dim3(blocks), dim3(256), 0, s, out, iters, 1e-9f);
  float best = 0.f;
  for (int t = 0; t < 3 && e == hipSuccess; ++t) {
    (void)hipEventRecord(a, s);
    hipLaunchKernelGGL(valu_probe_kernel, dim3(blocks), dim3(256), 0, s, out, iters, 1e-9f);
    (void)hipEventRecord(b, s);
    e = hipEventSynchronize(b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (e == hipSuccess && (best == 0.f || ms < best)) best = ms;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipFree(out);
  if (e != hipSuccess) return e;
  const double ms = best;
  const double waves = static_cast<double>(blocks) * 4;
  *wave_fma_per_s = waves * iters * kProbeChains / (ms * 1e-3);
  return hipSuccess;
}

}  // namespace hgsr
