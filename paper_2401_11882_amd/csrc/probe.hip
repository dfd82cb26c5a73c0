// Sustained VALU rates of the device, for the roofline context of the
// tracer kernels: plain FP32 FMA chains and v_exp_f32 chains, 16 (FMA) or 8
// (exp) independent chains per lane over a grid that fills every CU.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>

#include "../../include/drt.h"

extern "C" __attribute__((visibility("hidden"))) int drt_internal_fail(int code, const char* msg);

namespace {

constexpr int kIters = 2048;
constexpr int kBlocks = 8192;
constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void k_probe_fma(float* out, float a) {
  float x[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) x[i] = threadIdx.x * 1e-3f + i;
  for (int it = 0; it < kIters; ++it) {
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = fmaf(x[i], a, 0.25f);
  }
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < 16; ++i) s += x[i];
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_probe_exp(float* out) {
  float x[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) x[i] = -1.0f - threadIdx.x * 1e-6f - i * 0.01f;
  for (int it = 0; it < kIters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = -__builtin_amdgcn_exp2f(x[i]);  // stays in [-1, -0.5]
  }
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += x[i];
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

int fail_hip(hipError_t e, const char* what) {
  char buf[256];
  snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
  return drt_internal_fail(DRT_EHIP, buf);
}

}  // namespace

extern "C" int drt_valu_peak(double* fma_tflops, double* exp_tlanes) {
  if (!fma_tflops || !exp_tlanes) return drt_internal_fail(DRT_EINVAL, "NULL output pointer");
  float* d = nullptr;
  hipError_t e = hipMalloc(&d, sizeof(float) * kBlocks * kThreads);
  if (e != hipSuccess) return fail_hip(e, "probe buffer");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double best_fma = 0.0, best_exp = 0.0;
  if ((e = hipEventCreate(&e0)) == hipSuccess && (e = hipEventCreate(&e1)) == hipSuccess) {
    const double lanes = (double)kBlocks * kThreads * kIters;
    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
      for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        float ms = 0.0f;
        (void)hipEventRecord(e0, nullptr);
        if (k == 0) hipLaunchKernelGGL(k_probe_fma, dim3(kBlocks), dim3(kThreads), 0, nullptr, d, 0.5f);
        else hipLaunchKernelGGL(k_probe_exp, dim3(kBlocks), dim3(kThreads), 0, nullptr, d);
        if ((e = hipGetLastError()) != hipSuccess) break;
        (void)hipEventRecord(e1, nullptr);
        if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
        if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
        if (k == 0) best_fma = fmax(best_fma, 2.0 * 16.0 * lanes / (ms * 1e-3) / 1e12);
        else best_exp = fmax(best_exp, 8.0 * lanes / (ms * 1e-3) / 1e12);
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(d);
  if (e != hipSuccess) return fail_hip(e, "probe run");
  *fma_tflops = best_fma;
  *exp_tlanes = best_exp;
  return DRT_OK;
}
