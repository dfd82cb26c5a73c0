// Adam steps on points (transmitter positions) with a clamp to the box, and
// the geometric sharpness schedule of the transmitter optimisation.
#include "dev.h"
#include "trace.h"

namespace drt {

// One workgroup: every thread reads the old step count, updates its share of
// the n coordinates, and thread 0 writes the new count after a barrier.
__global__ __launch_bounds__(256) void k_adam_points(int n, float* __restrict__ x, const float* __restrict__ g,
                                                     float* __restrict__ m, float* __restrict__ v,
                                                     int32_t* __restrict__ step, float lr, float b1, float b2,
                                                     float eps, float lo, float hi) {
  const int t = step[0] + 1;
  const float bc1 = 1.0f - powf(b1, (float)t);
  const float bc2 = 1.0f - powf(b2, (float)t);
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float denom = sqrtf(vi) / sqrtf(bc2) + eps;
    const float xi = x[i] - (lr / bc1) * (mi / denom);
    x[i] = fminf(fmaxf(xi, lo), hi);
  }
  __syncthreads();
  if (threadIdx.x == 0) step[0] = t;
}

__global__ __launch_bounds__(256) void k_alpha_schedule(const int32_t* __restrict__ step, int n_iter, float a_first,
                                                        float a_last, float* __restrict__ alpha, int n) {
  const int i = min(max(step[0], 0), n_iter - 1);
  const float f = (float)i / (float)(n_iter - 1);
  const float a = a_first * exp2f(f * log2f(a_last / a_first));
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) alpha[j] = a;
}

// L = -min P and its seed: one workgroup finds the minimum and the lowest
// index attaining it (both independent of the reduction order), then writes
// -1 there and 0 elsewhere.
__global__ __launch_bounds__(1024) void k_min_seed(const float* __restrict__ P, int n, float* __restrict__ loss,
                                                   float* __restrict__ seed) {
  __shared__ float sv[1024];
  __shared__ int si[1024];
  float best = __builtin_inff();
  int bi = 0x7fffffff;
  for (int i = threadIdx.x; i < n; i += 1024) {
    const float p = P[i];
    if (p < best) {  // increasing i per thread: the first index of a tie stays
      best = p;
      bi = i;
    }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const float o = sv[threadIdx.x + w];
      const int oi = si[threadIdx.x + w];
      if (o < sv[threadIdx.x] || (o == sv[threadIdx.x] && oi < si[threadIdx.x])) {
        sv[threadIdx.x] = o;
        si[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const int am = si[0];
  if (threadIdx.x == 0 && loss) loss[0] = -sv[0];
  if (seed)
    for (int i = threadIdx.x; i < n; i += 1024) seed[i] = i == am ? -1.0f : 0.0f;
}

hipError_t launch_adam_points(int n, float* x, const float* grad, float* m, float* v, int32_t* step, float lr,
                              float b1, float b2, float eps, float lo, float hi, hipStream_t st) {
  hipLaunchKernelGGL(k_adam_points, dim3(1), dim3(256), 0, st, n, x, grad, m, v, step, lr, b1, b2, eps, lo, hi);
  return hipGetLastError();
}

hipError_t launch_alpha_schedule(const int32_t* step, int n_iter, float a_first, float a_last, float* alpha, int n,
                                 hipStream_t st) {
  const int blocks = (n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024;
  hipLaunchKernelGGL(k_alpha_schedule, dim3(blocks), dim3(256), 0, st, step, n_iter, a_first, a_last, alpha, n);
  return hipGetLastError();
}

hipError_t launch_min_seed(const float* power, int n, float* loss, float* seed, hipStream_t st) {
  hipLaunchKernelGGL(k_min_seed, dim3(1), dim3(1024), 0, st, power, n, loss, seed);
  return hipGetLastError();
}

}  // namespace drt
