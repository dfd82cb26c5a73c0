// Adam step on the transmitter position followed by a clamp to the box.
#include "dev.h"
#include "trace.h"

namespace drt {

__global__ void k_adam_tx(float* __restrict__ x, const float* __restrict__ g, float* __restrict__ m,
                          float* __restrict__ v, int32_t* __restrict__ step, float lr, float b1,
                          float b2, float eps, float lo, float hi) {
  const int i = threadIdx.x;
  const int t = step[0] + 1;  // every lane reads the old count before lane 0 writes
  if (i < 2) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float bc1 = 1.0f - powf(b1, (float)t);
    const float bc2 = 1.0f - powf(b2, (float)t);
    const float denom = sqrtf(vi) / sqrtf(bc2) + eps;
    const float xi = x[i] - (lr / bc1) * (mi / denom);
    x[i] = fminf(fmaxf(xi, lo), hi);
  }
  __syncthreads();
  if (i == 0) step[0] = t;
}

hipError_t launch_adam_tx(float* tx, const float* grad, float* m, float* v, int32_t* step, float lr,
                          float b1, float b2, float eps, float lo, float hi, hipStream_t st) {
  hipLaunchKernelGGL(k_adam_tx, dim3(1), dim3(64), 0, st, tx, grad, m, v, step, lr, b1, b2, eps, lo, hi);
  return hipGetLastError();
}

}  // namespace drt
