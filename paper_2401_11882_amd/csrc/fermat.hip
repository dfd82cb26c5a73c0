// Forward kernel of Fermat path tracing (Sec. V-B): power and loss partials
// of one scene, with the interaction points of order-1 and order-2
// candidates found by Newton on the path length (fermat.h) instead of the
// image method; line-of-sight paths are the same for both finders.
//
// Work decomposition as in k_forward: a workgroup owns a tile of 64
// receivers, its NW wavefronts take candidates c = w, w + NW, ...; one lane
// per receiver, candidate and wall wave-uniform.  No candidate screen,
// contribution cut or cache: every candidate is evaluated (the obstruction
// tests keep the exact culling and band skips of the image-method kernels).
// Per-lane sums are Kahan-compensated, cross-wave sums in a fixed order.
#include "fermat.h"
#include "trace.h"
#include "view.h"

namespace drt {

template <int NW, int MODE>
__global__ __launch_bounds__(NW * kWave) void k_forward_fermat(TraceArgs A, float* __restrict__ power,
                                                                float* __restrict__ loss_part, int loss_kind,
                                                                float log_eps, int max_iter, float inv_eps) {
  __shared__ float red[NW][2][kWave];
  const SceneView S = view_of(A);
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = uniform(threadIdx.x >> 6);
  const int tile = blockIdx.x;
  const int m = rx_of_lane(tile, lane, A.grid_nx);
  const bool live = m < A.n_rx;
  float rxx, rxy;
  receiver_of(A, m, live, rxx, rxy);
  const float txx = A.tx[0], txy = A.tx[1];
  float sum = 0.0f, comp = 0.0f;
#pragma unroll 1
  for (int c = wave; c < A.n_cand; c += NW) {
    const Cand cd = decode_candidate(c, A.n_walls);
    float v;
    if (cd.k == 0) v = path_power<0, MODE>(S, cd, txx, txy, rxx, rxy, live);
    else if (cd.k == 1) v = fermat_power<1, MODE>(S, cd, txx, txy, rxx, rxy, live, max_iter, inv_eps);
    else v = fermat_power<2, MODE>(S, cd, txx, txy, rxx, rxy, live, max_iter, inv_eps);
    kahan_add(sum, comp, v);
  }
  red[wave][0][lane] = sum;
  red[wave][1][lane] = comp;
  __syncthreads();
  if (wave == 0) {
    float s = 0.0f, cs = 0.0f;
#pragma unroll
    for (int w = 0; w < NW; ++w) kahan_add(s, cs, red[w][0][lane] - red[w][1][lane]);
    const float P = s - cs;
    float lp = 0.0f;
    if (live) {
      power[m] = P;
      if (loss_kind == 1) lp = P;
      else if (loss_kind == 2) lp = logf(P + log_eps);
    }
    if (loss_kind != 0) {
      const float tot = wave_sum(lp);
      if (lane == 0) loss_part[tile] = tot;
    }
  }
}

template <int NW>
static hipError_t fermat_nw(const TraceArgs& A, int n_tiles, float* power, float* loss_part, int loss_kind,
                            float log_eps, int max_iter, float inv_eps, hipStream_t st) {
  if (A.mode)
    hipLaunchKernelGGL((k_forward_fermat<NW, 1>), dim3(n_tiles), dim3(NW * kWave), 0, st, A, power, loss_part,
                       loss_kind, log_eps, max_iter, inv_eps);
  else
    hipLaunchKernelGGL((k_forward_fermat<NW, 0>), dim3(n_tiles), dim3(NW * kWave), 0, st, A, power, loss_part,
                       loss_kind, log_eps, max_iter, inv_eps);
  return hipGetLastError();
}

hipError_t launch_forward_fermat(const TraceArgs& A, int n_tiles, int nw, float* power, float* loss_part,
                                 int loss_kind, float log_eps, int max_iter, float inv_eps, hipStream_t st) {
  switch (nw) {
    case 2: return fermat_nw<2>(A, n_tiles, power, loss_part, loss_kind, log_eps, max_iter, inv_eps, st);
    case 4: return fermat_nw<4>(A, n_tiles, power, loss_part, loss_kind, log_eps, max_iter, inv_eps, st);
    case 8: return fermat_nw<8>(A, n_tiles, power, loss_part, loss_kind, log_eps, max_iter, inv_eps, st);
    case 16: return fermat_nw<16>(A, n_tiles, power, loss_part, loss_kind, log_eps, max_iter, inv_eps, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace drt
