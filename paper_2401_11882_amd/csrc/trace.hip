// Smoothed image-method tracer: forward, hand-written adjoint and the small
// reductions around them, for gfx950 (wave64).
//
// Work decomposition.  A workgroup owns one tile of 64 receivers (an 8x8
// block of a grid, or 64 consecutive receivers); its NW wavefronts split the
// candidate list (wave w takes chunks w, w+NW, ... of `cchunk` candidates).
// Inside a wavefront every lane is one receiver while the candidate and the
// wall being tested are wave-uniform, so wall records come in through scalar
// loads and candidate bookkeeping runs on the scalar unit.  Because a
// workgroup sees every candidate of its receivers, the power P(r) is complete
// at the end of the workgroup and the loss seed dL/dP(r) is formed there.
//
// Exact work skipping (no change to the FP32 result):
//  * a candidate whose interaction factor is exactly 0 in every lane (the
//    reflection points are far outside their segments, so an exponential
//    overflows and the reciprocal of the product is 0) skips all obstruction
//    tests, usually before any exponential is evaluated;
//  * an obstruction test whose leg and wall parameters are more than 18/alpha
//    outside [0, 1] has in(tau) in(upsilon) < 2^-25, so its factor rounds to
//    1.0f; it is decided on numerators before any reciprocal or exponential,
//    the wall parameter first, so a wavefront skips the rest of the test when
//    no lane is in the band.
//
// Contribution cache.  The forward kernel can record, per wavefront, the
// list of candidates with a nonzero contribution and the 64 per-lane values
// c = V / max(d^2, d_min^2).  The adjoint then needs only g(r) * c to start
// its reverse sweep, so it visits just those candidates and does not
// re-evaluate the forward.  A wavefront whose list would exceed the capacity
// marks it as overflowed and the adjoint re-evaluates that wavefront's
// candidates instead.
//
// Numerics.  in(x) = s(ax) s(a(1-x)) = 1 / ((1+E1)(1+E2)) with
// E1 = exp(-a x), E2 = exp(-a (1-x)).  An obstruction factor
// 1 - in(tau) in(ups) is formed as num / (1 + num) with
// num = n_t + n_u + n_t n_u, n_t = E1 + E2 + E1 E2: every term is positive,
// so deep shadows keep full relative precision.  Per-lane power sums over
// candidates are Kahan-compensated; every cross-lane / cross-wave /
// cross-block sum has a fixed order.
#include "path.h"
#include "screen.h"
#include "trace.h"
#include "view.h"

namespace drt {

// ---------------------------------------------------------------------------
// Forward kernel
// ---------------------------------------------------------------------------

template <int NW, int MODE, int MAXK>
__global__ __launch_bounds__(NW * kWave) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_forward(TraceArgs A, float* __restrict__ power,
                                                        float* __restrict__ seed,
                                                        float* __restrict__ loss_part, int loss_kind,
                                                        float log_eps) {
  __shared__ float red[NW][2][kWave];
  __shared__ float base[2][NW][kWave];  // each wavefront's power sum at the end of a phase
  extern __shared__ float fwd_boxes[];  // [NW][6 (max_order + 1)][64] leg boxes of screened candidates
  const SceneView S = view_of(A);
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = uniform(threadIdx.x >> 6);
  const int tile = blockIdx.x;
  const int m = rx_of_lane(tile, lane, A.grid_nx);
  const bool live = m < A.n_rx;
  float rxx, rxy;
  receiver_of(A, m, live, rxx, rxy);
  const float txx = A.tx[0], txy = A.tx[1];

  const int slot = tile * NW + wave;
  float* cache_c = A.cache_c ? A.cache_c + (size_t)slot * A.cache_cap * kWave : nullptr;
  int* cache_idx = A.cache_c ? A.cache_idx + (size_t)slot * A.cache_cap : nullptr;
  int nst = 0;

  float sum = 0.0f, comp = 0.0f;
  const RxBox box = rx_box(rxx, rxy, live);
  float* boxes = fwd_boxes + wave * 6 * (A.max_order + 1) * kWave;
  // The contribution cut compares each candidate with a lower bound of the
  // lane's P(r): the sum over all wavefronts at the end of the previous phase
  // (orders 0-1, then order 2 for order-3 scenes; shared through LDS), plus
  // this wavefront's own running sum since then.
  float cut_base = 0.0f, own_sync = 0.0f;
  auto visit = [&](int c, const Cand& cd, const float* Ix, const float* Iy, int j) {
    const float v = candidate_power_img<MODE, MAXK>(S, cd, Ix, Iy, txx, txy, rxx, rxy, live, boxes, j,
                                                    A.cut * (cut_base + (sum - comp) - own_sync));
    kahan_add(sum, comp, v);
    if (cache_c && ballot(v != 0.0f) != 0) {
      if (nst < A.cache_cap) {
        cache_c[(size_t)nst * kWave + lane] = v;
        if (lane == 0) cache_idx[nst] = c;
        if (lane < A.box_stride)
          A.cache_box[((size_t)slot * A.cache_cap + nst) * A.box_stride + lane] = boxes[lane * kWave + j];
      }
      ++nst;
    }
  };
  if constexpr (!uses_cut<MODE>()) {
    for_screened<MAXK>(S.walls, A.n_walls, 0, A.n_cand, S.dead_lim, A.screen != 0, wave, NW, A.cchunk, txx, txy,
                       box, S.cull_c, boxes, visit);
  } else {
    // one copy of the candidate code serves every phase (the loop is not
    // unrolled); base is double-buffered, so one barrier per phase suffices
    const CutPhases cp = cut_phases(A.n_walls, A.max_order, A.n_cand);
#pragma nounroll
    for (int ph = 0; ph < cp.n; ++ph) {
      const int b0 = ph == 0 ? 0 : (ph == 1 ? cp.end0 : cp.end1);
      const int b1 = ph == 0 ? cp.end0 : (ph == 1 ? cp.end1 : A.n_cand);
      for_screened<MAXK>(S.walls, A.n_walls, b0, b1, S.dead_lim, A.screen != 0, wave, NW, A.cchunk, txx, txy,
                         box, S.cull_c, boxes, visit);
      if (ph + 1 < cp.n) {
        own_sync = sum - comp;
        base[ph & 1][wave][lane] = own_sync;
        __syncthreads();
        float t = 0.0f;
#pragma unroll
        for (int w = 0; w < NW; ++w) t += base[ph & 1][w][lane];
        cut_base = t;
      }
    }
  }
  if (cache_c && lane == 0) A.cache_n[slot] = nst <= A.cache_cap ? nst : -1;
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
      if (loss_kind == 1) {
        lp = P;
        if (seed) seed[m] = 1.0f;
      } else if (loss_kind == 2) {
        lp = logf(P + log_eps);
        if (seed) seed[m] = -1.0f / ((float)A.n_rx * (P + log_eps));
      }
    }
    if (loss_kind != 0) {
      const float tot = wave_sum(lp);
      if (lane == 0) loss_part[tile] = tot;
    }
  }
}

// ---------------------------------------------------------------------------
// Adjoint kernel
// ---------------------------------------------------------------------------

template <int NW, int MODE>
__global__ __launch_bounds__(NW * kWave) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_backward(TraceArgs A, const float* __restrict__ gP,
                                                         float* __restrict__ part,
                                                         float* __restrict__ grad_rx, int reuse) {
  extern __shared__ float smem[];
  const SceneView S = view_of(A);
  const int ncol = 2 + 4 * A.n_walls;
  float* accs = smem;                           // [NW][ncol]
  float* rxr = smem + NW * ncol;                // [NW][2][64]
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = uniform(threadIdx.x >> 6);
  for (int i = threadIdx.x; i < NW * ncol; i += NW * kWave) accs[i] = 0.0f;
  __syncthreads();
  float* acc = accs + wave * ncol;

  const int tile = blockIdx.x;
  const int m = rx_of_lane(tile, lane, A.grid_nx);
  const bool live = m < A.n_rx;
  float rxx, rxy;
  receiver_of(A, m, live, rxx, rxy);
  const float g = live ? gP[m] : 0.0f;
  const float txx = A.tx[0], txy = A.tx[1];
  LaneGrad G{0.0f, 0.0f, 0.0f, 0.0f};

  if (ballot(g != 0.0f) != 0) {
    const int slot = tile * NW + wave;
    const int n_cached = (reuse && A.cache_c) ? A.cache_n[slot] : -1;
    if (n_cached >= 0) {
      const float* cache_c = A.cache_c + (size_t)slot * A.cache_cap * kWave;
      const int* cache_idx = A.cache_idx + (size_t)slot * A.cache_cap;
      for (int p = 0; p < n_cached; ++p) {
        const int c = cache_idx[p];
        const float Wl = g * cache_c[(size_t)p * kWave + lane];
        if (ballot(Wl != 0.0f) == 0) continue;
        const Cand cd = decode_candidate(c, A.n_walls);
        const float* gbox = A.cache_box + ((size_t)slot * A.cache_cap + p) * A.box_stride;
        candidate_adjoint_known<MODE>(S, cd, txx, txy, rxx, rxy, live, Wl, acc, lane, G, gbox);
      }
    } else {
      // re-evaluation of this wavefront's share as the forward split it into
      // phases, the cut against its own running sum
      float sum = 0.0f, comp = 0.0f;
      const CutPhases cp = cut_phases(A.n_walls, A.max_order, A.n_cand);
      const int nph = uses_cut<MODE>() ? cp.n : 1;
      const int stride = NW * A.cchunk;
      for (int part = 0; part < nph; ++part) {
        const int b0 = part == 0 ? 0 : (part == 1 ? cp.end0 : cp.end1);
        const int b1 = !uses_cut<MODE>() ? A.n_cand : (part == 0 ? cp.end0 : (part == 1 ? cp.end1 : A.n_cand));
        for (int c0 = b0 + wave * A.cchunk; c0 < b1; c0 += stride) {
          const int c1 = min(c0 + A.cchunk, b1);
          for (int c = c0; c < c1; ++c) {
            const Cand cd = decode_candidate(c, A.n_walls);
            kahan_add(sum, comp,
                      candidate_adjoint<MODE>(S, cd, txx, txy, rxx, rxy, live, g, acc, lane, G, A.cut * (sum - comp)));
          }
        }
      }
    }
  }
  {
    const float sx = wave_sum(G.tx_x), sy = wave_sum(G.tx_y);
    if (lane == 0) {
      acc[0] += sx;
      acc[1] += sy;
    }
  }
  rxr[(wave * 2 + 0) * kWave + lane] = G.rx_x;
  rxr[(wave * 2 + 1) * kWave + lane] = G.rx_y;
  __syncthreads();
  if (wave == 0 && live && grad_rx) {
    float sx = 0.0f, sy = 0.0f;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      sx += rxr[(w * 2 + 0) * kWave + lane];
      sy += rxr[(w * 2 + 1) * kWave + lane];
    }
    grad_rx[2 * m] = sx;
    grad_rx[2 * m + 1] = sy;
  }
  for (int col = threadIdx.x; col < ncol; col += NW * kWave) {
    float s = 0.0f;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += accs[w * ncol + col];
    part[(size_t)tile * ncol + col] = s;
  }
}

// ---------------------------------------------------------------------------
// Small kernels
// ---------------------------------------------------------------------------

// Wall records and culling data (see make_wall).
__global__ void k_prep_walls(const float* __restrict__ walls, int n, float c, WallRec* __restrict__ out,
                             WallBox* __restrict__ boxes) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  WallRec r;
  WallBox q;
  make_wall(walls[4 * j], walls[4 * j + 1], walls[4 * j + 2], walls[4 * j + 3], c, r, q);
  out[j] = r;
  boxes[j] = q;
}

// Column sums of part[n_rows][ncol] in FP64 with a fixed order: a workgroup
// of 1024 threads owns 32 columns; 32 row-groups each sum a strided row
// subset, then the 32 partials are added in order.
__global__ __launch_bounds__(1024) void k_reduce_cols(const float* __restrict__ part, int n_rows,
                                                      int ncol, float* __restrict__ out_head,
                                                      int n_head, float* __restrict__ out_tail) {
  __shared__ double sh[32][32];
  const int cl = threadIdx.x & 31, rg = threadIdx.x >> 5;
  const int col = blockIdx.x * 32 + cl;
  double s = 0.0;
  if (col < ncol) {
#pragma unroll 4
    for (int b = rg; b < n_rows; b += 32) s += (double)part[(size_t)b * ncol + col];
  }
  sh[rg][cl] = s;
  __syncthreads();
  if (rg == 0 && col < ncol) {
    double t = 0.0;
#pragma unroll
    for (int g = 0; g < 32; ++g) t += sh[g][cl];
    if (col < n_head) out_head[col] = (float)t;
    else out_tail[col - n_head] = (float)t;
  }
}

// scale * sum(part[0..n)) in FP64 with a fixed tree order; one block of 256.
__global__ void k_reduce_scalar(const float* __restrict__ part, int n, double scale,
                                float* __restrict__ out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += (double)part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = (float)(scale * sh[0]);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

hipError_t launch_prep_walls(const float* walls, int n, float cull_c, WallRec* out, WallBox* boxes,
                             hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_prep_walls, dim3((n + 255) / 256), dim3(256), 0, st, walls, n, cull_c, out,
                     boxes);
  return hipGetLastError();
}

template <int NW, int MAXK>
static void fwd_launch(const TraceArgs& A, int n_tiles, size_t lds, float* power, float* seed, float* loss_part,
                       int loss_kind, float log_eps, hipStream_t st) {
  if (A.mode)
    hipLaunchKernelGGL((k_forward<NW, 1, MAXK>), dim3(n_tiles), dim3(NW * kWave), lds, st, A, power, seed,
                       loss_part, loss_kind, log_eps);
  else
    hipLaunchKernelGGL((k_forward<NW, 0, MAXK>), dim3(n_tiles), dim3(NW * kWave), lds, st, A, power, seed,
                       loss_part, loss_kind, log_eps);
}

template <int NW>
static hipError_t fwd_nw(const TraceArgs& A, int n_tiles, float* power, float* seed, float* loss_part,
                         int loss_kind, float log_eps, hipStream_t st) {
  const size_t lds = forward_lds_bytes(NW, A.max_order) - sizeof(float) * NW * 2 * kWave;  // minus static
  // scenes up to order 2 run a kernel without the order-3 path code
  if (A.max_order <= 2) fwd_launch<NW, 2>(A, n_tiles, lds, power, seed, loss_part, loss_kind, log_eps, st);
  else fwd_launch<NW, 3>(A, n_tiles, lds, power, seed, loss_part, loss_kind, log_eps, st);
  return hipGetLastError();
}

hipError_t launch_forward(const TraceArgs& A, int n_tiles, int nw, float* power, float* seed,
                          float* loss_part, int loss_kind, float log_eps, hipStream_t st) {
  switch (nw) {
    case 2: return fwd_nw<2>(A, n_tiles, power, seed, loss_part, loss_kind, log_eps, st);
    case 4: return fwd_nw<4>(A, n_tiles, power, seed, loss_part, loss_kind, log_eps, st);
    case 8: return fwd_nw<8>(A, n_tiles, power, seed, loss_part, loss_kind, log_eps, st);
    case 16: return fwd_nw<16>(A, n_tiles, power, seed, loss_part, loss_kind, log_eps, st);
    default: return hipErrorInvalidValue;
  }
}

size_t forward_lds_bytes(int nw, int max_order) {
  return sizeof(float) * ((size_t)nw * 6 * (max_order + 1) * kWave + (size_t)nw * 2 * kWave);
}

size_t backward_lds_bytes(int nw, int n_walls) {
  return sizeof(float) * ((size_t)nw * (2 + 4 * (size_t)n_walls) + (size_t)nw * 2 * kWave);
}

template <int NW>
static hipError_t bwd_nw(const TraceArgs& A, int n_tiles, const float* gP, float* part, float* grad_rx,
                         int reuse, hipStream_t st) {
  const size_t lds = backward_lds_bytes(NW, A.n_walls);
  if (A.mode)
    hipLaunchKernelGGL((k_backward<NW, 1>), dim3(n_tiles), dim3(NW * kWave), lds, st, A, gP, part, grad_rx,
                       reuse);
  else
    hipLaunchKernelGGL((k_backward<NW, 0>), dim3(n_tiles), dim3(NW * kWave), lds, st, A, gP, part, grad_rx,
                       reuse);
  return hipGetLastError();
}

hipError_t launch_backward(const TraceArgs& A, int n_tiles, int nw, const float* gP, float* part,
                           float* grad_rx, int reuse, hipStream_t st) {
  switch (nw) {
    case 2: return bwd_nw<2>(A, n_tiles, gP, part, grad_rx, reuse, st);
    case 4: return bwd_nw<4>(A, n_tiles, gP, part, grad_rx, reuse, st);
    case 8: return bwd_nw<8>(A, n_tiles, gP, part, grad_rx, reuse, st);
    case 16: return bwd_nw<16>(A, n_tiles, gP, part, grad_rx, reuse, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_reduce_cols(const float* part, int n_rows, int ncol, float* out_head, int n_head,
                              float* out_tail, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_cols, dim3((ncol + 31) / 32), dim3(1024), 0, st, part, n_rows, ncol,
                     out_head, n_head, out_tail);
  return hipGetLastError();
}

hipError_t launch_reduce_scalar(const float* part, int n, double scale, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_scalar, dim3(1), dim3(256), 0, st, part, n, scale, out);
  return hipGetLastError();
}

}  // namespace drt
