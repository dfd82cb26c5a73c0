// 3D scenes of parallelogram panels: forward, adjoint and the per-panel
// gradient map, for gfx950 (wave64).  Same decomposition as the 2D tracer: a
// workgroup owns 64 receivers, its wavefronts split the candidates, every
// lane is one receiver, and the candidate and the panel under test are
// wave-uniform.  Exact skips: candidates screened out over the wavefront's
// receiver box (screen3.h); a candidate whose interaction factor is 0 in
// every lane stops before its exponentials; an obstruction test whose leg
// parameter, or panel coordinates, lie more than 18/alpha outside [0, 1] has
// the factor 1.0f and is skipped wave-wide; a candidate whose lanes are all
// fully blocked stops its panel loop.
#include "path3d.h"
#include "screen3.h"
#include "trace.h"
#include "trace3d.h"

namespace drt {

__device__ __forceinline__ Scene3View view3_of(const Trace3Args& A) {
  Scene3View S;
  S.panels = A.panels;
  S.boxes = A.boxes;
  S.cull_c = A.cull_c;
  S.n_panels = A.n_panels;
  S.mask_nb = A.mask_nb;
  S.alpha = A.alpha;
  S.a2 = A.a2;
  S.band_k = A.band_k;
  S.dmin2 = A.dmin2;
  S.a6 = A.alpha * (1.0f / 6.0f);
  S.a6h = S.a6 + 0.5f;
  S.a6m = 0.5f - S.a6;
  return S;
}

// Panel records and culling boxes from the corners (a, b, c).
__global__ void k_prep_panels(const float* __restrict__ pan, int n, float cull_c, PanelRec* __restrict__ out,
                              PanelBox* __restrict__ boxes) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const float* p = pan + 9 * (size_t)j;
  const float ax = p[0], ay = p[1], az = p[2];
  const float e1x = p[3] - ax, e1y = p[4] - ay, e1z = p[5] - az;
  const float e2x = p[6] - ax, e2y = p[7] - ay, e2z = p[8] - az;
  const float nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
  const float N = nx * nx + ny * ny + nz * nz;
  const float s = N > 0.0f ? 1.0f / N : 0.0f;
  PanelRec r;
  r.ax = ax;
  r.ay = ay;
  r.az = az;
  r.nx = nx;
  r.ny = ny;
  r.nz = nz;
  // m1 = (e2 x n) s, m2 = (n x e1) s
  r.m1x = (e2y * nz - e2z * ny) * s;
  r.m1y = (e2z * nx - e2x * nz) * s;
  r.m1z = (e2x * ny - e2y * nx) * s;
  r.m2x = (ny * e1z - nz * e1y) * s;
  r.m2y = (nz * e1x - nx * e1z) * s;
  r.m2z = (nx * e1y - ny * e1x) * s;
  r.s = s;
  r.nda = nx * ax + ny * ay + nz * az;
  r.pad0 = r.pad1 = 0.0f;
  out[j] = r;
  if (!boxes) return;
  // extended parallelogram a - c (e1 + e2) + [0, 1 + 2c] e1 + [0, 1 + 2c] e2
  const float k = 1.0f + 2.0f * cull_c;
  const float q0x = ax - cull_c * (e1x + e2x), q0y = ay - cull_c * (e1y + e2y), q0z = az - cull_c * (e1z + e2z);
  const float lox = q0x + fminf(0.0f, k * e1x) + fminf(0.0f, k * e2x);
  const float loy = q0y + fminf(0.0f, k * e1y) + fminf(0.0f, k * e2y);
  const float loz = q0z + fminf(0.0f, k * e1z) + fminf(0.0f, k * e2z);
  const float hix = q0x + fmaxf(0.0f, k * e1x) + fmaxf(0.0f, k * e2x);
  const float hiy = q0y + fmaxf(0.0f, k * e1y) + fmaxf(0.0f, k * e2y);
  const float hiz = q0z + fmaxf(0.0f, k * e1z) + fmaxf(0.0f, k * e2z);
  PanelBox q;
  q.cx = 0.5f * (lox + hix);
  q.cy = 0.5f * (loy + hiy);
  q.cz = 0.5f * (loz + hiz);
  const float hx = 0.5f * (hix - lox), hy = 0.5f * (hiy - loy), hz = 0.5f * (hiz - loz);
  q.hx = hx + 1e-5f * (fabsf(q.cx) + hx);
  q.hy = hy + 1e-5f * (fabsf(q.cy) + hy);
  q.hz = hz + 1e-5f * (fabsf(q.cz) + hz);
  if (!(N > 0.0f)) q.hx = q.hy = q.hz = -__builtin_inff();  // zero area: never tested
  q.nx = nx;
  q.ny = ny;
  q.nz = nz;
  q.nda = r.nda;
  q.scale = fabsf(ax) + fabsf(ay) + fabsf(az) + fabsf(e1x) + fabsf(e1y) + fabsf(e1z) + fabsf(e2x) + fabsf(e2y) +
            fabsf(e2z);
  q.pad = 0.0f;
  boxes[j] = q;
}

template <int NW, int MODE, int MAXK>
__global__ __launch_bounds__(NW * kWave) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_forward3(Trace3Args A, float* __restrict__ power,
                                                         float* __restrict__ seed, float* __restrict__ loss_part,
                                                         int loss_kind, float log_eps) {
  __shared__ float red[NW][2][kWave];
  __shared__ float base[NW][kWave];  // per-wave sums of orders 0-1
  __shared__ uint64_t mrec[NW][16];  // culling masks of the candidate being evaluated
  const Scene3View S = view3_of(A);
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = uniform(threadIdx.x >> 6);
  const int tile = blockIdx.x;
  const int m = rx_of_lane(tile, lane, A.grid_nx);
  const bool live = m < A.n_rx;
  const float rx = live ? A.rx[3 * m] : 0.5f, ry = live ? A.rx[3 * m + 1] : 0.5f, rz = live ? A.rx[3 * m + 2] : 0.5f;
  const float tx = A.tx[0], ty = A.tx[1], tz = A.tx[2];
  const int slot = tile * NW + wave;
  float* cache_c = A.cache_c ? A.cache_c + (size_t)slot * A.cache_cap * kWave : nullptr;
  int* cache_idx = A.cache_c ? A.cache_idx + (size_t)slot * A.cache_cap : nullptr;
  int nst = 0;
  float sum = 0.0f, comp = 0.0f;
  const RxBox3 box = rx_box3(rx, ry, rz, live);
  // parameter range beyond which an interaction factor is exactly 0
  const float lim = (MODE == kHardSigmoid ? kHardBandMargin / A.alpha : 128.0f / A.a2) * 1.00001f;
  // Contribution cut: every term is >= 0, so the orders 0-1 of all wavefronts
  // (summed through LDS after the first phase) plus this wavefront's running
  // sum of the later candidates bound P(r) from below.
  float cut_base = 0.0f, own1 = 0.0f;
  auto visit = [&](int c, const Cand& cd) {
    const float v = candidate_power3<MODE, MAXK>(S, cd, tx, ty, tz, rx, ry, rz, live, cache_c ? mrec[wave] : nullptr,
                                           A.cut * (cut_base + (sum - comp) - own1));
    kahan_add(sum, comp, v);
    if (cache_c && ballot(v != 0.0f) != 0) {
      if (nst < A.cache_cap) {
        cache_c[(size_t)nst * kWave + lane] = v;
        if (lane == 0) cache_idx[nst] = c;
        if (lane < A.mask_stride)
          A.cache_mask[((size_t)slot * A.cache_cap + nst) * A.mask_stride + lane] = mrec[wave][lane];
      }
      ++nst;
    }
  };
  // phase 0: candidates [0, n1) (orders 0-1), phase 1: [n1, C); one copy of
  // the candidate code serves both (the loop is not unrolled)
  if constexpr (!uses_cut<MODE>()) {
    for_screened3<MAXK>(A.panels, A.n_panels, 0, A.n_cand, lim, A.screen != 0, wave, NW, tx, ty, tz, box, visit);
  } else {
    const int n1 = min(A.n_cand, 1 + A.n_panels);
#pragma nounroll
    for (int ph = 0; ph < 2; ++ph) {
      for_screened3<MAXK>(A.panels, A.n_panels, ph ? n1 : 0, ph ? A.n_cand : n1, lim, A.screen != 0, wave, NW, tx, ty,
                    tz, box, visit);
      if (ph == 0) {
        own1 = sum - comp;
        base[wave][lane] = own1;
        __syncthreads();
#pragma unroll
        for (int w = 0; w < NW; ++w) cut_base += base[w][lane];
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
    if (loss_kind == 1 || loss_kind == 2) {
      const float tot = wave_sum(lp);
      if (lane == 0) loss_part[tile] = tot;
    }
  }
}

template <int NW, int MODE, int MAXK>
__global__ __launch_bounds__(NW * kWave) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_backward3(Trace3Args A, const float* __restrict__ gP,
                                                          float* __restrict__ part, float* __restrict__ grad_rx,
                                                          int reuse) {
  extern __shared__ float smem3[];
  const Scene3View S = view3_of(A);
  const int ncol = 3 + kPanelGrad * A.n_panels;
  float* accs = smem3;                 // [NW][ncol]
  float* rxr = smem3 + NW * ncol;      // [NW][3][64] per-wave receiver gradients
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = uniform(threadIdx.x >> 6);
  for (int i = threadIdx.x; i < NW * ncol; i += NW * kWave) accs[i] = 0.0f;
  __syncthreads();
  float* acc = accs + wave * ncol;
  const int tile = blockIdx.x;
  const int m = rx_of_lane(tile, lane, A.grid_nx);
  const bool live = m < A.n_rx;
  const float rx = live ? A.rx[3 * m] : 0.5f, ry = live ? A.rx[3 * m + 1] : 0.5f, rz = live ? A.rx[3 * m + 2] : 0.5f;
  const float g = live ? gP[m] : 0.0f;
  const float tx = A.tx[0], ty = A.tx[1], tz = A.tx[2];
  LaneGrad3 G{0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  if (ballot(g != 0.0f) != 0) {
    const int slot = tile * NW + wave;
    const int n_cached = (reuse && A.cache_c) ? A.cache_n[slot] : -1;
    if (n_cached >= 0) {
      const float* cache_c = A.cache_c + (size_t)slot * A.cache_cap * kWave;
      const int* cache_idx = A.cache_idx + (size_t)slot * A.cache_cap;
      for (int p = 0; p < n_cached; ++p) {
        const float Wl = g * cache_c[(size_t)p * kWave + lane];
        if (ballot(Wl != 0.0f) == 0) continue;
        const Cand cd = decode_candidate(cache_idx[p], A.n_panels);
        const uint64_t masks =
            lane < A.mask_stride ? A.cache_mask[((size_t)slot * A.cache_cap + p) * A.mask_stride + lane] : 0;
        candidate_adjoint3<MODE, MAXK>(S, cd, tx, ty, tz, rx, ry, rz, live, Wl, acc, lane, G, &masks);
      }
    } else if constexpr (!uses_cut<MODE>()) {
      for (int c = wave; c < A.n_cand; c += NW) {
        const Cand cd = decode_candidate(c, A.n_panels);
        const float Wl = g * candidate_power3<MODE, MAXK>(S, cd, tx, ty, tz, rx, ry, rz, live);
        if (ballot(Wl != 0.0f) == 0) continue;
        candidate_adjoint3<MODE, MAXK>(S, cd, tx, ty, tz, rx, ry, rz, live, Wl, acc, lane, G);
      }
    } else {
      // re-evaluation over the forward's share of candidates (orders 0-1,
      // then the rest), cut against this wavefront's own running sum
      const int n1 = min(A.n_cand, 1 + A.n_panels);
      float rs = 0.0f, rc = 0.0f;
      for (int part = 0; part < 2; ++part) {
        const int c0 = part == 0 ? 0 : n1, c1 = part == 0 ? n1 : A.n_cand;
        for (int c = c0 + wave; c < c1; c += NW) {
          const Cand cd = decode_candidate(c, A.n_panels);
          const float v = candidate_power3<MODE, MAXK>(S, cd, tx, ty, tz, rx, ry, rz, live, nullptr, A.cut * (rs - rc));
          kahan_add(rs, rc, v);
          const float Wl = g * v;
          if (ballot(Wl != 0.0f) == 0) continue;
          candidate_adjoint3<MODE, MAXK>(S, cd, tx, ty, tz, rx, ry, rz, live, Wl, acc, lane, G);
        }
      }
    }
  }
  {
    const float sx = wave_sum(G.tx), sy = wave_sum(G.ty), sz = wave_sum(G.tz);
    if (lane == 0) {
      acc[0] += sx;
      acc[1] += sy;
      acc[2] += sz;
    }
  }
  rxr[(wave * 3 + 0) * kWave + lane] = G.rx;
  rxr[(wave * 3 + 1) * kWave + lane] = G.ry;
  rxr[(wave * 3 + 2) * kWave + lane] = G.rz;
  __syncthreads();
  if (wave == 0 && live && grad_rx) {
    float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      s0 += rxr[(w * 3 + 0) * kWave + lane];
      s1 += rxr[(w * 3 + 1) * kWave + lane];
      s2 += rxr[(w * 3 + 2) * kWave + lane];
    }
    grad_rx[3 * m] = s0;
    grad_rx[3 * m + 1] = s1;
    grad_rx[3 * m + 2] = s2;
  }
  for (int col = threadIdx.x; col < ncol; col += NW * kWave) {
    float s = 0.0f;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += accs[w * ncol + col];
    part[(size_t)tile * ncol + col] = s;
  }
}

// Per panel: gradients with respect to the record (a, n, m1, m2, s) -> the
// corners.  With e1 = b - a, e2 = c - a, n = e1 x e2, N = n . n, s = 1 / N,
// m1 = (e2 x n) / N, m2 = (n x e1) / N; each product's vector-Jacobian
// product in turn, n's last.
__global__ void k_panel_grads(const float* __restrict__ gr, const float* __restrict__ pan, int n,
                              float* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const float* p = pan + 9 * (size_t)j;
  const float* g = gr + kPanelGrad * (size_t)j;
  const float e1x = p[3] - p[0], e1y = p[4] - p[1], e1z = p[5] - p[2];
  const float e2x = p[6] - p[0], e2y = p[7] - p[1], e2z = p[8] - p[2];
  const float nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
  const float N = nx * nx + ny * ny + nz * nz;
  float* o = out + 9 * (size_t)j;
  if (!(N > 0.0f)) {
    for (int k = 0; k < 9; ++k) o[k] = 0.0f;
    return;
  }
  const float s = 1.0f / N;
  const float v1x = e2y * nz - e2z * ny, v1y = e2z * nx - e2x * nz, v1z = e2x * ny - e2y * nx;  // e2 x n
  const float v2x = ny * e1z - nz * e1y, v2y = nz * e1x - nx * e1z, v2z = nx * e1y - ny * e1x;  // n x e1
  const float gm1x = g[6], gm1y = g[7], gm1z = g[8], gm2x = g[9], gm2y = g[10], gm2z = g[11];
  // N from s, m1 = v1 s, m2 = v2 s
  const float gN = -s * s * (g[12] + (gm1x * v1x + gm1y * v1y + gm1z * v1z) + (gm2x * v2x + gm2y * v2y + gm2z * v2z));
  const float gv1x = gm1x * s, gv1y = gm1y * s, gv1z = gm1z * s;
  const float gv2x = gm2x * s, gv2y = gm2y * s, gv2z = gm2z * s;
  float gnx = g[3] + 2.0f * gN * nx, gny = g[4] + 2.0f * gN * ny, gnz = g[5] + 2.0f * gN * nz;
  // v1 = e2 x n: g_e2 += n x gv1, g_n += gv1 x e2
  float ge2x = ny * gv1z - nz * gv1y, ge2y = nz * gv1x - nx * gv1z, ge2z = nx * gv1y - ny * gv1x;
  gnx += gv1y * e2z - gv1z * e2y;
  gny += gv1z * e2x - gv1x * e2z;
  gnz += gv1x * e2y - gv1y * e2x;
  // v2 = n x e1: g_n += e1 x gv2, g_e1 += gv2 x n
  gnx += e1y * gv2z - e1z * gv2y;
  gny += e1z * gv2x - e1x * gv2z;
  gnz += e1x * gv2y - e1y * gv2x;
  float ge1x = gv2y * nz - gv2z * ny, ge1y = gv2z * nx - gv2x * nz, ge1z = gv2x * ny - gv2y * nx;
  // n = e1 x e2: g_e1 += e2 x g_n, g_e2 += g_n x e1
  ge1x += e2y * gnz - e2z * gny;
  ge1y += e2z * gnx - e2x * gnz;
  ge1z += e2x * gny - e2y * gnx;
  ge2x += gny * e1z - gnz * e1y;
  ge2y += gnz * e1x - gnx * e1z;
  ge2z += gnx * e1y - gny * e1x;
  o[0] = g[0] - ge1x - ge2x;
  o[1] = g[1] - ge1y - ge2y;
  o[2] = g[2] - ge1z - ge2z;
  o[3] = ge1x;
  o[4] = ge1y;
  o[5] = ge1z;
  o[6] = ge2x;
  o[7] = ge2y;
  o[8] = ge2z;
}

hipError_t launch_prep_panels(const float* panels, int n, float cull_c, PanelRec* out, PanelBox* boxes,
                              hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_prep_panels, dim3((n + 255) / 256), dim3(256), 0, st, panels, n, cull_c, out, boxes);
  return hipGetLastError();
}

template <int NW, int MODE>
static hipError_t fwd3_nw(const Trace3Args& A, int n_tiles, float* power, float* seed, float* loss_part,
                          int loss_kind, float log_eps, hipStream_t st) {
  // scenes up to order 2 run a kernel without the order-3 path code (fewer
  // register spills, so less scratch traffic)
  if (A.max_order <= 2)
    hipLaunchKernelGGL((k_forward3<NW, MODE, 2>), dim3(n_tiles), dim3(NW * kWave), 0, st, A, power, seed, loss_part,
                       loss_kind, log_eps);
  else
    hipLaunchKernelGGL((k_forward3<NW, MODE, 3>), dim3(n_tiles), dim3(NW * kWave), 0, st, A, power, seed, loss_part,
                       loss_kind, log_eps);
  return hipGetLastError();
}

hipError_t launch_forward3(const Trace3Args& A, int n_tiles, int nw, float* power, float* seed, float* loss_part,
                           int loss_kind, float log_eps, hipStream_t st) {
  switch (nw) {
    case 2: return A.mode ? fwd3_nw<2, kHardSigmoid>(A, n_tiles, power, seed, loss_part, loss_kind, log_eps, st)
                     : fwd3_nw<2, kSigmoid>(A, n_tiles, power, seed, loss_part, loss_kind, log_eps, st);
    case 4: return A.mode ? fwd3_nw<4, kHardSigmoid>(A, n_tiles, power, seed, loss_part, loss_kind, log_eps, st)
                     : fwd3_nw<4, kSigmoid>(A, n_tiles, power, seed, loss_part, loss_kind, log_eps, st);
    case 8: return A.mode ? fwd3_nw<8, kHardSigmoid>(A, n_tiles, power, seed, loss_part, loss_kind, log_eps, st)
                     : fwd3_nw<8, kSigmoid>(A, n_tiles, power, seed, loss_part, loss_kind, log_eps, st);
    case 16: return A.mode ? fwd3_nw<16, kHardSigmoid>(A, n_tiles, power, seed, loss_part, loss_kind, log_eps, st)
                     : fwd3_nw<16, kSigmoid>(A, n_tiles, power, seed, loss_part, loss_kind, log_eps, st);
    default: return hipErrorInvalidValue;
  }
}

size_t backward3_lds_bytes(int nw, int n_panels) {
  return sizeof(float) * (size_t)nw * (3 + kPanelGrad * (size_t)n_panels + 3 * kWave);
}

template <int NW, int MODE>
static hipError_t bwd3_nw(const Trace3Args& A, int n_tiles, const float* gP, float* part, float* grad_rx, int reuse,
                          hipStream_t st) {
  const size_t lds = backward3_lds_bytes(NW, A.n_panels);
  if (A.max_order <= 2)
    hipLaunchKernelGGL((k_backward3<NW, MODE, 2>), dim3(n_tiles), dim3(NW * kWave), lds, st, A, gP, part, grad_rx,
                       reuse);
  else
    hipLaunchKernelGGL((k_backward3<NW, MODE, 3>), dim3(n_tiles), dim3(NW * kWave), lds, st, A, gP, part, grad_rx,
                       reuse);
  return hipGetLastError();
}

hipError_t launch_backward3(const Trace3Args& A, int n_tiles, int nw, const float* gP, float* part, float* grad_rx,
                            int reuse, hipStream_t st) {
  switch (nw) {
    case 2: return A.mode ? bwd3_nw<2, kHardSigmoid>(A, n_tiles, gP, part, grad_rx, reuse, st)
                     : bwd3_nw<2, kSigmoid>(A, n_tiles, gP, part, grad_rx, reuse, st);
    case 4: return A.mode ? bwd3_nw<4, kHardSigmoid>(A, n_tiles, gP, part, grad_rx, reuse, st)
                     : bwd3_nw<4, kSigmoid>(A, n_tiles, gP, part, grad_rx, reuse, st);
    case 8: return A.mode ? bwd3_nw<8, kHardSigmoid>(A, n_tiles, gP, part, grad_rx, reuse, st)
                     : bwd3_nw<8, kSigmoid>(A, n_tiles, gP, part, grad_rx, reuse, st);
    case 16: return A.mode ? bwd3_nw<16, kHardSigmoid>(A, n_tiles, gP, part, grad_rx, reuse, st)
                     : bwd3_nw<16, kSigmoid>(A, n_tiles, gP, part, grad_rx, reuse, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_panel_grads(const float* part, int n_tiles, int n_panels, const float* panels, float* tmp,
                              float* grad_tx, float* grad_panels, hipStream_t st) {
  hipError_t e = launch_reduce_cols(part, n_tiles, 3 + kPanelGrad * n_panels, grad_tx, 3, tmp, st);
  if (e != hipSuccess || n_panels <= 0) return e;
  hipLaunchKernelGGL(k_panel_grads, dim3((n_panels + 255) / 256), dim3(256), 0, st, tmp, panels, n_panels,
                     grad_panels);
  return hipGetLastError();
}

}  // namespace drt
