// Many scenes in one persistent launch: forward, loss seed and adjoint fused
// per work item.
//
// A work item is (scene, tile of 64 receivers).  Items are sorted by cost
// (candidates x receivers, longest first) on the host when the plan is made.
// The grid holds as many workgroups as fit on the GPU at once; each
// workgroup takes items from a device counter until the list is exhausted
// (every workgroup reaches that exit).  For its item the workgroup's NW
// wavefronts split the scene's candidates, record their nonzero
// contributions in the workgroup's own cache region, combine the per-wave
// power sums in LDS (so P(r) is complete), form dL/dP(r), and then run the
// adjoint from the recorded contributions.  Per-item gradient partials go to
// a per-item slot; a second kernel sums each scene's items in a fixed order,
// so results do not depend on which workgroup took which item.
#include "batched.h"
#include "path.h"
#include "screen.h"

namespace drt {

__global__ void k_batch_reset(int* counter) { *counter = 0; }

// Wall records and culling data for every wall of every scene (one
// workgroup per scene, alpha per scene).
__global__ void k_batch_prep(const float* __restrict__ walls, const int* __restrict__ wall_off,
                             const float* __restrict__ alpha, float cull_margin, WallRec* __restrict__ rec,
                             WallBox* __restrict__ boxes) {
  const int s = blockIdx.x;
  const float c = cull_margin / alpha[s];
  for (int j = wall_off[s] + threadIdx.x; j < wall_off[s + 1]; j += blockDim.x) {
    WallRec r;
    WallBox q;
    make_wall(walls[4 * j], walls[4 * j + 1], walls[4 * j + 2], walls[4 * j + 3], c, r, q);
    rec[j] = r;
    boxes[j] = q;
  }
}

// Receiver of a lane for tiles of tw x (64/tw) receivers on a row-major grid
// of nx columns (tw = 0 or nx = 0: 64 consecutive receivers).
__device__ __forceinline__ int batch_rx_of_lane(int tile, int lane, int nx, int tw) {
  if (nx > 0 && tw > 0) {
    const int th = kWave / tw;
    const int tpr = nx / tw;
    const int ty = tile / tpr;
    const int tx = tile - ty * tpr;
    return (ty * th + lane / tw) * nx + tx * tw + (lane % tw);
  }
  return tile * kWave + lane;
}

// MAXK: the highest order of the batch's candidates (2 covers orders 0..2;
// the code of higher orders is left out, which keeps register pressure at
// that order's).
template <int NW, int MODE, int MAXK>
__global__ __launch_bounds__(NW * kWave) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_batched(BatchArgs B) {
  extern __shared__ float smem[];
  __shared__ int item_sh;
  __shared__ float gsh[kWave];
  __shared__ float base[NW][kWave];  // each wavefront's power sum over the orders 0 and 1
  const int ncol_max = 2 + 4 * B.max_walls;
  float* accs = smem;                        // [NW][ncol_max]
  float* red = smem + NW * ncol_max;         // [NW][2][64]
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = uniform(threadIdx.x >> 6);
  // [NW][6 (max_order + 1)][64] leg boxes of screened candidates, when they fit
  float* boxes = B.box_lds ? red + NW * 2 * kWave + wave * 6 * (B.max_order + 1) * kWave : nullptr;
  const int slot = blockIdx.x * NW + wave;
  float* cache_c = B.cache_c ? B.cache_c + (size_t)slot * B.cache_cap * kWave : nullptr;
  int* cache_idx = B.cache_c ? B.cache_idx + (size_t)slot * B.cache_cap : nullptr;

  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) item_sh = atomicAdd(B.counter, 1);
    __syncthreads();
    const int it = item_sh;
    if (it >= B.n_items) break;
    const int s = B.items[2 * it], tile = B.items[2 * it + 1];
    const int w0 = B.wall_off[s], W = B.wall_off[s + 1] - w0;
    const int r0 = B.rx_off[s], R = B.rx_off[s + 1] - r0;
    const int ncol = 2 + 4 * W;
    const float alpha = B.alpha[s];
    SceneView S;
    S.walls = B.walls + w0;
    S.boxes = B.boxes + w0;
    S.n_walls = W;
    S.alpha = alpha;
    S.a2 = alpha * kLog2e;
    S.band_k = 1.0f + 2.0f * (MODE ? kHardBandMargin : kBandMargin) / alpha;
    S.cull_c = (MODE ? kHardCullMargin : kCullMargin) / alpha;
    S.dmin2 = B.dmin2;
    S.a6 = alpha * (1.0f / 6.0f);
    S.a6h = S.a6 + 0.5f;
    S.a6m = 0.5f - S.a6;
    S.dead_lim = (MODE ? kHardBandMargin / alpha : 128.0f / S.a2) * 1.00001f;
    S.cull = B.screen != 0;
    // number of candidates of this scene
    int n_cand = 1, term = 0;
    for (int k = 1; k <= B.max_order; ++k) {
      term = (k == 1) ? W : term * (W - 1);
      n_cand += term;
    }
    const float cutf = cut_factor(B.cut != 0.0f, n_cand);
    for (int i = threadIdx.x; i < NW * ncol; i += NW * kWave) accs[(i / ncol) * ncol_max + (i % ncol)] = 0.0f;

    const int m = batch_rx_of_lane(tile, lane, B.grid_nx[s], B.tile_w);
    const bool live = m < R;
    const float rxx = live ? B.rx[2 * (r0 + m)] : 0.5f;
    const float rxy = live ? B.rx[2 * (r0 + m) + 1] : 0.5f;
    const float txx = B.tx[2 * s], txy = B.tx[2 * s + 1];

    // -- forward over this wave's candidates, recording nonzero contributions
    float sum = 0.0f, comp = 0.0f;
    int nst = 0;
    const RxBox box = rx_box(rxx, rxy, live);
    // contribution cut against the orders 0 and 1 of every wavefront plus
    // this wavefront's running sum (see k_forward)
    float cut_base = 0.0f, own1 = 0.0f;
    auto visit = [&](int c, const Cand& cd, const float* Ix, const float* Iy, int j) {
      const float v = candidate_power_img<MODE, MAXK>(S, cd, Ix, Iy, txx, txy, rxx, rxy, live, boxes, j,
                                                cutf * (cut_base + (sum - comp) - own1));
      kahan_add(sum, comp, v);
      if (cache_c && B.loss_kind != 0 && ballot(v != 0.0f) != 0) {
        if (nst < B.cache_cap) {
          cache_c[(size_t)nst * kWave + lane] = v;
          if (lane == 0) cache_idx[nst] = c;
          if (boxes && lane < B.box_stride)
            B.cache_box[((size_t)slot * B.cache_cap + nst) * B.box_stride + lane] = boxes[lane * kWave + j];
        }
        ++nst;
      }
    };
    const int n1 = uses_cut<MODE>() ? min(n_cand, 1 + W) : 0;
#pragma nounroll
    for (int ph = uses_cut<MODE>() ? 0 : 1; ph < 2; ++ph) {
      for_screened(S.walls, W, ph ? n1 : 0, ph ? n_cand : n1, S.dead_lim, B.screen != 0, wave, NW, B.cchunk, txx,
                   txy, box, S.cull_c, boxes, visit);
      if (ph == 0) {
        own1 = sum - comp;
        base[wave][lane] = own1;
        __syncthreads();
#pragma unroll
        for (int w = 0; w < NW; ++w) cut_base += base[w][lane];
      }
    }
    red[(wave * 2 + 0) * kWave + lane] = sum;
    red[(wave * 2 + 1) * kWave + lane] = comp;
    __syncthreads();
    if (wave == 0) {
      float sp = 0.0f, cs = 0.0f;
#pragma unroll
      for (int w = 0; w < NW; ++w)
        kahan_add(sp, cs, red[(w * 2 + 0) * kWave + lane] - red[(w * 2 + 1) * kWave + lane]);
      const float P = sp - cs;
      float lp = 0.0f, g = 0.0f;
      if (live) {
        B.power[r0 + m] = P;
        if (B.loss_kind == 1) {
          lp = P;
          g = 1.0f;
        } else if (B.loss_kind == 2) {
          lp = logf(P + B.log_eps);
          g = -1.0f / ((float)R * (P + B.log_eps));
        }
      }
      if (B.loss_kind == 3) {
        // the scene's only tile: -min P, seeded at the lowest index attaining it
        const float pm = wave_min(live ? P : __builtin_inff());
        const uint64_t at = ballot(live && P == pm);
        const bool first = at != 0 && lane == __builtin_ctzll(at);
        g = first ? -1.0f : 0.0f;
        lp = first ? -pm : 0.0f;
      }
      gsh[lane] = g;
      const float tot = wave_sum(lp);
      if (lane == 0) B.loss_part[it] = tot;
    }
    if (B.loss_kind == 0) continue;  // forward only (the loop head synchronises)
    __syncthreads();

    // -- adjoint from the recorded contributions (or re-evaluation on overflow)
    const float g = gsh[lane];
    float* acc = accs + wave * ncol_max;
    LaneGrad G{0.0f, 0.0f, 0.0f, 0.0f};
    if (cache_c && nst <= B.cache_cap) {
      for (int p = 0; p < nst; ++p) {
        const int c = cache_idx[p];
        const float Wl = g * cache_c[(size_t)p * kWave + lane];
        if (ballot(Wl != 0.0f) == 0) continue;
        const Cand cd = decode_candidate(c, W);
        const float* gbox = boxes ? B.cache_box + ((size_t)slot * B.cache_cap + p) * B.box_stride : nullptr;
        candidate_adjoint_known<MODE, MAXK>(S, cd, txx, txy, rxx, rxy, live, Wl, acc, lane, G, gbox);
      }
    } else {
      // re-evaluation of this wavefront's share as the forward split it, the
      // cut against its own running sum
      float rs = 0.0f, rc = 0.0f;
      const int n1 = uses_cut<MODE>() ? min(n_cand, 1 + W) : 0;
      const int stride = NW * B.cchunk;
      for (int part = 0; part < 2; ++part) {
        const int b0 = part ? n1 : 0, b1 = part ? n_cand : n1;
        for (int c0 = b0 + wave * B.cchunk; c0 < b1; c0 += stride) {
          const int c1 = min(c0 + B.cchunk, b1);
          for (int c = c0; c < c1; ++c) {
            const Cand cd = decode_candidate(c, W);
            kahan_add(rs, rc,
                      candidate_adjoint<MODE, MAXK>(S, cd, txx, txy, rxx, rxy, live, g, acc, lane, G, cutf * (rs - rc)));
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
    __syncthreads();
    float* part = B.grad_part + B.part_off[it];
    for (int col = threadIdx.x; col < ncol; col += NW * kWave) {
      float v = 0.0f;
#pragma unroll
      for (int w = 0; w < NW; ++w) v += accs[w * ncol_max + col];
      part[col] = v;
    }
  }
}

// Per scene: loss and gradients summed over the scene's items in item order.
__global__ __launch_bounds__(256) void k_batch_reduce(BatchArgs B, float* __restrict__ loss,
                                                      float* __restrict__ grad_tx,
                                                      float* __restrict__ grad_walls) {
  const int s = blockIdx.x;
  const int i0 = B.scene_items[2 * s], i1 = i0 + B.scene_items[2 * s + 1];
  const int w0 = B.wall_off[s], W = B.wall_off[s + 1] - w0;
  const int ncol = 2 + 4 * W;
  for (int col = threadIdx.x; col < ncol; col += blockDim.x) {
    double t = 0.0;
    for (int it = i0; it < i1; ++it) t += (double)B.grad_part[B.part_off[it] + col];
    if (col < 2) grad_tx[2 * s + col] = (float)t;
    else grad_walls[4 * (size_t)w0 + (col - 2)] = (float)t;
  }
  if (threadIdx.x == 0 && loss) {
    double t = 0.0;
    for (int it = i0; it < i1; ++it) t += (double)B.loss_part[it];
    const int R = B.rx_off[s + 1] - B.rx_off[s];
    const double scale = B.loss_kind == 2 ? (R > 0 ? -1.0 / (double)R : 0.0) : 1.0;
    loss[s] = (float)(scale * t);
  }
}

static size_t batched_base_lds(int nw, int max_walls) {
  return sizeof(float) * ((size_t)nw * (2 + 4 * (size_t)max_walls) + (size_t)nw * 2 * kWave);
}

// The leg boxes of screened candidates go to LDS when the workgroup's total
// stays within 64 KiB; otherwise the boxes are formed from the lanes' legs.
bool batched_box_lds(int nw, int max_walls, int max_order) {
  return batched_base_lds(nw, max_walls) + sizeof(float) * (size_t)nw * 6 * (max_order + 1) * kWave <= 65536;
}

size_t batched_lds_bytes(int nw, int max_walls, int max_order) {
  return batched_base_lds(nw, max_walls) +
         (batched_box_lds(nw, max_walls, max_order) ? sizeof(float) * (size_t)nw * 6 * (max_order + 1) * kWave : 0);
}

template <int NW, int MAXK>
static hipError_t batched_nw_k(const BatchArgs& B, int n_blocks, hipStream_t st) {
  if (B.mode)
    hipLaunchKernelGGL((k_batched<NW, 1, MAXK>), dim3(n_blocks), dim3(NW * kWave),
                       batched_lds_bytes(NW, B.max_walls, B.max_order), st, B);
  else
    hipLaunchKernelGGL((k_batched<NW, 0, MAXK>), dim3(n_blocks), dim3(NW * kWave),
                       batched_lds_bytes(NW, B.max_walls, B.max_order), st, B);
  return hipGetLastError();
}

template <int NW>
static hipError_t batched_nw(const BatchArgs& B, int n_blocks, hipStream_t st) {
  return B.max_order <= 2 ? batched_nw_k<NW, 2>(B, n_blocks, st) : batched_nw_k<NW, 3>(B, n_blocks, st);
}

hipError_t launch_batched(const BatchArgs& B, int nw, int n_blocks, const float* walls_raw, const float* alpha,
                          int n_scenes, float* loss, float* grad_tx, float* grad_walls, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_prep, dim3(n_scenes), dim3(128), 0, st, walls_raw, B.wall_off, alpha,
                     B.mode ? kHardCullMargin : kCullMargin, const_cast<WallRec*>(B.walls),
                     const_cast<WallBox*>(B.boxes));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, st, B.counter);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  switch (nw) {
    case 4: e = batched_nw<4>(B, n_blocks, st); break;
    case 8: e = batched_nw<8>(B, n_blocks, st); break;
    case 16: e = batched_nw<16>(B, n_blocks, st); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  if (B.loss_kind == 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_reduce, dim3(n_scenes), dim3(256), 0, st, B, loss, grad_tx, grad_walls);
  return hipGetLastError();
}

// Resident workgroups per CU for a launch shape (the smaller of the two
// smoothing modes, so the persistent grid fits either).
template <int MAXK>
static void batched_fns(int nw, const void* (&fns)[2]) {
  if (nw == 4) {
    fns[0] = reinterpret_cast<const void*>(k_batched<4, 0, MAXK>);
    fns[1] = reinterpret_cast<const void*>(k_batched<4, 1, MAXK>);
  } else if (nw == 8) {
    fns[0] = reinterpret_cast<const void*>(k_batched<8, 0, MAXK>);
    fns[1] = reinterpret_cast<const void*>(k_batched<8, 1, MAXK>);
  } else {
    fns[0] = reinterpret_cast<const void*>(k_batched<16, 0, MAXK>);
    fns[1] = reinterpret_cast<const void*>(k_batched<16, 1, MAXK>);
  }
}

int batched_max_blocks_per_cu(int nw, int max_walls, int max_order) {
  const void* fns[2];
  if (max_order <= 2) batched_fns<2>(nw, fns);
  else batched_fns<3>(nw, fns);
  int best = 1 << 30;
  for (const void* fn : fns) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, nw * kWave, batched_lds_bytes(nw, max_walls, max_order)) !=
        hipSuccess)
      return 1;
    best = nb < best ? nb : best;
  }
  return best > 0 ? best : 1;
}

}  // namespace drt
