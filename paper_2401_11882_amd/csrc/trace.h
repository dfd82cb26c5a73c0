// Internal interface between the C ABI (api.hip) and the tracer kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace drt {

struct WallRec;
struct WallBox;

struct TraceArgs {
  const WallRec* walls;  // prepared wall records [n_walls]
  const WallBox* boxes;  // culling boxes [n_walls]
  const float* tx;       // [2]
  const float* rx;       // [n_rx][2]
  int n_walls;
  int n_rx;
  int grid_nx;           // 0 = consecutive receivers per wavefront
  int n_cand;
  int cchunk;            // candidates per chunk handed to one wavefront
  int screen;            // 1: drop candidates that are exactly 0 over a wavefront's receiver box
  float cut;             // contribution cut factor (kCutTotal / C, or 0 = off)
  int mode;              // 0 sigmoid, 1 hard sigmoid
  int max_order;
  float alpha;
  float a2;              // alpha * log2(e)
  float band_k;          // 1 + 2 * 18 / alpha: unsaturated-test band
  float cull_c;          // 20 / alpha: culling-box extension
  float dmin2;
  // contribution cache (all NULL when disabled): per (tile, wavefront) slot
  float* cache_c;    // [slots][cache_cap][64] per-lane contributions
  int* cache_idx;    // [slots][cache_cap] candidate index of each entry
  int* cache_n;      // [slots] entries, or -1 when the list overflowed
  int cache_cap;
  float* cache_box;  // [slots][cache_cap][box_stride] culling boxes of each entry's legs
  int box_stride;
};

hipError_t launch_prep_walls(const float* walls, int n, float cull_c, WallRec* out, WallBox* boxes,
                             hipStream_t st);
hipError_t launch_forward(const TraceArgs& A, int n_tiles, int nw, float* power, float* seed,
                          float* loss_part, int loss_kind, float log_eps, hipStream_t st);
hipError_t launch_forward_fermat(const TraceArgs& A, int n_tiles, int nw, float* power, float* loss_part,
                                 int loss_kind, float log_eps, int max_iter, float inv_eps, hipStream_t st);
hipError_t launch_backward(const TraceArgs& A, int n_tiles, int nw, const float* gP, float* part,
                           float* grad_rx, int reuse, hipStream_t st);
size_t backward_lds_bytes(int nw, int n_walls);
size_t forward_lds_bytes(int nw, int max_order);
hipError_t launch_reduce_cols(const float* part, int n_rows, int ncol, float* out_head, int n_head,
                              float* out_tail, hipStream_t st);
hipError_t launch_reduce_scalar(const float* part, int n, double scale, float* out, hipStream_t st);
hipError_t launch_adam_points(int n, float* x, const float* grad, float* m, float* v, int32_t* step, float lr,
                              float b1, float b2, float eps, float lo, float hi, hipStream_t st);
hipError_t launch_alpha_schedule(const int32_t* step, int n_iter, float a_first, float a_last, float* alpha, int n,
                                 hipStream_t st);
hipError_t launch_min_seed(const float* power, int n, float* loss, float* seed, hipStream_t st);

}  // namespace drt
