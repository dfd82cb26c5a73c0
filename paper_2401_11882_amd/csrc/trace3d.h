// Internal interface between the C ABI (api3d.hip) and the 3D tracer kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace drt {

struct PanelRec;
struct PanelBox;

struct Trace3Args {
  const PanelRec* panels;  // prepared panel records [n_panels]
  const PanelBox* boxes;   // culling boxes [n_panels], NULL: no culling
  float cull_c;            // 20 / alpha: culling extension of legs and panels
  int screen;              // 1: drop candidates that are exactly 0 over a wavefront's receiver box
  float cut;               // contribution cut factor (kCutTotal / C, or 0 = off)
  int mode;                // 0 sigmoid, 1 hard sigmoid
  const float* tx;         // [3]
  const float* rx;         // [n_rx][3]
  int n_panels;
  int n_rx;
  int grid_nx;             // 0 = consecutive receivers per wavefront
  int n_cand;
  int max_order;           // highest interaction order of the candidates
  float alpha;
  float a2;                // alpha * log2(e)
  float band_k;            // 1 + 2 * 18 / alpha
  float dmin2;
  // contribution cache (NULL when disabled): per (tile, wavefront) slot
  float* cache_c;          // [slots][cache_cap][64]
  int* cache_idx;          // [slots][cache_cap]
  int* cache_n;            // [slots], -1 when the list overflowed
  int cache_cap;
  uint64_t* cache_mask;    // [slots][cache_cap][mask_stride] culling masks of each entry
  int mask_stride;         // (max_order + 1) mask_nb <= 16
  int mask_nb;             // 64-panel batches: ceil(n_panels / 64)
};

hipError_t launch_prep_panels(const float* panels, int n, float cull_c, PanelRec* out, PanelBox* boxes,
                              hipStream_t st);
hipError_t launch_forward3(const Trace3Args& A, int n_tiles, int nw, float* power, float* seed, float* loss_part,
                           int loss_kind, float log_eps, hipStream_t st);
// grad_rx: [n_rx][3] or NULL.
hipError_t launch_backward3(const Trace3Args& A, int n_tiles, int nw, const float* gP, float* part, float* grad_rx,
                            int reuse, hipStream_t st);
// grad_tx[3] and grad_panels[n][9] from the fixed-order column sums of the
// per-tile partials [n_tiles][3 + 13 n] (tmp: 13 n floats).
hipError_t launch_panel_grads(const float* part, int n_tiles, int n_panels, const float* panels, float* tmp,
                              float* grad_tx, float* grad_panels, hipStream_t st);
size_t backward3_lds_bytes(int nw, int n_panels);

}  // namespace drt
