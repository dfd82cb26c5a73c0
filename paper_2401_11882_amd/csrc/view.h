// Scene view of a single-scene launch: the per-scene constants the device
// code reads, derived from the launch arguments.
#pragma once
#include "path.h"
#include "trace.h"

namespace drt {

__device__ __forceinline__ SceneView view_of(const TraceArgs& A) {
  SceneView S;
  S.walls = A.walls;
  S.boxes = A.boxes;
  S.n_walls = A.n_walls;
  S.alpha = A.alpha;
  S.a2 = A.a2;
  S.band_k = A.band_k;
  S.cull_c = A.cull_c;
  S.dmin2 = A.dmin2;
  S.a6 = A.alpha * (1.0f / 6.0f);
  S.a6h = S.a6 + 0.5f;
  S.a6m = 0.5f - S.a6;
  S.dead_lim = (A.mode ? kHardBandMargin / A.alpha : 128.0f / A.a2) * 1.00001f;
  S.cull = A.screen != 0;
  return S;
}

// Receiver m of a lane (live lanes only; others get a dummy point): from the
// array, or without one the centre ((i + 1/2) / nx, (j + 1/2) / ny) of cell
// m = j nx + i of the grid, computed in FP64 and rounded once to FP32.
__device__ __forceinline__ void receiver_of(const TraceArgs& A, int m, bool live, float& x, float& y) {
  if (!live) {
    x = y = 0.5f;
  } else if (A.rx) {
    x = A.rx[2 * m];
    y = A.rx[2 * m + 1];
  } else {
    const int nx = A.grid_nx, ny = A.n_rx / nx;
    const int j = m / nx, i = m - j * nx;
    x = (float)(((double)i + 0.5) / (double)nx);
    y = (float)(((double)j + 0.5) / (double)ny);
  }
}

}  // namespace drt
