// Internal interface of the batched persistent kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "dev.h"

namespace drt {

struct BatchArgs {
  const WallRec* walls;        // prepared records [sum W]
  const WallBox* boxes;        // culling boxes [sum W]
  const int* wall_off;         // [S+1] first wall of each scene
  const int* rx_off;           // [S+1] first receiver of each scene
  const int* grid_nx;          // [S] row length of a grid scene, 0 = consecutive receivers
  const float* rx;             // [sum R][2]
  const float* tx;             // [S][2]
  const float* alpha;          // [S]
  const int* items;            // [n_items][2] = (scene, tile), longest first
  int n_items;
  int* counter;                // work counter (reset before each launch)
  const int* scene_items;      // [S][2] = (first item, item count); a scene's items are contiguous
  const long long* part_off;   // [n_items] offset of each item's gradient partial (2 + 4 W floats)
  int max_order;
  int max_walls;
  float dmin2;
  float log_eps;
  int loss_kind;               // 1 = sum of power, 2 = -mean log(P + eps)
  float* power;                // [sum R]
  float* loss_part;            // [n_items]
  float* grad_part;            // [sum over items of 2 + 4 W]
  float* cache_c;              // [slots][cache_cap][64] (NULL = no cache)
  int* cache_idx;              // [slots][cache_cap]
  float* cache_box;            // [slots][cache_cap][box_stride] leg boxes of each entry
  int box_stride;
  int cache_cap;
  int cchunk;
  int screen;                  // candidate screen on / off
  float cut;                   // 1: contribution cut on (factor per scene), 0: off
  int mode;                    // 0 sigmoid, 1 hard sigmoid
  int box_lds;                 // 1: screened candidates' leg boxes kept in LDS
  int tile_w;                  // receivers per tile row on grid scenes (8, 16, 32)
};

hipError_t launch_batched(const BatchArgs& B, int nw, int n_blocks, const float* walls_raw, const float* alpha,
                          int n_scenes, float* loss, float* grad_tx, float* grad_walls, hipStream_t st);
size_t batched_lds_bytes(int nw, int max_walls, int max_order);
bool batched_box_lds(int nw, int max_walls, int max_order);
int batched_max_blocks_per_cu(int nw, int max_walls, int max_order);

}  // namespace drt
