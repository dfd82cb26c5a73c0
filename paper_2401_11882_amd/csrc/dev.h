// Device helpers shared by the tracer kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace drt {

constexpr int kWave = 64;
constexpr float kLog2e = 1.4426950408889634f;
// Above this, E / (1 + E) is taken as exactly 1 (it is within 1e-30 of it).
constexpr float kBig = 1e30f;

// Prepared wall record, 32 bytes: endpoint a, direction e = b - a, a x e.
struct WallRec {
  float ax, ay, ex, ey, axe, pad0, pad1, pad2;
};

// Axis-aligned box of a wall extended along itself by the culling band:
// [a - c e, b + c e], c = kCullMargin / alpha.
struct WallBox {
  float xmin, xmax, ymin, ymax;
};

// Obstruction tests are evaluated only when both parameters lie within
// kBandMargin / alpha of [0, 1]; the culling boxes use the wider kCullMargin
// so that a culled test is one the per-lane check would also skip.
constexpr float kBandMargin = 18.0f;
constexpr float kCullMargin = 20.0f;

__device__ __forceinline__ float ex2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ float uniformf(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// Sum over the 64 lanes of a wavefront with DPP; the total is returned as a
// wave-uniform value.  Steps: quad swaps, row shifts by 4 and 8 (lane 15 of
// each 16-lane row then holds the row sum), row broadcasts 15 and 31 (lane 63
// then holds the total).  Lanes whose DPP source is out of range add 0.
__device__ __forceinline__ float wave_sum(float x) {
  x += __builtin_amdgcn_update_dpp(0.0f, x, 0xb1, 0xf, 0xf, false);   // quad_perm [1,0,3,2]
  x += __builtin_amdgcn_update_dpp(0.0f, x, 0x4e, 0xf, 0xf, false);   // quad_perm [2,3,0,1]
  x += __builtin_amdgcn_update_dpp(0.0f, x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0.0f, x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0.0f, x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  x += __builtin_amdgcn_update_dpp(0.0f, x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

// Minimum / maximum over the 64 lanes (same DPP pattern as wave_sum; lanes
// whose source is out of range keep the identity).  Wave-uniform result.
__device__ __forceinline__ float wave_min(float x) {
  const float I = __builtin_inff();
  x = fminf(x, __builtin_amdgcn_update_dpp(I, x, 0xb1, 0xf, 0xf, false));
  x = fminf(x, __builtin_amdgcn_update_dpp(I, x, 0x4e, 0xf, 0xf, false));
  x = fminf(x, __builtin_amdgcn_update_dpp(I, x, 0x114, 0xf, 0xf, false));
  x = fminf(x, __builtin_amdgcn_update_dpp(I, x, 0x118, 0xf, 0xf, false));
  x = fminf(x, __builtin_amdgcn_update_dpp(I, x, 0x142, 0xa, 0xf, false));
  x = fminf(x, __builtin_amdgcn_update_dpp(I, x, 0x143, 0xc, 0xf, false));
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

__device__ __forceinline__ float wave_max(float x) {
  const float I = -__builtin_inff();
  x = fmaxf(x, __builtin_amdgcn_update_dpp(I, x, 0xb1, 0xf, 0xf, false));
  x = fmaxf(x, __builtin_amdgcn_update_dpp(I, x, 0x4e, 0xf, 0xf, false));
  x = fmaxf(x, __builtin_amdgcn_update_dpp(I, x, 0x114, 0xf, 0xf, false));
  x = fmaxf(x, __builtin_amdgcn_update_dpp(I, x, 0x118, 0xf, 0xf, false));
  x = fmaxf(x, __builtin_amdgcn_update_dpp(I, x, 0x142, 0xa, 0xf, false));
  x = fmaxf(x, __builtin_amdgcn_update_dpp(I, x, 0x143, 0xc, 0xf, false));
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

// Candidate index -> (order k, walls s[0..k-1]).  Candidates are ordered by
// order, then lexicographically: the first wall is a base-W digit, each later
// wall a base-(W-1) digit d mapped to d + (d >= previous wall), which skips a
// back-to-back repeat.  c must be < the candidate count.
struct Cand {
  int k;
  int s0, s1, s2;
};

__device__ __forceinline__ Cand decode_candidate(int c, int W) {
  Cand q{0, -1, -1, -1};
  if (c == 0) return q;
  c -= 1;
  if (c < W) {
    q.k = 1;
    q.s0 = c;
    return q;
  }
  c -= W;
  const int Wm = W - 1;
  const int n2 = W * Wm;
  if (c < n2) {
    q.k = 2;
    const int d1 = c / Wm;
    const int d2 = c - d1 * Wm;
    q.s0 = d1;
    q.s1 = d2 + (d2 >= d1);
    return q;
  }
  c -= n2;
  q.k = 3;
  const int Wm2 = Wm * Wm;
  const int d1 = c / Wm2;
  const int r = c - d1 * Wm2;
  const int d2 = r / Wm;
  const int d3 = r - d2 * Wm;
  q.s0 = d1;
  q.s1 = d2 + (d2 >= d1);
  q.s2 = d3 + (d3 >= q.s1);
  return q;
}

// Receiver index of a lane: 8x8 blocks on a row-major grid of nx columns, or
// 64 consecutive receivers.
__device__ __forceinline__ int rx_of_lane(int tile, int lane, int grid_nx) {
  if (grid_nx > 0) {
    const int tpr = grid_nx >> 3;
    const int ty = tile / tpr;
    const int tx = tile - ty * tpr;
    return ((ty << 3) + (lane >> 3)) * grid_nx + (tx << 3) + (lane & 7);
  }
  return tile * kWave + lane;
}

}  // namespace drt
