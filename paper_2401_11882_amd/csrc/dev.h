// Device helpers shared by the tracer kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace drt {

constexpr int kWave = 64;
constexpr float kLog2e = 1.4426950408889634f;
// Above this, E / (1 + E) is taken as exactly 1 (it is within 1e-30 of it).
constexpr float kBig = 1e30f;

// Prepared wall record, 32 bytes: endpoint a, direction e = b - a, a x e,
// 1 / |e|^2 (0 for a zero-length wall).
struct WallRec {
  float ax, ay, ex, ey, axe, inv_ee, pad1, pad2;
};

// Wall record at a wave-uniform index, read through the scalar data cache
// (constant address space, SGPR index) instead of 64 identical vector loads.
__device__ __forceinline__ WallRec load_wall(const WallRec* walls, int j) {
  typedef __attribute__((address_space(4))) const float* ConstF;
  const int ju = __builtin_amdgcn_readfirstlane(j);
  const ConstF p = (ConstF)(walls + ju);
  WallRec w;
  w.ax = p[0];
  w.ay = p[1];
  w.ex = p[2];
  w.ey = p[3];
  w.axe = p[4];
  w.inv_ee = p[5];
  w.pad1 = w.pad2 = 0.0f;
  return w;
}

// A wall extended along itself by the culling band, [a - c e, b + c e]
// (c = kCullMargin / alpha), with its normal n = perp(e) and n . p0: the data
// the culling test needs for one wall.
// Culling data of a wall: its segment extended by c |e| at both ends, as
// centre and half vector, the normal n = perp(e), n . centre, and the margin
// used against rounding in the normal-axis test.
struct WallBox {
  float cx, cy, hx, hy, nx, ny, nd, en;
};

// Record and culling data of the wall (a, b).
__device__ __forceinline__ void make_wall(float ax, float ay, float bx, float by, float c, WallRec& r,
                                          WallBox& q) {
  const float ex = bx - ax, ey = by - ay;
  r.ax = ax;
  r.ay = ay;
  r.ex = ex;
  r.ey = ey;
  r.axe = ax * ey - ay * ex;
  const float ee = ex * ex + ey * ey;
  r.inv_ee = ee > 0.0f ? 1.0f / ee : 0.0f;
  r.pad1 = r.pad2 = 0.0f;
  q.cx = 0.5f * (ax + bx);
  q.cy = 0.5f * (ay + by);
  q.hx = (0.5f + c) * ex;
  q.hy = (0.5f + c) * ey;
  q.nx = -ey;
  q.ny = ex;
  q.nd = q.nx * q.cx + q.ny * q.cy;
  q.en = 1e-5f * (fabsf(q.nx) + fabsf(q.ny) + fabsf(q.nd));
}

// Obstruction tests are evaluated only when both parameters lie within
// kBandMargin / alpha of [0, 1]; the culling boxes use the wider kCullMargin
// so that a culled test is one the per-lane check would also skip.
constexpr float kBandMargin = 18.0f;
constexpr float kCullMargin = 20.0f;
// Hard sigmoid: hs(x) hs(1 - x) is exactly 0 beyond 3 / alpha outside [0, 1].
constexpr float kHardBandMargin = 3.0f;
constexpr float kHardCullMargin = 4.0f;

__device__ __forceinline__ float ex2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ float uniformf(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// Smoothing of the comparisons (Sec. IV-B): sigmoid (Eq. 4) or hard sigmoid
// (Eq. 5-6, relu6(alpha x + 3) / 6 = clamp(x alpha / 6 + 1/2, 0, 1)).
constexpr int kSigmoid = 0;
constexpr int kHardSigmoid = 1;

__device__ __forceinline__ float med01(float x) { return __builtin_amdgcn_fmed3f(x, 0.0f, 1.0f); }

// Contribution cut: a lane drops a candidate as soon as its contribution is
// provably at most kCutTotal / C times the lane's running power sum (a lower
// bound of its P(r), every term being >= 0), C the scene's candidate count.
// The dropped terms of a receiver then add up to at most kCutTotal P(r) =
// 2^-24 P(r), no more than one FP32 rounding of P.
constexpr float kCutTotal = 0x1p-24f;

// Per-candidate cut factor of a scene with n_cand candidates (0: cut off).
__host__ __device__ inline float cut_factor(bool on, int n_cand) {
  return (on && n_cand > 0) ? kCutTotal / (float)n_cand : 0.0f;
}

// The cut serves the sigmoid smoothing.  Hard-sigmoid factors are already
// exactly 0 beyond a band of 3 / alpha, so those kernels are built without
// the cut and visit candidates in plain order (no first phase of orders 0-1).
template <int MODE>
constexpr bool uses_cut() {
  return MODE == kSigmoid;
}

// Candidate phases of the 2D kernels with the cut: the orders 0-1
// [0, end0), then the order 2 [end0, end1) when the scene also has order-3
// candidates, then the rest [end1, n_cand).  After each phase but the last
// the wavefronts of a workgroup add up their sums, the base of the bound.
struct CutPhases {
  int end0, end1, n;
};

__host__ __device__ inline CutPhases cut_phases(int n_walls, int max_order, int n_cand) {
  CutPhases p;
  p.end0 = n_cand < 1 + n_walls ? n_cand : 1 + n_walls;
  const int e2 = p.end0 + n_walls * (n_walls - 1);
  p.end1 = (max_order >= 3 && e2 < n_cand) ? e2 : n_cand;
  p.n = p.end1 < n_cand ? 3 : 2;
  return p;
}

// Lane l's 64-bit value (l wave-uniform).
__device__ __forceinline__ uint64_t readlane_u64(uint64_t x, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), l);
  return ((uint64_t)hi << 32) | lo;
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

// Four simultaneous maxima over the 64 lanes (a reduce-scatter): after two
// quad exchanges each lane holds one of the four quantities reduced over its
// quad (lane % 4 = 0: a, 1: c, 2: b, 3: d); two row rotations reduce over the
// 16-lane row, two permlane swaps over rows; four readlanes make the results
// wave-uniform.
__device__ __forceinline__ void wave_max4(float& a, float& b, float& c, float& d) {
  const int lane = __lane_id();
  const bool odd = lane & 1, hi2 = lane & 2;
  const float s0 = odd ? a : c, s1 = odd ? b : d;   // what the partner lane^1 keeps
  float o0 = odd ? c : a, o1 = odd ? d : b;
  o0 = fmaxf(o0, __builtin_amdgcn_update_dpp(s0, s0, 0xb1, 0xf, 0xf, false));  // quad_perm [1,0,3,2]
  o1 = fmaxf(o1, __builtin_amdgcn_update_dpp(s1, s1, 0xb1, 0xf, 0xf, false));
  const float s = hi2 ? o0 : o1;                                               // what lane^2 keeps
  float o = hi2 ? o1 : o0;
  o = fmaxf(o, __builtin_amdgcn_update_dpp(s, s, 0x4e, 0xf, 0xf, false));      // quad_perm [2,3,0,1]
  o = fmaxf(o, __builtin_amdgcn_update_dpp(o, o, 0x124, 0xf, 0xf, false));     // row_ror:4
  o = fmaxf(o, __builtin_amdgcn_update_dpp(o, o, 0x128, 0xf, 0xf, false));     // row_ror:8
  const auto h = __builtin_amdgcn_permlane32_swap(__float_as_uint(o), __float_as_uint(o), false, false);
  o = fmaxf(__uint_as_float(h[0]), __uint_as_float(h[1]));                     // lane ^ 32
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(o), __float_as_uint(o), false, false);
  o = fmaxf(__uint_as_float(r[0]), __uint_as_float(r[1]));                     // lane ^ 16
  a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(o), 0));
  c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(o), 1));
  b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(o), 2));
  d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(o), 3));
}

// Four simultaneous sums over the 64 lanes, the reduce-scatter of wave_max4
// with additions (fixed order, so deterministic).  Afterwards lane l holds
// the total of a, c, b or d for l % 4 = 0, 1, 2, 3.
__device__ __forceinline__ float wave_sum4(float a, float b, float c, float d) {
  const int lane = __lane_id();
  const bool odd = lane & 1, hi2 = lane & 2;
  const float s0 = odd ? a : c, s1 = odd ? b : d;
  float o0 = odd ? c : a, o1 = odd ? d : b;
  o0 += __builtin_amdgcn_update_dpp(s0, s0, 0xb1, 0xf, 0xf, false);  // quad_perm [1,0,3,2]
  o1 += __builtin_amdgcn_update_dpp(s1, s1, 0xb1, 0xf, 0xf, false);
  const float s = hi2 ? o0 : o1;
  float o = hi2 ? o1 : o0;
  o += __builtin_amdgcn_update_dpp(s, s, 0x4e, 0xf, 0xf, false);      // quad_perm [2,3,0,1]
  o += __builtin_amdgcn_update_dpp(o, o, 0x124, 0xf, 0xf, false);     // row_ror:4
  o += __builtin_amdgcn_update_dpp(o, o, 0x128, 0xf, 0xf, false);     // row_ror:8
  const auto h = __builtin_amdgcn_permlane32_swap(__float_as_uint(o), __float_as_uint(o), false, false);
  o = __uint_as_float(h[0]) + __uint_as_float(h[1]);                   // lane ^ 32
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(o), __float_as_uint(o), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);               // lane ^ 16
}

// Compensated sum; a zero term leaves the state as it is, so which zero
// contributions are visited does not change the result.
__device__ __forceinline__ void kahan_add(float& sum, float& comp, float x) {
  const float y = x - comp;
  const float t = sum + y;
  const float c = (t - sum) - y;
  sum = x != 0.0f ? t : sum;
  comp = x != 0.0f ? c : comp;
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
