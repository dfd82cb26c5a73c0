// Wavefront-level candidate screen: one lane per candidate, 64 candidates at
// a time, against the bounding box of the wavefront's live receivers.
//
// A candidate's interaction factor is exactly 0 at a receiver as soon as one
// back-trace parameter (t or u of some interaction) lies beyond
// -L or 1 + L with L = 128 / (alpha log2 e): the exponential of that
// parameter overflows and the reciprocal of the factor's denominator is 0
// (the per-lane check in the back-trace).  The screen proves this for every
// receiver of the box at once and drops such candidates, so the per-receiver
// work only runs for candidates that can be nonzero somewhere in the tile.
//
// Why corners suffice.  For the last interaction, t(r) and u(r) are ratios of
// affine functions of the receiver r with the common denominator
// den(r) = (I_K - r) x e.  Where den keeps one sign over a convex region the
// level sets {t = const} are lines, so the extremes over the region are taken
// at its vertices: the four corners of the box.  The reflection points of the
// receivers that stay alive then lie on the wall within the parameter range
// found, a segment; the previous interaction sees a ratio of affine functions
// of a point of that segment, whose extremes are at the two ends.  The screen
// walks the interactions backwards this way.  Wherever a denominator may
// change sign or is not clearly away from 0, or a wall is degenerate, it
// keeps the candidate.
//
// Margins.  Every bound is widened by 1e-4 of the ratio's condition number
// plus 1e-4 |t| and the threshold L by a relative 1e-5, so the screen never
// drops a candidate that the FP32 back-trace would keep (its rounding error
// is about 1e-7 of the same condition number); the result of a kernel with
// the screen is therefore the same as without it, apart from the order of
// the zero terms in the compensated sums.
#pragma once
#include "dev.h"

namespace drt {

struct RxBox {
  float x0, x1, y0, y1;  // wave-uniform
  bool empty;
};

// Bounding box of the live lanes' receivers.
__device__ __forceinline__ RxBox rx_box(float rxx, float rxy, bool live) {
  const float I = __builtin_inff();
  float a = live ? -rxx : -I, b = live ? rxx : -I, c = live ? -rxy : -I, d = live ? rxy : -I;
  wave_max4(a, b, c, d);
  RxBox B;
  B.empty = !(b >= -a);
  B.x0 = uniformf(-a);
  B.x1 = uniformf(b);
  B.y0 = uniformf(-c);
  B.y1 = uniformf(d);
  return B;
}

// Wall record at a per-lane index (vector loads).
__device__ __forceinline__ WallRec load_wall_lane(const WallRec* walls, int j) {
  const float4* p = reinterpret_cast<const float4*>(walls + j);
  const float4 a = p[0], b = p[1];
  WallRec w;
  w.ax = a.x;
  w.ay = a.y;
  w.ex = a.z;
  w.ey = a.w;
  w.axe = b.x;
  w.inv_ee = b.y;
  w.pad1 = w.pad2 = 0.0f;
  return w;
}

// Ranges of t and u over the points P[0..NP) for the back-trace towards image
// (Ix, Iy) across wall w.  Returns false when a denominator is not clearly
// nonzero with one sign at every point.
template <int NP>
__device__ __forceinline__ bool step_ranges(const WallRec& w, float Ix, float Iy, const float (&px)[NP],
                                            const float (&py)[NP], float& tlo, float& thi, float& ulo,
                                            float& uhi) {
  const float I = __builtin_inff();
  tlo = ulo = I;
  thi = uhi = -I;
  bool pos = true, neg = true;
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const float dx = Ix - px[q], dy = Iy - py[q];
    const float wx = w.ax - px[q], wy = w.ay - py[q];
    const float a1 = dx * w.ey, a2 = dy * w.ex;
    const float den = a1 - a2;
    const bool clear = fabsf(den) > 1e-2f * (fabsf(a1) + fabsf(a2));
    pos = pos & clear & (den > 0.0f);
    neg = neg & clear & (den < 0.0f);
    const float inv = 1.0f / den;
    const float b1 = wx * dy, b2 = wy * dx;
    const float c1 = wx * w.ey, c2 = wy * w.ex;
    const float t = (b1 - b2) * inv, u = (c1 - c2) * inv;
    const float ai = fabsf(inv);
    const float mt = 1e-4f * ((fabsf(b1) + fabsf(b2)) * ai + fabsf(t)) + 1e-6f;
    const float mu = 1e-4f * ((fabsf(c1) + fabsf(c2)) * ai + fabsf(u)) + 1e-6f;
    tlo = fminf(tlo, t - mt);
    thi = fmaxf(thi, t + mt);
    ulo = fminf(ulo, u - mu);
    uhi = fmaxf(uhi, u + mu);
  }
  return pos | neg;
}

// Box, in the frame of its own axis, around every leg from a point of the
// segment [A0, A1] to a point of the convex hull of B[0..3], extended by c of
// its length at both ends: the extended ends (1 + c) a - c b and
// (1 + c) b - c a are affine in (a, b), so their extremes along an axis come
// from the extremes of the two point sets.  Axis: from the middle of A to the
// middle of B.  Grown by a relative 1e-5 against rounding.  Stored as the
// fields ux, uy, umid, uh, vmid, vh at out[f * 64].
__device__ __forceinline__ void store_leg_box(float a0x, float a0y, float a1x, float a1y, const float (&bx)[4],
                                              const float (&by)[4], float c, float* out) {
  const float dx = 0.25f * ((bx[0] + bx[1]) + (bx[2] + bx[3])) - 0.5f * (a0x + a1x);
  const float dy = 0.25f * ((by[0] + by[1]) + (by[2] + by[3])) - 0.5f * (a0y + a1y);
  const float n2 = dx * dx + dy * dy;
  const float rn = n2 > 0.0f ? rsqrtf(n2) : 0.0f;
  const float ux = n2 > 0.0f ? dx * rn : 1.0f, uy = n2 > 0.0f ? dy * rn : 0.0f;
  const float pa0 = fmaf(ux, a0x, uy * a0y), pa1 = fmaf(ux, a1x, uy * a1y);
  const float qa0 = fmaf(ux, a0y, -uy * a0x), qa1 = fmaf(ux, a1y, -uy * a1x);
  float pbl = fmaf(ux, bx[0], uy * by[0]), pbh = pbl;
  float qbl = fmaf(ux, by[0], -uy * bx[0]), qbh = qbl;
#pragma unroll
  for (int j = 1; j < 4; ++j) {
    const float p = fmaf(ux, bx[j], uy * by[j]), q = fmaf(ux, by[j], -uy * bx[j]);
    pbl = fminf(pbl, p);
    pbh = fmaxf(pbh, p);
    qbl = fminf(qbl, q);
    qbh = fmaxf(qbh, q);
  }
  const float pal = fminf(pa0, pa1), pah = fmaxf(pa0, pa1), qal = fminf(qa0, qa1), qah = fmaxf(qa0, qa1);
  const float c1 = 1.0f + c;
  const float umin = fminf(fmaf(c1, pal, -c * pbh), fmaf(c1, pbl, -c * pah));
  const float umax = fmaxf(fmaf(c1, pah, -c * pbl), fmaf(c1, pbh, -c * pal));
  const float vmin = fminf(fmaf(c1, qal, -c * qbh), fmaf(c1, qbl, -c * qah));
  const float vmax = fmaxf(fmaf(c1, qah, -c * qbl), fmaf(c1, qbh, -c * qal));
  out[0] = ux;
  out[kWave] = uy;
  out[2 * kWave] = 0.5f * (umin + umax);
  out[3 * kWave] = 0.5f * (umax - umin) + 1e-5f * (1.0f + fmaxf(fabsf(umin), fabsf(umax)));
  out[4 * kWave] = 0.5f * (vmin + vmax);
  out[5 * kWave] = 0.5f * (vmax - vmin) + 1e-5f * (1.0f + fmaxf(fabsf(vmin), fabsf(vmax)));
}

// Screen of candidate cd (order <= 3) for the receivers in box B.  Fills the
// images I_1..I_K (Ix[i-1], Iy[i-1]) with the same arithmetic as the
// per-receiver setup.  Returns false only if every receiver in the box has a
// zero interaction factor.  With `out`, stores the culling box of every leg
// l = 0..K (fields at out[(6 l + f) * 64]): X_0 = tx, X_{K+1} in the box,
// and X_i on the part of its wall where it can lie at a receiver of the box
// with a nonzero factor (the whole range -L..1+L wherever the screen cannot
// tell, or when `test` is off).
template <int MAXK = 3>
__device__ __forceinline__ bool screen_candidate(const WallRec* walls, float lim, bool test, const Cand& cd,
                                                 float txx, float txy, const RxBox& B, float (&Ix)[3],
                                                 float (&Iy)[3], float c, float* out) {
#pragma unroll
  for (int i = 0; i < 3; ++i) Ix[i] = Iy[i] = 0.0f;
  const float cbx[4] = {B.x0, B.x1, B.x0, B.x1}, cby[4] = {B.y0, B.y0, B.y1, B.y1};
  if (cd.k == 0) {
    if (out) store_leg_box(txx, txy, txx, txy, cbx, cby, c, out);
    return true;
  }
  const int sv[3] = {cd.s0, cd.s1, cd.s2};
  WallRec w[3];
  float cx = txx, cy = txy;
  bool ok = true;
#pragma unroll
  for (int i = 0; i < MAXK; ++i) {
    if (i < cd.k) {
      w[i] = load_wall_lane(walls, sv[i]);
      const float nx = -w[i].ey, ny = w[i].ex;
      ok = ok && (w[i].inv_ee > 0.0f);
      const float h = ((cx - w[i].ax) * nx + (cy - w[i].ay) * ny) * w[i].inv_ee;
      cx = cx - 2.0f * h * nx;
      cy = cy - 2.0f * h * ny;
      Ix[i] = cx;
      Iy[i] = cy;
    } else {
      w[i] = w[0];
    }
  }
  if (!ok) return false;
  const float lo = -lim, hi = 1.0f + lim;
  bool known = test;
  // ends of the range of X_{i+1} (the box corners for i = K)
  float nx4[4], ny4[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    nx4[q] = cbx[q];
    ny4[q] = cby[q];
  }
  // interactions K..1, backwards
#pragma unroll
  for (int i = MAXK; i >= 1; --i) {
    if (i > cd.k) continue;
    const WallRec& wi = w[i - 1];
    float t0 = lo, t1 = hi;
    if (known) {
      float tlo, thi, ulo, uhi;
      bool sgn;
      if (i == cd.k) {
        sgn = step_ranges<4>(wi, Ix[i - 1], Iy[i - 1], nx4, ny4, tlo, thi, ulo, uhi);
      } else {
        const float px[2] = {nx4[0], nx4[1]}, py[2] = {ny4[0], ny4[1]};
        sgn = step_ranges<2>(wi, Ix[i - 1], Iy[i - 1], px, py, tlo, thi, ulo, uhi);
      }
      if (sgn) {
        if (thi < lo || tlo > hi || uhi < lo || ulo > hi) return false;
        t0 = fmaxf(tlo, lo);
        t1 = fminf(thi, hi);
      } else {
        known = false;
      }
    }
    const float x0 = fmaf(t0, wi.ex, wi.ax), y0 = fmaf(t0, wi.ey, wi.ay);
    const float x1 = fmaf(t1, wi.ex, wi.ax), y1 = fmaf(t1, wi.ey, wi.ay);
    if (out) store_leg_box(x0, y0, x1, y1, nx4, ny4, c, out + 6 * i * kWave);   // leg i: X_i -> X_{i+1}
    nx4[0] = nx4[2] = x0;
    ny4[0] = ny4[2] = y0;
    nx4[1] = nx4[3] = x1;
    ny4[1] = ny4[3] = y1;
  }
  if (out) store_leg_box(txx, txy, txx, txy, nx4, ny4, c, out);                  // leg 0: tx -> X_1
  return true;
}

// Calls fn(c, cd, Ix, Iy, j) (wave-uniform arguments: index, decoded walls,
// images I_1..I_K, the lane that screened it) for every candidate of this
// wavefront's share of [c_begin, n_cand) that survives the screen, in
// increasing candidate order.  The share: chunks of `cchunk` consecutive
// candidates from c_begin on, chunk q going to wavefront q mod nw.  With
// `boxes` (this wavefront's LDS area of 6 (K + 1) x 64 floats), every
// candidate's leg boxes are stored there.
template <int MAXK = 3, class Fn>
__device__ __forceinline__ void for_screened(const WallRec* walls, int n_walls, int c_begin, int n_cand, float lim,
                                             bool test, int wave, int nw, int cchunk, float txx, float txy,
                                             const RxBox& B, float cull_c, float* boxes, Fn&& fn) {
  if (B.empty) return;
  const int lane = __lane_id();
  for (int p0 = 0;; p0 += kWave) {
    const int q0 = p0 / cchunk;
    if (c_begin + (wave + nw * q0) * cchunk + (p0 - q0 * cchunk) >= n_cand) break;
    const int p = p0 + lane;
    const int pq = p / cchunk;
    const int c = c_begin + (wave + nw * pq) * cchunk + (p - pq * cchunk);
    Cand cd{0, -1, -1, -1};
    float Ix[3] = {0.0f, 0.0f, 0.0f}, Iy[3] = {0.0f, 0.0f, 0.0f};
    bool keep = false;
    if (c < n_cand) {
      cd = decode_candidate(c, n_walls);
      keep = screen_candidate<MAXK>(walls, lim, test, cd, txx, txy, B, Ix, Iy, cull_c, boxes ? boxes + lane : nullptr);
    }
    uint64_t m = ballot(keep);
    while (m) {
      const int j = __builtin_ctzll(m);
      m &= m - 1;
      Cand u;
      u.k = __builtin_amdgcn_readlane(cd.k, j);
      u.s0 = __builtin_amdgcn_readlane(cd.s0, j);
      u.s1 = __builtin_amdgcn_readlane(cd.s1, j);
      u.s2 = __builtin_amdgcn_readlane(cd.s2, j);
      const int cu = __builtin_amdgcn_readlane(c, j);
      float jx[3] = {0.0f, 0.0f, 0.0f}, jy[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int i = 0; i < MAXK; ++i) {
        jx[i] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(Ix[i]), j));
        jy[i] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(Iy[i]), j));
      }
      fn(cu, u, jx, jy, j);
    }
  }
}

}  // namespace drt
