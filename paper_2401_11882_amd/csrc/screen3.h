// Wavefront-level candidate screen for 3D panel scenes: one lane per
// candidate, 64 candidates at a time, against the bounding box of the
// wavefront's live receivers (the 3D counterpart of screen.h).
//
// A candidate's interaction factor is exactly 0 at a receiver as soon as one
// back-trace parameter (u, beta or gamma of some interaction) lies beyond -L
// or 1 + L, L = 128 / (alpha log2 e): its exponential overflows and the
// reciprocal of the factor's denominator is 0.  The screen proves this for
// every receiver of the box at once.
//
// Why corners suffice.  Back-tracing from a point p towards the image I
// across the plane of panel (a, n, m1, m2), with q = p - a and J = I - a:
//   den = (J - q) . n,   u = -(q . n) / den,
//   beta  = ((J . n)(q . m1) - (q . n)(J . m1)) / den,
//   gamma = ((J . n)(q . m2) - (q . n)(J . m2)) / den
// (the quadratic terms of (X - a) den cancel), all ratios of affine
// functions of p with one denominator.  Where den keeps one sign over a
// convex region their extremes lie at its vertices: the 8 corners of the
// receiver box for the last interaction, then the 4 corners of the
// parameter rectangle of the next panel (a + beta e1 + gamma e2) for the
// earlier ones.  Wherever a denominator may change sign or is not clearly
// away from 0, or a panel is degenerate, the candidate is kept.
//
// Margins as in 2D: every bound is widened by 1e-4 of the ratio's condition
// number plus 1e-4 of its value, and L by a relative 1e-5, so no candidate
// that the FP32 per-receiver back-trace keeps is dropped; results with and
// without the screen are the same.
#pragma once
#include "path3d.h"

namespace drt {

struct RxBox3 {
  float x0, x1, y0, y1, z0, z1;  // wave-uniform
  bool empty;
};

__device__ __forceinline__ RxBox3 rx_box3(float rx, float ry, float rz, bool live) {
  const float I = __builtin_inff();
  float a = live ? -rx : -I, b = live ? rx : -I, c = live ? -ry : -I, d = live ? ry : -I;
  float e = live ? -rz : -I, f = live ? rz : -I, g = -I, h = -I;
  wave_max4(a, b, c, d);
  wave_max4(e, f, g, h);
  RxBox3 B;
  B.empty = !(b >= -a);
  B.x0 = uniformf(-a);
  B.x1 = uniformf(b);
  B.y0 = uniformf(-c);
  B.y1 = uniformf(d);
  B.z0 = uniformf(-e);
  B.z1 = uniformf(f);
  return B;
}

// Panel record at a per-lane index (vector loads).
__device__ __forceinline__ PanelRec load_panel_lane(const PanelRec* panels, int j) {
  const float4* p = reinterpret_cast<const float4*>(panels + j);
  const float4 a = p[0], b = p[1], c = p[2], d = p[3];
  PanelRec r;
  r.ax = a.x;
  r.ay = a.y;
  r.az = a.z;
  r.nx = a.w;
  r.ny = b.x;
  r.nz = b.y;
  r.m1x = b.z;
  r.m1y = b.w;
  r.m1z = c.x;
  r.m2x = c.y;
  r.m2y = c.z;
  r.m2z = c.w;
  r.s = d.x;
  r.nda = d.y;
  r.pad0 = r.pad1 = 0.0f;
  return r;
}

// Ranges of u, beta, gamma over NP points p_q = corner(q) for the back-trace
// towards image I across panel w.  False when a denominator is not clearly
// nonzero with one sign at every point.
template <int NP, class Corner>
__device__ __forceinline__ bool step3_ranges(const PanelRec& w, float Ix, float Iy, float Iz, Corner&& corner,
                                             float (&lo)[3], float (&hi)[3]) {
  const float I = __builtin_inff();
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    lo[k] = I;
    hi[k] = -I;
  }
  const float Jx = Ix - w.ax, Jy = Iy - w.ay, Jz = Iz - w.az;
  const float Jn = dot3(Jx, Jy, Jz, w.nx, w.ny, w.nz);
  const float J1 = dot3(Jx, Jy, Jz, w.m1x, w.m1y, w.m1z);
  const float J2 = dot3(Jx, Jy, Jz, w.m2x, w.m2y, w.m2z);
  bool pos = true, neg = true;
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    float px, py, pz;
    corner(q, px, py, pz);
    const float qx = px - w.ax, qy = py - w.ay, qz = pz - w.az;
    const float qn = dot3(qx, qy, qz, w.nx, w.ny, w.nz);
    const float q1 = dot3(qx, qy, qz, w.m1x, w.m1y, w.m1z);
    const float q2 = dot3(qx, qy, qz, w.m2x, w.m2y, w.m2z);
    const float den = Jn - qn;
    const bool clear = fabsf(den) > 1e-2f * (fabsf(Jn) + fabsf(qn));
    pos = pos & clear & (den > 0.0f);
    neg = neg & clear & (den < 0.0f);
    const float inv = 1.0f / den, ai = fabsf(inv);
    const float b1 = Jn * q1, b2 = qn * J1, g1 = Jn * q2, g2 = qn * J2;
    const float v[3] = {-qn * inv, (b1 - b2) * inv, (g1 - g2) * inv};
    const float cnd[3] = {fabsf(qn) * ai, (fabsf(b1) + fabsf(b2)) * ai, (fabsf(g1) + fabsf(g2)) * ai};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float m = 1e-4f * (cnd[k] + fabsf(v[k])) + 1e-6f;
      lo[k] = fminf(lo[k], v[k] - m);
      hi[k] = fmaxf(hi[k], v[k] + m);
    }
  }
  return pos | neg;
}

// Screen of candidate cd (order <= 3) for the receivers in box B.  False only
// if every receiver in the box has a zero interaction factor.  Panel records
// are read again where needed rather than held, to keep registers free.
template <int MAXK = 3>
__device__ __forceinline__ bool screen_candidate3(const PanelRec* panels, float lim, const Cand& cd, float tx,
                                                  float ty, float tz, const RxBox3& B) {
  if (cd.k == 0) return true;
  const int sv[3] = {cd.s0, cd.s1, cd.s2};
  float Ix[3], Iy[3], Iz[3];
  float cx = tx, cy = ty, cz = tz;
  bool ok = true;
#pragma unroll
  for (int i = 0; i < MAXK; ++i) {
    if (i < cd.k) {
      const PanelRec w = load_panel_lane(panels, sv[i]);
      ok = ok && (w.s > 0.0f);
      const float h = dot3(cx - w.ax, cy - w.ay, cz - w.az, w.nx, w.ny, w.nz) * w.s;
      cx = fmaf(-2.0f * h, w.nx, cx);
      cy = fmaf(-2.0f * h, w.ny, cy);
      cz = fmaf(-2.0f * h, w.nz, cz);
    }
    Ix[i] = cx;
    Iy[i] = cy;
    Iz[i] = cz;
  }
  if (!ok) return false;
  const float L0 = -lim, L1 = 1.0f + lim;
  // the region of X_{i+1}: the receiver box for i = K, then the rectangle
  // [b0, b1] x [g0, g1] of panel coordinates of the next panel (base, e1, e2)
  float b0 = 0.0f, b1 = 0.0f, g0 = 0.0f, g1 = 0.0f;
  float ax = 0.0f, ay = 0.0f, az = 0.0f, e1x = 0.0f, e1y = 0.0f, e1z = 0.0f, e2x = 0.0f, e2y = 0.0f, e2z = 0.0f;
#pragma unroll
  for (int i = MAXK; i >= 1; --i) {
    if (i > cd.k) continue;
    const PanelRec wi = load_panel_lane(panels, sv[i - 1]);
    float lo[3], hi[3];
    bool sgn;
    if (i == cd.k) {
      sgn = step3_ranges<8>(wi, Ix[i - 1], Iy[i - 1], Iz[i - 1], [&](int q, float& x, float& y, float& z) {
        x = (q & 1) ? B.x1 : B.x0;
        y = (q & 2) ? B.y1 : B.y0;
        z = (q & 4) ? B.z1 : B.z0;
      }, lo, hi);
    } else {
      sgn = step3_ranges<4>(wi, Ix[i - 1], Iy[i - 1], Iz[i - 1], [&](int q, float& x, float& y, float& z) {
        const float bb = (q & 1) ? b1 : b0, gg = (q & 2) ? g1 : g0;
        x = fmaf(bb, e1x, fmaf(gg, e2x, ax));
        y = fmaf(bb, e1y, fmaf(gg, e2y, ay));
        z = fmaf(bb, e1z, fmaf(gg, e2z, az));
      }, lo, hi);
    }
    if (!sgn) return true;  // cannot tell: keep
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (hi[k] < L0 || lo[k] > L1) return false;
    // X_i lies where its panel coordinates stay within [-L, 1 + L]
    b0 = fmaxf(lo[1], L0);
    b1 = fminf(hi[1], L1);
    g0 = fmaxf(lo[2], L0);
    g1 = fminf(hi[2], L1);
    ax = wi.ax;
    ay = wi.ay;
    az = wi.az;
    // edges e1 = m2 x n, e2 = n x m1
    e1x = wi.m2y * wi.nz - wi.m2z * wi.ny;
    e1y = wi.m2z * wi.nx - wi.m2x * wi.nz;
    e1z = wi.m2x * wi.ny - wi.m2y * wi.nx;
    e2x = wi.ny * wi.m1z - wi.nz * wi.m1y;
    e2y = wi.nz * wi.m1x - wi.nx * wi.m1z;
    e2z = wi.nx * wi.m1y - wi.ny * wi.m1x;
  }
  return true;
}

// Calls fn(c, cd) (wave-uniform) for every candidate of this wavefront's
// share of [c_begin, n_cand) (c = c_begin + wave + nw p, p = 0, 1, ...) that
// survives the screen, in increasing order.
template <int MAXK = 3, class Fn>
__device__ __forceinline__ void for_screened3(const PanelRec* panels, int n_panels, int c_begin, int n_cand,
                                              float lim, bool test, int wave, int nw, float tx, float ty, float tz,
                                              const RxBox3& B, Fn&& fn) {
  if (B.empty) return;
  const int lane = __lane_id();
  for (int p0 = 0; c_begin + wave + nw * p0 < n_cand; p0 += kWave) {
    const int c = c_begin + wave + nw * (p0 + lane);
    Cand cd{0, -1, -1, -1};
    bool keep = false;
    if (c < n_cand) {
      cd = decode_candidate(c, n_panels);
      keep = !test || screen_candidate3<MAXK>(panels, lim, cd, tx, ty, tz, B);
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
      fn(__builtin_amdgcn_readlane(c, j), u);
    }
  }
}

}  // namespace drt
