// Per-(receiver, candidate) evaluation of the smoothed image-method path in
// 3D scenes of parallelogram panels, and its adjoint.  One lane = one
// receiver; the candidate and the panel under test are wave-uniform.
//
// A panel {a + beta (b - a) + gamma (c - a): beta, gamma in [0, 1]} keeps, in
// its prepared record, a, the normal n = (b - a) x (c - a), s = 1 / (n . n),
// n . a, and the vectors m1 = ((c - a) x n) s, m2 = (n x (b - a)) s with
// beta = (x - a) . m1 and gamma = (x - a) . m2 for x in its plane.  Every
// step is the 2D step with the wall replaced by the panel (the method does
// not depend on the dimension, Sec. VI): mirror across the plane, back-trace
// to the plane, the validity of an interaction in(beta) in(gamma) in(u) and
// the obstruction factor 1 - in(upsilon) in(beta) in(gamma), with in(x) =
// s(alpha x) s(alpha (1 - x)) and s the sigmoid (Sec. V-A, Eq. 3-4).
//
// The adjoint accumulates, per panel, the gradients with respect to the
// record's a, n, m1, m2 and s (13 numbers); a final kernel maps them to the
// corners a, b, c.
#pragma once
#include "dev.h"

namespace drt {

struct PanelRec {
  float ax, ay, az, nx, ny, nz, m1x, m1y, m1z, m2x, m2y, m2z, s, nda, pad0, pad1;
};

// Panel record at a wave-uniform index, through the scalar data cache (the
// records are written by an earlier launch).
__device__ __forceinline__ PanelRec load_panel(const PanelRec* panels, int j) {
  typedef __attribute__((address_space(4))) const float* ConstF;
  const int ju = __builtin_amdgcn_readfirstlane(j);
  const ConstF p = (ConstF)(panels + ju);
  PanelRec r;
  r.ax = p[0];
  r.ay = p[1];
  r.az = p[2];
  r.nx = p[3];
  r.ny = p[4];
  r.nz = p[5];
  r.m1x = p[6];
  r.m1y = p[7];
  r.m1z = p[8];
  r.m2x = p[9];
  r.m2y = p[10];
  r.m2z = p[11];
  r.s = p[12];
  r.nda = p[13];
  r.pad0 = r.pad1 = 0.0f;
  return r;
}

__device__ __forceinline__ float dot3(float ax, float ay, float az, float bx, float by, float bz) {
  return fmaf(ax, bx, fmaf(ay, by, az * bz));
}

// Culling data of a panel: the axis-aligned box of the panel extended by
// cull_c of each edge beyond both ends (centre c, half extents h, grown by a
// relative 1e-5), its plane (n, n . a) and the scale of its coordinates for
// the rounding margin of the plane test.
struct PanelBox {
  float cx, cy, cz, hx, hy, hz, nx, ny, nz, nda, scale, pad;
};

struct Scene3View {
  const PanelRec* panels;
  const PanelBox* boxes;  // NULL: no culling
  int n_panels;
  int mask_nb;            // 64-panel batches per leg in a recorded culling mask
  float alpha, a2, band_k, dmin2, cull_c;
  float a6, a6h, a6m;     // hard sigmoid: alpha / 6, alpha / 6 + 1/2, 1/2 - alpha / 6
};

// Hard sigmoid (Eq. 5-6): in(x) = hs(alpha x) hs(alpha (1 - x)) with
// hs(z) = clamp(z / 6 + 1/2, 0, 1); h1 = hs(alpha x), h2 = hs(alpha (1 - x)).
struct HardIn {
  float h1, h2, in, n;  // n = 1 - in = (1 - h1) + h1 (1 - h2), a sum of nonnegative terms
};

__device__ __forceinline__ HardIn hard_in(const Scene3View& S, float x) {
  HardIn r;
  r.h1 = med01(fmaf(S.a6, x, 0.5f));
  r.h2 = med01(fmaf(-S.a6, x, S.a6h));
  r.in = r.h1 * r.h2;
  r.n = fmaf(r.h1, med01(fmaf(S.a6, x, S.a6m)), med01(fmaf(-S.a6, x, 0.5f)));
  return r;
}

// d in(x) / dx divided by alpha / 6: h2 where hs(alpha x) is on its ramp,
// minus h1 where hs(alpha (1 - x)) is (0 on the flat parts; the kinks take 0).
__device__ __forceinline__ float ramp3(const HardIn& r) {
  return (((r.h1 > 0.0f) & (r.h1 < 1.0f)) ? r.h2 : 0.0f) - (((r.h2 > 0.0f) & (r.h2 < 1.0f)) ? r.h1 : 0.0f);
}

// d log in(x) / dx divided by alpha / 6 (on the ramps, where in(x) > 0).
__device__ __forceinline__ float dlog_ramp3(const HardIn& r) {
  return (((r.h1 > 0.0f) & (r.h1 < 1.0f)) ? rcp(r.h1) : 0.0f) - (((r.h2 > 0.0f) & (r.h2 < 1.0f)) ? rcp(r.h2) : 0.0f);
}

// Wave-uniform axis-aligned box around the extended legs
// [X_l - c D, X_{l+1} + c D] of the active lanes.  A panel whose extended box
// misses it, or whose plane does not cut it, cannot give an in-band test on
// that leg in any of those lanes: the crossing point would have to lie in
// both.
struct LegBox3 {
  float cx, cy, cz, hx, hy, hz;
  bool empty;
};

template <int K>
struct Path3 {
  static constexpr int KI = K > 0 ? K : 1;
  float Ix[K + 1], Iy[K + 1], Iz[K + 1];   // images (wave-uniform values)
  float Xx[K + 2], Xy[K + 2], Xz[K + 2];   // X_0 = tx .. X_{K+1} = r
  float u[KI], be[KI], ga[KI], inv[KI];    // interaction i at i - 1
  float dx[KI], dy[KI], dz[KI];            // d = I_i - X_{i+1}
  float h[KI];                             // mirror offsets ((I_{i-1} - a) . n) s
  int s[KI];
  int lo[K + 1], hi[K + 1];
  float F;
};

// d log in(x) / dx = alpha (E1 / (1 + E1) - E2 / (1 + E2)), E1 = e^(-alpha x), E2 = e^(-alpha (1 - x)).
__device__ __forceinline__ float dlog_in(float x, float alpha, float a2) {
  const float E1 = ex2(-a2 * x), E2 = ex2(fmaf(a2, x, -a2));
  const float r1 = E1 < kBig ? E1 * rcp(1.0f + E1) : 1.0f;
  const float r2 = E2 < kBig ? E2 * rcp(1.0f + E2) : 1.0f;
  return alpha * (r1 - r2);
}

// Images, back-trace and (if WANT_F) the interaction factors; with WANT_F,
// false as soon as every lane's factor is exactly 0.
template <int K, bool WANT_F, int MODE>
__device__ __forceinline__ bool setup3(const Scene3View& S, const Cand& cd, float tx, float ty, float tz,
                                       float rx, float ry, float rz, bool live, Path3<K>& P) {
  const int sv[3] = {cd.s0, cd.s1, cd.s2};
#pragma unroll
  for (int i = 0; i < Path3<K>::KI; ++i) P.s[i] = (i < K) ? sv[i] : -1;
#pragma unroll
  for (int l = 0; l <= K; ++l) {
    P.lo[l] = (l >= 1) ? sv[l - 1] : -1;
    P.hi[l] = (l + 1 <= K) ? sv[l] : -1;
  }
  P.Ix[0] = tx;
  P.Iy[0] = ty;
  P.Iz[0] = tz;
  bool ok = live;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const PanelRec w = load_panel(S.panels, P.s[i]);
    ok = ok && (w.s > 0.0f);
    const float h = dot3(P.Ix[i] - w.ax, P.Iy[i] - w.ay, P.Iz[i] - w.az, w.nx, w.ny, w.nz) * w.s;
    P.h[i] = h;
    P.Ix[i + 1] = fmaf(-2.0f * h, w.nx, P.Ix[i]);
    P.Iy[i + 1] = fmaf(-2.0f * h, w.ny, P.Iy[i]);
    P.Iz[i + 1] = fmaf(-2.0f * h, w.nz, P.Iz[i]);
  }
  P.Xx[0] = tx;
  P.Xy[0] = ty;
  P.Xz[0] = tz;
  P.Xx[K + 1] = rx;
  P.Xy[K + 1] = ry;
  P.Xz[K + 1] = rz;
  float F = ok ? 1.0f : 0.0f;
#pragma unroll
  for (int i = K; i >= 1; --i) {
    const PanelRec w = load_panel(S.panels, P.s[i - 1]);
    const float dx = P.Ix[i] - P.Xx[i + 1], dy = P.Iy[i] - P.Xy[i + 1], dz = P.Iz[i] - P.Xz[i + 1];
    const float den = dot3(dx, dy, dz, w.nx, w.ny, w.nz);
    const bool good = den != 0.0f;
    const float inv = good ? rcp(den) : 0.0f;
    const float u = (w.nda - dot3(P.Xx[i + 1], P.Xy[i + 1], P.Xz[i + 1], w.nx, w.ny, w.nz)) * inv;
    P.Xx[i] = fmaf(u, dx, P.Xx[i + 1]);
    P.Xy[i] = fmaf(u, dy, P.Xy[i + 1]);
    P.Xz[i] = fmaf(u, dz, P.Xz[i + 1]);
    const float qx = P.Xx[i] - w.ax, qy = P.Xy[i] - w.ay, qz = P.Xz[i] - w.az;
    const float be = dot3(qx, qy, qz, w.m1x, w.m1y, w.m1z);
    const float ga = dot3(qx, qy, qz, w.m2x, w.m2y, w.m2z);
    P.u[i - 1] = u;
    P.be[i - 1] = be;
    P.ga[i - 1] = ga;
    P.inv[i - 1] = inv;
    P.dx[i - 1] = dx;
    P.dy[i - 1] = dy;
    P.dz[i - 1] = dz;
    if constexpr (WANT_F && MODE == kHardSigmoid) {
      // exactly 0 beyond 3 / alpha outside [0, 1]
      F = good ? F : 0.0f;
      F *= (hard_in(S, be).in * hard_in(S, ga).in) * hard_in(S, u).in;
      if (ballot(F != 0.0f) == 0) {
        P.F = 0.0f;
        return false;
      }
    } else if constexpr (WANT_F) {
      F = good ? F : 0.0f;
      const float z1 = -S.a2 * be, z2 = fmaf(S.a2, be, -S.a2);
      const float z3 = -S.a2 * ga, z4 = fmaf(S.a2, ga, -S.a2);
      const float z5 = -S.a2 * u, z6 = fmaf(S.a2, u, -S.a2);
      const bool zero = (F == 0.0f) | (z1 >= 128.0f) | (z2 >= 128.0f) | (z3 >= 128.0f) | (z4 >= 128.0f) |
                        (z5 >= 128.0f) | (z6 >= 128.0f);
      if (ballot(!zero) == 0) {
        P.F = 0.0f;
        return false;
      }
      const float E1 = ex2(z1), E2 = ex2(z2), E3 = ex2(z3), E4 = ex2(z4), E5 = ex2(z5), E6 = ex2(z6);
      F *= rcp(((1.0f + E1) * (1.0f + E2)) * ((1.0f + E3) * (1.0f + E4)) * ((1.0f + E5) * (1.0f + E6)));
    }
  }
  P.F = F;
  return true;
}

// Sigmoid: 1 - in(ups) in(beta) in(gamma) = num / (1 + num) with
// num = (1 + n_u)(1 + n_b)(1 + n_g) - 1 expanded into positive terms,
// n_x = E1 + E2 + E1 E2 (E1 = e^(-alpha x), E2 = e^(-alpha (1 - x))).
struct Obs3 {
  float ups, be, ga, inv, qx, qy, qz, num;  // num: sigmoid num; hard sigmoid: the factor q itself
  // sigmoid: per parameter (ups, beta, gamma) E1 - E2 and A = (1 + E1)(1 + E2) = 1 + n
  float dE[3], A[3];
};

// Obstruction test of leg (X, D) by panel w: false if every lane's factor is
// 1.0f (a parameter more than band outside [0, 1]); the leg parameter first.
template <int MODE>
__device__ __forceinline__ bool obs3(const Scene3View& S, const PanelRec& w, float Xx, float Xy, float Xz, float Dx,
                                     float Dy, float Dz, bool act, Obs3& o, bool& in_band) {
  const float den = dot3(Dx, Dy, Dz, w.nx, w.ny, w.nz);
  const float num = w.nda - dot3(Xx, Xy, Xz, w.nx, w.ny, w.nz);  // (a - X) . n
  bool it = act && (fabsf(fmaf(2.0f, num, -den)) < S.band_k * fabsf(den));
  in_band = false;
  if (ballot(it) == 0) return false;
  o.inv = rcp(den);
  o.ups = num * o.inv;
  const float Hx = fmaf(o.ups, Dx, Xx), Hy = fmaf(o.ups, Dy, Xy), Hz = fmaf(o.ups, Dz, Xz);
  o.qx = Hx - w.ax;
  o.qy = Hy - w.ay;
  o.qz = Hz - w.az;
  o.be = dot3(o.qx, o.qy, o.qz, w.m1x, w.m1y, w.m1z);
  o.ga = dot3(o.qx, o.qy, o.qz, w.m2x, w.m2y, w.m2z);
  it = it && (fabsf(fmaf(2.0f, o.be, -1.0f)) < S.band_k) && (fabsf(fmaf(2.0f, o.ga, -1.0f)) < S.band_k);
  if (ballot(it) == 0) return false;
  in_band = it;
  if constexpr (MODE == kHardSigmoid) {
    // q = 1 - in_u in_b in_g = n_u + in_u (n_b + in_b n_g): nonnegative terms
    const HardIn u = hard_in(S, o.ups), b = hard_in(S, o.be), g = hard_in(S, o.ga);
    o.num = it ? fmaf(u.in, fmaf(b.in, g.n, b.n), u.n) : 1.0f;
  } else {
    if (it) {
      const float x[3] = {o.ups, o.be, o.ga};
      float n[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float E1 = ex2(-S.a2 * x[k]), E2 = ex2(fmaf(S.a2, x[k], -S.a2));
        n[k] = fmaf(E1, E2, E1 + E2);
        o.dE[k] = E1 - E2;
        o.A[k] = 1.0f + n[k];
      }
      const float t = fmaf(n[0], n[1], n[0] + n[1]);
      o.num = fmaf(t, n[2], t + n[2]);
    } else {
      o.num = kBig;
    }
  }
  return true;
}

template <int K>
__device__ __forceinline__ void leg_boxes3(const Path3<K>& P, bool act, float c, LegBox3 (&B)[K + 1]) {
  const float I = __builtin_inff();
  const bool none = ballot(act) == 0;
#pragma unroll
  for (int l = 0; l <= K; ++l) {
    const float Dx = P.Xx[l + 1] - P.Xx[l], Dy = P.Xy[l + 1] - P.Xy[l], Dz = P.Xz[l + 1] - P.Xz[l];
    const float p0x = fmaf(-c, Dx, P.Xx[l]), p0y = fmaf(-c, Dy, P.Xy[l]), p0z = fmaf(-c, Dz, P.Xz[l]);
    const float p1x = fmaf(c, Dx, P.Xx[l + 1]), p1y = fmaf(c, Dy, P.Xy[l + 1]), p1z = fmaf(c, Dz, P.Xz[l + 1]);
    // maxima of -lo and hi over the active lanes (others give -inf)
    float a = act ? -fminf(p0x, p1x) : -I, b = act ? -fminf(p0y, p1y) : -I;
    float cc = act ? -fminf(p0z, p1z) : -I, d = act ? fmaxf(p0x, p1x) : -I;
    float e = act ? fmaxf(p0y, p1y) : -I, f = act ? fmaxf(p0z, p1z) : -I, g = -I, h = -I;
    wave_max4(a, b, cc, d);
    wave_max4(e, f, g, h);
    B[l].empty = none;
    if (none) a = b = cc = d = e = f = 0.0f;
    const float hx = 0.5f * (d + a), hy = 0.5f * (e + b), hz = 0.5f * (f + cc);
    B[l].cx = uniformf(0.5f * (d - a));
    B[l].cy = uniformf(0.5f * (e - b));
    B[l].cz = uniformf(0.5f * (f - cc));
    B[l].hx = uniformf(hx + 1e-5f * (fabsf(B[l].cx) + hx));
    B[l].hy = uniformf(hy + 1e-5f * (fabsf(B[l].cy) + hy));
    B[l].hz = uniformf(hz + 1e-5f * (fabsf(B[l].cz) + hz));
  }
}

// Calls fn(panel, masks, bit) for every panel not culled for some leg, in
// increasing order; masks[l] bit `bit` says whether leg l needs the test (a
// leg's own end panels excluded).  Lane j checks panel b + j of each batch of
// 64.  Without culling data every panel is visited.
// The mask of batch i for leg l is word l * nb + i of a candidate's record
// (nb = S.mask_nb, (K + 1) nb <= 64 words).  With mask_out (the wavefront's
// LDS record) each computed mask is written there; with mask_in (one word per
// lane, lane = word) the masks are taken from it (the boxes are then not
// used), so an adjoint visits exactly the panels its forward visited.
template <int K, class Fn>
__device__ __forceinline__ void visit_panels(const Scene3View& S, const Path3<K>& P, const LegBox3 (&B)[K + 1],
                                             Fn&& fn, uint64_t* mask_out = nullptr,
                                             const uint64_t* mask_in = nullptr) {
  const int lane = threadIdx.x & (kWave - 1);
  for (int b = 0, bi = 0; b < S.n_panels; b += kWave, ++bi) {
    const int pj = b + lane;
    const bool valid = pj < S.n_panels;
    uint64_t m[K + 1];
    uint64_t uni = 0;
    if (mask_in) {
#pragma unroll
      for (int l = 0; l <= K; ++l) {
        m[l] = readlane_u64(*mask_in, l * S.mask_nb + bi);
        uni |= m[l];
      }
    } else if (S.boxes) {
      PanelBox q;
      if (valid) {
        q = S.boxes[pj];
      } else {
        q.cx = q.cy = q.cz = q.hx = q.hy = q.hz = q.nx = q.ny = q.nz = q.nda = q.scale = q.pad = 0.0f;
      }
      const float an = fabsf(q.nx) + fabsf(q.ny) + fabsf(q.nz);
#pragma unroll
      for (int l = 0; l <= K; ++l) {
        const LegBox3& L = B[l];
        const bool sep_box = (fabsf(q.cx - L.cx) > q.hx + L.hx) | (fabsf(q.cy - L.cy) > q.hy + L.hy) |
                             (fabsf(q.cz - L.cz) > q.hz + L.hz);
        const float ext = fmaf(fabsf(q.nx), L.hx, fmaf(fabsf(q.ny), L.hy, fabsf(q.nz) * L.hz));
        const float mar = 1e-5f * an * (fabsf(L.cx) + fabsf(L.cy) + fabsf(L.cz) + L.hx + L.hy + L.hz + q.scale);
        const bool sep_plane = fabsf(dot3(q.nx, q.ny, q.nz, L.cx, L.cy, L.cz) - q.nda) > ext + mar;
        const bool ov = valid & !L.empty & !sep_box & !sep_plane & (pj != P.lo[l]) & (pj != P.hi[l]);
        m[l] = ballot(ov);
        uni |= m[l];
        if (mask_out && lane == 0) mask_out[l * S.mask_nb + bi] = m[l];
      }
    } else {
#pragma unroll
      for (int l = 0; l <= K; ++l) {
        m[l] = ballot(valid & !B[l].empty & (pj != P.lo[l]) & (pj != P.hi[l]));
        uni |= m[l];
        if (mask_out && lane == 0) mask_out[l * S.mask_nb + bi] = m[l];
      }
    }
    while (uni) {
      const int j = __builtin_ctzll(uni);
      uni &= uni - 1;
      if (!fn(b + j, m, j)) return;
    }
  }
}

template <int K, int MODE>
__device__ __forceinline__ float obstruct_all3(const Scene3View& S, const Path3<K>& P, float V,
                                               uint64_t* mask_out = nullptr, float vcut = 0.0f) {
  const bool act = P.F != 0.0f;
  LegBox3 B[K + 1];
  if (S.boxes) {
    leg_boxes3<K>(P, act, S.cull_c, B);
  } else {
    const bool none = ballot(act) == 0;
#pragma unroll
    for (int l = 0; l <= K; ++l) B[l].empty = none;
  }
  visit_panels<K>(S, P, B, [&](int j, const uint64_t* m, int bit) {
    const PanelRec w = load_panel(S.panels, j);
    bool upd = false;
#pragma unroll
    for (int l = 0; l <= K; ++l) {
      if (((m[l] >> bit) & 1ull) == 0) continue;
      const float Dx = P.Xx[l + 1] - P.Xx[l], Dy = P.Xy[l + 1] - P.Xy[l], Dz = P.Xz[l + 1] - P.Xz[l];
      Obs3 o;
      bool ib;
      if (!obs3<MODE>(S, w, P.Xx[l], P.Xy[l], P.Xz[l], Dx, Dy, Dz, act, o, ib)) continue;
      if (ib) {
        if constexpr (MODE == kHardSigmoid) V *= o.num;
        else V *= o.num * rcp(1.0f + o.num);
        upd = true;
      }
    }
    // a lane whose product fell to its cut contributes nothing; once every
    // lane's product is 0 no further factor can change it
    if constexpr (uses_cut<MODE>()) V = V > vcut ? V : 0.0f;
    return ballot(upd) == 0 || ballot(V != 0.0f) != 0;
  }, mask_out);
  return V;
}

template <int K, int MODE>
__device__ __forceinline__ float path_power3(const Scene3View& S, const Cand& cd, float tx, float ty, float tz,
                                             float rx, float ry, float rz, bool live, uint64_t* mask_out,
                                             float scut) {
  Path3<K> P;
  if (!setup3<K, true, MODE>(S, cd, tx, ty, tz, rx, ry, rz, live, P)) return 0.0f;
  const float ex = rx - P.Ix[K], ey = ry - P.Iy[K], ez = rz - P.Iz[K];
  if constexpr (!uses_cut<MODE>()) {
    if (ballot(P.F != 0.0f) == 0) return 0.0f;
    const float V = obstruct_all3<K, MODE>(S, P, P.F, mask_out);
    return V / fmaxf(dot3(ex, ey, ez, ex, ey, ez), S.dmin2);
  } else {
    const float dd = fmaxf(dot3(ex, ey, ez, ex, ey, ez), S.dmin2);
    const float vcut = scut * dd;  // the contribution V / dd is below the cut once V <= vcut
    P.F = P.F > vcut ? P.F : 0.0f;
    if (ballot(P.F != 0.0f) == 0) return 0.0f;
    const float V = obstruct_all3<K, MODE>(S, P, P.F, mask_out, vcut);
    return V / dd;
  }
}

// Per-wave accumulator layout: [0..2] = d/dtx, [3 + 13 j + f] = d/d record of
// panel j with f: a (0..2), n (3..5), m1 (6..8), m2 (9..11), s (12).
constexpr int kPanelGrad = 13;

__device__ __forceinline__ void acc_panel(float* acc, int j, const float (&g)[kPanelGrad], int lane) {
  float* p = acc + 3 + kPanelGrad * j;
#pragma unroll
  for (int b = 0; b < 12; b += 4) {
    const float s = wave_sum4(g[b], g[b + 1], g[b + 2], g[b + 3]);
    if (lane < 4) p[b + ((lane & 1) << 1) + ((lane >> 1) & 1)] += s;
  }
  const float s12 = wave_sum(g[12]);
  if (lane == 0) p[12] += s12;
}

struct LaneGrad3 {
  float tx, ty, tz;  // transmitter (summed over lanes later)
  float rx, ry, rz;  // this lane's receiver
};

// Reverse sweep of one path given Wl = g(r) c (= dL / dlog V at this lane).
template <int K, int MODE>
__device__ __forceinline__ void path_adjoint3(const Scene3View& S, const Path3<K>& P, float Wl, float rx, float ry,
                                              float rz, float* acc, int lane, LaneGrad3& G,
                                              const uint64_t* mask_in = nullptr) {
  const bool act = Wl != 0.0f;
  // gradients of the path points X_0 .. X_{K+1} and of the images
  float gXx[K + 2], gXy[K + 2], gXz[K + 2], gIx[K + 1], gIy[K + 1], gIz[K + 1];
#pragma unroll
  for (int i = 0; i < K + 2; ++i) gXx[i] = gXy[i] = gXz[i] = 0.0f;
#pragma unroll
  for (int i = 0; i < K + 1; ++i) gIx[i] = gIy[i] = gIz[i] = 0.0f;

  // -- obstruction factors: d log q / d(ups, beta, gamma) = -L_x / num
  // culling masks recorded by the forward, or boxes around the legs of the
  // lanes with a nonzero W
  LegBox3 B[K + 1];
  if (mask_in) {
  } else if (S.boxes) {
    leg_boxes3<K>(P, act, S.cull_c, B);
  } else {
    const bool none = ballot(act) == 0;
#pragma unroll
    for (int l = 0; l <= K; ++l) B[l].empty = none;
  }
  visit_panels<K>(S, P, B, [&](int j, const uint64_t* m, int bit) {
    const PanelRec w = load_panel(S.panels, j);
    float g[kPanelGrad];
#pragma unroll
    for (int f = 0; f < kPanelGrad; ++f) g[f] = 0.0f;
    bool any = false;
#pragma unroll
    for (int l = 0; l <= K; ++l) {
      if (((m[l] >> bit) & 1ull) == 0) continue;
      const float Dx = P.Xx[l + 1] - P.Xx[l], Dy = P.Xy[l + 1] - P.Xy[l], Dz = P.Xz[l + 1] - P.Xz[l];
      Obs3 o;
      bool ib;
      if (!obs3<MODE>(S, w, P.Xx[l], P.Xy[l], P.Xz[l], Dx, Dy, Dz, act, o, ib)) continue;
      if (!ib) continue;
      float gu, gb, gg;  // Wl d log q / d(ups, beta, gamma)
      if constexpr (MODE == kHardSigmoid) {
        // q = 1 - in_u in_b in_g, dq/dx_u = -in'_u in_b in_g (likewise)
        const HardIn hu = hard_in(S, o.ups), hb = hard_in(S, o.be), hg = hard_in(S, o.ga);
        const float c = o.num > 0.0f ? -S.a6 * Wl * rcp(o.num) : 0.0f;
        gu = c * ramp3(hu) * (hb.in * hg.in);
        gb = c * ramp3(hb) * (hu.in * hg.in);
        gg = c * ramp3(hg) * (hu.in * hb.in);
      } else {
        // q = num / (1 + num), 1 + num = A_u A_b A_g: d log q / dx = alpha (E2 - E1) / (A_x num)
        // (E1, E2 <= e^18 within the band, so A_x num stays finite)
        const float c = -S.alpha * Wl;
        gu = c * o.dE[0] * rcp(o.A[0] * o.num);
        gb = c * o.dE[1] * rcp(o.A[1] * o.num);
        gg = c * o.dE[2] * rcp(o.A[2] * o.num);
      }
      // beta = q . m1, gamma = q . m2, q = X + ups D - a
      const float gqx = fmaf(gb, w.m1x, gg * w.m2x), gqy = fmaf(gb, w.m1y, gg * w.m2y),
                  gqz = fmaf(gb, w.m1z, gg * w.m2z);
      g[6] += gb * o.qx;
      g[7] += gb * o.qy;
      g[8] += gb * o.qz;
      g[9] += gg * o.qx;
      g[10] += gg * o.qy;
      g[11] += gg * o.qz;
      const float gut = gu + dot3(gqx, gqy, gqz, Dx, Dy, Dz);  // total d/d ups
      // ups = ((a - X) . n) / (D . n)
      const float gnum = gut * o.inv, gden = -gut * o.ups * o.inv;
      const float w0x = w.ax - P.Xx[l], w0y = w.ay - P.Xy[l], w0z = w.az - P.Xz[l];
      // d/dX_l: +gq (q) - gnum n (num) ; d/dD: ups gq + gden n
      const float gDx = fmaf(o.ups, gqx, gden * w.nx), gDy = fmaf(o.ups, gqy, gden * w.ny),
                  gDz = fmaf(o.ups, gqz, gden * w.nz);
      gXx[l] += gqx - gnum * w.nx - gDx;
      gXy[l] += gqy - gnum * w.ny - gDy;
      gXz[l] += gqz - gnum * w.nz - gDz;
      gXx[l + 1] += gDx;
      gXy[l + 1] += gDy;
      gXz[l + 1] += gDz;
      // panel record: a (q and num), n (num and den)
      g[0] += fmaf(gnum, w.nx, -gqx);
      g[1] += fmaf(gnum, w.ny, -gqy);
      g[2] += fmaf(gnum, w.nz, -gqz);
      g[3] += fmaf(gnum, w0x, gden * Dx);
      g[4] += fmaf(gnum, w0y, gden * Dy);
      g[5] += fmaf(gnum, w0z, gden * Dz);
      any = true;
    }
    if (ballot(any) != 0) acc_panel(acc, j, g, lane);
    return true;
  }, nullptr, mask_in);

  // -- image distance |r - I_K|^2 (zero gradient under the d_min floor)
  {
    const float ex = rx - P.Ix[K], ey = ry - P.Iy[K], ez = rz - P.Iz[K];
    const float d2 = dot3(ex, ey, ez, ex, ey, ez);
    if (d2 > S.dmin2) {
      const float f = 2.0f * Wl / d2;
      gIx[K] += f * ex;
      gIy[K] += f * ey;
      gIz[K] += f * ez;
      gXx[K + 1] -= f * ex;
      gXy[K + 1] -= f * ey;
      gXz[K + 1] -= f * ez;
    }
  }
  // -- interactions i = 1 .. K: the back-trace made X_i from X_{i+1}, so its
  // reverse runs from X_1 upwards (X_i's gradient is complete when reached)
#pragma unroll
  for (int i = 1; i <= K; ++i) {
    const PanelRec w = load_panel(S.panels, P.s[i - 1]);
    const float u = P.u[i - 1], inv = P.inv[i - 1];
    const float dx = P.dx[i - 1], dy = P.dy[i - 1], dz = P.dz[i - 1];
    float gb, gg, gu;  // Wl d log in / d(beta, gamma, u)
    if constexpr (MODE == kHardSigmoid) {
      const float aw = S.a6 * Wl;
      gb = aw * dlog_ramp3(hard_in(S, P.be[i - 1]));
      gg = aw * dlog_ramp3(hard_in(S, P.ga[i - 1]));
      gu = aw * dlog_ramp3(hard_in(S, u));
    } else {
      gb = Wl * dlog_in(P.be[i - 1], S.alpha, S.a2);
      gg = Wl * dlog_in(P.ga[i - 1], S.alpha, S.a2);
      gu = Wl * dlog_in(u, S.alpha, S.a2);
    }
    float g[kPanelGrad];
#pragma unroll
    for (int f = 0; f < kPanelGrad; ++f) g[f] = 0.0f;
    // beta = q . m1, gamma = q . m2 with q = X_i - a
    const float qx = P.Xx[i] - w.ax, qy = P.Xy[i] - w.ay, qz = P.Xz[i] - w.az;
    const float gqx = fmaf(gb, w.m1x, gg * w.m2x), gqy = fmaf(gb, w.m1y, gg * w.m2y),
                gqz = fmaf(gb, w.m1z, gg * w.m2z);
    g[6] = gb * qx;
    g[7] = gb * qy;
    g[8] = gb * qz;
    g[9] = gg * qx;
    g[10] = gg * qy;
    g[11] = gg * qz;
    g[0] = -gqx;
    g[1] = -gqy;
    g[2] = -gqz;
    const float gXix = gXx[i] + gqx, gXiy = gXy[i] + gqy, gXiz = gXz[i] + gqz;
    // X_i = X_{i+1} + u d
    const float gut = gu + dot3(gXix, gXiy, gXiz, dx, dy, dz);
    float gdx = u * gXix, gdy = u * gXiy, gdz = u * gXiz;
    gXx[i + 1] += gXix;
    gXy[i + 1] += gXiy;
    gXz[i + 1] += gXiz;
    // u = ((a - X_{i+1}) . n) / (d . n)
    const float gnum = gut * inv, gden = -gut * u * inv;
    const float wx = w.ax - P.Xx[i + 1], wy = w.ay - P.Xy[i + 1], wz = w.az - P.Xz[i + 1];
    g[0] += gnum * w.nx;
    g[1] += gnum * w.ny;
    g[2] += gnum * w.nz;
    gXx[i + 1] -= gnum * w.nx;
    gXy[i + 1] -= gnum * w.ny;
    gXz[i + 1] -= gnum * w.nz;
    g[3] = fmaf(gnum, wx, gden * dx);
    g[4] = fmaf(gnum, wy, gden * dy);
    g[5] = fmaf(gnum, wz, gden * dz);
    gdx = fmaf(gden, w.nx, gdx);
    gdy = fmaf(gden, w.ny, gdy);
    gdz = fmaf(gden, w.nz, gdz);
    // d = I_i - X_{i+1}
    gIx[i] += gdx;
    gIy[i] += gdy;
    gIz[i] += gdz;
    gXx[i + 1] -= gdx;
    gXy[i + 1] -= gdy;
    gXz[i + 1] -= gdz;
    acc_panel(acc, P.s[i - 1], g, lane);
  }
  G.tx += gXx[0];
  G.ty += gXy[0];
  G.tz += gXz[0];
  G.rx += gXx[K + 1];
  G.ry += gXy[K + 1];
  G.rz += gXz[K + 1];
  if (K == 0) {
    // I_0 is the transmitter itself
    G.tx += gIx[0];
    G.ty += gIy[0];
    G.tz += gIz[0];
    return;
  }
  // -- images, on wave-uniform values after one reduction over the lanes:
  // I_i = I_{i-1} - 2 h n with h = ((I_{i-1} - a) . n) s, for i = K .. 1
  float GIx[K + 1], GIy[K + 1], GIz[K + 1];
#pragma unroll
  for (int i = 1; i <= K; ++i) {
    GIx[i] = wave_sum(gIx[i]);
    GIy[i] = wave_sum(gIy[i]);
    GIz[i] = wave_sum(gIz[i]);
  }
  GIx[0] = GIy[0] = GIz[0] = 0.0f;
#pragma unroll
  for (int i = K; i >= 1; --i) {
    const PanelRec w = load_panel(S.panels, P.s[i - 1]);
    const float h = P.h[i - 1];
    const float pdx = P.Ix[i - 1] - w.ax, pdy = P.Iy[i - 1] - w.ay, pdz = P.Iz[i - 1] - w.az;
    const float gh = -2.0f * dot3(GIx[i], GIy[i], GIz[i], w.nx, w.ny, w.nz);
    const float ghs = gh * w.s;
    GIx[i - 1] += fmaf(ghs, w.nx, GIx[i]);
    GIy[i - 1] += fmaf(ghs, w.ny, GIy[i]);
    GIz[i - 1] += fmaf(ghs, w.nz, GIz[i]);
    if (lane == 0) {
      float* p = acc + 3 + kPanelGrad * P.s[i - 1];
      p[0] -= ghs * w.nx;
      p[1] -= ghs * w.ny;
      p[2] -= ghs * w.nz;
      p[3] += fmaf(-2.0f * h, GIx[i], ghs * pdx);
      p[4] += fmaf(-2.0f * h, GIy[i], ghs * pdy);
      p[5] += fmaf(-2.0f * h, GIz[i], ghs * pdz);
      p[12] += gh * dot3(pdx, pdy, pdz, w.nx, w.ny, w.nz);
    }
  }
  if (lane == 0) {
    acc[0] += GIx[0];
    acc[1] += GIy[0];
    acc[2] += GIz[0];
  }
}

template <int K, int MODE>
__device__ __forceinline__ void path_adjoint3_known(const Scene3View& S, const Cand& cd, float tx, float ty,
                                                    float tz, float rx, float ry, float rz, bool live, float Wl,
                                                    float* acc, int lane, LaneGrad3& G, const uint64_t* mask_in) {
  Path3<K> P;
  setup3<K, false, MODE>(S, cd, tx, ty, tz, rx, ry, rz, live, P);
  P.F = Wl != 0.0f ? 1.0f : 0.0f;
  path_adjoint3<K, MODE>(S, P, Wl, rx, ry, rz, acc, lane, G, mask_in);
}

// Contribution of candidate cd at this lane; with mask_out, its culling masks
// are kept there (see visit_panels).  A lane drops the candidate (returns 0)
// once its contribution is provably <= scut (the contribution cut).
// (MAXK: the highest order the caller's candidates can have; the code of
// higher orders is left out.)
template <int MODE, int MAXK = 3>
__device__ __forceinline__ float candidate_power3(const Scene3View& S, const Cand& cd, float tx, float ty,
                                                  float tz, float rx, float ry, float rz, bool live,
                                                  uint64_t* mask_out = nullptr, float scut = 0.0f) {
  static_assert(MAXK >= 1 && MAXK <= 3, "orders 1..3");
  switch (cd.k) {
    case 0: return path_power3<0, MODE>(S, cd, tx, ty, tz, rx, ry, rz, live, mask_out, scut);
    case 1: return path_power3<1, MODE>(S, cd, tx, ty, tz, rx, ry, rz, live, mask_out, scut);
    case 2:
      if constexpr (MAXK >= 2) return path_power3<2, MODE>(S, cd, tx, ty, tz, rx, ry, rz, live, mask_out, scut);
      else return 0.0f;
    default:
      if constexpr (MAXK >= 3) return path_power3<3, MODE>(S, cd, tx, ty, tz, rx, ry, rz, live, mask_out, scut);
      else return 0.0f;
  }
}

// Adjoint of candidate cd given Wl = g(r) c; with mask_in, the culling masks
// its forward recorded.
template <int MODE, int MAXK = 3>
__device__ __forceinline__ void candidate_adjoint3(const Scene3View& S, const Cand& cd, float tx, float ty,
                                                   float tz, float rx, float ry, float rz, bool live, float Wl,
                                                   float* acc, int lane, LaneGrad3& G,
                                                   const uint64_t* mask_in = nullptr) {
  static_assert(MAXK >= 1 && MAXK <= 3, "orders 1..3");
  switch (cd.k) {
    case 0: path_adjoint3_known<0, MODE>(S, cd, tx, ty, tz, rx, ry, rz, live, Wl, acc, lane, G, mask_in); break;
    case 1: path_adjoint3_known<1, MODE>(S, cd, tx, ty, tz, rx, ry, rz, live, Wl, acc, lane, G, mask_in); break;
    case 2:
      if constexpr (MAXK >= 2) path_adjoint3_known<2, MODE>(S, cd, tx, ty, tz, rx, ry, rz, live, Wl, acc, lane, G, mask_in);
      break;
    default:
      if constexpr (MAXK >= 3) path_adjoint3_known<3, MODE>(S, cd, tx, ty, tz, rx, ry, rz, live, Wl, acc, lane, G, mask_in);
      break;
  }
}

}  // namespace drt
