// Per-(receiver, candidate) evaluation of the smoothed image-method path and
// its adjoint, as inline device code shared by the single-scene and the
// batched kernels.  One lane = one receiver; the candidate and the wall under
// test are wave-uniform.
//
// Method (arXiv 2401.11882): image method in the relaxed scene (Sec. V,
// Sec. V-B); every validity comparison x0 > x1 smoothed as
// s(x0 - x1) = sigmoid(alpha (x0 - x1)) (Sec. V-A, Eq. 3, Eq. 4); power
// V / max(|r - I_k|^2, d_min^2) per path (Eq. 7 with identity coefficient).
//
// Exactness of the skips used below (none changes the FP32 result):
//  * exp2(z) is +inf for z >= 128, so an interaction whose exponent argument
//    reaches 128 has in(t) in(u) = 1 / inf = 0 exactly;
//  * an obstruction test with tau or upsilon more than 18/alpha outside
//    [0, 1] has in(tau) in(ups) < e^-18 < 2^-25, so 1 - in*in rounds to 1.0f.
#pragma once
#include "dev.h"

namespace drt {

struct SceneView {
  const WallRec* walls;  // prepared records [n_walls]
  const WallBox* boxes;  // culling boxes [n_walls]
  int n_walls;
  float alpha;
  float a2;      // alpha * log2(e)
  float band_k;  // 1 + 2 * kBandMargin / alpha
  float cull_c;  // kCullMargin / alpha
  float dmin2;
  float dead_lim;  // parameter range beyond which a factor is exactly 0 (see screen.h)
  float a6, a6h, a6m;  // hard sigmoid: alpha / 6, alpha / 6 + 1/2, 1/2 - alpha / 6
  int cull;        // 1: skip (wall, leg) tests whose factor is provably 1 (culling); 0: test all
};


template <int K>
struct Path {
  static constexpr int KI = K > 0 ? K : 1;
  float Ix[K + 1], Iy[K + 1];   // images I_0 = tx .. I_K (wave-uniform values)
  float Xx[K + 2], Xy[K + 2];   // X_0 = tx, X_1..X_K interaction points, X_{K+1} = r
  float t[KI], u[KI], inv[KI];  // interaction i (stored at i-1): wall and side parameters
  float dx[KI], dy[KI], wx[KI], wy[KI];
  int s[KI];                    // wall of interaction i
  int lo[K + 1], hi[K + 1];     // walls a leg is not tested against (its own ends)
  float F;                      // product of interaction factors
};

// E / (1 + E) = 1 - s, accurate for small E and exactly 1 for huge or infinite E.
__device__ __forceinline__ float one_minus_s(float E) { return E < kBig ? E * rcp(1.0f + E) : 1.0f; }

// Wall indices of candidate cd: interaction walls and, per leg, the walls
// the leg is not tested against (its own ends).
template <int K>
__device__ __forceinline__ void path_walls(const Cand& cd, Path<K>& P) {
  const int sv[3] = {cd.s0, cd.s1, cd.s2};
#pragma unroll
  for (int i = 0; i < Path<K>::KI; ++i) P.s[i] = (i < K) ? sv[i] : -1;
#pragma unroll
  for (int l = 0; l <= K; ++l) {
    P.lo[l] = (l >= 1) ? sv[l - 1] : -1;
    P.hi[l] = (l + 1 <= K) ? sv[l] : -1;
  }
}

// Images I_1..I_K of the transmitter (P.Ix[0], P.Iy[0]); false if a wall is
// degenerate.
template <int K>
__device__ __forceinline__ bool path_images(const SceneView& S, Path<K>& P) {
  bool ok = true;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const WallRec w = load_wall(S.walls, P.s[i]);
    const float nx = -w.ey, ny = w.ex;
    ok = ok && (w.inv_ee > 0.0f);
    const float h = ((P.Ix[i] - w.ax) * nx + (P.Iy[i] - w.ay) * ny) * w.inv_ee;
    P.Ix[i + 1] = P.Ix[i] - 2.0f * h * nx;
    P.Iy[i + 1] = P.Iy[i] - 2.0f * h * ny;
  }
  return ok;
}

// Back-trace from the receiver through the images and (if WANT_F) the
// interaction factors.  With WANT_F, returns false as soon as every lane's
// factor is exactly 0 (then P.F = 0 and the remaining fields are not filled).
template <int K, bool WANT_F, int MODE>
__device__ __forceinline__ bool back_trace(const SceneView& S, float rxx, float rxy, bool ok, Path<K>& P) {
  P.Xx[0] = P.Ix[0];
  P.Xy[0] = P.Iy[0];
  P.Xx[K + 1] = rxx;
  P.Xy[K + 1] = rxy;
  float F = ok ? 1.0f : 0.0f;
#pragma unroll
  for (int i = K; i >= 1; --i) {
    const WallRec w = load_wall(S.walls, P.s[i - 1]);
    const float dx = P.Ix[i] - P.Xx[i + 1], dy = P.Iy[i] - P.Xy[i + 1];
    const float wx = w.ax - P.Xx[i + 1], wy = w.ay - P.Xy[i + 1];
    const float den = dx * w.ey - dy * w.ex;
    const bool good = den != 0.0f;
    const float inv = good ? rcp(den) : 0.0f;
    const float t = (wx * dy - wy * dx) * inv;      // along the wall segment
    const float u = (wx * w.ey - wy * w.ex) * inv;  // between X_{i+1} and the image
    P.Xx[i] = fmaf(t, w.ex, w.ax);
    P.Xy[i] = fmaf(t, w.ey, w.ay);
    P.t[i - 1] = t;
    P.u[i - 1] = u;
    P.inv[i - 1] = inv;
    P.dx[i - 1] = dx;
    P.dy[i - 1] = dy;
    P.wx[i - 1] = wx;
    P.wy[i - 1] = wy;
    if (WANT_F) {
      F = good ? F : 0.0f;
      if constexpr (MODE == kSigmoid) {
        // exponents of E = exp(-alpha x) for x = t, 1 - t, u, 1 - u
        const float z1 = -S.a2 * t, z2 = fmaf(S.a2, t, -S.a2);
        const float z3 = -S.a2 * u, z4 = fmaf(S.a2, u, -S.a2);
        const bool zero = (F == 0.0f) | (z1 >= 128.0f) | (z2 >= 128.0f) | (z3 >= 128.0f) | (z4 >= 128.0f);
        if (ballot(!zero) == 0) {
          P.F = 0.0f;
          return false;
        }
        const float E1 = ex2(z1), E2 = ex2(z2), E3 = ex2(z3), E4 = ex2(z4);
        F *= rcp(((1.0f + E1) * (1.0f + E2)) * ((1.0f + E3) * (1.0f + E4)));
      } else {
        // hs(t) hs(1 - t) hs(u) hs(1 - u): exactly 0 beyond 3 / alpha outside [0, 1]
        F *= (med01(fmaf(S.a6, t, 0.5f)) * med01(fmaf(-S.a6, t, S.a6h))) *
             (med01(fmaf(S.a6, u, 0.5f)) * med01(fmaf(-S.a6, u, S.a6h)));
        if (ballot(F != 0.0f) == 0) {
          P.F = 0.0f;
          return false;
        }
      }
    }
  }
  P.F = F;
  return true;
}

// Images, back-trace and (if WANT_F) the interaction factors of candidate cd.
template <int K, bool WANT_F, int MODE>
__device__ __forceinline__ bool setup_path(const SceneView& S, const Cand& cd, float txx, float txy,
                                           float rxx, float rxy, bool live, Path<K>& P) {
  path_walls<K>(cd, P);
  P.Ix[0] = txx;
  P.Iy[0] = txy;
  const bool ok = path_images<K>(S, P);
  return back_trace<K, WANT_F, MODE>(S, rxx, rxy, live && ok, P);
}

struct LegGeom {
  float Dx, Dy, nXD, Xx, Xy;
};

template <int K>
__device__ __forceinline__ void leg_geoms(const Path<K>& P, LegGeom (&L)[K + 1]) {
#pragma unroll
  for (int l = 0; l <= K; ++l) {
    L[l].Dx = P.Xx[l + 1] - P.Xx[l];
    L[l].Dy = P.Xy[l + 1] - P.Xy[l];
    L[l].nXD = -(P.Xx[l] * L[l].Dy - P.Xy[l] * L[l].Dx);
    L[l].Xx = P.Xx[l];
    L[l].Xy = P.Xy[l];
  }
}

// Obstruction test of a leg by wall w, in two stages so a wavefront can stop
// after the first when no lane's tau is inside the band.
__device__ __forceinline__ bool tau_in_band(const LegGeom& L, const WallRec& w, float band_k, float& den,
                                            float& tn, float& kd) {
  den = L.Dx * w.ey - L.Dy * w.ex;
  tn = fmaf(w.ax, L.Dy, fmaf(-w.ay, L.Dx, L.nXD));  // (a - X) x D
  kd = band_k * fabsf(den);
  return fabsf(fmaf(2.0f, tn, -den)) < kd;
}

__device__ __forceinline__ bool ups_in_band(const LegGeom& L, const WallRec& w, float den, float kd,
                                            float& un) {
  un = fmaf(L.Xy, w.ex, fmaf(-L.Xx, w.ey, w.axe));  // (a - X) x e
  return fabsf(fmaf(2.0f, un, -den)) < kd;
}

struct ObsVals {
  float tau, ups, inv, E1, E2, E3, E4, nt, nu, num;
};

// 1 - in(tau) in(ups) = num / (1 + num), num = nt + nu + nt nu, nt = E1 + E2 + E1 E2.
__device__ __forceinline__ ObsVals obstruction_vals(float den, float tn, float un, float a2) {
  ObsVals o;
  o.inv = rcp(den);
  o.tau = tn * o.inv;
  o.ups = un * o.inv;
  o.E1 = ex2(-a2 * o.tau);
  o.E2 = ex2(fmaf(a2, o.tau, -a2));
  o.E3 = ex2(-a2 * o.ups);
  o.E4 = ex2(fmaf(a2, o.ups, -a2));
  o.nt = fmaf(o.E1, o.E2, o.E1 + o.E2);
  o.nu = fmaf(o.E3, o.E4, o.E3 + o.E4);
  o.num = fmaf(o.nt, o.nu, o.nt + o.nu);
  return o;
}

struct ObsGeom {
  float tau, ups, inv;
};

struct ObsHard {
  float tau, ups, inv, h1, h2, h3, h4, it, iu, q;
};

// Hard sigmoid: 1 - in(tau) in(ups) = nt + in(tau) nu with nt = 1 - in(tau) =
// (1 - h1) + h1 (1 - h2), h1 = hs(tau), h2 = hs(1 - tau) (likewise nu): all
// terms are nonnegative, so a nearly transparent factor keeps its precision.
__device__ __forceinline__ ObsHard obstruction_hard(const SceneView& S, float den, float tn, float un) {
  ObsHard o;
  o.inv = rcp(den);
  o.tau = tn * o.inv;
  o.ups = un * o.inv;
  o.h1 = med01(fmaf(S.a6, o.tau, 0.5f));
  o.h2 = med01(fmaf(-S.a6, o.tau, S.a6h));
  o.h3 = med01(fmaf(S.a6, o.ups, 0.5f));
  o.h4 = med01(fmaf(-S.a6, o.ups, S.a6h));
  const float d1 = med01(fmaf(-S.a6, o.tau, 0.5f)), d2 = med01(fmaf(S.a6, o.tau, S.a6m));
  const float d3 = med01(fmaf(-S.a6, o.ups, 0.5f)), d4 = med01(fmaf(S.a6, o.ups, S.a6m));
  const float nt = fmaf(o.h1, d2, d1), nu = fmaf(o.h3, d4, d3);
  o.it = o.h1 * o.h2;
  o.iu = o.h3 * o.h4;
  o.q = fmaf(o.it, nu, nt);
  return o;
}

// d hs(x) hs(1 - x) / dx divided by alpha / 6: h2 where hs(x) is on its ramp,
// minus h1 where hs(1 - x) is (0 on the flat parts; the kinks take 0).
__device__ __forceinline__ float hard_ramp(float h1, float h2) {
  return (((h1 > 0.0f) & (h1 < 1.0f)) ? h2 : 0.0f) - (((h2 > 0.0f) & (h2 < 1.0f)) ? h1 : 0.0f);
}

// Wave-uniform oriented box around the band-extended legs
// [X_l - c D, X_{l+1} + c D] of the live lanes: axis u along one live lane's
// leg, v = perp(u), extents from the lanes' projections (grown by a relative
// 1e-5 against rounding).  A wall whose band-extended segment is separated
// from it (separating axes u, v and the wall normal) cannot give an
// unsaturated test on that leg in any lane.
struct LegBox {
  float ux, uy, umid, uh, vmid, vh;  // wave-uniform (scalar registers)
  bool empty;
};

template <int K>
__device__ __forceinline__ void leg_boxes(const Path<K>& P, const LegGeom (&L)[K + 1], bool lane_live,
                                          float c, LegBox (&B)[K + 1]) {
  const float I = __builtin_inff();
  const uint64_t live = ballot(lane_live);
  const int src = live ? __builtin_ctzll(live) : 0;
#pragma unroll
  for (int l = 0; l <= K; ++l) {
    B[l].empty = live == 0;
    const float q0x = fmaf(-c, L[l].Dx, L[l].Xx), q0y = fmaf(-c, L[l].Dy, L[l].Xy);
    const float q1x = fmaf(c, L[l].Dx, P.Xx[l + 1]), q1y = fmaf(c, L[l].Dy, P.Xy[l + 1]);
    const float dx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(L[l].Dx), src));
    const float dy = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(L[l].Dy), src));
    const float n2 = dx * dx + dy * dy;
    const float rn = n2 > 0.0f ? rsqrtf(n2) : 0.0f;
    const float ux = uniformf(n2 > 0.0f ? dx * rn : 1.0f), uy = uniformf(n2 > 0.0f ? dy * rn : 0.0f);
    const float a0 = ux * q0x + uy * q0y, a1 = ux * q1x + uy * q1y;
    const float b0 = ux * q0y - uy * q0x, b1 = ux * q1y - uy * q1x;
    // maxima of -umin, umax, -vmin, vmax (dead lanes contribute -inf)
    float a = lane_live ? -fminf(a0, a1) : -I, b = lane_live ? fmaxf(a0, a1) : -I;
    float cc = lane_live ? -fminf(b0, b1) : -I, d = lane_live ? fmaxf(b0, b1) : -I;
    wave_max4(a, b, cc, d);
    if (B[l].empty) a = b = cc = d = 0.0f;
    const float eu = 1e-5f * (1.0f + fmaxf(fabsf(a), fabsf(b)));
    const float ev = 1e-5f * (1.0f + fmaxf(fabsf(cc), fabsf(d)));
    B[l].ux = ux;
    B[l].uy = uy;
    B[l].umid = uniformf(0.5f * (b - a));
    B[l].uh = uniformf(0.5f * (b + a) + eu);
    B[l].vmid = uniformf(0.5f * (d - cc));
    B[l].vh = uniformf(0.5f * (d + cc) + ev);
  }
}

// Separating-axis test of a wall's culling box q against a leg box (axis
// (ux, uy), centre (umid, vmid) and half extents (uh, vh) in that frame).
__device__ __forceinline__ bool sat_separated(const WallBox& q, float ux, float uy, float umid, float uh,
                                              float vmid, float vh) {
  const float uc = fmaf(ux, q.cx, uy * q.cy), uw = fabsf(fmaf(ux, q.hx, uy * q.hy));
  const float vc = fmaf(ux, q.cy, -uy * q.cx), vw = fabsf(fmaf(ux, q.hy, -uy * q.hx));
  const bool sep_u = fabsf(uc - umid) > uw + uh;
  const bool sep_v = fabsf(vc - vmid) > vw + vh;
  const float nu = fmaf(q.nx, ux, q.ny * uy), nv = fmaf(q.ny, ux, -q.nx * uy);
  const bool sep_n = fabsf(fmaf(umid, nu, fmaf(vmid, nv, -q.nd))) > fmaf(fabsf(nu), uh, fmaf(fabsf(nv), vh, q.en));
  return sep_u | sep_v | sep_n;
}

// Calls fn(wall, masks, bit) for every wall that is not separated from some
// leg box (every wall when S.cull is 0; walls in increasing order) until fn
// returns false; masks[l] bit
// `bit` tells whether leg l needs the test (its own end walls are excluded
// here).  Lane j of the wavefront checks wall b + j of each 64-wall batch.
// Separating axes: u and v (the wall's projection, centre +- half extent,
// against the box's) and the wall normal n (the box's range of n . x - n . a
// from its centre and half extents, against a relative margin).
template <int K, class Fn>
__device__ __forceinline__ void visit_walls(const SceneView& S, const Path<K>& P, const LegBox (&B)[K + 1],
                                            Fn&& fn) {
  const int lane = threadIdx.x & (kWave - 1);
  for (int b = 0; b < S.n_walls; b += kWave) {
    uint64_t m[K + 1];
    uint64_t uni = 0;
    const int r = S.n_walls - b;  // walls left (wave-uniform)
    if (K > 0 && (K + 1) * r <= kWave) {
      // short last batch: one pass over (leg, wall) pairs, lane = l r + i
      int ls = 0;
#pragma unroll
      for (int l = 1; l <= K; ++l) ls += lane >= l * r;
      const int wj = b + lane - ls * r;
      const bool valid = lane < (K + 1) * r;
      WallBox q;
      if (valid) {
        q = S.boxes[wj];
      } else {
        q.cx = q.cy = q.hx = q.hy = q.nx = q.ny = q.nd = q.en = 0.0f;
      }
      float ux = B[0].ux, uy = B[0].uy, umid = B[0].umid, uh = B[0].uh, vmid = B[0].vmid, vh = B[0].vh;
      bool empty = B[0].empty;
      int lo = P.lo[0], hi = P.hi[0];
#pragma unroll
      for (int l = 1; l <= K; ++l) {
        const bool t = ls == l;
        ux = t ? B[l].ux : ux;
        uy = t ? B[l].uy : uy;
        umid = t ? B[l].umid : umid;
        uh = t ? B[l].uh : uh;
        vmid = t ? B[l].vmid : vmid;
        vh = t ? B[l].vh : vh;
        empty = t ? B[l].empty : empty;
        lo = t ? P.lo[l] : lo;
        hi = t ? P.hi[l] : hi;
      }
      const bool ov = valid & (!S.cull | (!empty & !sat_separated(q, ux, uy, umid, uh, vmid, vh))) & (wj != lo) &
                      (wj != hi);
      const uint64_t M = ballot(ov);
      const uint64_t low = (1ull << r) - 1ull;
#pragma unroll
      for (int l = 0; l <= K; ++l) {
        m[l] = (M >> (l * r)) & low;
        uni |= m[l];
      }
    } else {
      const int wj = b + lane;
      const bool valid = wj < S.n_walls;
      WallBox q;
      if (valid) {
        q = S.boxes[wj];
      } else {
        q.cx = q.cy = q.hx = q.hy = q.nx = q.ny = q.nd = q.en = 0.0f;
      }
#pragma unroll
      for (int l = 0; l <= K; ++l) {
        const LegBox& L = B[l];
        const bool ov = valid & (!S.cull | (!L.empty & !sat_separated(q, L.ux, L.uy, L.umid, L.uh, L.vmid, L.vh))) &
                        (wj != P.lo[l]) & (wj != P.hi[l]);
        m[l] = ballot(ov);
        uni |= m[l];
      }
    }
    while (uni) {
      const int j = __builtin_ctzll(uni);
      uni &= uni - 1;
      if (!fn(b + j, m, j)) return;
    }
  }
}

// V times every obstruction factor of the path.
// With `boxes` (leg boxes stored by the candidate screen, fields of leg l at
// boxes[(6 l + f) * 64 + j]) the culling boxes are read from there; without,
// they are formed from the live lanes' legs.
template <int K, int MODE>
__device__ __forceinline__ float obstruct_all(const SceneView& S, const Path<K>& P, float V,
                                              const float* boxes = nullptr, int j = 0, float vcut = 0.0f) {
  LegGeom L[K + 1];
  leg_geoms<K>(P, L);
  LegBox B[K + 1];
  if (boxes) {
#pragma unroll
    for (int l = 0; l <= K; ++l) {
      const float* b = boxes + 6 * l * kWave + j;  // same address in every lane: to scalar registers
      B[l].ux = uniformf(b[0]);
      B[l].uy = uniformf(b[kWave]);
      B[l].umid = uniformf(b[2 * kWave]);
      B[l].uh = uniformf(b[3 * kWave]);
      B[l].vmid = uniformf(b[4 * kWave]);
      B[l].vh = uniformf(b[5 * kWave]);
      B[l].empty = false;
    }
  } else {
    leg_boxes<K>(P, L, P.F != 0.0f, S.cull_c, B);
  }
  visit_walls<K>(S, P, B, [&](int jw, const uint64_t* m, int j) {
    const WallRec w = load_wall(S.walls, jw);
    bool upd = false;
#pragma unroll
    for (int l = 0; l <= K; ++l) {
      if (((m[l] >> j) & 1ull) == 0) continue;
      float den, tn, kd, un;
      const bool it = tau_in_band(L[l], w, S.band_k, den, tn, kd);
      if (ballot(it) == 0) continue;
      if (it && ups_in_band(L[l], w, den, kd, un)) {
        if constexpr (MODE == kSigmoid) {
          const ObsVals o = obstruction_vals(den, tn, un, S.a2);
          V *= o.num * rcp(1.0f + o.num);
        } else {
          V *= obstruction_hard(S, den, tn, un).q;
        }
        upd = true;
      }
    }
    // a lane whose product fell to its cut contributes nothing; once every
    // lane's product is 0 no further factor can change it
    if constexpr (uses_cut<MODE>()) V = V > vcut ? V : 0.0f;
    return ballot(upd) == 0 || ballot(V != 0.0f) != 0;
  });
  return V;
}

// Contribution c = V / max(|r - I_K|^2, d_min^2) of candidate cd at this lane.
template <int K, int MODE>
__device__ __forceinline__ float path_power(const SceneView& S, const Cand& cd, float txx, float txy,
                                            float rxx, float rxy, bool live) {
  Path<K> P;
  if (!setup_path<K, true, MODE>(S, cd, txx, txy, rxx, rxy, live, P)) return 0.0f;
  if (ballot(P.F != 0.0f) == 0) return 0.0f;
  const float V = obstruct_all<K, MODE>(S, P, P.F);
  const float ex = rxx - P.Ix[K], ey = rxy - P.Iy[K];
  const float d2 = fmaf(ex, ex, ey * ey);
  return V / fmaxf(d2, S.dmin2);
}

// Same as path_power with the images I_1..I_K given (wave-uniform; the
// candidate's walls are known to be nondegenerate).
template <int K, int MODE>
__device__ __forceinline__ float path_power_img(const SceneView& S, const Cand& cd, const float* Ix,
                                                const float* Iy, float txx, float txy, float rxx, float rxy,
                                                bool live, const float* boxes, int j, float scut) {
  Path<K> P;
  path_walls<K>(cd, P);
  P.Ix[0] = txx;
  P.Iy[0] = txy;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    P.Ix[i + 1] = Ix[i];
    P.Iy[i + 1] = Iy[i];
  }
  if (!back_trace<K, true, MODE>(S, rxx, rxy, live, P)) return 0.0f;
  const float ex = rxx - P.Ix[K], ey = rxy - P.Iy[K];
  if constexpr (!uses_cut<MODE>()) {
    if (ballot(P.F != 0.0f) == 0) return 0.0f;
    const float V = obstruct_all<K, MODE>(S, P, P.F, boxes, j);
    return V / fmaxf(fmaf(ex, ex, ey * ey), S.dmin2);
  } else {
    const float dd = fmaxf(fmaf(ex, ex, ey * ey), S.dmin2);
    const float vcut = scut * dd;  // the contribution V / dd is below the cut once V <= vcut
    P.F = P.F > vcut ? P.F : 0.0f;
    if (ballot(P.F != 0.0f) == 0) return 0.0f;
    const float V = obstruct_all<K, MODE>(S, P, P.F, boxes, j, vcut);
    return V / dd;
  }
}

// Per-wave accumulator layout: [0,1] = d/dtx, [2 + 4j + c] = d/d walls[j][c].
// Lanes 0..3 add the wave totals of (dax, dbx, day, dby) to their entries.
__device__ __forceinline__ void acc_wall(float* acc, int j, float dax, float day, float dbx, float dby,
                                         int lane) {
  const float s = wave_sum4(dax, day, dbx, dby);
  if (lane < 4) acc[2 + 4 * j + ((lane & 1) << 1) + ((lane >> 1) & 1)] += s;
}

struct LaneGrad {
  float tx_x, tx_y, rx_x, rx_y;
};

// Reverse sweep of one path given Wl = g(r) * c (= dL/dlog V at this lane).
// Adds wall and transmitter gradients to the wave's accumulator and per-lane
// transmitter / receiver gradients to G.
// Leg boxes recorded by the forward (fields of leg l at gbox[6 l + f], the
// same address in every lane).  Vector loads, not the scalar data cache: in
// the batched kernel the same wavefront wrote these entries earlier in the
// launch, and only vector memory keeps that order.
template <int K>
__device__ __forceinline__ void load_leg_boxes(const float* gbox, LegBox (&B)[K + 1]) {
#pragma unroll
  for (int l = 0; l <= K; ++l) {
    B[l].ux = uniformf(gbox[6 * l]);
    B[l].uy = uniformf(gbox[6 * l + 1]);
    B[l].umid = uniformf(gbox[6 * l + 2]);
    B[l].uh = uniformf(gbox[6 * l + 3]);
    B[l].vmid = uniformf(gbox[6 * l + 4]);
    B[l].vh = uniformf(gbox[6 * l + 5]);
    B[l].empty = false;
  }
}

template <int K, int MODE>
__device__ __forceinline__ void path_adjoint_core(const SceneView& S, const Path<K>& P, float Wl,
                                                  float rxx, float rxy, float* acc, int lane,
                                                  LaneGrad& G, const float* gbox = nullptr) {
  const float ex = rxx - P.Ix[K], ey = rxy - P.Iy[K];
  const float d2 = fmaf(ex, ex, ey * ey);

  // -- obstruction tests, reverse: dlog q / dtau, dlog q / dups -> geometry
  LegGeom L[K + 1];
  leg_geoms<K>(P, L);
  float Sgwx[K + 1], Sgwy[K + 1], SgDx[K + 1], SgDy[K + 1];
#pragma unroll
  for (int l = 0; l <= K; ++l) Sgwx[l] = Sgwy[l] = SgDx[l] = SgDy[l] = 0.0f;
  const bool act = Wl != 0.0f;
  const float nalpha = -S.alpha;
  LegBox B[K + 1];
  if (gbox) load_leg_boxes<K>(gbox, B);
  else leg_boxes<K>(P, L, act, S.cull_c, B);
  visit_walls<K>(S, P, B, [&](int jw, const uint64_t* m, int j) {
    const WallRec w = load_wall(S.walls, jw);
    float gax = 0.0f, gay = 0.0f, gex = 0.0f, gey = 0.0f;
    bool any = false;
#pragma unroll
    for (int l = 0; l <= K; ++l) {
      if (((m[l] >> j) & 1ull) == 0) continue;
      float den, tn, kd, un;
      const bool it = tau_in_band(L[l], w, S.band_k, den, tn, kd) && act;
      if (ballot(it) == 0) continue;
      if (it && ups_in_band(L[l], w, den, kd, un)) {
        // gt, gu = Wl dlog q / dtau, Wl dlog q / dups
        float gt, gu;
        ObsGeom o;
        if constexpr (MODE == kSigmoid) {
          const ObsVals v = obstruction_vals(den, tn, un, S.a2);
          const float Ab = 1.0f + v.nt, Bb = 1.0f + v.nu;
          const float coef = nalpha * Wl * rcp(v.num * Ab * Bb);
          gt = coef * (v.E1 - v.E2) * Bb;
          gu = coef * (v.E3 - v.E4) * Ab;
          o = ObsGeom{v.tau, v.ups, v.inv};
        } else {
          const ObsHard v = obstruction_hard(S, den, tn, un);
          const float coef = v.q > 0.0f ? -S.a6 * Wl * rcp(v.q) : 0.0f;
          gt = coef * v.iu * hard_ramp(v.h1, v.h2);
          gu = coef * v.it * hard_ramp(v.h3, v.h4);
          o = ObsGeom{v.tau, v.ups, v.inv};
        }
        const float w0x = w.ax - L[l].Xx, w0y = w.ay - L[l].Xy;
        const float s = fmaf(gt, o.tau, gu * o.ups);
        const float gw0x = o.inv * fmaf(gt, L[l].Dy, gu * w.ey);
        const float gw0y = -o.inv * fmaf(gt, L[l].Dx, gu * w.ex);
        const float gDx = -o.inv * fmaf(gt, w0y, s * w.ey);
        const float gDy = o.inv * fmaf(gt, w0x, s * w.ex);
        const float gEx = o.inv * fmaf(-gu, w0y, s * L[l].Dy);
        const float gEy = o.inv * fmaf(gu, w0x, -s * L[l].Dx);
        Sgwx[l] += gw0x;
        Sgwy[l] += gw0y;
        SgDx[l] += gDx;
        SgDy[l] += gDy;
        gax += gw0x;
        gay += gw0y;
        gex += gEx;
        gey += gEy;
        any = true;
      }
    }
    if (ballot(any) != 0) acc_wall(acc, jw, gax - gex, gay - gey, gex, gey, lane);
    return true;
  });

  // -- gradients of the points X_0..X_{K+1} from the legs
  float gXx[K + 2], gXy[K + 2];
#pragma unroll
  for (int i = 0; i < K + 2; ++i) gXx[i] = gXy[i] = 0.0f;
#pragma unroll
  for (int l = 0; l <= K; ++l) {
    gXx[l] -= Sgwx[l] + SgDx[l];
    gXy[l] -= Sgwy[l] + SgDy[l];
    gXx[l + 1] += SgDx[l];
    gXy[l + 1] += SgDy[l];
  }
  // -- image distance |r - I_K|^2 (zero gradient under the d_min floor)
  float gIx[K + 1], gIy[K + 1];
#pragma unroll
  for (int i = 0; i <= K; ++i) gIx[i] = gIy[i] = 0.0f;
  if (d2 > S.dmin2) {
    const float f = 2.0f * Wl / d2;
    gIx[K] += f * ex;
    gIy[K] += f * ey;
    gXx[K + 1] -= f * ex;
    gXy[K + 1] -= f * ey;
  }
  // -- interactions i = 1..K: smoothed factors and back-trace, in order
#pragma unroll
  for (int i = 1; i <= K; ++i) {
    const WallRec w = load_wall(S.walls, P.s[i - 1]);
    const float t = P.t[i - 1], u = P.u[i - 1], inv = P.inv[i - 1];
    // gti, gu = Wl dlog f_i / dt, Wl dlog f_i / du
    float gti, gu;
    if constexpr (MODE == kSigmoid) {
      const float E1 = ex2(-S.a2 * t), E2 = ex2(fmaf(S.a2, t, -S.a2));
      const float E3 = ex2(-S.a2 * u), E4 = ex2(fmaf(S.a2, u, -S.a2));
      const float aw = S.alpha * Wl;
      gti = aw * (one_minus_s(E1) - one_minus_s(E2));
      gu = aw * (one_minus_s(E3) - one_minus_s(E4));
    } else {
      // d log hs(x) / dx = (alpha / 6) / hs(x) on the ramp, 0 on the flat parts
      const float h1 = med01(fmaf(S.a6, t, 0.5f)), h2 = med01(fmaf(-S.a6, t, S.a6h));
      const float h3 = med01(fmaf(S.a6, u, 0.5f)), h4 = med01(fmaf(-S.a6, u, S.a6h));
      const float aw = S.a6 * Wl;
      gti = aw * ((((h1 > 0.0f) & (h1 < 1.0f)) ? rcp(h1) : 0.0f) - (((h2 > 0.0f) & (h2 < 1.0f)) ? rcp(h2) : 0.0f));
      gu = aw * ((((h3 > 0.0f) & (h3 < 1.0f)) ? rcp(h3) : 0.0f) - (((h4 > 0.0f) & (h4 < 1.0f)) ? rcp(h4) : 0.0f));
    }
    // X_i = a + t e
    const float gt = gti + gXx[i] * w.ex + gXy[i] * w.ey;
    float gax = gXx[i], gay = gXy[i];
    float gex = t * gXx[i], gey = t * gXy[i];
    // t = (w x d)/den, u = (w x e)/den with w = a - X_{i+1}, d = I_i - X_{i+1}
    const float dx = P.dx[i - 1], dy = P.dy[i - 1], wx = P.wx[i - 1], wy = P.wy[i - 1];
    const float s = fmaf(gt, t, gu * u);
    const float gwx = inv * fmaf(gt, dy, gu * w.ey);
    const float gwy = -inv * fmaf(gt, dx, gu * w.ex);
    const float gdx = -inv * fmaf(gt, wy, s * w.ey);
    const float gdy = inv * fmaf(gt, wx, s * w.ex);
    gex += inv * fmaf(-gu, wy, s * dy);
    gey += inv * fmaf(gu, wx, -s * dx);
    gIx[i] += gdx;
    gIy[i] += gdy;
    gXx[i + 1] -= gdx + gwx;
    gXy[i + 1] -= gdy + gwy;
    gax += gwx;
    gay += gwy;
    acc_wall(acc, P.s[i - 1], gax - gex, gay - gey, gex, gey, lane);
  }
  // -- per-lane transmitter and receiver gradients
  G.tx_x += gXx[0];
  G.tx_y += gXy[0];
  G.rx_x += gXx[K + 1];
  G.rx_y += gXy[K + 1];
  if (K == 0) {
    // I_0 is the transmitter itself
    G.tx_x += gIx[0];
    G.tx_y += gIy[0];
  } else {
    // -- images: reduce over lanes, then mirror adjoint on uniform values
    float GIx[K + 1], GIy[K + 1];
#pragma unroll
    for (int i = 1; i <= K; ++i) {
      GIx[i] = wave_sum(gIx[i]);
      GIy[i] = wave_sum(gIy[i]);
    }
    GIx[0] = 0.0f;
    GIy[0] = 0.0f;
#pragma unroll
    for (int i = K; i >= 1; --i) {
      const WallRec w = load_wall(S.walls, P.s[i - 1]);
      const float nx = -w.ey, ny = w.ex;
      const float inn = w.inv_ee;
      const float px = P.Ix[i - 1] - w.ax, py = P.Iy[i - 1] - w.ay;
      const float h = (px * nx + py * ny) * inn;
      const float Gx = GIx[i], Gy = GIy[i];
      const float Gn = Gx * nx + Gy * ny;
      const float kk = 2.0f * Gn * inn;
      GIx[i - 1] += Gx - kk * nx;
      GIy[i - 1] += Gy - kk * ny;
      const float gax = kk * nx, gay = kk * ny;
      const float gnx = -2.0f * (Gn * (px - 2.0f * h * nx) * inn + h * Gx);
      const float gny = -2.0f * (Gn * (py - 2.0f * h * ny) * inn + h * Gy);
      const float gex = gny, gey = -gnx;
      if (lane == 0) {
        float* p = acc + 2 + 4 * P.s[i - 1];
        p[0] += gax - gex;
        p[1] += gay - gey;
        p[2] += gex;
        p[3] += gey;
      }
    }
    if (lane == 0) {
      acc[0] += GIx[0];
      acc[1] += GIy[0];
    }
  }
}

// Adjoint of one candidate, re-evaluating its forward value first.
template <int K, int MODE>
__device__ __forceinline__ float path_adjoint(const SceneView& S, const Cand& cd, float txx, float txy,
                                              float rxx, float rxy, bool live, float g, float* acc,
                                              int lane, LaneGrad& G, float scut) {
  Path<K> P;
  if (!setup_path<K, true, MODE>(S, cd, txx, txy, rxx, rxy, live, P)) return 0.0f;
  const float ex = rxx - P.Ix[K], ey = rxy - P.Iy[K];
  const float dd = fmaxf(fmaf(ex, ex, ey * ey), S.dmin2);
  const float vcut = scut * dd;
  if constexpr (uses_cut<MODE>()) P.F = P.F > vcut ? P.F : 0.0f;
  // lanes with g = 0 need neither their contribution nor their gradient
  if (ballot(P.F != 0.0f && g != 0.0f) == 0) return 0.0f;
  const float V = obstruct_all<K, MODE>(S, P, P.F, nullptr, 0, vcut);
  const float c = V / dd;
  const float Wl = g * c;
  if (ballot(Wl != 0.0f) != 0) path_adjoint_core<K, MODE>(S, P, Wl, rxx, rxy, acc, lane, G);
  return c;
}

// Adjoint of one candidate whose contribution c is already known.
template <int K, int MODE>
__device__ __forceinline__ void path_adjoint_known(const SceneView& S, const Cand& cd, float txx,
                                                   float txy, float rxx, float rxy, bool live, float Wl,
                                                   float* acc, int lane, LaneGrad& G, const float* gbox) {
  Path<K> P;
  setup_path<K, false, MODE>(S, cd, txx, txy, rxx, rxy, live, P);
  path_adjoint_core<K, MODE>(S, P, Wl, rxx, rxy, acc, lane, G, gbox);
}

template <int MODE>
__device__ __forceinline__ float candidate_power(const SceneView& S, const Cand& cd, float txx, float txy,
                                                 float rxx, float rxy, bool live) {
  switch (cd.k) {
    case 0: return path_power<0, MODE>(S, cd, txx, txy, rxx, rxy, live);
    case 1: return path_power<1, MODE>(S, cd, txx, txy, rxx, rxy, live);
    case 2: return path_power<2, MODE>(S, cd, txx, txy, rxx, rxy, live);
    default: return path_power<3, MODE>(S, cd, txx, txy, rxx, rxy, live);
  }
}

// MAXK: the highest order the caller's candidates can have (the code of
// higher orders is left out, which keeps register pressure at that order's).
template <int MODE, int MAXK = 3>
__device__ __forceinline__ float candidate_power_img(const SceneView& S, const Cand& cd, const float* Ix,
                                                     const float* Iy, float txx, float txy, float rxx,
                                                     float rxy, bool live, const float* boxes, int j,
                                                     float scut) {
  static_assert(MAXK >= 1 && MAXK <= 3, "orders 1..3");
  switch (cd.k) {
    case 0: return path_power_img<0, MODE>(S, cd, Ix, Iy, txx, txy, rxx, rxy, live, boxes, j, scut);
    case 1: return path_power_img<1, MODE>(S, cd, Ix, Iy, txx, txy, rxx, rxy, live, boxes, j, scut);
    case 2:
      if constexpr (MAXK >= 2) return path_power_img<2, MODE>(S, cd, Ix, Iy, txx, txy, rxx, rxy, live, boxes, j, scut);
      else return 0.0f;
    default:
      if constexpr (MAXK >= 3) return path_power_img<3, MODE>(S, cd, Ix, Iy, txx, txy, rxx, rxy, live, boxes, j, scut);
      else return 0.0f;
  }
}

// MAXK as in candidate_power_img: the highest order the caller's candidates
// can have.
template <int MODE, int MAXK = 3>
__device__ __forceinline__ float candidate_adjoint(const SceneView& S, const Cand& cd, float txx, float txy,
                                                   float rxx, float rxy, bool live, float g, float* acc,
                                                   int lane, LaneGrad& G, float scut) {
  static_assert(MAXK >= 2 && MAXK <= 3, "orders 2..3");
  switch (cd.k) {
    case 0: return path_adjoint<0, MODE>(S, cd, txx, txy, rxx, rxy, live, g, acc, lane, G, scut);
    case 1: return path_adjoint<1, MODE>(S, cd, txx, txy, rxx, rxy, live, g, acc, lane, G, scut);
    case 2: return path_adjoint<2, MODE>(S, cd, txx, txy, rxx, rxy, live, g, acc, lane, G, scut);
    default:
      if constexpr (MAXK >= 3) return path_adjoint<3, MODE>(S, cd, txx, txy, rxx, rxy, live, g, acc, lane, G, scut);
      else return 0.0f;
  }
}

template <int MODE, int MAXK = 3>
__device__ __forceinline__ void candidate_adjoint_known(const SceneView& S, const Cand& cd, float txx,
                                                        float txy, float rxx, float rxy, bool live,
                                                        float Wl, float* acc, int lane, LaneGrad& G,
                                                        const float* gbox = nullptr) {
  static_assert(MAXK >= 2 && MAXK <= 3, "orders 2..3");
  switch (cd.k) {
    case 0: path_adjoint_known<0, MODE>(S, cd, txx, txy, rxx, rxy, live, Wl, acc, lane, G, gbox); break;
    case 1: path_adjoint_known<1, MODE>(S, cd, txx, txy, rxx, rxy, live, Wl, acc, lane, G, gbox); break;
    case 2: path_adjoint_known<2, MODE>(S, cd, txx, txy, rxx, rxy, live, Wl, acc, lane, G, gbox); break;
    default:
      if constexpr (MAXK >= 3) path_adjoint_known<3, MODE>(S, cd, txx, txy, rxx, rxy, live, Wl, acc, lane, G, gbox);
      break;
  }
}

}  // namespace drt
