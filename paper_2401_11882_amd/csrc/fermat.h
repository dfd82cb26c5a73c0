// Fermat path tracing (FPT): the second path finder of Sec. V-B, per
// (receiver, candidate) lane, for candidates of order 1 and 2.
//
// The interaction points X_i = a_i + t_i e_i on the (infinite) lines of the
// candidate's walls are placed where the path length
//   l(t) = |X_1 - tx| + ... + |r - X_k|
// is smallest (Fermat's principle).  l is convex in t (a sum of norms of
// affine maps); each lane runs damped Newton on it from t = 1/2 with a
// halving line search.  The length has a kink where a leg shrinks to zero (a
// path through the corner of two adjacent walls), where Newton stalls, so the
// leg lengths are first smoothed to sqrt(|Q|^2 + delta^2) and delta is lowered
// in stages to 0, each stage starting from the last (continuation).  A wave
// leaves a stage when no live lane's step exceeds FP32 resolution.
//
// The finder's own discontinuity is its convergence check: the MPT loss, the
// squared residual of the law of reflection summed over the interactions,
//   L = sum_i |d_out - d_in + 2 (d_in . n) n|^2
// (d_in, d_out unit directions of the legs into and out of X_i, n the unit
// normal of the wall), is 0 on a valid path and 4 (d . n)^2 on a straight
// pass through a wall line; "L < eps" is smoothed as s(1 - L / eps) with the
// scene's sharpness (sigmoid or hard sigmoid).  The validity is then
//   V = prod_i in(t_i) * s(1 - L / eps) * obstruction factors of the legs
// (Sec. V-A, as for the image method), and the contribution V / max(l^2, d_min^2).
#pragma once
#include "path.h"

namespace drt {

template <int K>
struct FermatLines {
  float ax[K], ay[K], ex[K], ey[K], ee[K];
};

// Path length through the points on the lines at t, legs smoothed by d2.
template <int K>
__device__ __forceinline__ float fermat_length(const FermatLines<K>& W, const float (&t)[K], float txx, float txy,
                                               float rxx, float rxy, float d2) {
  float px = txx, py = txy, L = 0.0f;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const float x = fmaf(t[i], W.ex[i], W.ax[i]), y = fmaf(t[i], W.ey[i], W.ay[i]);
    const float dx = x - px, dy = y - py;
    L += sqrtf(fmaf(dx, dx, fmaf(dy, dy, d2)));
    px = x;
    py = y;
  }
  const float dx = rxx - px, dy = rxy - py;
  return L + sqrtf(fmaf(dx, dx, fmaf(dy, dy, d2)));
}

// Newton's iterations on the (smoothed) length; t in/out.
template <int K>
__device__ __forceinline__ void fermat_solve(const FermatLines<K>& W, float (&t)[K], float txx, float txy,
                                             float rxx, float rxy, bool lane_active, int max_iter) {
  constexpr int kStages = 4;
  const float stages[kStages] = {1e-2f, 1e-4f, 1e-6f, 0.0f};
#pragma unroll 1
  for (int st = 0; st < kStages; ++st) {
    const float d2 = stages[st];
#pragma unroll 1
    for (int it = 0; it < max_iter; ++it) {
      float xs[K + 2], ys[K + 2];
      xs[0] = txx;
      ys[0] = txy;
#pragma unroll
      for (int i = 0; i < K; ++i) {
        xs[i + 1] = fmaf(t[i], W.ex[i], W.ax[i]);
        ys[i + 1] = fmaf(t[i], W.ey[i], W.ay[i]);
      }
      xs[K + 1] = rxx;
      ys[K + 1] = rxy;
      float vx[K + 1], vy[K + 1], n[K + 1];
#pragma unroll
      for (int l = 0; l <= K; ++l) {
        const float qx = xs[l + 1] - xs[l], qy = ys[l + 1] - ys[l];
        n[l] = fmaxf(sqrtf(fmaf(qx, qx, fmaf(qy, qy, d2))), 1e-30f);
        const float in = 1.0f / n[l];
        vx[l] = qx * in;
        vy[l] = qy * in;
      }
      // gradient e_i . (v_{i-1} - v_i) and Hessian sum_l J^T (I - v v^T) J / n_l
      float g[K], s[K];
      float h00, h01 = 0.0f, h11 = 0.0f;
      {
        const float ve0 = vx[0] * W.ex[0] + vy[0] * W.ey[0], ve1 = vx[1] * W.ex[0] + vy[1] * W.ey[0];
        g[0] = ve0 - ve1;
        h00 = (W.ee[0] - ve0 * ve0) / n[0] + (W.ee[0] - ve1 * ve1) / n[1];
      }
      if constexpr (K == 2) {
        const float ve1 = vx[1] * W.ex[1] + vy[1] * W.ey[1], ve2 = vx[2] * W.ex[1] + vy[2] * W.ey[1];
        g[1] = ve1 - ve2;
        h11 = (W.ee[1] - ve1 * ve1) / n[1] + (W.ee[1] - ve2 * ve2) / n[2];
        const float v1e0 = vx[1] * W.ex[0] + vy[1] * W.ey[0];
        h01 = (-(W.ex[0] * W.ex[1] + W.ey[0] * W.ey[1]) + v1e0 * ve1) / n[1];
        const float det = h00 * h11 - h01 * h01;
        if (det > 1e-30f * (h00 * h11) && det > 0.0f) {
          const float id = 1.0f / det;
          s[0] = (h11 * g[0] - h01 * g[1]) * id;
          s[1] = (h00 * g[1] - h01 * g[0]) * id;
        } else {
          const float tr = 1.0f / fmaxf(h00 + h11, 1e-30f);
          s[0] = g[0] * tr;
          s[1] = g[1] * tr;
        }
      } else {
        s[0] = h00 > 0.0f ? g[0] / h00 : 0.0f;
      }
      // halving line search on the same (smoothed) length; a step that does not
      // raise it beyond FP32 rounding is taken
      float L0 = 0.0f;
#pragma unroll
      for (int l = 0; l <= K; ++l) L0 += n[l];
      float lam = 1.0f;
      bool found = false;
#pragma unroll 1
      for (int m = 0; m < 16; ++m) {
        float tc[K];
#pragma unroll
        for (int i = 0; i < K; ++i) tc[i] = fmaf(-lam, s[i], t[i]);
        if (fermat_length<K>(W, tc, txx, txy, rxx, rxy, d2) <= L0 * (1.0f + 4e-7f)) {
          found = true;
          break;
        }
        lam *= 0.5f;
      }
      bool moved = false;
      if (found) {
#pragma unroll
        for (int i = 0; i < K; ++i) {
          const float d = lam * s[i];
          moved |= fabsf(d) > 2e-7f * (1.0f + fabsf(t[i]));
          t[i] -= d;
        }
      }
      if (ballot(lane_active && moved) == 0) break;
    }
  }
}

// Contribution of candidate cd at this lane with Fermat path tracing.
template <int K, int MODE>
__device__ __forceinline__ float fermat_power(const SceneView& S, const Cand& cd, float txx, float txy, float rxx,
                                              float rxy, bool live, int max_iter, float inv_eps) {
  Path<K> P;
  path_walls<K>(cd, P);
  FermatLines<K> W;
  bool ok = live;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const WallRec w = load_wall(S.walls, P.s[i]);
    W.ax[i] = w.ax;
    W.ay[i] = w.ay;
    W.ex[i] = w.ex;
    W.ey[i] = w.ey;
    W.ee[i] = fmaf(w.ex, w.ex, w.ey * w.ey);
    ok = ok && (w.inv_ee > 0.0f);
  }
  if (ballot(ok) == 0) return 0.0f;
  float t[K];
#pragma unroll
  for (int i = 0; i < K; ++i) t[i] = 0.5f;
  fermat_solve<K>(W, t, txx, txy, rxx, rxy, ok, max_iter);

  // points, legs and the MPT loss at the solution (unsmoothed lengths)
  P.Xx[0] = txx;
  P.Xy[0] = txy;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    P.Xx[i + 1] = fmaf(t[i], W.ex[i], W.ax[i]);
    P.Xy[i + 1] = fmaf(t[i], W.ey[i], W.ay[i]);
  }
  P.Xx[K + 1] = rxx;
  P.Xy[K + 1] = rxy;
  float ux[K + 1], uy[K + 1], len = 0.0f;
#pragma unroll
  for (int l = 0; l <= K; ++l) {
    const float qx = P.Xx[l + 1] - P.Xx[l], qy = P.Xy[l + 1] - P.Xy[l];
    const float nl = sqrtf(fmaf(qx, qx, qy * qy));
    ok = ok && (nl > 0.0f);
    const float in = nl > 0.0f ? 1.0f / nl : 0.0f;
    ux[l] = qx * in;
    uy[l] = qy * in;
    len += nl;
  }
  float Lm = 0.0f;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const float rn = W.ee[i] > 0.0f ? rsqrtf(W.ee[i]) : 0.0f;
    const float nx = -W.ey[i] * rn, ny = W.ex[i] * rn;
    const float dn = ux[i] * nx + uy[i] * ny;
    const float rx_ = fmaf(2.0f * dn, nx, ux[i + 1] - ux[i]), ry_ = fmaf(2.0f * dn, ny, uy[i + 1] - uy[i]);
    Lm = fmaf(rx_, rx_, fmaf(ry_, ry_, Lm));
  }
  // interaction factors in(t_i) and the smoothed check s(1 - L / eps)
  float F = ok ? 1.0f : 0.0f;
  const float zc = 1.0f - Lm * inv_eps;
  if constexpr (MODE == kSigmoid) {
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const float E1 = ex2(-S.a2 * t[i]), E2 = ex2(fmaf(S.a2, t[i], -S.a2));
      F *= rcp((1.0f + E1) * (1.0f + E2));
    }
    F *= rcp(1.0f + ex2(-S.a2 * zc));
  } else {
#pragma unroll
    for (int i = 0; i < K; ++i) F *= med01(fmaf(S.a6, t[i], 0.5f)) * med01(fmaf(-S.a6, t[i], S.a6h));
    F *= med01(fmaf(S.a6, zc, 0.5f));
  }
  P.F = F;
  if (ballot(F != 0.0f) == 0) return 0.0f;
  const float V = obstruct_all<K, MODE>(S, P, F);
  return V / fmaxf(len * len, S.dmin2);
}

}  // namespace drt
