// Smoothed image-method tracer: forward, hand-written adjoint and the small
// reductions around them, for gfx950 (wave64).
//
// Work decomposition.  A workgroup owns one tile of 64 receivers (an 8x8
// block of a grid, or 64 consecutive receivers); its NW wavefronts split the
// candidate list (wave w takes chunks w, w+NW, ... of `cchunk` candidates).
// Inside a wavefront every lane is one receiver while the candidate and the
// wall being tested are wave-uniform, so wall records come in through scalar
// loads and candidate bookkeeping runs on the scalar unit.  Because a
// workgroup sees every candidate of its receivers, the power P(r) is complete
// at the end of the workgroup and the loss seed dL/dP(r) is formed there.
//
// Exact work skipping (no change to the FP32 result):
//  * a candidate whose interaction factor is exactly 0 in every lane (the
//    reflection points are far outside their segments, so prod (1+E) overflows
//    and its reciprocal is 0) skips all obstruction tests;
//  * an obstruction test whose leg and wall parameters are more than 18/alpha
//    outside [0, 1] has in(tau) in(upsilon) < 2^-25, so its factor rounds to
//    1.0f; it is decided on numerators before any reciprocal or exponential.
//
// Numerics.  in(x) = s(ax) s(a(1-x)) = 1 / ((1+E1)(1+E2)) with
// E1 = exp(-a x), E2 = exp(-a (1-x)).  An obstruction factor
// 1 - in(tau) in(ups) is formed as num / (1 + num) with
// num = n_t + n_u + n_t n_u, n_t = E1 + E2 + E1 E2: every term is positive,
// so deep shadows keep full relative precision.  Per-lane power sums over
// candidates are Kahan-compensated; every cross-lane / cross-wave /
// cross-block sum has a fixed order.
#include "dev.h"
#include "trace.h"

namespace drt {

// ---------------------------------------------------------------------------
// Per-candidate path state (images, back-traced points, interaction data)
// ---------------------------------------------------------------------------

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

// E1 = exp(-alpha x), E2 = exp(-alpha (1 - x)); either may be +inf, then
// 1 / ((1+E1)(1+E2)) is exactly 0 (no NaN: both are >= 0).
__device__ __forceinline__ void inside_pair(float x, float a2, float& E1, float& E2) {
  E1 = ex2(-a2 * x);
  E2 = ex2(fmaf(a2, x, -a2));
}

// E / (1 + E) = 1 - s, accurate for small E and exactly 1 for huge or infinite E.
__device__ __forceinline__ float one_minus_s(float E) { return E < kBig ? E * rcp(1.0f + E) : 1.0f; }

template <int K>
__device__ __forceinline__ void setup_path(const TraceArgs& A, const Cand& cd, float txx, float txy,
                                           float rxx, float rxy, bool live, Path<K>& P) {
  const int sv[3] = {cd.s0, cd.s1, cd.s2};
#pragma unroll
  for (int i = 0; i < Path<K>::KI; ++i) P.s[i] = (i < K) ? sv[i] : -1;
  P.Ix[0] = txx;
  P.Iy[0] = txy;
  bool ok = live;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const WallRec w = A.walls[P.s[i]];
    const float nx = -w.ey, ny = w.ex;
    const float nn = nx * nx + ny * ny;
    ok = ok && (nn > 0.0f);
    const float h = ((P.Ix[i] - w.ax) * nx + (P.Iy[i] - w.ay) * ny) / (nn > 0.0f ? nn : 1.0f);
    P.Ix[i + 1] = P.Ix[i] - 2.0f * h * nx;
    P.Iy[i + 1] = P.Iy[i] - 2.0f * h * ny;
  }
  P.Xx[0] = txx;
  P.Xy[0] = txy;
  P.Xx[K + 1] = rxx;
  P.Xy[K + 1] = rxy;
  float F = ok ? 1.0f : 0.0f;
#pragma unroll
  for (int i = K; i >= 1; --i) {
    const WallRec w = A.walls[P.s[i - 1]];
    const float dx = P.Ix[i] - P.Xx[i + 1], dy = P.Iy[i] - P.Xy[i + 1];
    const float wx = w.ax - P.Xx[i + 1], wy = w.ay - P.Xy[i + 1];
    const float den = dx * w.ey - dy * w.ex;
    const bool good = den != 0.0f;
    const float inv = good ? rcp(den) : 0.0f;
    const float t = (wx * dy - wy * dx) * inv;     // along the wall segment
    const float u = (wx * w.ey - wy * w.ex) * inv; // between X_{i+1} and the image
    F = good ? F : 0.0f;
    P.Xx[i] = fmaf(t, w.ex, w.ax);
    P.Xy[i] = fmaf(t, w.ey, w.ay);
    float E1, E2, E3, E4;
    inside_pair(t, A.a2, E1, E2);
    inside_pair(u, A.a2, E3, E4);
    F *= rcp(((1.0f + E1) * (1.0f + E2)) * ((1.0f + E3) * (1.0f + E4)));
    P.t[i - 1] = t;
    P.u[i - 1] = u;
    P.inv[i - 1] = inv;
    P.dx[i - 1] = dx;
    P.dy[i - 1] = dy;
    P.wx[i - 1] = wx;
    P.wy[i - 1] = wy;
  }
  P.F = F;
#pragma unroll
  for (int l = 0; l <= K; ++l) {
    P.lo[l] = (l >= 1) ? sv[l - 1] : -1;
    P.hi[l] = (l + 1 <= K) ? sv[l] : -1;
  }
}

// Geometry of one (leg, wall) obstruction test.  Returns true when the test
// is unsaturated (both parameters within 18/alpha of [0, 1]).
struct LegGeom {
  float Dx, Dy, nXD, Xx, Xy;
};

__device__ __forceinline__ bool obstruction_live(const LegGeom& L, const WallRec& w, float band_k,
                                                 float& den, float& tn, float& un) {
  den = L.Dx * w.ey - L.Dy * w.ex;
  tn = fmaf(w.ax, L.Dy, fmaf(-w.ay, L.Dx, L.nXD));     // (a - X) x D
  un = fmaf(L.Xy, w.ex, fmaf(-L.Xx, w.ey, w.axe));     // (a - X) x e
  const float kd = band_k * fabsf(den);
  return (fabsf(fmaf(2.0f, tn, -den)) < kd) & (fabsf(fmaf(2.0f, un, -den)) < kd);
}

struct ObsVals {
  float tau, ups, inv, E1, E2, E3, E4, nt, nu, num;
};

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

// V times every obstruction factor of the path.
template <int K>
__device__ __forceinline__ float obstruct_all(const TraceArgs& A, const Path<K>& P, float V) {
  LegGeom L[K + 1];
  leg_geoms<K>(P, L);
  for (int j = 0; j < A.n_walls; ++j) {
    const WallRec w = A.walls[j];
#pragma unroll
    for (int l = 0; l <= K; ++l) {
      if (j == P.lo[l] || j == P.hi[l]) continue;
      float den, tn, un;
      if (obstruction_live(L[l], w, A.band_k, den, tn, un)) {
        const ObsVals o = obstruction_vals(den, tn, un, A.a2);
        V *= o.num * rcp(1.0f + o.num);
      }
    }
  }
  return V;
}

template <int K>
__device__ __forceinline__ float path_power(const TraceArgs& A, const Cand& cd, float txx, float txy,
                                            float rxx, float rxy, bool live) {
  Path<K> P;
  setup_path<K>(A, cd, txx, txy, rxx, rxy, live, P);
  if (ballot(P.F != 0.0f) == 0) return 0.0f;
  const float V = obstruct_all<K>(A, P, P.F);
  const float ex = rxx - P.Ix[K], ey = rxy - P.Iy[K];
  const float d2 = fmaf(ex, ex, ey * ey);
  return V / fmaxf(d2, A.dmin2);
}

__device__ __forceinline__ void kahan_add(float& sum, float& comp, float x) {
  const float y = x - comp;
  const float t = sum + y;
  comp = (t - sum) - y;
  sum = t;
}

// ---------------------------------------------------------------------------
// Forward kernel
// ---------------------------------------------------------------------------

template <int NW>
__global__ __launch_bounds__(NW * kWave) void k_forward(TraceArgs A, float* __restrict__ power,
                                                        float* __restrict__ seed,
                                                        float* __restrict__ loss_part, int loss_kind,
                                                        float log_eps) {
  __shared__ float red[NW][2][kWave];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = uniform(threadIdx.x >> 6);
  const int tile = blockIdx.x;
  const int m = rx_of_lane(tile, lane, A.grid_nx);
  const bool live = m < A.n_rx;
  const float rxx = live ? A.rx[2 * m] : 0.5f;
  const float rxy = live ? A.rx[2 * m + 1] : 0.5f;
  const float txx = A.tx[0], txy = A.tx[1];

  float sum = 0.0f, comp = 0.0f;
  const int stride = NW * A.cchunk;
  for (int c0 = wave * A.cchunk; c0 < A.n_cand; c0 += stride) {
    const int c1 = min(c0 + A.cchunk, A.n_cand);
    for (int c = c0; c < c1; ++c) {
      const Cand cd = decode_candidate(c, A.n_walls);
      float v;
      switch (cd.k) {
        case 0: v = path_power<0>(A, cd, txx, txy, rxx, rxy, live); break;
        case 1: v = path_power<1>(A, cd, txx, txy, rxx, rxy, live); break;
        case 2: v = path_power<2>(A, cd, txx, txy, rxx, rxy, live); break;
        default: v = path_power<3>(A, cd, txx, txy, rxx, rxy, live); break;
      }
      kahan_add(sum, comp, v);
    }
  }
  red[wave][0][lane] = sum;
  red[wave][1][lane] = comp;
  __syncthreads();
  if (wave == 0) {
    float s = 0.0f, cs = 0.0f;
#pragma unroll
    for (int w = 0; w < NW; ++w) kahan_add(s, cs, red[w][0][lane] - red[w][1][lane]);
    const float P = s - cs;
    float lp = 0.0f;
    if (live) {
      power[m] = P;
      if (loss_kind == 1) {
        lp = P;
        if (seed) seed[m] = 1.0f;
      } else if (loss_kind == 2) {
        lp = logf(P + log_eps);
        if (seed) seed[m] = -1.0f / ((float)A.n_rx * (P + log_eps));
      }
    }
    if (loss_kind != 0) {
      const float tot = wave_sum(lp);
      if (lane == 0) loss_part[tile] = tot;
    }
  }
}

// ---------------------------------------------------------------------------
// Adjoint kernel
// ---------------------------------------------------------------------------

// Per-wave LDS accumulator layout: [0,1] = d/dtx, [2 + 4j + c] = d/d walls[j][c].
__device__ __forceinline__ void acc_wall(float* acc, int j, float dax, float day, float dbx, float dby,
                                         int lane) {
  const float s0 = wave_sum(dax), s1 = wave_sum(day), s2 = wave_sum(dbx), s3 = wave_sum(dby);
  if (lane == 0) {
    float* p = acc + 2 + 4 * j;
    p[0] += s0;
    p[1] += s1;
    p[2] += s2;
    p[3] += s3;
  }
}

template <int K>
__device__ __forceinline__ void path_adjoint(const TraceArgs& A, const Cand& cd, float txx, float txy,
                                             float rxx, float rxy, bool live, float g, float* acc,
                                             int lane, float& gtx_x, float& gtx_y, float& grx_x,
                                             float& grx_y) {
  Path<K> P;
  setup_path<K>(A, cd, txx, txy, rxx, rxy, live, P);
  if (ballot(P.F != 0.0f && g != 0.0f) == 0) return;
  const float V = obstruct_all<K>(A, P, P.F);
  const float ex = rxx - P.Ix[K], ey = rxy - P.Iy[K];
  const float d2 = fmaf(ex, ex, ey * ey);
  const float D2 = fmaxf(d2, A.dmin2);
  const float Wl = g * (V / D2);  // dL/d(log V) for this lane
  if (ballot(Wl != 0.0f) == 0) return;

  // -- obstruction tests, reverse: dlog q / dtau, dlog q / dups -> geometry
  LegGeom L[K + 1];
  leg_geoms<K>(P, L);
  float Sgwx[K + 1], Sgwy[K + 1], SgDx[K + 1], SgDy[K + 1];
#pragma unroll
  for (int l = 0; l <= K; ++l) Sgwx[l] = Sgwy[l] = SgDx[l] = SgDy[l] = 0.0f;
  const bool act = Wl != 0.0f;
  const float nalpha = -A.alpha;
  for (int j = 0; j < A.n_walls; ++j) {
    const WallRec w = A.walls[j];
    float gax = 0.0f, gay = 0.0f, gex = 0.0f, gey = 0.0f;
    bool any = false;
#pragma unroll
    for (int l = 0; l <= K; ++l) {
      if (j == P.lo[l] || j == P.hi[l]) continue;
      float den, tn, un;
      if (obstruction_live(L[l], w, A.band_k, den, tn, un) && act) {
        const ObsVals o = obstruction_vals(den, tn, un, A.a2);
        const float Ab = 1.0f + o.nt, Bb = 1.0f + o.nu;
        const float coef = nalpha * Wl * rcp(o.num * Ab * Bb);
        const float gt = coef * (o.E1 - o.E2) * Bb;
        const float gu = coef * (o.E3 - o.E4) * Ab;
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
    if (ballot(any) != 0) acc_wall(acc, j, gax - gex, gay - gey, gex, gey, lane);
  }

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
  if (d2 > A.dmin2) {
    const float f = 2.0f * Wl / d2;
    gIx[K] += f * ex;
    gIy[K] += f * ey;
    gXx[K + 1] -= f * ex;
    gXy[K + 1] -= f * ey;
  }
  // -- interactions i = 1..K: smoothed factors and back-trace, in order
#pragma unroll
  for (int i = 1; i <= K; ++i) {
    const WallRec w = A.walls[P.s[i - 1]];
    const float t = P.t[i - 1], u = P.u[i - 1], inv = P.inv[i - 1];
    float E1, E2, E3, E4;
    inside_pair(t, A.a2, E1, E2);
    inside_pair(u, A.a2, E3, E4);
    const float aw = A.alpha * Wl;
    const float gti = aw * (one_minus_s(E1) - one_minus_s(E2));
    const float gu = aw * (one_minus_s(E3) - one_minus_s(E4));
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
  gtx_x += gXx[0];
  gtx_y += gXy[0];
  grx_x += gXx[K + 1];
  grx_y += gXy[K + 1];
  if (K == 0) {
    // I_0 is the transmitter itself
    gtx_x += gIx[0];
    gtx_y += gIy[0];
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
      const WallRec w = A.walls[P.s[i - 1]];
      const float nx = -w.ey, ny = w.ex;
      const float nn = nx * nx + ny * ny;
      const float px = P.Ix[i - 1] - w.ax, py = P.Iy[i - 1] - w.ay;
      const float h = (px * nx + py * ny) / nn;
      const float Gx = GIx[i], Gy = GIy[i];
      const float Gn = Gx * nx + Gy * ny;
      const float kk = 2.0f * Gn / nn;
      GIx[i - 1] += Gx - kk * nx;
      GIy[i - 1] += Gy - kk * ny;
      const float gax = kk * nx, gay = kk * ny;
      const float gnx = -2.0f * (Gn * (px - 2.0f * h * nx) / nn + h * Gx);
      const float gny = -2.0f * (Gn * (py - 2.0f * h * ny) / nn + h * Gy);
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

template <int NW>
__global__ __launch_bounds__(NW * kWave) void k_backward(TraceArgs A, const float* __restrict__ gP,
                                                         float* __restrict__ part,
                                                         float* __restrict__ grad_rx) {
  extern __shared__ float smem[];
  const int ncol = 2 + 4 * A.n_walls;
  float* accs = smem;                           // [NW][ncol]
  float* rxr = smem + NW * ncol;                // [NW][2][64]
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = uniform(threadIdx.x >> 6);
  for (int i = threadIdx.x; i < NW * ncol; i += NW * kWave) accs[i] = 0.0f;
  __syncthreads();
  float* acc = accs + wave * ncol;

  const int tile = blockIdx.x;
  const int m = rx_of_lane(tile, lane, A.grid_nx);
  const bool live = m < A.n_rx;
  const float rxx = live ? A.rx[2 * m] : 0.5f;
  const float rxy = live ? A.rx[2 * m + 1] : 0.5f;
  const float g = live ? gP[m] : 0.0f;
  const float txx = A.tx[0], txy = A.tx[1];
  float gtx_x = 0.0f, gtx_y = 0.0f, grx_x = 0.0f, grx_y = 0.0f;

  if (ballot(g != 0.0f) != 0) {
    const int stride = NW * A.cchunk;
    for (int c0 = wave * A.cchunk; c0 < A.n_cand; c0 += stride) {
      const int c1 = min(c0 + A.cchunk, A.n_cand);
      for (int c = c0; c < c1; ++c) {
        const Cand cd = decode_candidate(c, A.n_walls);
        switch (cd.k) {
          case 0: path_adjoint<0>(A, cd, txx, txy, rxx, rxy, live, g, acc, lane, gtx_x, gtx_y, grx_x, grx_y); break;
          case 1: path_adjoint<1>(A, cd, txx, txy, rxx, rxy, live, g, acc, lane, gtx_x, gtx_y, grx_x, grx_y); break;
          case 2: path_adjoint<2>(A, cd, txx, txy, rxx, rxy, live, g, acc, lane, gtx_x, gtx_y, grx_x, grx_y); break;
          default: path_adjoint<3>(A, cd, txx, txy, rxx, rxy, live, g, acc, lane, gtx_x, gtx_y, grx_x, grx_y); break;
        }
      }
    }
  }
  {
    const float sx = wave_sum(gtx_x), sy = wave_sum(gtx_y);
    if (lane == 0) {
      acc[0] += sx;
      acc[1] += sy;
    }
  }
  rxr[(wave * 2 + 0) * kWave + lane] = grx_x;
  rxr[(wave * 2 + 1) * kWave + lane] = grx_y;
  __syncthreads();
  if (wave == 0 && live && grad_rx) {
    float sx = 0.0f, sy = 0.0f;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      sx += rxr[(w * 2 + 0) * kWave + lane];
      sy += rxr[(w * 2 + 1) * kWave + lane];
    }
    grad_rx[2 * m] = sx;
    grad_rx[2 * m + 1] = sy;
  }
  for (int col = threadIdx.x; col < ncol; col += NW * kWave) {
    float s = 0.0f;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += accs[w * ncol + col];
    part[(size_t)tile * ncol + col] = s;
  }
}

// ---------------------------------------------------------------------------
// Small kernels
// ---------------------------------------------------------------------------

__global__ void k_prep_walls(const float* __restrict__ walls, int n, WallRec* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const float ax = walls[4 * j], ay = walls[4 * j + 1];
  const float ex = walls[4 * j + 2] - ax, ey = walls[4 * j + 3] - ay;
  WallRec r;
  r.ax = ax;
  r.ay = ay;
  r.ex = ex;
  r.ey = ey;
  r.axe = ax * ey - ay * ex;
  r.pad0 = r.pad1 = r.pad2 = 0.0f;
  out[j] = r;
}

// Column sums of part[n_rows][ncol] in FP64, fixed row order.
__global__ void k_reduce_cols(const float* __restrict__ part, int n_rows, int ncol,
                              float* __restrict__ out_head, int n_head, float* __restrict__ out_tail) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= ncol) return;
  double s = 0.0;
  for (int b = 0; b < n_rows; ++b) s += (double)part[(size_t)b * ncol + col];
  if (col < n_head) out_head[col] = (float)s;
  else out_tail[col - n_head] = (float)s;
}

// scale * sum(part[0..n)) in FP64 with a fixed tree order; one block of 256.
__global__ void k_reduce_scalar(const float* __restrict__ part, int n, double scale,
                                float* __restrict__ out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += (double)part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = (float)(scale * sh[0]);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

hipError_t launch_prep_walls(const float* walls, int n, WallRec* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_prep_walls, dim3((n + 255) / 256), dim3(256), 0, st, walls, n, out);
  return hipGetLastError();
}

template <int NW>
static hipError_t fwd_nw(const TraceArgs& A, int n_tiles, float* power, float* seed, float* loss_part,
                         int loss_kind, float log_eps, hipStream_t st) {
  hipLaunchKernelGGL(k_forward<NW>, dim3(n_tiles), dim3(NW * kWave), 0, st, A, power, seed, loss_part,
                     loss_kind, log_eps);
  return hipGetLastError();
}

hipError_t launch_forward(const TraceArgs& A, int n_tiles, int nw, float* power, float* seed,
                          float* loss_part, int loss_kind, float log_eps, hipStream_t st) {
  switch (nw) {
    case 2: return fwd_nw<2>(A, n_tiles, power, seed, loss_part, loss_kind, log_eps, st);
    case 4: return fwd_nw<4>(A, n_tiles, power, seed, loss_part, loss_kind, log_eps, st);
    case 8: return fwd_nw<8>(A, n_tiles, power, seed, loss_part, loss_kind, log_eps, st);
    case 16: return fwd_nw<16>(A, n_tiles, power, seed, loss_part, loss_kind, log_eps, st);
    default: return hipErrorInvalidValue;
  }
}

size_t backward_lds_bytes(int nw, int n_walls) {
  return sizeof(float) * ((size_t)nw * (2 + 4 * (size_t)n_walls) + (size_t)nw * 2 * kWave);
}

template <int NW>
static hipError_t bwd_nw(const TraceArgs& A, int n_tiles, const float* gP, float* part, float* grad_rx,
                         hipStream_t st) {
  const size_t lds = backward_lds_bytes(NW, A.n_walls);
  hipLaunchKernelGGL(k_backward<NW>, dim3(n_tiles), dim3(NW * kWave), lds, st, A, gP, part, grad_rx);
  return hipGetLastError();
}

hipError_t launch_backward(const TraceArgs& A, int n_tiles, int nw, const float* gP, float* part,
                           float* grad_rx, hipStream_t st) {
  switch (nw) {
    case 2: return bwd_nw<2>(A, n_tiles, gP, part, grad_rx, st);
    case 4: return bwd_nw<4>(A, n_tiles, gP, part, grad_rx, st);
    case 8: return bwd_nw<8>(A, n_tiles, gP, part, grad_rx, st);
    case 16: return bwd_nw<16>(A, n_tiles, gP, part, grad_rx, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_reduce_cols(const float* part, int n_rows, int ncol, float* out_head, int n_head,
                              float* out_tail, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_cols, dim3((ncol + 255) / 256), dim3(256), 0, st, part, n_rows, ncol,
                     out_head, n_head, out_tail);
  return hipGetLastError();
}

hipError_t launch_reduce_scalar(const float* part, int n, double scale, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_scalar, dim3(1), dim3(256), 0, st, part, n, scale, out);
  return hipGetLastError();
}

}  // namespace drt
