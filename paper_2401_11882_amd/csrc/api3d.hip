// C ABI of the 3D tracer (scenes of parallelogram panels): argument checks,
// workspace layout, launches.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>

#include "../../include/drt.h"
#include "dev.h"
#include "path3d.h"
#include "trace.h"
#include "trace3d.h"

extern "C" __attribute__((visibility("hidden"))) int drt_internal_fail(int code, const char* msg);
extern "C" __attribute__((visibility("hidden"))) int64_t drt_internal_cache_limit(void);
extern "C" __attribute__((visibility("hidden"))) int drt_internal_screen(void);
extern "C" __attribute__((visibility("hidden"))) int drt_internal_cut(void);

namespace {

int failf(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int failf(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  return drt_internal_fail(code, buf);
}

int hip_fail(hipError_t e, const char* what) { return failf(DRT_EHIP, "%s: %s", what, hipGetErrorString(e)); }

constexpr size_t kAlign = 256;
constexpr size_t kMaxLds = 48 * 1024;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int64_t count_candidates(int64_t P, int K) {
  int64_t total = 1, term = 0;
  for (int k = 1; k <= K; ++k) {
    term = (k == 1) ? P : term * (P - 1);
    total += term;
  }
  return total;
}

struct Plan3 {
  int n_tiles;
  int nw;
  int ncol;       // 3 + 13 P
  int cache_cap;  // 0 = no contribution cache
  size_t off_panels, off_boxes, off_loss, off_seed, off_grad, off_tmp, off_cache_c, off_cache_idx, off_cache_n,
      off_cache_mask, total;
  int mask_nb;      // 64-panel batches: max(1, ceil(P / 64))
  int mask_stride;  // culling-mask words per cache entry: (max_order + 1) mask_nb
};

// A cache entry's culling masks occupy one 64-bit register per lane.
static_assert((DRT_MAX_ORDER + 1) * ((DRT3_MAX_PANELS + 63) / 64) <= 64, "culling masks exceed one wavefront");

int check_scene3(const drt3_scene* s) {
  if (!s) return failf(DRT_EINVAL, "scene is NULL");
  if (s->n_panels < 0 || s->n_panels > DRT3_MAX_PANELS)
    return failf(DRT_EINVAL, "n_panels=%d outside [0, %d]", s->n_panels, DRT3_MAX_PANELS);
  if (s->n_panels > 0 && !s->panels_dev) return failf(DRT_EINVAL, "panels_dev is NULL");
  if (!s->tx_dev) return failf(DRT_EINVAL, "tx_dev is NULL");
  if (s->n_rx < 0) return failf(DRT_EINVAL, "n_rx=%d is negative", s->n_rx);
  if (s->n_rx > 0 && !s->rx_dev) return failf(DRT_EINVAL, "rx_dev is NULL");
  if (s->max_order < 0 || s->max_order > DRT_MAX_ORDER)
    return failf(DRT_EINVAL, "max_order=%d outside [0, %d]", s->max_order, DRT_MAX_ORDER);
  if (!std::isfinite(s->alpha) || !(s->alpha > 0.0f)) return failf(DRT_EINVAL, "alpha must be finite and > 0");
  if (!std::isfinite(s->d_min) || !(s->d_min > 0.0f)) return failf(DRT_EINVAL, "d_min must be finite and > 0");
  if (s->smoothing != DRT_SIGMOID && s->smoothing != DRT_HARD_SIGMOID)
    return failf(DRT_ENOTSUP, "smoothing=%d not supported", s->smoothing);
  if (s->rx_grid_nx != 0) {
    const int nx = s->rx_grid_nx;
    if (nx < 0 || nx % 8 != 0 || s->n_rx % (8 * nx) != 0)
      return failf(DRT_EINVAL, "rx_grid_nx=%d needs nx %% 8 == 0 and n_rx %% (8 nx) == 0", nx);
  }
  if (count_candidates(s->n_panels, s->max_order) > 0x7fffffffLL)
    return failf(DRT_EINVAL, "candidate count exceeds 2^31-1");
  return DRT_OK;
}

Plan3 make_plan3(const drt3_scene* s) {
  Plan3 p{};
  p.n_tiles = (s->n_rx + drt::kWave - 1) / drt::kWave;
  p.nw = p.n_tiles < 512 ? 16 : (p.n_tiles < 2048 ? 8 : 4);
  while (p.nw > 2 && drt::backward3_lds_bytes(p.nw, s->n_panels) > kMaxLds) p.nw >>= 1;
  p.ncol = 3 + drt::kPanelGrad * s->n_panels;
  const size_t P1 = s->n_panels > 0 ? (size_t)s->n_panels : 1;
  const size_t T1 = p.n_tiles > 0 ? (size_t)p.n_tiles : 1;
  size_t off = 0;
  p.off_panels = off;
  off = align_up(off + sizeof(drt::PanelRec) * P1);
  p.off_boxes = off;
  off = align_up(off + sizeof(drt::PanelBox) * P1);
  p.off_loss = off;
  off = align_up(off + sizeof(float) * T1);
  p.off_seed = off;
  off = align_up(off + sizeof(float) * (size_t)(s->n_rx > 0 ? s->n_rx : 1));
  p.off_grad = off;
  off = align_up(off + sizeof(float) * (size_t)p.ncol * T1);
  p.off_tmp = off;
  off = align_up(off + sizeof(float) * drt::kPanelGrad * P1);
  // contribution cache: a wavefront meets at most ceil(n1 / nw) + ceil((C - n1) / nw)
  // candidates (orders 0-1, n1 = 1 + P of them, then the rest)
  const int64_t n_cand = count_candidates(s->n_panels, s->max_order);
  const int64_t n1 = std::min<int64_t>(n_cand, 1 + (int64_t)s->n_panels);
  const int64_t per_wave = (n1 + p.nw - 1) / p.nw + (n_cand - n1 + p.nw - 1) / p.nw;
  const int64_t slots = (int64_t)p.n_tiles * p.nw;
  p.mask_nb = s->n_panels > 0 ? (s->n_panels + drt::kWave - 1) / drt::kWave : 1;
  p.mask_stride = (s->max_order + 1) * p.mask_nb;
  const int64_t entry = (int64_t)drt::kWave * sizeof(float) + sizeof(int) + (int64_t)p.mask_stride * sizeof(uint64_t);
  const int64_t limit = drt_internal_cache_limit();
  int64_t cap = per_wave;
  if (slots > 0 && limit > 0) {
    const int64_t fit = (limit - slots * (int64_t)sizeof(int)) / (slots * entry);
    if (fit < cap) cap = fit;
  } else {
    cap = 0;
  }
  p.cache_cap = cap > 0 ? (int)cap : 0;
  p.off_cache_c = off;
  off = align_up(off + sizeof(float) * (size_t)slots * p.cache_cap * drt::kWave);
  p.off_cache_idx = off;
  off = align_up(off + sizeof(int) * (size_t)slots * p.cache_cap);
  p.off_cache_n = off;
  off = align_up(off + sizeof(int) * (size_t)(p.cache_cap > 0 ? slots : 0));
  p.off_cache_mask = off;
  off = align_up(off + sizeof(uint64_t) * (size_t)slots * p.cache_cap * p.mask_stride);
  p.total = off;
  return p;
}

drt::Trace3Args make_args3(const drt3_scene* s, const Plan3& p, void* ws) {
  drt::Trace3Args A{};
  char* w = static_cast<char*>(ws);
  A.panels = reinterpret_cast<const drt::PanelRec*>(w + p.off_panels);
  A.boxes = drt_internal_screen() ? reinterpret_cast<const drt::PanelBox*>(w + p.off_boxes) : nullptr;
  const bool hard = s->smoothing == DRT_HARD_SIGMOID;
  A.mode = hard ? 1 : 0;
  A.cull_c = (hard ? drt::kHardCullMargin : drt::kCullMargin) / s->alpha;
  A.screen = drt_internal_screen();
  A.cut = drt::cut_factor(drt_internal_cut() != 0, (int)count_candidates(s->n_panels, s->max_order));
  A.tx = s->tx_dev;
  A.rx = s->rx_dev;
  A.n_panels = s->n_panels;
  A.n_rx = s->n_rx;
  A.grid_nx = s->rx_grid_nx;
  A.n_cand = (int)count_candidates(s->n_panels, s->max_order);
  A.max_order = s->max_order;
  A.alpha = s->alpha;
  A.a2 = s->alpha * drt::kLog2e;
  A.band_k = 1.0f + 2.0f * (hard ? drt::kHardBandMargin : drt::kBandMargin) / s->alpha;
  A.dmin2 = s->d_min * s->d_min;
  if (p.cache_cap > 0) {
    A.cache_c = reinterpret_cast<float*>(w + p.off_cache_c);
    A.cache_idx = reinterpret_cast<int*>(w + p.off_cache_idx);
    A.cache_n = reinterpret_cast<int*>(w + p.off_cache_n);
    A.cache_cap = p.cache_cap;
    A.cache_mask = reinterpret_cast<uint64_t*>(w + p.off_cache_mask);
    A.mask_stride = p.mask_stride;
  }
  A.mask_nb = p.mask_nb;
  return A;
}

int check_ws3(const Plan3& p, void* ws, size_t ws_bytes) {
  if (!ws) return failf(DRT_EWORKSPACE, "workspace is NULL");
  if (ws_bytes < p.total) return failf(DRT_EWORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, p.total);
  if (reinterpret_cast<uintptr_t>(ws) % 16 != 0) return failf(DRT_EWORKSPACE, "workspace not 16-byte aligned");
  return DRT_OK;
}

int check_loss3(int32_t loss_kind, float log_eps) {
  if (loss_kind < DRT_LOSS_NONE || loss_kind > DRT_LOSS_NEG_MIN_POWER)
    return failf(DRT_EINVAL, "loss_kind=%d unknown", loss_kind);
  if (loss_kind == DRT_LOSS_NEG_MEAN_LOG_POWER && (!std::isfinite(log_eps) || !(log_eps > 0.0f)))
    return failf(DRT_EINVAL, "log_eps must be finite and > 0");
  return DRT_OK;
}

int prep3(const drt3_scene* s, const Plan3& p, void* ws, hipStream_t st) {
  char* w = static_cast<char*>(ws);
  const float cull_c = (s->smoothing == DRT_HARD_SIGMOID ? drt::kHardCullMargin : drt::kCullMargin) / s->alpha;
  hipError_t e = drt::launch_prep_panels(s->panels_dev, s->n_panels, cull_c,
                                         reinterpret_cast<drt::PanelRec*>(w + p.off_panels),
                                         reinterpret_cast<drt::PanelBox*>(w + p.off_boxes), st);
  return e == hipSuccess ? DRT_OK : hip_fail(e, "prep_panels launch");
}

int enqueue_forward3(const drt3_scene* s, const Plan3& p, const drt::Trace3Args& A, int32_t loss_kind,
                     float log_eps, float* power, float* loss, float* seed, void* ws, hipStream_t st) {
  int rc = prep3(s, p, ws, st);
  if (rc) return rc;
  float* loss_part = reinterpret_cast<float*>(static_cast<char*>(ws) + p.off_loss);
  const bool min_loss = loss_kind == DRT_LOSS_NEG_MIN_POWER;
  hipError_t e;
  if (p.n_tiles > 0) {
    e = drt::launch_forward3(A, p.n_tiles, p.nw, power, min_loss ? nullptr : seed, loss_part,
                             min_loss ? DRT_LOSS_NONE : loss_kind, log_eps, st);
    if (e != hipSuccess) return hip_fail(e, "forward3 launch");
  }
  if (min_loss) {
    e = drt::launch_min_seed(power, s->n_rx, loss, seed, st);
    return e == hipSuccess ? DRT_OK : hip_fail(e, "min-loss launch");
  }
  if (loss_kind != DRT_LOSS_NONE && loss) {
    const double scale =
        loss_kind == DRT_LOSS_NEG_MEAN_LOG_POWER ? (s->n_rx > 0 ? -1.0 / (double)s->n_rx : 0.0) : 1.0;
    e = drt::launch_reduce_scalar(loss_part, p.n_tiles, scale, loss, st);
    if (e != hipSuccess) return hip_fail(e, "loss reduction launch");
  }
  return DRT_OK;
}

int enqueue_backward3(const drt3_scene* s, const Plan3& p, const drt::Trace3Args& A, const float* gP, float* gtx,
                      float* gpanels, float* grx, int reuse, void* ws, hipStream_t st) {
  char* w = static_cast<char*>(ws);
  float* part = reinterpret_cast<float*>(w + p.off_grad);
  hipError_t e;
  if (p.n_tiles > 0) {
    e = drt::launch_backward3(A, p.n_tiles, p.nw, gP, part, grx, reuse, st);
    if (e != hipSuccess) return hip_fail(e, "backward3 launch");
  }
  e = drt::launch_panel_grads(part, p.n_tiles, s->n_panels, s->panels_dev, reinterpret_cast<float*>(w + p.off_tmp),
                              gtx, gpanels, st);
  return e == hipSuccess ? DRT_OK : hip_fail(e, "panel gradient launch");
}

}  // namespace

extern "C" {

int drt3_workspace_size(const drt3_scene* scene, size_t* bytes) {
  int rc = check_scene3(scene);
  if (rc) return rc;
  if (!bytes) return failf(DRT_EINVAL, "bytes is NULL");
  *bytes = make_plan3(scene).total;
  return DRT_OK;
}

int drt3_forward(const drt3_scene* scene, int32_t loss_kind, float log_eps, float* power_dev, float* loss_dev,
                 float* seed_dev, void* ws_dev, size_t ws_bytes, void* stream) {
  int rc = check_scene3(scene);
  if (rc) return rc;
  if ((rc = check_loss3(loss_kind, log_eps))) return rc;
  if (scene->n_rx > 0 && !power_dev) return failf(DRT_EINVAL, "power_dev is NULL");
  if (seed_dev && loss_kind == DRT_LOSS_NONE) return failf(DRT_EINVAL, "seed_dev needs a loss_kind");
  if (loss_kind == DRT_LOSS_NEG_MIN_POWER && scene->n_rx < 1) return failf(DRT_EINVAL, "min loss needs n_rx >= 1");
  const Plan3 p = make_plan3(scene);
  if ((rc = check_ws3(p, ws_dev, ws_bytes))) return rc;
  const drt::Trace3Args A = make_args3(scene, p, ws_dev);
  return enqueue_forward3(scene, p, A, loss_kind, log_eps, power_dev, loss_dev, seed_dev, ws_dev,
                          static_cast<hipStream_t>(stream));
}

int drt3_backward(const drt3_scene* scene, const float* grad_power_dev, int32_t flags, float* grad_tx_dev,
                  float* grad_panels_dev, float* grad_rx_dev, void* ws_dev, size_t ws_bytes, void* stream) {
  int rc = check_scene3(scene);
  if (rc) return rc;
  if (flags & ~DRT_BWD_REUSE_FORWARD) return failf(DRT_EINVAL, "unknown flags 0x%x", flags);
  if (scene->n_rx > 0 && !grad_power_dev) return failf(DRT_EINVAL, "grad_power_dev is NULL");
  if (!grad_tx_dev) return failf(DRT_EINVAL, "grad_tx_dev is NULL");
  if (scene->n_panels > 0 && !grad_panels_dev) return failf(DRT_EINVAL, "grad_panels_dev is NULL");
  const Plan3 p = make_plan3(scene);
  if ((rc = check_ws3(p, ws_dev, ws_bytes))) return rc;
  const drt::Trace3Args A = make_args3(scene, p, ws_dev);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool reuse = (flags & DRT_BWD_REUSE_FORWARD) != 0;
  // (with the flag, the panel records the forward wrote into this workspace
  // are still those of this scene)
  if (!reuse && (rc = prep3(scene, p, ws_dev, st))) return rc;
  return enqueue_backward3(scene, p, A, grad_power_dev, grad_tx_dev, grad_panels_dev, grad_rx_dev, reuse ? 1 : 0,
                           ws_dev, st);
}

int drt3_forward_backward(const drt3_scene* scene, int32_t loss_kind, float log_eps, float* power_dev,
                          float* loss_dev, float* grad_tx_dev, float* grad_panels_dev, float* grad_rx_dev,
                          void* ws_dev, size_t ws_bytes, void* stream) {
  int rc = check_scene3(scene);
  if (rc) return rc;
  if ((rc = check_loss3(loss_kind, log_eps))) return rc;
  if (loss_kind == DRT_LOSS_NONE) return failf(DRT_EINVAL, "forward_backward needs a loss_kind");
  if (loss_kind == DRT_LOSS_NEG_MIN_POWER && scene->n_rx < 1) return failf(DRT_EINVAL, "min loss needs n_rx >= 1");
  if (scene->n_rx > 0 && !power_dev) return failf(DRT_EINVAL, "power_dev is NULL");
  if (!grad_tx_dev) return failf(DRT_EINVAL, "grad_tx_dev is NULL");
  if (scene->n_panels > 0 && !grad_panels_dev) return failf(DRT_EINVAL, "grad_panels_dev is NULL");
  const Plan3 p = make_plan3(scene);
  if ((rc = check_ws3(p, ws_dev, ws_bytes))) return rc;
  const drt::Trace3Args A = make_args3(scene, p, ws_dev);
  hipStream_t st = static_cast<hipStream_t>(stream);
  float* seed = reinterpret_cast<float*>(static_cast<char*>(ws_dev) + p.off_seed);
  rc = enqueue_forward3(scene, p, A, loss_kind, log_eps, power_dev, loss_dev, seed, ws_dev, st);
  if (rc) return rc;
  return enqueue_backward3(scene, p, A, seed, grad_tx_dev, grad_panels_dev, grad_rx_dev, 1, ws_dev, st);
}

}  // extern "C"
