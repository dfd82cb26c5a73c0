// C ABI of the tracer library: argument checks, workspace layout, launches.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "../../include/drt.h"
#include "dev.h"
#include "trace.h"

// Scratch of the allocation-free entry point drt_forward_backward_noalloc
// (64 MiB per device; see scratch_of_current_device).
constexpr size_t kScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(DRT_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// Launch shape overrides (0 = automatic).
int g_nw_override = 0;
int g_cchunk_override = 0;
// Largest contribution cache placed in a workspace (bytes); 0 disables it.
int64_t g_cache_limit = 32LL << 30;
int g_screen = 1;
int g_cut = 1;

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int64_t count_candidates(int64_t W, int K) {
  int64_t total = 1, term = 0;
  for (int k = 1; k <= K; ++k) {
    term = (k == 1) ? W : term * (W - 1);
    total += term;
  }
  return total;
}

struct Plan {
  int n_tiles;
  int nw;
  int cchunk;
  int ncol;       // 2 + 4 W
  int cache_cap;  // 0 = no contribution cache
  size_t off_walls, off_boxes, off_loss, off_seed, off_grad, off_cache_c, off_cache_idx, off_cache_n, off_cache_box,
      total;
  int box_stride;  // floats of leg boxes per cache entry: 6 (max_order + 1)
};

int pick_nw(int n_tiles, int n_walls, int max_order) {
  int nw = g_nw_override;
  if (nw == 0) nw = n_tiles < 512 ? 16 : (n_tiles < 2048 ? 8 : 4);
  while (nw > 2 && (drt::backward_lds_bytes(nw, n_walls) > 48 * 1024 ||
                    drt::forward_lds_bytes(nw, max_order) > 48 * 1024))
    nw >>= 1;
  return nw;
}

int check_scene(const drt_scene* s) {
  if (!s) return fail(DRT_EINVAL, "scene is NULL");
  if (s->n_walls < 0 || s->n_walls > DRT_MAX_WALLS)
    return fail(DRT_EINVAL, "n_walls=%d outside [0, %d]", s->n_walls, DRT_MAX_WALLS);
  if (s->n_walls > 0 && !s->walls_dev) return fail(DRT_EINVAL, "walls_dev is NULL");
  if (!s->tx_dev) return fail(DRT_EINVAL, "tx_dev is NULL");
  if (s->n_rx < 0) return fail(DRT_EINVAL, "n_rx=%d is negative", s->n_rx);
  if (s->n_rx > 0 && !s->rx_dev && s->rx_grid_nx <= 0)
    return fail(DRT_EINVAL, "rx_dev is NULL and rx_grid_nx is 0 (no receiver array and no grid)");
  if (s->max_order < 0 || s->max_order > DRT_MAX_ORDER)
    return fail(DRT_EINVAL, "max_order=%d outside [0, %d]", s->max_order, DRT_MAX_ORDER);
  if (!std::isfinite(s->alpha) || !(s->alpha > 0.0f))
    return fail(DRT_EINVAL, "alpha must be finite and > 0");
  if (!std::isfinite(s->d_min) || !(s->d_min > 0.0f))
    return fail(DRT_EINVAL, "d_min must be finite and > 0");
  if (s->smoothing != DRT_SIGMOID && s->smoothing != DRT_HARD_SIGMOID)
    return fail(DRT_ENOTSUP, "smoothing=%d not supported", s->smoothing);
  if (s->rx_grid_nx != 0) {
    const int nx = s->rx_grid_nx;
    if (nx < 0 || nx % 8 != 0 || s->n_rx % (8 * nx) != 0)
      return fail(DRT_EINVAL, "rx_grid_nx=%d needs nx %% 8 == 0 and n_rx %% (8 nx) == 0", nx);
  }
  if (count_candidates(s->n_walls, s->max_order) > 0x7fffffffLL)
    return fail(DRT_EINVAL, "candidate count exceeds 2^31-1");
  return DRT_OK;
}

// cache_limit: largest contribution cache placed in the workspace (bytes).
Plan make_plan(const drt_scene* s, int64_t cache_limit) {
  Plan p{};
  p.n_tiles = (s->n_rx + drt::kWave - 1) / drt::kWave;
  p.nw = pick_nw(p.n_tiles, s->n_walls, s->max_order);
  p.cchunk = g_cchunk_override > 0 ? g_cchunk_override : 1;
  p.ncol = 2 + 4 * s->n_walls;
  size_t off = 0;
  p.off_walls = off;
  off = align_up(off + sizeof(drt::WallRec) * (size_t)(s->n_walls > 0 ? s->n_walls : 1));
  p.off_boxes = off;
  off = align_up(off + sizeof(drt::WallBox) * (size_t)(s->n_walls > 0 ? s->n_walls : 1));
  p.off_loss = off;
  off = align_up(off + sizeof(float) * (size_t)(p.n_tiles > 0 ? p.n_tiles : 1));
  p.off_seed = off;
  off = align_up(off + sizeof(float) * (size_t)(s->n_rx > 0 ? s->n_rx : 1));
  p.off_grad = off;
  off = align_up(off + sizeof(float) * (size_t)p.ncol * (size_t)(p.n_tiles > 0 ? p.n_tiles : 1));
  // contribution cache: the forward visits the candidates in at most three
  // phases, each split into chunks over the wavefronts, so a wavefront meets
  // at most ceil(C / (nw cchunk)) + 3 chunks
  const int64_t n_cand = count_candidates(s->n_walls, s->max_order);
  const int64_t span = (int64_t)p.nw * p.cchunk;
  const int64_t per_wave = ((n_cand + span - 1) / span + 3) * p.cchunk;
  const int64_t slots = (int64_t)p.n_tiles * p.nw;
  p.box_stride = 6 * (s->max_order + 1);
  const int64_t entry = (int64_t)drt::kWave * sizeof(float) + sizeof(int) + (int64_t)p.box_stride * sizeof(float);
  int64_t cap = per_wave;
  if (slots > 0 && cache_limit > 0) {
    const int64_t fit = (cache_limit - slots * (int64_t)sizeof(int)) / (slots * entry);
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
  p.off_cache_box = off;
  off = align_up(off + sizeof(float) * (size_t)slots * p.cache_cap * p.box_stride);
  p.total = off;
  return p;
}

drt::TraceArgs make_args(const drt_scene* s, const Plan& p, void* ws) {
  drt::TraceArgs A{};
  A.walls = reinterpret_cast<const drt::WallRec*>(static_cast<char*>(ws) + p.off_walls);
  A.boxes = reinterpret_cast<const drt::WallBox*>(static_cast<char*>(ws) + p.off_boxes);
  A.tx = s->tx_dev;
  A.rx = s->rx_dev;
  A.n_walls = s->n_walls;
  A.n_rx = s->n_rx;
  A.grid_nx = s->rx_grid_nx;
  A.n_cand = (int)count_candidates(s->n_walls, s->max_order);
  A.cchunk = p.cchunk;
  A.screen = g_screen;
  A.cut = drt::cut_factor(g_cut != 0, A.n_cand);
  A.alpha = s->alpha;
  A.a2 = s->alpha * drt::kLog2e;
  const bool hard = s->smoothing == DRT_HARD_SIGMOID;
  A.mode = hard ? 1 : 0;
  A.max_order = s->max_order;
  A.band_k = 1.0f + 2.0f * (hard ? drt::kHardBandMargin : drt::kBandMargin) / s->alpha;
  A.cull_c = (hard ? drt::kHardCullMargin : drt::kCullMargin) / s->alpha;
  A.dmin2 = s->d_min * s->d_min;
  if (p.cache_cap > 0) {
    char* w = static_cast<char*>(ws);
    A.cache_c = reinterpret_cast<float*>(w + p.off_cache_c);
    A.cache_idx = reinterpret_cast<int*>(w + p.off_cache_idx);
    A.cache_n = reinterpret_cast<int*>(w + p.off_cache_n);
    A.cache_box = reinterpret_cast<float*>(w + p.off_cache_box);
    A.cache_cap = p.cache_cap;
    A.box_stride = p.box_stride;
  }
  return A;
}

int check_ws(const Plan& p, void* ws, size_t ws_bytes) {
  if (!ws) return fail(DRT_EWORKSPACE, "workspace is NULL");
  if (ws_bytes < p.total)
    return fail(DRT_EWORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, p.total);
  if (reinterpret_cast<uintptr_t>(ws) % 16 != 0) return fail(DRT_EWORKSPACE, "workspace not 16-byte aligned");
  return DRT_OK;
}

int check_loss(int32_t loss_kind, float log_eps) {
  if (loss_kind < DRT_LOSS_NONE || loss_kind > DRT_LOSS_NEG_MIN_POWER)
    return fail(DRT_EINVAL, "loss_kind=%d unknown", loss_kind);
  if (loss_kind == DRT_LOSS_NEG_MEAN_LOG_POWER && (!std::isfinite(log_eps) || !(log_eps > 0.0f)))
    return fail(DRT_EINVAL, "log_eps must be finite and > 0");
  return DRT_OK;
}

// Enqueue: prep walls, forward (power, seed, per-tile loss partials), loss.
int enqueue_forward(const drt_scene* s, const Plan& p, const drt::TraceArgs& A, int32_t loss_kind,
                    float log_eps, float* power, float* loss, float* seed, void* ws, hipStream_t st) {
  char* w = static_cast<char*>(ws);
  hipError_t e = drt::launch_prep_walls(s->walls_dev, s->n_walls, A.cull_c,
                                        reinterpret_cast<drt::WallRec*>(w + p.off_walls),
                                        reinterpret_cast<drt::WallBox*>(w + p.off_boxes), st);
  if (e != hipSuccess) return hip_fail(e, "prep_walls launch");
  float* loss_part = reinterpret_cast<float*>(w + p.off_loss);
  const bool min_loss = loss_kind == DRT_LOSS_NEG_MIN_POWER;
  if (p.n_tiles > 0) {
    e = drt::launch_forward(A, p.n_tiles, p.nw, power, min_loss ? nullptr : seed, loss_part,
                            min_loss ? DRT_LOSS_NONE : loss_kind, log_eps, st);
    if (e != hipSuccess) return hip_fail(e, "forward launch");
  }
  if (min_loss) {
    e = drt::launch_min_seed(power, s->n_rx, loss, seed, st);
    if (e != hipSuccess) return hip_fail(e, "min-loss launch");
    return DRT_OK;
  }
  if (loss_kind != DRT_LOSS_NONE && loss) {
    const double scale = loss_kind == DRT_LOSS_NEG_MEAN_LOG_POWER
                             ? (s->n_rx > 0 ? -1.0 / (double)s->n_rx : 0.0)
                             : 1.0;
    e = drt::launch_reduce_scalar(loss_part, p.n_tiles, scale, loss, st);
    if (e != hipSuccess) return hip_fail(e, "loss reduction launch");
  }
  return DRT_OK;
}

int enqueue_backward(const drt_scene* s, const Plan& p, const drt::TraceArgs& A, const float* gP,
                     float* gtx, float* gwalls, float* grx, int reuse, void* ws, hipStream_t st) {
  char* w = static_cast<char*>(ws);
  float* part = reinterpret_cast<float*>(w + p.off_grad);
  hipError_t e;
  if (p.n_tiles > 0) {
    e = drt::launch_backward(A, p.n_tiles, p.nw, gP, part, grx, reuse, st);
    if (e != hipSuccess) return hip_fail(e, "backward launch");
  }
  e = drt::launch_reduce_cols(part, p.n_tiles, p.ncol, gtx, 2, gwalls, st);
  if (e != hipSuccess) return hip_fail(e, "gradient reduction launch");
  return DRT_OK;
}

int check_forward_backward(const drt_scene* scene, int32_t loss_kind, float log_eps, const float* power_dev,
                           const float* grad_tx_dev, const float* grad_walls_dev) {
  int rc = check_scene(scene);
  if (rc) return rc;
  if ((rc = check_loss(loss_kind, log_eps))) return rc;
  if (loss_kind == DRT_LOSS_NONE) return fail(DRT_EINVAL, "forward_backward needs a loss_kind");
  if (loss_kind == DRT_LOSS_NEG_MIN_POWER && scene->n_rx < 1) return fail(DRT_EINVAL, "min loss needs n_rx >= 1");
  if (scene->n_rx > 0 && !power_dev) return fail(DRT_EINVAL, "power_dev is NULL");
  if (!grad_tx_dev) return fail(DRT_EINVAL, "grad_tx_dev is NULL");
  if (scene->n_walls > 0 && !grad_walls_dev) return fail(DRT_EINVAL, "grad_walls_dev is NULL");
  return DRT_OK;
}

// Forward, seed (kept in the workspace) and adjoint from the recorded contributions.
int enqueue_forward_backward(const drt_scene* scene, const Plan& p, int32_t loss_kind, float log_eps,
                             float* power_dev, float* loss_dev, float* grad_tx_dev, float* grad_walls_dev,
                             float* grad_rx_dev, void* ws, hipStream_t st) {
  const drt::TraceArgs A = make_args(scene, p, ws);
  float* seed = reinterpret_cast<float*>(static_cast<char*>(ws) + p.off_seed);
  int rc = enqueue_forward(scene, p, A, loss_kind, log_eps, power_dev, loss_dev, seed, ws, st);
  if (rc) return rc;
  return enqueue_backward(scene, p, A, seed, grad_tx_dev, grad_walls_dev, grad_rx_dev, 1, ws, st);
}

// Scratch memory of drt_forward_backward_noalloc: a device array that every
// GPU the library runs on holds for the life of the process.  Host code must
// never pass the array's name to a kernel (on the host it is only a stand-in
// for the symbol); it uses the address hipGetSymbolAddress returns for the
// current device, looked up once per device.  Nothing in it needs to start
// at zero: every kernel writes what it later reads within the same call.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_of_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(DRT_EINVAL, "device index %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(DRT_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return DRT_OK;
}

}  // namespace

extern "C" {

// Error reporting shared with the other translation units of the library.
__attribute__((visibility("hidden"))) int drt_internal_fail(int code, const char* msg) {
  g_err = msg ? msg : "";
  return code;
}

__attribute__((visibility("hidden"))) int64_t drt_internal_cache_limit(void) { return g_cache_limit; }
__attribute__((visibility("hidden"))) int drt_internal_screen(void) { return g_screen; }
__attribute__((visibility("hidden"))) int drt_internal_cut(void) { return g_cut; }

int drt_abi_version(void) { return DRT_ABI_VERSION; }

const char* drt_status_string(int status) {
  switch (status) {
    case DRT_OK: return "ok";
    case DRT_EINVAL: return "invalid argument";
    case DRT_EWORKSPACE: return "workspace missing or too small";
    case DRT_ENOTSUP: return "not supported";
    case DRT_EHIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char* drt_last_error(void) { return g_err.c_str(); }

int drt_set_launch_config(int32_t nw, int32_t cchunk) {
  if (!(nw == 0 || nw == 2 || nw == 4 || nw == 8 || nw == 16))
    return fail(DRT_EINVAL, "nw=%d must be 0, 2, 4, 8 or 16", nw);
  if (cchunk < 0) return fail(DRT_EINVAL, "cchunk=%d is negative", cchunk);
  g_nw_override = nw;
  g_cchunk_override = cchunk;
  return DRT_OK;
}

int drt_set_cache_limit(int64_t bytes) {
  if (bytes < 0) return fail(DRT_EINVAL, "cache limit %lld is negative", (long long)bytes);
  g_cache_limit = bytes;
  return DRT_OK;
}

int drt_set_screen(int32_t enabled) {
  if (enabled != 0 && enabled != 1) return fail(DRT_EINVAL, "screen flag %d must be 0 or 1", enabled);
  g_screen = enabled;
  return DRT_OK;
}

int drt_set_cut(int32_t enabled) {
  if (enabled != 0 && enabled != 1) return fail(DRT_EINVAL, "cut flag %d must be 0 or 1", enabled);
  g_cut = enabled;
  return DRT_OK;
}

int drt_num_candidates(int32_t n_walls, int32_t max_order, int64_t* count) {
  if (!count) return fail(DRT_EINVAL, "count is NULL");
  if (n_walls < 0 || n_walls > DRT_MAX_WALLS || max_order < 0 || max_order > DRT_MAX_ORDER)
    return fail(DRT_EINVAL, "n_walls=%d / max_order=%d out of range", n_walls, max_order);
  *count = count_candidates(n_walls, max_order);
  return DRT_OK;
}

int drt_workspace_size(const drt_scene* scene, size_t* bytes) {
  int rc = check_scene(scene);
  if (rc) return rc;
  if (!bytes) return fail(DRT_EINVAL, "bytes is NULL");
  *bytes = make_plan(scene, g_cache_limit).total;
  return DRT_OK;
}

int drt_cache_layout(const drt_scene* scene, int64_t* slots, int64_t* capacity, int64_t* off_idx,
                     int64_t* off_n) {
  int rc = check_scene(scene);
  if (rc) return rc;
  if (!slots || !capacity || !off_idx || !off_n) return fail(DRT_EINVAL, "NULL output pointer");
  const Plan p = make_plan(scene, g_cache_limit);
  *slots = (int64_t)p.n_tiles * p.nw;
  *capacity = p.cache_cap;
  *off_idx = (int64_t)p.off_cache_idx;
  *off_n = (int64_t)p.off_cache_n;
  return DRT_OK;
}

int drt_forward(const drt_scene* scene, int32_t loss_kind, float log_eps, float* power_dev,
                float* loss_dev, float* seed_dev, void* ws_dev, size_t ws_bytes, void* stream) {
  int rc = check_scene(scene);
  if (rc) return rc;
  if ((rc = check_loss(loss_kind, log_eps))) return rc;
  if (scene->n_rx > 0 && !power_dev) return fail(DRT_EINVAL, "power_dev is NULL");
  if (seed_dev && loss_kind == DRT_LOSS_NONE) return fail(DRT_EINVAL, "seed_dev needs a loss_kind");
  if (loss_kind == DRT_LOSS_NEG_MIN_POWER && scene->n_rx < 1) return fail(DRT_EINVAL, "min loss needs n_rx >= 1");
  const Plan p = make_plan(scene, g_cache_limit);
  if ((rc = check_ws(p, ws_dev, ws_bytes))) return rc;
  const drt::TraceArgs A = make_args(scene, p, ws_dev);
  return enqueue_forward(scene, p, A, loss_kind, log_eps, power_dev, loss_dev, seed_dev, ws_dev,
                         static_cast<hipStream_t>(stream));
}

int drt_backward(const drt_scene* scene, const float* grad_power_dev, int32_t flags,
                 float* grad_tx_dev, float* grad_walls_dev, float* grad_rx_dev, void* ws_dev,
                 size_t ws_bytes, void* stream) {
  int rc = check_scene(scene);
  if (rc) return rc;
  if (flags & ~DRT_BWD_REUSE_FORWARD) return fail(DRT_EINVAL, "unknown flags 0x%x", flags);
  if (scene->n_rx > 0 && !grad_power_dev) return fail(DRT_EINVAL, "grad_power_dev is NULL");
  if (!grad_tx_dev) return fail(DRT_EINVAL, "grad_tx_dev is NULL");
  if (scene->n_walls > 0 && !grad_walls_dev) return fail(DRT_EINVAL, "grad_walls_dev is NULL");
  const Plan p = make_plan(scene, g_cache_limit);
  if ((rc = check_ws(p, ws_dev, ws_bytes))) return rc;
  const drt::TraceArgs A = make_args(scene, p, ws_dev);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool reuse = (flags & DRT_BWD_REUSE_FORWARD) != 0;
  if (!reuse) {
    // (with the flag, the wall records and culling boxes the forward wrote
    // into this workspace are still those of this scene)
    char* w = static_cast<char*>(ws_dev);
    hipError_t e = drt::launch_prep_walls(scene->walls_dev, scene->n_walls, A.cull_c,
                                          reinterpret_cast<drt::WallRec*>(w + p.off_walls),
                                          reinterpret_cast<drt::WallBox*>(w + p.off_boxes), st);
    if (e != hipSuccess) return hip_fail(e, "prep_walls launch");
  }
  return enqueue_backward(scene, p, A, grad_power_dev, grad_tx_dev, grad_walls_dev, grad_rx_dev, reuse ? 1 : 0,
                          ws_dev, st);
}

int drt_forward_backward(const drt_scene* scene, int32_t loss_kind, float log_eps, float* power_dev,
                         float* loss_dev, float* grad_tx_dev, float* grad_walls_dev,
                         float* grad_rx_dev, void* ws_dev, size_t ws_bytes, void* stream) {
  int rc = check_forward_backward(scene, loss_kind, log_eps, power_dev, grad_tx_dev, grad_walls_dev);
  if (rc) return rc;
  const Plan p = make_plan(scene, g_cache_limit);
  if ((rc = check_ws(p, ws_dev, ws_bytes))) return rc;
  return enqueue_forward_backward(scene, p, loss_kind, log_eps, power_dev, loss_dev, grad_tx_dev, grad_walls_dev,
                                  grad_rx_dev, ws_dev, static_cast<hipStream_t>(stream));
}

int drt_forward_backward_noalloc(const drt_scene* scene, int32_t loss_kind, float log_eps, float* power_dev,
                                 float* loss_dev, float* grad_tx_dev, float* grad_walls_dev,
                                 float* grad_rx_dev, void* stream) {
  int rc = check_forward_backward(scene, loss_kind, log_eps, power_dev, grad_tx_dev, grad_walls_dev);
  if (rc) return rc;
  // everything but the contribution cache must fit; the cache gets what is left
  const Plan bare = make_plan(scene, 0);
  if (bare.total > kScratchBytes)
    return fail(DRT_EINVAL,
                "scene needs %zu bytes of scratch (n_walls=%d, n_rx=%d); the allocation-free entry point holds "
                "%zu: use drt_forward_backward with a caller workspace",
                bare.total, scene->n_walls, scene->n_rx, kScratchBytes);
  int64_t room = (int64_t)(kScratchBytes - bare.total) - 4 * (int64_t)kAlign;
  if (room > g_cache_limit) room = g_cache_limit;
  Plan p = make_plan(scene, room > 0 ? room : 0);
  if (p.total > kScratchBytes) p = bare;
  void* ws = nullptr;
  if ((rc = scratch_of_current_device(&ws))) return rc;
  return enqueue_forward_backward(scene, p, loss_kind, log_eps, power_dev, loss_dev, grad_tx_dev, grad_walls_dev,
                                  grad_rx_dev, ws, static_cast<hipStream_t>(stream));
}

int drt_forward_fermat(const drt_scene* scene, int32_t max_iter, float conv_eps, int32_t loss_kind,
                       float log_eps, float* power_dev, float* loss_dev, void* ws_dev, size_t ws_bytes,
                       void* stream) {
  int rc = check_scene(scene);
  if (rc) return rc;
  if (scene->max_order > 2) return fail(DRT_ENOTSUP, "Fermat path tracing covers max_order <= 2 (got %d)",
                                        scene->max_order);
  if (max_iter < 1 || max_iter > 64) return fail(DRT_EINVAL, "max_iter=%d outside [1, 64]", max_iter);
  if (!std::isfinite(conv_eps) || !(conv_eps > 0.0f)) return fail(DRT_EINVAL, "conv_eps must be finite and > 0");
  if ((rc = check_loss(loss_kind, log_eps))) return rc;
  if (loss_kind == DRT_LOSS_NEG_MIN_POWER) return fail(DRT_ENOTSUP, "loss_kind NEG_MIN_POWER not offered here");
  if (scene->n_rx > 0 && !power_dev) return fail(DRT_EINVAL, "power_dev is NULL");
  const Plan p = make_plan(scene, g_cache_limit);
  if ((rc = check_ws(p, ws_dev, ws_bytes))) return rc;
  const drt::TraceArgs A = make_args(scene, p, ws_dev);
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws_dev);
  hipError_t e = drt::launch_prep_walls(scene->walls_dev, scene->n_walls, A.cull_c,
                                        reinterpret_cast<drt::WallRec*>(w + p.off_walls),
                                        reinterpret_cast<drt::WallBox*>(w + p.off_boxes), st);
  if (e != hipSuccess) return hip_fail(e, "prep_walls launch");
  float* loss_part = reinterpret_cast<float*>(w + p.off_loss);
  if (p.n_tiles > 0) {
    e = drt::launch_forward_fermat(A, p.n_tiles, p.nw, power_dev, loss_part, loss_kind, log_eps, max_iter,
                                   1.0f / conv_eps, st);
    if (e != hipSuccess) return hip_fail(e, "Fermat forward launch");
  }
  if (loss_kind != DRT_LOSS_NONE && loss_dev) {
    const double scale = loss_kind == DRT_LOSS_NEG_MEAN_LOG_POWER
                             ? (scene->n_rx > 0 ? -1.0 / (double)scene->n_rx : 0.0)
                             : 1.0;
    e = drt::launch_reduce_scalar(loss_part, p.n_tiles, scale, loss_dev, st);
    if (e != hipSuccess) return hip_fail(e, "loss reduction launch");
  }
  return DRT_OK;
}

int drt_adam_tx(float* tx_dev, const float* grad_dev, float* m_dev, float* v_dev, int32_t* step_dev,
                float lr, float b1, float b2, float eps, float lo, float hi, void* stream) {
  return drt_adam_points(1, tx_dev, grad_dev, m_dev, v_dev, step_dev, lr, b1, b2, eps, lo, hi, stream);
}

int drt_alpha_schedule(const int32_t* step_dev, int32_t n_iter, float a_first, float a_last, float* alpha_dev,
                       int32_t n, void* stream) {
  if (!step_dev || !alpha_dev) return fail(DRT_EINVAL, "NULL pointer argument");
  if (n_iter < 2) return fail(DRT_EINVAL, "n_iter=%d must be >= 2", n_iter);
  if (n < 1) return fail(DRT_EINVAL, "n=%d must be >= 1", n);
  if (!(a_first > 0.0f) || !(a_last > 0.0f) || !std::isfinite(a_first) || !std::isfinite(a_last))
    return fail(DRT_EINVAL, "a_first / a_last must be finite and > 0");
  hipError_t e = drt::launch_alpha_schedule(step_dev, n_iter, a_first, a_last, alpha_dev, n,
                                            static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "alpha schedule launch");
  return DRT_OK;
}

int drt_adam_points(int32_t n_points, float* tx_dev, const float* grad_dev, float* m_dev, float* v_dev,
                    int32_t* step_dev, float lr, float b1, float b2, float eps, float lo, float hi, void* stream) {
  if (n_points < 1) return fail(DRT_EINVAL, "n_points=%d must be >= 1", n_points);
  if (!tx_dev || !grad_dev || !m_dev || !v_dev || !step_dev)
    return fail(DRT_EINVAL, "NULL pointer argument");
  if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(DRT_EINVAL, "lr must be finite and > 0");
  if (!(b1 >= 0.0f && b1 < 1.0f) || !(b2 >= 0.0f && b2 < 1.0f))
    return fail(DRT_EINVAL, "betas must lie in [0, 1)");
  if (!(eps > 0.0f) || !std::isfinite(eps)) return fail(DRT_EINVAL, "eps must be finite and > 0");
  if (!(lo <= hi)) return fail(DRT_EINVAL, "lo > hi");
  hipError_t e = drt::launch_adam_points(2 * n_points, tx_dev, grad_dev, m_dev, v_dev, step_dev, lr, b1, b2, eps,
                                         lo, hi, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "adam launch");
  return DRT_OK;
}

}  // extern "C"
