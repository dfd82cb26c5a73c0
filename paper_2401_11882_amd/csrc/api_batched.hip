// C ABI for many scenes in one persistent launch: plans (work list, device
// buffers, launch shape) and the autotuner that picks the launch shape.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/drt.h"
#include "batched.h"

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

int64_t n_candidates(int64_t W, int K) {
  int64_t total = 1, term = 0;
  for (int k = 1; k <= K; ++k) {
    term = (k == 1) ? W : term * (W - 1);
    total += term;
  }
  return total;
}

template <class T>
T* dev_alloc(size_t n, hipError_t& e) {
  void* p = nullptr;
  e = hipMalloc(&p, n * sizeof(T) + 16);
  return static_cast<T*>(p);
}

}  // namespace

struct drt_plan {
  int device = 0;
  int n_scenes = 0;
  int max_order = 0;
  int max_walls = 0;
  int n_cu = 0;
  int64_t sum_walls = 0, sum_rx = 0;
  int64_t max_cand = 0;
  std::vector<int> wall_off, rx_off, grid_nx;
  std::vector<int> items, scene_items;
  std::vector<long long> part_off;
  long long part_total = 0;
  std::string signature;
  drt_plan_config cfg{8, 1, 0, 8};
  int blocks = 0;
  int cache_cap = 0;
  int64_t cache_limit = 32LL << 30;
  // device buffers (owned)
  int *d_wall_off = nullptr, *d_rx_off = nullptr, *d_grid_nx = nullptr, *d_items = nullptr;
  int *d_scene_items = nullptr, *d_counter = nullptr, *d_cache_idx = nullptr;
  long long* d_part_off = nullptr;
  drt::WallRec* d_rec = nullptr;
  drt::WallBox* d_boxes = nullptr;
  float *d_loss_part = nullptr, *d_grad_part = nullptr, *d_cache_c = nullptr, *d_cache_box = nullptr;
  size_t cache_bytes = 0;
};

namespace {

// Largest workgroup LDS footprint the batched kernel is launched with.
constexpr size_t kMaxBatchedLds = 64 * 1024;

void free_plan(drt_plan* p) {
  void* bufs[] = {p->d_wall_off, p->d_rx_off, p->d_grid_nx, p->d_items, p->d_scene_items, p->d_counter,
                  p->d_cache_idx, p->d_part_off, p->d_rec, p->d_boxes, p->d_loss_part, p->d_grad_part,
                  p->d_cache_c, p->d_cache_box};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
}

// Device grid_nx for a tile width: a scene keeps 2D tiles only when its grid
// divides into tw x (64/tw) tiles.
std::vector<int> grid_for_tile(const drt_plan* p, int tw) {
  std::vector<int> g(p->n_scenes, 0);
  for (int s = 0; s < p->n_scenes; ++s) {
    const int nx = p->grid_nx[s];
    const int R = p->rx_off[s + 1] - p->rx_off[s];
    const int th = 64 / tw;
    if (nx > 0 && nx % tw == 0 && R % nx == 0 && (R / nx) % th == 0) g[s] = nx;
  }
  return g;
}

int apply_config(drt_plan* p, const drt_plan_config& c) {
  if (!(c.nw == 4 || c.nw == 8 || c.nw == 16)) return failf(DRT_EINVAL, "nw=%d must be 4, 8 or 16", c.nw);
  if (c.cchunk < 1 || c.cchunk > 64) return failf(DRT_EINVAL, "cchunk=%d outside [1, 64]", c.cchunk);
  if (!(c.tile_w == 8 || c.tile_w == 16 || c.tile_w == 32)) return failf(DRT_EINVAL, "tile_w=%d must be 8, 16 or 32", c.tile_w);
  if (drt::batched_lds_bytes(c.nw, p->max_walls, p->max_order) > kMaxBatchedLds)
    return failf(DRT_EINVAL, "nw=%d needs %zu bytes of LDS for %d walls (limit %zu)", c.nw,
                 drt::batched_lds_bytes(c.nw, p->max_walls, p->max_order), p->max_walls, kMaxBatchedLds);
  const int maxb = drt::batched_max_blocks_per_cu(c.nw, p->max_walls, p->max_order);
  const int bpc = c.blocks_per_cu <= 0 ? maxb : std::min(c.blocks_per_cu, maxb);
  const int blocks = bpc * p->n_cu;
  // contribution cache: one region per wavefront slot of the persistent grid
  // the forward visits the orders 0 and 1 first, then the rest, each part in
  // chunks over the wavefronts: at most one extra chunk per wavefront
  const int64_t per_wave =
      ((p->max_cand + (int64_t)c.nw * c.cchunk - 1) / ((int64_t)c.nw * c.cchunk) + 1) * c.cchunk;
  const int64_t slots = (int64_t)blocks * c.nw;
  const int box_stride = 6 * (p->max_order + 1);
  const int64_t entry = 64 * (int64_t)sizeof(float) + (int64_t)sizeof(int) + (int64_t)box_stride * sizeof(float);
  int64_t cap = per_wave;
  if (p->cache_limit <= 0) cap = 0;
  else cap = std::min<int64_t>(cap, p->cache_limit / (slots * entry));
  const size_t need_c = (size_t)slots * (size_t)cap * 64 * sizeof(float);
  const size_t need_i = (size_t)slots * (size_t)cap * sizeof(int);
  const size_t need_b = (size_t)slots * (size_t)cap * box_stride * sizeof(float);
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return failf(DRT_EHIP, "hipSetDevice: %s", hipGetErrorString(e));
  if (need_c + need_i + need_b > p->cache_bytes) {
    if (p->d_cache_c) (void)hipFree(p->d_cache_c);
    if (p->d_cache_idx) (void)hipFree(p->d_cache_idx);
    if (p->d_cache_box) (void)hipFree(p->d_cache_box);
    p->d_cache_c = nullptr;
    p->d_cache_idx = nullptr;
    p->d_cache_box = nullptr;
    p->cache_bytes = 0;
    if (cap > 0) {
      p->d_cache_c = dev_alloc<float>(need_c / sizeof(float), e);
      if (e != hipSuccess) return failf(DRT_EHIP, "cache allocation (%zu bytes): %s", need_c, hipGetErrorString(e));
      p->d_cache_idx = dev_alloc<int>(need_i / sizeof(int), e);
      if (e != hipSuccess) return failf(DRT_EHIP, "cache index allocation: %s", hipGetErrorString(e));
      p->d_cache_box = dev_alloc<float>(need_b / sizeof(float), e);
      if (e != hipSuccess) return failf(DRT_EHIP, "cache box allocation: %s", hipGetErrorString(e));
      p->cache_bytes = need_c + need_i + need_b;
    }
  }
  const std::vector<int> g = grid_for_tile(p, c.tile_w);
  e = hipMemcpy(p->d_grid_nx, g.data(), sizeof(int) * g.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return failf(DRT_EHIP, "grid upload: %s", hipGetErrorString(e));
  p->cfg = c;
  p->cfg.blocks_per_cu = bpc;
  p->blocks = blocks;
  p->cache_cap = (int)cap;
  return DRT_OK;
}

int check_batch(const drt_plan* p, const drt_batch* b) {
  if (!p) return failf(DRT_EINVAL, "plan is NULL");
  if (!b) return failf(DRT_EINVAL, "batch is NULL");
  if (p->sum_walls > 0 && !b->walls_dev) return failf(DRT_EINVAL, "walls_dev is NULL");
  if (!b->tx_dev || !b->alpha_dev) return failf(DRT_EINVAL, "tx_dev / alpha_dev is NULL");
  if (p->sum_rx > 0 && !b->rx_dev) return failf(DRT_EINVAL, "rx_dev is NULL");
  if (!std::isfinite(b->d_min) || !(b->d_min > 0.0f)) return failf(DRT_EINVAL, "d_min must be finite and > 0");
  if (b->smoothing != DRT_SIGMOID && b->smoothing != DRT_HARD_SIGMOID)
    return failf(DRT_ENOTSUP, "smoothing=%d not supported", b->smoothing);
  return DRT_OK;
}

drt::BatchArgs make_args(const drt_plan* p, const drt_batch* b, int loss_kind, float log_eps, float* power) {
  drt::BatchArgs B{};
  B.walls = p->d_rec;
  B.boxes = p->d_boxes;
  B.wall_off = p->d_wall_off;
  B.rx_off = p->d_rx_off;
  B.grid_nx = p->d_grid_nx;
  B.rx = b->rx_dev;
  B.tx = b->tx_dev;
  B.alpha = b->alpha_dev;
  B.items = p->d_items;
  B.n_items = (int)(p->items.size() / 2);
  B.counter = p->d_counter;
  B.scene_items = p->d_scene_items;
  B.part_off = p->d_part_off;
  B.max_order = p->max_order;
  B.max_walls = p->max_walls;
  B.dmin2 = b->d_min * b->d_min;
  B.log_eps = log_eps;
  B.loss_kind = loss_kind;
  B.power = power;
  B.loss_part = p->d_loss_part;
  B.grad_part = p->d_grad_part;
  B.cache_c = p->cache_cap > 0 ? p->d_cache_c : nullptr;
  B.cache_idx = p->cache_cap > 0 ? p->d_cache_idx : nullptr;
  B.cache_box = p->cache_cap > 0 ? p->d_cache_box : nullptr;
  B.box_stride = 6 * (p->max_order + 1);
  B.cache_cap = p->cache_cap;
  B.cchunk = p->cfg.cchunk;
  B.screen = drt_internal_screen();
  B.cut = drt_internal_cut() ? 1.0f : 0.0f;
  B.mode = b->smoothing == DRT_HARD_SIGMOID ? 1 : 0;
  B.box_lds = drt::batched_box_lds(p->cfg.nw, p->max_walls, p->max_order) ? 1 : 0;
  B.tile_w = p->cfg.tile_w;
  return B;
}

int enqueue(drt_plan* p, const drt_batch* b, int loss_kind, float log_eps, float* power, float* loss,
            float* gtx, float* gw, hipStream_t st) {
  const drt::BatchArgs B = make_args(p, b, loss_kind, log_eps, power);
  hipError_t e = drt::launch_batched(B, p->cfg.nw, p->blocks, b->walls_dev, b->alpha_dev, p->n_scenes, loss,
                                     gtx, gw, st);
  if (e != hipSuccess) return failf(DRT_EHIP, "batched launch: %s", hipGetErrorString(e));
  return DRT_OK;
}

int check_outputs(const drt_plan* p, int loss_kind, float log_eps, float* power, float* gtx, float* gw) {
  if (loss_kind < DRT_LOSS_NONE || loss_kind > DRT_LOSS_NEG_MIN_POWER)
    return failf(DRT_EINVAL, "loss_kind=%d unknown", loss_kind);
  if (loss_kind == DRT_LOSS_NEG_MIN_POWER)
    for (int s = 0; s < p->n_scenes; ++s) {
      const int R = p->rx_off[s + 1] - p->rx_off[s];
      if (R < 1 || R > 64) return failf(DRT_EINVAL, "min loss needs 1..64 receivers per scene (scene %d has %d)", s, R);
    }
  if (loss_kind == DRT_LOSS_NONE) {
    if (p->sum_rx > 0 && !power) return failf(DRT_EINVAL, "power_dev is NULL");
    return DRT_OK;
  }
  if (loss_kind == DRT_LOSS_NEG_MEAN_LOG_POWER && (!std::isfinite(log_eps) || !(log_eps > 0.0f)))
    return failf(DRT_EINVAL, "log_eps must be finite and > 0");
  if (p->sum_rx > 0 && !power) return failf(DRT_EINVAL, "power_dev is NULL");
  if (!gtx) return failf(DRT_EINVAL, "grad_tx_dev is NULL");
  if (p->sum_walls > 0 && !gw) return failf(DRT_EINVAL, "grad_walls_dev is NULL");
  return DRT_OK;
}

bool read_tuned(const char* path, const std::string& sig, drt_plan_config* out) {
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    std::istringstream ss(line);
    std::string s;
    drt_plan_config c{};
    double ms = 0.0;
    if (ss >> s >> c.nw >> c.cchunk >> c.blocks_per_cu >> c.tile_w >> ms && s == sig) {
      *out = c;  // the last matching line wins
      found = true;
    }
  }
  return found;
}

}  // namespace

extern "C" {

int drt_plan_create(const drt_batch_shape* shape, const char* tune_cache_path, drt_plan** out) {
  if (!out) return failf(DRT_EINVAL, "out is NULL");
  *out = nullptr;
  if (!shape) return failf(DRT_EINVAL, "shape is NULL");
  const int S = shape->n_scenes;
  if (S <= 0) return failf(DRT_EINVAL, "n_scenes=%d must be > 0", S);
  if (!shape->n_walls || !shape->n_rx) return failf(DRT_EINVAL, "n_walls / n_rx arrays are NULL");
  if (shape->max_order < 0 || shape->max_order > DRT_MAX_ORDER)
    return failf(DRT_EINVAL, "max_order=%d outside [0, %d]", shape->max_order, DRT_MAX_ORDER);
  drt_plan* p = new (std::nothrow) drt_plan();
  if (!p) return failf(DRT_EINVAL, "out of host memory");
  p->n_scenes = S;
  p->max_order = shape->max_order;
  p->cache_limit = drt_internal_cache_limit();
  p->wall_off.assign(S + 1, 0);
  p->rx_off.assign(S + 1, 0);
  p->grid_nx.assign(S, 0);
  uint64_t h = 1469598103934665603ULL;  // FNV-1a over the per-scene shape
  auto mix = [&h](int64_t v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (uint64_t)((v >> (8 * i)) & 0xff);
      h *= 1099511628211ULL;
    }
  };
  for (int s = 0; s < S; ++s) {
    const int W = shape->n_walls[s], R = shape->n_rx[s];
    const int nx = shape->rx_grid_nx ? shape->rx_grid_nx[s] : 0;
    if (W < 0 || W > DRT_MAX_WALLS || R < 0 || nx < 0) {
      delete p;
      return failf(DRT_EINVAL, "scene %d: n_walls=%d n_rx=%d grid_nx=%d out of range", s, W, R, nx);
    }
    if (n_candidates(W, shape->max_order) > 0x7fffffffLL) {
      delete p;
      return failf(DRT_EINVAL, "scene %d: candidate count exceeds 2^31-1", s);
    }
    p->wall_off[s + 1] = p->wall_off[s] + W;
    p->rx_off[s + 1] = p->rx_off[s] + R;
    p->grid_nx[s] = nx;
    p->max_walls = std::max(p->max_walls, W);
    p->max_cand = std::max<int64_t>(p->max_cand, n_candidates(W, shape->max_order));
    mix(W);
    mix(R);
    mix(nx);
  }
  p->sum_walls = p->wall_off[S];
  p->sum_rx = p->rx_off[S];
  if (p->sum_walls > 0x7fffffffLL || p->sum_rx > 0x3fffffffLL) {
    delete p;
    return failf(DRT_EINVAL, "batch too large");
  }
  // work items, longest first (cost = candidates of the scene), scene-contiguous
  std::vector<int> order(S);
  for (int s = 0; s < S; ++s) order[s] = s;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const int64_t ca = n_candidates(p->wall_off[a + 1] - p->wall_off[a], p->max_order);
    const int64_t cb = n_candidates(p->wall_off[b + 1] - p->wall_off[b], p->max_order);
    return ca > cb;
  });
  p->scene_items.assign(2 * S, 0);
  for (int s : order) {
    const int R = p->rx_off[s + 1] - p->rx_off[s];
    const int W = p->wall_off[s + 1] - p->wall_off[s];
    const int tiles = (R + 63) / 64;
    p->scene_items[2 * s] = (int)(p->items.size() / 2);
    p->scene_items[2 * s + 1] = tiles;
    for (int t = 0; t < tiles; ++t) {
      p->items.push_back(s);
      p->items.push_back(t);
      p->part_off.push_back(p->part_total);
      p->part_total += 2 + 4 * W;
    }
  }
  hipError_t e = hipGetDevice(&p->device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, p->device);
  hipDeviceProp_t prop;
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, p->device);
  if (e != hipSuccess) {
    delete p;
    return failf(DRT_EHIP, "device query: %s", hipGetErrorString(e));
  }
  {
    std::ostringstream sig;
    sig << prop.gcnArchName << "-cu" << p->n_cu << "-S" << S << "-W" << p->sum_walls << "-R" << p->sum_rx << "-K"
        << p->max_order << "-h" << std::hex << h;
    p->signature = sig.str();
    for (char& c : p->signature)
      if (c == ' ' || c == ':') c = '_';
  }
  const size_t n_items = p->items.size() / 2;
  p->d_wall_off = dev_alloc<int>(S + 1, e);
  if (e == hipSuccess) p->d_rx_off = dev_alloc<int>(S + 1, e);
  if (e == hipSuccess) p->d_grid_nx = dev_alloc<int>(S, e);
  if (e == hipSuccess) p->d_items = dev_alloc<int>(std::max<size_t>(2 * n_items, 2), e);
  if (e == hipSuccess) p->d_scene_items = dev_alloc<int>(2 * S, e);
  if (e == hipSuccess) p->d_counter = dev_alloc<int>(1, e);
  if (e == hipSuccess) p->d_part_off = dev_alloc<long long>(std::max<size_t>(n_items, 1), e);
  if (e == hipSuccess) p->d_rec = dev_alloc<drt::WallRec>(std::max<int64_t>(p->sum_walls, 1), e);
  if (e == hipSuccess) p->d_boxes = dev_alloc<drt::WallBox>(std::max<int64_t>(p->sum_walls, 1), e);
  if (e == hipSuccess) p->d_loss_part = dev_alloc<float>(std::max<size_t>(n_items, 1), e);
  if (e == hipSuccess) p->d_grad_part = dev_alloc<float>(std::max<long long>(p->part_total, 1), e);
  if (e == hipSuccess)
    e = hipMemcpy(p->d_wall_off, p->wall_off.data(), sizeof(int) * (S + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d_rx_off, p->rx_off.data(), sizeof(int) * (S + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess && n_items)
    e = hipMemcpy(p->d_items, p->items.data(), sizeof(int) * 2 * n_items, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(p->d_scene_items, p->scene_items.data(), sizeof(int) * 2 * S, hipMemcpyHostToDevice);
  if (e == hipSuccess && n_items)
    e = hipMemcpy(p->d_part_off, p->part_off.data(), sizeof(long long) * n_items, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    free_plan(p);
    delete p;
    return failf(DRT_EHIP, "plan buffers: %s", hipGetErrorString(e));
  }
  // default shape: 8 wavefronts, fewer when the wall accumulators do not fit
  drt_plan_config c{8, 1, 0, 8};
  while (c.nw > 4 && drt::batched_lds_bytes(c.nw, p->max_walls, p->max_order) > kMaxBatchedLds) c.nw >>= 1;
  read_tuned(tune_cache_path, p->signature, &c);
  int rc = apply_config(p, c);
  if (rc != DRT_OK) {
    free_plan(p);
    delete p;
    return rc;
  }
  *out = p;
  return DRT_OK;
}

int drt_plan_destroy(drt_plan* plan) {
  if (!plan) return DRT_OK;
  (void)hipSetDevice(plan->device);
  (void)hipDeviceSynchronize();
  free_plan(plan);
  delete plan;
  return DRT_OK;
}

int drt_plan_get_config(const drt_plan* plan, drt_plan_config* cfg) {
  if (!plan || !cfg) return failf(DRT_EINVAL, "NULL argument");
  *cfg = plan->cfg;
  return DRT_OK;
}

int drt_plan_set_config(drt_plan* plan, const drt_plan_config* cfg) {
  if (!plan || !cfg) return failf(DRT_EINVAL, "NULL argument");
  return apply_config(plan, *cfg);
}

int drt_plan_info(const drt_plan* plan, int64_t* n_items, int64_t* path_evals, int32_t* cache_cap) {
  if (!plan) return failf(DRT_EINVAL, "plan is NULL");
  if (n_items) *n_items = (int64_t)(plan->items.size() / 2);
  if (path_evals) {
    int64_t t = 0;
    for (int s = 0; s < plan->n_scenes; ++s)
      t += (int64_t)(plan->rx_off[s + 1] - plan->rx_off[s]) *
           n_candidates(plan->wall_off[s + 1] - plan->wall_off[s], plan->max_order);
    *path_evals = t;
  }
  if (cache_cap) *cache_cap = plan->cache_cap;
  return DRT_OK;
}

int drt_batched_forward_backward(drt_plan* plan, const drt_batch* batch, int32_t loss_kind, float log_eps,
                                 float* power_dev, float* loss_dev, float* grad_tx_dev, float* grad_walls_dev,
                                 void* stream) {
  int rc = check_batch(plan, batch);
  if (rc) return rc;
  if ((rc = check_outputs(plan, loss_kind, log_eps, power_dev, grad_tx_dev, grad_walls_dev))) return rc;
  return enqueue(plan, batch, loss_kind, log_eps, power_dev, loss_dev, grad_tx_dev, grad_walls_dev,
                 static_cast<hipStream_t>(stream));
}

int drt_batched_autotune(drt_plan* plan, const drt_batch* batch, int32_t loss_kind, float log_eps,
                         float* power_dev, float* loss_dev, float* grad_tx_dev, float* grad_walls_dev,
                         const char* cache_path, void* stream) {
  int rc = check_batch(plan, batch);
  if (rc) return rc;
  if ((rc = check_outputs(plan, loss_kind, log_eps, power_dev, grad_tx_dev, grad_walls_dev))) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return failf(DRT_EHIP, "event creation failed");
  const drt_plan_config start = plan->cfg;
  drt_plan_config best = start;
  float best_ms = 1e30f;
  int run_rc = DRT_OK;
  const int nws[] = {4, 8, 16};
  const int chunks[] = {1, 4};
  const int tiles[] = {8, 16};
  for (int nw : nws)
    for (int cc : chunks)
      for (int tw : tiles) {
        const int maxb = drt::batched_max_blocks_per_cu(nw, plan->max_walls, plan->max_order);
        // powers of two below the resident maximum, and the maximum itself
        for (int bpc = 1; bpc <= maxb; bpc = (bpc < maxb && 2 * bpc > maxb) ? maxb : 2 * bpc) {
          drt_plan_config c{nw, cc, bpc, tw};
          if (run_rc != DRT_OK || apply_config(plan, c) != DRT_OK) continue;
          float ms = 1e30f;
          for (int rep = 0; rep < 3; ++rep) {
            hipEventRecord(e0, st);
            run_rc = enqueue(plan, batch, loss_kind, log_eps, power_dev, loss_dev, grad_tx_dev, grad_walls_dev, st);
            hipEventRecord(e1, st);
            if (run_rc == DRT_OK && hipEventSynchronize(e1) != hipSuccess)
              run_rc = failf(DRT_EHIP, "autotune run failed");
            if (run_rc != DRT_OK) break;
            float t = 0.0f;
            hipEventElapsedTime(&t, e0, e1);
            if (rep > 0) ms = std::min(ms, t);  // first run warms up
          }
          if (run_rc != DRT_OK) break;
          if (ms < best_ms) {
            best_ms = ms;
            best = plan->cfg;
          }
        }
      }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (run_rc != DRT_OK) {
    apply_config(plan, start);
    return run_rc;
  }
  if ((rc = apply_config(plan, best)) != DRT_OK) return rc;
  if (cache_path) {
    FILE* f = fopen(cache_path, "a");
    if (f) {
      fprintf(f, "%s %d %d %d %d %.4f\n", plan->signature.c_str(), best.nw, best.cchunk, best.blocks_per_cu,
              best.tile_w, best_ms);
      fclose(f);
    }
  }
  return DRT_OK;
}

}  // extern "C"
