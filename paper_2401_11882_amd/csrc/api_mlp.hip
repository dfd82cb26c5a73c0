// C ABI of the learned surrogate: handle with device buffers, training step
// (forward, MSE, backward, Adam), gradients, inference and tx scan.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "../../include/drt.h"
#include "mlp.h"

extern "C" __attribute__((visibility("hidden"))) int drt_internal_fail(int code, const char* msg);

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

drt::MlpLayout make_layout() {
  drt::MlpLayout L{};
  int off = 0, boff = 0;
  for (int l = 0; l < drt::kMlpHidden; ++l) {
    L.fan_in[l] = l == 0 ? drt::kMlpIn : drt::kMlpWidth;
    L.w_off[l] = off;
    off += L.fan_in[l] * drt::kMlpWidth;
    L.b_off[l] = off;
    off += drt::kMlpWidth;
    L.bf_off[l] = boff;
    boff += L.fan_in[l] * drt::kMlpWidth;
  }
  L.head_w = off;
  off += drt::kMlpWidth;
  L.head_b = off;
  off += 1;
  L.n_params = off;
  L.n_bf = boff;
  return L;
}

}  // namespace

// Tiles of the fused forward per scan launch (the tile-sum buffer's size).
constexpr int kMaxTiles = 1 << 20;

struct drt_mlp {
  int device = 0;
  int max_batch = 0;
  int max_slices = 0;
  drt::MlpLayout L{};
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr, *Bf = nullptr;
  int* step = nullptr;
  __bf16 *wbf = nullptr, *wtbf = nullptr;
  // transposed copies for the weight gradients: X0^T [128][max_batch],
  // H_l^T [256][max_batch] (l = 0..3), dZ_l^T [256][max_batch] (l = 0..4)
  __bf16 *X0T = nullptr, *HT = nullptr, *dZT = nullptr;
  float *yhat = nullptr, *dw_part = nullptr;
  float *hw_part = nullptr, *hs_part = nullptr;  // per 64-row tile: head-weight gradient [256], (sum g, sum d^2)
  double* tile_sum = nullptr;  // [kMaxTiles] per-tile yhat sums of the scan
  float* db_part = nullptr;    // [5][max_slices][256] bias-gradient partials
};

namespace {

void free_mlp(drt_mlp* h) {
  void* bufs[] = {h->p, h->g, h->m, h->v, h->Bf, h->step, h->wbf, h->wtbf, h->X0T, h->HT,
                  h->dZT, h->yhat, h->dw_part, h->hw_part, h->hs_part, h->tile_sum, h->db_part};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
}

#define HIPCHK(expr, what)                                                            \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) return failf(DRT_EHIP, "%s: %s", what, hipGetErrorString(e_)); \
  } while (0)

drt::FusedArgs fused_args(drt_mlp* h, long long n) {
  drt::FusedArgs a{};
  a.R = 1;
  a.n = n;
  a.Bf = h->Bf;
  a.wt = h->wtbf;
  a.p = h->p;
  a.L = h->L;
  a.yhat = h->yhat;
  return a;
}

// Adam arguments of a training step at learning rate lr (torch defaults
// for the rest).
drt::AdamArgs adam_args(drt_mlp* h, float lr) {
  return drt::AdamArgs{h->p, h->m, h->v, h->step, lr, 0.9f, 0.999f, 1e-8f, h->wbf, h->wtbf};
}

// Forward + MSE + backward on rows [0, n) of v/y; gradients into h->g, loss
// (mean squared error over n) into loss_dev; with adam.p set, the Adam step
// count is advanced and every parameter updated as its gradient is formed.
int enqueue_grads(drt_mlp* h, const float* v, const float* y, const int32_t* rows, int n, float* loss_dev,
                  const drt::AdamArgs& adam, hipStream_t st) {
  const drt::MlpLayout& L = h->L;
  const int W = drt::kMlpWidth;
  const long long ldt = h->max_batch;
  // forward, head and input gradients per 64-row tile in one kernel: the
  // transposed operands of the weight gradients and the head's partial sums
  drt::TrainArgs ta{};
  ta.v = v;
  ta.y = y;
  ta.rows = rows;
  ta.Bf = h->Bf;
  ta.wt = h->wtbf;
  ta.w = h->wbf;
  ta.p = h->p;
  ta.L = L;
  ta.inv_total = 1.0f / (float)n;
  ta.n = n;
  ta.X0T = h->X0T;
  ta.HT = h->HT;
  ta.ht_stride = ldt * W;
  ta.dZT = h->dZT;
  ta.dzt_stride = ldt * W;
  ta.hw_part = h->hw_part;
  ta.hs_part = h->hs_part;
  ta.step = adam.p ? h->step : nullptr;
  HIPCHK(drt::launch_mlp_train(ta, st), "training pass");
  // weight and bias gradients of every hidden layer: slices of at least
  // kSliceRows rows, at most max_slices of them; then every sum, the head's
  // and the loss included, each followed by its parameter's update
  constexpr int kSliceRows = 512;
  drt::DwArgs dw{};
  dw.X0T = h->X0T;
  dw.HT = h->HT;
  dw.ht_stride = ldt * W;
  dw.dZT = h->dZT;
  dw.dzt_stride = ldt * W;
  dw.n = n;
  dw.slice_rows = std::max(kSliceRows, ((n + h->max_slices - 1) / h->max_slices + 31) / 32 * 32);
  dw.n_slices = (n + dw.slice_rows - 1) / dw.slice_rows;
  dw.L = L;
  dw.part = h->dw_part;
  dw.part_b = h->db_part;
  drt::HeadFold hf{h->hw_part, h->hs_part, n / drt::mlp_train_rows(), 1.0 / (double)n, loss_dev};
  HIPCHK(drt::launch_mlp_dw(dw, h->g, hf, adam, st), "weight gradients");
  return DRT_OK;
}

int check_rows(const drt_mlp* h, int64_t n) {
  if (!h) return failf(DRT_EINVAL, "mlp is NULL");
  if (n <= 0 || n > h->max_batch || n % 64 != 0)
    return failf(DRT_EINVAL, "rows=%lld must be a positive multiple of 64 and <= max_batch=%d", (long long)n,
                 h->max_batch);
  return DRT_OK;
}

}  // namespace

extern "C" {

int drt_mlp_num_params(int64_t* n) {
  if (!n) return failf(DRT_EINVAL, "n is NULL");
  *n = make_layout().n_params;
  return DRT_OK;
}

int drt_mlp_create(const float* fourier_B_host, const float* params_host, int32_t max_batch, drt_mlp** out) {
  if (!out) return failf(DRT_EINVAL, "out is NULL");
  *out = nullptr;
  if (!fourier_B_host || !params_host) return failf(DRT_EINVAL, "NULL host array");
  if (max_batch <= 0 || max_batch % 64 != 0 || max_batch > (1 << 24))
    return failf(DRT_EINVAL, "max_batch=%d must be a positive multiple of 64 up to 2^24", max_batch);
  drt_mlp* h = new (std::nothrow) drt_mlp();
  if (!h) return failf(DRT_EINVAL, "out of host memory");
  h->L = make_layout();
  h->max_batch = max_batch;
  h->max_slices = 32;
  const size_t P = h->L.n_params, nb = (size_t)max_batch, W = drt::kMlpWidth;
  hipError_t e = hipGetDevice(&h->device);
  auto alloc = [&e](void** ptr, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(ptr, bytes);
  };
  alloc((void**)&h->p, P * 4);
  alloc((void**)&h->g, P * 4);
  alloc((void**)&h->m, P * 4);
  alloc((void**)&h->v, P * 4);
  alloc((void**)&h->Bf, drt::kMlpFreq * 4 * 4);
  alloc((void**)&h->step, 16);
  alloc((void**)&h->wbf, (size_t)h->L.n_bf * 2);
  alloc((void**)&h->wtbf, (size_t)h->L.n_bf * 2);
  alloc((void**)&h->X0T, nb * drt::kMlpIn * 2);
  alloc((void**)&h->HT, nb * W * 2 * (drt::kMlpHidden - 1));
  alloc((void**)&h->dZT, nb * W * 2 * drt::kMlpHidden);
  alloc((void**)&h->yhat, nb * 4);
  alloc((void**)&h->dw_part, (size_t)drt::kMlpHidden * h->max_slices * W * W * 4);
  alloc((void**)&h->hw_part, nb / drt::mlp_train_rows() * W * 4);
  alloc((void**)&h->hs_part, nb / drt::mlp_train_rows() * 2 * 4);
  alloc((void**)&h->tile_sum, (size_t)kMaxTiles * sizeof(double));
  alloc((void**)&h->db_part, (size_t)drt::kMlpHidden * h->max_slices * W * 4);
  if (e == hipSuccess) e = hipMemcpy(h->p, params_host, P * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(h->Bf, fourier_B_host, drt::kMlpFreq * 4 * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(h->m, 0, P * 4);
  if (e == hipSuccess) e = hipMemset(h->v, 0, P * 4);
  if (e == hipSuccess) e = hipMemset(h->g, 0, P * 4);
  if (e == hipSuccess) e = hipMemset(h->step, 0, 16);
  if (e == hipSuccess) e = drt::launch_mlp_copies(h->p, h->L.n_params, h->L, h->wbf, h->wtbf, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_mlp(h);
    delete h;
    return failf(DRT_EHIP, "mlp buffers: %s", hipGetErrorString(e));
  }
  *out = h;
  return DRT_OK;
}

int drt_mlp_destroy(drt_mlp* mlp) {
  if (!mlp) return DRT_OK;
  (void)hipSetDevice(mlp->device);
  (void)hipDeviceSynchronize();
  free_mlp(mlp);
  delete mlp;
  return DRT_OK;
}

int drt_mlp_get_params(const drt_mlp* mlp, float* params_host) {
  if (!mlp || !params_host) return failf(DRT_EINVAL, "NULL argument");
  hipError_t e = hipMemcpy(params_host, mlp->p, (size_t)mlp->L.n_params * 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return failf(DRT_EHIP, "download: %s", hipGetErrorString(e));
  return DRT_OK;
}

int drt_mlp_set_params(drt_mlp* mlp, const float* params_host) {
  if (!mlp || !params_host) return failf(DRT_EINVAL, "NULL argument");
  hipError_t e = hipMemcpy(mlp->p, params_host, (size_t)mlp->L.n_params * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = drt::launch_mlp_copies(mlp->p, mlp->L.n_params, mlp->L, mlp->wbf, mlp->wtbf, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return failf(DRT_EHIP, "upload: %s", hipGetErrorString(e));
  return DRT_OK;
}

int drt_mlp_grads(drt_mlp* mlp, const float* v_dev, const float* y_dev, int64_t n, float* grads_dev,
                  float* loss_dev, void* stream) {
  int rc = check_rows(mlp, n);
  if (rc) return rc;
  if (!v_dev || !y_dev) return failf(DRT_EINVAL, "v_dev / y_dev is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = enqueue_grads(mlp, v_dev, y_dev, nullptr, (int)n, loss_dev, drt::AdamArgs{}, st))) return rc;
  if (grads_dev) HIPCHK(hipMemcpyAsync(grads_dev, mlp->g, (size_t)mlp->L.n_params * 4, hipMemcpyDeviceToDevice, st),
                        "grad copy");
  return DRT_OK;
}

int drt_mlp_train_step(drt_mlp* mlp, const float* v_dev, const float* y_dev, int64_t n, float lr,
                       float* loss_dev, void* stream) {
  int rc = check_rows(mlp, n);
  if (rc) return rc;
  if (!v_dev || !y_dev) return failf(DRT_EINVAL, "v_dev / y_dev is NULL");
  if (!(lr > 0.0f) || !std::isfinite(lr)) return failf(DRT_EINVAL, "lr must be finite and > 0");
  hipStream_t st = static_cast<hipStream_t>(stream);
  return enqueue_grads(mlp, v_dev, y_dev, nullptr, (int)n, loss_dev, adam_args(mlp, lr), st);
}

int drt_mlp_train_step_rows(drt_mlp* mlp, const float* v_dev, const float* y_dev, const int32_t* rows_dev,
                            int64_t n, float lr, float* loss_dev, void* stream) {
  int rc = check_rows(mlp, n);
  if (rc) return rc;
  if (!v_dev || !y_dev || !rows_dev) return failf(DRT_EINVAL, "v_dev / y_dev / rows_dev is NULL");
  if (!(lr > 0.0f) || !std::isfinite(lr)) return failf(DRT_EINVAL, "lr must be finite and > 0");
  hipStream_t st = static_cast<hipStream_t>(stream);
  return enqueue_grads(mlp, v_dev, y_dev, rows_dev, (int)n, loss_dev, adam_args(mlp, lr), st);
}

int drt_mlp_forward(drt_mlp* mlp, const float* v_dev, int64_t n, float* yhat_dev, void* stream) {
  if (!mlp) return failf(DRT_EINVAL, "mlp is NULL");
  if (n < 0) return failf(DRT_EINVAL, "n is negative");
  if (n > 0 && (!v_dev || !yhat_dev)) return failf(DRT_EINVAL, "v_dev / yhat_dev is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  // one fused launch over all rows: the activations never leave the workgroup
  drt::FusedArgs fa = fused_args(mlp, n);
  fa.v = v_dev;
  fa.yhat = yhat_dev;
  HIPCHK(drt::launch_mlp_fused(fa, st), "fused forward");
  return DRT_OK;
}

int drt_mlp_scan(drt_mlp* mlp, const float* tx_dev, int32_t n_tx, const float* rx_dev, int32_t n_rx,
                 float* F_dev, void* stream) {
  if (!mlp) return failf(DRT_EINVAL, "mlp is NULL");
  if (n_tx < 0 || n_rx <= 0 || n_rx > mlp->max_batch)
    return failf(DRT_EINVAL, "n_tx=%d n_rx=%d (need 0 < n_rx <= max_batch=%d)", n_tx, n_rx, mlp->max_batch);
  if (n_tx > 0 && (!tx_dev || !rx_dev || !F_dev)) return failf(DRT_EINVAL, "NULL device array");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int tile = drt::mlp_fused_rows();
  if (n_rx % tile == 0) {
    // whole tiles per transmitter: the fused forward sums each tile's yhat and
    // the means follow from the tile sums, kMaxTiles tiles per launch
    const int tiles_per_tx = n_rx / tile;
    const int per = std::max(1, kMaxTiles / tiles_per_tx);
    for (int t0 = 0; t0 < n_tx; t0 += per) {
      const int nt = std::min(per, n_tx - t0);
      drt::FusedArgs fa = fused_args(mlp, (long long)nt * n_rx);
      fa.yhat = nullptr;
      fa.tile_sum = mlp->tile_sum;
      fa.tx = tx_dev;
      fa.rx = rx_dev;
      fa.R = n_rx;
      fa.row0 = (long long)t0 * n_rx;
      HIPCHK(drt::launch_mlp_fused(fa, st), "fused forward");
      HIPCHK(drt::launch_tile_mean(mlp->tile_sum, nt, tiles_per_tx, n_rx, F_dev + t0, st), "tile means");
    }
    return DRT_OK;
  }
  const int per = mlp->max_batch / n_rx;  // transmitters per chunk
  for (int t0 = 0; t0 < n_tx; t0 += per) {
    const int nt = std::min(per, n_tx - t0);
    const int rows = nt * n_rx;
    drt::FusedArgs fa = fused_args(mlp, rows);
    fa.tx = tx_dev;
    fa.rx = rx_dev;
    fa.R = n_rx;
    fa.row0 = (long long)t0 * n_rx;
    HIPCHK(drt::launch_mlp_fused(fa, st), "fused forward");
    HIPCHK(drt::launch_segment_mean(mlp->yhat, nt, n_rx, F_dev + t0, st), "segment mean");
  }
  return DRT_OK;
}

int drt_log_targets(const float* power_dev, int64_t n, float eps, float* y_dev, void* stream) {
  if (n < 0) return failf(DRT_EINVAL, "n is negative");
  if (n > 0 && (!power_dev || !y_dev)) return failf(DRT_EINVAL, "NULL device array");
  if (!(eps > 0.0f) || !std::isfinite(eps)) return failf(DRT_EINVAL, "eps must be finite and > 0");
  if (n == 0) return DRT_OK;
  HIPCHK(drt::launch_log_eps(power_dev, n, eps, y_dev, static_cast<hipStream_t>(stream)), "log targets");
  return DRT_OK;
}

}  // extern "C"
