// Internal interface of the surrogate MLP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace drt {

constexpr int kMlpHidden = 5;     // hidden layers of width 256 (128 -> 256, then 256 -> 256 x 4)
constexpr int kMlpWidth = 256;
constexpr int kMlpIn = 128;       // 64 Fourier frequencies -> sin, cos
constexpr int kMlpFreq = 64;

struct MlpLayout {
  int w_off[kMlpHidden];   // flat offset of W_l [in][out]
  int b_off[kMlpHidden];   // flat offset of b_l [out]
  int fan_in[kMlpHidden];
  int bf_off[kMlpHidden];  // offset of layer l in the bf16 weight copies
  int head_w, head_b;      // flat offsets of w5 [256], b5 [1]
  int n_params;
  int n_bf;                // elements per bf16 copy
};

// Fused forward of rows [0, n): features from v [n][4] (v != NULL) or from
// the pairs (tx[(row0 + row) / R], rx[(row0 + row) % R]); hidden layers from
// the bf16 W^T copies wt and the FP32 biases in p; yhat [n] out.
struct FusedArgs {
  const float* v;
  const float* tx;
  const float* rx;
  int R;
  long long row0;
  long long n;
  const float* Bf;
  const __bf16* wt;
  const float* p;
  MlpLayout L;
  float* yhat;
  double* tile_sum;  // [n / fused rows] or NULL: per-tile sums of yhat (yhat may then be NULL)
};

hipError_t launch_mlp_fused(const FusedArgs& a, hipStream_t st);
// Rows per workgroup tile of the fused kernels.
int mlp_fused_rows();
// F[t] = sum of tile_sum[t tiles_per_tx .. + tiles_per_tx) / R.
hipError_t launch_tile_mean(const double* tile_sum, int n_tx, int tiles_per_tx, int R, float* F, hipStream_t st);

// Training pass of rows [0, n) (n % 64 == 0): features of v [n][4], the
// forward through the bf16 W^T copies wt, the head with targets y (squared
// error, output gradient g = 2 (yhat - y) inv_total), and the input
// gradients through the bf16 W copies w.  Out, transposed in blocks of 32
// rows (element (col, row) of an operand with C columns at
// (row / 32) 32 C + 32 col + row % 32): X0T (C = 128), HT [4][ht_stride]
// (H_l, l = 0..3, C = 256), dZT [5][dzt_stride] (dZ_l, C = 256); per tile t
// of mlp_train_rows() rows: hw_part[t][i] = sum_m g_m H_4[m][i]
// and hs_part[t] = (sum_m g_m, sum_m (yhat_m - y_m)^2); yhat [n] if not NULL.
struct TrainArgs {
  const float* v;
  const float* y;
  const int32_t* rows;  // NULL: row m is sample m; else sample rows[m]
  const float* Bf;
  const __bf16* wt;
  const __bf16* w;
  const float* p;
  MlpLayout L;
  float inv_total;
  long long n;
  __bf16* X0T;
  __bf16* HT;
  long long ht_stride;
  __bf16* dZT;
  long long dzt_stride;
  float* hw_part;
  float* hs_part;
  float* yhat;
  int* step;  // not NULL: step[0] += 1, the Adam step count of the update that follows
};

hipError_t launch_mlp_train(const TrainArgs& a, hipStream_t st);
// Rows per tile of the training pass.
int mlp_train_rows();

// The head's part of the gradient sums: g[head_w + i] = sum_t hw_part[t][i],
// g[head_b] = sum_t hs_part[t][0], loss[0] = inv_n sum_t hs_part[t][1]
// (fixed order; hw_part NULL: nothing; loss NULL: no loss).
struct HeadFold {
  const float* hw_part;
  const float* hs_part;
  int tiles;
  double inv_n;
  float* loss;
};

// Adam (torch semantics) applied to each gradient element as its sum is
// formed, at step t = step[0] (counted up by the training pass), with the
// BF16 copies of W and W^T (fragment order) rewritten.  p NULL: no update.
struct AdamArgs {
  float* p;
  float* m;
  float* v;
  const int* step;
  float lr, b1, b2, eps;
  __bf16* wbf;
  __bf16* wtbf;
};

// Weight and bias gradients of the hidden layers from the transposed
// operands X0T, HT [4][ht_stride] and dZT [5][dzt_stride] (blocks of 32 rows
// as written by the training pass):
// partials over slices of slice_rows rows (weights into part, biases -- the
// row sums of dZ_l^T -- into part_b), then the in-order slice sums into g
// (W_l at w_off_l, b_l at b_off_l), the head's sums (HeadFold), and with
// adam.p set the parameter update of every element (AdamArgs).  n and
// slice_rows are multiples of 32, n_slices = ceil(n / slice_rows).
struct DwArgs {
  const __bf16* X0T;
  const __bf16* HT;
  long long ht_stride;
  const __bf16* dZT;
  long long dzt_stride;
  long long n;
  int slice_rows;
  int n_slices;
  MlpLayout L;
  float* part;    // [5][n_slices][256][256]
  float* part_b;  // [5][n_slices][256]
};

hipError_t launch_mlp_dw(const DwArgs& a, float* g, const HeadFold& hf, const AdamArgs& adam, hipStream_t st);
hipError_t launch_segment_mean(const float* yhat, int T, int R, float* F, hipStream_t st);
hipError_t launch_mlp_copies(const float* p, int n, const MlpLayout& L, __bf16* wbf, __bf16* wtbf,
                             hipStream_t st);
hipError_t launch_log_eps(const float* P, long long n, float eps, float* y, hipStream_t st);

}  // namespace drt
