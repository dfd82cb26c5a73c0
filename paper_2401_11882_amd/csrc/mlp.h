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
// the bf16 W^T copies wt and the FP32 biases in p; yhat [n] out; optional
// X0 [n][128] and H [5][h_stride] (layer l at H + l h_stride, [n][256]) out,
// and the transposed inputs of the weight gradients, X0T [128][ld_t] and
// HT [4][ht_stride] (H_l^T [256][ld_t] for l = 0..3; ld_t % 8 == 0).
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
  __bf16* X0;
  __bf16* H;
  long long h_stride;
  __bf16* X0T;
  __bf16* HT;
  long long ht_stride;
  long long ld_t;
  double* tile_sum;  // [n / fused rows] or NULL: per-tile sums of yhat (yhat may then be NULL)
};

hipError_t launch_mlp_fused(const FusedArgs& a, hipStream_t st);
// Rows per workgroup tile of the fused kernels.
int mlp_fused_rows();
// F[t] = sum of tile_sum[t tiles_per_tx .. + tiles_per_tx) / R.
hipError_t launch_tile_mean(const double* tile_sum, int n_tx, int tiles_per_tx, int R, float* F, hipStream_t st);

// Input gradients of hidden layers 4..1 from dz4 [n][256] (the head's
// gradient), masks H [5][h_stride] ([n][256] per layer), weights w (bf16
// W [in][out] copies); every dZ_l stored transposed at dZT + l dzt_stride
// ([256][ld]).  n % 8 == 0.
struct DxArgs {
  const __bf16* dz4;
  const __bf16* H;
  long long h_stride;
  const __bf16* w;
  MlpLayout L;
  __bf16* dZT;
  long long dzt_stride;
  long long ld;
  long long n;
};

hipError_t launch_mlp_dx(const DxArgs& a, hipStream_t st);

// Weight and bias gradients of the hidden layers from the transposed
// operands X0T [128][ld], HT [4][ht_stride] and dZT [5][dzt_stride]:
// partials over slices of slice_rows rows (weights into part, biases -- the
// row sums of dZ_l^T -- into part_b), then the in-order slice sums into g
// (W_l at w_off_l, b_l at b_off_l).  n and slice_rows are
// multiples of 32, n_slices = ceil(n / slice_rows).
struct DwArgs {
  const __bf16* X0T;
  const __bf16* HT;
  long long ht_stride;
  const __bf16* dZT;
  long long dzt_stride;
  long long ld;
  long long n;
  int slice_rows;
  int n_slices;
  MlpLayout L;
  float* part;    // [5][n_slices][256][256]
  float* part_b;  // [5][n_slices][256]
};

hipError_t launch_mlp_dw(const DwArgs& a, float* g, hipStream_t st);
hipError_t launch_head(const __bf16* H, int n, const float* w, const float* b, const float* y, float inv_total,
                       float* yhat, float* loss_part, float* gout, __bf16* dZ, hipStream_t st);
// out[col] = sum_m X[m][col] * (wt ? wt[m] : 1) through per-chunk partials
// (part: colsum_chunks(M) x N floats), fixed order.
int colsum_chunks(int M);
hipError_t launch_colsum(const __bf16* X, int M, int N, const float* wt, float* part, float* out, hipStream_t st);
hipError_t launch_sum_scalar(const float* x, int n, double scale, float* out, hipStream_t st);
hipError_t launch_segment_mean(const float* yhat, int T, int R, float* F, hipStream_t st);
hipError_t launch_adam_mlp(float* p, const float* gr, float* m, float* v, int* step, int n, float lr, float b1,
                           float b2, float eps, const MlpLayout& L, __bf16* wbf, __bf16* wtbf, hipStream_t st);
hipError_t launch_mlp_copies(const float* p, int n, const MlpLayout& L, __bf16* wbf, __bf16* wtbf,
                             hipStream_t st);
hipError_t launch_log_eps(const float* P, long long n, float eps, float* y, hipStream_t st);

}  // namespace drt
