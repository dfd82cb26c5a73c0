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

struct GemmArgs {
  const __bf16* A;
  int lda;
  const __bf16* B;
  int ldb;
  int M, N, K;
  int k_split;
  const float* bias;     // [N] or NULL
  int relu;
  const __bf16* mask;    // [M][N] or NULL: zero where mask <= 0
  float* out_f32;        // [slices][M][N] or NULL
  __bf16* out_bf16;      // [M][N] or NULL
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
};

hipError_t launch_mlp_fused(const FusedArgs& a, hipStream_t st);
// out[c][r] = in[r][c], bf16 [n][cols] -> [cols][ld]; n % 64 == 0, cols % 64 == 0.
hipError_t launch_transpose_bf16(const __bf16* in, int n, int cols, __bf16* out, long long ld, hipStream_t st);
hipError_t launch_gemm(const GemmArgs& g, bool a_mc, bool b_nc, int n_slices, hipStream_t st);
hipError_t launch_head(const __bf16* H, int n, const float* w, const float* b, const float* y, float inv_total,
                       float* yhat, float* loss_part, float* gout, __bf16* dZ, hipStream_t st);
// out[col] = sum_m X[m][col] * (wt ? wt[m] : 1) through per-chunk partials
// (part: colsum_chunks(M) x N floats), fixed order.
int colsum_chunks(int M);
hipError_t launch_colsum(const __bf16* X, int M, int N, const float* wt, float* part, float* out, hipStream_t st);
hipError_t launch_sum_slices(const float* part, int n_slices, int n, float* out, hipStream_t st);
hipError_t launch_sum_scalar(const float* x, int n, double scale, float* out, hipStream_t st);
hipError_t launch_segment_mean(const float* yhat, int T, int R, float* F, hipStream_t st);
hipError_t launch_adam_mlp(float* p, const float* gr, float* m, float* v, int* step, int n, float lr, float b1,
                           float b2, float eps, const MlpLayout& L, __bf16* wbf, __bf16* wtbf, hipStream_t st);
hipError_t launch_mlp_copies(const float* p, int n, const MlpLayout& L, __bf16* wbf, __bf16* wtbf,
                             hipStream_t st);
hipError_t launch_log_eps(const float* P, long long n, float eps, float* y, hipStream_t st);

}  // namespace drt
