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

hipError_t launch_features(const float* v, const float* tx, const float* rx, int R, long long row0, int n,
                           const float* Bf, __bf16* X0, hipStream_t st);
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
