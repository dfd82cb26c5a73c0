// Learned surrogate of the log smoothed power map: Fourier features
// gamma(v) = [sin(2 pi B v), cos(2 pi B v)] of v = (tx, rx) and a 6-layer ReLU
// MLP (128 -> 256 x 5 -> 1), trained and evaluated with BF16 MFMA
// (v_mfma_f32_16x16x32_bf16) and FP32 accumulation.
//
// Layouts (row-major): features X0 [n][128] bf16; hidden activations
// H_l [n][256] bf16; weights of hidden layer l as bf16 in two copies,
// W [in][out] and W^T [out][in]; master weights, biases, Adam moments FP32 in
// one flat vector: per hidden layer W_l [in][out] then b_l [out], then the
// head w5 [256], b5 [1].
#include "dev.h"
#include "mlp.h"

namespace drt {

typedef __bf16 bf16;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

// ---------------------------------------------------------------------------
// Fused forward: features, the five hidden layers and the head of a tile of
// ROWS rows (128, or 64 for small batches) in one workgroup of kFusedWaves
// wavefronts.  The tile's
// activations stay in LDS (bf16, [row][k]) from layer to layer and are read
// by every wavefront; wavefront w owns output columns 64 w .. 64 w + 63 of
// every row, so its weight fragments (W^T rows of those columns) are its own
// and come straight from global memory (L2-resident: 640 KB for all five
// layers), one k-step ahead, with no LDS traffic or barrier inside a layer.
// Per 32-k step a wavefront issues (ROWS / 16) x 4 MFMA 16x16x32 (row
// tiles x 4 column tiles), k in increasing steps of 32, FP32 accumulation.
// After a layer every wavefront has finished reading its inputs (barrier),
// the new activations (bias, ReLU, bf16) overwrite them in place, and
// optionally go to global memory for the backward pass.  The head is k_head's
// per-row dot product (4 columns per lane, then the wave sum).
// ---------------------------------------------------------------------------
constexpr int kFusedWaves = 4;
constexpr int kFusedRows = 128;
constexpr int ALD = 256 + 8;    // activation row stride (bf16): 132 dwords, rows 4 banks apart

// Row-major store of the tile's first `cols` activation columns, 16 bytes
// per thread (rows past n are not stored).
template <int ROWS = kFusedRows>
__device__ __forceinline__ void store_tile(const bf16* act, int cols, long long tile0, long long n, bf16* out) {
  const int per_row = cols / 8;
  for (int i = threadIdx.x; i < ROWS * per_row; i += kFusedWaves * 64) {
    const int r = i / per_row, c8 = (i - r * per_row) * 8;
    if (tile0 + r < n)
      *reinterpret_cast<uint4*>(out + (tile0 + r) * cols + c8) = *reinterpret_cast<const uint4*>(&act[r * ALD + c8]);
  }
}

// Transposed store out[col][tile0 + r] (row stride ld): 8 rows of one column
// per thread, 16 bytes (rows past n are zero; ld and tile0 are multiples of 8).
template <int ROWS = kFusedRows>
__device__ __forceinline__ void store_tile_t(const bf16* act, int cols, long long tile0, long long n, bf16* out,
                                             long long ld) {
  constexpr int kChunks = ROWS / 8;
  for (int i = threadIdx.x; i < cols * kChunks; i += kFusedWaves * 64) {
    const int col = i / kChunks, r8 = (i - col * kChunks) * 8;
    if (tile0 + r8 >= n) continue;
    bf16x8 v;
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = tile0 + r8 + q < n ? act[(r8 + q) * ALD + col] : (bf16)0.0f;
    *reinterpret_cast<bf16x8*>(out + (size_t)col * ld + tile0 + r8) = v;
  }
}

template <int ROWS>
__global__ __launch_bounds__(kFusedWaves * 64, 2) void k_mlp_fused(FusedArgs a) {
  __shared__ __attribute__((aligned(16))) bf16 act[ROWS * ALD];
  constexpr int kRT = ROWS / 16;  // row tiles
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const long long tile0 = (long long)blockIdx.x * ROWS;

  // features of the tile's rows (rows past n get zeros and are never stored)
  for (int i = tid; i < ROWS * 64; i += kFusedWaves * 64) {
    const int r = i >> 6, f = i & 63;
    const long long row = tile0 + r;
    float s = 0.0f, c = 0.0f;
    if (row < a.n) {
      float x0, x1, x2, x3;
      if (a.v) {
        x0 = a.v[4 * row];
        x1 = a.v[4 * row + 1];
        x2 = a.v[4 * row + 2];
        x3 = a.v[4 * row + 3];
      } else {
        const long long g = a.row0 + row;
        const int t = (int)(g / a.R), q = (int)(g % a.R);
        x0 = a.tx[2 * t];
        x1 = a.tx[2 * t + 1];
        x2 = a.rx[2 * q];
        x3 = a.rx[2 * q + 1];
      }
      const float tt = a.Bf[4 * f] * x0 + a.Bf[4 * f + 1] * x1 + a.Bf[4 * f + 2] * x2 + a.Bf[4 * f + 3] * x3;
      sincospif(2.0f * tt, &s, &c);
    }
    act[r * ALD + f] = (bf16)s;
    act[r * ALD + 64 + f] = (bf16)c;
  }
  __syncthreads();
  if (a.X0) store_tile<ROWS>(act, 128, tile0, a.n, a.X0);
  if (a.X0T) store_tile_t<ROWS>(act, 128, tile0, a.n, a.X0T, a.ld_t);

  const int kq = 8 * (lane >> 4);  // this lane's 8-wide k slot within a 32-k step
  const int c0 = wave * 64;        // this wavefront's first output column
#pragma unroll 1
  for (int l = 0; l < kMlpHidden; ++l) {
    const int K = a.L.fan_in[l];
    const bf16* Wt = a.wt + a.L.bf_off[l];  // [256][K]
    const float* bias = a.p + a.L.b_off[l];
    const int nks = K / 32;
    floatx4 acc[kRT][4];
#pragma unroll
    for (int i = 0; i < kRT; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = (floatx4){0.0f, 0.0f, 0.0f, 0.0f};
    // weight fragments of k-step 0; then each step loads the next one's
    bf16x8 bw[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      bw[j] = *reinterpret_cast<const bf16x8*>(Wt + (size_t)(c0 + 16 * j + (lane & 15)) * K + kq);
#pragma unroll 1
    for (int ks = 0; ks < nks; ++ks) {
      bf16x8 bn[4];
      const int kn = ks + 1 < nks ? ks + 1 : ks;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        bn[j] = *reinterpret_cast<const bf16x8*>(Wt + (size_t)(c0 + 16 * j + (lane & 15)) * K + kn * 32 + kq);
#pragma unroll
      for (int i = 0; i < kRT; ++i) {
        const bf16x8 af = *reinterpret_cast<const bf16x8*>(&act[(16 * i + (lane & 15)) * ALD + ks * 32 + kq]);
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[j], af, acc[i][j], 0, 0, 0);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) bw[j] = bn[j];
    }
    __syncthreads();  // every wavefront is past its last read of this layer's inputs
    // (weights as the first MFMA operand: a lane holds 4 consecutive output
    // columns of one row, written to the activations as 8 bytes)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = c0 + 16 * j + 4 * (lane >> 4);
      float b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) b[q] = bias[col + q];
#pragma unroll
      for (int i = 0; i < kRT; ++i) {
        bf16x4 v;
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = (bf16)fmaxf(acc[i][j][q] + b[q], 0.0f);
        *reinterpret_cast<bf16x4*>(&act[(16 * i + (lane & 15)) * ALD + col]) = v;
      }
    }
    __syncthreads();
    if (a.H) store_tile<ROWS>(act, 256, tile0, a.n, a.H + (size_t)l * a.h_stride);
    if (a.HT && l + 1 < kMlpHidden)
      store_tile_t<ROWS>(act, 256, tile0, a.n, a.HT + (size_t)l * a.ht_stride, a.ld_t);
  }
  // head: rows of this wavefront, k_head's order
  const float* hw = a.p + a.L.head_w;
  float wv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) wv[q] = hw[lane * 4 + q];
  const float hb = a.p[a.L.head_b];
  constexpr int kRowsPerWave = ROWS / kFusedWaves;
  double wsum = 0.0;  // lane 0: this wavefront's rows, in order
#pragma unroll 1
  for (int i = 0; i < kRowsPerWave; ++i) {
    const int r = wave * kRowsPerWave + i;
    float part = 0.0f;
#pragma unroll
    for (int q = 0; q < 4; ++q) part = fmaf((float)act[r * ALD + lane * 4 + q], wv[q], part);
    const float yh = wave_sum(part) + hb;
    if (lane == 0 && tile0 + r < a.n) {
      if (a.yhat) a.yhat[tile0 + r] = yh;
      wsum += (double)yh;
    }
  }
  if (a.tile_sum) {
    // the tile's sum of yhat, wavefronts in order (for per-transmitter means)
    __shared__ double ws[kFusedWaves];
    if (lane == 0) ws[wave] = wsum;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < kFusedWaves; ++w) t += ws[w];
      a.tile_sum[blockIdx.x] = t;
    }
  }
}

// F[t] = (sum over the tiles of transmitter t, in order) / R: the mean of
// yhat over its R receivers from the fused forward's tile sums.
__global__ void k_tile_mean(const double* __restrict__ tile_sum, int n_tx, int tiles_per_tx, int R,
                            float* __restrict__ F) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tx) return;
  double s = 0.0;
  for (int j = 0; j < tiles_per_tx; ++j) s += tile_sum[(size_t)t * tiles_per_tx + j];
  F[t] = (float)(s / R);
}

// ---------------------------------------------------------------------------
// Input gradients of the hidden layers, 4 down to 1, fused over the layers
// like the forward: a workgroup takes kDxRows rows of dZ_4 (the head's
// gradient, row-major bf16) into LDS and forms
//   dZ_{l-1} = (dZ_l W_l^T) * (H_{l-1} > 0)
// in place, wavefront w owning columns 64 w .. 64 w + 63 with the weight
// fragments (rows of W_l [in][out]) straight from global memory, k in steps of
// 32, FP32 accumulation.  Each dZ_l (l = 4..0) is stored transposed, dZT + l dzt_stride
// ([256][ld]), for the weight and bias gradients.
// ---------------------------------------------------------------------------
constexpr int kDxRows = 64;  // rows per workgroup of k_mlp_dx: more workgroups for small batches

__global__ __launch_bounds__(kFusedWaves * 64, 2) void k_mlp_dx(DxArgs a) {
  __shared__ __attribute__((aligned(16))) bf16 act[kDxRows * ALD];
  constexpr int kRT = kDxRows / 16;  // row tiles
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const long long tile0 = (long long)blockIdx.x * kDxRows;
  for (int i = tid; i < kDxRows * 32; i += kFusedWaves * 64) {
    const int r = i >> 5, c8 = (i & 31) * 8;
    uint4 v = {0u, 0u, 0u, 0u};
    if (tile0 + r < a.n) v = *reinterpret_cast<const uint4*>(a.dz4 + (tile0 + r) * 256 + c8);
    *reinterpret_cast<uint4*>(&act[r * ALD + c8]) = v;
  }
  __syncthreads();
  store_tile_t<kDxRows>(act, 256, tile0, a.n, a.dZT + (size_t)(kMlpHidden - 1) * a.dzt_stride, a.ld);
  const int kq = 8 * (lane >> 4);
  const int c0 = wave * 64;
#pragma unroll 1
  for (int l = kMlpHidden - 1; l >= 1; --l) {
    const bf16* Wl = a.w + a.L.bf_off[l];  // W_l [in = 256][out = 256]
    const bf16* mask = a.H + (size_t)(l - 1) * a.h_stride;
    floatx4 acc[kRT][4];
#pragma unroll
    for (int i = 0; i < kRT; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = (floatx4){0.0f, 0.0f, 0.0f, 0.0f};
    bf16x8 bw[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      bw[j] = *reinterpret_cast<const bf16x8*>(Wl + (size_t)(c0 + 16 * j + (lane & 15)) * 256 + kq);
#pragma unroll 1
    for (int ks = 0; ks < 8; ++ks) {
      bf16x8 bn[4];
      const int kn = ks + 1 < 8 ? ks + 1 : ks;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        bn[j] = *reinterpret_cast<const bf16x8*>(Wl + (size_t)(c0 + 16 * j + (lane & 15)) * 256 + kn * 32 + kq);
#pragma unroll
      for (int i = 0; i < kRT; ++i) {
        const bf16x8 af = *reinterpret_cast<const bf16x8*>(&act[(16 * i + (lane & 15)) * ALD + ks * 32 + kq]);
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[j], af, acc[i][j], 0, 0, 0);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) bw[j] = bn[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = c0 + 16 * j + 4 * (lane >> 4);
#pragma unroll
      for (int i = 0; i < kRT; ++i) {
        bf16x4 v;
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = (bf16)acc[i][j][q];
        *reinterpret_cast<bf16x4*>(&act[(16 * i + (lane & 15)) * ALD + col]) = v;
      }
    }
    __syncthreads();
    // ReLU derivative of layer l - 1, 16 bytes at a time (rows past n become 0)
    for (int c = tid; c < kDxRows * 32; c += kFusedWaves * 64) {
      const int r = c >> 5, c8 = (c & 31) * 8;
      bf16x8 v = *reinterpret_cast<const bf16x8*>(&act[r * ALD + c8]);
      bf16x8 mk = {};
      if (tile0 + r < a.n) mk = *reinterpret_cast<const bf16x8*>(mask + (tile0 + r) * 256 + c8);
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = (float)mk[q] > 0.0f ? v[q] : (bf16)0.0f;
      *reinterpret_cast<bf16x8*>(&act[r * ALD + c8]) = v;
    }
    __syncthreads();
    store_tile_t<kDxRows>(act, 256, tile0, a.n, a.dZT + (size_t)(l - 1) * a.dzt_stride, a.ld);
  }
}

// ---------------------------------------------------------------------------
// Weight-gradient partials of all five hidden layers in one launch:
//   part[l][s][i][o] = sum over the rows r of slice s of X_l^T[i][r] dZ_l^T[o][r]
// and the bias partials part_b[l][s][o] = sum over those rows of dZ_l^T[o][r]
// (X_0 = the features, X_l = H_{l-1}), both operands contiguous in r.  A work
// item is (layer, block of 128 rows i, slice); the X^T tile of a 32-row step
// is staged in LDS (double-buffered) for the workgroup's 4 wavefronts, each
// wavefront owning 64 columns o whose dZ^T fragments come straight from
// global memory.  k in increasing steps of 32 within a slice.
// ---------------------------------------------------------------------------
constexpr int XLD = 32 + 8;     // staged X^T step row stride (bf16)

__global__ __launch_bounds__(kFusedWaves * 64, 2) void k_mlp_dw(DwArgs a) {
  __shared__ __attribute__((aligned(16))) bf16 xs[2][128 * XLD];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  // decode the work item: layer 0 has one block of 128 rows (fan-in 128), the others two
  int item = blockIdx.x / a.n_slices;
  const int s = blockIdx.x - item * a.n_slices;
  const int l = item == 0 ? 0 : 1 + (item - 1) / 2;
  const int rb = item == 0 ? 0 : (item - 1) % 2;
  const bf16* XT = l == 0 ? a.X0T : a.HT + (size_t)(l - 1) * a.ht_stride;
  const bf16* DT = a.dZT + (size_t)l * a.dzt_stride;
  const long long r0 = (long long)s * a.slice_rows;
  const long long r1 = r0 + a.slice_rows < a.n ? r0 + a.slice_rows : a.n;
  const int nks = (int)((r1 - r0) / 32);
  const int kq = 8 * (lane >> 4);
  const int c0 = wave * 64;
  // staging: thread -> (row i of the block, 16-row half of the step)
  const int si = tid >> 1, sh = (tid & 1) * 16;
  const bf16* xsrc = XT + (size_t)(128 * rb + si) * a.ld + r0 + sh;
  floatx4 acc[8][4];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (floatx4){0.0f, 0.0f, 0.0f, 0.0f};
  // the first block of each layer also sums its dZ^T fragments: bias partials
  const bool bias = rb == 0;
  float bsum[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  if (nks > 0) {
    const uint4* src = reinterpret_cast<const uint4*>(xsrc);
    uint4* dst = reinterpret_cast<uint4*>(&xs[0][si * XLD + sh]);
    dst[0] = src[0];
    dst[1] = src[1];
  }
  bf16x8 bw[4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
    bw[j] = *reinterpret_cast<const bf16x8*>(DT + (size_t)(c0 + 16 * j + (lane & 15)) * a.ld + r0 + kq);
  __syncthreads();
#pragma unroll 1
  for (int ks = 0; ks < nks; ++ks) {
    const int buf = ks & 1;
    const bool more = ks + 1 < nks;
    uint4 nx0, nx1;
    bf16x8 bn[4];
    if (more) {
      const uint4* src = reinterpret_cast<const uint4*>(xsrc + (ks + 1) * 32);
      nx0 = src[0];
      nx1 = src[1];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        bn[j] = *reinterpret_cast<const bf16x8*>(DT + (size_t)(c0 + 16 * j + (lane & 15)) * a.ld + r0 +
                                                 (ks + 1) * 32 + kq);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const bf16x8 af = *reinterpret_cast<const bf16x8*>(&xs[buf][(16 * i + (lane & 15)) * XLD + kq]);
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[j], af, acc[i][j], 0, 0, 0);
    }
    if (bias) {
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int q = 0; q < 8; ++q) bsum[j] += (float)bw[j][q];
    }
    if (more) {
      uint4* dst = reinterpret_cast<uint4*>(&xs[buf ^ 1][si * XLD + sh]);
      dst[0] = nx0;
      dst[1] = nx1;
#pragma unroll
      for (int j = 0; j < 4; ++j) bw[j] = bn[j];
    }
    __syncthreads();
  }
  if (bias) {
    // lanes l, l ^ 16, l ^ 32, l ^ 48 hold the four 8-row slots of column o
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float b = bsum[j];
      b += __shfl_xor(b, 16);
      b += __shfl_xor(b, 32);
      if (lane < 16) a.part_b[((size_t)l * a.n_slices + s) * 256 + c0 + 16 * j + lane] = b;
    }
  }
  // (dZ^T as the first MFMA operand: a lane holds 4 consecutive columns o of one row i)
  float* out = a.part + ((size_t)l * a.n_slices + s) * 256 * 256;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int o = c0 + 16 * j + 4 * (lane >> 4);
#pragma unroll
    for (int i = 0; i < 8; ++i)
      *reinterpret_cast<floatx4*>(out + (size_t)(128 * rb + 16 * i + (lane & 15)) * 256 + o) = acc[i][j];
  }
}

// Weight and bias gradients from the partials, slices in order:
// g[w_off_l + i 256 + o] = sum_s part[l][s][i][o], g[b_off_l + o] = sum_s part_b[l][s][o].
__global__ void k_mlp_dw_sum(const float* __restrict__ part, const float* __restrict__ part_b, int n_slices,
                             MlpLayout L, float* __restrict__ g) {
  const int l = blockIdx.y;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;  // i 256 + o within layer l, then the 256 biases
  const int nw = L.fan_in[l] * 256;
  if (e < nw) {
    const float* p = part + (size_t)l * n_slices * 256 * 256 + e;
    float s = 0.0f;
    for (int z = 0; z < n_slices; ++z) s += p[(size_t)z * 256 * 256];
    g[L.w_off[l] + e] = s;
  } else if (e < nw + 256) {
    const float* p = part_b + (size_t)l * n_slices * 256 + (e - nw);
    float s = 0.0f;
    for (int z = 0; z < n_slices; ++z) s += p[(size_t)z * 256];
    g[L.b_off[l] + e - nw] = s;
  }
}

// ---------------------------------------------------------------------------
// Head: yhat = H[m] . w + b (FP32).  Training: d = yhat - y, loss_part[m] = d^2,
// g[m] = 2 d / n_total, dZ[m][i] = bf16(g w[i] (H[m][i] > 0)).
// One wavefront per row; 4 rows per workgroup.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_head(const bf16* __restrict__ H, int n, const float* __restrict__ w,
                                              const float* __restrict__ b, const float* __restrict__ y,
                                              float inv_total, float* __restrict__ yhat,
                                              float* __restrict__ loss_part, float* __restrict__ gout,
                                              bf16* __restrict__ dZ) {
  const int lane = threadIdx.x & 63;
  const int m = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (m >= n) return;  // whole wavefront leaves together
  float h[4], wv[4];
  float part = 0.0f;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    h[q] = (float)H[(size_t)m * 256 + lane * 4 + q];
    wv[q] = w[lane * 4 + q];
    part = fmaf(h[q], wv[q], part);
  }
  const float yh = wave_sum(part) + b[0];
  if (yhat && lane == 0) yhat[m] = yh;
  if (y) {
    const float d = yh - y[m];
    const float gm = 2.0f * d * inv_total;
    if (lane == 0) {
      loss_part[m] = d * d;
      gout[m] = gm;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) dZ[(size_t)m * 256 + lane * 4 + q] = (bf16)(h[q] > 0.0f ? gm * wv[q] : 0.0f);
  }
}

// part[chunk][col] = sum over the chunk's kColChunk rows m of
// X[m][col] * (wt ? wt[m] : 1); one workgroup per (chunk, 256 columns).
// Thread (row lane r, column group g) reads 8 columns at once (16 bytes) of
// rows r, r + 8, ... in order; the 8 row lanes are then added in order
// through LDS (fixed order overall, with k_colsum_fold).  N % 8 == 0.
constexpr int kColChunk = 128;

__global__ __launch_bounds__(256) void k_colsum_part(const bf16* __restrict__ X, int M, int N,
                                                     const float* __restrict__ wt, float* __restrict__ part) {
  __shared__ float sh[8][256];
  const int cg = threadIdx.x & 31, rl = threadIdx.x >> 5;
  const int col0 = blockIdx.y * 256 + cg * 8;
  const int m0 = blockIdx.x * kColChunk, m1 = min(M, m0 + kColChunk);
  float s[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  if (col0 < N) {
    int m = m0 + rl;
    // four rows' loads in flight, then their products in row order (the
    // order of the plain loop below)
    for (; m + 24 < m1; m += 32) {
      uint4 raw[4];
      float w[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        raw[q] = *reinterpret_cast<const uint4*>(X + (size_t)(m + 8 * q) * N + col0);
        w[q] = wt ? wt[m + 8 * q] : 1.0f;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const bf16* x = reinterpret_cast<const bf16*>(&raw[q]);
#pragma unroll
        for (int k = 0; k < 8; ++k) s[k] = fmaf((float)x[k], w[q], s[k]);
      }
    }
    for (; m < m1; m += 8) {
      const uint4 raw = *reinterpret_cast<const uint4*>(X + (size_t)m * N + col0);
      const bf16* x = reinterpret_cast<const bf16*>(&raw);
      const float w = wt ? wt[m] : 1.0f;
#pragma unroll
      for (int k = 0; k < 8; ++k) s[k] = fmaf((float)x[k], w, s[k]);
    }
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) sh[rl][cg * 8 + k] = s[k];
  __syncthreads();
  const int col = blockIdx.y * 256 + threadIdx.x;
  if (col < N) {
    float t = 0.0f;
#pragma unroll
    for (int r = 0; r < 8; ++r) t += sh[r][threadIdx.x];
    part[(size_t)blockIdx.x * N + col] = t;
  }
}

// out[col] = sum over chunks of part[chunk][col]: 32 columns per workgroup,
// 8 threads per column each adding every 8th chunk in order, then the 8
// partials in order.
__global__ __launch_bounds__(256) void k_colsum_fold(const float* __restrict__ part, int chunks, int N,
                                                     float* __restrict__ out) {
  __shared__ float sh[8][32];
  const int c = threadIdx.x & 31, q = threadIdx.x >> 5;
  const int col = blockIdx.x * 32 + c;
  float s = 0.0f;
  if (col < N) {
    int z = q;
    // eight loads in flight, then the adds in chunk order
    for (; z + 56 < chunks; z += 64) {
      float v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = part[(size_t)(z + 8 * j) * N + col];
#pragma unroll
      for (int j = 0; j < 8; ++j) s += v[j];
    }
    for (; z < chunks; z += 8) s += part[(size_t)z * N + col];
  }
  sh[q][c] = s;
  __syncthreads();
  if (q == 0 && col < N) {
    float t = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) t += sh[k][c];
    out[col] = t;
  }
}

// scale * sum(x[0..n)) in FP64, fixed tree order; one workgroup of 1024.
__global__ __launch_bounds__(1024) void k_sum_scalar(const float* __restrict__ x, int n, double scale,
                                                     float* __restrict__ out) {
  __shared__ double sh[1024];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) s += (double)x[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = (float)(scale * sh[0]);
}

// Segment means: F[t] = mean of yhat[t * R .. t * R + R).  One workgroup per t.
__global__ void k_segment_mean(const float* __restrict__ yhat, int R, float* __restrict__ F) {
  __shared__ double sh[256];
  const float* p = yhat + (size_t)blockIdx.x * R;
  double s = 0.0;
  for (int i = threadIdx.x; i < R; i += 256) s += (double)p[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) F[blockIdx.x] = (float)(sh[0] / R);
}

// Adam on the flat FP32 parameters (torch semantics) with t = step[0] + 1,
// then BF16 copies W [in][out] and W^T [out][in] of the hidden layers.
__global__ void k_adam_mlp(float* __restrict__ p, const float* __restrict__ gr, float* __restrict__ m,
                           float* __restrict__ v, const int* __restrict__ step, int n, float lr, float b1,
                           float b2, float eps, MlpLayout L, bf16* __restrict__ wbf, bf16* __restrict__ wtbf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int t = step[0] + 1;
  const float gi = gr[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float bc1 = 1.0f - powf(b1, (float)t);
  const float bc2 = 1.0f - powf(b2, (float)t);
  const float pi = p[i] - (lr / bc1) * (mi / (sqrtf(vi) / sqrtf(bc2) + eps));
  p[i] = pi;
#pragma unroll
  for (int l = 0; l < kMlpHidden; ++l) {
    const int off = L.w_off[l], fi = L.fan_in[l];
    if (i >= off && i < off + fi * 256) {
      const int r = (i - off) / 256, c = (i - off) % 256;
      wbf[L.bf_off[l] + r * 256 + c] = (bf16)pi;
      wtbf[L.bf_off[l] + c * fi + r] = (bf16)pi;
    }
  }
}

__global__ void k_step_inc(int* step) { step[0] += 1; }

// Same bf16 copies without an update (after loading parameters).
__global__ void k_mlp_copies(const float* __restrict__ p, int n, MlpLayout L, bf16* __restrict__ wbf,
                             bf16* __restrict__ wtbf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int l = 0; l < kMlpHidden; ++l) {
    const int off = L.w_off[l], fi = L.fan_in[l];
    if (i >= off && i < off + fi * 256) {
      const int r = (i - off) / 256, c = (i - off) % 256;
      wbf[L.bf_off[l] + r * 256 + c] = (bf16)p[i];
      wtbf[L.bf_off[l] + c * fi + r] = (bf16)p[i];
    }
  }
}

// y = log(P + eps)
__global__ void k_log_eps(const float* __restrict__ P, long long n, float eps, float* __restrict__ y) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = logf(P[i] + eps);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

hipError_t launch_mlp_fused(const FusedArgs& a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  // tiles of 64 rows while there are too few of 128 to fill the chip twice
  // (training batches); per-tile sums always use tiles of kFusedRows
  if (!a.tile_sum && a.n < 2LL * 256 * kFusedRows) {
    hipLaunchKernelGGL(k_mlp_fused<kFusedRows / 2>, dim3((unsigned)((a.n + kFusedRows / 2 - 1) / (kFusedRows / 2))),
                       dim3(kFusedWaves * 64), 0, st, a);
  } else {
    hipLaunchKernelGGL(k_mlp_fused<kFusedRows>, dim3((unsigned)((a.n + kFusedRows - 1) / kFusedRows)),
                       dim3(kFusedWaves * 64), 0, st, a);
  }
  return hipGetLastError();
}

int mlp_fused_rows() { return kFusedRows; }

hipError_t launch_tile_mean(const double* tile_sum, int n_tx, int tiles_per_tx, int R, float* F, hipStream_t st) {
  if (n_tx <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_mean, dim3((n_tx + 255) / 256), dim3(256), 0, st, tile_sum, n_tx, tiles_per_tx, R, F);
  return hipGetLastError();
}

hipError_t launch_mlp_dx(const DxArgs& a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_dx, dim3((unsigned)((a.n + kDxRows - 1) / kDxRows)), dim3(kFusedWaves * 64), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_mlp_dw(const DwArgs& a, float* g, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  if (a.n % 32 != 0 || a.slice_rows % 32 != 0 || a.ld % 8 != 0) return hipErrorInvalidValue;
  // items: layer 0 (one block of 128 inputs) + layers 1..4 (two blocks each)
  const int items = 1 + 2 * (kMlpHidden - 1);
  hipLaunchKernelGGL(k_mlp_dw, dim3(items * a.n_slices), dim3(kFusedWaves * 64), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_dw_sum, dim3(257, kMlpHidden), dim3(256), 0, st, a.part, a.part_b, a.n_slices, a.L, g);
  return hipGetLastError();
}

hipError_t launch_head(const bf16* H, int n, const float* w, const float* b, const float* y, float inv_total,
                       float* yhat, float* loss_part, float* gout, bf16* dZ, hipStream_t st) {
  hipLaunchKernelGGL(k_head, dim3((n + 3) / 4), dim3(256), 0, st, H, n, w, b, y, inv_total, yhat, loss_part, gout,
                     dZ);
  return hipGetLastError();
}

int colsum_chunks(int M) { return (M + kColChunk - 1) / kColChunk; }

hipError_t launch_colsum(const bf16* X, int M, int N, const float* wt, float* part, float* out, hipStream_t st) {
  const int chunks = colsum_chunks(M);
  if (chunks <= 0 || N <= 0) return hipSuccess;
  if (N % 8 != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_colsum_part, dim3(chunks, (N + 255) / 256), dim3(256), 0, st, X, M, N, wt, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_colsum_fold, dim3((N + 31) / 32), dim3(256), 0, st, part, chunks, N, out);
  return hipGetLastError();
}

hipError_t launch_sum_scalar(const float* x, int n, double scale, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_scalar, dim3(1), dim3(1024), 0, st, x, n, scale, out);
  return hipGetLastError();
}

hipError_t launch_segment_mean(const float* yhat, int T, int R, float* F, hipStream_t st) {
  hipLaunchKernelGGL(k_segment_mean, dim3(T), dim3(256), 0, st, yhat, R, F);
  return hipGetLastError();
}

hipError_t launch_adam_mlp(float* p, const float* gr, float* m, float* v, int* step, int n, float lr, float b1,
                           float b2, float eps, const MlpLayout& L, bf16* wbf, bf16* wtbf, hipStream_t st) {
  hipLaunchKernelGGL(k_adam_mlp, dim3((n + 255) / 256), dim3(256), 0, st, p, gr, m, v, step, n, lr, b1, b2, eps, L,
                     wbf, wtbf);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_step_inc, dim3(1), dim3(1), 0, st, step);
  return hipGetLastError();
}

hipError_t launch_mlp_copies(const float* p, int n, const MlpLayout& L, bf16* wbf, bf16* wtbf, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_copies, dim3((n + 255) / 256), dim3(256), 0, st, p, n, L, wbf, wtbf);
  return hipGetLastError();
}

hipError_t launch_log_eps(const float* P, long long n, float eps, float* y, hipStream_t st) {
  hipLaunchKernelGGL(k_log_eps, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, P, n, eps, y);
  return hipGetLastError();
}

}  // namespace drt
