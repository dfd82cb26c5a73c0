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
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

// ---------------------------------------------------------------------------
// C[M x N] = A[M x K] . B[K x N], BF16 in, FP32 accumulate.
//   A(m, k) = A[m * lda + k]          (A_MC = false)
//           = A[k * lda + m]          (A_MC = true)
//   B(k, n) = B[n * ldb + k]          (B_NC = false)
//           = B[k * ldb + n]          (B_NC = true)
// Tile 64 x 64 x 64 per workgroup of 4 wavefronts (2 x 2, 32 x 32 each, as
// 2 x 2 MFMA 16x16x32 tiles).  Both operand tiles sit in LDS with k
// contiguous so every fragment is one 16-byte LDS read.  gridDim.z splits K
// (k_split per slice); slice z writes out_f32 + z * M * N.
// Epilogue: + bias[n], ReLU, * (mask[m][n] > 0), then FP32 and/or BF16 out.
// Requires N % 64 == 0, K % 64 == 0, k_split % 64 == 0, lda / ldb % 8 == 0.
// ---------------------------------------------------------------------------
constexpr int GT = 64;          // tile edge
constexpr int GLD = GT + 8;     // LDS row stride (bf16), 144 bytes

template <bool A_MC, bool B_NC>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) bf16 As[GT * GLD];
  __shared__ __attribute__((aligned(16))) bf16 Bs[GT * GLD];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int m0 = blockIdx.x * GT, n0 = blockIdx.y * GT;
  const int kb = blockIdx.z * g.k_split;
  const int ke = min(g.K, kb + g.k_split);
  const bf16x8 zero8 = {};

  floatx4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (floatx4){0.0f, 0.0f, 0.0f, 0.0f};

  for (int k0 = kb; k0 < ke; k0 += GT) {
    // stage A tile rows m0..m0+63, k0..k0+63 into As[m][k]
#pragma unroll
    for (int rep = 0; rep < 2; ++rep) {
      const int c = t + rep * 256;
      if (!A_MC) {
        const int r = c >> 3, kc = (c & 7) * 8;
        bf16x8 val = zero8;
        if (m0 + r < g.M) val = *reinterpret_cast<const bf16x8*>(g.A + (size_t)(m0 + r) * g.lda + k0 + kc);
        *reinterpret_cast<bf16x8*>(&As[r * GLD + kc]) = val;
      } else {
        const int kr = c >> 3, mc = (c & 7) * 8;
        bf16x8 val = zero8;
        if (m0 + mc < g.M) val = *reinterpret_cast<const bf16x8*>(g.A + (size_t)(k0 + kr) * g.lda + m0 + mc);
#pragma unroll
        for (int j = 0; j < 8; ++j) As[(mc + j) * GLD + kr] = val[j];
      }
    }
    // stage B tile n0..n0+63, k0..k0+63 into Bs[n][k]
#pragma unroll
    for (int rep = 0; rep < 2; ++rep) {
      const int c = t + rep * 256;
      if (!B_NC) {
        const int r = c >> 3, kc = (c & 7) * 8;
        const bf16x8 val = *reinterpret_cast<const bf16x8*>(g.B + (size_t)(n0 + r) * g.ldb + k0 + kc);
        *reinterpret_cast<bf16x8*>(&Bs[r * GLD + kc]) = val;
      } else {
        const int kr = c >> 3, nc = (c & 7) * 8;
        const bf16x8 val = *reinterpret_cast<const bf16x8*>(g.B + (size_t)(k0 + kr) * g.ldb + n0 + nc);
#pragma unroll
        for (int j = 0; j < 8; ++j) Bs[(nc + j) * GLD + kr] = val[j];
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GT; kk += 32) {
      bf16x8 af[2], bfr[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int r = wm * 32 + i * 16 + (lane & 15);
        af[i] = *reinterpret_cast<const bf16x8*>(&As[r * GLD + kk + 8 * (lane >> 4)]);
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int r = wn * 32 + j * 16 + (lane & 15);
        bfr[j] = *reinterpret_cast<const bf16x8*>(&Bs[r * GLD + kk + 8 * (lane >> 4)]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }

  float* outf = g.out_f32 ? g.out_f32 + (size_t)blockIdx.z * g.M * g.N : nullptr;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn * 32 + j * 16 + (lane & 15);
      const float bias = g.bias ? g.bias[col] : 0.0f;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + v;
        if (row >= g.M) continue;
        float x = acc[i][j][v] + bias;
        if (g.relu) x = fmaxf(x, 0.0f);
        if (g.mask && !((float)g.mask[(size_t)row * g.N + col] > 0.0f)) x = 0.0f;
        if (outf) outf[(size_t)row * g.N + col] = x;
        if (g.out_bf16) g.out_bf16[(size_t)row * g.N + col] = (bf16)x;
      }
    }
}

// ---------------------------------------------------------------------------
// Fused forward: features, the five hidden layers and the head of a tile of
// kFusedRows rows in one workgroup.  The tile's activations stay in LDS
// (bf16, [row][k]) from layer to layer; each layer's weights W^T [256][in]
// stream through LDS in chunks of 32 k (double-buffered, shared by the
// workgroup's 8 wavefronts).  Wavefront w owns rows 16 w .. 16 w + 15 of the
// tile and all 256 output columns: 16 MFMA 16x16x32 accumulators, k in
// increasing steps of 32 -- the accumulation order of k_gemm, so every
// activation is bitwise the one of the layer-by-layer path.  After a layer's
// last chunk every wavefront has finished reading the activations, and the
// new ones (bias, ReLU, bf16) overwrite them in place; optionally they also
// go to global memory for the backward pass.  The head is k_head's per-row
// dot product (4 columns per lane, then the wave sum).
// ---------------------------------------------------------------------------
constexpr int kFusedWaves = 8;
constexpr int kFusedRows = 16 * kFusedWaves;
constexpr int ALD = 256 + 8;    // activation row stride (bf16): 132 dwords, rows 4 banks apart
constexpr int WKC = 32;         // k per staged weight chunk
constexpr int WLD = WKC + 8;    // weight chunk row stride (bf16): 20 dwords

// Row-major store of the tile's first `cols` activation columns, 16 bytes
// per thread (rows past n are not stored).
__device__ __forceinline__ void store_tile(const bf16* act, int cols, long long tile0, long long n, bf16* out) {
  const int per_row = cols / 8;
  for (int i = threadIdx.x; i < kFusedRows * per_row; i += kFusedWaves * 64) {
    const int r = i / per_row, c8 = (i - r * per_row) * 8;
    if (tile0 + r < n)
      *reinterpret_cast<uint4*>(out + (tile0 + r) * cols + c8) = *reinterpret_cast<const uint4*>(&act[r * ALD + c8]);
  }
}

// Transposed store out[col][tile0 + r] (row stride ld): 8 rows of one column
// per thread, 16 bytes (rows past n are zero; ld and tile0 are multiples of 8).
__device__ __forceinline__ void store_tile_t(const bf16* act, int cols, long long tile0, long long n, bf16* out,
                                             long long ld) {
  constexpr int kChunks = kFusedRows / 8;
  for (int i = threadIdx.x; i < cols * kChunks; i += kFusedWaves * 64) {
    const int col = i / kChunks, r8 = (i - col * kChunks) * 8;
    if (tile0 + r8 >= n) continue;
    bf16x8 v;
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = tile0 + r8 + q < n ? act[(r8 + q) * ALD + col] : (bf16)0.0f;
    *reinterpret_cast<bf16x8*>(out + (size_t)col * ld + tile0 + r8) = v;
  }
}

__global__ __launch_bounds__(kFusedWaves * 64) void k_mlp_fused(FusedArgs a) {
  __shared__ __attribute__((aligned(16))) bf16 act[kFusedRows * ALD];
  __shared__ __attribute__((aligned(16))) bf16 wch[2][256 * WLD];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const long long tile0 = (long long)blockIdx.x * kFusedRows;

  // features of the tile's rows (rows past n get zeros and are never stored)
  for (int i = tid; i < kFusedRows * 64; i += kFusedWaves * 64) {
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
  if (a.X0 || a.X0T) {
    __syncthreads();
    if (a.X0) store_tile(act, 128, tile0, a.n, a.X0);
    if (a.X0T) store_tile_t(act, 128, tile0, a.n, a.X0T, a.ld_t);
  }

  const int ar = wave * 16 + (lane & 15);  // this lane's A row in the tile
  const int kq = 8 * (lane >> 4);          // and its 8-wide k slot within a 32-k step
  // staging of a weight chunk (256 columns x 32 k): thread -> (output column, 16-k half)
  const int sc = tid >> 1, sh = (tid & 1) * 16;
#pragma unroll 1
  for (int l = 0; l < kMlpHidden; ++l) {
    const int K = a.L.fan_in[l];
    const bf16* Wt = a.wt + a.L.bf_off[l];  // [256][K]
    const float* bias = a.p + a.L.b_off[l];
    const int nch = K / WKC;
    {
      const uint4* src = reinterpret_cast<const uint4*>(Wt + (size_t)sc * K + sh);
      uint4* dst = reinterpret_cast<uint4*>(&wch[0][sc * WLD + sh]);
      dst[0] = src[0];
      dst[1] = src[1];
    }
    __syncthreads();  // features / previous layer's outputs and chunk 0 in place
    floatx4 acc[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[j] = (floatx4){0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 1
    for (int kc = 0; kc < nch; ++kc) {
      const int buf = kc & 1;
      uint4 nx0, nx1;
      const bool more = kc + 1 < nch;
      if (more) {
        const uint4* src = reinterpret_cast<const uint4*>(Wt + (size_t)sc * K + (kc + 1) * WKC + sh);
        nx0 = src[0];
        nx1 = src[1];
      }
      const bf16x8 af = *reinterpret_cast<const bf16x8*>(&act[ar * ALD + kc * WKC + kq]);
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const bf16x8 bfr = *reinterpret_cast<const bf16x8*>(&wch[buf][(j * 16 + (lane & 15)) * WLD + kq]);
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bfr, acc[j], 0, 0, 0);
      }
      if (more) {
        uint4* dst = reinterpret_cast<uint4*>(&wch[buf ^ 1][sc * WLD + sh]);
        dst[0] = nx0;
        dst[1] = nx1;
      }
      __syncthreads();
    }
    // every wavefront is past its last read of this layer's inputs
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int col = j * 16 + (lane & 15);
      const float b = bias[col];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = wave * 16 + 4 * (lane >> 4) + q;
        act[r * ALD + col] = (bf16)fmaxf(acc[j][q] + b, 0.0f);
      }
    }
    __syncthreads();
    if (a.H) store_tile(act, 256, tile0, a.n, a.H + (size_t)l * a.h_stride);
    if (a.HT && l + 1 < kMlpHidden) store_tile_t(act, 256, tile0, a.n, a.HT + (size_t)l * a.ht_stride, a.ld_t);
  }
  // head: rows of this wavefront, k_head's order
  const float* hw = a.p + a.L.head_w;
  float wv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) wv[q] = hw[lane * 4 + q];
  const float hb = a.p[a.L.head_b];
#pragma unroll 1
  for (int i = 0; i < 16; ++i) {
    const int r = wave * 16 + i;
    float part = 0.0f;
#pragma unroll
    for (int q = 0; q < 4; ++q) part = fmaf((float)act[r * ALD + lane * 4 + q], wv[q], part);
    const float yh = wave_sum(part) + hb;
    if (lane == 0 && tile0 + r < a.n) a.yhat[tile0 + r] = yh;
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

// out[c][r] = in[r][c] for a bf16 [n][cols] matrix (out row stride ld):
// 64 x 64 tiles through LDS, 16-byte loads and stores.  n % 64 == 0.
__global__ __launch_bounds__(256) void k_transpose_bf16(const bf16* __restrict__ in, int n, int cols,
                                                        bf16* __restrict__ out, long long ld) {
  __shared__ bf16 t[64][64 + 8];
  const int r0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
#pragma unroll
  for (int rep = 0; rep < 2; ++rep) {
    const int i = threadIdx.x + rep * 256;
    const int r = i >> 3, c8 = (i & 7) * 8;
    const bf16x8 v = *reinterpret_cast<const bf16x8*>(in + (size_t)(r0 + r) * cols + c0 + c8);
#pragma unroll
    for (int q = 0; q < 8; ++q) t[r][c8 + q] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int rep = 0; rep < 2; ++rep) {
    const int i = threadIdx.x + rep * 256;
    const int c = i >> 3, r8 = (i & 7) * 8;
    bf16x8 v;
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = t[r8 + q][c];
    *reinterpret_cast<bf16x8*>(out + (size_t)(c0 + c) * ld + r0 + r8) = v;
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

// out[i] = sum_z part[z * n + i] in order.
__global__ void k_sum_slices(const float* __restrict__ part, int n_slices, int n, float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.0f;
  int z = 0;
  // eight loads in flight, then the adds in slice order (the order of a
  // plain loop, so the sum is the same)
  for (; z + 8 <= n_slices; z += 8) {
    float v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = part[(size_t)(z + q) * n + i];
#pragma unroll
    for (int q = 0; q < 8; ++q) s += v[q];
  }
  for (; z < n_slices; ++z) s += part[(size_t)z * n + i];
  out[i] = s;
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

hipError_t launch_gemm(const GemmArgs& g, bool a_mc, bool b_nc, int n_slices, hipStream_t st) {
  const dim3 grid((g.M + GT - 1) / GT, g.N / GT, n_slices);
  if (!a_mc && !b_nc) hipLaunchKernelGGL((k_gemm<false, false>), grid, dim3(256), 0, st, g);
  else if (a_mc && b_nc) hipLaunchKernelGGL((k_gemm<true, true>), grid, dim3(256), 0, st, g);
  else if (a_mc) hipLaunchKernelGGL((k_gemm<true, false>), grid, dim3(256), 0, st, g);
  else hipLaunchKernelGGL((k_gemm<false, true>), grid, dim3(256), 0, st, g);
  return hipGetLastError();
}

hipError_t launch_mlp_fused(const FusedArgs& a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  const unsigned tiles = (unsigned)((a.n + kFusedRows - 1) / kFusedRows);
  hipLaunchKernelGGL(k_mlp_fused, dim3(tiles), dim3(kFusedWaves * 64), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_head(const bf16* H, int n, const float* w, const float* b, const float* y, float inv_total,
                       float* yhat, float* loss_part, float* gout, bf16* dZ, hipStream_t st) {
  hipLaunchKernelGGL(k_head, dim3((n + 3) / 4), dim3(256), 0, st, H, n, w, b, y, inv_total, yhat, loss_part, gout,
                     dZ);
  return hipGetLastError();
}

hipError_t launch_transpose_bf16(const bf16* in, int n, int cols, bf16* out, long long ld, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (n % 64 != 0 || cols % 64 != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_transpose_bf16, dim3(n / 64, cols / 64), dim3(256), 0, st, in, n, cols, out, ld);
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

hipError_t launch_sum_slices(const float* part, int n_slices, int n, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_slices, dim3((n + 255) / 256), dim3(256), 0, st, part, n_slices, n, out);
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
