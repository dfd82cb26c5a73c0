// Learned surrogate of the log smoothed power map: Fourier features
// gamma(v) = [sin(2 pi B v), cos(2 pi B v)] of v = (tx, rx) and a 6-layer ReLU
// MLP (128 -> 256 x 5 -> 1), trained and evaluated with BF16 MFMA
// (v_mfma_f32_16x16x32_bf16) and FP32 accumulation.
//
// Layouts: activations of a row tile in LDS, row-major bf16; the inputs of
// the weight gradients (features, hidden activations, their gradients)
// transposed in blocks of 32 rows; weights of hidden layer l as bf16 in two
// copies, W and W^T, in MFMA fragment order (frag_off); master weights,
// biases, Adam moments FP32 in one flat vector: per hidden layer
// W_l [in][out] then b_l [out], then the head w5 [256], b5 [1].
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
// and the new activations (bias, ReLU, bf16) overwrite them in place.  The
// head is a per-row dot product in FP32 over the last layer's registers
// (4 columns per lane, then a pairwise tree over the 64 column groups), with
// the same sums in the same order as the training pass's wave sum.
// ---------------------------------------------------------------------------
constexpr int kFusedWaves = 4;
constexpr int kFusedRows = 128;
constexpr int ALD = 256 + 8;    // activation row stride (bf16): 132 dwords, rows 4 banks apart
constexpr int kTrainRows = 32;  // rows per workgroup of the training pass (tile of the head's partial sums)

// The bf16 weight copies are stored in MFMA fragment order.  A copy is read
// as a matrix M [256][K] whose rows are the product's output columns c
// (W^T for the forward, W for the backward).  The operand of k-step ks,
// column tile j of the wavefront that owns columns 64 s .. 64 s + 63 is 64
// lanes x 8 consecutive k (lane = 16 (k / 8 % 4) + c % 16); those 1024
// bytes are contiguous, so one load instruction reads whole cache lines.
__device__ __forceinline__ size_t frag_off(int c, int k, int K) {
  return ((((size_t)(c >> 6) * (K >> 5) + (k >> 5)) * 4 + ((c >> 4) & 3)) * 64 + ((((k >> 3) & 3) << 4) | (c & 15))) * 8 +
         (k & 7);
}

// ReLU on the bit pattern: a float with its sign bit set (a negative value or
// -0) becomes +0 and any other is kept, as fmaxf(x, 0) gives for every non-NaN
// x, in one integer max (fmaxf first quietens its operand: a second instruction)
__device__ __forceinline__ float relu(float x) {
  return __builtin_bit_cast(float, max(__builtin_bit_cast(int, x), 0));
}

// Two floats rounded to BF16 (nearest even) in one register, x in the low
// half: the packed conversion the compiler emits for a pair, written out
// because it does not pair conversions whose result is then bit-cast.
__device__ __forceinline__ uint32_t cvt_pk_bf16(float x, float y) {
  uint32_t r;
  asm("v_cvt_pk_bf16_f32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(y));
  return r;
}

// ReLU of four values rounded to BF16: rounding keeps the sign, so the
// patterns with the sign bit set (negative values, -0, negative NaN) become
// +0 by an integer max on each 16-bit half, as rounding relu(x) gives for
// every x; two packed maxima where the float form takes four.
__device__ __forceinline__ bf16x4 relu_bf16x4(const floatx4& x) {
  typedef __attribute__((__vector_size__(2 * sizeof(short)))) short shortx2;
  const shortx2 lo = __builtin_bit_cast(shortx2, cvt_pk_bf16(x[0], x[1]));
  const shortx2 hi = __builtin_bit_cast(shortx2, cvt_pk_bf16(x[2], x[3]));
  const uint2 u = {__builtin_bit_cast(uint32_t, __builtin_elementwise_max(lo, (shortx2){0, 0})),
                   __builtin_bit_cast(uint32_t, __builtin_elementwise_max(hi, (shortx2){0, 0}))};
  return __builtin_bit_cast(bf16x4, u);
}

// x plus x of the lane 16 apart (lanes 0..15 pair with 16..31, 32..47 with
// 48..63), and x plus x of the lane 32 apart: each lane gets the pair's sum.
__device__ __forceinline__ float pair_sum16(float x) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float pair_sum32(float x) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Workgroup barrier that orders LDS only, so that global loads stay in
// flight across it (used where no wavefront reads global memory that
// another wavefront of the workgroup writes in the same launch).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// This lane's operand of (wavefront s, k-step ks, column tile j).
__device__ __forceinline__ const bf16* frag_ptr(const bf16* M, int K, int s, int ks, int j, int lane) {
  return M + ((((size_t)s * (K >> 5) + ks) * 4 + j) * 64 + lane) * 8;
}

// The transposed operands of the weight gradients are stored in blocks of
// kTB rows: element (col, row) of an operand with `cols` columns is at
// (row / kTB) cols kTB + col kTB + row % kTB, so a block is one contiguous
// piece (every 32-row k-step of the weight-gradient product reads one block).
constexpr int kTB = 32;

// Transposed store of the tile's first `cols` columns (cols % 4 == 0; ROWS
// and tile0 multiples of kTB; every row of the tile is below n).  A work item
// is 4 columns x 8 rows: eight 8-byte LDS reads (one row's 4 columns each)
// are transposed in registers into four 16-byte stores (one column's 8 rows
// each); adjacent lanes write adjacent 16-byte pieces.
template <int ROWS>
__device__ __forceinline__ void store_tile_t(const bf16* act, int cols, long long tile0, bf16* out) {
  static_assert(ROWS % kTB == 0, "whole blocks");
  constexpr int kChunks = ROWS / 8;
  for (int it = threadIdx.x; it < (cols / 4) * kChunks; it += kFusedWaves * 64) {
    const int g = it / kChunks, r8 = (it - g * kChunks) * 8;
    uint32_t d[8][2];
#pragma unroll
    for (int rr = 0; rr < 8; ++rr) {
      const uint2 x = *reinterpret_cast<const uint2*>(&act[(r8 + rr) * ALD + 4 * g]);
      d[rr][0] = x.x;  // columns 4g, 4g + 1
      d[rr][1] = x.y;  // columns 4g + 2, 4g + 3
    }
    const long long row = tile0 + r8;
    bf16* blk = out + (size_t)(row / kTB) * cols * kTB + row % kTB;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      uint4 o;
      uint32_t* ow = reinterpret_cast<uint32_t*>(&o);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t a0 = d[2 * k][c >> 1], a1 = d[2 * k + 1][c >> 1];
        ow[k] = (c & 1) ? ((a0 >> 16) | (a1 & 0xffff0000u)) : ((a0 & 0xffffu) | (a1 << 16));
      }
      *reinterpret_cast<uint4*>(blk + (size_t)(4 * g + c) * kTB) = o;
    }
  }
}

// Fourier features of rows tile0 .. tile0 + ROWS - 1 into act[r][0..127]
// (sin, then cos; rows past n get zeros).  The rows' inputs and B are first
// staged in LDS with one coalesced load per element, so the feature loop
// itself waits on no global load.  x(r, e): input e (0..3) of row r.
template <int ROWS, class X>
__device__ __forceinline__ void tile_features(bf16* act, float (*xin)[4], float (*bfs)[4], const float* Bf,
                                              long long tile0, long long n, X&& x) {
  const int tid = threadIdx.x;
  constexpr int kPer = (ROWS * 4 + kFusedWaves * 64 - 1) / (kFusedWaves * 64);
  float xv[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int e = tid + u * kFusedWaves * 64;
    const long long row = tile0 + (e >> 2);
    xv[u] = (e < ROWS * 4 && row < n) ? x(row, e & 3) : 0.0f;
  }
  const float bv = Bf[tid];  // kMlpFreq x 4 = 256 values, one per thread
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int e = tid + u * kFusedWaves * 64;
    if (e < ROWS * 4) xin[e >> 2][e & 3] = xv[u];
  }
  bfs[tid >> 2][tid & 3] = bv;
  __syncthreads();
  // thread (wavefront w, lane f) makes feature f of rows w, w + kFusedWaves,
  // ...: row f of B is read once, the rows' inputs are wave-uniform reads, and
  // the row limit is wave-uniform
  const int f = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const float b0 = bfs[f][0], b1 = bfs[f][1], b2 = bfs[f][2], b3 = bfs[f][3];
  const int rows_in = (int)(n - tile0 < ROWS ? n - tile0 : ROWS);  // rows r < rows_in exist
#pragma unroll 4
  for (int u = 0; u < ROWS / kFusedWaves; ++u) {
    const int r = w + kFusedWaves * u;
    // every row is evaluated (rows past n hold zero inputs) so that the
    // unrolled rows' input reads are in flight together; those rows store 0
    const float tt = b0 * xin[r][0] + b1 * xin[r][1] + b2 * xin[r][2] + b3 * xin[r][3];
    // sin / cos of 2 pi tt by the hardware's revolution-scaled sine and
    // cosine on the fractional part (exact), as BF16 features
    const float fr = __builtin_amdgcn_fractf(tt);
    const bool in = r < rows_in;
    act[r * ALD + f] = (bf16)(in ? __builtin_amdgcn_sinf(fr) : 0.0f);
    act[r * ALD + 64 + f] = (bf16)(in ? __builtin_amdgcn_cosf(fr) : 0.0f);
  }
}

template <int ROWS>
__global__ __launch_bounds__(kFusedWaves * 64, 2) void k_mlp_fused(FusedArgs a) {
  __shared__ __attribute__((aligned(16))) bf16 act[ROWS * ALD];
  constexpr int kRT = ROWS / 16;  // row tiles
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const long long tile0 = (long long)blockIdx.x * ROWS;

  // head parameters now, so their loads are long done when the head runs
  static_assert(kFusedWaves * 64 == kMlpWidth, "one head weight per thread");
  __shared__ __attribute__((aligned(16))) float hws[kMlpWidth];
  hws[tid] = a.p[a.L.head_w + tid];
  const float hb = a.p[a.L.head_b];
  __shared__ float xin[ROWS][4], bfs[kMlpFreq][4];
  if (a.v) {
    tile_features<ROWS>(act, xin, bfs, a.Bf, tile0, a.n, [&](long long row, int e) { return a.v[4 * row + e]; });
  } else {
    // row g pairs transmitter g / R with receiver g % R: the tile's first row
    // is divided once and its other rows step on from there (R >= 1, so at
    // most ROWS steps; none where R is a multiple of ROWS, as row0 is a
    // multiple of R)
    const long long g0 = a.row0 + tile0;
    const long long q0 = g0 / a.R, r0 = g0 % a.R;
    tile_features<ROWS>(act, xin, bfs, a.Bf, tile0, a.n, [&](long long row, int e) {
      long long q = q0, rr = r0 + (row - tile0);
      while (rr >= a.R) {
        rr -= a.R;
        ++q;
      }
      return e < 2 ? a.tx[2 * q + e] : a.rx[2 * rr + e - 2];
    });
  }
  __syncthreads();

  const int kq = 8 * (lane >> 4);  // this lane's 8-wide k slot within a 32-k step
  const int c0 = wave * 64;        // this wavefront's first output column
#pragma unroll 1
  for (int l = 0; l < kMlpHidden; ++l) {
    const int K = a.L.fan_in[l];
    const bf16* Wt = a.wt + a.L.bf_off[l];  // [256][K]
    const float* bias = a.p + a.L.b_off[l];
    const int nks = K / 32;
    // the accumulators start at the bias of their 4 columns (weights as the
    // first MFMA operand: a lane holds 4 consecutive output columns of one
    // row): the first step's multiplications take it as their addend, so no
    // copy of it into the accumulators is made
    floatx4 bq[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = c0 + 16 * j + 4 * (lane >> 4);
      bq[j] = (floatx4){bias[col], bias[col + 1], bias[col + 2], bias[col + 3]};
    }
    floatx4 acc[kRT][4];
    // weight fragments in two register sets, named apart (the loop body is
    // written out twice): the next k-step's fragments load into one while the
    // multiplications use the other.  nks (4 or 8) is even; the last request
    // is clamped to the last step, so the wait counts stay static.
    // (a scheduling barrier after each request keeps the compiler from
    // sinking it to just before its use)
    auto wload = [&](bf16x8 (&w)[4], int k) {
#pragma unroll
      for (int j = 0; j < 4; ++j) w[j] = *reinterpret_cast<const bf16x8*>(frag_ptr(Wt, K, wave, k, j, lane));
      __builtin_amdgcn_sched_barrier(0);
    };
    auto wmul = [&](const bf16x8 (&w)[4], int k) {
#pragma unroll
      for (int i = 0; i < kRT; ++i) {
        const bf16x8 af = *reinterpret_cast<const bf16x8*>(&act[(16 * i + (lane & 15)) * ALD + k * 32 + kq]);
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[j], af, acc[i][j], 0, 0, 0);
      }
    };
    auto wmul0 = [&](const bf16x8 (&w)[4]) {  // step 0: the bias as the addend
#pragma unroll
      for (int i = 0; i < kRT; ++i) {
        const bf16x8 af = *reinterpret_cast<const bf16x8*>(&act[(16 * i + (lane & 15)) * ALD + kq]);
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[j], af, bq[j], 0, 0, 0);
      }
    };
    bf16x8 wa[4], wb[4];
    wload(wa, 0);
    // nks (4 or 8) is even; the first pair of steps is written out
    wload(wb, 1);
    wmul0(wa);
    wload(wa, 2 < nks ? 2 : 1);
    wmul(wb, 1);
#pragma unroll 1
    for (int ks = 2; ks < nks; ks += 2) {
      wload(wb, ks + 1);
      wmul(wa, ks);
      wload(wa, ks + 2 < nks ? ks + 2 : ks + 1);
      wmul(wb, ks + 1);
    }
    if (l + 1 == kMlpHidden) {
      // The head's dot product of each row from the registers, summed as one
      // balanced tree of pairs over the 64 four-column groups (group G holds
      // columns 4 G .. 4 G + 3, a chain of fused multiply-adds from zero;
      // here G = 16 wave + 4 j + lane / 16): its lowest level pairs lanes 16
      // apart, the next lanes 32 apart, the next two this lane's column
      // tiles j, the last two the wavefronts (below, through LDS).
      float4 hw4[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) hw4[j] = *reinterpret_cast<const float4*>(&hws[c0 + 16 * j + 4 * (lane >> 4)]);
#pragma unroll
      for (int i = 0; i < kRT; ++i) {
        uint32_t t[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const bf16x4 h = relu_bf16x4(acc[i][j]);
          float p = 0.0f;
          p = fmaf((float)h[0], hw4[j].x, p);
          p = fmaf((float)h[1], hw4[j].y, p);
          p = fmaf((float)h[2], hw4[j].z, p);
          p = fmaf((float)h[3], hw4[j].w, p);
          t[j] = __float_as_uint(p);
        }
        // lanes 16 apart: swapping rows between tiles 0 and 1 (2 and 3)
        // leaves tile 0's (2's) pair sums in rows 0 and 2, tile 1's (3's) in
        // rows 1 and 3; lanes 32 apart: then row k holds tile k's sum
        const auto a01 = __builtin_amdgcn_permlane16_swap(t[0], t[1], false, false);
        const auto a23 = __builtin_amdgcn_permlane16_swap(t[2], t[3], false, false);
        const float s01 = __uint_as_float(a01[0]) + __uint_as_float(a01[1]);
        const float s23 = __uint_as_float(a23[0]) + __uint_as_float(a23[1]);
        const auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(s01), __float_as_uint(s23), false, false);
        // tiles (0, 1) and (2, 3), then the two pairs
        const float v = pair_sum32(pair_sum16(__uint_as_float(b[0]) + __uint_as_float(b[1])));
        if (lane < 16) xin[16 * i + lane][wave] = v;
      }
      break;
    }
    __syncthreads();  // every wavefront is past its last read of this layer's inputs
    // ReLU, BF16, 4 columns of one row per lane written as 8 bytes
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = c0 + 16 * j + 4 * (lane >> 4);
#pragma unroll
      for (int i = 0; i < kRT; ++i)
        *reinterpret_cast<bf16x4*>(&act[(16 * i + (lane & 15)) * ALD + col]) = relu_bf16x4(acc[i][j]);
    }
    __syncthreads();
  }
  // xin[r][w] now holds wavefront w's sum for row r (the inputs were last
  // read before the first layer): the tree's last two levels and the bias
  __syncthreads();
  float* yhs = &bfs[0][0];  // ROWS values (the features' B is no longer read)
  static_assert(ROWS <= kMlpFreq * 4, "yhat of the tile fits in the features' B");
  if (tid < ROWS) {
    const float yh = ((xin[tid][0] + xin[tid][1]) + (xin[tid][2] + xin[tid][3])) + hb;
    yhs[tid] = yh;
    if (a.yhat && tile0 + tid < a.n) a.yhat[tile0 + tid] = yh;
  }
  if (a.tile_sum) {
    // the tile's sum of yhat: each wavefront's quarter of the rows in order,
    // then the wavefronts in order (for per-transmitter means)
    constexpr int kRowsPerWave = ROWS / kFusedWaves;
    __shared__ double ws[kFusedWaves];
    __syncthreads();
    if (lane == 0) {
      double wsum = 0.0;
      for (int i = 0; i < kRowsPerWave; ++i) {
        const int r = wave * kRowsPerWave + i;
        if (tile0 + r < a.n) wsum += (double)yhs[r];
      }
      ws[wave] = wsum;
    }
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < kFusedWaves; ++w) t += ws[w];
      a.tile_sum[blockIdx.x] = t;
    }
  }
}

// ---------------------------------------------------------------------------
// Training pass of one tile of ROWS rows in one workgroup: the fused
// forward (features, five hidden layers), the head with the squared error
// and its output gradient, and the input-gradient chain
//   dZ_{l-1} = (dZ_l W_l^T) * (H_{l-1} > 0),  l = 4 .. 1,
// all on the tile's activations in LDS.  The ReLU masks of layers 0..3 stay
// in LDS (4 bits per byte); no row-major activation leaves the workgroup.  Out: the
// transposed operands of the weight gradients (X0T, HT_0..3, dZT_0..4), and
// per tile the partial sums of the head's gradients (sum_m g_m H_4[m][i] and
// sum_m g_m) and of the squared errors.
//
// Nine products of the tile (5 forward with W_l^T, 4 backward with W_l) run
// through one loop.  Wavefront w owns output columns 64 w .. 64 w + 63; its
// operand of a whole product (8 k-steps x 4 column tiles of bf16x8, 128
// VGPRs) sits in registers and is reloaded for the next product as soon as
// the multiplications are issued, so the loads are in flight during the
// epilogue and the stores.  Tiles are small (32 rows) so that two
// workgroups share a CU and one's products overlap the other's epilogue.
// ---------------------------------------------------------------------------
struct WSlice {
  bf16x8 f[8][4];  // [k-step][column tile]
};

// Rows c0 .. c0 + 63 of M [256][K] (K = 128 or 256, fragment order), this
// lane's operands of every k-step.  K is a compile-time constant, so the
// requests are issued back to back with no branch between them (a branch
// per k-step made the compiler wait for each group before the next).
template <int K>
__device__ __forceinline__ void load_wslice(WSlice& s, const bf16* M, int c0, int lane) {
  static_assert(K == kMlpIn || K == kMlpWidth, "fan-in");
#pragma unroll
  for (int ks = 0; ks < K / 32; ++ks)
#pragma unroll
    for (int j = 0; j < 4; ++j) s.f[ks][j] = *reinterpret_cast<const bf16x8*>(frag_ptr(M, K, c0 >> 6, ks, j, lane));
}

// Product p of the training pass: the matrix ([256][K], rows = output
// columns) and K.  p = 0..4: W_p^T; p = 5..8: W_{9-p} (backward).
__device__ __forceinline__ const bf16* train_matrix(const TrainArgs& a, int p, int& K) {
  if (p < kMlpHidden) {
    K = a.L.fan_in[p];
    return a.wt + a.L.bf_off[p];
  }
  K = kMlpWidth;
  return a.w + a.L.bf_off[2 * kMlpHidden - 1 - p];
}

template <int ROWS>
__global__ __launch_bounds__(kFusedWaves * 64, 2) void k_mlp_train(TrainArgs a) {
  constexpr int kRT = ROWS / 16;  // row tiles
  __shared__ __attribute__((aligned(16))) bf16 act[ROWS * ALD];
  __shared__ uint8_t mnib[kMlpHidden - 1][ROWS][kMlpWidth / 4];  // H_l > 0, l = 0..3: bit c % 4 of byte c / 4
  __shared__ float hwp[kFusedWaves][kMlpWidth];              // per-wavefront head-weight gradient partials
  __shared__ float hsp[kFusedWaves][2];                      // per-wavefront sums of g and of d^2
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const long long tile0 = (long long)blockIdx.x * ROWS;
  // the step count of the update this pass feeds (read by a later launch only)
  if (a.step && blockIdx.x == 0 && tid == 0) a.step[0] += 1;

  // head parameters and this wavefront's targets now, so their loads are
  // long done when the head runs (lane i < 16: row 16 wave + i)
  constexpr int kRowsPerWave = ROWS / kFusedWaves;
  const float* hw = a.p + a.L.head_w;
  float wv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) wv[q] = hw[lane * 4 + q];
  const float hb = a.p[a.L.head_b];
  const long long yrow = tile0 + wave * kRowsPerWave + (lane & (kRowsPerWave - 1));
  const float yv = yrow < a.n ? a.y[a.rows ? (long long)a.rows[yrow] : yrow] : 0.0f;
  // the hidden layers' biases, staged in LDS for the epilogues
  __shared__ __attribute__((aligned(16))) float bsh[kMlpHidden][kMlpWidth];
#pragma unroll
  for (int l = 0; l < kMlpHidden; ++l) bsh[l][tid] = a.p[a.L.b_off[l] + tid];
  __shared__ float xin[ROWS][4], bfs[kMlpFreq][4];
  tile_features<ROWS>(act, xin, bfs, a.Bf, tile0, a.n, [&](long long row, int e) {
    return a.v[4 * (a.rows ? (long long)a.rows[row] : row) + e];
  });
  __syncthreads();
  store_tile_t<ROWS>(act, kMlpIn, tile0, a.X0T);

  const int kq = 8 * (lane >> 4);
  const int c0 = wave * 64;
  WSlice ws;
  {
    int K;  // product 0 (W_0^T) has the features' fan-in, every other product 256
    const bf16* M = train_matrix(a, 0, K);
    load_wslice<kMlpIn>(ws, M, c0, lane);
  }
#pragma unroll 1
  for (int p = 0; p < 2 * kMlpHidden - 1; ++p) {
    int K;
    (void)train_matrix(a, p, K);
    floatx4 acc[kRT][4];
#pragma unroll
    for (int i = 0; i < kRT; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = (floatx4){0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      if (ks * 32 < K) {
#pragma unroll
        for (int i = 0; i < kRT; ++i) {
          const bf16x8 af = *reinterpret_cast<const bf16x8*>(&act[(16 * i + (lane & 15)) * ALD + ks * 32 + kq]);
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ws.f[ks][j], af, acc[i][j], 0, 0, 0);
        }
      }
    }
    // the next product's operand, in flight during the epilogue and the stores
    if (p + 1 < 2 * kMlpHidden - 1) {
      int Kn;
      const bf16* Mn = train_matrix(a, p + 1, Kn);
      load_wslice<kMlpWidth>(ws, Mn, c0, lane);
    }
    __syncthreads();  // every wavefront is past its last read of this product's input
    if (p < kMlpHidden) {
      // forward: bias, ReLU, bf16; a lane holds 4 consecutive columns of one row
      // (and writes their ReLU mask as one byte)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = c0 + 16 * j + 4 * (lane >> 4);
        const float4 b = *reinterpret_cast<const float4*>(&bsh[p][col]);
        const float bq[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
        for (int i = 0; i < kRT; ++i) {
          bf16x4 v;
          uint32_t m = 0;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            v[q] = (bf16)relu(acc[i][j][q] + bq[q]);
            m |= ((float)v[q] > 0.0f ? 1u : 0u) << q;
          }
          if (p < kMlpHidden - 1) mnib[p][16 * i + (lane & 15)][col / 4] = (uint8_t)m;
          *reinterpret_cast<bf16x4*>(&act[(16 * i + (lane & 15)) * ALD + col]) = v;
        }
      }
    } else {
      // backward: dZ_{l-1} = bf16(dZ_l W_l^T) masked by H_{l-1} > 0, l = 9 - p
      const int lm = 2 * kMlpHidden - 2 - p;  // l - 1
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = c0 + 16 * j + 4 * (lane >> 4);
#pragma unroll
        for (int i = 0; i < kRT; ++i) {
          const uint32_t m = mnib[lm][16 * i + (lane & 15)][col / 4];
          bf16x4 v;
#pragma unroll
          for (int q = 0; q < 4; ++q) v[q] = ((m >> q) & 1u) ? (bf16)acc[i][j][q] : (bf16)0.0f;
          *reinterpret_cast<bf16x4*>(&act[(16 * i + (lane & 15)) * ALD + col]) = v;
        }
      }
    }
    __syncthreads();
    if (p < kMlpHidden - 1) {
      store_tile_t<ROWS>(act, kMlpWidth, tile0, a.HT + (size_t)p * a.ht_stride);
    } else if (p == kMlpHidden - 1) {
      // head on this wavefront's rows: yhat = H_4 . w + b, d = yhat - y,
      // g = 2 d / n_total, dZ_4 = bf16(g w (H_4 > 0)) in place (each row is
      // read and written by the same lanes)
      float gw[4] = {0.0f, 0.0f, 0.0f, 0.0f};
      float gsum = 0.0f, lsum = 0.0f;
#pragma unroll
      for (int i = 0; i < kRowsPerWave; ++i) {
        const int r = wave * kRowsPerWave + i;
        const bool in = tile0 + r < a.n;
        float h[4], part = 0.0f;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          h[q] = (float)act[r * ALD + lane * 4 + q];
          part = fmaf(h[q], wv[q], part);
        }
        const float yh = wave_sum(part) + hb;
        const float d = in ? yh - __int_as_float(__builtin_amdgcn_readlane(__float_as_int(yv), i)) : 0.0f;
        const float gm = 2.0f * d * a.inv_total;
        if (in && a.yhat && lane == 0) a.yhat[tile0 + r] = yh;
        gsum += gm;
        lsum = fmaf(d, d, lsum);
        bf16x4 dz;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          gw[q] = fmaf(gm, h[q], gw[q]);
          dz[q] = (bf16)(h[q] > 0.0f ? gm * wv[q] : 0.0f);
        }
        *reinterpret_cast<bf16x4*>(&act[r * ALD + lane * 4]) = dz;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) hwp[wave][lane * 4 + q] = gw[q];
      if (lane == 0) {
        hsp[wave][0] = gsum;
        hsp[wave][1] = lsum;
      }
      __syncthreads();
      // the tile's partials, wavefronts in order
      {
        float t = 0.0f;
#pragma unroll
        for (int w = 0; w < kFusedWaves; ++w) t += hwp[w][tid];
        a.hw_part[(size_t)blockIdx.x * kMlpWidth + tid] = t;
        if (tid < 2) {
          float u = 0.0f;
#pragma unroll
          for (int w = 0; w < kFusedWaves; ++w) u += hsp[w][tid];
          a.hs_part[2 * (size_t)blockIdx.x + tid] = u;
        }
      }
      store_tile_t<ROWS>(act, kMlpWidth, tile0, a.dZT + (size_t)(kMlpHidden - 1) * a.dzt_stride);
    } else {
      const int lm = 2 * kMlpHidden - 2 - p;
      store_tile_t<ROWS>(act, kMlpWidth, tile0, a.dZT + (size_t)lm * a.dzt_stride);
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
// Weight-gradient partials of all five hidden layers in one launch:
//   part[l][s][i][o] = sum over the rows r of slice s of X_l^T[i][r] dZ_l^T[o][r]
// and the bias partials part_b[l][s][o] = sum over those rows of dZ_l^T[o][r]
// (X_0 = the features, X_l = H_{l-1}), both operands contiguous in r.  A work
// item is (layer, block of 128 rows i, half of the 256 columns o, slice): the
// halves double the workgroups, so two or more share a CU and cover each
// other's loads and barriers.  The X^T tile of a 32-row step is staged in LDS
// (double-buffered) for the workgroup's 4 wavefronts, each wavefront owning
// 32 columns o whose dZ^T fragments come straight from global memory.  k in
// increasing steps of 32 within a slice.
// ---------------------------------------------------------------------------
constexpr int XLD = 32 + 8;     // staged X^T step row stride (bf16)

__global__ __launch_bounds__(kFusedWaves * 64, 2) void k_mlp_dw(DwArgs a) {
  __shared__ __attribute__((aligned(16))) bf16 xs[2][128 * XLD];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  // decode the work item: half oh of the outputs o; layer 0 has one block
  // of 128 rows i (fan-in 128), the others two
  int item = blockIdx.x / a.n_slices;
  const int s = blockIdx.x - item * a.n_slices;
  const int oh = item & 1;
  item >>= 1;
  const int l = item == 0 ? 0 : 1 + (item - 1) / 2;
  const int rb = item == 0 ? 0 : (item - 1) % 2;
  const bf16* XT = l == 0 ? a.X0T : a.HT + (size_t)(l - 1) * a.ht_stride;
  const bf16* DT = a.dZT + (size_t)l * a.dzt_stride;
  const long long r0 = (long long)s * a.slice_rows;
  const long long r1 = r0 + a.slice_rows < a.n ? r0 + a.slice_rows : a.n;
  const int nks = (int)((r1 - r0) / 32);
  const int kq = 8 * (lane >> 4);
  const int c0 = 128 * oh + 32 * wave;  // this wavefront's 32 columns o
  // k-step ks (rows r0 + 32 ks ..) is block b0 + ks of both operands
  const long long b0 = r0 / kTB;
  const int xcols = l == 0 ? kMlpIn : kMlpWidth;
  // staging: thread -> (row i of the block, 16-row half of the step)
  const int si = tid >> 1, sh = (tid & 1) * 16;
  const bf16* xsrc = XT + (size_t)b0 * xcols * kTB + (size_t)(128 * rb + si) * kTB + sh;
  const size_t xstep = (size_t)xcols * kTB, dstep = (size_t)kMlpWidth * kTB;
  const bf16* dsrc = DT + (size_t)b0 * dstep + kq;
  floatx4 acc[8][2];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (floatx4){0.0f, 0.0f, 0.0f, 0.0f};
  // the first block of each layer also sums its dZ^T fragments: bias partials
  const bool bias = rb == 0;
  float bsum[2] = {0.0f, 0.0f};
  // pipeline, two k-steps deep: at step ks the X^T piece and the dZ^T
  // fragments of step ks + 2 are requested, the X^T piece of step ks + 1
  // (requested one step earlier) goes to the other LDS buffer, and the
  // barriers order LDS only, so the requests stay in flight across them
  auto xload = [&](int ks, uint4& x0, uint4& x1) {
    const uint4* src = reinterpret_cast<const uint4*>(xsrc + (size_t)ks * xstep);
    x0 = src[0];
    x1 = src[1];
  };
  auto dload = [&](int ks, bf16x8 (&d)[2]) {
#pragma unroll
    for (int j = 0; j < 2; ++j)
      d[j] = *reinterpret_cast<const bf16x8*>(dsrc + (size_t)ks * dstep + (size_t)(c0 + 16 * j + (lane & 15)) * kTB);
  };
  // three register sets for each operand, rotated by name (the loop body
  // is written out three times), so no copy waits for a load in flight
  uint4 X0a = {}, X0b = {}, X1a = {}, X1b = {}, X2a = {}, X2b = {};
  bf16x8 D0[2] = {}, D1[2] = {}, D2[2] = {};
  if (nks > 0) {
    xload(0, X0a, X0b);
    dload(0, D0);
  }
  if (nks > 1) {
    xload(1, X1a, X1b);
    dload(1, D1);
  }
  if (nks > 0) {
    uint4* dst = reinterpret_cast<uint4*>(&xs[0][si * XLD + sh]);
    dst[0] = X0a;
    dst[1] = X0b;
  }
  lds_barrier();
  // step ks: request step ks + 2 into (dl, xl), multiply with dc and LDS
  // buffer ks % 2, store the X^T piece of step ks + 1 (xw) to the other buffer
  auto step = [&](int ks, const bf16x8 (&dc)[2], bf16x8 (&dl)[2], uint4& xl0, uint4& xl1, const uint4& xw0,
                  const uint4& xw1) __attribute__((always_inline)) {
    const int buf = ks & 1;
    // (always issued, clamped to the last step, so the wait counts are static)
    const int kn = ks + 2 < nks ? ks + 2 : nks - 1;
    xload(kn, xl0, xl1);
    dload(kn, dl);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const bf16x8 af = *reinterpret_cast<const bf16x8*>(&xs[buf][(16 * i + (lane & 15)) * XLD + kq]);
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(dc[j], af, acc[i][j], 0, 0, 0);
    }
    if (bias) {
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int q = 0; q < 8; ++q) bsum[j] += (float)dc[j][q];
    }
    if (ks + 1 < nks) {
      uint4* dst = reinterpret_cast<uint4*>(&xs[buf ^ 1][si * XLD + sh]);
      dst[0] = xw0;
      dst[1] = xw1;
    }
    lds_barrier();
  };
#pragma unroll 1
  for (int ks = 0; ks < nks; ks += 3) {
    step(ks, D0, D2, X2a, X2b, X1a, X1b);
    if (ks + 1 < nks) step(ks + 1, D1, D0, X0a, X0b, X2a, X2b);
    if (ks + 2 < nks) step(ks + 2, D2, D1, X1a, X1b, X0a, X0b);
  }
  if (bias) {
    // lanes l, l ^ 16, l ^ 32, l ^ 48 hold the four 8-row slots of column o
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      float b = bsum[j];
      b += __shfl_xor(b, 16);
      b += __shfl_xor(b, 32);
      if (lane < 16) a.part_b[((size_t)l * a.n_slices + s) * 256 + c0 + 16 * j + lane] = b;
    }
  }
  // (dZ^T as the first MFMA operand: a lane holds 4 consecutive columns o of one row i)
  float* out = a.part + ((size_t)l * a.n_slices + s) * 256 * 256;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int o = c0 + 16 * j + 4 * (lane >> 4);
#pragma unroll
    for (int i = 0; i < 8; ++i)
      *reinterpret_cast<floatx4*>(out + (size_t)(128 * rb + 16 * i + (lane & 15)) * 256 + o) = acc[i][j];
  }
}

// One element of Adam (torch semantics) at step t with gradient gi: updates
// p[i], m[i], v[i] and returns the new p[i].
__device__ __forceinline__ float adam_elem(const AdamArgs& ad, int t, int i, float gi) {
  const float mi = ad.b1 * ad.m[i] + (1.0f - ad.b1) * gi;
  const float vi = ad.b2 * ad.v[i] + (1.0f - ad.b2) * gi * gi;
  ad.m[i] = mi;
  ad.v[i] = vi;
  const float bc1 = 1.0f - powf(ad.b1, (float)t);
  const float bc2 = 1.0f - powf(ad.b2, (float)t);
  const float pi = ad.p[i] - (ad.lr / bc1) * (mi / (sqrtf(vi) / sqrtf(bc2) + ad.eps));
  ad.p[i] = pi;
  return pi;
}

// Weight and bias gradients from the partials, slices in order:
// g[w_off_l + i 256 + o] = sum_s part[l][s][i][o], g[b_off_l + o] = sum_s part_b[l][s][o];
// with ad.p set, each element's Adam update follows its sum at once (and
// for hidden-layer weights the two BF16 copies).
__global__ void k_mlp_dw_sum(const float* __restrict__ part, const float* __restrict__ part_b, int n_slices,
                             MlpLayout L, float* __restrict__ g, HeadFold hf, AdamArgs ad) {
  const int l = blockIdx.y;
  if (l == kMlpHidden) {
    // the head (blocks 0..8 of the last row; fixed order throughout):
    // block b < 8: g[head_w + i], i = 32 b .. 32 b + 31, thread (i, z)
    // adding tiles z, z + 8, ... with eight loads in flight, then the eight
    // z in order; block 8: g[head_b] and the loss from the per-tile sums in
    // FP64 (strided per thread, then a tree).
    __shared__ double dsh[256];
    if (!hf.hw_part || blockIdx.x > 8) return;
    const int tid = threadIdx.x;
    if (blockIdx.x < 8) {
      const int i = 32 * blockIdx.x + (tid & 31), z = tid >> 5;
      float s = 0.0f;
      int t = z;
      for (; t + 56 < hf.tiles; t += 64) {
        float v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = hf.hw_part[(size_t)(t + 8 * k) * kMlpWidth + i];
#pragma unroll
        for (int k = 0; k < 8; ++k) s += v[k];
      }
      for (; t < hf.tiles; t += 8) s += hf.hw_part[(size_t)t * kMlpWidth + i];
      float* sh = reinterpret_cast<float*>(dsh);
      sh[tid] = s;
      __syncthreads();
      if (z == 0) {
        float u = 0.0f;
#pragma unroll
        for (int k = 0; k < 8; ++k) u += sh[32 * k + (tid & 31)];
        g[L.head_w + i] = u;
        if (ad.p) (void)adam_elem(ad, ad.step[0], L.head_w + i, u);
      }
      return;
    }
    for (int c = 0; c < 2; ++c) {
      double u = 0.0;
      for (int t = tid; t < hf.tiles; t += 256) u += (double)hf.hs_part[2 * (size_t)t + c];
      dsh[tid] = u;
      __syncthreads();
      for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) dsh[tid] += dsh[tid + w];
        __syncthreads();
      }
      if (tid == 0) {
        if (c == 0) {
          const float gb = (float)dsh[0];
          g[L.head_b] = gb;
          if (ad.p) (void)adam_elem(ad, ad.step[0], L.head_b, gb);
        } else if (hf.loss) {
          hf.loss[0] = (float)(dsh[0] * hf.inv_n);
        }
      }
      __syncthreads();
    }
    return;
  }
  const int e = blockIdx.x * blockDim.x + threadIdx.x;  // i 256 + o within layer l, then the 256 biases
  const int nw = L.fan_in[l] * 256;
  if (e < nw) {
    const float* p = part + (size_t)l * n_slices * 256 * 256 + e;
    float s = 0.0f;
    for (int z = 0; z < n_slices; ++z) s += p[(size_t)z * 256 * 256];
    g[L.w_off[l] + e] = s;
    if (ad.p) {
      const float pi = adam_elem(ad, ad.step[0], L.w_off[l] + e, s);
      const int r = e >> 8, c = e & 255;  // W[r][c]: input r, output c
      ad.wbf[L.bf_off[l] + frag_off(r, c, 256)] = (bf16)pi;         // W: rows = inputs, k = outputs
      ad.wtbf[L.bf_off[l] + frag_off(c, r, L.fan_in[l])] = (bf16)pi;  // W^T: rows = outputs, k = inputs
    }
  } else if (e < nw + 256) {
    const float* p = part_b + (size_t)l * n_slices * 256 + (e - nw);
    float s = 0.0f;
    for (int z = 0; z < n_slices; ++z) s += p[(size_t)z * 256];
    g[L.b_off[l] + e - nw] = s;
    if (ad.p) (void)adam_elem(ad, ad.step[0], L.b_off[l] + e - nw, s);
  }
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
      wbf[L.bf_off[l] + frag_off(r, c, 256)] = (bf16)p[i];
      wtbf[L.bf_off[l] + frag_off(c, r, fi)] = (bf16)p[i];
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

hipError_t launch_mlp_train(const TrainArgs& a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  if (a.n % kTrainRows != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mlp_train<kTrainRows>, dim3((unsigned)(a.n / kTrainRows)), dim3(kFusedWaves * 64), 0, st, a);
  return hipGetLastError();
}

int mlp_train_rows() { return kTrainRows; }

hipError_t launch_mlp_dw(const DwArgs& a, float* g, const HeadFold& hf, const AdamArgs& adam, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  if (a.n % kTB != 0 || a.slice_rows % kTB != 0) return hipErrorInvalidValue;
  // items: layer 0 (one block of 128 inputs) + layers 1..4 (two blocks each)
  const int items = 2 * (1 + 2 * (kMlpHidden - 1));  // (layer, row block) x two halves of the outputs
  hipLaunchKernelGGL(k_mlp_dw, dim3(items * a.n_slices), dim3(kFusedWaves * 64), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_dw_sum, dim3(257, kMlpHidden + 1), dim3(256), 0, st, a.part, a.part_b, a.n_slices, a.L, g,
                     hf, adam);
  return hipGetLastError();
}

hipError_t launch_segment_mean(const float* yhat, int T, int R, float* F, hipStream_t st) {
  hipLaunchKernelGGL(k_segment_mean, dim3(T), dim3(256), 0, st, yhat, R, F);
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
