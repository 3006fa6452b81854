// Device side of the learned collision closure: a 19-64-64-19 perceptron
// evaluated per wave of 64 voxels with bfloat16 matrix-core instructions
// (v_mfma_f32_32x32x16_bf16, FP32 accumulation), tanh-form GELU, and the
// projection of its output onto the second-order Hermite space.
//
// Per wave, layer k computes Z[64 voxels x N] = A[64 x K] W[K x N] + b as
// 2 (voxel tiles) x N/32 (column tiles) x K/16 (k chunks) MFMAs.  Activations
// go through the wave's own LDS region (bf16, padded rows); weights sit in
// LDS in operand order, shared by the workgroup.
#pragma once
#ifdef LBM_Q27
#error "the closure network is a D3Q19 network"
#endif
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_common.h"
#include "lattice.h"

namespace lbm {
inline namespace LBM_LATTICE_NS {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

constexpr int kMlpHidden = 64;
constexpr int kMlpInPad = 32;   // 19 inputs padded to two k chunks of 16
constexpr int kMlpOutPad = 32;  // 19 outputs padded to one column tile
constexpr int kActStride = kMlpHidden + 8;  // bf16 per LDS activation row (padding against bank conflicts)
constexpr int kOutStride = kMlpOutPad + 1;  // floats per LDS output row
constexpr int kWaveLdsBytes = 64 * kActStride * 2;  // activations; the output tile aliases it
static_assert(64 * kOutStride * 4 <= kWaveLdsBytes, "output tile must fit the activation region");

// packed bf16 weights in operand order: [k chunk][column tile][lane][8]
constexpr int kW1Elems = (kMlpInPad / 16) * (kMlpHidden / 32) * 64 * 8;   // 2048
constexpr int kW2Elems = (kMlpHidden / 16) * (kMlpHidden / 32) * 64 * 8;  // 4096
constexpr int kW3Elems = (kMlpHidden / 16) * (kMlpOutPad / 32) * 64 * 8;  // 2048
constexpr int kWPackedElems = kW1Elems + kW2Elems + kW3Elems;            // 8192 bf16 = 16 KB
// GELU as a table of linear pieces: kGeluSegs pieces of width
// 1/kGeluPerUnit centred on -8, -8 + 1/kGeluPerUnit, ..., each (slope,
// intercept) as two floats; the table follows the packed weights in device
// memory and in LDS.
constexpr int kGeluPerUnit = 32;
constexpr int kGeluSegs = 16 * kGeluPerUnit;                       // 512
constexpr int kGeluTabBytes = kGeluSegs * 8;                       // 4 KB
constexpr int kWStageElems = kWPackedElems + kGeluTabBytes / 2;    // weights + table, in bf16 units
constexpr int kBiasFloats = kMlpHidden + kMlpHidden + kMlpOutPad;          // 160
constexpr int kStdFloats = 4 * 32;  // in_mean, in_inv_std, out_std, out_mean (19 used of 32)

// Number of trained parameters and their order in flat parameter arrays:
// W1 [19][64], b1 [64], W2 [64][64], b2 [64], W3 [64][19], b3 [19].
constexpr int kMlpW1 = 0, kMlpB1 = kMlpW1 + 19 * 64, kMlpW2 = kMlpB1 + 64, kMlpB2 = kMlpW2 + 64 * 64,
              kMlpW3 = kMlpB2 + 64, kMlpB3 = kMlpW3 + 64 * 19, kMlpParams = kMlpB3 + 19;  // 6675

// Lane layout of v_mfma_f32_32x32x16_bf16 (A: 32x16, B: 16x32, D: 32x32):
// lane l holds A[l%32][8(l/32) + j] and B[8(l/32) + j][l%32] for j = 0..7,
// and D[8(r/4) + 4(l/32) + r%4][l%32] in accumulator element r = 0..15.
__device__ __forceinline__ int mfma_a_row(int l) { return l & 31; }
__device__ __forceinline__ int mfma_k0(int l) { return 8 * (l >> 5); }
__device__ __forceinline__ int mfma_d_row(int l, int r) { return 8 * (r >> 2) + 4 * (l >> 5) + (r & 3); }
__device__ __forceinline__ int mfma_d_col(int l) { return l & 31; }

// Position of weight W[k][n] (k < K, n < N) in the packed operand order.
__host__ __device__ inline int packed_index(int k, int n, int N) {
  const int kc = k / 16, kk = k % 16, nt = n / 32, nn = n % 32;
  const int lane = nn + 32 * (kk / 8), j = kk % 8;
  return ((kc * (N / 32) + nt) * 64 + lane) * 8 + j;
}

struct MlpView {
  const __bf16 *w;         // packed weights (global), kWPackedElems
  const float *bias;       // b1 [64], b2 [64], b3 [32] (global)
  const float *stdz;       // in_mean, in_inv_std, out_std, out_mean, 32 each
  unsigned long long *fallbacks;  // fallback counter (64-bit: a long run exceeds 2^32 updates)
};

// tanh-form GELU, written as x * sigmoid(2 sqrt(2/pi) (x + 0.044715 x^3))
__device__ __forceinline__ float gelu_f(float x) {
  // exp(-2z) = 2^(x (c1 + c2 x^2)), z = sqrt(2/pi) (x + 0.044715 x^3):
  // c1 = -2 sqrt(2/pi) / ln 2, c2 = 0.044715 c1; then x * sigmoid(2z) with
  // the hardware exp2 and reciprocal (about 1 ulp each; the result is
  // rounded to bf16 for the next layer)
  constexpr float c1 = -2.0f * 0.7978845608028654f * 1.4426950408889634f;
  constexpr float c2 = 0.044715f * c1;
  const float e = __builtin_amdgcn_exp2f(x * fmaf(c2, x * x, c1));
  return x * __builtin_amdgcn_rcpf(1.0f + e);
}

// tanh-form GELU from the table of linear pieces in LDS (tab: the
// (slope, intercept) pairs; piece j spans a width 1/32 centred on
// -8 + j/32 and interpolates the function with its error centred, at most
// 5e-5 away from it, below the bf16 rounding of the result).  Arguments
// beyond the table use the outermost piece: 0 below, x above.  The piece
// index is round(32 (x + 8)): one FMA adds 2^23 as well, which leaves that
// integer in the low mantissa bits of the rounded sum (x 32 is exact, so
// the FMA rounds once; a tie takes the even piece, and both neighbours
// agree there to 5e-5), and the clamped bit pattern shifted by 3 is the
// byte offset of the piece plus a constant that one shift-and-add removes.
__device__ __forceinline__ float gelu_tab(float x, const float2 *tab) {
  constexpr float kTwo23 = 8388608.0f;
  static_assert(8.0f * kGeluPerUnit + kTwo23 == 8388864.0f, "the offset must be exact at 2^23");
  const float t = __builtin_amdgcn_fmed3f(fmaf(x, (float)kGeluPerUnit, 8.0f * kGeluPerUnit + kTwo23), kTwo23,
                                          kTwo23 + (float)(kGeluSegs - 1));
  const uint32_t off = (__float_as_uint(t) << 3) - (__float_as_uint(kTwo23) << 3);
  const float2 c = *(const float2 *)((const char *)tab + off);
  return fmaf(c.x, x, c.y);
}

// derivative of gelu_f
__device__ __forceinline__ float gelu_grad_f(float x) {
  const float k2 = 2.0f * 0.7978845608028654f;
  const float z = k2 * fmaf(0.044715f * x, x * x, x);
  const float sg = 1.0f / (1.0f + __expf(-z));
  const float dz = k2 * fmaf(3.0f * 0.044715f, x * x, 1.0f);
  return sg + x * sg * (1.0f - sg) * dz;
}

// One dense layer on the wave's LDS activations.  act: [64][kActStride] bf16
// (K columns used); wl: packed weights in LDS; acc[t][n]: D tiles.
template <int K, int N>
__device__ __forceinline__ void mfma_layer(const __bf16 *act, const __bf16 *wl, const float *bias,
                                           f32x16_t (&acc)[2][N / 32], int lane) {
#pragma unroll
  for (int n = 0; n < N / 32; ++n) {
    const float bv = bias[32 * n + mfma_d_col(lane)];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[t][n][r] = bv;
  }
#pragma unroll
  for (int kc = 0; kc < K / 16; ++kc) {
    bf16x8_t a[2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
      a[t] = *(const bf16x8_t *)(act + (32 * t + mfma_a_row(lane)) * kActStride + 16 * kc + mfma_k0(lane));
#pragma unroll
    for (int n = 0; n < N / 32; ++n) {
      const bf16x8_t b = *(const bf16x8_t *)(wl + ((kc * (N / 32) + n) * 64 + lane) * 8);
#pragma unroll
      for (int t = 0; t < 2; ++t) acc[t][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[t], b, acc[t][n], 0, 0, 0);
    }
  }
}

// Where the training forward keeps its intermediates (per sample, 288
// floats): standardized input as rounded to bf16 [32], z1 [64], h1 [64],
// z2 [64], h2 [64].  Null for inference.
constexpr int kSaveX = 0, kSaveZ1 = 32, kSaveH1 = 96, kSaveZ2 = 160, kSaveH2 = 224, kSaveFloats = 288;

// Orders LDS traffic of one wave: all earlier LDS accesses complete before
// later ones issue, and the compiler may not move memory accesses across.
__device__ __forceinline__ void wave_lds_sync() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// GELU of hidden accumulators, written back as the next layer's bf16
// activations (and, when training, z and h to `save`).
__device__ __forceinline__ void hidden_out(__bf16 *act, const f32x16_t (&acc)[2][2], const float2 *gtab, int lane,
                                           float *save, int64_t row0, int zoff, int hoff, int64_t nvalid) {
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int n = 0; n < 2; ++n)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 32 * t + mfma_d_row(lane, r), col = 32 * n + mfma_d_col(lane);
        const float z = acc[t][n][r];
        const __bf16 hb = (__bf16)gelu_tab(z, gtab);
        act[row * kActStride + col] = hb;
        if (save && row0 + row < nvalid) {
          save[(row0 + row) * kSaveFloats + zoff + col] = z;
          save[(row0 + row) * kSaveFloats + hoff + col] = (float)hb;
        }
      }
}

// Network forward for one wave: lane v brings the 19 standardized inputs of
// its voxel or sample v (x) and receives the 19 raw outputs before
// de-standardization (yt).  act is the wave's LDS region, wl the packed
// weights in LDS, bias the b1|b2|b3 array.  With `save`, intermediates of
// rows row0.. (< nvalid) go to the training buffer.
__device__ __forceinline__ void mlp_forward_wave(const float (&x)[Q], float (&yt)[Q], __bf16 *act,
                                                 const __bf16 *wl, const float *bias, int lane,
                                                 float *save = nullptr, int64_t row0 = 0,
                                                 int64_t nvalid = 0) {
#pragma unroll
  for (int k = 0; k < kMlpInPad; ++k) {
    const __bf16 v = (__bf16)(k < Q ? x[k] : 0.0f);
    act[lane * kActStride + k] = v;
    if (save && row0 + lane < nvalid) save[(row0 + lane) * kSaveFloats + kSaveX + k] = (float)v;
  }
  wave_lds_sync();
  f32x16_t h[2][2];
  mfma_layer<kMlpInPad, kMlpHidden>(act, wl, bias, h, lane);
  wave_lds_sync();
  const float2 *gtab = (const float2 *)(wl + kWPackedElems);
  hidden_out(act, h, gtab, lane, save, row0, kSaveZ1, kSaveH1, nvalid);
  wave_lds_sync();
  mfma_layer<kMlpHidden, kMlpHidden>(act, wl + kW1Elems, bias + kMlpHidden, h, lane);
  wave_lds_sync();
  hidden_out(act, h, gtab, lane, save, row0, kSaveZ2, kSaveH2, nvalid);
  wave_lds_sync();
  f32x16_t o[2][1];
  mfma_layer<kMlpHidden, kMlpOutPad>(act, wl + kW1Elems + kW2Elems, bias + 2 * kMlpHidden, o, lane);
  wave_lds_sync();
  float *out = (float *)act;  // the output tile reuses the activation region
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) out[(32 * t + mfma_d_row(lane, r)) * kOutStride + mfma_d_col(lane)] = o[t][0][r];
  wave_lds_sync();
#pragma unroll
  for (int i = 0; i < Q; ++i) yt[i] = out[lane * kOutStride + i];
  wave_lds_sync();
}

// ----------------------------------------------- register-resident forward --
// Inference form of the same network with no activation traffic through LDS.
// The product is taken transposed, Z^T = W^T X^T: the weights are the A
// operand (their packed order is already the A order of W^T) and the 64
// voxels of the wave form two 32-wide B / D column tiles.  A lane then holds,
// in accumulator element r of tile (m, t), feature 32m + 8(r/4) + 4h + r%4 of
// voxel 32t + l%32 (h = lane / 32).  The next layer's B operand needs, per
// 16-feature chunk, features 8h..8h+7 of that voxel: each lane already has
// half of them, and one v_permlane32_swap per register pair exchanges the
// other half with lane l ^ 32.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
  const bf16x2_t v = {(__bf16)lo, (__bf16)hi};
  return __builtin_bit_cast(uint32_t, v);
}

// swap the upper 32 lanes of x with the lower 32 lanes of y
__device__ __forceinline__ void swap_halves(uint32_t &x, uint32_t &y) {
  const auto r = __builtin_amdgcn_permlane32_swap(x, y, false, false);
  x = r[0];
  y = r[1];
}

// bias of accumulator element r (feature 32m + 8(r/4) + 4h + r%4)
__device__ __forceinline__ void bias_init(f32x16_t &acc, const float *bias, int m, int h) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float4 b4 = *(const float4 *)(bias + 32 * m + 8 * q + 4 * h);
    acc[4 * q + 0] = b4.x;
    acc[4 * q + 1] = b4.y;
    acc[4 * q + 2] = b4.z;
    acc[4 * q + 3] = b4.w;
  }
}

// B operands (two voxel tiles) of one 16-feature chunk c of a hidden layer
// from the GELU'd accumulators of feature tile c/2.
__device__ __forceinline__ void hidden_chunk(const f32x16_t &z0, const f32x16_t &z1, int c, const float2 *gtab,
                                             bf16x8_t &b0, bf16x8_t &b1) {
  const int r0 = 8 * (c & 1);
  uint32_t x[2][2], y[2][2];  // [tile][dword]
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    x[0][k] = pack_bf16(gelu_tab(z0[r0 + 2 * k], gtab), gelu_tab(z0[r0 + 2 * k + 1], gtab));
    y[0][k] = pack_bf16(gelu_tab(z0[r0 + 4 + 2 * k], gtab), gelu_tab(z0[r0 + 4 + 2 * k + 1], gtab));
    x[1][k] = pack_bf16(gelu_tab(z1[r0 + 2 * k], gtab), gelu_tab(z1[r0 + 2 * k + 1], gtab));
    y[1][k] = pack_bf16(gelu_tab(z1[r0 + 4 + 2 * k], gtab), gelu_tab(z1[r0 + 4 + 2 * k + 1], gtab));
  }
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int k = 0; k < 2; ++k) swap_halves(x[t][k], y[t][k]);
  const u32x4_t w0 = {x[0][0], x[0][1], y[0][0], y[0][1]};
  const u32x4_t w1 = {x[1][0], x[1][1], y[1][0], y[1][1]};
  b0 = __builtin_bit_cast(bf16x8_t, w0);
  b1 = __builtin_bit_cast(bf16x8_t, w1);
}

// One output tile m of a layer: acc[t] = W^T[m] B[t] + bias over KC chunks
// of 16 inputs; bk[c][t] are the B operands of chunk c.
template <int KC, int MT>
__device__ __forceinline__ void layer_tile(const __bf16 *wl, const float *bias, const bf16x8_t (&bk)[KC][2],
                                           int m, f32x16_t (&acc)[2], int lane) {
  bias_init(acc[0], bias, m, lane >> 5);
  acc[1] = acc[0];
#pragma unroll
  for (int c = 0; c < KC; ++c) {
    const bf16x8_t a = *(const bf16x8_t *)(wl + ((c * MT + m) * 64 + lane) * 8);
#pragma unroll
    for (int t = 0; t < 2; ++t) acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bk[c][t], acc[t], 0, 0, 0);
  }
}

// Network forward of the wave's 64 voxels (lane v brings voxel v's 19
// standardized inputs x and receives its 19 raw outputs yt), weights packed
// in LDS (wl), biases b1|b2|b3 in global memory.
__device__ __forceinline__ void mlp_forward_wave_reg(const float (&x)[Q], float (&yt)[Q], const __bf16 *wl,
                                                     const float *bias, int lane) {
  const float2 *gtab = (const float2 *)(wl + kWPackedElems);
  // layer 1 operands: chunk c holds features 16c..16c+15; the lane's own
  // features 16c..16c+7 (F0) and 16c+8..16c+15 (F1) are swapped across
  // halves so that F0-slot registers form tile 0 and F1-slot registers tile 1
  bf16x8_t b1[2][2];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    uint32_t f0[4], f1[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i0 = 16 * c + 2 * k, i1 = 16 * c + 8 + 2 * k;
      f0[k] = pack_bf16(i0 < Q ? x[i0] : 0.0f, i0 + 1 < Q ? x[i0 + 1] : 0.0f);
      f1[k] = pack_bf16(i1 < Q ? x[i1] : 0.0f, i1 + 1 < Q ? x[i1 + 1] : 0.0f);
      swap_halves(f0[k], f1[k]);
    }
    const u32x4_t w0 = {f0[0], f0[1], f0[2], f0[3]};
    const u32x4_t w1 = {f1[0], f1[1], f1[2], f1[3]};
    b1[c][0] = __builtin_bit_cast(bf16x8_t, w0);
    b1[c][1] = __builtin_bit_cast(bf16x8_t, w1);
  }
  // hidden layers one 32-feature tile at a time, each tile turned into the
  // next layer's two 16-feature chunks right away
  bf16x8_t b2[4][2], b3[4][2];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    f32x16_t z[2];
    layer_tile<2, 2>(wl, bias, b1, m, z, lane);
    hidden_chunk(z[0], z[1], 2 * m, gtab, b2[2 * m][0], b2[2 * m][1]);
    hidden_chunk(z[0], z[1], 2 * m + 1, gtab, b2[2 * m + 1][0], b2[2 * m + 1][1]);
  }
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    f32x16_t z[2];
    layer_tile<4, 2>(wl + kW1Elems, bias + kMlpHidden, b2, m, z, lane);
    hidden_chunk(z[0], z[1], 2 * m, gtab, b3[2 * m][0], b3[2 * m][1]);
    hidden_chunk(z[0], z[1], 2 * m + 1, gtab, b3[2 * m + 1][0], b3[2 * m + 1][1]);
  }
  f32x16_t o[1][2];
  layer_tile<4, 1>(wl + kW1Elems + kW2Elems, bias + 2 * kMlpHidden, b3, 0, o[0], lane);
  // gather the voxel's outputs: element r (= 4q + r%4) of tile t holds
  // output 8q + 4h + r%4 of voxel 32t + l%32, so each lane keeps the half of
  // its own voxel's outputs it holds and receives the other half from lane
  // l ^ 32 (a lane shuffle: a 32-lane swap of accumulator elements was
  // merged into one by the compiler)
  const bool lo = lane < 32;
  float ox[11], oy[11];
#pragma unroll
  for (int r = 0; r < 11; ++r) {
    const float give = lo ? o[0][1][r] : o[0][0][r];
    const float recv = __shfl_xor(give, 32, 64);
    ox[r] = lo ? o[0][0][r] : recv;  // outputs 8q + r%4
    oy[r] = lo ? recv : o[0][1][r];  // outputs 8q + 4 + r%4
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int r = 4 * (i / 8) + (i & 3);
    yt[i] = (i & 4) ? oy[r] : ox[r];
  }
}

// Copies the packed weights and the GELU table (20 KB) from global memory to
// LDS (wl holds kWStageElems), and with bl the biases b1|b2|b3 too (bl holds
// kBiasFloats); every thread of the workgroup must call it before any wave
// returns.
__device__ __forceinline__ void stage_weights(__bf16 *wl, const __bf16 *wg, float *bl = nullptr,
                                              const float *bg = nullptr) {
  const uint4 *src = (const uint4 *)wg;
  uint4 *dst = (uint4 *)wl;
  for (int k = threadIdx.x; k < kWStageElems / 8; k += blockDim.x) dst[k] = src[k];
  if (bl)
    for (int k = threadIdx.x; k < kBiasFloats; k += blockDim.x) bl[k] = bg[k];
  __syncthreads();
}

// Q-weighted second moment A = sum_j Q_j y_j (Q_j = c_j c_j - c_s^2 I) as
// (xx, yy, zz, xy, xz, yz): the coordinates of y's second-order Hermite
// part, P(y) = hermite2(A).
__device__ __forceinline__ void q_stress(const float (&y)[Q], float (&a)[6]) {
  float s = y[0];
#pragma unroll
  for (int i = 1; i < Q; ++i) s = s + y[i];
  const float p78 = y[7] + y[8], p910 = y[9] + y[10], p1112 = y[11] + y[12];
  const float p1314 = y[13] + y[14], p1516 = y[15] + y[16], p1718 = y[17] + y[18];
  const float s3 = s * (1.0f / 3.0f);
  a[0] = (y[1] + y[2]) + p78 + p910 + p1112 + p1314 - s3;
  a[1] = (y[3] + y[4]) + p78 + p910 + p1516 + p1718 - s3;
  a[2] = (y[5] + y[6]) + p1112 + p1314 + p1516 + p1718 - s3;
  // the off-diagonal sums pair opposite directions (c_a c_b is even in c)
  a[3] = p78 - p910;
  a[4] = p1112 - p1314;
  a[5] = p1516 - p1718;
}

// Second-order Hermite projection, P(y)_i = w_i/(2 c_s^4) Q_i : sum_j Q_j y_j:
// keeps the stress-like part of y and drops mass, momentum and every
// higher (ghost) moment.
__device__ __forceinline__ void project_out(float (&y)[Q]) {
  float a[6];
  q_stress(y, a);
  hermite2(a[0], a[1], a[2], a[3], a[4], a[5], y);
}

}  // inline namespace
}  // namespace lbm
