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
  unsigned int *fallbacks;  // fallback counter
};

// tanh-form GELU, written as x * sigmoid(2 sqrt(2/pi) (x + 0.044715 x^3))
__device__ __forceinline__ float gelu_f(float x) {
  const float k2 = 2.0f * 0.7978845608028654f;
  const float z = k2 * fmaf(0.044715f * x, x * x, x);
  // x * sigmoid(2z) with the hardware reciprocal (about 1 ulp; the result
  // is rounded to bf16 for the next layer) instead of an IEEE division
  return x * __builtin_amdgcn_rcpf(1.0f + __expf(-z));
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
__device__ __forceinline__ void hidden_out(__bf16 *act, const f32x16_t (&acc)[2][2], int lane,
                                           float *save, int64_t row0, int zoff, int hoff, int64_t nvalid) {
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int n = 0; n < 2; ++n)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 32 * t + mfma_d_row(lane, r), col = 32 * n + mfma_d_col(lane);
        const float z = acc[t][n][r];
        const __bf16 hb = (__bf16)gelu_f(z);
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
  hidden_out(act, h, lane, save, row0, kSaveZ1, kSaveH1, nvalid);
  wave_lds_sync();
  mfma_layer<kMlpHidden, kMlpHidden>(act, wl + kW1Elems, bias + kMlpHidden, h, lane);
  wave_lds_sync();
  hidden_out(act, h, lane, save, row0, kSaveZ2, kSaveH2, nvalid);
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

// Copies the packed weights (16 KB) from global memory to LDS; every thread
// of the workgroup must call it before any wave returns.
__device__ __forceinline__ void stage_weights(__bf16 *wl, const __bf16 *wg) {
  const uint4 *src = (const uint4 *)wg;
  uint4 *dst = (uint4 *)wl;
  for (int k = threadIdx.x; k < kWPackedElems / 8; k += blockDim.x) dst[k] = src[k];
  __syncthreads();
}

// Second-order Hermite projection, P(y)_i = w_i/(2 c_s^4) Q_i : sum_j Q_j y_j:
// keeps the stress-like part of y and drops mass, momentum and every
// higher (ghost) moment.
__device__ __forceinline__ void project_out(float (&y)[Q]) {
  float s = y[0];
#pragma unroll
  for (int i = 1; i < Q; ++i) s = s + y[i];
  const float p78 = y[7] + y[8], p910 = y[9] + y[10], p1112 = y[11] + y[12];
  const float p1314 = y[13] + y[14], p1516 = y[15] + y[16], p1718 = y[17] + y[18];
  const float s3 = s * (1.0f / 3.0f);
  const float pxx = (y[1] + y[2]) + p78 + p910 + p1112 + p1314 - s3;
  const float pyy = (y[3] + y[4]) + p78 + p910 + p1516 + p1718 - s3;
  const float pzz = (y[5] + y[6]) + p1112 + p1314 + p1516 + p1718 - s3;
  // the off-diagonal sums pair opposite directions (c_a c_b is even in c)
  const float pxy = p78 - p910, pxz = p1112 - p1314, pyz = p1516 - p1718;
  hermite2(pxx, pyy, pzz, pxy, pxz, pyz, y);
}

}  // inline namespace
}  // namespace lbm
