// Training and utility kernels of the learned collision closure.
//
// A training step on a batch of populations f [B][19]:
//   k_mlp_fwd     per wave of 64 samples: g = (f - f^eq)/rho, standardize, network
//                 forward on the matrix cores (the inference code path),
//                 projection, squared error against the regularized target
//                 f1/rho, and the loss gradient with respect to the raw
//                 outputs (dyt); intermediates go to `save`;
//   k_mlp_bwd_mfma    per wave of 64 samples: back through layers 3 and 2
//                 (dz2, dz1) on the matrix cores with the bf16 weights the
//                 forward used;
//   k_mlp_wgrad_mfma  per chunk of 128 samples: weight gradients on the
//                 matrix cores, bias gradients as column sums, one partial
//                 gradient per chunk;
//   k_mlp_grad_final  per parameter: the chunk partials summed in order;
//   k_mlp_adam    per parameter: Adam on the FP32 master weights;
//   k_mlp_pack    master weights -> bf16 operand-order copy + biases.
// Everything is deterministic (fixed summation orders, no atomics).
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "launch.h"
#include "mlp_device.h"

namespace lbm {
inline namespace LBM_LATTICE_NS {

namespace {

__device__ __forceinline__ float bf16_value(float v) { return (float)(__bf16)v; }

// mean of out_std^2 (the loss normalization)
__device__ __forceinline__ float s2_of(const float *stdz) {
  float s2 = 0.0f;
#pragma unroll
  for (int i = 0; i < Q; ++i) s2 = fmaf(stdz[64 + i], stdz[64 + i], s2);
  return s2 * (1.0f / Q);
}

// populations f (FP32, unshifted) of one sample -> shifted h
__device__ __forceinline__ void load_sample(const float *f, int64_t k, float (&h)[Q]) {
#pragma unroll
  for (int i = 0; i < Q; ++i) h[i] = f[k * Q + i] - weight_f(i);
}

// standardized closure inputs x = ((f - f^eq)/rho - mean) / std and the moments
__device__ __forceinline__ Moments closure_inputs(const float (&h)[Q], const float *stdz, float (&x)[Q],
                                                  bool &out_of_range) {
  const Moments m = moments(h);
  float heq[Q];
  equilibrium(m, heq);
  const float ir = 1.0f / m.rho;
  out_of_range = false;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float g = (h[i] - heq[i]) * ir;
    x[i] = (g - stdz[i]) * stdz[32 + i];
    out_of_range = out_of_range || fabsf(x[i]) > 8.0f;
  }
  return m;
}

}  // namespace

// ------------------------------------------------------------ forward/loss --
__global__ __launch_bounds__(256) void k_mlp_fwd(const float *f, const int64_t *idx, int64_t n, const __bf16 *wg,
                                                 const float *bias, const float *stdz, float *save,
                                                 float *dyt, float *yout, double *partial) {
  __shared__ __attribute__((aligned(16))) __bf16 wl[kWStageElems];
  __shared__ __attribute__((aligned(16))) __bf16 act[4][64 * kActStride];
  stage_weights(wl, wg);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * 64;
  const int64_t k = row0 + lane;
  const bool valid = k < n;
  float h[Q], x[Q], yt[Q];
  if (valid) load_sample(f, idx ? idx[k] : k, h);
  else
#pragma unroll
    for (int i = 0; i < Q; ++i) h[i] = 0.0f;
  bool oor;
  const Moments m = closure_inputs(h, stdz, x, oor);
  mlp_forward_wave(x, yt, act[wave], wl, bias, lane, save, row0, save ? n : 0);
  float y[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) y[i] = fmaf(yt[i], stdz[64 + i], stdz[96 + i]);
  if (yout && valid)
#pragma unroll
    for (int i = 0; i < Q; ++i) yout[k * Q + i] = y[i];
  if (!dyt) return;
  // target: the regularized non-equilibrium part per unit density
  float f1[Q];
  f1_projection(h, m, f1);
  const float ir = 1.0f / m.rho;
  project_out(y);
  float d[Q];
  double e = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    d[i] = valid ? y[i] - f1[i] * ir : 0.0f;
    e += (double)d[i] * (double)d[i];
  }
  e = e / (double)s2_of(stdz);
  // loss = mean d^2 / s2 with s2 the mean target variance (scale-free loss);
  // dL/dP = 2 d / (n 19 s2).  With P = M y, M_ij = w_i (Q_i : Q_j) / (2 c_s^4),
  // dL/dy_j = sum_i dL/dP_i M_ij = P(w o dL/dP)_j / w_j.
  const float s2 = s2_of(stdz);
  const float sc = 2.0f / ((float)(n * Q) * s2);
  float z[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) z[i] = d[i] * sc * weight_f(i);
  project_out(z);
  if (valid)
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const float inv_w = i == 0 ? 3.0f : (i < 7 ? 18.0f : 36.0f);
      dyt[k * Q + i] = z[i] * inv_w * stdz[64 + i];
    }
  for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
  if (lane == 0 && partial) partial[blockIdx.x * 4 + wave] = e;
}

// ---------------------------------------------- matrix-core backward pass --
// Products C[m][n] = sum_k A[m][k] B[n][k] of bf16 operands held in LDS as
// rows (A: [M][lda], B: [N][ldb], k contiguous, FP32 accumulation) on
// v_mfma_f32_32x32x16_bf16: lane l loads A row m0 + l%32 and B row
// n0 + l%32, eight k values each from k0 + 8 (l/32); element r of the
// result tile is C[m0 + 8(r/4) + 4(l/32) + r%4][n0 + l%32].
__device__ __forceinline__ void mfma_nt(const __bf16 *A, int lda, int m0, const __bf16 *B, int ldb, int n0, int K,
                                        f32x16_t &acc, int lane) {
  const __bf16 *pa = A + (m0 + (lane & 31)) * lda + 8 * (lane >> 5);
  const __bf16 *pb = B + (n0 + (lane & 31)) * ldb + 8 * (lane >> 5);
  for (int k = 0; k < K; k += 16) {
    const bf16x8_t a = *(const bf16x8_t *)(pa + k);
    const bf16x8_t b = *(const bf16x8_t *)(pb + k);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
}

__device__ __forceinline__ int tile_row(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

constexpr int kBwdRows = 64;                 // samples per wave
constexpr int kLd32 = 32 + 8, kLd64 = 64 + 8;  // LDS row strides (bf16), padded against bank conflicts

// Back through layers 3 and 2 for 256 samples per workgroup (64 per wave):
//   dz2 = (dyt W3^T) o gelu'(z2),  dz1 = (dz2 W2^T) o gelu'(z1),
// products on the matrix cores with the bf16 weights the forward used and
// dyt, dz2 rounded to bf16; dz1 and dz2 leave in FP32.
__global__ __launch_bounds__(256) void k_mlp_bwd_mfma(int64_t n, const float *params, const float *save,
                                                      const float *dyt, float *dz1, float *dz2) {
  __shared__ __attribute__((aligned(16))) __bf16 w3[64 * kLd32];   // W3 [a][j]
  __shared__ __attribute__((aligned(16))) __bf16 w2[64 * kLd64];   // W2 [a][b]
  __shared__ __attribute__((aligned(16))) __bf16 rows[4][kBwdRows * kLd64];  // per wave: dyt, then dz2
  for (int k = threadIdx.x; k < 64 * 32; k += blockDim.x) {
    const int a = k >> 5, j = k & 31;
    w3[a * kLd32 + j] = (__bf16)(j < Q ? params[kMlpW3 + a * 19 + j] : 0.0f);
  }
  for (int k = threadIdx.x; k < 64 * 64; k += blockDim.x) w2[(k >> 6) * kLd64 + (k & 63)] = (__bf16)params[kMlpW2 + k];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * kBwdRows;
  __bf16 *rw = rows[wave];
  // this wave's dyt rows [64][32], zero beyond the batch and beyond 19
  for (int k = lane; k < kBwdRows * 32; k += 64) {
    const int si = k >> 5, j = k & 31;
    const int64_t sg = row0 + si;
    rw[si * kLd32 + j] = (__bf16)(sg < n && j < Q ? dyt[sg * Q + j] : 0.0f);
  }
  __syncthreads();
  // dz2 tiles: samples 32t.., features 32u..
  f32x16_t acc[2][2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      acc[t][u] = {};
      mfma_nt(rw, kLd32, 32 * t, w3, kLd32, 32 * u, 32, acc[t][u], lane);
    }
  wave_lds_sync();  // the dyt rows are read; the region now takes dz2
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int si = 32 * t + tile_row(lane, r), a = 32 * u + (lane & 31);
        const int64_t sg = row0 + si;
        float d = 0.0f;
        if (sg < n) {
          d = acc[t][u][r] * gelu_grad_f(save[sg * kSaveFloats + kSaveZ2 + a]);
          dz2[sg * 64 + a] = d;
        }
        rw[si * kLd64 + a] = (__bf16)d;
      }
  wave_lds_sync();
  // dz1 tiles
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      acc[t][u] = {};
      mfma_nt(rw, kLd64, 32 * t, w2, kLd64, 32 * u, 64, acc[t][u], lane);
    }
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int si = 32 * t + tile_row(lane, r), a = 32 * u + (lane & 31);
        const int64_t sg = row0 + si;
        if (sg < n) dz1[sg * 64 + a] = acc[t][u][r] * gelu_grad_f(save[sg * kSaveFloats + kSaveZ1 + a]);
      }
}

constexpr int kWgradChunk = 128;          // samples per workgroup of the weight-gradient pass
constexpr int kLdS = kWgradChunk + 8;     // LDS row stride (bf16) of transposed operands

// Stages rows [s0, s0 + kWgradChunk) of a [n][ld] FP32 array, columns
// [c0, c0 + cols) (zero beyond nc valid columns and beyond the batch), into
// LDS transposed: dst[c][s] in bf16.
__device__ __forceinline__ void stage_t(__bf16 *dst, int rowsd, const float *src, int ld, int c0, int nc, int64_t s0,
                                        int64_t n) {
  for (int k = threadIdx.x; k < rowsd * kWgradChunk; k += blockDim.x) {
    const int c = k / kWgradChunk, si = k % kWgradChunk;
    const int64_t sg = s0 + si;
    dst[c * kLdS + si] = (__bf16)(sg < n && c < nc ? src[sg * ld + c0 + c] : 0.0f);
  }
}

// Weight and bias gradients of one chunk of kWgradChunk samples, into
// partial[chunk][kMlpParams]:
//   W1[i][a] = sum x_i dz1_a,  W2[a][b] = sum h1_a dz2_b,  W3[a][j] = sum h2_a dyt_j
// as matrix-core products over the chunk (bf16 operands, FP32 accumulation),
// biases as FP32 column sums in sample order.
__global__ __launch_bounds__(256) void k_mlp_wgrad_mfma(int64_t n, const float *save, const float *dyt,
                                                        const float *dz1, const float *dz2, float *partial) {
  __shared__ __attribute__((aligned(16))) __bf16 lds[(32 + 64 + 64 + 32) * kLdS];
  __bf16 *sx = lds, *sd1 = lds + 32 * kLdS, *sh2 = lds + 96 * kLdS, *sdy = lds + 160 * kLdS;
  const int64_t s0 = (int64_t)blockIdx.x * kWgradChunk;
  float *out = partial + (size_t)blockIdx.x * kMlpParams;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // phase 1: W1 (waves 0, 1) and W3 (waves 2, 3)
  stage_t(sx, 32, save, kSaveFloats, kSaveX, Q, s0, n);
  stage_t(sd1, 64, dz1, 64, 0, 64, s0, n);
  stage_t(sh2, 64, save, kSaveFloats, kSaveH2, 64, s0, n);
  stage_t(sdy, 32, dyt, Q, 0, Q, s0, n);
  __syncthreads();
  {
    f32x16_t acc = {};
    if (wave < 2) {  // W1 tile: inputs 0..31 x features 32 wave..
      mfma_nt(sx, kLdS, 0, sd1, kLdS, 32 * wave, kWgradChunk, acc, lane);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = tile_row(lane, r), a = 32 * wave + (lane & 31);
        if (i < Q) out[kMlpW1 + i * 64 + a] = acc[r];
      }
    } else {  // W3 tile: features 32 (wave - 2).. x outputs 0..31
      mfma_nt(sh2, kLdS, 32 * (wave - 2), sdy, kLdS, 0, kWgradChunk, acc, lane);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int a = 32 * (wave - 2) + tile_row(lane, r), j = lane & 31;
        if (j < Q) out[kMlpW3 + a * 19 + j] = acc[r];
      }
    }
  }
  // biases: column sums in sample order (FP32)
  {
    const int t = threadIdx.x;
    const int64_t s1 = s0 + kWgradChunk < n ? s0 + kWgradChunk : n;
    float acc = 0.0f;
    if (t < 64) {
      for (int64_t sg = s0; sg < s1; ++sg) acc += dz1[sg * 64 + t];
      out[kMlpB1 + t] = acc;
    } else if (t < 128) {
      for (int64_t sg = s0; sg < s1; ++sg) acc += dz2[sg * 64 + (t - 64)];
      out[kMlpB2 + t - 64] = acc;
    } else if (t < 128 + Q) {
      for (int64_t sg = s0; sg < s1; ++sg) acc += dyt[sg * Q + (t - 128)];
      out[kMlpB3 + t - 128] = acc;
    }
  }
  __syncthreads();
  // phase 2: W2 (one 32x32 tile per wave)
  __bf16 *sh1 = lds, *sd2 = lds + 64 * kLdS;
  stage_t(sh1, 64, save, kSaveFloats, kSaveH1, 64, s0, n);
  stage_t(sd2, 64, dz2, 64, 0, 64, s0, n);
  __syncthreads();
  f32x16_t acc = {};
  const int mt = wave >> 1, nt = wave & 1;
  mfma_nt(sh1, kLdS, 32 * mt, sd2, kLdS, 32 * nt, kWgradChunk, acc, lane);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int a = 32 * mt + tile_row(lane, r), b = 32 * nt + (lane & 31);
    out[kMlpW2 + a * 64 + b] = acc[r];
  }
}

// Sum of the chunk partials in chunk order.
__global__ void k_mlp_grad_final(const float *partial, int nchunks, float *grads) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpParams) return;
  float acc = 0.0f;
  for (int c = 0; c < nchunks; ++c) acc += partial[(size_t)c * kMlpParams + p];
  grads[p] = acc;
}

__global__ void k_loss_final(const double *partial, int64_t nw, int64_t n, double *loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double e = 0.0;
  for (int64_t k = 0; k < nw; ++k) e += partial[k];
  *loss = e / (double)(n * Q);
}

// -------------------------------------------------------------- optimizer --
__global__ void k_mlp_adam(float *params, const float *grads, float *m, float *v, float lr, float b1c,
                           float b2c) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpParams) return;
  const float g = grads[p];
  const float mm = 0.9f * m[p] + 0.1f * g;
  const float vv = 0.999f * v[p] + 0.001f * g * g;
  m[p] = mm;
  v[p] = vv;
  params[p] -= lr * (mm / b1c) / (sqrtf(vv / b2c) + 1e-8f);
}

// splitmix64 (Steele, Lea and Flood 2014), a counter-based generator.
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// He-uniform initial weights U(-sqrt(6/fan_in), +sqrt(6/fan_in)), zero
// biases; parameter p draws 53 bits of splitmix64(seed ^ splitmix64(p)).
__global__ void k_mlp_init(float *params, uint64_t seed) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpParams) return;
  constexpr double kLim19 = 0.5619514869490163;   // sqrt(6/19)
  constexpr double kLim64 = 0.30618621784789724;  // sqrt(6/64)
  double lim = 0.0;
  if (p < kMlpB1) lim = kLim19;
  else if ((p >= kMlpW2 && p < kMlpB2) || (p >= kMlpW3 && p < kMlpB3)) lim = kLim64;
  const uint64_t r = mix64(seed ^ mix64((uint64_t)p));
  const double u = (double)(r >> 11) * (1.0 / 9007199254740992.0);  // [0, 1)
  params[p] = (float)((2.0 * u - 1.0) * lim);
}

// master weights -> packed bf16 operand order and padded biases
__global__ void k_mlp_pack(const float *params, __bf16 *wp, float *bias) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < kMlpInPad * kMlpHidden) {  // W1 padded to 32 rows
    const int k = t / kMlpHidden, a = t % kMlpHidden;
    wp[packed_index(k, a, kMlpHidden)] = (__bf16)(k < Q ? params[kMlpW1 + k * 64 + a] : 0.0f);
  }
  if (t < kMlpHidden * kMlpHidden) {
    const int k = t / 64, a = t % 64;
    wp[kW1Elems + packed_index(k, a, kMlpHidden)] = (__bf16)params[kMlpW2 + k * 64 + a];
  }
  if (t < kMlpHidden * kMlpOutPad) {  // W3 padded to 32 columns
    const int k = t / kMlpOutPad, j = t % kMlpOutPad;
    wp[kW1Elems + kW2Elems + packed_index(k, j, kMlpOutPad)] = (__bf16)(j < Q ? params[kMlpW3 + k * 19 + j] : 0.0f);
  }
  if (t < 64) {
    bias[t] = params[kMlpB1 + t];
    bias[64 + t] = params[kMlpB2 + t];
  }
  if (t < 32) bias[128 + t] = t < Q ? params[kMlpB3 + t] : 0.0f;
}

// ------------------------------------------------------ standardization --
// Per-component mean and standard deviation of the inputs g = (f - f^eq)/rho
// and of the targets f1/rho, FP64 sums in a fixed order.
__global__ __launch_bounds__(256) void k_stats_partial(const float *f, int64_t n, double *partial) {
  __shared__ double sh[256];
  double acc[4 * Q];
  for (int k = 0; k < 4 * Q; ++k) acc[k] = 0.0;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x) {
    float h[Q], f1[Q];
    load_sample(f, s, h);
    const Moments m = moments(h);
    float heq[Q];
    equilibrium(m, heq);
    f1_projection(h, m, f1);
    const float ir = 1.0f / m.rho;
    for (int i = 0; i < Q; ++i) {
      const double g = (double)((h[i] - heq[i]) * ir);
      const double t = (double)(f1[i] * ir);
      acc[i] += g;
      acc[Q + i] += g * g;
      acc[2 * Q + i] += t;
      acc[3 * Q + i] += t * t;
    }
  }
  for (int k = 0; k < 4 * Q; ++k) {
    sh[threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * 4 * Q + k] = sh[0];
    __syncthreads();
  }
}

__global__ void k_stats_final(const double *partial, int nblk, int64_t n, float *stdz) {
  const int i = threadIdx.x;
  if (i >= 32) return;
  if (i >= Q) {
    stdz[i] = 0.0f;
    stdz[32 + i] = 1.0f;
    stdz[64 + i] = 1.0f;
    stdz[96 + i] = 0.0f;
    return;
  }
  double s[4] = {0, 0, 0, 0};
  for (int b = 0; b < nblk; ++b)
    for (int k = 0; k < 4; ++k) s[k] += partial[(int64_t)b * 4 * Q + k * Q + i];
  const double mg = s[0] / n, vg = fmax(s[1] / n - mg * mg, 0.0);
  const double mt = s[2] / n, vt = fmax(s[3] / n - mt * mt, 0.0);
  const double sg = sqrt(vg) > 1e-12 ? sqrt(vg) : 1.0;
  const double st = sqrt(vt) > 1e-12 ? sqrt(vt) : 1.0;
  stdz[i] = (float)mg;
  stdz[32 + i] = (float)(1.0 / sg);
  stdz[64 + i] = (float)st;
  stdz[96 + i] = (float)mt;
}

// sum of out_std^2 in the order of s2_of, for the solver's judge
__global__ void k_mlp_derive(const float *stdz, float *s2) {
  float v = 0.0f;
  for (int i = 0; i < Q; ++i) v = fmaf(stdz[64 + i], stdz[64 + i], v);
  *s2 = v;
}

// ---------------------------------------------------------------- launch --
static int64_t waves_blocks(int64_t n) { return (n + 255) / 256; }

hipError_t mlp_pack(const MlpBuffers &B, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_pack, dim3(16), dim3(256), 0, s, B.params, (__bf16 *)B.wpacked, B.bias);
  return hipGetLastError();
}

hipError_t mlp_fit_standardization(const MlpBuffers &B, const float *f, int64_t n, hipStream_t s) {
  const int nblk = 64;
  hipLaunchKernelGGL(k_stats_partial, dim3(nblk), dim3(256), 0, s, f, n, B.partial);
  hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(32), 0, s, B.partial, nblk, n, B.stdz);
  return mlp_derive(B, s);
}

hipError_t mlp_derive(const MlpBuffers &B, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_derive, dim3(1), dim3(1), 0, s, (const float *)B.stdz, B.s2);
  return hipGetLastError();
}

hipError_t mlp_forward(const MlpBuffers &B, const float *f, int64_t n, float *y, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_fwd, dim3((unsigned)waves_blocks(n)), dim3(256), 0, s, f, (const int64_t *)nullptr, n,
                     (const __bf16 *)B.wpacked, B.bias, B.stdz, (float *)nullptr, (float *)nullptr, y,
                     (double *)nullptr);
  return hipGetLastError();
}

hipError_t mlp_gradients(const MlpBuffers &B, const float *f, const int64_t *idx, int64_t n, double *loss,
                         hipStream_t s) {
  if (n <= 0 || n > B.batch_max) return hipErrorInvalidValue;
  const unsigned nb = (unsigned)waves_blocks(n);
  hipLaunchKernelGGL(k_mlp_fwd, dim3(nb), dim3(256), 0, s, f, idx, n, (const __bf16 *)B.wpacked, B.bias, B.stdz,
                     B.save, B.dyt, (float *)nullptr, B.partial);
  hipLaunchKernelGGL(k_mlp_bwd_mfma, dim3(nb), dim3(256), 0, s, n, B.params, B.save, B.dyt, B.dz1, B.dz2);
  const int nchunks = (int)((n + kWgradChunk - 1) / kWgradChunk);
  hipLaunchKernelGGL(k_mlp_wgrad_mfma, dim3(nchunks), dim3(256), 0, s, n, B.save, B.dyt, B.dz1, B.dz2, B.gpartial);
  hipLaunchKernelGGL(k_mlp_grad_final, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, B.gpartial, nchunks,
                     B.grads);
  if (loss) hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, B.partial, (int64_t)nb * 4, n, loss);
  return hipGetLastError();
}

hipError_t mlp_adam(const MlpBuffers &B, const float *grads, float lr, int32_t t, hipStream_t s) {
  const float b1c = 1.0f - powf(0.9f, (float)t), b2c = 1.0f - powf(0.999f, (float)t);
  hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, B.params, grads, B.adam_m,
                     B.adam_v, lr, b1c, b2c);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return mlp_pack(B, s);
}

hipError_t mlp_init(const MlpBuffers &B, uint64_t seed, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_init, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, B.params, seed);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return mlp_pack(B, s);
}

}  // inline namespace
}  // namespace lbm
