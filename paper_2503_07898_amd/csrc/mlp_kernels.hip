// Training and utility kernels of the learned collision closure.
//
// A training step on a batch of populations f [B][19]:
//   k_mlp_fwd     per wave of 64 samples: g = (f - f^eq)/rho, standardize, network
//                 forward on the matrix cores (the inference code path),
//                 projection, squared error against the regularized target
//                 f1/rho, and the loss gradient with respect to the raw
//                 outputs (dyt); intermediates go to `save`;
//   k_mlp_bwd     per sample: back through layers 3 and 2 (dz2, dz1) with the
//                 bf16 weights the forward used;
//   k_mlp_wgrad   per parameter: sums over the batch in a fixed order;
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
  __shared__ __attribute__((aligned(16))) __bf16 wl[kWPackedElems];
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

// ------------------------------------------------------- hidden backward --
// W2 and W3 as the forward used them (rounded to bf16), from the masters.
__global__ __launch_bounds__(256) void k_mlp_bwd(int64_t n, const float *params, const float *save,
                                                 const float *dyt, float *dz1, float *dz2) {
  __shared__ float w2[64 * 64], w3[64 * 19];
  for (int k = threadIdx.x; k < 64 * 64; k += blockDim.x) w2[k] = bf16_value(params[kMlpW2 + k]);
  for (int k = threadIdx.x; k < 64 * 19; k += blockDim.x) w3[k] = bf16_value(params[kMlpW3 + k]);
  __syncthreads();
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const float *sv = save + s * kSaveFloats;
  float g[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) g[j] = dyt[s * Q + j];
  float d2[64];
  for (int a = 0; a < 64; ++a) {
    float acc = 0.0f;
#pragma unroll
    for (int j = 0; j < Q; ++j) acc = fmaf(g[j], w3[a * 19 + j], acc);
    const float z = sv[kSaveZ2 + a];
    d2[a] = acc * gelu_grad_f(z);
    dz2[s * 64 + a] = d2[a];
  }
  for (int a = 0; a < 64; ++a) {
    float acc = 0.0f;
    for (int b = 0; b < 64; ++b) acc = fmaf(d2[b], w2[a * 64 + b], acc);
    dz1[s * 64 + a] = acc * gelu_grad_f(sv[kSaveZ1 + a]);
  }
}

// --------------------------------------------------------- weight grads --
__global__ __launch_bounds__(256) void k_mlp_wgrad(int64_t n, const float *save, const float *dyt,
                                                   const float *dz1, const float *dz2, float *grads) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpParams) return;
  float acc = 0.0f;
  if (p < kMlpB1) {  // W1[i][a] = sum x_i dz1_a
    const int i = p / 64, a = p % 64;
    for (int64_t s = 0; s < n; ++s) acc = fmaf(save[s * kSaveFloats + kSaveX + i], dz1[s * 64 + a], acc);
  } else if (p < kMlpW2) {
    const int a = p - kMlpB1;
    for (int64_t s = 0; s < n; ++s) acc += dz1[s * 64 + a];
  } else if (p < kMlpB2) {  // W2[a][b] = sum h1_a dz2_b
    const int a = (p - kMlpW2) / 64, b = (p - kMlpW2) % 64;
    for (int64_t s = 0; s < n; ++s) acc = fmaf(save[s * kSaveFloats + kSaveH1 + a], dz2[s * 64 + b], acc);
  } else if (p < kMlpW3) {
    const int b = p - kMlpB2;
    for (int64_t s = 0; s < n; ++s) acc += dz2[s * 64 + b];
  } else if (p < kMlpB3) {  // W3[a][j] = sum h2_a dyt_j
    const int a = (p - kMlpW3) / 19, j = (p - kMlpW3) % 19;
    for (int64_t s = 0; s < n; ++s) acc = fmaf(save[s * kSaveFloats + kSaveH2 + a], dyt[s * Q + j], acc);
  } else {
    const int j = p - kMlpB3;
    for (int64_t s = 0; s < n; ++s) acc += dyt[s * Q + j];
  }
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
  hipLaunchKernelGGL(k_mlp_bwd, dim3(nb), dim3(256), 0, s, n, B.params, B.save, B.dyt, B.dz1, B.dz2);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, n, B.save, B.dyt, B.dz1,
                     B.dz2, B.grads);
  if (loss) hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, B.partial, (int64_t)nb * 4, n, loss);
  return hipGetLastError();
}

hipError_t mlp_adam(const MlpBuffers &B, float lr, int32_t t, hipStream_t s) {
  const float b1c = 1.0f - powf(0.9f, (float)t), b2c = 1.0f - powf(0.999f, (float)t);
  hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, B.params, B.grads, B.adam_m,
                     B.adam_v, lr, b1c, b2c);
  return mlp_pack(B, s);
}

}  // inline namespace
}  // namespace lbm
