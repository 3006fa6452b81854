// Off-hot-path kernels of liblbm: equilibrium initialisation, macroscopic
// read-out, population checkpoint read/write and FP64 reductions.  All of
// them visit slots in storage order and exchange data in canonical order
// through the slot -> canonical index map.
#include <hip/hip_runtime.h>

#include <mutex>

#include "device_common.h"
#include "launch.h"

namespace lbm {
inline namespace LBM_LATTICE_NS {

__device__ __forceinline__ int64_t canon_of(const SlotArgs &A, int64_t slot) {
  return A.canon ? (int64_t)A.canon[slot] : slot;
}

// index of population i of a slot: block-interleaved for block layouts,
// separate planes for the dense lexicographic arm
__device__ __forceinline__ size_t uidx(const SlotArgs &A, int i, int64_t slot) {
  return A.blocked ? pidx(i, (uint32_t)slot) : (size_t)i * A.S + (size_t)slot;
}

// FP64 equilibrium, shifted: f^eq_i - w_i = w_i (drho + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u))
template <class ST>
__global__ void k_init_eq(SlotArgs A, const double *rho, const double *u) {
  using T = typename ST::T;
  const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= A.nslots) return;
  const int64_t c = canon_of(A, slot);
  T *pa = (T *)A.pop_a, *pb = (T *)A.pop_b;
  if (c < 0) {
    for (int i = 0; i < Q; ++i) {
      pa[uidx(A, i, slot)] = ST::from_double(0.0);
      pb[uidx(A, i, slot)] = ST::from_double(0.0);
    }
    return;
  }
  const double r = rho[c], ux = u[c], uy = u[A.n + c], uz = u[2 * A.n + c];
  const double uu = ux * ux + uy * uy + uz * uz;
  for (int i = 0; i < Q; ++i) {
    const double cu = kCx[i] * ux + kCy[i] * uy + kCz[i] * uz;
    const double h = weight_d(i) * ((r - 1.0) + r * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
    const T v = ST::from_double(h);
    pa[uidx(A, i, slot)] = v;
    pb[uidx(A, i, slot)] = v;
  }
}

template <class ST>
__global__ void k_read_macro(SlotArgs A, void *rho_out, void *u_out, int f64) {
  using T = typename ST::T;
  const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= A.nslots) return;
  const int64_t c = canon_of(A, slot);
  if (c < 0) return;
  const T *p = (const T *)A.pop_a;
  double d = 0, jx = 0, jy = 0, jz = 0;
  for (int i = 0; i < Q; ++i) {
    const double h = ST::to_double(p[uidx(A, i, slot)]);
    d += h;
    jx += kCx[i] * h;
    jy += kCy[i] * h;
    jz += kCz[i] * h;
  }
  const double r = 1.0 + d;
  const double ir = 1.0 / r;  // one FP64 division per voxel
  if (f64) {
    double *ro = (double *)rho_out, *uo = (double *)u_out;
    ro[c] = r;
    uo[c] = jx * ir;
    uo[A.n + c] = jy * ir;
    uo[2 * A.n + c] = jz * ir;
  } else {
    float *ro = (float *)rho_out, *uo = (float *)u_out;
    ro[c] = (float)r;
    uo[c] = (float)(jx * ir);
    uo[A.n + c] = (float)(jy * ir);
    uo[2 * A.n + c] = (float)(jz * ir);
  }
}

template <class ST>
__global__ void k_read_pop(SlotArgs A, double *f) {
  using T = typename ST::T;
  const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= A.nslots) return;
  const int64_t c = canon_of(A, slot);
  if (c < 0) return;
  const T *p = (const T *)A.pop_a;
  for (int i = 0; i < Q; ++i) f[(size_t)i * A.n + c] = weight_d(i) + ST::to_double(p[uidx(A, i, slot)]);
}

template <class ST>
__global__ void k_write_pop(SlotArgs A, const double *f) {
  using T = typename ST::T;
  const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= A.nslots) return;
  const int64_t c = canon_of(A, slot);
  if (c < 0) return;
  T *p = (T *)A.pop_a;
  for (int i = 0; i < Q; ++i) p[uidx(A, i, slot)] = ST::from_double(f[(size_t)i * A.n + c] - weight_d(i));
}

// Sums of one 64-slot row (mass, momentum, kinetic energy), computed by one
// wave: per-lane moments, then a butterfly in a fixed order.  Every lane
// ends with the same five totals.
template <class ST>
__device__ __forceinline__ void row_sums(const SlotArgs &A, int64_t row, int lane, double (&v)[5]) {
  using T = typename ST::T;
  const int64_t slot = row * 64 + lane;
  for (int k = 0; k < 5; ++k) v[k] = 0.0;
  if (slot < A.nslots && canon_of(A, slot) >= 0) {
    const T *p = (const T *)A.pop_a;
    double d = 0, jx = 0, jy = 0, jz = 0;
    for (int i = 0; i < Q; ++i) {
      const double h = ST::to_double(p[uidx(A, i, slot)]);
      d += h;
      jx += kCx[i] * h;
      jy += kCy[i] * h;
      jz += kCz[i] * h;
    }
    const double r = 1.0 + d;
    v[0] = r;
    v[1] = jx;
    v[2] = jy;
    v[3] = jz;
    v[4] = 0.5 * (jx * jx + jy * jy + jz * jz) / r;
  }
  for (int k = 0; k < 5; ++k) {
    double x = v[k];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    v[k] = x;
  }
}

// Per 64-slot row partial sums, times weight; one wave per row.
template <class ST>
__global__ __launch_bounds__(256) void k_reduce_partial(SlotArgs A, double weight, double *partial) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);  // one row of 64 slots per wave
  if (row * 64 >= A.nslots) return;
  const int lane = threadIdx.x & 63;
  double v[5];
  row_sums<ST>(A, row, lane, v);
  if (lane == 0)
    for (int k = 0; k < 5; ++k) partial[row * 5 + k] = weight * v[k];
}

// Fixed LDS tree over the 256 threads' five accumulators; thread k < 5
// writes total k to out5.
__device__ __forceinline__ void tree5(const double (&acc)[5], double *out5) {
  __shared__ double sh[5][256];
  const int t = threadIdx.x;
  for (int k = 0; k < 5; ++k) sh[k][t] = acc[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w)
      for (int k = 0; k < 5; ++k) sh[k][t] += sh[k][t + w];
    __syncthreads();
  }
  if (t < 5) out5[t] = sh[t][0];
}

// Fixed-order sum of rows [r0, r1) of a [rows][5] array by one 256-thread
// workgroup: thread t adds rows r0 + t, r0 + t + 256, ... in turn, then the
// fixed LDS tree; the result does not depend on timing.
__device__ __forceinline__ void sum_rows(const double *in, int64_t r0, int64_t r1, double *out5) {
  const int t = threadIdx.x;
  double acc[5] = {0, 0, 0, 0, 0};
  for (int64_t r = r0 + t; r < r1; r += 256)
    for (int k = 0; k < 5; ++k) acc[k] += in[r * 5 + k];
  tree5(acc, out5);
}

// Second pass: chunks of kReduceChunk partial rows, one workgroup each.
__global__ __launch_bounds__(256) void k_reduce_mid(const double *partial, int64_t rows, double *mid) {
  const int64_t r0 = (int64_t)blockIdx.x * kReduceChunk;
  const int64_t r1 = r0 + kReduceChunk < rows ? r0 + kReduceChunk : rows;
  sum_rows(partial, r0, r1, mid + (int64_t)blockIdx.x * 5);
}

// Third pass: the chunk sums, one workgroup.
__global__ __launch_bounds__(256) void k_reduce_final(const double *mid, int64_t nmid, double *out5) {
  sum_rows(mid, 0, nmid, out5);
}

// First and second pass fused, for lbm_reduce_noalloc: workgroup c sums
// the rows [c kReduceChunk, (c + 1) kReduceChunk) of all levels in the
// order k_reduce_mid adds the stored row partials -- thread t = 64 w + i
// adds rows r0 + t, r0 + t + 256, ... -- but without storing them: wave w
// computes those rows one after another and lane i keeps the totals of the
// rows that are thread t's.  The chunk sums are bitwise those of the
// partial/mid passes.
template <class ST>
__global__ __launch_bounds__(256) void k_reduce_chunk(ReduceLevels R, double *mid) {
  const int64_t rows = R.row0[R.nlevels];
  const int64_t r0 = (int64_t)blockIdx.x * kReduceChunk;
  const int64_t r1 = r0 + kReduceChunk < rows ? r0 + kReduceChunk : rows;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double acc[5] = {0, 0, 0, 0, 0};
  for (int64_t base = r0 + wave * 64; base < r1; base += 256) {
    for (int i = 0; i < 64 && base + i < r1; ++i) {
      const int64_t r = base + i;
      int l = 0;
      while (l + 1 < R.nlevels && r >= R.row0[l + 1]) ++l;
      double v[5];
      row_sums<ST>(R.a[l], r - R.row0[l], lane, v);
      if (lane == i)
        for (int k = 0; k < 5; ++k) acc[k] += R.weight[l] * v[k];
    }
  }
  tree5(acc, mid + (int64_t)blockIdx.x * 5);
}

// The chunk sums of lbm_reduce_noalloc.  Each GPU holds its own copy; the
// host reaches it only through the address hipGetSymbolAddress returns on
// that device.
static __device__ __align__(256) double scratch[kNoAllocMidRows * 5];

template <template <class> class K, class... Args>
static hipError_t dispatch(int storage, dim3 g, dim3 b, hipStream_t s, Args... args) {
  switch (storage) {
    case LBM_F32: hipLaunchKernelGGL(K<StoreF32>::fn, g, b, 0, s, args...); break;
    case LBM_F16_SHIFTED: hipLaunchKernelGGL(K<StoreF16>::fn, g, b, 0, s, args...); break;
    case LBM_BF16_SHIFTED: hipLaunchKernelGGL(K<StoreBF16>::fn, g, b, 0, s, args...); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class ST> struct InitK { static constexpr auto fn = k_init_eq<ST>; };
template <class ST> struct MacroK { static constexpr auto fn = k_read_macro<ST>; };
template <class ST> struct RPopK { static constexpr auto fn = k_read_pop<ST>; };
template <class ST> struct WPopK { static constexpr auto fn = k_write_pop<ST>; };
template <class ST> struct RedK { static constexpr auto fn = k_reduce_partial<ST>; };
template <class ST> struct ChunkK { static constexpr auto fn = k_reduce_chunk<ST>; };

static dim3 grid_for(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

hipError_t launch_init_equilibrium(const SlotArgs &A, const double *rho, const double *u, hipStream_t s) {
  if (A.nslots == 0) return hipSuccess;
  return dispatch<InitK>(A.storage, grid_for(A.nslots), dim3(256), s, A, rho, u);
}
hipError_t launch_read_macroscopic(const SlotArgs &A, void *rho, void *u, int out_f64, hipStream_t s) {
  if (A.nslots == 0) return hipSuccess;
  return dispatch<MacroK>(A.storage, grid_for(A.nslots), dim3(256), s, A, rho, u, out_f64);
}
hipError_t launch_read_populations(const SlotArgs &A, double *f, hipStream_t s) {
  if (A.nslots == 0) return hipSuccess;
  return dispatch<RPopK>(A.storage, grid_for(A.nslots), dim3(256), s, A, f);
}
hipError_t launch_write_populations(const SlotArgs &A, const double *f, hipStream_t s) {
  if (A.nslots == 0) return hipSuccess;
  return dispatch<WPopK>(A.storage, grid_for(A.nslots), dim3(256), s, A, f);
}
hipError_t launch_reduce_partial(const SlotArgs &A, double weight, double *partial, hipStream_t s) {
  const int64_t rows = (A.nslots + 63) / 64;
  if (rows == 0) return hipSuccess;
  return dispatch<RedK>(A.storage, dim3((unsigned)((rows + 3) / 4)), dim3(256), s, A, weight, partial);
}
hipError_t launch_reduce_final(const double *partial, int64_t rows, double *mid, double *out5, hipStream_t s) {
  const int64_t nmid = reduce_mid_rows(rows);
  hipLaunchKernelGGL(k_reduce_mid, dim3((unsigned)nmid), dim3(256), 0, s, partial, rows, mid);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, s, mid, nmid, out5);
  return hipGetLastError();
}

// Device address of `scratch` on the current device, looked up once per
// device (the array's host-side name is not a device address).
static hipError_t scratch_address(double **out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static double *addr[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = (double *)p;
  }
  *out = addr[dev];
  return hipSuccess;
}

hipError_t launch_reduce_noalloc(const ReduceLevels &R, double *out5, hipStream_t s) {
  const int64_t nmid = reduce_mid_rows(R.row0[R.nlevels]);
  if (nmid > kNoAllocMidRows) return hipErrorInvalidValue;  // the caller checks the limit first
  double *mid = nullptr;
  hipError_t e = scratch_address(&mid);
  if (e != hipSuccess) return e;
  e = dispatch<ChunkK>(R.a[0].storage, dim3((unsigned)nmid), dim3(256), s, R, mid);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, s, (const double *)mid, nmid, out5);
  return hipGetLastError();
}

}  // inline namespace
}  // namespace lbm
