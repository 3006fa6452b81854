// Device-side building blocks shared by every liblbm kernel: population
// storage codecs, the collision operators and the per-link boundary rules.
// All arithmetic is FP32 on shifted populations h_i = f_i - w_i.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "lattice.h"
#include "launch.h"

namespace lbm {
inline namespace LBM_LATTICE_NS {

// ---------------------------------------------------------------- storage --
// Populations are stored shifted by the lattice weight.  FP32 keeps h as a
// float; the 16-bit forms round h to nearest-even in binary16 or bfloat16.

struct StoreF32 {
  using T = float;
  static __device__ __forceinline__ float load(const T *p, size_t i) { return p[i]; }
  static __device__ __forceinline__ float decode(T v) { return v; }
  static __device__ __forceinline__ void store(T *p, size_t i, float v) {
    __builtin_nontemporal_store(v, p + i);
  }
  static __device__ __forceinline__ float to_float(T v) { return v; }
  static __device__ __forceinline__ T from_double(double d) { return (float)d; }
  static __device__ __forceinline__ double to_double(T v) { return (double)v; }
};

// binary16 conversion f32 -> f16, round to nearest-even.  Written as one
// instruction so the compiler cannot merge it into a preceding FMA
// (v_fma_mixlo_f16 rounds once from the exact product), which would make
// the rounding depend on the surrounding code of each kernel.
__device__ __forceinline__ uint16_t f16_rne(float v) {
  uint32_t r;
  asm("v_cvt_f16_f32 %0, %1" : "=v"(r) : "v"(v));
  return (uint16_t)r;
}

struct StoreF16 {
  using T = uint16_t;
  static __device__ __forceinline__ float load(const T *p, size_t i) {
    return (float)__builtin_bit_cast(_Float16, p[i]);
  }
  static __device__ __forceinline__ float decode(T v) { return (float)__builtin_bit_cast(_Float16, v); }
  static __device__ __forceinline__ void store(T *p, size_t i, float v) {
    __builtin_nontemporal_store(f16_rne(v), p + i);
  }
  static __device__ __forceinline__ T from_double(double d) {
    return __builtin_bit_cast(uint16_t, (_Float16)d);
  }
  static __device__ __forceinline__ double to_double(T v) {
    return (double)(float)__builtin_bit_cast(_Float16, v);
  }
};

// bfloat16 keeps the top 16 bits of an IEEE float.
__device__ __forceinline__ uint16_t bf16_rne(float v) {
  uint32_t u = __float_as_uint(v);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

struct StoreBF16 {
  using T = uint16_t;
  static __device__ __forceinline__ float load(const T *p, size_t i) {
    return __uint_as_float((uint32_t)p[i] << 16);
  }
  static __device__ __forceinline__ float decode(T v) { return __uint_as_float((uint32_t)v << 16); }
  static __device__ __forceinline__ void store(T *p, size_t i, float v) {
    __builtin_nontemporal_store(bf16_rne(v), p + i);
  }
  // round a double to 8 significant bits (nearest-even) without passing
  // through float, so the result is correctly rounded
  static __device__ __forceinline__ T from_double(double d) {
    uint64_t b = (uint64_t)__double_as_longlong(d);
    b += ((1ull << 44) - 1) + ((b >> 45) & 1ull);
    b &= ~((1ull << 45) - 1);
    float f = (float)__longlong_as_double((long long)b);
    return (uint16_t)(__float_as_uint(f) >> 16);
  }
  static __device__ __forceinline__ double to_double(T v) {
    return (double)__uint_as_float((uint32_t)v << 16);
  }
};

// ------------------------------------------------------ population layout --
// Block layouts interleave the populations per block: the 64 slots of block
// b in direction i are the 64 consecutive values starting at (b Q + i) 64, so
// a block's Q rows form one contiguous span of Q x 64 values and every row
// is still one coalesced wave access.  (The dense lexicographic arm keeps Q
// separate planes of nx ny nz values.)
__device__ __forceinline__ size_t pidx(int i, uint32_t slot) {
  return ((size_t)(slot >> 6) * Q + (size_t)i) * 64 + (slot & 63u);
}

// ------------------------------------------------------- compile-time loop --
template <int I, int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// ---------------------------------------------------------------- moments --
struct Moments {
  float drho, rho, ux, uy, uz;
};

// rho - 1 = sum h, rho u = sum c h (the weights carry no momentum)
__device__ __forceinline__ Moments moments(const float (&h)[Q]) {
  Moments m;
  float s = h[0];
#pragma unroll
  for (int i = 1; i < Q; ++i) s = s + h[i];
#ifndef LBM_Q27
  const float jx = (h[1] - h[2]) + (h[7] - h[8]) + (h[9] - h[10]) + (h[11] - h[12]) + (h[13] - h[14]);
  const float jy = (h[3] - h[4]) + (h[7] - h[8]) + (h[10] - h[9]) + (h[15] - h[16]) + (h[17] - h[18]);
  const float jz = (h[5] - h[6]) + (h[11] - h[12]) + (h[14] - h[13]) + (h[15] - h[16]) + (h[18] - h[17]);
#else
  // opposite pairs (i, i+1) for odd i: c_i (h_i - h_i+1)
  float jx = 0.0f, jy = 0.0f, jz = 0.0f;
  static_for<1, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    if constexpr (kOpp[i] > i) {
      const float d = h[i] - h[kOpp[i]];
      if constexpr (kCx[i] > 0) jx = jx + d; else if constexpr (kCx[i] < 0) jx = jx - d;
      if constexpr (kCy[i] > 0) jy = jy + d; else if constexpr (kCy[i] < 0) jy = jy - d;
      if constexpr (kCz[i] > 0) jz = jz + d; else if constexpr (kCz[i] < 0) jz = jz - d;
    }
  });
#endif
  m.drho = s;
  m.rho = 1.0f + s;
  const float ir = 1.0f / m.rho;
  m.ux = jx * ir;
  m.uy = jy * ir;
  m.uz = jz * ir;
  return m;
}

// c_i . u for direction i
template <int I>
__device__ __forceinline__ float cdotu(float ux, float uy, float uz) {
  constexpr int cx = kCx[I], cy = kCy[I], cz = kCz[I];
  float r = 0.0f;
  bool first = true;
  auto acc = [&](int c, float v) {
    if (c == 0) return;
    if (first) { r = c > 0 ? v : -v; first = false; }
    else r = c > 0 ? r + v : r - v;
  };
  acc(cx, ux);
  acc(cy, uy);
  acc(cz, uz);
  return r;
}

// Shifted second-order equilibrium h^eq_i = f^eq_i - w_i,
//   f^eq_i = w_i rho (1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u.u).
// Computed per opposite pair: a = drho + rho (4.5 (c.u)^2 - 1.5 u.u),
// b = 3 rho c.u, h^eq = w (a +- b).
__device__ __forceinline__ void equilibrium(const Moments &m, float (&heq)[Q]) {
  const float usq15 = 1.5f * ((m.ux * m.ux + m.uy * m.uy) + m.uz * m.uz);
  const float rho3 = 3.0f * m.rho;
  heq[0] = weight_f(0) * fmaf(-m.rho, usq15, m.drho);
  static_for<1, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    if constexpr (kOpp[i] > i) {
      const float cu = cdotu<i>(m.ux, m.uy, m.uz);
      const float a = fmaf(m.rho, fmaf(4.5f * cu, cu, -usq15), m.drho);
      const float b = rho3 * cu;
      heq[i] = weight_f(i) * (a + b);
      heq[kOpp[i]] = weight_f(i) * (a - b);
    }
  });
}

// Hermite projection of the non-equilibrium part onto second order:
//   Pi_ab = sum_i c_ia c_ib h_i - drho/3 delta_ab - rho u_a u_b
//   f1_i  = 4.5 w_i (c_i . Pi . c_i - tr(Pi)/3)
__device__ __forceinline__ void hermite2(float pxx, float pyy, float pzz, float pxy, float pxz, float pyz,
                                         float (&f1)[Q]) {
  // f1_i = w_i / (2 c_s^4) Q_i : P with Q_i = c_i c_i - I/3
  const float tr3 = (pxx + pyy + pzz) * (1.0f / 3.0f);
#ifdef LBM_Q27
  // c_i c_i : P - tr P / 3 for every direction, per opposite pair
  static_for<0, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    if constexpr (i == 0 || kOpp[i] > i) {
      constexpr int cx = kCx[i], cy = kCy[i], cz = kCz[i];
      float q = -tr3;
      if constexpr (cx != 0) q = q + pxx;
      if constexpr (cy != 0) q = q + pyy;
      if constexpr (cz != 0) q = q + pzz;
      if constexpr (cx * cy != 0) q = fmaf((float)(2 * cx * cy), pxy, q);
      if constexpr (cx * cz != 0) q = fmaf((float)(2 * cx * cz), pxz, q);
      if constexpr (cy * cz != 0) q = fmaf((float)(2 * cy * cz), pyz, q);
      f1[i] = (4.5f * weight_f(i)) * q;
      if constexpr (i != 0) f1[kOpp[i]] = f1[i];
    }
  });
#else
  const float k1 = 4.5f * weight_f(1), k2 = 4.5f * weight_f(7);
  f1[0] = 4.5f * weight_f(0) * -tr3;
  f1[1] = f1[2] = k1 * (pxx - tr3);
  f1[3] = f1[4] = k1 * (pyy - tr3);
  f1[5] = f1[6] = k1 * (pzz - tr3);
  const float exy = pxx + pyy - tr3, exz = pxx + pzz - tr3, eyz = pyy + pzz - tr3;
  f1[7] = f1[8] = k2 * (exy + 2.0f * pxy);
  f1[9] = f1[10] = k2 * (exy - 2.0f * pxy);
  f1[11] = f1[12] = k2 * (exz + 2.0f * pxz);
  f1[13] = f1[14] = k2 * (exz - 2.0f * pxz);
  f1[15] = f1[16] = k2 * (eyz + 2.0f * pyz);
  f1[17] = f1[18] = k2 * (eyz - 2.0f * pyz);
#endif
}

#ifndef LBM_Q27
// Non-equilibrium stress Pi = sum_i c_i c_i (h_i - h^eq_i) of a D3Q19
// voxel as (xx, yy, zz, xy, xz, yz).
__device__ __forceinline__ void neq_stress(const float (&h)[Q], const Moments &m, float (&p)[6]) {
  const float p78 = h[7] + h[8], p910 = h[9] + h[10], p1112 = h[11] + h[12];
  const float p1314 = h[13] + h[14], p1516 = h[15] + h[16], p1718 = h[17] + h[18];
  const float sxx = (h[1] + h[2]) + p78 + p910 + p1112 + p1314;
  const float syy = (h[3] + h[4]) + p78 + p910 + p1516 + p1718;
  const float szz = (h[5] + h[6]) + p1112 + p1314 + p1516 + p1718;
  const float d3 = m.drho * (1.0f / 3.0f);
  p[0] = sxx - d3 - m.rho * m.ux * m.ux;
  p[1] = syy - d3 - m.rho * m.uy * m.uy;
  p[2] = szz - d3 - m.rho * m.uz * m.uz;
  p[3] = (p78 - p910) - m.rho * m.ux * m.uy;
  p[4] = (p1112 - p1314) - m.rho * m.ux * m.uz;
  p[5] = (p1516 - p1718) - m.rho * m.uy * m.uz;
}

// Squared Euclidean norm of the D3Q19 Hermite vector hermite2(P), summed in
// closed form over the lattice: the rest population gives (1.5 t)^2 with
// t = tr P / 3, each axis pair 2 (P_aa - t)^2 / 16, each edge plane ab
// 2 ((e + 2 P_ab)^2 + (e - 2 P_ab)^2) / 64 with e = P_aa + P_bb - t.
__device__ __forceinline__ float hermite2_norm2(float pxx, float pyy, float pzz, float pxy, float pxz,
                                                float pyz) {
  const float t = (pxx + pyy + pzz) * (1.0f / 3.0f);
  const float ax = pxx - t, ay = pyy - t, az = pzz - t;
  const float exy = pxx + pyy - t, exz = pxx + pzz - t, eyz = pyy + pzz - t;
  float s = 2.25f * (t * t);
  s = fmaf(0.125f, ax * ax + ay * ay + az * az, s);
  s = fmaf(0.0625f, exy * exy + exz * exz + eyz * eyz, s);
  s = fmaf(0.25f, pxy * pxy + pxz * pxz + pyz * pyz, s);
  return s;
}
#endif

__device__ __forceinline__ void f1_projection(const float (&h)[Q], const Moments &m, float (&f1)[Q]) {
#ifdef LBM_Q27
  // second moments of h over opposite pairs (c c is even in c)
  float sxx = 0.0f, syy = 0.0f, szz = 0.0f, sxy = 0.0f, sxz = 0.0f, syz = 0.0f;
  static_for<1, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    if constexpr (kOpp[i] > i) {
      constexpr int cx = kCx[i], cy = kCy[i], cz = kCz[i];
      const float p = h[i] + h[kOpp[i]];
      if constexpr (cx != 0) sxx = sxx + p;
      if constexpr (cy != 0) syy = syy + p;
      if constexpr (cz != 0) szz = szz + p;
      if constexpr (cx * cy > 0) sxy = sxy + p; else if constexpr (cx * cy < 0) sxy = sxy - p;
      if constexpr (cx * cz > 0) sxz = sxz + p; else if constexpr (cx * cz < 0) sxz = sxz - p;
      if constexpr (cy * cz > 0) syz = syz + p; else if constexpr (cy * cz < 0) syz = syz - p;
    }
  });
  const float d3 = m.drho * (1.0f / 3.0f);
  hermite2(sxx - d3 - m.rho * m.ux * m.ux, syy - d3 - m.rho * m.uy * m.uy, szz - d3 - m.rho * m.uz * m.uz,
           sxy - m.rho * m.ux * m.uy, sxz - m.rho * m.ux * m.uz, syz - m.rho * m.uy * m.uz, f1);
#else
  float p[6];
  neq_stress(h, m, p);
  hermite2(p[0], p[1], p[2], p[3], p[4], p[5], f1);
#endif
}

enum : int { kCollBGK = 0, kCollRegularized = 1, kCollMLP = 2 };

// BGK: h* = h + omega (h^eq - h)
__device__ __forceinline__ void collide_bgk(float (&h)[Q], float omega) {
  const Moments m = moments(h);
  float heq[Q];
  equilibrium(m, heq);
#pragma unroll
  for (int i = 0; i < Q; ++i) h[i] = fmaf(omega, heq[i] - h[i], h[i]);
}

// Regularized: h* = h^eq + (1 - omega) f1(h)
__device__ __forceinline__ void collide_regularized_m(float (&h)[Q], const Moments &m, float omega) {
  float heq[Q], f1[Q];
  equilibrium(m, heq);
  f1_projection(h, m, f1);
  const float r = 1.0f - omega;
#pragma unroll
  for (int i = 0; i < Q; ++i) h[i] = fmaf(r, f1[i], heq[i]);
}

__device__ __forceinline__ void collide_regularized(float (&h)[Q], float omega) {
  const Moments m = moments(h);
  collide_regularized_m(h, m, omega);
}

// ------------------------------------------------------- boundary rules ---
// Classification of one pulled link of voxel (gx,gy,gz) in direction I
// against the box faces (reading of the tie-break: a moving wall wins over
// a stationary wall, which wins over a regularized face).
enum : int { kLinkInside = 0, kLinkBounce = 1, kLinkMoving = 2, kLinkUnknown = 3 };

struct LinkClass {
  int kind;
  int face;     // face id for kLinkUnknown
  float extra;  // moving-wall correction for kLinkMoving
};

// c_i . u_w with a wall velocity from the face table (face known at compile time)
template <int I>
__device__ __forceinline__ float moving_wall_term(const FaceParams &fp, int face) {
  const float cu = cdotu<I>(fp.val[face][0], fp.val[face][1], fp.val[face][2]);
  return (6.0f * weight_f(I)) * cu;  // 2 w_i (c_i . u_w) / c_s^2, wall density 1
}

// REC: the moving-wall velocity comes from the voxel's boundary record rv
// (indirect indexing of the bitmask layout) instead of the face table.
template <int I, bool REC = false>
__device__ __forceinline__ LinkClass classify_link(const FaceParams &fp, int gx, int gy, int gz,
                                                   int nx, int ny, int nz, const float *rv = nullptr) {
  constexpr int c[3] = {kCx[I], kCy[I], kCz[I]};
  const int g[3] = {gx, gy, gz};
  const int n[3] = {nx, ny, nz};
  LinkClass r{kLinkInside, -1, 0.0f};
  bool moving = false, wall = false;
  int reg = -1;
  float extra = 0.0f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (c[a] == 0) continue;
    const int face = 2 * a + (c[a] > 0 ? 0 : 1);  // compile-time after unrolling
    const bool crossed = !((fp.periodic >> a) & 1) && (c[a] > 0 ? g[a] == 0 : g[a] == n[a] - 1);
    if (!crossed) continue;
    const int k = fp.kind[face];
    if (k == LBM_BC_MOVING_WALL) {
      if (!moving) {
        if constexpr (REC) extra = (6.0f * weight_f(I)) * cdotu<I>(rv[0], rv[1], rv[2]);
        else extra = moving_wall_term<I>(fp, face);
      }
      moving = true;
    } else if (k == LBM_BC_BOUNCE_BACK) {
      wall = true;
    } else {
      reg = face;
    }
  }
  if (moving) { r.kind = kLinkMoving; r.extra = extra; }
  else if (wall) r.kind = kLinkBounce;
  else if (reg >= 0) { r.kind = kLinkUnknown; r.face = reg; }
  return r;
}

// Face parameter with a lane-dependent face id, by selection (no indexed
// private memory).
__device__ __forceinline__ float face_val(const FaceParams &fp, int face, int k) {
  float r = fp.val[0][k];
#pragma unroll
  for (int f = 1; f < 6; ++f) r = face == f ? fp.val[f][k] : r;
  return r;
}
__device__ __forceinline__ int face_kind(const FaceParams &fp, int face) {
  int r = fp.kind[0];
#pragma unroll
  for (int f = 1; f < 6; ++f) r = face == f ? fp.kind[f] : r;
  return r;
}

// Regularized velocity/pressure face (Latt et al. 2008) for a voxel whose
// links in `unknown` come from outside across `face`; h holds the known
// pulled values.  Computes rho (velocity face) or the normal velocity
// (pressure face) from the tangential and outgoing sums, rebuilds the unknown
// populations by non-equilibrium bounce-back, regularizes and relaxes:
// h* = h^eq + (1 - omega) f1.
// REC: the face value comes from the voxel's boundary record rv.
template <bool REC = false>
__device__ __forceinline__ void regularized_face(float (&h)[Q], uint32_t unknown, int face,
                                                 const FaceParams &fp, float omega,
                                                 const float *rv = nullptr) {
  const int axis = face >> 1;
  const float sgn = (face & 1) ? 1.0f : -1.0f;
  // per axis: sums over c_a = 0, c_a > 0 and c_a < 0 (index sets fixed at
  // compile time), then pick the face's axis and orientation
  float s0[3] = {0.0f, 0.0f, 0.0f}, sp[3] = {0.0f, 0.0f, 0.0f}, sm[3] = {0.0f, 0.0f, 0.0f};
  static_for<0, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    constexpr int c[3] = {kCx[i], kCy[i], kCz[i]};
#pragma unroll
    for (int a2 = 0; a2 < 3; ++a2) {
      if (c[a2] == 0) s0[a2] = s0[a2] + h[i];
      else if (c[a2] > 0) sp[a2] = sp[a2] + h[i];
      else sm[a2] = sm[a2] + h[i];
    }
  });
  const float sT = axis == 0 ? s0[0] : (axis == 1 ? s0[1] : s0[2]);
  const float sOp = axis == 0 ? sp[0] : (axis == 1 ? sp[1] : sp[2]);
  const float sOm = axis == 0 ? sm[0] : (axis == 1 ? sm[1] : sm[2]);
  const float sO = (face & 1) ? sOp : sOm;  // populations leaving through the face
  const float X = sT + 2.0f * sO;  // = rho (1 + u.n) - 1
  Moments m;
  auto value = [&](int k) { return REC ? rv[k] : face_val(fp, face, k); };
  if (face_kind(fp, face) == LBM_BC_REG_VELOCITY) {
    m.ux = value(0);
    m.uy = value(1);
    m.uz = value(2);
    const float un = sgn * (axis == 0 ? m.ux : (axis == 1 ? m.uy : m.uz));
    m.drho = (X - un) / (1.0f + un);
    m.rho = 1.0f + m.drho;
  } else {
    m.rho = value(0);
    m.drho = m.rho - 1.0f;
    const float un = (X - m.drho) / m.rho;
    m.ux = axis == 0 ? sgn * un : 0.0f;
    m.uy = axis == 1 ? sgn * un : 0.0f;
    m.uz = axis == 2 ? sgn * un : 0.0f;
  }
  float heq[Q];
  equilibrium(m, heq);
  static_for<1, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    if ((unknown >> i) & 1u) h[i] = h[kOpp[i]] + (heq[i] - heq[kOpp[i]]);
  });
  float f1[Q];
  f1_projection(h, m, f1);
  const float r = 1.0f - omega;
#pragma unroll
  for (int i = 0; i < Q; ++i) h[i] = fmaf(r, f1[i], heq[i]);
}

// ------------------------------------------------------------ utilities ---
// Workgroup order of the block kernels.  The hardware deals workgroup k to
// XCD k % 8; the logical workgroups (4 consecutive Morton-ordered blocks
// each) are cut into chunks of kXcdChunk, and XCD x takes chunks x, x + 8,
// x + 16, ... in turn.  A chunk (64 blocks, a 4x4x4-block Morton cube of a
// dense grid) stays on one XCD and its L2,
// and at any moment the eight XCDs work on neighbouring chunks, so the rows
// that blocks pull across chunk faces are fetched once into the shared
// Infinity Cache for all of them and the DRAM traffic of the chip covers
// one compact region.  (Contiguous eighths of the range per XCD measured
// 6% slower on the FP32 interior kernel; chunks of 4, 8 and 32 workgroups
// 1-2%, 0.5-1% and 0-3% slower over the whole steps.)
// The grid is padded to whole rounds of 8 chunks (xcd_grid); the padding
// workgroups map past the last block and exit.
constexpr int kXcdChunk = 16;
__host__ __device__ constexpr int xcd_grid(int nwg) {
  return (nwg + 8 * kXcdChunk - 1) / (8 * kXcdChunk) * (8 * kXcdChunk);
}
__device__ __forceinline__ int xcd_remap(int k) {
  const int x = k & 7, i = k >> 3;
  return ((i / kXcdChunk) * 8 + x) * kXcdChunk + i % kXcdChunk;
}

}  // inline namespace
}  // namespace lbm
