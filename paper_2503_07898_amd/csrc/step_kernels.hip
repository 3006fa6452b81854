// Fused pull collide-and-stream kernels of liblbm (gfx950).
//
// Block layouts: one wave64 per 4^3-voxel block, lane = voxel x+4y+16z,
// four blocks per 256-thread workgroup.  Populations are block-interleaved
// (pidx): each block's Q rows of 64 values are contiguous, so every
// population load of a wave is one 256-byte (FP32) or 128-byte (16-bit) row
// of its own block plus the face and edge rows of the neighbour blocks it
// pulls across.  Neighbour block slots and bounce masks are wave-uniform and
// come through scalar loads.
//
// Kernels per group (the disaggregated design's group-specific operations):
//   full      -- every pulled source is a fluid voxel; no masks, no checks;
//   masked    -- non-boundary blocks with obstacles or stationary walls:
//                halfway bounce-back where the bounce mask says so;
//   boundary  -- blocks with moving-wall or regularized-face voxels; carries
//                the per-lane face logic and the regularized reconstruction.
//   jump      -- multires blocks next to a resolution jump: every source is
//                read through a precomputed gather table (explosion and
//                coalescence as pulls), then collided.
// The single-kernel comparison arm of block-sparse grids launches the
// boundary kernel over every block.  The dense comparison arm is the
// lexicographic kernel.  The unfused multires baseline runs the same gathers
// with FUSED = false (store the pulled populations) followed by the
// collision-only kernel.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "launch.h"
#ifndef LBM_Q27
#include "mlp_device.h"
#endif

namespace lbm {
inline namespace LBM_LATTICE_NS {

// Slot of the source of lane `lane` in direction I (pull from x - c_I).
// Uniform neighbour slots nbv[d-1] for lattice directions d = 1..Q-1; the
// source block is chosen per lane by which block faces the pull crosses.
template <int I>
__device__ __forceinline__ uint32_t pull_slot(int lane, int own, const int32_t (&nbv)[kNbr]) {
  constexpr int cx = kCx[I], cy = kCy[I], cz = kCz[I];
  const int lx = lane & 3, ly = (lane >> 2) & 3, lz = lane >> 4;
  const bool ox = cx != 0 && lx == (cx > 0 ? 0 : 3);
  const bool oy = cy != 0 && ly == (cy > 0 ? 0 : 3);
  const bool oz = cz != 0 && lz == (cz > 0 ? 0 : 3);
  int b = own;
  if constexpr (cx != 0) b = ox ? nbv[dir_of(-cx, 0, 0) - 1] : b;
  if constexpr (cy != 0) b = oy ? nbv[dir_of(0, -cy, 0) - 1] : b;
  if constexpr (cz != 0) b = oz ? nbv[dir_of(0, 0, -cz) - 1] : b;
  if constexpr (cx != 0 && cy != 0) b = (ox && oy) ? nbv[dir_of(-cx, -cy, 0) - 1] : b;
  if constexpr (cx != 0 && cz != 0) b = (ox && oz) ? nbv[dir_of(-cx, 0, -cz) - 1] : b;
  if constexpr (cy != 0 && cz != 0) b = (oy && oz) ? nbv[dir_of(0, -cy, -cz) - 1] : b;
  if constexpr (cx != 0 && cy != 0 && cz != 0) b = (ox && oy && oz) ? nbv[dir_of(-cx, -cy, -cz) - 1] : b;
  const int local = ((lx - cx) & 3) | (((ly - cy) & 3) << 2) | (((lz - cz) & 3) << 4);
  return (uint32_t)(b * 64 + local);
}

template <int COLL>
__device__ __forceinline__ void collide(float (&h)[Q], float omega) {
  if constexpr (COLL == kCollRegularized) collide_regularized(h, omega);
  else collide_bgk(h, omega);
}

// ------------------------------------------------------ interior kernels --
// Per-block body of the interior kernels (b is wave-uniform).
template <class ST, int COLL, bool MASKED, bool FUSED>
__device__ __forceinline__ void interior_block(const StepArgs &a, int b) {
  using T = typename ST::T;
  const int lane = threadIdx.x & 63;
  const T *__restrict__ src = (const T *)a.src;
  T *__restrict__ dst = (T *)a.dst;
  const uint32_t own_slot = (uint32_t)b * 64u + (uint32_t)lane;

  int32_t nbv[kNbr];
#pragma unroll
  for (int d = 0; d < kNbr; ++d) nbv[d] = a.nbr[(size_t)b * kNbr + d];
  uint64_t bm[kNbr];
  if constexpr (MASKED) {
#pragma unroll
    for (int d = 0; d < kNbr; ++d) bm[d] = a.bbm[(size_t)b * kNbr + d];
  }

  float h[Q];
  h[0] = ST::load(src, pidx(0, own_slot));
  static_for<1, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    uint32_t slot = pull_slot<i>(lane, b, nbv);
    uint32_t plane = i;
    if constexpr (MASKED) {
      if ((bm[i - 1] >> lane) & 1ull) {  // halfway bounce-back
        slot = own_slot;
        plane = kOpp[i];
      }
    }
    h[i] = ST::load(src, pidx(plane, slot));
  });

  if constexpr (FUSED) collide<COLL>(h, a.omega);

#pragma unroll
  for (int i = 0; i < Q; ++i) ST::store(dst, pidx(i, own_slot), h[i]);
}

template <class ST, int COLL, bool MASKED, bool FUSED>
__global__ __launch_bounds__(256) void k_block_interior(StepArgs a, int32_t g0, int32_t n) {
  const int wg = xcd_remap(blockIdx.x);
  const int b = __builtin_amdgcn_readfirstlane(g0 + wg * 4 + (int)(threadIdx.x >> 6));
  if (b >= g0 + n) return;
  interior_block<ST, COLL, MASKED, FUSED>(a, b);
}

// Bitmask-based grouping: every block of the level is visited, the run-time
// bit of the block selects the non-boundary ones (bounce masks cover the
// blocks that the memory-based layout separates as "full").
template <class ST, int COLL>
__global__ __launch_bounds__(256) void k_block_interior_bits(StepArgs a, int32_t g0, int32_t n) {
  const int wg = xcd_remap(blockIdx.x);
  const int b = __builtin_amdgcn_readfirstlane(g0 + wg * 4 + (int)(threadIdx.x >> 6));
  if (b >= g0 + n) return;
  if ((a.bbits[b >> 5] >> (b & 31)) & 1u) return;
  interior_block<ST, COLL, true, true>(a, b);
}

#ifndef LBM_Q27  // D3Q19 only
// ------------------------------------------ 32-bit pull offsets (closure) --
// For population buffers of at most 4 GiB the byte offset of every pull fits
// in 32 bits, and it splits into a per-lane part that does not depend on the
// direction and wave-uniform parts selected per lane by bit masks.  Lane v of
// block b pulling direction I reads byte
//   S (v + Q 64 b) + S (64 I - c_I.(1, 4, 16))
//   + sum over the block faces the pull crosses of a uniform delta,
// where crossing face x moves the source to block n_x (delta S Q 64 (n_x - b)
// + 4 c_x S, the wrap of the x coordinate), and an edge pull adds a second
// order term so that the sum lands in the edge neighbour's block.  All of it
// is taken modulo 2^32, and the true offset is below 2^32.  One AND and one
// add per crossed face replace the 64-bit slot arithmetic, which keeps the
// vector-instruction count of the issue-bound closure kernel down.  (The
// HBM-bound interior kernels keep the 64-bit form: the 32-bit one, built for
// them too, left their whole steps unchanged within 1.5%.)
struct LaneFaces {
  uint32_t x0, x3, y0, y3, z0, z3;  // all ones where the lane sits on that face of its block
  template <int C> __device__ __forceinline__ uint32_t x() const { return C > 0 ? x0 : x3; }
  template <int C> __device__ __forceinline__ uint32_t y() const { return C > 0 ? y0 : y3; }
  template <int C> __device__ __forceinline__ uint32_t z() const { return C > 0 ? z0 : z3; }
};

__device__ __forceinline__ LaneFaces lane_faces(int lane) {
  const auto all = [](bool c) { return c ? ~0u : 0u; };
  return {all((lane & 3) == 0), all((lane & 3) == 3), all((lane & 12) == 0),
          all((lane & 12) == 12), all(lane < 16), all(lane >= 48)};
}

// if_set where the lane's bit of the wave-uniform mask is set, else if_clear:
// one select that reads the mask from its scalar registers (as C++ the test
// of bit `lane` becomes a 64-bit shift, an AND and a compare per direction)
__device__ __forceinline__ uint32_t lane_select(uint64_t mask, uint32_t if_set, uint32_t if_clear) {
  uint32_t r;
  asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(if_clear), "v"(if_set), "s"(mask));
  return r;
}

// byte offset of lane's pull source in direction I; `base` = S (lane + Q 64 own)
template <int I, int S>
__device__ __forceinline__ uint32_t pull_off32(uint32_t base, const LaneFaces &lf, int own,
                                               const int32_t (&nbv)[kNbr]) {
  constexpr int cx = kCx[I], cy = kCy[I], cz = kCz[I];
  static_assert(!(cx != 0 && cy != 0 && cz != 0), "D3Q19 has no corner directions");
  constexpr uint32_t QS = (uint32_t)(Q * 64 * S);
  const uint32_t own_q = (uint32_t)own * QS;
  const auto delta = [&](int d, int wrap) { return (uint32_t)nbv[d - 1] * QS - own_q + (uint32_t)(wrap * S); };
  uint32_t off = base + (uint32_t)((64 * I - (cx + 4 * cy + 16 * cz)) * S);
  uint32_t dx = 0, dy = 0, dz = 0;
  if constexpr (cx != 0) {
    dx = delta(dir_of(-cx, 0, 0), 4 * cx);
    off += lf.x<cx>() & dx;
  }
  if constexpr (cy != 0) {
    dy = delta(dir_of(0, -cy, 0), 16 * cy);
    off += lf.y<cy>() & dy;
  }
  if constexpr (cz != 0) {
    dz = delta(dir_of(0, 0, -cz), 64 * cz);
    off += lf.z<cz>() & dz;
  }
  if constexpr (cx != 0 && cy != 0) off += (lf.x<cx>() & lf.y<cy>()) & (delta(dir_of(-cx, -cy, 0), 4 * cx + 16 * cy) - dx - dy);
  if constexpr (cx != 0 && cz != 0) off += (lf.x<cx>() & lf.z<cz>()) & (delta(dir_of(-cx, 0, -cz), 4 * cx + 64 * cz) - dx - dz);
  if constexpr (cy != 0 && cz != 0) off += (lf.y<cy>() & lf.z<cz>()) & (delta(dir_of(0, -cy, -cz), 16 * cy + 64 * cz) - dy - dz);
  return off;
}

// ------------------------------------------ interior kernel, learned closure --
// Same gather as k_block_interior; the collision evaluates the closure
// network for the wave's 64 voxels on the matrix cores, projects its output
// to zero mass and momentum, and falls back per voxel to the regularized
// operator when a standardized input leaves [-8, 8], a population turns
// negative, or the closure's non-equilibrium part strays more than the
// judge tolerance from the regularized operator's.  The packed weights, the
// GELU table and the biases are staged in LDS once per workgroup.  Three
// waves per SIMD (at most 168 registers): the network's accumulators then
// stay in ordinary registers (no accumulator-register reads) and a third
// wave hides more of the LDS and matrix-core latency.

// The pulls of block b (wave-uniform) into raw, issued without waiting.
// NARROW: population buffers of at most 4 GiB (32-bit pull offsets).
template <class ST, bool MASKED, bool NARROW>
__device__ __forceinline__ void closure_gather(const StepArgs &a, int b, int lane, typename ST::T (&raw)[Q]) {
  using T = typename ST::T;
  const T *__restrict__ src = (const T *)a.src;
  const uint32_t own_slot = (uint32_t)b * 64u + (uint32_t)lane;
  int32_t nbv[kNbr];
#pragma unroll
  for (int d = 0; d < kNbr; ++d) nbv[d] = a.nbr[(size_t)b * kNbr + d];
  uint64_t bm[kNbr];
  if constexpr (MASKED) {
#pragma unroll
    for (int d = 0; d < kNbr; ++d) bm[d] = a.bbm[(size_t)b * kNbr + d];
  }
  // all stored values first, then their decoding: under the register limit
  // of three waves per SIMD this keeps the 19 loads of 16-bit storage in
  // flight together instead of one converted value at a time
  if constexpr (NARROW) {
    constexpr int S = (int)sizeof(T);
    const LaneFaces lf = lane_faces(lane);
    const uint32_t base = (uint32_t)lane * S + (uint32_t)b * (uint32_t)(Q * 64 * S);
    const char *src8 = (const char *)src;
    raw[0] = *(const T *)(src8 + base);
    static_for<1, Q>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      uint32_t off = pull_off32<i, S>(base, lf, b, nbv);
      if constexpr (MASKED) off = lane_select(bm[i - 1], base + (uint32_t)(kOpp[i] * 64 * S), off);
      raw[i] = *(const T *)(src8 + off);
    });
  } else {
    raw[0] = src[pidx(0, own_slot)];
    static_for<1, Q>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      uint32_t slot = pull_slot<i>(lane, b, nbv);
      uint32_t plane = i;
      if constexpr (MASKED) {
        if ((bm[i - 1] >> lane) & 1ull) {
          slot = own_slot;
          plane = kOpp[i];
        }
      }
      raw[i] = src[pidx(plane, slot)];
    });
  }
}

// The closure update of block b from its pulled populations raw.
template <class ST, bool MASKED>
__device__ __forceinline__ void closure_update(const StepArgs &a, int b, int lane, const typename ST::T (&raw)[Q],
                                               const __bf16 *wl, const float *bl) {
  using T = typename ST::T;
  T *__restrict__ dst = (T *)a.dst;
  float h[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) h[i] = ST::decode(raw[i]);
  const bool fluid = MASKED ? ((a.fmask[b] >> lane) & 1ull) != 0 : true;

  // closure inputs g = (f - f^eq)/rho, standardized.  What the rest of the
  // update needs of the populations -- the moments and the non-equilibrium
  // stress (the regularized operator's input, for the judge and the
  // fallback) -- is taken now, so the populations are dead while the
  // network runs (fewer live registers, more waves per SIMD); the
  // equilibrium is recomputed afterwards, bit for bit the same.
  const Moments m = moments(h);
  const float *sd = a.mlp_stdz;
  const float ir = 1.0f / m.rho;
  float x[Q];
  float xmax = 0.0f;  // largest |x_i|: one max per input instead of a compare
  {
    float heq[Q];
    equilibrium(m, heq);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const float g = (h[i] - heq[i]) * ir;
      x[i] = fluid ? (g - sd[i]) * sd[32 + i] : 0.0f;
      xmax = fmaxf(xmax, fabsf(x[i]));
    }
  }
  const bool out_of_range = xmax > 8.0f;
  float pneq[6];
  neq_stress(h, m, pneq);
  float y[Q];
  mlp_forward_wave_reg(x, y, wl, bl, lane);
#pragma unroll
  for (int i = 0; i < Q; ++i) y[i] = fmaf(y[i], sd[64 + i], sd[96 + i]);
  float ys[6];  // second-order Hermite coordinates of the closure's output
  q_stress(y, ys);
  hermite2(ys[0], ys[1], ys[2], ys[3], ys[4], ys[5], y);
  // the regularized operator judges the closure: its non-equilibrium part
  // f1/rho must lie within judge (relative L2) of the closure's, with the
  // typical target size as floor for voxels near equilibrium.  Both are
  // second-order Hermite vectors, so their distance and the target's size
  // are taken from the six stress coordinates in closed form.
  bool off = false;
  if (a.mlp_judge > 0.0f) {
    float ps[6], ds[6];  // coordinates of f1/rho and of the difference
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      ps[k] = pneq[k] * ir;
      ds[k] = ys[k] - ps[k];
    }
    const float d2 = hermite2_norm2(ds[0], ds[1], ds[2], ds[3], ds[4], ds[5]);
    const float t2 = hermite2_norm2(ps[0], ps[1], ps[2], ps[3], ps[4], ps[5]);
    off = d2 > a.mlp_judge * a.mlp_judge * (t2 + *a.mlp_s2);  // s2: sum of out_std^2, kept beside stdz
  }
  float heq[Q];
  equilibrium(m, heq);
  const float r = (1.0f - a.omega) * m.rho;
  bool negative = false;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    h[i] = fmaf(r, y[i], heq[i]);
    // w_i + h_i < 0 in FP32 exactly when h_i < -w_i: the rounded sum keeps
    // the sign of the exact one, which is a multiple of h_i's unit in the
    // last place and so never underflows.  (A minimum per weight class and
    // three compares issue fewer instructions but measured 3-5% slower: the
    // chains of minima sit on the path to the stores.)
    negative = negative || (h[i] < -weight_f(i));
  }
  const bool fb = fluid && (out_of_range || negative || off);
  if (fb) {
    // the regularized operator: f^eq + (1 - omega) f1, f1 from the stress
    float f1[Q];
    hermite2(pneq[0], pneq[1], pneq[2], pneq[3], pneq[4], pneq[5], f1);
    const float rr = 1.0f - a.omega;
#pragma unroll
    for (int i = 0; i < Q; ++i) h[i] = fmaf(rr, f1[i], heq[i]);
  }
  const uint64_t bal = __ballot(fb);
  if (lane == 0 && bal) atomicAdd(a.mlp_fallbacks, (unsigned long long)__popcll(bal));
  T *dstb = dst + (size_t)b * (Q * 64);  // the block's rows, from a wave-uniform base
#pragma unroll
  for (int i = 0; i < Q; ++i) ST::store(dstb, (size_t)(i * 64 + lane), h[i]);
}

// PB blocks per wave, the wave's k-th block being g0 + 4 PB wg + 4 k + wave
// (the workgroup's four waves work on four consecutive blocks at a time).
// The pulls of the next block are issued before the current block's update,
// and nothing inside the update waits on a vector-memory load (weights,
// table and biases come from LDS, the standardization through scalar
// loads), so the one in-order counter of vector-memory loads does not tie
// the update to the next block's pulls.  With 16-bit storage the compiled
// kernel still waits for both blocks' pulls before the first network (it
// packs the 16-bit values two to a register as they arrive), so what two
// blocks per wave buy there is 38 pulls in flight per wave instead of 19.
template <class ST, bool MASKED, bool NARROW, int PB>
__global__ __launch_bounds__(256, 3) void k_block_interior_mlp(StepArgs a, int32_t g0, int32_t n) {
  using T = typename ST::T;
  __shared__ __attribute__((aligned(16))) __bf16 wl[kWStageElems];
  // the biases sit in LDS as well: a global load inside the network would
  // make its wait (one in-order counter) wait for the next block's pulls too
  __shared__ __attribute__((aligned(16))) float bl[kBiasFloats];
  stage_weights(wl, (const __bf16 *)a.mlp_w, bl, a.mlp_bias);
  const int wg = xcd_remap(blockIdx.x);
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int b0 = __builtin_amdgcn_readfirstlane(g0 + wg * 4 * PB + wave);
  if (b0 >= g0 + n) return;
  T raw[2][Q];
  closure_gather<ST, MASKED, NARROW>(a, b0, lane, raw[0]);
#pragma unroll
  for (int k = 0; k < PB; ++k) {
    const int b = b0 + 4 * k;
    if (k + 1 < PB && b + 4 < g0 + n) closure_gather<ST, MASKED, NARROW>(a, b + 4, lane, raw[(k + 1) & 1]);
    closure_update<ST, MASKED>(a, b, lane, raw[k & 1], wl, bl);
    if (b + 4 >= g0 + n) break;
  }
}

#endif  // LBM_Q27

// ------------------------------------------------------ boundary kernel --
// Per-block body of the boundary kernels.  REC: boundary values from the
// voxel's indirect record (bitmask layout) instead of the face table.
template <class ST, int COLL, bool FUSED, bool REC>
__device__ __forceinline__ void boundary_block(const StepArgs &a, int b) {
  using T = typename ST::T;
  const int lane = threadIdx.x & 63;
  const T *__restrict__ src = (const T *)a.src;
  T *__restrict__ dst = (T *)a.dst;
  const uint32_t own_slot = (uint32_t)b * 64u + (uint32_t)lane;

  int32_t nbv[kNbr];
  uint64_t bm[kNbr];
#pragma unroll
  for (int d = 0; d < kNbr; ++d) {
    nbv[d] = a.nbr[(size_t)b * kNbr + d];
    bm[d] = a.bbm[(size_t)b * kNbr + d];
  }
  const int packed = a.coords[b];
  const int gx = (packed & 1023) * 4 + (lane & 3);
  const int gy = ((packed >> 10) & 1023) * 4 + ((lane >> 2) & 3);
  const int gz = ((packed >> 20) & 1023) * 4 + (lane >> 4);

  float rv[3] = {0.0f, 0.0f, 0.0f};
  if constexpr (REC) {
    const int32_t id = a.vid[own_slot];
    if (id >= 0) {
      rv[0] = a.vrec[4 * id];
      rv[1] = a.vrec[4 * id + 1];
      rv[2] = a.vrec[4 * id + 2];
    }
  }

  float h[Q];
  uint32_t unknown = 0;
  int rface = 0;
  h[0] = ST::load(src, pidx(0, own_slot));
  static_for<1, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    const LinkClass lc = classify_link<i, REC>(a.fp, gx, gy, gz, a.nx, a.ny, a.nz, rv);
    uint32_t slot = pull_slot<i>(lane, b, nbv);
    uint32_t plane = i;
    if (lc.kind != kLinkInside || ((bm[i - 1] >> lane) & 1ull)) {
      slot = own_slot;
      plane = kOpp[i];
    }
    float v = ST::load(src, pidx(plane, slot));
    if (lc.kind == kLinkMoving) v = v + lc.extra;
    if (lc.kind == kLinkUnknown) {
      unknown |= 1u << i;
      rface = lc.face;
    }
    h[i] = v;
  });

  if constexpr (FUSED) {
    if (unknown) regularized_face<REC>(h, unknown, rface, a.fp, a.omega, rv);
    else collide<COLL>(h, a.omega);
  }

#pragma unroll
  for (int i = 0; i < Q; ++i) ST::store(dst, pidx(i, own_slot), h[i]);
}

template <class ST, int COLL, bool FUSED>
__global__ __launch_bounds__(256) void k_block_boundary(StepArgs a, int32_t g0, int32_t n) {
  const int wg = xcd_remap(blockIdx.x);
  const int b = __builtin_amdgcn_readfirstlane(g0 + wg * 4 + (int)(threadIdx.x >> 6));
  if (b >= g0 + n) return;
  boundary_block<ST, COLL, FUSED, false>(a, b);
}

// Bitmask-based grouping: visits every block, keeps the boundary ones.
template <class ST, int COLL>
__global__ __launch_bounds__(256) void k_block_boundary_bits(StepArgs a, int32_t g0, int32_t n) {
  const int wg = xcd_remap(blockIdx.x);
  const int b = __builtin_amdgcn_readfirstlane(g0 + wg * 4 + (int)(threadIdx.x >> 6));
  if (b >= g0 + n) return;
  if (!((a.bbits[b >> 5] >> (b & 31)) & 1u)) return;
  boundary_block<ST, COLL, true, true>(a, b);
}

// ------------------------------------------------- collision-only kernel --
// In place on a buffer of pulled populations (the unfused multires
// baseline).  HEAVY blocks re-derive, from their coordinates, which links
// came from a regularized face and rebuild those populations.
template <class ST, int COLL, bool HEAVY>
__global__ __launch_bounds__(256) void k_block_collide(StepArgs a, int32_t g0, int32_t n) {
  using T = typename ST::T;
  const int wg = xcd_remap(blockIdx.x);
  const int b = __builtin_amdgcn_readfirstlane(g0 + wg * 4 + (int)(threadIdx.x >> 6));
  if (b >= g0 + n) return;
  const int lane = threadIdx.x & 63;
  T *__restrict__ buf = (T *)a.dst;
  const uint32_t own_slot = (uint32_t)b * 64u + (uint32_t)lane;
  float h[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) h[i] = ST::load(buf, pidx(i, own_slot));
  if constexpr (HEAVY) {
    const int packed = a.coords[b];
    const int gx = (packed & 1023) * 4 + (lane & 3);
    const int gy = ((packed >> 10) & 1023) * 4 + ((lane >> 2) & 3);
    const int gz = ((packed >> 20) & 1023) * 4 + (lane >> 4);
    uint32_t unknown = 0;
    int rface = 0;
    static_for<1, Q>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      const LinkClass lc = classify_link<i>(a.fp, gx, gy, gz, a.nx, a.ny, a.nz);
      if (lc.kind == kLinkUnknown) {
        unknown |= 1u << i;
        rface = lc.face;
      }
    });
    if (unknown) regularized_face(h, unknown, rface, a.fp, a.omega);
    else collide<COLL>(h, a.omega);
  } else {
    collide<COLL>(h, a.omega);
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) ST::store(buf, pidx(i, own_slot), h[i]);
}

#ifndef LBM_Q27  // D3Q19 only
// ----------------------------------------------- multires jump kernel ---
// Blocks next to a resolution jump.  Each (voxel, direction) has one table
// entry per substep phase: a tagged slot in one of five buffers, or a list
// of 8 such entries whose mean is taken (coalescence onto the 2x2x2
// footprint of a coarse voxel).  Explosion, re-entry and coalescence are all
// gathers, so no atomics and no second pass are needed.
// The five source buffers come in as wave-uniform 64-bit values held in
// scalar registers, and the per-lane choice is a chain of selects between
// them (an indexed read of the argument block, or of a table the compiler
// builds in LDS when the bases sit in an array or structure, would add a
// dependent memory load to every gather: that form measured 20-35% slower
// on the sphere grids).
template <class ST>
__device__ __forceinline__ float mr_fetch(uint64_t p0, uint64_t p1, uint64_t p2, uint64_t p3, uint64_t p4,
                                          uint32_t e, int plane, int opp_plane) {
  using T = typename ST::T;
  const uint32_t tag = e >> 29;
  const uint32_t slot = e & ((1u << 28) - 1u);
  const int pl = (e >> 28) & 1u ? opp_plane : plane;
  uint64_t base = p0;
  base = tag == 1u ? p1 : base;
  base = tag == 2u ? p2 : base;
  base = tag == 3u ? p3 : base;
  base = tag == 4u ? p4 : base;
  return ST::decode(((const __attribute__((address_space(1))) T *)base)[pidx(pl, slot)]);
}

constexpr int kJumpGroup = 4;  // directions whose coalescence lists load together

// Per-block body of the jump kernel (b is wave-uniform).
template <class ST, int COLL, bool FUSED>
__device__ __forceinline__ void mr_jump_block(const StepArgs &a, const MrArgs &m, int b) {
  using T = typename ST::T;
  const int lane = threadIdx.x & 63;
  T *__restrict__ dst = (T *)a.dst;
  const uint32_t own_slot = (uint32_t)b * 64u + (uint32_t)lane;
  const uint32_t *tab = m.jtab + ((size_t)b * 2 + m.phase) * Q * 64 + lane;
  // the five bases as plain 64-bit values (a structure or array of them
  // held in memory lets the compiler turn the selects into a per-lane table
  // in LDS, a dependent LDS read in front of every gather)
  const uint64_t p0 = (uint64_t)m.src[0], p1 = (uint64_t)m.src[1], p2 = (uint64_t)m.src[2],
                 p3 = (uint64_t)m.src[3], p4 = (uint64_t)m.src[4];
  // three rounds of independent loads: the table entries, the direct
  // gathers, then the coalescence lists
  uint32_t e[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) e[i] = tab[i * 64];
  float h[Q];
  static_for<0, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    // a lane with a list entry reads slot 0 of the first buffer here (a
    // valid address) and takes its list mean below
    h[i] = mr_fetch<ST>(p0, p1, p2, p3, p4, (e[i] >> 29) == 7u ? 0u : e[i], i, kOpp[i]);
  });
  // Coalescence lists, kJumpGroup directions at a time: every lane of a
  // group with a list in the wave loads list entries (lanes without one
  // read list 0, which exists then), then all the gathers are issued
  // together, so a wave waits for two memory round trips per group rather
  // than two per direction.  The mean is summed in a fixed order.
  static_for<0, (Q + kJumpGroup - 1) / kJumpGroup>([&](auto gc) {
    constexpr int i0 = decltype(gc)::value * kJumpGroup;
    constexpr int G = Q - i0 < kJumpGroup ? Q - i0 : kJumpGroup;
    bool lst[G];
    bool any = false;
#pragma unroll
    for (int k = 0; k < G; ++k) {
      lst[k] = (e[i0 + k] >> 29) == 7u;
      any = any || lst[k];
    }
    if (__builtin_amdgcn_ballot_w64(any) != 0) {
      uint32_t ent[G][8];
#pragma unroll
      for (int k = 0; k < G; ++k) {
        const uint32_t li = lst[k] ? (e[i0 + k] & ((1u << 28) - 1u)) : 0u;
        const uint4 *p = (const uint4 *)(m.jlist + (size_t)li * 8);
        const uint4 ea = p[0], eb = p[1];
        ent[k][0] = ea.x; ent[k][1] = ea.y; ent[k][2] = ea.z; ent[k][3] = ea.w;
        ent[k][4] = eb.x; ent[k][5] = eb.y; ent[k][6] = eb.z; ent[k][7] = eb.w;
      }
      float v[G][8];
#pragma unroll
      for (int k = 0; k < G; ++k)
#pragma unroll
        for (int j = 0; j < 8; ++j) v[k][j] = mr_fetch<ST>(p0, p1, p2, p3, p4, ent[k][j], i0 + k, kOpp[i0 + k]);
#pragma unroll
      for (int k = 0; k < G; ++k) {
        float sum = v[k][0];
#pragma unroll
        for (int j = 1; j < 8; ++j) sum = sum + v[k][j];
        if (lst[k]) h[i0 + k] = sum * 0.125f;
      }
    }
  });
  if constexpr (FUSED) collide<COLL>(h, a.omega);
#pragma unroll
  for (int i = 0; i < Q; ++i) ST::store(dst, pidx(i, own_slot), h[i]);
}

template <class ST, int COLL, bool FUSED>
__global__ __launch_bounds__(256) void k_mr_jump(StepArgs a, MrArgs m, int32_t g0, int32_t n) {
  const int wg = xcd_remap(blockIdx.x);
  const int b = __builtin_amdgcn_readfirstlane(g0 + wg * 4 + (int)(threadIdx.x >> 6));
  if (b >= g0 + n) return;
  mr_jump_block<ST, COLL, FUSED>(a, m, b);
}

// One launch for all groups of a small multires level update: the groups
// are independent within the update, and a level that holds fewer blocks
// than the chip holds waves is bound by the dispatch and drain of each
// launch rather than by occupancy.  Workgroups take the groups in storage
// order [jump | boundary | masked | full] (cnt[g] blocks each, four per
// workgroup); consecutive workgroups go to different XCDs, which spreads
// every group over the whole chip.  Each block runs the body of its
// group's own kernel.
// JFUSED selects the jump group's form separately (the paper's schedule
// streams jump blocks unfused while the uniform groups are fused).
template <class ST, int COLL, bool FUSED, bool JFUSED>
__device__ __forceinline__ void level_merged_body(const StepArgs &a, const MrArgs &m, int32_t nj, int32_t nbd,
                                                  int32_t nm, int32_t nf, int k) {
  const int wave = (int)(threadIdx.x >> 6);
  const int wj = (nj + 3) >> 2, wb = (nbd + 3) >> 2, wm = (nm + 3) >> 2;
  if (k < wj) {
    const int b = __builtin_amdgcn_readfirstlane(k * 4 + wave);
    if (b < nj) mr_jump_block<ST, COLL, JFUSED>(a, m, b);
    return;
  }
  k -= wj;
  if (k < wb) {
    const int b = __builtin_amdgcn_readfirstlane(k * 4 + wave);
    if (b < nbd) boundary_block<ST, COLL, FUSED, false>(a, nj + b);
    return;
  }
  k -= wb;
  if (k < wm) {
    const int b = __builtin_amdgcn_readfirstlane(k * 4 + wave);
    if (b < nm) interior_block<ST, COLL, true, FUSED>(a, nj + nbd + b);
    return;
  }
  k -= wm;
  const int b = __builtin_amdgcn_readfirstlane(k * 4 + wave);
  if (b < nf) interior_block<ST, COLL, false, FUSED>(a, nj + nbd + nm + b);
}

template <class ST, int COLL, bool FUSED, bool JFUSED = FUSED>
__global__ __launch_bounds__(256) void k_level_merged(StepArgs a, MrArgs m, int32_t nj, int32_t nbd, int32_t nm,
                                                      int32_t nf) {
  // the chunked XCD order over all groups; padding workgroups land past the
  // last full block and exit
  level_merged_body<ST, COLL, FUSED, JFUSED>(a, m, nj, nbd, nm, nf, xcd_remap(blockIdx.x));
}

// Two merged level updates with no buffer in common between one's writes
// and the other's reads or writes -- a coarse level's update and the next
// substep of a level two or more levels finer, or of the finer level's
// second substep, whose reads are the coarse level's current state and
// not the buffer being written -- in one launch: the first update's
// workgroups, then the second's.
template <class ST, int COLL>
__global__ __launch_bounds__(256) void k_level_pair(StepArgs a0, MrArgs m0, int4 c0, StepArgs a1, MrArgs m1,
                                                    int4 c1) {
  const int k = xcd_remap(blockIdx.x);  // padding lands past the second update's last block
  const int w0 = ((c0.x + 3) >> 2) + ((c0.y + 3) >> 2) + ((c0.z + 3) >> 2) + ((c0.w + 3) >> 2);
  if (k < w0) level_merged_body<ST, COLL, true, true>(a0, m0, c0.x, c0.y, c0.z, c0.w, k);
  else level_merged_body<ST, COLL, true, true>(a1, m1, c1.x, c1.y, c1.z, c1.w, k - w0);
}

#endif  // LBM_Q27

// ---------------------------------------------- dense lexicographic arm ---
// One thread per voxel of an all-fluid box stored as [19][nx*ny*nz] with
// x fastest; face rules evaluated inline for every voxel.
template <class ST, int COLL>
__global__ __launch_bounds__(256) void k_lex(StepArgs a) {
  using T = typename ST::T;
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int y = blockIdx.y * 4 + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= a.nx || y >= a.ny) return;
  const T *__restrict__ src = (const T *)a.src;
  T *__restrict__ dst = (T *)a.dst;
  const uint32_t S = a.S;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const uint32_t own = (uint32_t)x + (uint32_t)nx * ((uint32_t)y + (uint32_t)ny * (uint32_t)z);

  float h[Q];
  uint32_t unknown = 0;
  int rface = 0;
  h[0] = ST::load(src, own);
  static_for<1, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    const LinkClass lc = classify_link<i>(a.fp, x, y, z, nx, ny, nz);
    int sx = x - kCx[i], sy = y - kCy[i], sz = z - kCz[i];
    sx = sx < 0 ? sx + nx : (sx >= nx ? sx - nx : sx);
    sy = sy < 0 ? sy + ny : (sy >= ny ? sy - ny : sy);
    sz = sz < 0 ? sz + nz : (sz >= nz ? sz - nz : sz);
    uint32_t slot = (uint32_t)sx + (uint32_t)nx * ((uint32_t)sy + (uint32_t)ny * (uint32_t)sz);
    uint32_t plane = i;
    if (lc.kind != kLinkInside) {
      slot = own;
      plane = kOpp[i];
    }
    float v = ST::load(src + (size_t)plane * S, slot);
    if (lc.kind == kLinkMoving) v = v + lc.extra;
    if (lc.kind == kLinkUnknown) {
      unknown |= 1u << i;
      rface = lc.face;
    }
    h[i] = v;
  });

  if (unknown) regularized_face(h, unknown, rface, a.fp, a.omega);
  else collide<COLL>(h, a.omega);

#pragma unroll
  for (int i = 0; i < Q; ++i) ST::store(dst + (size_t)i * S, own, h[i]);
}

#ifndef LBM_Q27  // D3Q19 only
// ------------------------------------------------------ training sampler --
// splitmix64 (Steele, Lea and Flood 2014), a counter-based generator.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

// Sample k draws block slots uniformly from [b0, b0 + nb) and lanes
// uniformly, rejecting non-fluid voxels, and writes the pre-collision
// populations the collision operator would see there (the pull of the
// interior kernels, bounce-back included), unshifted FP32 [n][19].
template <class ST>
__global__ void k_sample_pre(StepArgs a, int32_t b0, int32_t nb, uint64_t seed, int64_t n, float *out) {
  using T = typename ST::T;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int b = b0, lane = 0;
  for (int attempt = 0; attempt < 4096; ++attempt) {
    const uint64_t r = splitmix64(seed ^ splitmix64((uint64_t)k * 4096u + (uint64_t)attempt));
    const int bb = b0 + (int)((r >> 6) % (uint64_t)nb);
    const int ll = (int)(r & 63u);
    b = bb;
    lane = ll;
    if ((a.fmask[bb] >> ll) & 1ull) break;
  }
  const T *src = (const T *)a.src;
  int32_t nbv[kNbr];
  for (int d = 0; d < kNbr; ++d) nbv[d] = a.nbr[(size_t)b * kNbr + d];
  const uint32_t own = (uint32_t)b * 64u + (uint32_t)lane;
  out[k * Q] = weight_f(0) + ST::load(src, pidx(0, own));
  static_for<1, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    uint32_t slot = pull_slot<i>(lane, b, nbv);
    uint32_t plane = i;
    if ((a.bbm[(size_t)b * kNbr + i - 1] >> lane) & 1ull) {
      slot = own;
      plane = kOpp[i];
    }
    out[k * Q + i] = weight_f(i) + ST::load(src, pidx(plane, slot));
  });
}

hipError_t launch_sample_pre(const StepArgs &a, int32_t storage, int32_t b0, int32_t nb, uint64_t seed, int64_t n,
                             float *out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const dim3 g((unsigned)((n + 255) / 256)), blk(256);
  switch (storage) {
    case LBM_F32: hipLaunchKernelGGL(k_sample_pre<StoreF32>, g, blk, 0, s, a, b0, nb, seed, n, out); break;
    case LBM_F16_SHIFTED: hipLaunchKernelGGL(k_sample_pre<StoreF16>, g, blk, 0, s, a, b0, nb, seed, n, out); break;
    case LBM_BF16_SHIFTED: hipLaunchKernelGGL(k_sample_pre<StoreBF16>, g, blk, 0, s, a, b0, nb, seed, n, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#endif  // LBM_Q27

// --------------------------------------------------------------- launch --
template <class ST, int COLL>
static hipError_t launch_t(const Launch &L, hipStream_t s) {
  if (L.kind == kKernelLex) {
    dim3 blk(64, 4, 1);
    dim3 grd((L.args.nx + 63) / 64, (L.args.ny + 3) / 4, L.args.nz);
    hipLaunchKernelGGL((k_lex<ST, COLL>), grd, blk, L.lds, s, L.args);
    return hipGetLastError();
  }
  const int32_t g0 = L.first, n = L.count;
  if (n <= 0) return hipSuccess;
  const dim3 grd(xcd_grid((n + 3) / 4)), blk(256);  // the block kernels' order (xcd_remap)
  const bool f = L.fused != 0;
  switch (L.kind) {
    case kKernelFull:
      if (f) hipLaunchKernelGGL((k_block_interior<ST, COLL, false, true>), grd, blk, L.lds, s, L.args, g0, n);
      else hipLaunchKernelGGL((k_block_interior<ST, COLL, false, false>), grd, blk, L.lds, s, L.args, g0, n);
      break;
    case kKernelMasked:
      if (f) hipLaunchKernelGGL((k_block_interior<ST, COLL, true, true>), grd, blk, L.lds, s, L.args, g0, n);
      else hipLaunchKernelGGL((k_block_interior<ST, COLL, true, false>), grd, blk, L.lds, s, L.args, g0, n);
      break;
    case kKernelBoundary:
      if (f) hipLaunchKernelGGL((k_block_boundary<ST, COLL, true>), grd, blk, L.lds, s, L.args, g0, n);
      else hipLaunchKernelGGL((k_block_boundary<ST, COLL, false>), grd, blk, L.lds, s, L.args, g0, n);
      break;
#ifndef LBM_Q27
    case kKernelJump:
      if (f) hipLaunchKernelGGL((k_mr_jump<ST, COLL, true>), grd, blk, 0, s, L.args, L.mr, g0, n);
      else hipLaunchKernelGGL((k_mr_jump<ST, COLL, false>), grd, blk, 0, s, L.args, L.mr, g0, n);
      break;
    case kKernelLevelMerged: {
      const int32_t *c = L.gcount;
      const dim3 gm(xcd_grid((c[0] + 3) / 4 + (c[1] + 3) / 4 + (c[2] + 3) / 4 + (c[3] + 3) / 4));
      if (g0 != 0 || c[0] + c[1] + c[2] + c[3] != n) return hipErrorInvalidValue;
      if (L.fused == 2)  // uniform groups fused, jump group streamed only
        hipLaunchKernelGGL((k_level_merged<ST, COLL, true, false>), gm, blk, 0, s, L.args, L.mr, c[0], c[1], c[2],
                           c[3]);
      else if (f)
        hipLaunchKernelGGL((k_level_merged<ST, COLL, true>), gm, blk, 0, s, L.args, L.mr, c[0], c[1], c[2], c[3]);
      else hipLaunchKernelGGL((k_level_merged<ST, COLL, false>), gm, blk, 0, s, L.args, L.mr, c[0], c[1], c[2], c[3]);
      break;
    }
    case kKernelLevelPair: {
      const int32_t *c = L.gcount, *d = L.gcount2;
      const dim3 gm(xcd_grid((c[0] + 3) / 4 + (c[1] + 3) / 4 + (c[2] + 3) / 4 + (c[3] + 3) / 4 + (d[0] + 3) / 4 +
                    (d[1] + 3) / 4 + (d[2] + 3) / 4 + (d[3] + 3) / 4));
      if (!f) return hipErrorInvalidValue;
      hipLaunchKernelGGL((k_level_pair<ST, COLL>), gm, blk, 0, s, L.args, L.mr, make_int4(c[0], c[1], c[2], c[3]),
                         L.args2, L.mr2, make_int4(d[0], d[1], d[2], d[3]));
      break;
    }
#endif
    case kKernelCollide:
      hipLaunchKernelGGL((k_block_collide<ST, COLL, false>), grd, blk, L.lds, s, L.args, g0, n);
      break;
    case kKernelInteriorBits:
      hipLaunchKernelGGL((k_block_interior_bits<ST, COLL>), grd, blk, L.lds, s, L.args, g0, n);
      break;
    case kKernelBoundaryBits:
      hipLaunchKernelGGL((k_block_boundary_bits<ST, COLL>), grd, blk, L.lds, s, L.args, g0, n);
      break;
    case kKernelCollideHeavy:
      hipLaunchKernelGGL((k_block_collide<ST, COLL, true>), grd, blk, L.lds, s, L.args, g0, n);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#ifndef LBM_Q27
template <class ST>
static hipError_t launch_mlp(const Launch &L, hipStream_t s) {
  const int32_t g0 = L.first, n = L.count;
  if (n <= 0) return hipSuccess;
  const dim3 blk(256);
  // 32-bit pull offsets while a population buffer spans at most 4 GiB
  const bool narrow = (uint64_t)L.args.S * Q * sizeof(typename ST::T) <= (1ull << 32) && !L.wide;
  if (L.kind == kKernelFull) {
    // two blocks per wave with 16-bit storage (measured +8%); a second FP32
    // block's pulls do not fit beside the network in the registers of three
    // waves per SIMD (spills: 9% slower)
    constexpr int PB = sizeof(typename ST::T) == 2 ? 2 : 1;
    const dim3 grd(xcd_grid((n + 4 * PB - 1) / (4 * PB)));
    if (narrow) hipLaunchKernelGGL((k_block_interior_mlp<ST, false, true, PB>), grd, blk, 0, s, L.args, g0, n);
    else hipLaunchKernelGGL((k_block_interior_mlp<ST, false, false, PB>), grd, blk, 0, s, L.args, g0, n);
  } else {  // the masked kernels hold bounce masks too: one block per wave
    const dim3 grd(xcd_grid((n + 3) / 4));
    if (narrow) hipLaunchKernelGGL((k_block_interior_mlp<ST, true, true, 1>), grd, blk, 0, s, L.args, g0, n);
    else hipLaunchKernelGGL((k_block_interior_mlp<ST, true, false, 1>), grd, blk, 0, s, L.args, g0, n);
  }
  return hipGetLastError();
}
#endif

hipError_t launch_one(const Launch &L, int32_t storage, int32_t collision, hipStream_t s) {
  if (collision == kCollMLP) {
#ifdef LBM_Q27
    return hipErrorInvalidValue;  // the closure is a D3Q19 network
#else
    // the closure runs on the non-boundary groups; every other kernel uses
    // the regularized operator it was trained to imitate
    if (L.kind == kKernelLevelMerged || L.kind == kKernelLevelPair)
      return hipErrorInvalidValue;  // never scheduled with the closure
    if (L.fused && (L.kind == kKernelFull || L.kind == kKernelMasked)) {
      switch (storage) {
        case LBM_F32: return launch_mlp<StoreF32>(L, s);
        case LBM_F16_SHIFTED: return launch_mlp<StoreF16>(L, s);
        case LBM_BF16_SHIFTED: return launch_mlp<StoreBF16>(L, s);
      }
      return hipErrorInvalidValue;
    }
    collision = kCollRegularized;
#endif
  }
  const bool reg = collision == kCollRegularized;
  switch (storage) {
    case LBM_F32: return reg ? launch_t<StoreF32, kCollRegularized>(L, s) : launch_t<StoreF32, kCollBGK>(L, s);
    case LBM_F16_SHIFTED: return reg ? launch_t<StoreF16, kCollRegularized>(L, s) : launch_t<StoreF16, kCollBGK>(L, s);
    case LBM_BF16_SHIFTED: return reg ? launch_t<StoreBF16, kCollRegularized>(L, s) : launch_t<StoreBF16, kCollBGK>(L, s);
  }
  return hipErrorInvalidValue;
}

}  // inline namespace
}  // namespace lbm
