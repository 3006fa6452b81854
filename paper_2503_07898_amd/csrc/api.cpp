// C ABI of liblbm (declarations and contracts in include/lbm.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "grid.h"
#include "launch.h"
#include "lattice.h"

using namespace lbm;

namespace {

thread_local std::string g_err;

lbm_status fail(lbm_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

lbm_status hip_fail(hipError_t e, const char *what) {
  return fail(LBM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

enum State { kCreated = 0, kCommitted = 1, kBound = 2, kReady = 3 };

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t storage_bytes(int st) { return st == LBM_F32 ? 4 : 2; }

}  // namespace

struct lbm_grid {
  lbm_grid_desc desc{};
  std::vector<uint8_t> fluid;
  FaceBC faces[6];
  int state = kCreated;
  bool lex = false;
  BlockLevel L;
  int64_t S = 0;        // slots per population plane
  int64_t n_fluid = 0;
  // workspace layout (byte offsets)
  size_t off_pop[2] = {0, 0}, off_nbr = 0, off_bbm = 0, off_coords = 0, off_canon = 0,
         off_partial = 0, total = 0;
  char *ws = nullptr;
  int cur = 0;  // index of the buffer holding the current populations
  std::vector<int32_t> packed_coords;
};

extern "C" {

const char *lbm_last_error(void) { return g_err.c_str(); }

lbm_status lbm_grid_create(const lbm_grid_desc *d, lbm_grid **out) {
  if (!d || !out) return fail(LBM_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (d->nx <= 0 || d->ny <= 0 || d->nz <= 0)
    return fail(LBM_ERR_INVALID_ARG, "box sizes must be positive");
  if (!(d->tau > 0.5) || !std::isfinite(d->tau))
    return fail(LBM_ERR_INVALID_ARG, "tau must be finite and > 1/2");
  if (d->storage < LBM_F32 || d->storage > LBM_BF16_SHIFTED)
    return fail(LBM_ERR_INVALID_ARG, "unknown storage");
  if (d->collision < LBM_BGK || d->collision > LBM_MLP)
    return fail(LBM_ERR_INVALID_ARG, "unknown collision");
  if (d->collision == LBM_MLP)
    return fail(LBM_ERR_UNSUPPORTED, "the MLP closure is selected with lbm_set_collision");
  if (d->schedule != LBM_PLAIN_SINGLE_KERNEL && d->schedule != LBM_DISAGG)
    return fail(LBM_ERR_INVALID_ARG, "unknown schedule");
  if (d->kind == LBM_MULTIRES) return fail(LBM_ERR_UNSUPPORTED, "multires grids are not built yet");
  if (d->kind != LBM_DENSE && d->kind != LBM_BLOCK_SPARSE)
    return fail(LBM_ERR_INVALID_ARG, "unknown grid kind");
  if (d->num_levels != 1) return fail(LBM_ERR_INVALID_ARG, "dense and block-sparse grids have 1 level");
  const int64_t nv = (int64_t)d->nx * d->ny * d->nz;
  if (nv * 19 >= ((int64_t)1 << 32)) return fail(LBM_ERR_INVALID_ARG, "box too large for 32-bit offsets");
  lbm_grid *g = new (std::nothrow) lbm_grid;
  if (!g) return fail(LBM_ERR_OUT_OF_MEMORY, "host allocation failed");
  g->desc = *d;
  g->desc.fluid_mask = nullptr;
  g->desc.level_map = nullptr;
  try {
    g->fluid.assign((size_t)nv, 1);
  } catch (...) {
    delete g;
    return fail(LBM_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
  if (d->fluid_mask) {
    for (int64_t i = 0; i < nv; ++i) g->fluid[i] = d->fluid_mask[i] ? 1 : 0;
    if (d->kind == LBM_DENSE) {
      for (int64_t i = 0; i < nv; ++i)
        if (!g->fluid[i]) {
          delete g;
          return fail(LBM_ERR_INVALID_ARG, "dense grids must be all fluid; use LBM_BLOCK_SPARSE for obstacles");
        }
    }
  }
  g->lex = d->kind == LBM_DENSE && d->schedule == LBM_PLAIN_SINGLE_KERNEL;
  if (!g->lex && (d->nx % 4 || d->ny % 4 || d->nz % 4)) {
    delete g;
    return fail(LBM_ERR_INVALID_ARG, "block layouts need box sizes that are multiples of 4");
  }
  *out = g;
  return LBM_OK;
}

lbm_status lbm_set_boundary(lbm_grid *g, lbm_face face, lbm_bc kind, const double value[3]) {
  if (!g) return fail(LBM_ERR_INVALID_ARG, "null grid");
  if (g->state != kCreated) return fail(LBM_ERR_STATE, "boundaries are set before commit");
  if ((int)face < 0 || (int)face > 5) return fail(LBM_ERR_INVALID_ARG, "bad face");
  if ((int)kind < 0 || (int)kind > 3) return fail(LBM_ERR_INVALID_ARG, "bad boundary kind");
  if (g->desc.periodic[(int)face / 2]) return fail(LBM_ERR_INVALID_ARG, "face lies on a periodic axis");
  if ((kind == LBM_BC_REG_VELOCITY || kind == LBM_BC_REG_PRESSURE || kind == LBM_BC_MOVING_WALL) && !value)
    return fail(LBM_ERR_INVALID_ARG, "this boundary kind needs a value");
  if (kind == LBM_BC_REG_PRESSURE && !(value[0] > 0)) return fail(LBM_ERR_INVALID_ARG, "outlet density must be > 0");
  g->faces[face].kind = kind;
  for (int a = 0; a < 3; ++a) g->faces[face].value[a] = value ? value[a] : 0.0;
  return LBM_OK;
}

lbm_status lbm_grid_commit(lbm_grid *g, size_t *bytes) {
  if (!g || !bytes) return fail(LBM_ERR_INVALID_ARG, "null argument");
  if (g->state != kCreated) return fail(LBM_ERR_STATE, "grid already committed");
  const lbm_grid_desc &d = g->desc;
  // a voxel may not need two regularized faces
  for (int f1 = 0; f1 < 6; ++f1)
    for (int f2 = f1 + 1; f2 < 6; ++f2) {
      auto reg = [&](int f) {
        return g->faces[f].kind == LBM_BC_REG_VELOCITY || g->faces[f].kind == LBM_BC_REG_PRESSURE;
      };
      if (!reg(f1) || !reg(f2) || f1 / 2 == f2 / 2) continue;
      const int a1 = f1 / 2, a2 = f2 / 2;
      const int n[3] = {d.nx, d.ny, d.nz};
      const int v1 = (f1 & 1) ? n[a1] - 1 : 0, v2 = (f2 & 1) ? n[a2] - 1 : 0;
      for (int64_t z = 0; z < d.nz; ++z)
        for (int64_t y = 0; y < d.ny; ++y)
          for (int64_t x = 0; x < d.nx; ++x) {
            const int64_t p[3] = {x, y, z};
            if (p[a1] == v1 && p[a2] == v2 && g->fluid[x + d.nx * (y + (int64_t)d.ny * z)])
              return fail(LBM_ERR_INVALID_ARG, "a fluid voxel touches two regularized faces");
          }
    }
  const size_t es = storage_bytes(d.storage);
  if (g->lex) {
    g->S = (int64_t)d.nx * d.ny * d.nz;
    g->n_fluid = g->S;
    size_t off = 0;
    for (int k = 0; k < 2; ++k) {
      g->off_pop[k] = off;
      off = align256(off + (size_t)g->S * Q * es);
    }
    g->off_partial = off;
    off = align256(off + (size_t)((g->S + 63) / 64) * 5 * sizeof(double));
    g->total = off;
  } else {
    std::string e = build_block_level(g->L, d.nx, d.ny, d.nz, d.periodic, g->fluid, g->faces,
                                      d.kind == LBM_DENSE);
    if (!e.empty()) return fail(LBM_ERR_INVALID_ARG, "%s", e.c_str());
    const BlockLevel &L = g->L;
    g->S = L.nblocks * 64;
    g->n_fluid = L.n_fluid;
    g->packed_coords.resize(L.nblocks);
    for (int64_t b = 0; b < L.nblocks; ++b)
      g->packed_coords[b] = L.coords[3 * b] | (L.coords[3 * b + 1] << 10) | (L.coords[3 * b + 2] << 20);
    size_t off = 0;
    for (int k = 0; k < 2; ++k) {
      g->off_pop[k] = off;
      off = align256(off + (size_t)g->S * Q * es);
    }
    g->off_nbr = off;
    off = align256(off + (size_t)L.nblocks * 18 * 4);
    g->off_bbm = off;
    off = align256(off + (size_t)L.nblocks * 18 * 8);
    g->off_coords = off;
    off = align256(off + (size_t)L.nblocks * 4);
    g->off_canon = off;
    off = align256(off + (size_t)g->S * 4);
    g->off_partial = off;
    off = align256(off + (size_t)L.nblocks * 5 * sizeof(double));
    g->total = off;
  }
  *bytes = g->total;
  g->state = kCommitted;
  return LBM_OK;
}

lbm_status lbm_grid_bind(lbm_grid *g, void *ws, size_t bytes, void *stream) {
  if (!g || !ws) return fail(LBM_ERR_INVALID_ARG, "null argument");
  if (g->state != kCommitted) return fail(LBM_ERR_STATE, "bind needs a committed, unbound grid");
  if (bytes < g->total) return fail(LBM_ERR_INVALID_ARG, "workspace too small (%zu < %zu)", bytes, g->total);
  if (((uintptr_t)ws) & 255) return fail(LBM_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  g->ws = (char *)ws;
  hipStream_t s = (hipStream_t)stream;
  if (!g->lex) {
    const BlockLevel &L = g->L;
    hipError_t e;
    // synchronous copies: the host tables may be freed by the caller afterwards
    if ((e = hipMemcpyAsync(g->ws + g->off_nbr, L.nbr.data(), L.nbr.size() * 4, hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(g->ws + g->off_bbm, L.bbm.data(), L.bbm.size() * 8, hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(g->ws + g->off_coords, g->packed_coords.data(), g->packed_coords.size() * 4,
                            hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(g->ws + g->off_canon, L.canon.data(), L.canon.size() * 4, hipMemcpyHostToDevice, s)) ||
        (e = hipStreamSynchronize(s)))
      return hip_fail(e, "uploading index tables");
  }
  g->state = kBound;
  return LBM_OK;
}

lbm_status lbm_num_voxels(const lbm_grid *g, int32_t level, int64_t *n) {
  if (!g || !n) return fail(LBM_ERR_INVALID_ARG, "null argument");
  if (g->state < kCommitted) return fail(LBM_ERR_STATE, "commit first");
  if (level != 0) return fail(LBM_ERR_INVALID_ARG, "level out of range");
  *n = g->n_fluid;
  return LBM_OK;
}

static SlotArgs slot_args(const lbm_grid *g) {
  SlotArgs A{};
  A.pop_a = g->ws + g->off_pop[g->cur];
  A.pop_b = g->ws + g->off_pop[1 - g->cur];
  A.S = (uint32_t)g->S;
  A.nslots = g->S;
  A.canon = g->lex ? nullptr : (const int32_t *)(g->ws + g->off_canon);
  A.n = g->n_fluid;
  A.storage = g->desc.storage;
  return A;
}

lbm_status lbm_init_equilibrium(lbm_grid *g, int32_t level, const double *rho, const double *u, void *stream) {
  if (!g || !rho || !u) return fail(LBM_ERR_INVALID_ARG, "null argument");
  if (g->state < kBound) return fail(LBM_ERR_STATE, "bind first");
  if (level != 0) return fail(LBM_ERR_INVALID_ARG, "level out of range");
  hipError_t e = launch_init_equilibrium(slot_args(g), rho, u, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "init_equilibrium");
  g->state = kReady;
  return LBM_OK;
}

static StepLaunch make_step(const lbm_grid *g) {
  StepLaunch L{};
  const lbm_grid_desc &d = g->desc;
  L.args.S = (uint32_t)g->S;
  L.args.nx = d.nx;
  L.args.ny = d.ny;
  L.args.nz = d.nz;
  L.args.omega = (float)(1.0 / d.tau);
  for (int f = 0; f < 6; ++f) {
    L.args.fp.kind[f] = g->faces[f].kind;
    for (int a = 0; a < 3; ++a) L.args.fp.val[f][a] = (float)g->faces[f].value[a];
  }
  L.args.fp.periodic = (d.periodic[0] ? 1 : 0) | (d.periodic[1] ? 2 : 0) | (d.periodic[2] ? 4 : 0);
  L.storage = d.storage;
  L.collision = d.collision == LBM_REGULARIZED ? 1 : 0;
  L.lex = g->lex;
  if (!g->lex) {
    L.args.nbr = (const int32_t *)(g->ws + g->off_nbr);
    L.args.bbm = (const uint64_t *)(g->ws + g->off_bbm);
    L.args.coords = (const int32_t *)(g->ws + g->off_coords);
    const auto &gc = g->L.group_count;
    if (d.schedule == LBM_PLAIN_SINGLE_KERNEL) {
      L.nlaunch = 1;
      L.kind[0] = kKernelBoundary;
      L.first[0] = 0;
      L.count[0] = (int32_t)g->L.nblocks;
    } else {
      // largest group first; the groups are independent within a step
      const int32_t first[3] = {0, (int32_t)gc[0], (int32_t)(gc[0] + gc[1])};
      const int32_t kind[3] = {kKernelBoundary, kKernelMasked, kKernelFull};
      int order[3] = {2, 1, 0};
      L.nlaunch = 0;
      for (int k : order)
        if (gc[k] > 0) {
          L.kind[L.nlaunch] = kind[k];
          L.first[L.nlaunch] = first[k];
          L.count[L.nlaunch] = (int32_t)gc[k];
          ++L.nlaunch;
        }
    }
  }
  return L;
}

lbm_status lbm_step(lbm_grid *g, int32_t n, void *stream) {
  if (!g) return fail(LBM_ERR_INVALID_ARG, "null grid");
  if (g->state < kReady) return fail(LBM_ERR_STATE, "initialise the populations first");
  if (n < 0) return fail(LBM_ERR_INVALID_ARG, "negative step count");
  StepLaunch L = make_step(g);
  for (int32_t k = 0; k < n; ++k) {
    L.args.src = g->ws + g->off_pop[g->cur];
    L.args.dst = g->ws + g->off_pop[1 - g->cur];
    hipError_t e = launch_step(L, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "step launch");
    g->cur = 1 - g->cur;
  }
  return LBM_OK;
}

lbm_status lbm_step_launches(const lbm_grid *g, int64_t *blocks_out, int32_t max, int32_t *n) {
  if (!g || !n) return fail(LBM_ERR_INVALID_ARG, "null argument");
  if (g->state < kCommitted) return fail(LBM_ERR_STATE, "commit first");
  StepLaunch L = make_step(g);
  if (g->lex) {
    *n = 1;
    if (blocks_out && max >= 1) blocks_out[0] = (g->S + 63) / 64;
    return LBM_OK;
  }
  *n = L.nlaunch;
  for (int k = 0; k < L.nlaunch && k < max && blocks_out; ++k) blocks_out[k] = L.count[k];
  return LBM_OK;
}

lbm_status lbm_launch_group(lbm_grid *g, int32_t k, void *stream) {
  if (!g) return fail(LBM_ERR_INVALID_ARG, "null grid");
  if (g->state < kReady) return fail(LBM_ERR_STATE, "initialise the populations first");
  StepLaunch L = make_step(g);
  L.args.src = g->ws + g->off_pop[g->cur];
  L.args.dst = g->ws + g->off_pop[1 - g->cur];
  if (g->lex) {
    if (k != 0) return fail(LBM_ERR_INVALID_ARG, "launch index out of range");
  } else {
    if (k < 0 || k >= L.nlaunch) return fail(LBM_ERR_INVALID_ARG, "launch index out of range");
    L.kind[0] = L.kind[k];
    L.first[0] = L.first[k];
    L.count[0] = L.count[k];
    L.nlaunch = 1;
  }
  hipError_t e = launch_step(L, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "launch_group");
  return LBM_OK;
}

lbm_status lbm_read_macroscopic(lbm_grid *g, int32_t level, void *rho, void *u, int32_t f64, void *stream) {
  if (!g || !rho || !u) return fail(LBM_ERR_INVALID_ARG, "null argument");
  if (g->state < kReady) return fail(LBM_ERR_STATE, "initialise the populations first");
  if (level != 0) return fail(LBM_ERR_INVALID_ARG, "level out of range");
  hipError_t e = launch_read_macroscopic(slot_args(g), rho, u, f64 ? 1 : 0, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "read_macroscopic");
  return LBM_OK;
}

lbm_status lbm_read_populations(lbm_grid *g, int32_t level, double *f, void *stream) {
  if (!g || !f) return fail(LBM_ERR_INVALID_ARG, "null argument");
  if (g->state < kReady) return fail(LBM_ERR_STATE, "initialise the populations first");
  if (level != 0) return fail(LBM_ERR_INVALID_ARG, "level out of range");
  hipError_t e = launch_read_populations(slot_args(g), f, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "read_populations");
  return LBM_OK;
}

lbm_status lbm_write_populations(lbm_grid *g, int32_t level, const double *f, void *stream) {
  if (!g || !f) return fail(LBM_ERR_INVALID_ARG, "null argument");
  if (g->state < kBound) return fail(LBM_ERR_STATE, "bind first");
  if (level != 0) return fail(LBM_ERR_INVALID_ARG, "level out of range");
  // slots of non-fluid voxels are never read by any kernel, so only fluid
  // slots are written
  hipError_t e = launch_write_populations(slot_args(g), f, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "write_populations");
  g->state = kReady;
  return LBM_OK;
}

lbm_status lbm_reduce(lbm_grid *g, double *out5, void *stream) {
  if (!g || !out5) return fail(LBM_ERR_INVALID_ARG, "null argument");
  if (g->state < kReady) return fail(LBM_ERR_STATE, "initialise the populations first");
  SlotArgs A = slot_args(g);
  double *partial = (double *)(g->ws + g->off_partial);
  hipError_t e = launch_reduce_partial(A, 1.0, partial, (hipStream_t)stream);
  if (e == hipSuccess) e = launch_reduce_final(partial, (A.nslots + 63) / 64, out5, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "reduce");
  return LBM_OK;
}

lbm_status lbm_get_index_map(const lbm_grid *g, int32_t level, lbm_map which, void *out, size_t *count) {
  if (!g || !count) return fail(LBM_ERR_INVALID_ARG, "null argument");
  if (g->state < kCommitted) return fail(LBM_ERR_STATE, "commit first");
  if (level != 0) return fail(LBM_ERR_INVALID_ARG, "level out of range");
  if (g->lex) return fail(LBM_ERR_UNSUPPORTED, "the lexicographic dense arm has no block maps");
  const BlockLevel &L = g->L;
  size_t n = 0;
  switch (which) {
    case LBM_MAP_GROUPS: {
      n = 4;
      if (out) {
        int64_t *o = (int64_t *)out;
        o[0] = L.group_count[0];
        o[1] = L.group_count[1];
        o[2] = L.group_count[2];
        o[3] = L.nblocks;
      }
      break;
    }
    case LBM_MAP_COORDS: n = L.coords.size(); if (out) memcpy(out, L.coords.data(), n * 4); break;
    case LBM_MAP_NEIGHBOURS: n = L.nbr.size(); if (out) memcpy(out, L.nbr.data(), n * 4); break;
    case LBM_MAP_FLUIDMASK: n = L.fmask.size(); if (out) memcpy(out, L.fmask.data(), n * 8); break;
    case LBM_MAP_CANONICAL: {
      n = L.canon.size();
      if (out) {
        int64_t *o = (int64_t *)out;
        for (size_t i = 0; i < n; ++i) o[i] = L.canon[i];
      }
      break;
    }
    default: return fail(LBM_ERR_INVALID_ARG, "unknown map");
  }
  *count = n;
  return LBM_OK;
}

lbm_status lbm_grid_destroy(lbm_grid *g) {
  delete g;
  return LBM_OK;
}

}  // extern "C"
