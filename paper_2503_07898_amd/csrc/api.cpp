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
#include "mlp_device.h"

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

// Device-side layout and time state of one level.
struct LevelRT {
  const BlockLevel *L = nullptr;  // null for the lexicographic dense arm
  const MultiresLevel *M = nullptr;
  int32_t nx = 0, ny = 0, nz = 0;  // level box in level voxels
  int64_t S = 0;                   // slots per population plane
  int64_t n_fluid = 0;
  double tau = 0.6;
  int nbuf = 2;
  size_t off_pop[3] = {0, 0, 0};
  size_t off_nbr = 0, off_bbm = 0, off_coords = 0, off_canon = 0, off_jtab = 0, off_jlist = 0, off_fmask = 0;
  size_t off_bbits = 0, off_vid = 0, off_vrec = 0;  // bitmask layout
  int64_t partial_row0 = 0;        // first row of this level in the reduction partials
  int cur = 0, prev = 2, nxt = 1;  // roles of the population buffers
  std::vector<int32_t> packed;
};

}  // namespace

struct lbm_mlp {
  size_t total = 0;
  float judge = 0.01f;  // relative L2 tolerance of the closure against the regularized f1
  size_t off_params = 0, off_m = 0, off_v = 0, off_grads = 0, off_w = 0, off_bias = 0, off_stdz = 0,
         off_fb = 0, off_save = 0, off_dyt = 0, off_dz1 = 0, off_dz2 = 0, off_partial = 0, off_loss = 0,
         off_gpartial = 0, off_s2 = 0;
  char *ws = nullptr;
  MlpBuffers B{};
};

// Lattice-specific launchers (the kernels are compiled once per lattice).
struct LatticeLaunchers {
  hipError_t (*one)(const Launch &, int32_t, int32_t, hipStream_t);
  hipError_t (*init_eq)(const SlotArgs &, const double *, const double *, hipStream_t);
  hipError_t (*read_macro)(const SlotArgs &, void *, void *, int, hipStream_t);
  hipError_t (*read_pop)(const SlotArgs &, double *, hipStream_t);
  hipError_t (*write_pop)(const SlotArgs &, const double *, hipStream_t);
  hipError_t (*reduce_partial)(const SlotArgs &, double, double *, hipStream_t);
  hipError_t (*reduce_final)(const double *, int64_t, double *, double *, hipStream_t);
  hipError_t (*reduce_noalloc)(const ReduceLevels &, double *, hipStream_t);
};
#define LBM_LAUNCHERS_OF(ns)                                                                          \
  LatticeLaunchers {                                                                                  \
    &ns::launch_one, &ns::launch_init_equilibrium, &ns::launch_read_macroscopic,                      \
        &ns::launch_read_populations, &ns::launch_write_populations, &ns::launch_reduce_partial,      \
        &ns::launch_reduce_final, &ns::launch_reduce_noalloc                                          \
  }

// Multires levels up to this many blocks run each update as one launch by
// default: 8,192 waves fill the chip at eight waves per SIMD, so a smaller
// level's separate group launches are bound by their dispatch and drain,
// not by occupancy.
constexpr int64_t kMergeMaxBlocks = 8192;

struct lbm_grid {
  lbm_grid_desc desc{};
  int32_t q = 19;  // lattice
  int64_t merge_max = kMergeMaxBlocks;  // multires: merged level updates up to this many blocks
  int32_t residency = LBM_RESIDENCY_AUTO;  // workgroups per CU of the block kernels, 0 = no cap
  bool lds_sized = false;                  // lds_of filled for the current device
  int32_t wide = 0;                        // 1: 64-bit pull addressing whatever the buffer size
  uint32_t lds_of[9] = {};                 // LDS bytes per workgroup that cap residency at w
  LatticeLaunchers ops = LBM_LAUNCHERS_OF(lbm::k19);
  int32_t collision = LBM_BGK;
  const lbm_mlp *mlp = nullptr;
  std::vector<uint8_t> fluid;
  std::vector<uint8_t> level_map;
  FaceBC faces[6];
  int state = kCreated;
  bool lex = false;
  BlockLevel single;              // dense / block-sparse
  std::vector<MultiresLevel> mr;  // multires
  std::vector<LevelRT> lv;
  // launch lists of one step, one per buffer-role state met so far (roles
  // cycle with a period of at most 6 steps); cleared when the collision, the
  // closure or the merge limit changes
  struct StepPlan {
    std::vector<int32_t> roles_in, roles_out;  // (cur, prev, nxt) of every level
    std::vector<Launch> launches;
  };
  std::vector<StepPlan> plans;
  size_t off_partial = 0, off_mid = 0, off_check = 0, total = 0;
  int64_t partial_rows = 0;
  char *ws = nullptr;
};

namespace {

void *pop_ptr(const lbm_grid *g, const LevelRT &r, int role) { return g->ws + r.off_pop[role]; }

StepArgs level_args(const lbm_grid *g, const LevelRT &r) {
  StepArgs a{};
  a.S = (uint32_t)r.S;
  a.nx = r.nx;
  a.ny = r.ny;
  a.nz = r.nz;
  a.omega = (float)(1.0 / r.tau);
  for (int f = 0; f < 6; ++f) {
    a.fp.kind[f] = g->faces[f].kind;
    for (int k = 0; k < 3; ++k) a.fp.val[f][k] = (float)g->faces[f].value[k];
  }
  const uint8_t *p = g->desc.periodic;
  a.fp.periodic = (p[0] ? 1 : 0) | (p[1] ? 2 : 0) | (p[2] ? 4 : 0);
  if (r.L) {
    a.nbr = (const int32_t *)(g->ws + r.off_nbr);
    a.bbm = (const uint64_t *)(g->ws + r.off_bbm);
    a.coords = (const int32_t *)(g->ws + r.off_coords);
    a.fmask = (const uint64_t *)(g->ws + r.off_fmask);
    if (!r.L->grouped) {
      a.bbits = (const uint32_t *)(g->ws + r.off_bbits);
      a.vid = (const int32_t *)(g->ws + r.off_vid);
      a.vrec = (const float *)(g->ws + r.off_vrec);
    }
  }
  if (g->mlp) {
    a.mlp_w = g->mlp->B.wpacked;
    a.mlp_bias = g->mlp->B.bias;
    a.mlp_stdz = g->mlp->B.stdz;
    a.mlp_s2 = g->mlp->B.s2;
    a.mlp_fallbacks = g->mlp->B.fallbacks;
    a.mlp_judge = g->mlp->judge;
  }
  return a;
}

// Launches of one level update with the level's current buffer roles.
void level_update(const lbm_grid *g, const std::vector<LevelRT> &lv, int l, int substep,
                  std::vector<Launch> &out) {
  const LevelRT &r = lv[l];
  StepArgs a = level_args(g, r);
  a.src = pop_ptr(g, r, r.cur);
  a.dst = pop_ptr(g, r, r.nxt);
  if (g->lex) {
    Launch x{};
    x.kind = kKernelLex;
    x.fused = 1;
    x.count = (int32_t)((r.S + 63) / 64);
    x.args = a;
    out.push_back(x);
    return;
  }
  const auto &gc = r.L->group_count;
  const int32_t first[4] = {0, (int32_t)gc[0], (int32_t)(gc[0] + gc[1]), (int32_t)(gc[0] + gc[1] + gc[2])};
  const int32_t nb = (int32_t)r.L->nblocks;
  const bool multires = g->desc.kind == LBM_MULTIRES;
  const bool plain = g->desc.schedule == LBM_PLAIN_SINGLE_KERNEL;
  auto push = [&](int32_t kind, int32_t fused, int32_t f0, int32_t n) {
    if (n <= 0) return;
    Launch x{};
    x.kind = kind;
    x.fused = fused;
    x.first = f0;
    x.count = n;
    x.args = a;
    if (kind == kKernelJump || kind == kKernelLevelMerged) {
      MrArgs &m = x.mr;
      const LevelRT *fr = l > 0 ? &lv[l - 1] : nullptr;
      const LevelRT *cr = l + 1 < (int)lv.size() ? &lv[l + 1] : nullptr;
      m.src[0] = pop_ptr(g, r, r.cur);
      m.src[1] = pop_ptr(g, r, r.prev);
      m.src[2] = fr ? pop_ptr(g, *fr, fr->cur) : m.src[0];
      m.src[3] = fr ? pop_ptr(g, *fr, fr->prev) : m.src[0];
      m.src[4] = cr ? pop_ptr(g, *cr, cr->cur) : m.src[0];
      m.stride[0] = m.stride[1] = (uint32_t)r.S;
      m.stride[2] = m.stride[3] = fr ? (uint32_t)fr->S : (uint32_t)r.S;
      m.stride[4] = cr ? (uint32_t)cr->S : (uint32_t)r.S;
      m.jtab = (const uint32_t *)(g->ws + r.off_jtab);
      m.jlist = (const uint32_t *)(g->ws + r.off_jlist);
      m.phase = substep == 2 ? 1 : 0;
    }
    out.push_back(x);
  };
  if (!multires) {
    if (plain) {
      push(kKernelBoundary, 1, 0, nb);  // the naive single kernel
    } else if (!r.L->grouped) {
      // bitmask-based grouping: both kernels over every block
      push(kKernelInteriorBits, 1, 0, nb);
      push(kKernelBoundaryBits, 1, 0, nb);
    } else {
      // largest group first; the groups are independent within a step
      push(kKernelFull, 1, first[3], (int32_t)gc[3]);
      push(kKernelMasked, 1, first[2], (int32_t)gc[2]);
      push(kKernelBoundary, 1, first[1], (int32_t)gc[1]);
    }
    return;
  }
  // a level with fewer blocks than the chip holds waves at once runs its
  // independent group kernels as one launch (the closure keeps its own
  // kernels)
  const bool merge = nb <= g->merge_max && g->collision != LBM_MLP;
  auto push_merged = [&](int32_t fused) {
    push(kKernelLevelMerged, fused, 0, nb);
    for (int k = 0; k < 4; ++k) out.back().gcount[k] = (int32_t)gc[k];
  };
  if (g->desc.schedule == LBM_DISAGG_UNIFORM_FUSED && l > 0) {
    // the paper's schedule: uniform groups fused, the jump group streamed
    // (gathers stored) and then collided in place; the groups are
    // independent, so the jump collision may follow the uniform kernels
    if (merge) {
      push_merged(2);
    } else {
      push(kKernelFull, 1, first[3], (int32_t)gc[3]);
      push(kKernelMasked, 1, first[2], (int32_t)gc[2]);
      push(kKernelBoundary, 1, first[1], (int32_t)gc[1]);
      push(kKernelJump, 0, first[0], (int32_t)gc[0]);
    }
    push(kKernelCollide, 1, first[0], (int32_t)gc[0]);
    return;
  }
  if (plain && l > 0) {
    // unfused baseline: streaming kernels, then collision in place
    if (merge) {
      push_merged(0);
    } else {
      push(kKernelJump, 0, first[0], (int32_t)gc[0]);
      push(kKernelBoundary, 0, first[1], (int32_t)gc[1]);
      push(kKernelMasked, 0, first[2], (int32_t)gc[2]);
      push(kKernelFull, 0, first[3], (int32_t)gc[3]);
    }
    push(kKernelCollide, 1, first[0], (int32_t)gc[0]);
    push(kKernelCollideHeavy, 1, first[1], (int32_t)gc[1]);
    push(kKernelCollide, 1, first[2], (int32_t)(gc[2] + gc[3]));
    return;
  }
  // fused collide-and-stream on every group (the jump group through its tables)
  if (merge) {
    push_merged(1);
    return;
  }
  push(kKernelFull, 1, first[3], (int32_t)gc[3]);
  push(kKernelMasked, 1, first[2], (int32_t)gc[2]);
  push(kKernelBoundary, 1, first[1], (int32_t)gc[1]);
  push(kKernelJump, 1, first[0], (int32_t)gc[0]);
}

void rotate(LevelRT &r) {
  if (r.nbuf == 2) {
    std::swap(r.cur, r.nxt);
  } else {
    const int old_prev = r.prev;
    r.prev = r.cur;
    r.cur = r.nxt;
    r.nxt = old_prev;
  }
}

// Level-recursive schedule: the finer level's first substep, this level's
// update, the finer level's second substep, then the buffer rotation.
void level_schedule(const lbm_grid *g, std::vector<LevelRT> &lv, int l, int substep,
                    std::vector<Launch> &out) {
  if (l > 0) level_schedule(g, lv, l - 1, 1, out);
  level_update(g, lv, l, substep, out);
  if (l > 0) level_schedule(g, lv, l - 1, 2, out);
  rotate(lv[l]);
}

// Buffers a launch reads and writes (for the independence test below).
void launch_buffers(const Launch &x, std::vector<const void *> &rd, std::vector<const void *> &wr) {
  rd.assign({x.args.src});
  if (x.kind == kKernelJump || x.kind == kKernelLevelMerged)
    for (int t = 0; t < 5; ++t) rd.push_back(x.mr.src[t]);
  wr.assign({x.args.dst});
}

bool disjoint(const std::vector<const void *> &a, const std::vector<const void *> &b) {
  for (const void *p : a)
    for (const void *q : b)
      if (p == q) return false;
  return true;
}

// Launches of one (coarse) step; lv is advanced to the state after it.
// Consecutive fused merged level updates that share no buffer between one's
// writes and the other's reads or writes run as one launch (on a 3-level
// grid of small levels: 7 level updates in 4 launches).
void step_launches(const lbm_grid *g, std::vector<LevelRT> &lv, std::vector<Launch> &out) {
  std::vector<Launch> seq;
  level_schedule(g, lv, (int)lv.size() - 1, 0, seq);
  out.clear();
  std::vector<const void *> r0, w0, r1, w1;
  for (size_t k = 0; k < seq.size(); ++k) {
    const Launch &a = seq[k];
    if (k + 1 < seq.size() && a.kind == kKernelLevelMerged && a.fused == 1 &&
        seq[k + 1].kind == kKernelLevelMerged && seq[k + 1].fused == 1) {
      const Launch &b = seq[k + 1];
      launch_buffers(a, r0, w0);
      launch_buffers(b, r1, w1);
      if (disjoint(w0, r1) && disjoint(w0, w1) && disjoint(w1, r0)) {
        Launch x = a;
        x.kind = kKernelLevelPair;
        x.count = a.count + b.count;
        for (int t = 0; t < 4; ++t) x.gcount2[t] = b.gcount[t];
        x.args2 = b.args;
        x.mr2 = b.mr;
        out.push_back(x);
        ++k;
        continue;
      }
    }
    out.push_back(a);
  }
}

SlotArgs slot_args(const lbm_grid *g, const LevelRT &r) {
  SlotArgs A{};
  A.pop_a = pop_ptr(g, r, r.cur);
  A.pop_b = pop_ptr(g, r, r.nxt);
  A.S = (uint32_t)r.S;
  A.nslots = r.S;
  A.canon = r.L ? (const int32_t *)(g->ws + r.off_canon) : nullptr;
  A.n = r.n_fluid;
  A.storage = g->desc.storage;
  A.blocked = r.L ? 1 : 0;
  return A;
}

lbm_status check_level(const lbm_grid *g, int32_t level) {
  if (level < 0 || level >= (int32_t)g->lv.size()) return fail(LBM_ERR_INVALID_ARG, "level out of range");
  return LBM_OK;
}

int32_t coll_code(const lbm_grid *g) {
  return g->collision == LBM_MLP ? 2 : (g->collision == LBM_REGULARIZED ? 1 : 0);
}

std::vector<int32_t> roles_of(const std::vector<LevelRT> &lv) {
  std::vector<int32_t> r;
  r.reserve(3 * lv.size());
  for (const LevelRT &x : lv) {
    r.push_back(x.cur);
    r.push_back(x.prev);
    r.push_back(x.nxt);
  }
  return r;
}

// The launch plan of the next step from the grid's current buffer roles,
// built (from a copy of the level state) the first time those roles occur.
const lbm_grid::StepPlan &step_plan(lbm_grid *g) {
  const std::vector<int32_t> key = roles_of(g->lv);
  for (const auto &p : g->plans)
    if (p.roles_in == key) return p;
  lbm_grid::StepPlan p;
  p.roles_in = key;
  std::vector<LevelRT> next = g->lv;
  step_launches(g, next, p.launches);
  p.roles_out = roles_of(next);
  g->plans.push_back(std::move(p));
  return g->plans.back();
}

// The closure's GELU, 0.5 x (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3))), as
// kGeluSegs linear pieces over [-8, 8): piece j on [x0, x0 + h] is the
// chord through its end points lowered by the mean of the largest and
// smallest deviation of the function from the chord (sampled), which
// halves the worst error.  (slope, intercept) per piece, FP64 -> FP32.
std::vector<float> gelu_table() {
  auto gelu = [](double x) { return 0.5 * x * (1.0 + std::tanh(0.7978845608028654 * (x + 0.044715 * x * x * x))); };
  std::vector<float> t(2 * kGeluSegs);
  const double h = 1.0 / kGeluPerUnit;
  for (int j = 0; j < kGeluSegs; ++j) {  // piece j is centred on -8 + j h
    const double x0 = -8.0 + (j - 0.5) * h, x1 = x0 + h;
    const double a = (gelu(x1) - gelu(x0)) / h, b = gelu(x0) - a * x0;
    double dmin = 0.0, dmax = 0.0;
    for (int k = 1; k < 64; ++k) {
      const double x = x0 + h * k / 64.0, d = gelu(x) - (a * x + b);
      dmin = std::min(dmin, d);
      dmax = std::max(dmax, d);
    }
    t[2 * j] = (float)a;
    t[2 * j + 1] = (float)(b + 0.5 * (dmin + dmax));
  }
  return t;
}

}  // namespace

extern "C" {

const char *lbm_last_error(void) { return g_err.c_str(); }

lbm_status lbm_grid_create(const lbm_grid_desc *d, lbm_grid **out) {
  if (!d || !out) return fail(LBM_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (d->nx <= 0 || d->ny <= 0 || d->nz <= 0) return fail(LBM_ERR_INVALID_ARG, "box sizes must be positive");
  if (!(d->tau > 0.5) || !std::isfinite(d->tau)) return fail(LBM_ERR_INVALID_ARG, "tau must be finite and > 1/2");
  if (d->storage < LBM_F32 || d->storage > LBM_BF16_SHIFTED) return fail(LBM_ERR_INVALID_ARG, "unknown storage");
  if (d->collision < LBM_BGK || d->collision > LBM_MLP) return fail(LBM_ERR_INVALID_ARG, "unknown collision");
  if (d->collision == LBM_MLP)
    return fail(LBM_ERR_UNSUPPORTED, "the MLP closure is selected with lbm_set_collision");
  if (d->schedule != LBM_PLAIN_SINGLE_KERNEL && d->schedule != LBM_DISAGG && d->schedule != LBM_DISAGG_BITMASK &&
      d->schedule != LBM_DISAGG_UNIFORM_FUSED)
    return fail(LBM_ERR_INVALID_ARG, "unknown schedule");
  if (d->schedule == LBM_DISAGG_BITMASK && d->kind == LBM_MULTIRES)
    return fail(LBM_ERR_UNSUPPORTED, "bitmask-based grouping is built for dense and block-sparse grids");
  if (d->schedule == LBM_DISAGG_UNIFORM_FUSED && d->kind != LBM_MULTIRES)
    return fail(LBM_ERR_INVALID_ARG, "LBM_DISAGG_UNIFORM_FUSED is a multires schedule");
  if (d->lattice != 0 && d->lattice != 19 && d->lattice != 27)
    return fail(LBM_ERR_INVALID_ARG, "lattice must be 19 or 27");
  if (d->lattice == 27 && d->kind == LBM_MULTIRES)
    return fail(LBM_ERR_UNSUPPORTED, "multires grids are built for D3Q19");
  if (d->kind != LBM_DENSE && d->kind != LBM_BLOCK_SPARSE && d->kind != LBM_MULTIRES)
    return fail(LBM_ERR_INVALID_ARG, "unknown grid kind");
  if (d->kind != LBM_MULTIRES && d->num_levels != 1)
    return fail(LBM_ERR_INVALID_ARG, "dense and block-sparse grids have 1 level");
  if (d->kind == LBM_MULTIRES && (d->num_levels < 2 || !d->level_map))
    return fail(LBM_ERR_INVALID_ARG, "multires grids need num_levels >= 2 and a level map");
  const int64_t nv = (int64_t)d->nx * d->ny * d->nz;
  if (d->kind == LBM_DENSE && d->schedule == LBM_PLAIN_SINGLE_KERNEL && nv >= ((int64_t)1 << 31))
    return fail(LBM_ERR_INVALID_ARG, "box too large for 32-bit slot indices");
  lbm_grid *g = new (std::nothrow) lbm_grid;
  if (!g) return fail(LBM_ERR_OUT_OF_MEMORY, "host allocation failed");
  g->desc = *d;
  g->collision = d->collision;
  g->desc.fluid_mask = nullptr;
  g->desc.level_map = nullptr;
  try {
    g->fluid.assign((size_t)nv, 1);
    if (d->fluid_mask)
      for (int64_t i = 0; i < nv; ++i) g->fluid[i] = d->fluid_mask[i] ? 1 : 0;
    if (d->kind == LBM_MULTIRES) g->level_map.assign(d->level_map, d->level_map + nv);
  } catch (...) {
    delete g;
    return fail(LBM_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
  if (d->kind == LBM_DENSE && d->fluid_mask) {
    for (int64_t i = 0; i < nv; ++i)
      if (!g->fluid[i]) {
        delete g;
        return fail(LBM_ERR_INVALID_ARG, "dense grids must be all fluid; use LBM_BLOCK_SPARSE for obstacles");
      }
  }
  g->lex = d->kind == LBM_DENSE && d->schedule == LBM_PLAIN_SINGLE_KERNEL;
  if (d->lattice == 27) {
    g->q = 27;
    g->ops = LBM_LAUNCHERS_OF(lbm::k27);
  }
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
  auto reg = [&](int f) {
    return g->faces[f].kind == LBM_BC_REG_VELOCITY || g->faces[f].kind == LBM_BC_REG_PRESSURE;
  };
  for (int f1 = 0; f1 < 6; ++f1)
    for (int f2 = f1 + 1; f2 < 6; ++f2) {
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
  g->lv.clear();
  if (g->lex) {
    LevelRT r;
    r.nx = d.nx; r.ny = d.ny; r.nz = d.nz;
    r.S = (int64_t)d.nx * d.ny * d.nz;
    r.n_fluid = r.S;
    r.tau = d.tau;
    g->lv.push_back(r);
  } else if (d.kind != LBM_MULTIRES) {
    std::string e = build_block_level(g->single, d.nx, d.ny, d.nz, d.periodic, g->fluid, g->faces,
                                      d.kind == LBM_DENSE, nullptr, d.schedule != LBM_DISAGG_BITMASK, g->q);
    if (!e.empty()) return fail(LBM_ERR_INVALID_ARG, "%s", e.c_str());
    LevelRT r;
    r.L = &g->single;
    r.nx = d.nx; r.ny = d.ny; r.nz = d.nz;
    r.tau = d.tau;
    g->lv.push_back(r);
  } else {
    std::string e = build_multires(g->mr, d.nx, d.ny, d.nz, d.num_levels, d.periodic, g->level_map,
                                   g->fluid, g->faces, d.tau);
    if (!e.empty()) return fail(LBM_ERR_INVALID_ARG, "%s", e.c_str());
    for (int l = 0; l < d.num_levels; ++l) {
      LevelRT r;
      r.L = &g->mr[l].L;
      r.M = &g->mr[l];
      r.nx = d.nx >> l; r.ny = d.ny >> l; r.nz = d.nz >> l;
      r.tau = g->mr[l].tau;
      r.nbuf = 3;
      r.cur = 0; r.prev = 1; r.nxt = 2;
      g->lv.push_back(r);
    }
  }
  // workspace layout
  size_t off = 0;
  g->partial_rows = 0;
  for (LevelRT &r : g->lv) {
    if (r.L) {
      r.S = r.L->nblocks * 64;
      r.n_fluid = r.L->n_fluid;
      r.packed.resize(r.L->nblocks);
      for (int64_t b = 0; b < r.L->nblocks; ++b)
        r.packed[b] = r.L->coords[3 * b] | (r.L->coords[3 * b + 1] << 10) | (r.L->coords[3 * b + 2] << 20);
    }
    for (int k = 0; k < r.nbuf; ++k) {
      r.off_pop[k] = off;
      off = align256(off + (size_t)r.S * g->q * es);
    }
    if (r.nbuf == 2) r.off_pop[2] = r.off_pop[0];  // the third role is unused
    if (r.L) {
      r.off_nbr = off;
      off = align256(off + r.L->nbr.size() * 4);
      r.off_bbm = off;
      off = align256(off + r.L->bbm.size() * 8);
      r.off_coords = off;
      off = align256(off + r.packed.size() * 4);
      r.off_canon = off;
      off = align256(off + r.L->canon.size() * 4);
      r.off_fmask = off;
      off = align256(off + r.L->fmask.size() * 8);
      if (!r.L->grouped) {
        r.off_bbits = off;
        off = align256(off + r.L->bbits.size() * 4);
        r.off_vid = off;
        off = align256(off + r.L->vid.size() * 4);
        r.off_vrec = off;
        off = align256(off + r.L->vrec.size() * 4);
      }
    }
    if (r.M) {
      r.off_jtab = off;
      off = align256(off + r.M->jtab.size() * 4);
      r.off_jlist = off;
      off = align256(off + r.M->jlist.size() * 4 + 4);
    }
    r.partial_row0 = g->partial_rows;
    g->partial_rows += (r.S + 63) / 64;
  }
  g->off_partial = off;
  off = align256(off + (size_t)g->partial_rows * 5 * sizeof(double));
  g->off_mid = off;  // chunk sums of the second reduction pass
  off = align256(off + (size_t)reduce_mid_rows(g->partial_rows) * 5 * sizeof(double));
  g->off_check = off;  // five doubles for lbm_check
  off = align256(off + 5 * sizeof(double));
  g->total = off;
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
  hipError_t e = hipSuccess;
  auto up = [&](size_t off, const void *src, size_t n) {
    if (e == hipSuccess && n) e = hipMemcpyAsync(g->ws + off, src, n, hipMemcpyHostToDevice, s);
  };
  for (const LevelRT &r : g->lv) {
    if (!r.L) continue;
    up(r.off_nbr, r.L->nbr.data(), r.L->nbr.size() * 4);
    up(r.off_bbm, r.L->bbm.data(), r.L->bbm.size() * 8);
    up(r.off_coords, r.packed.data(), r.packed.size() * 4);
    up(r.off_canon, r.L->canon.data(), r.L->canon.size() * 4);
    up(r.off_fmask, r.L->fmask.data(), r.L->fmask.size() * 8);
    if (!r.L->grouped) {
      up(r.off_bbits, r.L->bbits.data(), r.L->bbits.size() * 4);
      up(r.off_vid, r.L->vid.data(), r.L->vid.size() * 4);
      up(r.off_vrec, r.L->vrec.data(), r.L->vrec.size() * 4);
    }
    if (r.M) {
      up(r.off_jtab, r.M->jtab.data(), r.M->jtab.size() * 4);
      up(r.off_jlist, r.M->jlist.data(), r.M->jlist.size() * 4);
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "uploading index tables");
  g->state = kBound;
  return LBM_OK;
}

lbm_status lbm_num_voxels(const lbm_grid *g, int32_t level, int64_t *n) {
  if (!g || !n) return fail(LBM_ERR_INVALID_ARG, "null argument");
  if (g->state < kCommitted) return fail(LBM_ERR_STATE, "commit first");
  if (lbm_status s = check_level(g, level)) return s;
  *n = g->lv[level].n_fluid;
  return LBM_OK;
}

lbm_status lbm_init_equilibrium(lbm_grid *g, int32_t level, const double *rho, const double *u, void *stream) {
  if (!g || !rho || !u) return fail(LBM_ERR_INVALID_ARG, "null argument");
  if (g->state < kBound) return fail(LBM_ERR_STATE, "bind first");
  if (lbm_status s = check_level(g, level)) return s;
  LevelRT &r = g->lv[level];
  SlotArgs A = slot_args(g, r);
  hipError_t e = g->ops.init_eq(A, rho, u, (hipStream_t)stream);
  if (e == hipSuccess && r.nbuf == 3) {
    // the buffer one step back starts equal to the current state
    A.pop_b = pop_ptr(g, r, r.prev);
    e = g->ops.init_eq(A, rho, u, (hipStream_t)stream);
  }
  if (e != hipSuccess) return hip_fail(e, "init_equilibrium");
  g->state = kReady;
  return LBM_OK;
}

// LDS bytes per workgroup that leave room for at most w workgroups on one
// CU of the current device (1 KiB steps), w = 1..8; 0 requests none
static lbm_status size_residency(lbm_grid *g) {
  int dev = 0, per_cu = 0, per_wg = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&per_wg, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return hip_fail(e, "LDS size query");
  g->lds_of[0] = 0;
  for (int w = 1; w <= 8; ++w) {
    const int64_t b = ((int64_t)per_cu / w) / 1024 * 1024;
    g->lds_of[w] = (uint32_t)(b < per_wg ? b : (int64_t)per_wg / 1024 * 1024);
  }
  g->lds_sized = true;
  return LBM_OK;
}

// Workgroups per CU of each block kernel under LBM_RESIDENCY_AUTO (0: no
// cap), from sweeps of every kernel kind, storage and lattice on MI355X.
// Launches of fewer than 16384 blocks are not capped: with under 16
// workgroups per CU they need every wave slot for loads in flight.
static int32_t auto_residency(const Launch &x, int32_t storage, int32_t q) {
  if (x.count < 16384) return 0;
  const bool f32 = storage == LBM_F32, q19 = q == 19;
  switch (x.kind) {
    case kKernelFull: return f32 ? 5 : (q19 ? 6 : 5);
    case kKernelMasked: return f32 ? 5 : (q19 ? 6 : 0);
    case kKernelInteriorBits: return q19 ? (f32 ? 5 : 7) : 0;
    case kKernelBoundary: return q19 ? (f32 ? 6 : 7) : 0;
    default: return 0;
  }
}

static uint32_t residency_lds(const lbm_grid *g, const Launch &x) {
  // the multires jump and merged-level kernels run uncapped: they serve
  // levels too small to fill the chip (the merged forms by construction),
  // where every cap measured slower
  if (x.kind == kKernelJump || x.kind == kKernelLevelMerged || x.kind == kKernelLevelPair) return 0;
  const int32_t w = g->residency >= 0 ? g->residency : auto_residency(x, g->desc.storage, g->q);
  return g->lds_of[w < 0 ? 0 : (w > 8 ? 8 : w)];
}

lbm_status lbm_step(lbm_grid *g, int32_t n, void *stream) {
  if (!g) return fail(LBM_ERR_INVALID_ARG, "null grid");
  if (g->state < kReady) return fail(LBM_ERR_STATE, "initialise the populations first");
  if (n < 0) return fail(LBM_ERR_INVALID_ARG, "negative step count");
  const float judge = g->mlp ? g->mlp->judge : 0.0f;  // may change between steps
  if (!g->lds_sized) {
    if (lbm_status st = size_residency(g)) return st;
  }
  for (int32_t k = 0; k < n; ++k) {
    const lbm_grid::StepPlan &p = step_plan(g);
    for (Launch x : p.launches) {
      x.args.mlp_judge = judge;
      x.lds = residency_lds(g, x);
      x.wide = g->wide;
      hipError_t e = g->ops.one(x, g->desc.storage, coll_code(g), (hipStream_t)stream);
      if (e != hipSuccess) return hip_fail(e, "step launch");
    }
    for (size_t l = 0; l < g->lv.size(); ++l) {
      g->lv[l].cur = p.roles_out[3 * l];
      g->lv[l].prev = p.roles_out[3 * l + 1];
      g->lv[l].nxt = p.roles_out[3 * l + 2];
    }
  }
  return LBM_OK;
}

lbm_status lbm_step_launches(const lbm_grid *g, int64_t *blocks_out, int32_t max, int32_t *n) {
  if (!g || !n) return fail(LBM_ERR_INVALID_ARG, "null argument");
  if (g->state < kCommitted) return fail(LBM_ERR_STATE, "commit first");
  std::vector<LevelRT> tmp = g->lv;
  std::vector<Launch> launches;
  step_launches(g, tmp, launches);
  *n = (int32_t)launches.size();
  for (int k = 0; k < (int)launches.size() && k < max && blocks_out; ++k) blocks_out[k] = launches[k].count;
  return LBM_OK;
}

lbm_status lbm_launch_group(lbm_grid *g, int32_t k, void *stream) {
  if (!g) return fail(LBM_ERR_INVALID_ARG, "null grid");
  if (g->state < kReady) return fail(LBM_ERR_STATE, "initialise the populations first");
  std::vector<LevelRT> tmp = g->lv;
  std::vector<Launch> launches;
  step_launches(g, tmp, launches);
  if (k < 0 || k >= (int32_t)launches.size()) return fail(LBM_ERR_INVALID_ARG, "launch index out of range");
  if (!g->lds_sized) {
    if (lbm_status st = size_residency(g)) return st;
  }
  launches[k].lds = residency_lds(g, launches[k]);
  launches[k].wide = g->wide;
  hipError_t e = g->ops.one(launches[k], g->desc.storage, coll_code(g), (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "launch_group");
  return LBM_OK;
}

lbm_status lbm_read_macroscopic(lbm_grid *g, int32_t level, void *rho, void *u, int32_t f64, void *stream) {
  if (!g || !rho || !u) return fail(LBM_ERR_INVALID_ARG, "null argument");
  if (g->state < kReady) return fail(LBM_ERR_STATE, "initialise the populations first");
  if (lbm_status s = check_level(g, level)) return s;
  hipError_t e = g->ops.read_macro(slot_args(g, g->lv[level]), rho, u, f64 ? 1 : 0, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "read_macroscopic");
  return LBM_OK;
}

lbm_status lbm_read_populations(lbm_grid *g, int32_t level, double *f, void *stream) {
  if (!g || !f) return fail(LBM_ERR_INVALID_ARG, "null argument");
  if (g->state < kReady) return fail(LBM_ERR_STATE, "initialise the populations first");
  if (lbm_status s = check_level(g, level)) return s;
  hipError_t e = g->ops.read_pop(slot_args(g, g->lv[level]), f, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "read_populations");
  return LBM_OK;
}

lbm_status lbm_write_populations(lbm_grid *g, int32_t level, const double *f, void *stream) {
  if (!g || !f) return fail(LBM_ERR_INVALID_ARG, "null argument");
  if (g->state < kBound) return fail(LBM_ERR_STATE, "bind first");
  if (lbm_status s = check_level(g, level)) return s;
  // slots of non-fluid voxels are never read by any kernel, so only fluid
  // slots are written
  LevelRT &r = g->lv[level];
  SlotArgs A = slot_args(g, r);
  hipError_t e = g->ops.write_pop(A, f, (hipStream_t)stream);
  if (e == hipSuccess && r.nbuf == 3) {
    A.pop_a = pop_ptr(g, r, r.prev);
    e = g->ops.write_pop(A, f, (hipStream_t)stream);
  }
  if (e != hipSuccess) return hip_fail(e, "write_populations");
  g->state = kReady;
  return LBM_OK;
}

lbm_status lbm_reduce(lbm_grid *g, double *out5, void *stream) {
  if (!g || !out5) return fail(LBM_ERR_INVALID_ARG, "null argument");
  if (g->state < kReady) return fail(LBM_ERR_STATE, "initialise the populations first");
  double *partial = (double *)(g->ws + g->off_partial);
  hipError_t e = hipSuccess;
  for (size_t l = 0; l < g->lv.size() && e == hipSuccess; ++l) {
    const LevelRT &r = g->lv[l];
    e = g->ops.reduce_partial(slot_args(g, r), (double)(1ll << (3 * l)), partial + r.partial_row0 * 5,
                              (hipStream_t)stream);
  }
  if (e == hipSuccess)
    e = g->ops.reduce_final(partial, g->partial_rows, (double *)(g->ws + g->off_mid), out5, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "reduce");
  return LBM_OK;
}

lbm_status lbm_reduce_noalloc(lbm_grid *g, double *out5, void *stream) {
  if (!g || !out5) return fail(LBM_ERR_INVALID_ARG, "null argument");
  if (g->state < kCommitted) return fail(LBM_ERR_STATE, "commit, bind and initialise the grid first");
  if ((int)g->lv.size() > kReduceMaxLevels) return fail(LBM_ERR_UNSUPPORTED, "more than %d levels", kReduceMaxLevels);
  const int64_t nmid = reduce_mid_rows(g->partial_rows);
  if (nmid > kNoAllocMidRows)
    return fail(LBM_ERR_INVALID_ARG, "grid too large for lbm_reduce_noalloc: %lld slots, limit %lld",
                (long long)g->partial_rows * 64, (long long)(kNoAllocMidRows * kReduceChunk * 64));
  if (g->state < kReady) return fail(LBM_ERR_STATE, "initialise the populations first");
  ReduceLevels R{};
  R.nlevels = (int32_t)g->lv.size();
  for (int l = 0; l < R.nlevels; ++l) {
    const LevelRT &r = g->lv[l];
    R.a[l] = slot_args(g, r);
    R.weight[l] = (double)(1ll << (3 * l));
    R.row0[l] = r.partial_row0;
  }
  R.row0[R.nlevels] = g->partial_rows;
  hipError_t e = g->ops.reduce_noalloc(R, out5, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "reduce_noalloc");
  return LBM_OK;
}

lbm_status lbm_check(lbm_grid *g, void *stream) {
  if (!g) return fail(LBM_ERR_INVALID_ARG, "null grid");
  if (g->state < kReady) return fail(LBM_ERR_STATE, "initialise the populations first");
  double *d = (double *)(g->ws + g->off_check);
  if (lbm_status st = lbm_reduce(g, d, stream)) return st;
  double h[5];
  hipError_t e = hipMemcpyAsync(h, d, sizeof h, hipMemcpyDeviceToHost, (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "check");
  for (int k = 0; k < 5; ++k)
    if (!std::isfinite(h[k]))
      return fail(LBM_ERR_NUMERIC, "non-finite populations (mass %g, momentum %g %g %g, energy %g)", h[0], h[1],
                  h[2], h[3], h[4]);
  return LBM_OK;
}

lbm_status lbm_get_index_map(const lbm_grid *g, int32_t level, lbm_map which, void *out, size_t *count) {
  if (!g || !count) return fail(LBM_ERR_INVALID_ARG, "null argument");
  if (g->state < kCommitted) return fail(LBM_ERR_STATE, "commit first");
  if (lbm_status s = check_level(g, level)) return s;
  if (g->lex) return fail(LBM_ERR_UNSUPPORTED, "the lexicographic dense arm has no block maps");
  const BlockLevel &L = *g->lv[level].L;
  size_t n = 0;
  switch (which) {
    case LBM_MAP_GROUPS: {
      n = 5;
      if (out) {
        int64_t *o = (int64_t *)out;
        for (int k = 0; k < 4; ++k) o[k] = L.group_count[k];
        o[4] = L.nblocks;
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
    case LBM_MAP_BOUNDARY_BITS: n = L.bbits.size(); if (out) memcpy(out, L.bbits.data(), n * 4); break;
    case LBM_MAP_RECORD_IDS: n = L.vid.size(); if (out) memcpy(out, L.vid.data(), n * 4); break;
    default: return fail(LBM_ERR_INVALID_ARG, "unknown map");
  }
  *count = n;
  return LBM_OK;
}

// ------------------------------------------------------ learned closure --

lbm_status lbm_mlp_create(lbm_mlp **out, size_t *bytes) {
  if (!out || !bytes) return fail(LBM_ERR_INVALID_ARG, "null argument");
  lbm_mlp *m = new (std::nothrow) lbm_mlp;
  if (!m) return fail(LBM_ERR_OUT_OF_MEMORY, "host allocation failed");
  const int64_t bmax = LBM_MLP_BATCH_MAX;
  size_t off = 0;
  auto take = [&](size_t &o, size_t n) {
    o = off;
    off = align256(off + n);
  };
  take(m->off_params, kMlpParams * 4);
  take(m->off_m, kMlpParams * 4);
  take(m->off_v, kMlpParams * 4);
  take(m->off_grads, kMlpParams * 4);
  take(m->off_w, kWPackedElems * 2 + kGeluTabBytes);  // packed weights, then the GELU table
  take(m->off_bias, kBiasFloats * 4);
  take(m->off_stdz, kStdFloats * 4);
  take(m->off_s2, 4);
  take(m->off_fb, 256);
  take(m->off_save, (size_t)bmax * kSaveFloats * 4);
  take(m->off_dyt, (size_t)bmax * Q * 4);
  take(m->off_dz1, (size_t)bmax * 64 * 4);
  take(m->off_dz2, (size_t)bmax * 64 * 4);
  take(m->off_partial, 8192 * 8);
  take(m->off_gpartial, (size_t)((bmax + 127) / 128) * kMlpParams * 4);
  take(m->off_loss, 64);
  m->total = off;
  m->B.batch_max = bmax;
  *out = m;
  *bytes = m->total;
  return LBM_OK;
}

lbm_status lbm_mlp_bind(lbm_mlp *m, void *dev, size_t bytes, void *stream) {
  if (!m || !dev) return fail(LBM_ERR_INVALID_ARG, "null argument");
  if (m->ws) return fail(LBM_ERR_STATE, "closure already bound");
  if (bytes < m->total) return fail(LBM_ERR_INVALID_ARG, "buffer too small (%zu < %zu)", bytes, m->total);
  if (((uintptr_t)dev) & 255) return fail(LBM_ERR_INVALID_ARG, "buffer must be 256-byte aligned");
  m->ws = (char *)dev;
  MlpBuffers &B = m->B;
  B.params = (float *)(m->ws + m->off_params);
  B.adam_m = (float *)(m->ws + m->off_m);
  B.adam_v = (float *)(m->ws + m->off_v);
  B.grads = (float *)(m->ws + m->off_grads);
  B.wpacked = m->ws + m->off_w;
  B.bias = (float *)(m->ws + m->off_bias);
  B.stdz = (float *)(m->ws + m->off_stdz);
  B.s2 = (float *)(m->ws + m->off_s2);
  B.fallbacks = (unsigned long long *)(m->ws + m->off_fb);
  B.save = (float *)(m->ws + m->off_save);
  B.dyt = (float *)(m->ws + m->off_dyt);
  B.dz1 = (float *)(m->ws + m->off_dz1);
  B.dz2 = (float *)(m->ws + m->off_dz2);
  B.partial = (double *)(m->ws + m->off_partial);
  B.gpartial = (float *)(m->ws + m->off_gpartial);
  hipStream_t s = (hipStream_t)stream;
  std::vector<float> zeros(kMlpParams, 0.0f), stdz(kStdFloats, 0.0f);
  for (int i = 0; i < 32; ++i) {
    stdz[32 + i] = 1.0f;
    stdz[64 + i] = 1.0f;
  }
  const uint32_t zero_count[64] = {0};
  hipError_t e = hipMemcpyAsync(B.params, zeros.data(), kMlpParams * 4, hipMemcpyHostToDevice, s);
  if (!e) e = hipMemcpyAsync(B.adam_m, zeros.data(), kMlpParams * 4, hipMemcpyHostToDevice, s);
  if (!e) e = hipMemcpyAsync(B.adam_v, zeros.data(), kMlpParams * 4, hipMemcpyHostToDevice, s);
  if (!e) e = hipMemcpyAsync(B.stdz, stdz.data(), kStdFloats * 4, hipMemcpyHostToDevice, s);
  if (!e) e = mlp_derive(B, s);
  if (!e) e = hipMemcpyAsync(B.fallbacks, zero_count, sizeof zero_count, hipMemcpyHostToDevice, s);
  const std::vector<float> gtab = gelu_table();
  if (!e) e = hipMemcpyAsync(m->ws + m->off_w + kWPackedElems * 2, gtab.data(), kGeluTabBytes,
                             hipMemcpyHostToDevice, s);
  if (!e) e = mlp_pack(B, s);
  if (!e) e = hipStreamSynchronize(s);
  if (e) return hip_fail(e, "mlp_bind");
  return LBM_OK;
}

lbm_status lbm_mlp_set_params(lbm_mlp *m, const float *host, void *stream) {
  if (!m || !host) return fail(LBM_ERR_INVALID_ARG, "null argument");
  if (!m->ws) return fail(LBM_ERR_STATE, "bind the closure first");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(m->B.params, host, kMlpParams * 4, hipMemcpyHostToDevice, s);
  if (!e) e = mlp_pack(m->B, s);
  if (!e) e = hipStreamSynchronize(s);
  if (e) return hip_fail(e, "mlp_set_params");
  return LBM_OK;
}

lbm_status lbm_mlp_get_params(lbm_mlp *m, float *host, void *stream) {
  if (!m || !host) return fail(LBM_ERR_INVALID_ARG, "null argument");
  if (!m->ws) return fail(LBM_ERR_STATE, "bind the closure first");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(host, m->B.params, kMlpParams * 4, hipMemcpyDeviceToHost, s);
  if (!e) e = hipStreamSynchronize(s);
  if (e) return hip_fail(e, "mlp_get_params");
  return LBM_OK;
}

lbm_status lbm_mlp_set_standardization(lbm_mlp *m, const float *host, void *stream) {
  if (!m || !host) return fail(LBM_ERR_INVALID_ARG, "null argument");
  if (!m->ws) return fail(LBM_ERR_STATE, "bind the closure first");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(m->B.stdz, host, kStdFloats * 4, hipMemcpyHostToDevice, s);
  if (!e) e = mlp_derive(m->B, s);
  if (!e) e = hipStreamSynchronize(s);
  if (e) return hip_fail(e, "mlp_set_standardization");
  return LBM_OK;
}

lbm_status lbm_mlp_get_standardization(lbm_mlp *m, float *host, void *stream) {
  if (!m || !host) return fail(LBM_ERR_INVALID_ARG, "null argument");
  if (!m->ws) return fail(LBM_ERR_STATE, "bind the closure first");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(host, m->B.stdz, kStdFloats * 4, hipMemcpyDeviceToHost, s);
  if (!e) e = hipStreamSynchronize(s);
  if (e) return hip_fail(e, "mlp_get_standardization");
  return LBM_OK;
}

lbm_status lbm_mlp_fit_standardization(lbm_mlp *m, const float *f, int64_t n, void *stream) {
  if (!m || !f || n <= 0) return fail(LBM_ERR_INVALID_ARG, "bad argument");
  if (!m->ws) return fail(LBM_ERR_STATE, "bind the closure first");
  hipError_t e = mlp_fit_standardization(m->B, f, n, (hipStream_t)stream);
  if (e) return hip_fail(e, "mlp_fit_standardization");
  return LBM_OK;
}

lbm_status lbm_mlp_forward(lbm_mlp *m, const float *f, int64_t n, float *y, void *stream) {
  if (!m || !f || !y || n < 0) return fail(LBM_ERR_INVALID_ARG, "bad argument");
  if (!m->ws) return fail(LBM_ERR_STATE, "bind the closure first");
  hipError_t e = mlp_forward(m->B, f, n, y, (hipStream_t)stream);
  if (e) return hip_fail(e, "mlp_forward");
  return LBM_OK;
}

lbm_status lbm_mlp_gradients(lbm_mlp *m, const float *f, const int64_t *idx, int64_t n, float *grads, double *loss,
                             void *stream) {
  if (!m || !f) return fail(LBM_ERR_INVALID_ARG, "null argument");
  if (n <= 0 || n > LBM_MLP_BATCH_MAX) return fail(LBM_ERR_INVALID_ARG, "batch size must be 1..%d", LBM_MLP_BATCH_MAX);
  if (!m->ws) return fail(LBM_ERR_STATE, "bind the closure first");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = mlp_gradients(m->B, f, idx, n, loss, s);
  if (!e && grads) e = hipMemcpyAsync(grads, m->B.grads, kMlpParams * 4, hipMemcpyDeviceToDevice, s);
  if (e) return hip_fail(e, "mlp_gradients");
  return LBM_OK;
}

lbm_status lbm_mlp_train_step(lbm_mlp *m, const float *f, const int64_t *idx, int64_t n, float lr, int32_t t,
                              double *loss, void *stream) {
  if (!m || !f) return fail(LBM_ERR_INVALID_ARG, "null argument");
  if (n <= 0 || n > LBM_MLP_BATCH_MAX) return fail(LBM_ERR_INVALID_ARG, "batch size must be 1..%d", LBM_MLP_BATCH_MAX);
  if (t < 1 || !(lr > 0)) return fail(LBM_ERR_INVALID_ARG, "need t >= 1 and lr > 0");
  if (!m->ws) return fail(LBM_ERR_STATE, "bind the closure first");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = mlp_gradients(m->B, f, idx, n, loss, s);
  if (!e) e = mlp_adam(m->B, m->B.grads, lr, t, s);
  if (e) return hip_fail(e, "mlp_train_step");
  return LBM_OK;
}

lbm_status lbm_mlp_adam(lbm_mlp *m, const float *grads, float lr, int32_t t, void *stream) {
  if (!m || !grads) return fail(LBM_ERR_INVALID_ARG, "null argument");
  if (t < 1 || !(lr > 0)) return fail(LBM_ERR_INVALID_ARG, "need t >= 1 and lr > 0");
  if (!m->ws) return fail(LBM_ERR_STATE, "bind the closure first");
  hipError_t e = mlp_adam(m->B, grads, lr, t, (hipStream_t)stream);
  if (e) return hip_fail(e, "mlp_adam");
  return LBM_OK;
}

lbm_status lbm_mlp_init_params(lbm_mlp *m, uint64_t seed, void *stream) {
  if (!m) return fail(LBM_ERR_INVALID_ARG, "null argument");
  if (!m->ws) return fail(LBM_ERR_STATE, "bind the closure first");
  hipError_t e = mlp_init(m->B, seed, (hipStream_t)stream);
  if (e) return hip_fail(e, "mlp_init_params");
  return LBM_OK;
}

lbm_status lbm_mlp_set_judge(lbm_mlp *m, double rel_tol) {
  if (!m || !(rel_tol >= 0.0) || !std::isfinite(rel_tol)) return fail(LBM_ERR_INVALID_ARG, "bad judge tolerance");
  m->judge = (float)rel_tol;
  return LBM_OK;
}

lbm_status lbm_mlp_fallbacks(lbm_mlp *m, uint64_t *count, int32_t reset, void *stream) {
  if (!m || !count) return fail(LBM_ERR_INVALID_ARG, "null argument");
  if (!m->ws) return fail(LBM_ERR_STATE, "bind the closure first");
  hipStream_t s = (hipStream_t)stream;
  uint64_t c = 0;
  hipError_t e = hipMemcpyAsync(&c, m->B.fallbacks, sizeof c, hipMemcpyDeviceToHost, s);
  if (!e) e = hipStreamSynchronize(s);
  if (!e && reset) {
    const uint64_t z = 0;
    e = hipMemcpyAsync(m->B.fallbacks, &z, sizeof z, hipMemcpyHostToDevice, s);
    if (!e) e = hipStreamSynchronize(s);
  }
  if (e) return hip_fail(e, "mlp_fallbacks");
  *count = c;
  return LBM_OK;
}

lbm_status lbm_mlp_destroy(lbm_mlp *m) {
  delete m;
  return LBM_OK;
}

lbm_status lbm_set_collision(lbm_grid *g, lbm_collision c, const lbm_mlp *m) {
  if (!g) return fail(LBM_ERR_INVALID_ARG, "null grid");
  if (c < LBM_BGK || c > LBM_MLP) return fail(LBM_ERR_INVALID_ARG, "unknown collision");
  if (c == LBM_MLP) {
    if (!m || !m->ws) return fail(LBM_ERR_INVALID_ARG, "LBM_MLP needs a bound closure");
    if (g->lex || g->desc.kind == LBM_MULTIRES || g->desc.schedule != LBM_DISAGG || g->q != 19)
      return fail(LBM_ERR_UNSUPPORTED,
                  "the closure runs on D3Q19 dense or block-sparse grids in the disaggregated schedule");
    g->mlp = m;
  }
  g->collision = c;
  g->plans.clear();
  return LBM_OK;
}

lbm_status lbm_set_merge_limit(lbm_grid *g, int64_t max_blocks) {
  if (!g) return fail(LBM_ERR_INVALID_ARG, "null grid");
  if (max_blocks < 0) return fail(LBM_ERR_INVALID_ARG, "the merge limit must be >= 0");
  g->merge_max = max_blocks;
  g->plans.clear();
  return LBM_OK;
}

lbm_status lbm_set_residency(lbm_grid *g, int32_t wg_per_cu) {
  if (!g) return fail(LBM_ERR_INVALID_ARG, "null grid");
  if (wg_per_cu < LBM_RESIDENCY_AUTO || wg_per_cu > 8)
    return fail(LBM_ERR_INVALID_ARG, "workgroups per CU must be LBM_RESIDENCY_AUTO or in 0..8");
  g->residency = wg_per_cu;
  return LBM_OK;
}

lbm_status lbm_set_wide_addressing(lbm_grid *g, int32_t wide) {
  if (!g) return fail(LBM_ERR_INVALID_ARG, "null grid");
  if (wide != 0 && wide != 1) return fail(LBM_ERR_INVALID_ARG, "wide must be 0 or 1");
  g->wide = wide;
  return LBM_OK;
}

lbm_status lbm_sample_populations(lbm_grid *g, int32_t level, uint64_t seed, int64_t n, float *f, void *stream) {
  if (!g || !f || n < 0) return fail(LBM_ERR_INVALID_ARG, "bad argument");
  if (g->state < kReady) return fail(LBM_ERR_STATE, "initialise the populations first");
  if (lbm_status st = check_level(g, level)) return st;
  const LevelRT &r = g->lv[level];
  if (!r.L) return fail(LBM_ERR_UNSUPPORTED, "sampling needs a block layout");
  if (!r.L->grouped) return fail(LBM_ERR_UNSUPPORTED, "sampling needs the memory-grouped layout");
  if (g->q != 19) return fail(LBM_ERR_UNSUPPORTED, "sampling feeds the D3Q19 closure");
  const auto &gc = r.L->group_count;
  const int32_t b0 = (int32_t)(gc[0] + gc[1]), nb = (int32_t)(gc[2] + gc[3]);
  if (nb <= 0) return fail(LBM_ERR_INVALID_ARG, "the level has no non-boundary blocks");
  StepArgs a = level_args(g, r);
  a.src = pop_ptr(g, r, r.cur);
  hipError_t e = launch_sample_pre(a, g->desc.storage, b0, nb, seed, n, f, (hipStream_t)stream);
  if (e) return hip_fail(e, "sample_populations");
  return LBM_OK;
}

lbm_status lbm_grid_destroy(lbm_grid *g) {
  delete g;
  return LBM_OK;
}

}  // extern "C"
