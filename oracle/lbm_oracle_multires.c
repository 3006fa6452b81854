/*
 * FP64 CPU oracle for the multi-resolution D3Q19 update.
 *
 * TEST INFRASTRUCTURE ONLY (see lbm_oracle.c).  Shares nothing with the GPU
 * library.  Built into the same liboracle.so as lbm_oracle.c, whose
 * equilibrium, collision and Hermite helpers it reuses.
 *
 * What it follows: section "Disaggregation on a Multi-resolution Domain" and
 * the multi-resolution evaluation ("Improving Multi-resolution LBM Kernel
 * Fusion"): one uniform grid per level; per time step an *explosion*
 * (collision results of a coarse level feed the finer level) and a
 * *coalescence* (streamed data of the finer level merges into the coarser
 * one).  The paper gives neither operator's formulas; this file implements
 * the reading written down in the design notes ("M"), chosen so that mass
 * is conserved exactly:
 *
 *  - level l voxels are cubes of 2^l finest cells (l = 0 finest); the level
 *    map is block aligned and 2:1 balanced; solids exist at level 0 only;
 *  - level l advances in steps of 2^l finest steps, tau_l - 1/2 =
 *    (tau_coarsest - 1/2) * 2^(L-1-l); no rescaling of non-equilibrium parts;
 *  - inside one step of level l, the finer level takes two substeps.  Coarse
 *    territory seen from the finer level holds "virtual" fine populations:
 *    at the start of the coarse step each equals the coarse post-collision
 *    value of its cell (explosion) and they stream without colliding;
 *  - a coarse voxel receives, per direction, the average of the 8 virtual
 *    values that land on its 2x2x2 footprint at the end of the two substeps
 *    (coalescence).
 *
 * Time bookkeeping: every level keeps its post-collision field at the
 * current time ("cur") and one step earlier ("prev").  The coarse update of
 * level l runs between the two substeps of level l-1, when level l-1 holds
 * cur = f*(t + dt/2) and prev = f*(t).
 *
 * Layout (oracle only): per level a dense box (nx>>l, ny>>l, nz>>l) of 19
 * doubles per cell, x fastest; cells that are not active at that level hold
 * unused values.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_Q 19
#define ORC_MAXL 6

/* shared with lbm_oracle.c (same library) */
void orc_lattice(int32_t *c, double *w, int32_t *opp);
void orc_equilibrium(double rho, const double *u, double *feq);
void orc_moments(const double *f, double *rho, double *u);
void orc_f1(const double *f, const double *feq, double *f1);

enum { MR_BB = 0, MR_MOVING = 1, MR_REG_VEL = 2, MR_REG_PRES = 3 };

typedef struct {
  int32_t nx, ny, nz; /* finest box */
  int32_t levels;
  int32_t periodic[3];
  const uint8_t *level_map; /* finest resolution */
  const uint8_t *fluid;     /* finest resolution, NULL = all fluid */
  int32_t bc_kind[6];
  double bc_val[6][3];
  double tau_coarsest;
  int32_t collision; /* 0 BGK, 1 regularized */
} orc_mr_grid;

typedef struct {
  double *cur[ORC_MAXL];
  double *prev[ORC_MAXL];
  double *nxt[ORC_MAXL];
} orc_mr_state;

static int C[ORC_Q][3];
static double W[ORC_Q];
static int OPP[ORC_Q];
static int lattice_ready = 0;

static void mr_lattice(void) {
  if (lattice_ready) return;
  int32_t c[3 * ORC_Q], opp[ORC_Q];
  orc_lattice(c, W, opp);
  for (int i = 0; i < ORC_Q; ++i) {
    for (int a = 0; a < 3; ++a) C[i][a] = c[3 * i + a];
    OPP[i] = opp[i];
  }
  lattice_ready = 1;
}

static int dim(const orc_mr_grid *g, int l, int a) {
  int n = a == 0 ? g->nx : (a == 1 ? g->ny : g->nz);
  return n >> l;
}

/* Wraps level-l coordinates on periodic axes; returns 0 if the point lies
 * outside the box across a non-periodic face (and sets *face). */
static int wrap(const orc_mr_grid *g, int l, int p[3], int *face) {
  for (int a = 0; a < 3; ++a) {
    int n = dim(g, l, a);
    if (p[a] < 0 || p[a] >= n) {
      if (g->periodic[a]) {
        p[a] = ((p[a] % n) + n) % n;
      } else {
        if (face) *face = 2 * a + (p[a] >= n ? 1 : 0);
        return 0;
      }
    }
  }
  return 1;
}

/* level that owns the finest-resolution cube of level-l cell p (in-box):
 * l = active at level l, > l = part of a coarser cell, < l = refined */
static int territory(const orc_mr_grid *g, int l, const int p[3]) {
  size_t x = (size_t)p[0] << l, y = (size_t)p[1] << l, z = (size_t)p[2] << l;
  return g->level_map[x + (size_t)g->nx * (y + (size_t)g->ny * z)];
}

static int fluid_at(const orc_mr_grid *g, int l, const int p[3]) {
  if (!g->fluid || l > 0) return 1;
  return g->fluid[(size_t)p[0] + (size_t)g->nx * ((size_t)p[1] + (size_t)g->ny * p[2])];
}

static size_t cell_index(const orc_mr_grid *g, int l, const int p[3]) {
  return (size_t)p[0] + (size_t)dim(g, l, 0) * ((size_t)p[1] + (size_t)dim(g, l, 1) * p[2]);
}

static double tau_at(const orc_mr_grid *g, int l) {
  return 0.5 + (g->tau_coarsest - 0.5) * (double)(1 << (g->levels - 1 - l));
}

/* Value of direction i arriving at level-l voxel x by a same-resolution
 * pull, including explosion from the coarser level at substep s (1 or 2 of
 * the level-(l+1) step; 0 on the coarsest level).  Returns 0 and sets
 * *unknown_face when the link needs the regularized face rule. */
static int plain_pull(const orc_mr_grid *g, const orc_mr_state *st, int l, const int x[3], int i,
                      int s, double *val, int *unknown_face) {
  const double *own = st->cur[l] + cell_index(g, l, x) * ORC_Q;
  int q[3] = {x[0] - C[i][0], x[1] - C[i][1], x[2] - C[i][2]};
  /* faces crossed by the link, with the single-level tie-break: moving
   * wall, then stationary wall, then regularized */
  int crossed = 0, moving = -1, wall = -1, reg = -1;
  for (int a = 0; a < 3; ++a) {
    int n = dim(g, l, a);
    if (q[a] < 0 || q[a] >= n) {
      if (g->periodic[a]) continue;
      crossed = 1;
      int f = 2 * a + (q[a] >= n ? 1 : 0);
      int k = g->bc_kind[f];
      if (k == MR_MOVING) { if (moving < 0) moving = f; }
      else if (k == MR_BB) { if (wall < 0) wall = f; }
      else reg = f;
    }
  }
  if (crossed) {
    if (moving >= 0) {
      const double *uw = g->bc_val[moving];
      double cu = C[i][0] * uw[0] + C[i][1] * uw[1] + C[i][2] * uw[2];
      *val = own[OPP[i]] + 6.0 * W[i] * cu;
    } else if (wall >= 0) {
      *val = own[OPP[i]];
    } else {
      *unknown_face = reg;
      *val = 0.0;
      return 0;
    }
    return 1;
  }
  wrap(g, l, q, NULL);
  int t = territory(g, l, q);
  if (t == l) {
    if (fluid_at(g, l, q)) *val = st->cur[l][cell_index(g, l, q) * ORC_Q + i];
    else *val = own[OPP[i]];
    return 1;
  }
  if (t == l + 1) {
    /* explosion: virtual fine populations in coarse territory */
    int cq[3] = {q[0] >> 1, q[1] >> 1, q[2] >> 1};
    if (s == 1) {
      *val = st->cur[l + 1][cell_index(g, l + 1, cq) * ORC_Q + i];
      return 1;
    }
    /* substep 2: the virtual value at q arrived from r = q - c_i during
     * substep 1 -- a real level-l voxel's post-collision value at the start
     * of the coarse step, or the virtual (exploded) value of r */
    int r[3] = {q[0] - C[i][0], q[1] - C[i][1], q[2] - C[i][2]};
    wrap(g, l, r, NULL);
    if (territory(g, l, r) == l) {
      *val = st->prev[l][cell_index(g, l, r) * ORC_Q + i];
    } else {
      int cr[3] = {r[0] >> 1, r[1] >> 1, r[2] >> 1};
      *val = st->cur[l + 1][cell_index(g, l + 1, cr) * ORC_Q + i];
    }
    return 1;
  }
  /* finer territory is handled by coalescence before this is reached */
  *val = NAN;
  return 1;
}

/* Direction i arriving at level-l voxel x for this level-l step. */
static int arrive(const orc_mr_grid *g, const orc_mr_state *st, int l, const int x[3], int i, int s,
                  double *val, int *unknown_face) {
  if (l > 0 && i > 0) {
    /* coalescence applies if some footprint point sees finer territory one
     * or two fine cells upstream */
    int any = 0;
    double v8[8];
    int kind8[8];
    for (int d = 0; d < 8; ++d) {
      int p[3] = {2 * x[0] + (d & 1), 2 * x[1] + ((d >> 1) & 1), 2 * x[2] + (d >> 2)};
      int a1[3] = {p[0] - C[i][0], p[1] - C[i][1], p[2] - C[i][2]};
      int a2[3] = {p[0] - 2 * C[i][0], p[1] - 2 * C[i][1], p[2] - 2 * C[i][2]};
      kind8[d] = 0;
      if (wrap(g, l - 1, a1, NULL) && territory(g, l - 1, a1) == l - 1) {
        v8[d] = st->cur[l - 1][cell_index(g, l - 1, a1) * ORC_Q + i]; /* f*(t + dt/2) */
        kind8[d] = 1;
        any = 1;
      } else if (wrap(g, l - 1, a2, NULL) && territory(g, l - 1, a2) == l - 1) {
        v8[d] = st->prev[l - 1][cell_index(g, l - 1, a2) * ORC_Q + i]; /* f*(t) */
        kind8[d] = 2;
        any = 1;
      }
    }
    if (any) {
      double coarse = 0.0;
      int have_coarse = 0;
      double sum = 0.0;
      for (int d = 0; d < 8; ++d) {
        if (kind8[d] == 0) {
          if (!have_coarse) {
            int uf = -1;
            if (!plain_pull(g, st, l, x, i, s, &coarse, &uf)) return 0; /* excluded by validation */
            have_coarse = 1;
          }
          sum += coarse;
        } else {
          sum += v8[d];
        }
      }
      *val = sum / 8.0;
      return 1;
    }
  }
  if (i == 0) {
    *val = st->cur[l][cell_index(g, l, x) * ORC_Q];
    return 1;
  }
  return plain_pull(g, st, l, x, i, s, val, unknown_face);
}

static void mr_collide(const orc_mr_grid *g, int l, double *f, const int *unknown, int reg_face,
                       double *out) {
  const double tau = tau_at(g, l);
  double feq[ORC_Q], f1[ORC_Q], rho, u[3];
  if (reg_face >= 0) {
    /* regularized face, as in the single-level oracle */
    int axis = reg_face / 2;
    double n[3] = {0, 0, 0};
    n[axis] = (reg_face % 2) ? 1.0 : -1.0;
    double sT = 0, sO = 0;
    for (int i = 0; i < ORC_Q; ++i) {
      double cn = C[i][0] * n[0] + C[i][1] * n[1] + C[i][2] * n[2];
      if (cn == 0) sT += f[i];
      else if (cn > 0) sO += f[i];
    }
    if (g->bc_kind[reg_face] == MR_REG_VEL) {
      for (int a = 0; a < 3; ++a) u[a] = g->bc_val[reg_face][a];
      rho = (sT + 2 * sO) / (1.0 + u[0] * n[0] + u[1] * n[1] + u[2] * n[2]);
    } else {
      rho = g->bc_val[reg_face][0];
      double un = (sT + 2 * sO) / rho - 1.0;
      for (int a = 0; a < 3; ++a) u[a] = un * n[a];
    }
    orc_equilibrium(rho, u, feq);
    for (int i = 0; i < ORC_Q; ++i)
      if (unknown[i]) f[i] = feq[i] + f[OPP[i]] - feq[OPP[i]];
    orc_f1(f, feq, f1);
    for (int i = 0; i < ORC_Q; ++i) out[i] = feq[i] + (1.0 - 1.0 / tau) * f1[i];
    return;
  }
  orc_moments(f, &rho, u);
  orc_equilibrium(rho, u, feq);
  if (g->collision == 1) {
    orc_f1(f, feq, f1);
    for (int i = 0; i < ORC_Q; ++i) out[i] = feq[i] + (1.0 - 1.0 / tau) * f1[i];
  } else {
    for (int i = 0; i < ORC_Q; ++i) out[i] = f[i] - (f[i] - feq[i]) / tau;
  }
}

static int update_level(const orc_mr_grid *g, orc_mr_state *st, int l, int s) {
  const int n0 = dim(g, l, 0), n1 = dim(g, l, 1), n2 = dim(g, l, 2);
  int err = 0;
#pragma omp parallel for collapse(2) schedule(static) reduction(| : err)
  for (int z = 0; z < n2; ++z)
    for (int y = 0; y < n1; ++y)
      for (int x = 0; x < n0; ++x) {
        int p[3] = {x, y, z};
        if (territory(g, l, p) != l || !fluid_at(g, l, p)) continue;
        double f[ORC_Q];
        int unknown[ORC_Q], reg_face = -1;
        for (int i = 0; i < ORC_Q; ++i) {
          int uf = -1;
          unknown[i] = 0;
          if (!arrive(g, st, l, p, i, s, &f[i], &uf)) {
            unknown[i] = 1;
            if (reg_face >= 0 && reg_face != uf) err |= 1;
            reg_face = uf;
          }
        }
        mr_collide(g, l, f, unknown, reg_face, st->nxt[l] + cell_index(g, l, p) * ORC_Q);
      }
  return err;
}

static void rotate(orc_mr_state *st, int l) {
  double *old_prev = st->prev[l];
  st->prev[l] = st->cur[l];
  st->cur[l] = st->nxt[l];
  st->nxt[l] = old_prev;
}

static int level_step(const orc_mr_grid *g, orc_mr_state *st, int l, int s) {
  int err = 0;
  if (l > 0) err |= level_step(g, st, l - 1, 1);
  err |= update_level(g, st, l, s);
  if (l > 0) err |= level_step(g, st, l - 1, 2);
  rotate(st, l);
  return err;
}

/* n coarse steps.  cur/prev/nxt are caller-owned arrays per level (the
 * function rotates the pointers it is given and reports the final order in
 * `which_cur`: which_cur[l] = 0, 1 or 2 for the array holding the current
 * field among (a, b, c) as passed). */
int orc_mr_run(const orc_mr_grid *g, double **a, double **b, double **c, int32_t nsteps,
               int32_t *which_cur) {
  mr_lattice();
  if (g->levels < 1 || g->levels > ORC_MAXL) return -2;
  orc_mr_state st;
  for (int l = 0; l < g->levels; ++l) {
    st.cur[l] = a[l];
    st.prev[l] = b[l];
    st.nxt[l] = c[l];
  }
  int err = 0;
  for (int k = 0; k < nsteps; ++k) err |= level_step(g, &st, g->levels - 1, 0);
  for (int l = 0; l < g->levels; ++l) which_cur[l] = st.cur[l] == a[l] ? 0 : (st.cur[l] == b[l] ? 1 : 2);
  return err ? -1 : 0;
}

/* Mass sum_l 8^l sum_x sum_i f of the current fields. */
double orc_mr_mass(const orc_mr_grid *g, double **cur) {
  double m = 0.0;
  for (int l = 0; l < g->levels; ++l) {
    const int n0 = dim(g, l, 0), n1 = dim(g, l, 1), n2 = dim(g, l, 2);
    double ml = 0.0;
    for (int z = 0; z < n2; ++z)
      for (int y = 0; y < n1; ++y)
        for (int x = 0; x < n0; ++x) {
          int p[3] = {x, y, z};
          if (territory(g, l, p) != l || !fluid_at(g, l, p)) continue;
          const double *f = cur[l] + cell_index(g, l, p) * ORC_Q;
          for (int i = 0; i < ORC_Q; ++i) ml += f[i];
        }
    m += ml * (double)(1 << (3 * l));
  }
  return m;
}
