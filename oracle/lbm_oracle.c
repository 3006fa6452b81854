/*
 * FP64 CPU oracle for the D3Q19 (and D3Q27) collide-and-stream update.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * statement of what the GPU library computes.  It shares no code, header,
 * table or helper with the library under paper_2503_07898_amd/ and is built
 * separately with gcc.  Only tests/, the smoke check and the CPU-baseline leg
 * of bench.py load it.
 *
 * What it follows:
 *  - Evaluation section, first paragraph: LBM populations f_i on a D3Q19
 *    lattice, a collide step (BGK single relaxation time) and a stream step
 *    along the q directions.  The lattice, equilibrium and BGK forms are the
 *    textbook ones the paper cites (Krueger et al. 2016).
 *  - "Improving LBM register allocation": halfway bounce-back on obstacle
 *    surfaces and regularized inflow/outflow faces (Latt et al. 2008).
 *  - "Improving LBM scalability", benchmarking paragraph: lid-driven cavity,
 *    read as bounce-back walls plus a moving-wall bounce-back lid.
 *  - Regularized collision operator (an addition of this library; the same
 *    Hermite projection the regularized boundary uses).
 *
 * State convention: the stored field is the post-collision population f* of
 * every fluid voxel.  One step gathers f_i(x) = f*_i(x - c_i) (or the
 * boundary rule), then collides.  Starting from f* = f^eq, which is a fixed
 * point of both collision operators, the moments after n steps equal those of
 * the pre-collision field of the collide-then-stream formulation.
 *
 * Layout (oracle only): dense box arrays, voxel v = x + nx*(y + ny*z), 19
 * doubles per voxel (array of structures).  Solid voxels hold unused values.
 *
 * Where the paper is silent (lattice order, equilibrium order, moving-wall
 * form, regularized-boundary formulas, tie-breaks at edges) the readings are
 * the ones listed in the design notes; each is marked "reading" below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Built twice: as the D3Q19 oracle (default) and, with -DORC_D3Q27, as the
 * D3Q27 oracle (the lattice of the paper's block-sparse register study). */
#ifndef ORC_D3Q27
#define ORC_Q 19

/* Reading: direction order 0 rest, 1-6 faces (+x,-x,+y,-y,+z,-z), 7-18 edges,
 * opposite pairs (1,2),(3,4),...,(17,18). */
static const int orc_c[ORC_Q][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static const double orc_w[ORC_Q] = {
    1.0 / 3.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
#else
#define ORC_Q 27

/* Reading: the D3Q19 order followed by the 8 corners in opposite pairs
 * (19,20),...,(25,26); weights 8/27, 2/27, 1/54, 1/216 (textbook D3Q27). */
static const int orc_c[ORC_Q][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
    {1, 1, 1}, {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
    {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1}};

static const double orc_w[ORC_Q] = {
    8.0 / 27.0,
    2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0,
    1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0,
    1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0,
    1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0,
    1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0};
#endif

static const double orc_cs2 = 1.0 / 3.0;

/* opposite direction: found by search, not by a hand-written table */
static int orc_opp(int i) {
  for (int j = 0; j < ORC_Q; ++j)
    if (orc_c[j][0] == -orc_c[i][0] && orc_c[j][1] == -orc_c[i][1] &&
        orc_c[j][2] == -orc_c[i][2])
      return j;
  return -1;
}

/* face ids: 2*axis + (1 if the max side) */
enum { ORC_BB = 0, ORC_MOVING = 1, ORC_REG_VEL = 2, ORC_REG_PRES = 3 };
enum { ORC_BGK = 0, ORC_REGULARIZED = 1 };

typedef struct {
  int32_t nx, ny, nz;
  int32_t periodic[3];
  const uint8_t *fluid; /* nx*ny*nz, 1 = fluid; NULL = all fluid */
  int32_t bc_kind[6];
  double bc_val[6][3];
  double tau;
  int32_t collision;
} orc_grid;

void orc_lattice(int32_t *c, double *w, int32_t *opp) {
  for (int i = 0; i < ORC_Q; ++i) {
    for (int a = 0; a < 3; ++a) c[3 * i + a] = orc_c[i][a];
    w[i] = orc_w[i];
    opp[i] = orc_opp(i);
  }
}

/* second-order equilibrium, f_i^eq = w_i rho (1 + c.u/cs2 + (c.u)^2/(2cs4) - u.u/(2cs2)) */
void orc_equilibrium(double rho, const double *u, double *feq) {
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < ORC_Q; ++i) {
    double cu = orc_c[i][0] * u[0] + orc_c[i][1] * u[1] + orc_c[i][2] * u[2];
    feq[i] = orc_w[i] * rho *
             (1.0 + cu / orc_cs2 + cu * cu / (2.0 * orc_cs2 * orc_cs2) -
              uu / (2.0 * orc_cs2));
  }
}

void orc_moments(const double *f, double *rho, double *u) {
  double r = 0, j[3] = {0, 0, 0};
  for (int i = 0; i < ORC_Q; ++i) {
    r += f[i];
    for (int a = 0; a < 3; ++a) j[a] += orc_c[i][a] * f[i];
  }
  *rho = r;
  for (int a = 0; a < 3; ++a) u[a] = j[a] / r;
}

/* BGK: f* = f - (f - f^eq)/tau */
void orc_collide_bgk(const double *f, double tau, double *out) {
  double rho, u[3], feq[ORC_Q];
  orc_moments(f, &rho, u);
  orc_equilibrium(rho, u, feq);
  for (int i = 0; i < ORC_Q; ++i) out[i] = f[i] - (f[i] - feq[i]) / tau;
}

/* Hermite projection of the non-equilibrium part:
 * Pi_ab = sum_j c_ja c_jb (f_j - feq_j)
 * f1_i  = w_i / (2 cs^4) * sum_ab (c_ia c_ib - cs2 delta_ab) Pi_ab */
void orc_f1(const double *f, const double *feq, double *f1) {
  double pi[3][3] = {{0}};
  for (int j = 0; j < ORC_Q; ++j) {
    double fn = f[j] - feq[j];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) pi[a][b] += orc_c[j][a] * orc_c[j][b] * fn;
  }
  for (int i = 0; i < ORC_Q; ++i) {
    double s = 0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        s += (orc_c[i][a] * orc_c[i][b] - (a == b ? orc_cs2 : 0.0)) * pi[a][b];
    f1[i] = orc_w[i] / (2.0 * orc_cs2 * orc_cs2) * s;
  }
}

/* regularized collision: f* = f^eq + (1 - 1/tau) f1 */
void orc_collide_regularized(const double *f, double tau, double *out) {
  double rho, u[3], feq[ORC_Q], f1[ORC_Q];
  orc_moments(f, &rho, u);
  orc_equilibrium(rho, u, feq);
  orc_f1(f, feq, f1);
  for (int i = 0; i < ORC_Q; ++i) out[i] = feq[i] + (1.0 - 1.0 / tau) * f1[i];
}

static int orc_is_fluid(const orc_grid *g, int x, int y, int z) {
  if (!g->fluid) return 1;
  return g->fluid[(size_t)x + (size_t)g->nx * ((size_t)y + (size_t)g->ny * z)] != 0;
}

/* Result codes of one voxel update. */
#define ORC_OK 0
#define ORC_ERR_GEOMETRY (-1)

/*
 * One voxel of one step.  fin is the post-collision field of the previous
 * step, out receives the 19 new post-collision values of voxel (x,y,z).
 */
static int orc_update_voxel(const orc_grid *g, const double *fin, int x, int y,
                            int z, double *out) {
  const int n[3] = {g->nx, g->ny, g->nz};
  const int p[3] = {x, y, z};
  const size_t v = (size_t)x + (size_t)n[0] * ((size_t)y + (size_t)n[1] * z);
  const double *own = fin + v * ORC_Q;
  double f[ORC_Q];
  int unknown[ORC_Q];
  int reg_face = -1;

  for (int i = 0; i < ORC_Q; ++i) {
    int s[3];
    int crossed[3] = {-1, -1, -1}; /* face id crossed on each axis, or -1 */
    int any_crossed = 0;
    for (int a = 0; a < 3; ++a) {
      s[a] = p[a] - orc_c[i][a];
      if (s[a] < 0 || s[a] >= n[a]) {
        if (g->periodic[a]) {
          s[a] = (s[a] + n[a]) % n[a];
        } else {
          crossed[a] = 2 * a + (s[a] >= n[a] ? 1 : 0);
          any_crossed = 1;
        }
      }
    }
    unknown[i] = 0;
    if (!any_crossed) {
      if (orc_is_fluid(g, s[0], s[1], s[2])) {
        size_t sv = (size_t)s[0] + (size_t)n[0] * ((size_t)s[1] + (size_t)n[1] * s[2]);
        f[i] = fin[sv * ORC_Q + i];
      } else {
        f[i] = own[orc_opp(i)]; /* halfway bounce-back on a solid voxel */
      }
      continue;
    }
    /* Reading (tie-break): a moving wall wins over every other face, then a
     * stationary wall, and only links that cross regularized faces alone are
     * unknown. */
    int moving = -1, wall = -1, reg = -1, nreg = 0;
    for (int a = 0; a < 3; ++a) {
      if (crossed[a] < 0) continue;
      int k = g->bc_kind[crossed[a]];
      if (k == ORC_MOVING && moving < 0) moving = crossed[a];
      else if (k == ORC_BB && wall < 0) wall = crossed[a];
      else if (k == ORC_REG_VEL || k == ORC_REG_PRES) { reg = crossed[a]; ++nreg; }
    }
    if (moving >= 0) {
      /* moving-wall bounce-back, wall density 1:
       * f_i = f*_opp + 2 w_i (c_i . u_w) / cs2 */
      const double *uw = g->bc_val[moving];
      double cu = orc_c[i][0] * uw[0] + orc_c[i][1] * uw[1] + orc_c[i][2] * uw[2];
      f[i] = own[orc_opp(i)] + 2.0 * orc_w[i] * cu / orc_cs2;
    } else if (wall >= 0) {
      f[i] = own[orc_opp(i)];
    } else {
      if (nreg != 1) return ORC_ERR_GEOMETRY;
      if (reg_face >= 0 && reg_face != reg) return ORC_ERR_GEOMETRY;
      reg_face = reg;
      unknown[i] = 1;
      f[i] = 0.0;
    }
  }

  if (reg_face < 0) {
    if (g->collision == ORC_REGULARIZED) orc_collide_regularized(f, g->tau, out);
    else orc_collide_bgk(f, g->tau, out);
    return ORC_OK;
  }

  /* Regularized boundary (Latt et al. 2008), on face reg_face with outward
   * normal nrm.  T: c.n = 0, O: c.n > 0 (known), U: c.n < 0 (sources outside). */
  const int axis = reg_face / 2;
  double nrm[3] = {0, 0, 0};
  nrm[axis] = (reg_face % 2) ? 1.0 : -1.0;
  double sT = 0, sO = 0;
  for (int i = 0; i < ORC_Q; ++i) {
    double cn = orc_c[i][0] * nrm[0] + orc_c[i][1] * nrm[1] + orc_c[i][2] * nrm[2];
    if (cn == 0) sT += f[i];
    else if (cn > 0) sO += f[i];
  }
  double rho, u[3];
  if (g->bc_kind[reg_face] == ORC_REG_VEL) {
    for (int a = 0; a < 3; ++a) u[a] = g->bc_val[reg_face][a];
    double un = u[0] * nrm[0] + u[1] * nrm[1] + u[2] * nrm[2];
    rho = (sT + 2.0 * sO) / (1.0 + un);
  } else {
    rho = g->bc_val[reg_face][0];
    double un = (sT + 2.0 * sO) / rho - 1.0;
    for (int a = 0; a < 3; ++a) u[a] = un * nrm[a];
  }
  double feq[ORC_Q], f1[ORC_Q];
  orc_equilibrium(rho, u, feq);
  /* non-equilibrium bounce-back of the unknown populations */
  for (int i = 0; i < ORC_Q; ++i)
    if (unknown[i]) {
      int o = orc_opp(i);
      f[i] = feq[i] + (f[o] - feq[o]);
    }
  orc_f1(f, feq, f1);
  for (int i = 0; i < ORC_Q; ++i) out[i] = feq[i] + (1.0 - 1.0 / g->tau) * f1[i];
  return ORC_OK;
}

/* One step over every fluid voxel.  Returns 0, or a negative code if the
 * geometry has a link that crosses two regularized faces. */
int orc_step(const orc_grid *g, const double *fin, double *fout) {
  int err = 0;
#pragma omp parallel for collapse(2) schedule(static) reduction(| : err)
  for (int z = 0; z < g->nz; ++z)
    for (int y = 0; y < g->ny; ++y)
      for (int x = 0; x < g->nx; ++x) {
        if (!orc_is_fluid(g, x, y, z)) continue;
        size_t v = (size_t)x + (size_t)g->nx * ((size_t)y + (size_t)g->ny * z);
        if (orc_update_voxel(g, fin, x, y, z, fout + v * ORC_Q) != ORC_OK) err |= 1;
      }
  return err ? ORC_ERR_GEOMETRY : ORC_OK;
}

/* n steps with ping-pong between f and work; the result ends in f. */
int orc_run(const orc_grid *g, double *f, double *work, int32_t nsteps) {
  size_t nv = (size_t)g->nx * g->ny * g->nz;
  for (int s = 0; s < nsteps; ++s) {
    int r = orc_step(g, f, work);
    if (r) return r;
    memcpy(f, work, nv * ORC_Q * sizeof(double));
  }
  return ORC_OK;
}

/* Updates of a list of voxels only (linear box indices); out is [n][19].
 * Used to check single outputs of a large GPU run one by one. */
int orc_step_voxels(const orc_grid *g, const double *fin, const int64_t *vox,
                    int64_t nvox, double *out) {
  int err = 0;
#pragma omp parallel for schedule(static) reduction(| : err)
  for (int64_t k = 0; k < nvox; ++k) {
    int64_t v = vox[k];
    int x = (int)(v % g->nx);
    int y = (int)((v / g->nx) % g->ny);
    int z = (int)(v / ((int64_t)g->nx * g->ny));
    if (orc_update_voxel(g, fin, x, y, z, out + k * ORC_Q) != ORC_OK) err |= 1;
  }
  return err ? ORC_ERR_GEOMETRY : ORC_OK;
}

/* f^eq(rho(x), u(x)) on every voxel; rho [nv], u [nv][3]. */
void orc_init_equilibrium(const orc_grid *g, const double *rho, const double *u,
                          double *f) {
  size_t nv = (size_t)g->nx * g->ny * g->nz;
#pragma omp parallel for schedule(static)
  for (size_t v = 0; v < nv; ++v) orc_equilibrium(rho[v], u + 3 * v, f + v * ORC_Q);
}

/* rho, u of every voxel (solid voxels included; their values are unused). */
void orc_macroscopic(const orc_grid *g, const double *f, double *rho, double *u) {
  size_t nv = (size_t)g->nx * g->ny * g->nz;
#pragma omp parallel for schedule(static)
  for (size_t v = 0; v < nv; ++v) orc_moments(f + v * ORC_Q, rho + v, u + 3 * v);
}
