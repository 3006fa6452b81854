/*
 * lbm.h -- C ABI of liblbm.so, a D3Q19 lattice-Boltzmann collide-and-stream
 * library for AMD Instinct MI355X (gfx950) built around the disaggregated
 * data-structure design of "Disaggregated Design for GPU-Based Volumetric
 * Data Structures" (arXiv 2503.07898).
 *
 * The paper's method (section "Disaggregated Design Method", Definition 1):
 * pick properties that matter for a performance objective, classify voxels
 * into groups by them, map each group to memory with an ordinary locality
 * order, and run a group-specific operation on each group.  This library
 * applies it to the three grid kinds of that section:
 *   - dense grids ("Disaggregation on a Dense Domain"): a shell group of
 *     blocks that touch a non-periodic box face and an interior group;
 *   - block-sparse grids of 4^3-voxel blocks ("Disaggregation on a Sparse
 *     Domain", memory-based grouping): boundary blocks stored first, then
 *     non-boundary blocks, one kernel per group;
 *   - multi-resolution grids ("Disaggregation on a Multi-resolution
 *     Domain"): per level, blocks near a resolution jump and uniform blocks,
 *     with collide and stream fused on the uniform ones.
 * The update itself is the LBM of the evaluation section: D3Q19 (D3Q27 on
 * request), BGK collision, halfway bounce-back on obstacles, regularized
 * inflow/outflow faces, and a moving-wall lid for the lid-driven cavity.
 *
 * Conventions shared by every call
 *   - Every function returns an lbm_status and never aborts.  On failure,
 *     lbm_last_error() returns a message for the calling thread.
 *   - The library never allocates device memory and never creates streams.
 *     The caller allocates one device workspace whose size lbm_grid_commit
 *     reports and passes it to lbm_grid_bind; it must stay valid until
 *     lbm_grid_destroy.  Device pointers passed to other calls are caller
 *     owned as well.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Device work is enqueued asynchronously on it; host-side results
 *     (sizes, index maps) are returned synchronously.
 *   - Call order: create -> set_boundary* -> commit -> bind -> init or
 *     write_populations -> step / read / reduce.  Calls made out of order
 *     return LBM_ERR_STATE.
 *   - Voxel coordinates: x fastest, then y, then z.  "Canonical order" of a
 *     level lists its fluid voxels in that lexicographic order of level
 *     coordinates; every array exchanged with the caller uses it.  The
 *     internal grouped layout stays private and is exposed only through
 *     lbm_get_index_map.
 *   - Lattice direction order: 0 rest; 1..6 = +x,-x,+y,-y,+z,-z;
 *     7..18 = (+1,+1,0),(-1,-1,0),(+1,-1,0),(-1,+1,0),(+1,0,+1),(-1,0,-1),
 *     (+1,0,-1),(-1,0,+1),(0,+1,+1),(0,-1,-1),(0,+1,-1),(0,-1,+1).
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBM_OK = 0,
  LBM_ERR_INVALID_ARG = -1,
  LBM_ERR_OUT_OF_MEMORY = -2, /* host allocation failed */
  LBM_ERR_HIP = -3,           /* a HIP runtime call failed; message holds hipGetErrorString */
  LBM_ERR_STATE = -4,         /* call out of order */
  LBM_ERR_UNSUPPORTED = -5,   /* valid request the library does not implement */
  LBM_ERR_NUMERIC = -6        /* non-finite values found by lbm_check */
} lbm_status;

/* Message of the last failure on the calling thread ("" if none). */
const char *lbm_last_error(void);

typedef struct lbm_grid lbm_grid; /* opaque host object owned by the library */

typedef enum { LBM_DENSE = 0, LBM_BLOCK_SPARSE = 1, LBM_MULTIRES = 2 } lbm_grid_kind;

/* Population storage.  The shifted forms store h_i = f_i - w_i rounded to
 * nearest-even in binary16 / bfloat16; arithmetic is FP32 in every form. */
typedef enum { LBM_F32 = 0, LBM_F16_SHIFTED = 1, LBM_BF16_SHIFTED = 2 } lbm_storage;

/* Collision operator for non-boundary voxels: BGK (evaluation section),
 * the regularized operator (Hermite projection of the non-equilibrium part,
 * the same projection the regularized faces use), or a learned MLP closure. */
typedef enum { LBM_BGK = 0, LBM_REGULARIZED = 1, LBM_MLP = 2 } lbm_collision;

/* LBM_PLAIN_SINGLE_KERNEL: the comparison arm of each grid kind --
 *   dense: one kernel over a lexicographic structure-of-arrays box;
 *   block-sparse: the "naive" single kernel (table dissBlock) that carries
 *     every boundary rule and so the boundary register demand everywhere;
 *   multires: collision and streaming as separate kernels at every level
 *     except the finest (the unfused baseline of the multires evaluation).
 * LBM_DISAGG: the disaggregated groups, one specialized kernel per group
 *   (memory-based grouping: each group contiguous, "Disaggregation on a
 *   Sparse Domain", table dissBlock).
 * LBM_DISAGG_BITMASK: the bitmask-based grouping of the same section, for
 *   dense and block-sparse grids: blocks stay in one Morton order, a bit per
 *   block marks the boundary blocks, and two kernels each run over every
 *   block and skip the blocks of the other kind at run time.  Boundary
 *   values reach the boundary kernel through indirect indexing: a 32-bit id
 *   per voxel slot selects the voxel's entry in a contiguous buffer of
 *   boundary-voxel records.  Not with LBM_MLP, not for sampling.
 * LBM_DISAGG_UNIFORM_FUSED: multires only, the paper's own multires
 *   schedule ("Improving Multi-resolution LBM Kernel Fusion"): at every
 *   level above the finest, blocks of the uniform groups run the fused
 *   collide-and-stream kernels while jump blocks keep separate streaming
 *   (their gathers, stored) and collision kernels; the finest level is
 *   fused throughout, as in the other two multires schedules.  LBM_DISAGG
 *   fuses the jump blocks as well (their explosion and coalescence sources
 *   are precomputed gathers).  All three give the same FP32 result bit for
 *   bit. */
typedef enum {
  LBM_PLAIN_SINGLE_KERNEL = 0,
  LBM_DISAGG = 1,
  LBM_DISAGG_BITMASK = 2,
  LBM_DISAGG_UNIFORM_FUSED = 3
} lbm_schedule;

typedef struct {
  lbm_grid_kind kind;
  int32_t nx, ny, nz;        /* finest-level box in voxels; block grids need multiples of 4
                                (multires: of 4 * 2^(num_levels-1)) */
  uint8_t periodic[3];       /* per axis x, y, z: 1 = periodic */
  int32_t num_levels;        /* 1 for dense and block-sparse */
  const uint8_t *fluid_mask; /* host, nx*ny*nz, 1 = fluid, NULL = all fluid.  Dense grids
                                must be all fluid. Read during create only. */
  const uint8_t *level_map;  /* multires: host, nx*ny*nz level of each finest voxel
                                (0 = finest), else NULL. Read during create only. */
  double tau;                /* relaxation time (multires: of the coarsest level) */
  lbm_storage storage;
  lbm_collision collision;
  lbm_schedule schedule;
  int32_t lattice;           /* velocity set: 19 (D3Q19, also 0) or 27 (D3Q27, the lattice of
                                the block-sparse register study); D3Q27 is built for dense
                                and block-sparse grids with BGK or regularized collision.
                                Population arrays are [q][N] with q = the lattice. */
} lbm_grid_desc;

/* Builds the host side of a grid: classification into groups, locality
 * order per group, index and neighbour tables (Definition 1, steps 2-3).
 * Errors: LBM_ERR_INVALID_ARG for bad sizes or masks (message says which). */
lbm_status lbm_grid_create(const lbm_grid_desc *desc, lbm_grid **out);

typedef enum { LBM_XMIN = 0, LBM_XMAX, LBM_YMIN, LBM_YMAX, LBM_ZMIN, LBM_ZMAX } lbm_face;

/* Boundary kinds of the evaluation section: halfway bounce-back walls, a
 * moving-wall lid (lid-driven cavity; value = wall velocity, wall density 1),
 * and the regularized velocity inlet (value = u) / pressure outlet
 * (value[0] = density) of the wind-tunnel case.  Every face of a
 * non-periodic axis defaults to bounce-back.  Solid voxels inside the box are
 * always bounce-back. */
typedef enum {
  LBM_BC_BOUNCE_BACK = 0,
  LBM_BC_MOVING_WALL = 1,
  LBM_BC_REG_VELOCITY = 2,
  LBM_BC_REG_PRESSURE = 3
} lbm_bc;

lbm_status lbm_set_boundary(lbm_grid *g, lbm_face face, lbm_bc kind, const double value[3]);

/* Finishes classification (the boundary kinds decide the groups of a
 * block-sparse grid) and reports the device workspace size in bytes.
 * Errors: LBM_ERR_INVALID_ARG if a voxel would need two regularized faces. */
lbm_status lbm_grid_commit(lbm_grid *g, size_t *workspace_bytes);

/* Hands the library a device workspace of at least the committed size
 * (256-byte aligned) and uploads the index tables into it on `stream`. */
lbm_status lbm_grid_bind(lbm_grid *g, void *workspace, size_t bytes, void *stream);

/* Number of fluid voxels of a level (canonical array length). */
lbm_status lbm_num_voxels(const lbm_grid *g, int32_t level, int64_t *n);

/* Sets every fluid voxel of `level` to f^eq(rho, u); rho_dev [N] and
 * u_dev [3][N] are FP64 device arrays in canonical order. */
lbm_status lbm_init_equilibrium(lbm_grid *g, int32_t level, const double *rho_dev,
                                const double *u_dev, void *stream);

/* Advances n_steps time steps (multires: coarse steps).  Each step is the
 * fused pull collide-and-stream of every group, ping-ponging population
 * buffers inside the workspace.  Multires grids follow the level-recursive
 * schedule: a level-l step (2^l finest steps, tau_l - 1/2 = (tau - 1/2)
 * 2^(L-1-l)) runs the finer level's first substep, its own update, then the
 * finer level's second substep.  Explosion (coarse post-collision values
 * feeding the finer level) and coalescence (the finer level's streamed
 * values merging into coarse voxels, as the mean over the 2x2x2 footprint)
 * are gathers of the jump-group kernel; uniform blocks run the fused kernels
 * of the single-level grids.  A step only launches kernels on `stream` (no
 * allocation, memset or host synchronization after the first step of a
 * grid), so it can be captured into a HIP graph: the graph holds the
 * launches with the buffer roles they had, and the roles repeat every 2
 * steps (dense, block-sparse) or every 3 coarse steps (multires), so a
 * graph of a multiple of that many steps replays as further steps. */
lbm_status lbm_step(lbm_grid *g, int32_t n_steps, void *stream);

/* Density and velocity of every fluid voxel of `level` in canonical order,
 * computed in FP64 from the stored post-collision populations.  rho_dev [N],
 * u_dev [3][N]; out_is_f64 = 1 writes doubles, 0 writes floats. */
lbm_status lbm_read_macroscopic(lbm_grid *g, int32_t level, void *rho_dev, void *u_dev,
                                int32_t out_is_f64, void *stream);

/* FP64 reductions over all levels: out5_dev[0] = mass sum f,
 * [1..3] = momentum sum c f, [4] = kinetic energy sum rho |u|^2 / 2.
 * Multires levels weight each voxel by its volume 8^level.  Deterministic
 * (fixed-order two-pass sum). */
lbm_status lbm_reduce(lbm_grid *g, double *out5_dev, void *stream);

/* lbm_reduce for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same sums, bitwise equal to lbm_reduce's, computed without the
 * reduction scratch of the grid's workspace.  Its chunk sums live in a
 * device array of the library, 4096 rows of five doubles (160 KiB) per GPU,
 * held until the process ends; grids of more than 4096 x 2048 x 64 =
 * 536,870,912 slots (all levels together) are rejected with
 * LBM_ERR_INVALID_ARG, grids of more than 8 levels with LBM_ERR_UNSUPPORTED.
 * Allocates nothing (no hipMalloc, no host-side device allocation).  Every
 * call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (on different streams, or from different threads) race; calls on one
 * stream are ordered.  out5_dev: five doubles in device memory, written
 * asynchronously on `stream`. */
lbm_status lbm_reduce_noalloc(lbm_grid *g, double *out5_dev, void *stream);

/* Health check: runs the reductions above into the grid's workspace, waits
 * for the stream and returns LBM_ERR_NUMERIC if any sum is not finite.  A
 * NaN or infinite population anywhere makes the mass sum non-finite, so
 * this detects every blown-up state (the kernels themselves never test for
 * it).  Synchronizes `stream`; off the timed loop. */
lbm_status lbm_check(lbm_grid *g, void *stream);

/* Post-collision populations of `level` as FP64 [q][N] in canonical order. */
lbm_status lbm_read_populations(lbm_grid *g, int32_t level, double *f_dev, void *stream);
/* Overwrites the populations of `level` from FP64 [q][N] canonical order
 * (checkpoint restore); values are rounded to the storage format. */
lbm_status lbm_write_populations(lbm_grid *g, int32_t level, const double *f_dev, void *stream);

/* Index maps of the internal layout, copied to host memory.  Pass
 * host_out = NULL to query the element count in *count.
 *   LBM_MAP_GROUPS     int64 [5]: blocks per group in storage order (jump, boundary,
 *                      masked, full) and the total; "jump" blocks hold a voxel
 *                      next to a resolution jump (multires only), "boundary"
 *                      blocks a voxel next to a moving-wall or regularized face
 *                      (dense grids: a voxel on any non-periodic face), "masked"
 *                      blocks pull from some non-fluid source, "full" blocks
 *                      do not
 *   LBM_MAP_COORDS     int32 [nblocks][3]: block coordinates, in storage order
 *   LBM_MAP_NEIGHBOURS int32 [nblocks][q-1]: slot of the neighbour block in
 *                      direction 1..q-1 of the grid's lattice, -1 = none
 *   LBM_MAP_FLUIDMASK  uint64 [nblocks]: bit x+4y+16z set for fluid voxels
 *   LBM_MAP_CANONICAL  int64 [nblocks*64]: canonical index of each slot, -1 = not fluid
 *   LBM_MAP_BOUNDARY_BITS uint32 [(nblocks+31)/32]: bit b set if storage block b is a
 *                      boundary-group block
 *   LBM_MAP_RECORD_IDS int32 [nblocks*64]: bitmask layout only (else empty): boundary
 *                      record of each slot, -1 = none */
typedef enum {
  LBM_MAP_GROUPS = 0,
  LBM_MAP_COORDS = 1,
  LBM_MAP_NEIGHBOURS = 2,
  LBM_MAP_FLUIDMASK = 3,
  LBM_MAP_CANONICAL = 4,
  LBM_MAP_BOUNDARY_BITS = 5,
  LBM_MAP_RECORD_IDS = 6
} lbm_map;
lbm_status lbm_get_index_map(const lbm_grid *g, int32_t level, lbm_map which, void *host_out,
                             size_t *count);

/* Kernel launches one lbm_step issues per (coarse) time step, and the blocks
 * each of them covers (for checking the structure of table dissBlock; a
 * merged multires level update, see lbm_set_merge_limit, covers all blocks
 * of its level).
 * blocks_out[max] receives block counts per launch; *n receives the launch
 * count. */
lbm_status lbm_step_launches(const lbm_grid *g, int64_t *blocks_out, int32_t max, int32_t *n);

/* ------------------------------------------------- learned collision closure
 * A 19-64-64-19 perceptron with tanh-form GELU activations (an addition of
 * this library; the paper has no learned component).  Input: the
 * standardized non-equilibrium part per unit density of a voxel,
 * g = (f - f^eq(rho, u))/rho; output: an
 * estimate y of the regularized operator's non-equilibrium part per unit
 * density, projected onto the second-order Hermite space (no mass, momentum
 * or higher-order content: P(y)_i = w_i/(2 c_s^4) Q_i : sum_j Q_j y_j with
 * Q_i = c_i c_i - c_s^2 I); post-collision state
 * f* = f^eq + (1 - 1/tau) rho P(y).  Inference and training forward run on
 * the matrix cores in bfloat16 with FP32 accumulation; FP32 master weights
 * are trained with Adam (beta 0.9 / 0.999, eps 1e-8) on the mean squared
 * error of P(y) against f1/rho divided by the mean target variance (a
 * scale-free loss; the raw error is of order 1e-9).  Parameters are flat FP32 arrays of
 * LBM_MLP_PARAMS values: W1 [19][64], b1 [64], W2 [64][64], b2 [64],
 * W3 [64][19], b3 [19] (row-major, W_k indexed [input][output]).
 * Standardization: 128 floats, in_mean [32] | in_inv_std [32] |
 * out_std [32] | out_mean [32] (first 19 of each used). */
#define LBM_MLP_PARAMS 6675
#define LBM_MLP_BATCH_MAX 8192
typedef struct lbm_mlp lbm_mlp;

/* Creates a closure object and reports the device buffer it needs. */
lbm_status lbm_mlp_create(lbm_mlp **out, size_t *bytes_needed);
/* Binds caller-owned device memory (256-byte aligned); clears optimizer
 * state and the fallback counter, sets identity standardization. */
lbm_status lbm_mlp_bind(lbm_mlp *m, void *device_buffer, size_t bytes, void *stream);
/* Copies LBM_MLP_PARAMS host floats into the master weights (synchronous). */
lbm_status lbm_mlp_set_params(lbm_mlp *m, const float *host_params, void *stream);
lbm_status lbm_mlp_get_params(lbm_mlp *m, float *host_params, void *stream);
/* 128 host floats (layout above), synchronous. */
lbm_status lbm_mlp_set_standardization(lbm_mlp *m, const float *host_stdz, void *stream);
lbm_status lbm_mlp_get_standardization(lbm_mlp *m, float *host_stdz, void *stream);
/* Per-component mean and standard deviation of the inputs g and targets
 * f1/rho over n populations f_dev [n][19] (FP32, unshifted). */
lbm_status lbm_mlp_fit_standardization(lbm_mlp *m, const float *f_dev, int64_t n, void *stream);
/* Network output y (de-standardized, before projection) for n populations. */
lbm_status lbm_mlp_forward(lbm_mlp *m, const float *f_dev, int64_t n, float *y_dev, void *stream);
/* Loss and gradients of one batch of n <= LBM_MLP_BATCH_MAX populations:
 * rows idx_dev[0..n) of f_dev (int64 device array), or rows 0..n-1 when
 * idx_dev is NULL.  grads_dev [LBM_MLP_PARAMS] and loss_dev (one double)
 * may be NULL. */
lbm_status lbm_mlp_gradients(lbm_mlp *m, const float *f_dev, const int64_t *idx_dev, int64_t n,
                             float *grads_dev, double *loss_dev, void *stream);
/* One training step on such a batch: gradients, then Adam step t (t >= 1)
 * with learning rate lr on the FP32 master weights, then the bf16 copy. */
lbm_status lbm_mlp_train_step(lbm_mlp *m, const float *f_dev, const int64_t *idx_dev, int64_t n,
                              float lr, int32_t t, double *loss_dev, void *stream);
/* Adam step t (t >= 1, learning rate lr > 0; beta 0.9 / 0.999, eps 1e-8)
 * on caller-supplied gradients grads_dev [LBM_MLP_PARAMS] (FP32, device;
 * e.g. from lbm_mlp_gradients, possibly combined by the caller), then the
 * bf16 copy of the weights.  Asynchronous on `stream`. */
lbm_status lbm_mlp_adam(lbm_mlp *m, const float *grads_dev, float lr, int32_t t, void *stream);
/* Seeded initial weights on the device: He-uniform
 * U(-sqrt(6/fan_in), +sqrt(6/fan_in)) per layer (fan_in 19, 64, 64), zero
 * biases; weight p takes 53 bits of splitmix64(seed ^ splitmix64(p))
 * (Steele, Lea and Flood 2014), so a seed fixes the network on any device.
 * Asynchronous on `stream`; optimizer state is left as it is. */
lbm_status lbm_mlp_init_params(lbm_mlp *m, uint64_t seed, void *stream);
/* Tolerance of the run-time judge (default 0.01): a voxel keeps the
 * closure's update only if |P(y) - f1/rho|_2^2 <= rel_tol^2 (|f1/rho|_2^2 +
 * |out_std|_2^2), with f1 the regularized operator's non-equilibrium part
 * and out_std the output scale of the standardization (the floor lets voxels
 * near equilibrium keep small absolute deviations); 0 switches the judge off
 * (the range and positivity tests remain).  Near tau = 1/2 an overshoot of
 * the regularized stress by more than 1/(1 - 1/tau) - 1 (1.5% at
 * tau = 0.5038) is unstable, which the default keeps out.  Takes effect at
 * the next step of every grid that uses this closure. */
lbm_status lbm_mlp_set_judge(lbm_mlp *m, double rel_tol);
/* Voxels that fell back to the regularized operator since bind/reset. */
lbm_status lbm_mlp_fallbacks(lbm_mlp *m, uint64_t *host_count, int32_t reset, void *stream);
lbm_status lbm_mlp_destroy(lbm_mlp *m);

/* Switches a committed dense or block-sparse grid (disaggregated schedule)
 * to another collision operator.  LBM_MLP needs a bound closure and applies
 * it to the non-boundary groups; blocks of the boundary group then use the
 * regularized operator.  The closure must outlive its use by the grid. */
lbm_status lbm_set_collision(lbm_grid *g, lbm_collision c, const lbm_mlp *m);

/* Launch shape of multires level updates (a tuning knob; results are bit
 * for bit the same either way).  The groups of one level update are
 * independent (section on multi-resolution kernel fusion), so a level with
 * at most max_blocks blocks runs all of them as one launch; larger levels
 * launch one kernel per group.  Default 8192 (the chip's wave slots at
 * eight waves per SIMD); 0 keeps one launch per group everywhere.  Dense
 * and block-sparse grids always launch per group.  Any grid state; takes
 * effect at the next step.  max_blocks < 0 is LBM_ERR_INVALID_ARG. */
lbm_status lbm_set_merge_limit(lbm_grid *g, int64_t max_blocks);

/* Residency cap of the stepping kernels (a tuning knob; results are bit for
 * bit the same either way).  Each 256-thread workgroup of the block kernels
 * (every kernel of lbm_step except the closure's and the multires jump and
 * merged-level kernels, which always run uncapped) requests LDS it never
 * touches, (LDS per CU) / wg_per_cu bytes rounded down to 1 KiB, so that at
 * most wg_per_cu workgroups (4 waves each) sit on one compute unit.  The
 * HBM bytes stay the same; fewer requests in flight raise the rate at which
 * HBM serves them (a plain 19-row-per-wave copy measures 5.99 TB/s at 4
 * workgroups per CU against 5.78 at 8), as long as enough remain to cover
 * the latency.  0 removes the cap (registers then allow up to 8 per CU);
 * LBM_RESIDENCY_AUTO (the default) takes a per-kernel value measured on
 * MI355X for the kernel kind, storage and lattice.  Any grid state; takes
 * effect at the next launch.  Values outside LBM_RESIDENCY_AUTO..8 are
 * LBM_ERR_INVALID_ARG. */
#define LBM_RESIDENCY_AUTO (-1)
lbm_status lbm_set_residency(lbm_grid *g, int32_t wg_per_cu);

/* Pull addressing of the learned-closure kernel (a diagnostic knob; results
 * are bit for bit the same either way).  While a population buffer spans at
 * most 4 GiB the kernel forms each pull's address as a 32-bit byte offset
 * over the buffer's start, built from wave-uniform neighbour deltas and
 * per-lane face masks (fewer vector instructions in a kernel bound by their
 * issue); larger buffers use 64-bit slot arithmetic.  wide = 1 forces the
 * 64-bit form at any size, so that it can be checked against the 32-bit one
 * on grids of every size; 0 (the default) restores the automatic choice.
 * Any grid state; takes effect at the next launch.  Other values are
 * LBM_ERR_INVALID_ARG. */
lbm_status lbm_set_wide_addressing(lbm_grid *g, int32_t wide);

/* n pre-collision population sets (FP32, unshifted, [n][19]: the values the
 * collision operator of the next step receives, pulled from the current
 * post-collision field with bounce-back) of fluid voxels drawn uniformly
 * with replacement from the non-boundary groups of `level` (counter-based
 * splitmix64 stream from `seed`) -- the training data of the closure.
 * Needs a block layout. */
lbm_status lbm_sample_populations(lbm_grid *g, int32_t level, uint64_t seed, int64_t n, float *f_dev,
                                  void *stream);

/* Measurement hook: enqueues launch k (0-based, in lbm_step_launches order) of
 * one step on its own -- it reads the current populations and writes the
 * other buffer, which does not become current.  Lets a caller time one
 * group's kernel in isolation. */
lbm_status lbm_launch_group(lbm_grid *g, int32_t k, void *stream);

lbm_status lbm_grid_destroy(lbm_grid *g);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
