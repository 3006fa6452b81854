// Launch descriptors shared between the C-ABI layer and the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/lbm.h"
#include "lattice.h"

namespace lbm {

// Per-face boundary parameters: face id 2*axis + side (side 1 = max face),
// kinds as lbm_bc, value = wall/inlet velocity or outlet density.
struct FaceParams {
  int32_t kind[6];
  float val[6][3];
  int32_t periodic;  // bit a set if axis a is periodic
};

struct StepArgs {
  const void *src;           // populations read (post-collision of the last step), S slots
  void *dst;                 // populations written; block layouts index both with pidx
  uint32_t S;                // plane stride in slots
  const int32_t *nbr;        // [nblocks][Q-1] neighbour block slots (-1 = none)
  const uint64_t *bbm;       // [nblocks][Q-1] bounce masks
  const int32_t *coords;     // [nblocks] packed bx | by << 10 | bz << 20
  int32_t nx, ny, nz;        // box in voxels
  float omega;               // 1 / tau
  FaceParams fp;
  const uint64_t *fmask;     // [nblocks] fluid voxels of each block
  // learned closure (interior groups when the collision is LBM_MLP)
  const void *mlp_w;              // packed bf16 weights
  const float *mlp_bias;          // b1 | b2 | b3
  const float *mlp_stdz;          // in_mean | in_inv_std | out_std | out_mean (32 each)
  const float *mlp_s2;            // sum of out_std^2 over the 19 outputs (the judge's floor)
  unsigned long long *mlp_fallbacks;  // voxels that fell back to the regularized operator (64-bit)
  float mlp_judge;                // relative L2 tolerance against the regularized f1 (0 = off)
  // bitmask-based grouping
  const uint32_t *bbits;          // [(nblocks+31)/32] bit set = boundary block
  const int32_t *vid;             // [S] boundary record of the slot, -1 = none
  const float *vrec;              // [nrec][4] record values
};

enum KernelKind : int32_t {
  kKernelBoundary = 0,      // heavy-boundary group (also the naive single kernel)
  kKernelMasked = 1,        // non-boundary blocks with bounce-back sources
  kKernelFull = 2,          // blocks whose every source is fluid
  kKernelJump = 3,          // multires blocks next to a resolution jump (table gather)
  kKernelCollide = 4,       // collision only, in place (unfused multires baseline)
  kKernelCollideHeavy = 5,  // collision only for heavy-boundary blocks
  kKernelLex = 6,           // dense lexicographic single kernel
  kKernelInteriorBits = 7,  // bitmask grouping: all blocks, non-boundary ones processed
  kKernelBoundaryBits = 8,  // bitmask grouping: all blocks, boundary ones processed
  kKernelLevelMerged = 9,   // every group of a small multires level in one launch
  kKernelLevelPair = 10      // two independent merged level updates (fused) in one launch
};

// Sources of the multires jump gather, indexed by table tag: own level now,
// own level one step back, finer level now, finer one step back, coarser now.
struct MrArgs {
  const void *src[5];
  uint32_t stride[5];      // slots per buffer (informational)
  const uint32_t *jtab;   // [njump][2][19][64]
  const uint32_t *jlist;  // [nlist][8]
  int32_t phase;          // 0 or 1
};

struct Launch {
  int32_t kind;
  int32_t fused;          // 0: store the gathered (pre-collision) populations only; 2 (merged
                          // level launch): uniform groups fused, jump group stored only
  int32_t first, count;   // block range of the launch
  uint32_t lds;           // dynamic LDS bytes the kernel never touches: requested only to cap the
                          // workgroups resident per CU (0: no cap)
  int32_t wide;           // 1: 64-bit pull addressing in every kernel that has both forms
  int32_t gcount[4];      // kKernelLevelMerged: blocks of the jump, boundary, masked, full groups
  StepArgs args;
  MrArgs mr;
  // kKernelLevelPair: the second level update (its group counts, arguments)
  int32_t gcount2[4];
  StepArgs args2;
  MrArgs mr2;
};

// ---- learned closure: training and utility launches (mlp_kernels.hip) ----
struct MlpBuffers {
  float *params;      // [kMlpParams] FP32 master weights
  float *adam_m;      // [kMlpParams]
  float *adam_v;      // [kMlpParams]
  float *grads;       // [kMlpParams]
  void *wpacked;      // packed bf16 weights
  float *bias;        // b1 | b2 | b3 (padded)
  float *stdz;        // standardization, 4 x 32
  float *s2;          // sum of out_std^2, derived from stdz by mlp_derive whenever stdz changes
  unsigned long long *fallbacks;
  float *save;        // [batch_max][288] forward intermediates
  float *dyt;         // [batch_max][19]
  float *dz1;         // [batch_max][64]
  float *dz2;         // [batch_max][64]
  double *partial;    // reduction partials
  float *gpartial;    // [batch_max / 128][kMlpParams] per-chunk weight gradients
  int64_t batch_max;
};

LBM_NAMESPACE_K19 {  // D3Q19 only
hipError_t mlp_pack(const MlpBuffers &B, hipStream_t s);
hipError_t mlp_fit_standardization(const MlpBuffers &B, const float *f, int64_t n, hipStream_t s);
// the values derived from the standardization (B.s2)
hipError_t mlp_derive(const MlpBuffers &B, hipStream_t s);
hipError_t mlp_forward(const MlpBuffers &B, const float *f, int64_t n, float *y, hipStream_t s);
hipError_t mlp_gradients(const MlpBuffers &B, const float *f, const int64_t *idx, int64_t n, double *loss,
                         hipStream_t s);
// Adam step t on `grads` (B.grads or a caller's array), then the bf16 copy
hipError_t mlp_adam(const MlpBuffers &B, const float *grads, float lr, int32_t t, hipStream_t s);
// seeded He-uniform weights and zero biases, then the bf16 copy
hipError_t mlp_init(const MlpBuffers &B, uint64_t seed, hipStream_t s);
hipError_t launch_sample_pre(const StepArgs &a, int32_t storage, int32_t b0, int32_t nb, uint64_t seed, int64_t n,
                             float *out, hipStream_t s);
}  // namespace k19

// FP64 reductions run in three fixed-order passes: one partial row per 64
// slots, sums of kReduceChunk rows, then one sum of those.
constexpr int64_t kReduceChunk = 2048;
inline int64_t reduce_mid_rows(int64_t rows) { return rows > 0 ? (rows + kReduceChunk - 1) / kReduceChunk : 1; }

// Utility kernels over a slot range [0, nslots) with an optional canonical
// map (NULL = identity, every slot fluid).
struct SlotArgs {
  void *pop_a;               // current buffer
  void *pop_b;               // other buffer (init writes both)
  uint32_t S;                // plane stride
  int64_t nslots;            // slots to visit (multiple of 64 for block layouts)
  const int32_t *canon;      // [nslots] or NULL
  int64_t n;                 // canonical length
  int32_t storage;
  int32_t blocked;           // 1: block-interleaved populations, 0: planes of S
};

// The reduction without workspace scratch (lbm_reduce_noalloc): the same
// fixed-order sums, the first two passes fused per chunk of kReduceChunk
// rows, the chunk sums kept in a device array of kNoAllocMidRows rows of five
// doubles that the library holds for the life of the process.
constexpr int kReduceMaxLevels = 8;
constexpr int64_t kNoAllocMidRows = 4096;
struct ReduceLevels {
  SlotArgs a[kReduceMaxLevels];
  double weight[kReduceMaxLevels];
  int64_t row0[kReduceMaxLevels + 1];  // first partial row of each level; row0[nlevels] = all rows
  int32_t nlevels;
};

// Launchers built once per lattice (step_kernels.hip and util_kernels.hip
// are compiled for D3Q19 into k19 and for D3Q27 into k27).
#define LBM_DECLARE_LATTICE_LAUNCHERS                                                                  \
  hipError_t launch_one(const Launch &L, int32_t storage, int32_t collision, hipStream_t s);           \
  hipError_t launch_init_equilibrium(const SlotArgs &A, const double *rho, const double *u,             \
                                     hipStream_t s);                                                   \
  hipError_t launch_read_macroscopic(const SlotArgs &A, void *rho, void *u, int out_f64, hipStream_t s); \
  hipError_t launch_read_populations(const SlotArgs &A, double *f, hipStream_t s);                      \
  hipError_t launch_write_populations(const SlotArgs &A, const double *f, hipStream_t s);               \
  /* partial sums per 64-slot group (weighted by `weight`) into partial[first_row..] */                 \
  hipError_t launch_reduce_partial(const SlotArgs &A, double weight, double *partial, hipStream_t s);   \
  hipError_t launch_reduce_final(const double *partial, int64_t rows, double *mid, double *out5, hipStream_t s); \
  hipError_t launch_reduce_noalloc(const ReduceLevels &R, double *out5, hipStream_t s);

LBM_NAMESPACE_K19 {
LBM_DECLARE_LATTICE_LAUNCHERS
}
LBM_NAMESPACE_K27 {
LBM_DECLARE_LATTICE_LAUNCHERS
}

}  // namespace lbm
