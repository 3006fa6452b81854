// Host-side grid representation of liblbm (internal).
#pragma once
#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lbm.h"

namespace lbm {

// Groups of the block layouts, in storage order.  The classification
// follows the paper's disaggregated design: blocks next to a resolution jump
// (multires only), heavy-boundary blocks, then non-boundary blocks split by
// whether any voxel pulls from a non-fluid source ("masked") or none does
// ("full").
enum BlockGroup : int {
  kGroupJump = 0,
  kGroupBoundary = 1,
  kGroupMasked = 2,
  kGroupFull = 3,
  kNumGroups = 4
};

struct FaceBC {
  int32_t kind = LBM_BC_BOUNCE_BACK;
  double value[3] = {0, 0, 0};
};

// One uniform block-sparse level: 4^3-voxel blocks in grouped Morton order.
struct BlockLevel {
  int32_t nx = 0, ny = 0, nz = 0;     // level box in level voxels
  int32_t nbx = 0, nby = 0, nbz = 0;  // level box in blocks
  int64_t nblocks = 0;
  std::array<int64_t, kNumGroups> group_count{};
  std::vector<int32_t> coords;     // [nblocks][3]
  std::vector<int32_t> nbr;        // [nblocks][q-1] (D3Q19: face and edge blocks; D3Q27: + corners)
  std::vector<uint64_t> fmask;     // [nblocks]
  std::vector<uint64_t> bbm;       // [nblocks][q-1]: lanes whose source is not a fluid voxel
  std::vector<int32_t> canon;      // [nblocks*64]: canonical index or -1
  std::vector<int32_t> slot_of_block;  // [nbz][nby][nbx] -> block slot or -1
  int64_t n_fluid = 0;
  bool grouped = true;             // memory-based grouping (else one Morton order)
  std::vector<uint8_t> group;      // [nblocks] BlockGroup of each storage slot
  std::vector<uint32_t> bbits;     // [(nblocks+31)/32] bit set = boundary-group block
  // bitmask layout only: indirect boundary records
  std::vector<int32_t> vid;        // [nblocks*64] record of the voxel, -1 = none
  std::vector<float> vrec;         // [nrec][4] value of the voxel's valued face (u or rho), 0
};

uint64_t morton_key(uint32_t bx, uint32_t by, uint32_t bz);

// Active blocks, classification, Morton order per group, neighbour tables,
// bounce masks and canonical indices of one level.  `fluid` is the level's
// voxel mask (nx*ny*nz, x fastest).  `dense` selects the shell/interior
// classification; otherwise blocks with a voxel next to a moving-wall or
// regularized face form the boundary group.  Returns "" or an error message.
// `jump` (optional, same shape as fluid) marks voxels next to a resolution
// jump; blocks holding one form the first group.
// `grouped` = false keeps all blocks in one Morton order (bitmask-based
// grouping) and builds the per-voxel indirect ids and boundary records.
// `q` selects the lattice (19 or 27), which fixes the neighbour directions.
std::string build_block_level(BlockLevel &L, int32_t nx, int32_t ny, int32_t nz,
                              const uint8_t periodic[3], const std::vector<uint8_t> &fluid,
                              const FaceBC faces[6], bool dense,
                              const std::vector<uint8_t> *jump = nullptr, bool grouped = true,
                              int q = 19);

// ---------------------------------------------------------------- multires
// Source-list entry of the jump tables: bits 31..29 buffer tag, bit 28 use
// the opposite population plane, bits 27..0 slot.  Tag kTagList means bits
// 27..0 index a list of 8 entries whose mean is the value (coalescence).
enum : uint32_t {
  kTagLevelCur = 0,
  kTagLevelPrev = 1,
  kTagFinerCur = 2,
  kTagFinerPrev = 3,
  kTagCoarserCur = 4,
  kTagList = 7
};
constexpr uint32_t kEntryOpp = 1u << 28;
constexpr uint32_t kSlotMask = (1u << 28) - 1;
inline uint32_t make_entry(uint32_t tag, uint32_t slot, bool opp) {
  return (tag << 29) | (opp ? kEntryOpp : 0u) | (slot & kSlotMask);
}

struct MultiresLevel {
  BlockLevel L;
  double tau = 0.6;
  // [njump][2 phases][19][64] entries (phase 0: first substep of the coarser
  // level's step, 1: second; the coarsest level uses phase 0 only)
  std::vector<uint32_t> jtab;
  std::vector<uint32_t> jlist;  // [nlist][8]
};

// Validates a multires descriptor and builds every level: active masks,
// jump voxels, grouped block maps and the jump gather tables.
std::string build_multires(std::vector<MultiresLevel> &levels, int32_t nx, int32_t ny, int32_t nz,
                           int32_t num_levels, const uint8_t periodic[3],
                           const std::vector<uint8_t> &level_map, const std::vector<uint8_t> &fluid,
                           const FaceBC faces[6], double tau_coarsest);

}  // namespace lbm
