// Host-side grid representation of liblbm (internal).
#pragma once
#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lbm.h"

namespace lbm {

// Groups of the block layouts, in storage order.  The classification
// follows the paper's disaggregated design: heavy-boundary blocks, then
// non-boundary blocks split by whether any voxel pulls from a non-fluid
// source ("masked") or none does ("full").
enum BlockGroup : int { kGroupBoundary = 0, kGroupMasked = 1, kGroupFull = 2, kNumGroups = 3 };

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
  std::vector<int32_t> nbr;        // [nblocks][18]
  std::vector<uint64_t> fmask;     // [nblocks]
  std::vector<uint64_t> bbm;       // [nblocks][18]: lanes whose source is not a fluid voxel
  std::vector<int32_t> canon;      // [nblocks*64]: canonical index or -1
  std::vector<int32_t> slot_of_block;  // [nbz][nby][nbx] -> block slot or -1
  int64_t n_fluid = 0;
};

uint64_t morton_key(uint32_t bx, uint32_t by, uint32_t bz);

// Active blocks, classification, Morton order per group, neighbour tables,
// bounce masks and canonical indices of one level.  `fluid` is the level's
// voxel mask (nx*ny*nz, x fastest).  `dense` selects the shell/interior
// classification; otherwise blocks with a voxel next to a moving-wall or
// regularized face form the boundary group.  Returns "" or an error message.
std::string build_block_level(BlockLevel &L, int32_t nx, int32_t ny, int32_t nz,
                              const uint8_t periodic[3], const std::vector<uint8_t> &fluid,
                              const FaceBC faces[6], bool dense);

}  // namespace lbm
