// Host grid builder: classification and locality mapping of the
// disaggregated block layout (Definition 1, steps 2 and 3; block-sparse
// grids managed by a space-filling curve; memory-based grouping with the
// boundary group stored first, or bitmask-based grouping with one Morton
// order and indirect boundary records).
#include <algorithm>
#include <cstring>

#include "grid.h"
#include "lattice.h"

namespace lbm {

uint64_t morton_key(uint32_t bx, uint32_t by, uint32_t bz) {
  // spread the low 21 bits of v so that bit b lands at bit 3b
  auto spread = [](uint64_t v) {
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
  };
  return spread(bx) | (spread(by) << 1) | (spread(bz) << 2);
}

static bool heavy_face(const FaceBC &f) {
  return f.kind == LBM_BC_MOVING_WALL || f.kind == LBM_BC_REG_VELOCITY ||
         f.kind == LBM_BC_REG_PRESSURE;
}

std::string build_block_level(BlockLevel &L, int32_t nx, int32_t ny, int32_t nz,
                              const uint8_t periodic[3], const std::vector<uint8_t> &fluid,
                              const FaceBC faces[6], bool dense, const std::vector<uint8_t> *jump,
                              bool grouped, int q) {
  const LatticeDesc lat = lattice_desc(q);
  const int NQ = lat.q, NB = lat.q - 1;
  if (!grouped && jump) return "the bitmask layout has no resolution jumps";
  if (nx <= 0 || ny <= 0 || nz <= 0 || nx % 4 || ny % 4 || nz % 4)
    return "block grids need positive sizes that are multiples of 4";
  if (nx / 4 >= 1024 || ny / 4 >= 1024 || nz / 4 >= 1024)
    return "block grids are limited to 4092 voxels per axis";
  L = BlockLevel{};
  L.nx = nx; L.ny = ny; L.nz = nz;
  L.nbx = nx / 4; L.nby = ny / 4; L.nbz = nz / 4;
  const int64_t nvox = (int64_t)nx * ny * nz;
  if ((int64_t)fluid.size() != nvox) return "fluid mask has the wrong size";
  auto fl = [&](int64_t x, int64_t y, int64_t z) -> bool {
    return fluid[(size_t)(x + nx * (y + (int64_t)ny * z))] != 0;
  };
  const int64_t nbtot = (int64_t)L.nbx * L.nby * L.nbz;

  // per-block fluid masks (and jump-voxel flags) over the whole block box
  std::vector<uint64_t> bm(nbtot, 0);
  std::vector<uint8_t> bj(jump ? nbtot : 0, 0);
  for (int64_t z = 0; z < nz; ++z)
    for (int64_t y = 0; y < ny; ++y)
      for (int64_t x = 0; x < nx; ++x)
        if (fl(x, y, z)) {
          int64_t b = x / 4 + L.nbx * (y / 4 + (int64_t)L.nby * (z / 4));
          bm[b] |= 1ull << ((x & 3) + 4 * (y & 3) + 16 * (z & 3));
          if (jump && (*jump)[(size_t)(x + nx * (y + (int64_t)ny * z))]) bj[b] = 1;
        }

  const int nb3[3] = {L.nbx, L.nby, L.nbz};
  auto bid = [&](int bx, int by, int bz) -> int64_t {
    return bx + (int64_t)L.nbx * (by + (int64_t)L.nby * bz);
  };
  // neighbour block id in lattice direction d, or -1 (outside a non-periodic box)
  auto nb_id = [&](int bx, int by, int bz, int d) -> int64_t {
    int q[3] = {bx + lat.cx[d], by + lat.cy[d], bz + lat.cz[d]};
    for (int a = 0; a < 3; ++a) {
      if (q[a] < 0 || q[a] >= nb3[a]) {
        if (!periodic[a]) return -1;
        q[a] = (q[a] + nb3[a]) % nb3[a];
      }
    }
    return bid(q[0], q[1], q[2]);
  };

  // voxels next to heavy faces (moving wall, regularized inlet/outlet)
  auto block_has_heavy = [&](int bx, int by, int bz) -> bool {
    uint64_t m = bm[bid(bx, by, bz)];
    if (!m) return false;
    for (int f = 0; f < 6; ++f) {
      int axis = f / 2, side = f % 2;
      if (periodic[axis] || !heavy_face(faces[f])) continue;
      int b[3] = {bx, by, bz};
      if (b[axis] != (side ? nb3[axis] - 1 : 0)) continue;
      int l = side ? 3 : 0;  // local layer on that face
      for (int k = 0; k < 64; ++k) {
        int lc[3] = {k & 3, (k >> 2) & 3, k >> 4};
        if (lc[axis] == l && ((m >> k) & 1)) return true;
      }
    }
    return false;
  };

  std::vector<std::pair<uint64_t, int64_t>> grp[kNumGroups];
  for (int bz = 0; bz < L.nbz; ++bz)
    for (int by = 0; by < L.nby; ++by)
      for (int bx = 0; bx < L.nbx; ++bx) {
        int64_t b = bid(bx, by, bz);
        if (!bm[b]) continue;
        int g;
        if (jump && bj[b]) {
          grp[kGroupJump].push_back({morton_key(bx, by, bz), b});
          continue;
        }
        bool shell = (!periodic[0] && (bx == 0 || bx == L.nbx - 1)) ||
                     (!periodic[1] && (by == 0 || by == L.nby - 1)) ||
                     (!periodic[2] && (bz == 0 || bz == L.nbz - 1));
        if (dense ? shell : block_has_heavy(bx, by, bz)) {
          g = kGroupBoundary;
        } else {
          bool full = bm[b] == ~0ull;
          for (int d = 1; d < NQ && full; ++d) {
            int64_t n = nb_id(bx, by, bz, d);
            if (n < 0 || bm[n] != ~0ull) full = false;
          }
          g = full ? kGroupFull : kGroupMasked;
        }
        grp[g].push_back({morton_key(bx, by, bz), b});
      }

  L.slot_of_block.assign(nbtot, -1);
  L.grouped = grouped;
  std::vector<int64_t> order;
  std::vector<uint8_t> gid_of(nbtot, 0);
  for (int g = 0; g < kNumGroups; ++g) {
    std::sort(grp[g].begin(), grp[g].end());
    L.group_count[g] = (int64_t)grp[g].size();
    for (auto &kv : grp[g]) gid_of[kv.second] = (uint8_t)g;
  }
  if (grouped) {
    for (int g = 0; g < kNumGroups; ++g)
      for (auto &kv : grp[g]) order.push_back(kv.second);
  } else {
    std::vector<std::pair<uint64_t, int64_t>> all;
    for (int g = 0; g < kNumGroups; ++g) all.insert(all.end(), grp[g].begin(), grp[g].end());
    std::sort(all.begin(), all.end());
    for (auto &kv : all) order.push_back(kv.second);
  }
  for (size_t s = 0; s < order.size(); ++s) L.slot_of_block[order[s]] = (int32_t)s;
  L.nblocks = (int64_t)order.size();
  if (L.nblocks == 0) return "the grid has no fluid voxel";
  if (L.nblocks * 64 >= (int64_t)1 << 31) return "too many blocks for 32-bit slot indices";

  L.group.resize(L.nblocks);
  L.bbits.assign((L.nblocks + 31) / 32, 0u);
  for (int64_t s = 0; s < L.nblocks; ++s) {
    L.group[s] = gid_of[order[s]];
    if (L.group[s] == kGroupBoundary) L.bbits[s >> 5] |= 1u << (s & 31);
  }

  L.coords.resize(L.nblocks * 3);
  L.nbr.assign(L.nblocks * NB, -1);
  L.fmask.resize(L.nblocks);
  L.bbm.assign(L.nblocks * NB, 0);
  for (int64_t s = 0; s < L.nblocks; ++s) {
    int64_t b = order[s];
    int bx = (int)(b % L.nbx), by = (int)((b / L.nbx) % L.nby), bz = (int)(b / ((int64_t)L.nbx * L.nby));
    L.coords[3 * s] = bx; L.coords[3 * s + 1] = by; L.coords[3 * s + 2] = bz;
    L.fmask[s] = bm[b];
    int64_t nbid[27];
    nbid[0] = b;
    for (int d = 1; d < NQ; ++d) {
      int64_t n = nb_id(bx, by, bz, d);
      nbid[d] = n;
      if (n >= 0 && L.slot_of_block[n] >= 0) L.nbr[s * NB + d - 1] = L.slot_of_block[n];
    }
    // bounce masks: lane l of direction i pulls from l - c_i
    for (int i = 1; i < NQ; ++i) {
      uint64_t m = 0;
      for (int l = 0; l < 64; ++l) {
        int p[3] = {(l & 3) - lat.cx[i], ((l >> 2) & 3) - lat.cy[i], (l >> 4) - lat.cz[i]};
        int o[3];
        for (int a = 0; a < 3; ++a) o[a] = p[a] < 0 ? -1 : (p[a] > 3 ? 1 : 0);
        int64_t src_block = b;
        if (o[0] || o[1] || o[2]) src_block = nbid[lat.dir(o[0], o[1], o[2])];
        bool ok = src_block >= 0 &&
                  ((bm[src_block] >> ((p[0] & 3) + 4 * (p[1] & 3) + 16 * (p[2] & 3))) & 1);
        if (!ok) m |= 1ull << l;
      }
      L.bbm[s * NB + i - 1] = m;
    }
  }

  // canonical order: fluid voxels, x fastest
  L.canon.assign(L.nblocks * 64, -1);
  int64_t c = 0;
  for (int64_t z = 0; z < nz; ++z)
    for (int64_t y = 0; y < ny; ++y)
      for (int64_t x = 0; x < nx; ++x)
        if (fl(x, y, z)) {
          int64_t s = L.slot_of_block[x / 4 + L.nbx * (y / 4 + (int64_t)L.nby * (z / 4))];
          L.canon[s * 64 + (x & 3) + 4 * (y & 3) + 16 * (z & 3)] = (int32_t)c++;
        }
  L.n_fluid = c;

  if (!grouped) {
    // indirect boundary records: every fluid voxel of a boundary block that
    // lies on a moving-wall or regularized face gets one record holding that
    // face's value (wall / inlet velocity, or outlet density in component 0)
    L.vid.assign(L.nblocks * 64, -1);
    for (int64_t s = 0; s < L.nblocks; ++s) {
      if (L.group[s] != kGroupBoundary) continue;
      const int bx = L.coords[3 * s], by = L.coords[3 * s + 1], bz = L.coords[3 * s + 2];
      for (int l = 0; l < 64; ++l) {
        if (!((L.fmask[s] >> l) & 1)) continue;
        const int g[3] = {bx * 4 + (l & 3), by * 4 + ((l >> 2) & 3), bz * 4 + (l >> 4)};
        const int n3[3] = {nx, ny, nz};
        int valued = -1;
        for (int f = 0; f < 6; ++f) {
          const int a = f / 2;
          if (periodic[a] || !heavy_face(faces[f])) continue;
          if (g[a] != ((f & 1) ? n3[a] - 1 : 0)) continue;
          if (valued >= 0) return "the bitmask layout needs every voxel on at most one moving-wall or regularized face";
          valued = f;
        }
        if (valued < 0) continue;
        L.vid[s * 64 + l] = (int32_t)(L.vrec.size() / 4);
        for (int k = 0; k < 3; ++k) L.vrec.push_back((float)faces[valued].value[k]);
        L.vrec.push_back(0.0f);
      }
    }
    if (L.vrec.empty()) L.vrec.assign(4, 0.0f);  // keep the buffer non-empty
  }
  return "";
}

}  // namespace lbm
