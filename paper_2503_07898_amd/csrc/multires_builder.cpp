// Host builder of multi-resolution grids ("Disaggregation on a
// Multi-resolution Domain"): one block-sparse grid per level, the distance
// property that splits each level into blocks next to a resolution jump and
// uniform blocks, and the transition tables that express explosion and
// coalescence as gathers.
//
// Reading of the inter-level operators (the paper names them, explosion and
// coalescence, without formulas): coarse territory seen from the finer level
// holds virtual fine populations that start, at the beginning of the coarse
// step, as the coarse post-collision value of their cell and stream without
// colliding; a coarse voxel takes, per direction, the mean of the 8 virtual
// values that land on its 2x2x2 footprint after the two fine substeps.  Every
// source of a jump voxel is therefore a fixed slot in one of five buffers
// (own level now and one step back, finer level now and one step back,
// coarser level now), which the tables below record per voxel, direction and
// substep.
#include <algorithm>
#include <cmath>
#include <string>

#include "grid.h"
#include "lattice.h"

namespace lbm {

namespace {

struct Box {
  int32_t n[3];
  uint8_t per[3];
  const std::vector<uint8_t> *lm;
  const std::vector<uint8_t> *fl;
  int32_t L;

  int dim(int l, int a) const { return n[a] >> l; }
  // wraps level-l coordinates; false if outside a non-periodic face
  bool wrap(int l, int p[3]) const {
    for (int a = 0; a < 3; ++a) {
      const int m = dim(l, a);
      if (p[a] < 0 || p[a] >= m) {
        if (!per[a]) return false;
        p[a] = ((p[a] % m) + m) % m;
      }
    }
    return true;
  }
  // level owning the finest cube of level-l cell p (in box)
  int terr(int l, const int p[3]) const {
    const size_t x = (size_t)p[0] << l, y = (size_t)p[1] << l, z = (size_t)p[2] << l;
    return (*lm)[x + (size_t)n[0] * (y + (size_t)n[1] * z)];
  }
  bool fluid0(const int p[3]) const {
    return (*fl)[(size_t)p[0] + (size_t)n[0] * ((size_t)p[1] + (size_t)n[1] * p[2])] != 0;
  }
  bool active(int l, const int p[3]) const { return terr(l, p) == l && (l > 0 || fluid0(p)); }
};

}  // namespace

std::string build_multires(std::vector<MultiresLevel> &levels, int32_t nx, int32_t ny, int32_t nz,
                           int32_t L, const uint8_t periodic[3], const std::vector<uint8_t> &level_map,
                           const std::vector<uint8_t> &fluid, const FaceBC faces[6],
                           double tau_coarsest) {
  if (L < 2 || L > 6) return "multires grids need 2 to 6 levels";
  const int top = 4 << (L - 1);
  if (nx <= 0 || ny <= 0 || nz <= 0 || nx % top || ny % top || nz % top)
    return "multires box sizes must be multiples of 4 * 2^(levels-1)";
  const int64_t nv = (int64_t)nx * ny * nz;
  if ((int64_t)level_map.size() != nv || (int64_t)fluid.size() != nv) return "level map has the wrong size";
  Box B{{nx, ny, nz}, {periodic[0], periodic[1], periodic[2]}, &level_map, &fluid, L};

  // ---- finest-block level array: uniform per 4^3 block, aligned, balanced
  const int fb[3] = {nx / 4, ny / 4, nz / 4};
  std::vector<int8_t> LV((size_t)fb[0] * fb[1] * fb[2]);
  for (int64_t bz = 0; bz < fb[2]; ++bz)
    for (int64_t by = 0; by < fb[1]; ++by)
      for (int64_t bx = 0; bx < fb[0]; ++bx) {
        int v0 = -1;
        for (int k = 0; k < 64; ++k) {
          int64_t x = bx * 4 + (k & 3), y = by * 4 + ((k >> 2) & 3), z = bz * 4 + (k >> 4);
          int v = level_map[(size_t)(x + nx * (y + (int64_t)ny * z))];
          if (v >= L) return "level map value out of range";
          if (v0 < 0) v0 = v;
          else if (v != v0) return "level map is not uniform over 4^3 finest blocks";
          if (v > 0 && !fluid[(size_t)(x + nx * (y + (int64_t)ny * z))])
            return "solid voxels must lie on the finest level";
        }
        LV[(size_t)(bx + fb[0] * (by + (int64_t)fb[1] * bz))] = (int8_t)v0;
      }
  auto lv_at = [&](int64_t bx, int64_t by, int64_t bz) {
    return (int)LV[(size_t)(bx + fb[0] * (by + (int64_t)fb[1] * bz))];
  };
  for (int64_t bz = 0; bz < fb[2]; ++bz)
    for (int64_t by = 0; by < fb[1]; ++by)
      for (int64_t bx = 0; bx < fb[0]; ++bx) {
        const int l = lv_at(bx, by, bz);
        const int64_t s = (int64_t)1 << l;  // a level-l block spans s finest blocks
        const int64_t ox = bx / s * s, oy = by / s * s, oz = bz / s * s;
        for (int64_t z = oz; z < oz + s; ++z)
          for (int64_t y = oy; y < oy + s; ++y)
            for (int64_t x = ox; x < ox + s; ++x)
              if (lv_at(x, y, z) != l) return "level map is not aligned to the blocks of each level";
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              int q[3] = {(int)bx + dx, (int)by + dy, (int)bz + dz};
              bool in = true;
              for (int a = 0; a < 3; ++a)
                if (q[a] < 0 || q[a] >= fb[a]) {
                  if (!periodic[a]) in = false;
                  else q[a] = (q[a] + fb[a]) % fb[a];
                }
              if (in && std::abs(lv_at(q[0], q[1], q[2]) - l) > 1)
                return "level map is not 2:1 balanced over neighbouring blocks";
            }
      }
  // solids keep two finest cells away from coarser territory
  for (int64_t z = 0; z < nz; ++z)
    for (int64_t y = 0; y < ny; ++y)
      for (int64_t x = 0; x < nx; ++x) {
        if (fluid[(size_t)(x + nx * (y + (int64_t)ny * z))]) continue;
        for (int dz = -2; dz <= 2; ++dz)
          for (int dy = -2; dy <= 2; ++dy)
            for (int dx = -2; dx <= 2; ++dx) {
              int q[3] = {(int)x + dx, (int)y + dy, (int)z + dz};
              if (B.wrap(0, q) && B.terr(0, q) > 0)
                return "solid voxels must stay two cells away from coarser levels";
            }
      }

  // ---- per level: active and jump masks, block maps
  levels.assign(L, MultiresLevel{});
  std::vector<std::vector<uint8_t>> act(L), jmp(L);
  for (int l = 0; l < L; ++l) {
    const int n0 = B.dim(l, 0), n1 = B.dim(l, 1), n2 = B.dim(l, 2);
    act[l].assign((size_t)n0 * n1 * n2, 0);
    jmp[l].assign((size_t)n0 * n1 * n2, 0);
    for (int z = 0; z < n2; ++z)
      for (int y = 0; y < n1; ++y)
        for (int x = 0; x < n0; ++x) {
          int p[3] = {x, y, z};
          if (!B.active(l, p)) continue;
          const size_t v = (size_t)x + (size_t)n0 * ((size_t)y + (size_t)n1 * z);
          act[l][v] = 1;
          bool j = false;
          // distance 0 to a resolution jump: some pulled neighbour lies in
          // coarser territory (explosion) or finer territory (coalescence)
          for (int i = 1; i < Q && !j; ++i) {
            int q[3] = {x - kCx[i], y - kCy[i], z - kCz[i]};
            if (B.wrap(l, q) && B.terr(l, q) != l) j = true;
          }
          if (j) {
            for (int a = 0; a < 3; ++a)
              if (!periodic[a] && (p[a] < 2 || p[a] >= B.dim(l, a) - 2))
                return "resolution jumps must stay two cells away from non-periodic faces";
            jmp[l][v] = 1;
          }
        }
    std::string e = build_block_level(levels[l].L, n0, n1, n2, periodic, act[l], faces, false, &jmp[l]);
    if (!e.empty()) return "level " + std::to_string(l) + ": " + e;
    levels[l].tau = 0.5 + (tau_coarsest - 0.5) * (double)(1 << (L - 1 - l));
    if (levels[l].L.nblocks * 64 > (int64_t)kSlotMask) return "too many slots for the jump tables";
  }

  // ---- jump tables
  auto slot_of = [&](int l, const int p[3]) -> uint32_t {
    const BlockLevel &BL = levels[l].L;
    const int64_t b = BL.slot_of_block[(size_t)(p[0] / 4 + BL.nbx * (p[1] / 4 + (int64_t)BL.nby * (p[2] / 4)))];
    return (uint32_t)(b * 64 + (p[0] & 3) + 4 * (p[1] & 3) + 16 * (p[2] & 3));
  };
  for (int l = 0; l < L; ++l) {
    MultiresLevel &M = levels[l];
    const BlockLevel &BL = M.L;
    const int64_t nj = BL.group_count[kGroupJump];
    M.jtab.assign((size_t)nj * 2 * Q * 64, 0);
    M.jlist.clear();
    for (int64_t s = 0; s < nj; ++s) {
      for (int lane = 0; lane < 64; ++lane) {
        int W[3] = {BL.coords[3 * s] * 4 + (lane & 3), BL.coords[3 * s + 1] * 4 + ((lane >> 2) & 3),
                    BL.coords[3 * s + 2] * 4 + (lane >> 4)};
        const uint32_t own = (uint32_t)(s * 64 + lane);
        const bool on = B.active(l, W);
        for (int ph = 0; ph < 2; ++ph) {
          const int sub = (l == L - 1) ? 0 : ph + 1;
          for (int i = 0; i < Q; ++i) {
            uint32_t &out = M.jtab[(((size_t)s * 2 + ph) * Q + i) * 64 + lane];
            if (!on || i == 0) {
              out = make_entry(kTagLevelCur, own, false);
              continue;
            }
            // same-resolution pull, with explosion from the coarser level
            auto plain = [&](uint32_t &e) -> std::string {
              int q[3] = {W[0] - kCx[i], W[1] - kCy[i], W[2] - kCz[i]};
              if (!B.wrap(l, q)) {
                const int face = [&] {
                  for (int a = 0; a < 3; ++a)
                    if (q[a] < 0) return 2 * a;
                    else if (q[a] >= B.dim(l, a)) return 2 * a + 1;
                  return 0;
                }();
                if (faces[face].kind != LBM_BC_BOUNCE_BACK)
                  return "a block next to a resolution jump touches a moving-wall or regularized face";
                e = make_entry(kTagLevelCur, own, true);
                return "";
              }
              const int t = B.terr(l, q);
              if (t == l) {
                e = B.active(l, q) ? make_entry(kTagLevelCur, slot_of(l, q), false)
                                   : make_entry(kTagLevelCur, own, true);
              } else if (t == l + 1) {
                if (sub == 1) {
                  int cq[3] = {q[0] >> 1, q[1] >> 1, q[2] >> 1};
                  e = make_entry(kTagCoarserCur, slot_of(l + 1, cq), false);
                } else {
                  int r[3] = {q[0] - kCx[i], q[1] - kCy[i], q[2] - kCz[i]};
                  if (!B.wrap(l, r)) return "re-entry path leaves the box";
                  if (B.terr(l, r) == l) {
                    e = make_entry(kTagLevelPrev, slot_of(l, r), false);
                  } else {
                    int cr[3] = {r[0] >> 1, r[1] >> 1, r[2] >> 1};
                    if (B.terr(l + 1, cr) != l + 1) return "explosion source is not on the coarser level";
                    e = make_entry(kTagCoarserCur, slot_of(l + 1, cr), false);
                  }
                }
              } else {
                return "unexpected finer source outside coalescence";
              }
              return "";
            };
            uint32_t list[8];
            bool any_fine = false;
            if (l > 0) {
              for (int d = 0; d < 8; ++d) {
                int p[3] = {2 * W[0] + (d & 1), 2 * W[1] + ((d >> 1) & 1), 2 * W[2] + (d >> 2)};
                int a1[3] = {p[0] - kCx[i], p[1] - kCy[i], p[2] - kCz[i]};
                int a2[3] = {p[0] - 2 * kCx[i], p[1] - 2 * kCy[i], p[2] - 2 * kCz[i]};
                list[d] = 0xffffffffu;
                if (B.wrap(l - 1, a1) && B.terr(l - 1, a1) == l - 1) {
                  list[d] = make_entry(kTagFinerCur, slot_of(l - 1, a1), false);
                  any_fine = true;
                } else if (B.wrap(l - 1, a2) && B.terr(l - 1, a2) == l - 1) {
                  list[d] = make_entry(kTagFinerPrev, slot_of(l - 1, a2), false);
                  any_fine = true;
                }
              }
            }
            uint32_t e = 0;
            std::string err = "";
            if (!any_fine) {
              err = plain(e);
              out = e;
            } else {
              uint32_t coarse = 0;
              bool have = false;
              for (int d = 0; d < 8 && err.empty(); ++d)
                if (list[d] == 0xffffffffu) {
                  if (!have) {
                    err = plain(coarse);
                    have = true;
                  }
                  list[d] = coarse;
                }
              const uint32_t idx = (uint32_t)(M.jlist.size() / 8);
              M.jlist.insert(M.jlist.end(), list, list + 8);
              out = make_entry(kTagList, idx, false);
            }
            if (!err.empty()) return "level " + std::to_string(l) + ": " + err;
          }
        }
      }
    }
  }
  return "";
}

}  // namespace lbm
