// Velocity sets of the library (host and device).
//
// D3Q19: 0 rest; 1..6 faces +x,-x,+y,-y,+z,-z; 7..18 edges in opposite
// pairs; weights 1/3, 1/18, 1/36 (the lattice of the evaluation section).
// D3Q27: the D3Q19 order followed by the 8 corners in opposite pairs
// 19..26; weights 8/27, 2/27, 1/54, 1/216 (the lattice of the block-sparse
// register study).  c_s^2 = 1/3 for both.
//
// Device code is compiled once per lattice: with LBM_Q27 defined the
// kernels see D3Q27 as the current lattice, otherwise D3Q19.  The current
// lattice lives in an inline namespace (k19 / k27) so that the two builds
// of every kernel and helper carry different symbol names and can be linked
// into one library; host code reaches either set by its namespace.
#pragma once
#include <cstdint>

#if defined(__HIPCC__)
#define LBM_HD __host__ __device__
#else
#define LBM_HD
#endif

namespace lbm {

namespace d3q19 {
constexpr int Q = 19;
constexpr int kCx[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int kCy[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int kCz[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
constexpr int kOpp[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
LBM_HD constexpr double weight_d(int i) { return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }
LBM_HD constexpr float weight_f(int i) { return i == 0 ? 1.0f / 3.0f : (i < 7 ? 1.0f / 18.0f : 1.0f / 36.0f); }
}  // namespace d3q19

namespace d3q27 {
constexpr int Q = 27;
constexpr int kCx[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0,
                        1, -1, 1, -1, 1, -1, -1, 1};
constexpr int kCy[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1,
                        1, -1, 1, -1, -1, 1, 1, -1};
constexpr int kCz[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1,
                        1, -1, -1, 1, 1, -1, 1, -1};
constexpr int kOpp[Q] = {0,  2,  1,  4,  3,  6,  5,  8,  7,  10, 9,  12, 11, 14,
                         13, 16, 15, 18, 17, 20, 19, 22, 21, 24, 23, 26, 25};
LBM_HD constexpr double weight_d(int i) {
  return i == 0 ? 8.0 / 27.0 : (i < 7 ? 2.0 / 27.0 : (i < 19 ? 1.0 / 54.0 : 1.0 / 216.0));
}
LBM_HD constexpr float weight_f(int i) {
  return i == 0 ? 8.0f / 27.0f : (i < 7 ? 2.0f / 27.0f : (i < 19 ? 1.0f / 54.0f : 1.0f / 216.0f));
}
}  // namespace d3q27

#ifdef LBM_Q27
#define LBM_LATTICE_NS k27
// reopen either lattice's namespace with the inline-ness it has in this build
#define LBM_NAMESPACE_K19 namespace k19
#define LBM_NAMESPACE_K27 inline namespace k27
inline namespace k27 {
using namespace d3q27;
#else
#define LBM_LATTICE_NS k19
#define LBM_NAMESPACE_K19 inline namespace k19
#define LBM_NAMESPACE_K27 namespace k27
inline namespace k19 {
using namespace d3q19;
#endif

// Direction index of a lattice vector in the current set, -1 if absent.
LBM_HD constexpr int dir_of(int cx, int cy, int cz) {
  for (int i = 0; i < Q; ++i)
    if (kCx[i] == cx && kCy[i] == cy && kCz[i] == cz) return i;
  return -1;
}
constexpr int kNbr = Q - 1;  // neighbour blocks a block pulls from (one per direction)

}  // inline namespace

// Host description of either lattice (the grid builder takes it at run time).
struct LatticeDesc {
  int q;
  const int *cx, *cy, *cz, *opp;
  int dir(int x, int y, int z) const {
    for (int i = 0; i < q; ++i)
      if (cx[i] == x && cy[i] == y && cz[i] == z) return i;
    return -1;
  }
};
inline LatticeDesc lattice_desc(int q) {
  if (q == 27) return {27, d3q27::kCx, d3q27::kCy, d3q27::kCz, d3q27::kOpp};
  return {19, d3q19::kCx, d3q19::kCy, d3q19::kCz, d3q19::kOpp};
}

}  // namespace lbm
