// D3Q19 velocity set of the library (host and device).
//
// Order: 0 rest; 1..6 faces +x,-x,+y,-y,+z,-z; 7..18 edges in opposite
// pairs.  Weights 1/3 (rest), 1/18 (faces), 1/36 (edges); c_s^2 = 1/3
// (the lattice of the evaluation section, textbook form).
#pragma once
#include <cstdint>

#if defined(__HIPCC__)
#define LBM_HD __host__ __device__
#else
#define LBM_HD
#endif

namespace lbm {

constexpr int Q = 19;
constexpr int kCx[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int kCy[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int kCz[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
constexpr int kOpp[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};

LBM_HD constexpr double weight_d(int i) {
  return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
}
LBM_HD constexpr float weight_f(int i) {
  return i == 0 ? 1.0f / 3.0f : (i < 7 ? 1.0f / 18.0f : 1.0f / 36.0f);
}

// Direction index of a lattice vector, -1 if it is not in the set.
LBM_HD constexpr int dir_of(int cx, int cy, int cz) {
  for (int i = 0; i < Q; ++i)
    if (kCx[i] == cx && kCy[i] == cy && kCz[i] == cz) return i;
  return -1;
}

}  // namespace lbm
