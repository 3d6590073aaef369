// Velocity sets of the paper's Table 1 (Section 2.3) as compile-time tables.
//
// Order convention (the paper fixes only the groups): index 0 is the rest
// velocity, then opposite pairs (i, i+1) for odd i: the six faces, the twelve
// edges, the eight corners.  D3Q19 is the first 19 entries of D3Q27 and D3Q7
// the first 7, so a D3Q27 x D3Q19 pair shares direction indices 0..18.
#pragma once
#include <cstdint>

namespace stgv {

template <int Q> struct Stencil;

template <> struct Stencil<27> {
  static constexpr int q = 27;
  static constexpr int ex[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0,
                                 1, -1, 1, -1, 1, -1, -1, 1};
  static constexpr int ey[27] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1,
                                 1, -1, 1, -1, -1, 1, 1, -1};
  static constexpr int ez[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1,
                                 1, -1, -1, 1, 1, -1, 1, -1};
  // 8/27, 2/27, 1/54, 1/216
  static constexpr double w[27] = {
      8.0 / 27, 2.0 / 27, 2.0 / 27, 2.0 / 27, 2.0 / 27, 2.0 / 27, 2.0 / 27,
      1.0 / 54, 1.0 / 54, 1.0 / 54, 1.0 / 54, 1.0 / 54, 1.0 / 54, 1.0 / 54, 1.0 / 54,
      1.0 / 54, 1.0 / 54, 1.0 / 54, 1.0 / 54,
      1.0 / 216, 1.0 / 216, 1.0 / 216, 1.0 / 216, 1.0 / 216, 1.0 / 216, 1.0 / 216, 1.0 / 216};
  static constexpr double cs2 = 1.0 / 3.0;
};

template <> struct Stencil<19> {
  static constexpr int q = 19;
  static constexpr int ex[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  static constexpr int ey[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  static constexpr int ez[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  // 1/3, 1/18, 1/36
  static constexpr double w[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                                   1.0 / 18, 1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                   1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                   1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  static constexpr double cs2 = 1.0 / 3.0;
};

template <> struct Stencil<15> {
  static constexpr int q = 15;
  static constexpr int ex[15] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1};
  static constexpr int ey[15] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1};
  static constexpr int ez[15] = {0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1, 1, -1};
  // 2/9, 1/9, 1/72
  static constexpr double w[15] = {2.0 / 9,  1.0 / 9,  1.0 / 9,  1.0 / 9,  1.0 / 9,
                                   1.0 / 9,  1.0 / 9,  1.0 / 72, 1.0 / 72, 1.0 / 72,
                                   1.0 / 72, 1.0 / 72, 1.0 / 72, 1.0 / 72, 1.0 / 72};
  static constexpr double cs2 = 1.0 / 3.0;
};

template <> struct Stencil<7> {
  static constexpr int q = 7;
  static constexpr int ex[7] = {0, 1, -1, 0, 0, 0, 0};
  static constexpr int ey[7] = {0, 0, 0, 1, -1, 0, 0};
  static constexpr int ez[7] = {0, 0, 0, 0, 0, 1, -1};
  // 1/4, 1/8 with c_s = 1/2
  static constexpr double w[7] = {1.0 / 4, 1.0 / 8, 1.0 / 8, 1.0 / 8, 1.0 / 8, 1.0 / 8, 1.0 / 8};
  static constexpr double cs2 = 1.0 / 4.0;
};

// Opposite direction under the pairing convention above.
constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

}  // namespace stgv
