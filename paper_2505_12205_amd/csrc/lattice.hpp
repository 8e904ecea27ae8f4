// lattice.hpp -- compile-time D2Q9 / D3Q19 tables for the gfx950 kernels.
//
// Velocity order is the column order of the moment matrices of the paper's
// appendix A (their momentum rows fix e_x, e_y, e_z); weights from Eq.
// weights (D3Q19) and the isotropic D2Q9 set 4/9, 1/9, 1/36.
#pragma once

namespace lbm {

template <int Q>
struct Lat;

template <>
struct Lat<9> {
  static constexpr int D = 2;
  static constexpr int AX = 1;  // streamwise axis of inlet/outlet (y)
  static constexpr int NH = 2;  // inlet unknowns with a tangential component
  static constexpr int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  static constexpr int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  static constexpr int ez[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  static constexpr float w[9] = {4.f / 9, 1.f / 9, 1.f / 9, 1.f / 9, 1.f / 9,
                                 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36};
  static constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
};

template <>
struct Lat<19> {
  static constexpr int D = 3;
  static constexpr int AX = 2;  // streamwise axis of inlet/outlet (z)
  static constexpr int NH = 4;
  static constexpr int ex[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  static constexpr int ey[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  static constexpr int ez[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  static constexpr float w[19] = {1.f / 3,  1.f / 18, 1.f / 18, 1.f / 18, 1.f / 18,
                                  1.f / 18, 1.f / 18, 1.f / 36, 1.f / 36, 1.f / 36,
                                  1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36,
                                  1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36};
  static constexpr int opp[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
};

template <int Q>
__host__ __device__ constexpr int ecomp(int a, int d) {
  return d == 0 ? Lat<Q>::ex[a] : (d == 1 ? Lat<Q>::ey[a] : Lat<Q>::ez[a]);
}

// index of the velocity with components (x, y, z); -1 if none
template <int Q>
__host__ __device__ constexpr int find_vel(int x, int y, int z) {
  for (int b = 0; b < Q; ++b)
    if (Lat<Q>::ex[b] == x && Lat<Q>::ey[b] == y && Lat<Q>::ez[b] == z) return b;
  return -1;
}

// velocity a with the components of the axes in `mask` (bit d) reversed
template <int Q>
__host__ __device__ constexpr int reflect(int a, int mask) {
  return find_vel<Q>((mask & 1) ? -Lat<Q>::ex[a] : Lat<Q>::ex[a],
                     (mask & 2) ? -Lat<Q>::ey[a] : Lat<Q>::ey[a],
                     (mask & 4) ? -Lat<Q>::ez[a] : Lat<Q>::ez[a]);
}

}  // namespace lbm
