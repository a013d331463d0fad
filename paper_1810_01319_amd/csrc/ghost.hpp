// ghost.hpp -- indexing of the ghost shell of a block and the physical
// boundary map of a ghost cell's global index (device helpers shared by the
// refresh kernels and their adjoint).
#pragma once
#include <hip/hip_runtime.h>

#include "layout.hpp"

namespace amr {

// Flat ghost index -> padded (a, b, c): 3 full z-layers, N middle layers
// (3 full rows, N rows of 3+3 cells, 3 full rows), 3 full z-layers.
template <int N>
__device__ inline void ghost_decode(int g, int& a, int& b, int& c) {
  constexpr int M = N + 2 * kGhost;
  constexpr int L2 = M * M;
  constexpr int SLAB = 3 * L2;
  constexpr int MID = 6 * M + 6 * N;
  if (g < SLAB) {
    c = g / L2;
    const int r = g - c * L2;
    b = r / M;
    a = r - b * M;
    return;
  }
  g -= SLAB;
  if (g < N * MID) {
    const int cz = g / MID;
    int r = g - cz * MID;
    c = kGhost + cz;
    if (r < 3 * M) {
      b = r / M;
      a = r - b * M;
      return;
    }
    r -= 3 * M;
    if (r < 6 * N) {
      const int row = r / 6;
      const int t = r - row * 6;
      b = kGhost + row;
      a = t < 3 ? t : N + t;
      return;
    }
    r -= 6 * N;
    const int row = r / M;
    b = N + kGhost + row;
    a = r - row * M;
    return;
  }
  g -= N * MID;
  const int cz = g / L2;
  const int r = g - cz * L2;
  c = N + kGhost + cz;
  b = r / M;
  a = r - b * M;
}

template <int N>
__device__ inline int dir_code(int a, int b, int c) {
  const int sx = a < kGhost ? 0 : (a < N + kGhost ? 1 : 2);
  const int sy = b < kGhost ? 0 : (b < N + kGhost ? 1 : 2);
  const int sz = c < kGhost ? 0 : (c < N + kGhost ? 1 : 2);
  return sx + 3 * sy + 9 * sz;
}

// Phase-2 tasks of kind K (0: faces, 1: edges, 2: corners): a task is the
// ghost region of one direction (neighbour code) of one leaf, SIZE cells.
template <int N, int K>
struct P2Region {
  static constexpr int SIZE = K == 0 ? 3 * N * N : (K == 1 ? 9 * N : 27);
  // cells sharing one coarse parent: along a ghost axis the 3 cells form the
  // groups {1 cell, 2 cells} (low side) or {2, 1} (high side), along an
  // interior axis N / 2 pairs; GROUPS per region
  static constexpr int GROUPS = p2_groups(N, K);
  static constexpr int WAVES = p2_waves(N, K);  // a task takes whole waves
  static_assert(WAVES <= (1 << kP2SubBits), "wave-in-task index does not fit its bits");
};

// Group j along an axis of region class cl (0: low ghost slab, 1: interior,
// 2: high ghost slab): its first padded index and its number of cells.  The
// padded index a is the global index i N - 3 + a (N even), so the cells
// 2 p + 1, 2 p + 2 of the padded range share the coarse parent.
template <int N>
__device__ inline void p2_group(int cl, int j, int& first, int& n) {
  if (cl == 1) {
    first = kGhost + 2 * j;
    n = 2;
  } else if (cl == 0) {
    first = j == 0 ? 0 : 1;
    n = j == 0 ? 1 : 2;
  } else {
    first = j == 0 ? N + kGhost : N + kGhost + 2;
    n = j == 0 ? 2 : 1;
  }
}

// Global level-l index of a ghost cell after the physical boundary: periodic
// wraps, outflow clamps to the nearest domain cell.
template <int N>
__device__ inline int bc_index(const InstParams& ip, int l, int ax, int p) {
  const int n = (ip.root[ax] << l) * N;
  if (p >= 0 && p < n) return p;
  if (ip.bc[ax] == 0) return p < 0 ? p + n : p - n;
  return p < 0 ? 0 : n - 1;
}


}  // namespace amr
