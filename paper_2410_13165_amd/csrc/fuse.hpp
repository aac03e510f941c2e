// Shared pieces of the two-step (fused) passes: tile shapes, the LDS plane
// slots of the step-1 values, and the tile order (kernels.hip forward passes,
// adjoint.hip adjoint passes).  D = 3 only; the passes march along x_3.
#pragma once

#include <hip/hip_runtime.h>

#include "engine.hpp"

namespace lbm {

// Compute units of the current device (cached per device; 256 on MI355X).
inline int device_cus() {
  static int cache[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cache[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n <= 0)
      n = 256;
    cache[dev] = n;
  }
  return cache[dev];
}

// x_3 planes per block.  The passes run one block per CU (the LDS holds one
// tile) and a block of zc planes takes zc + 2 iterations (it recomputes two
// step-1 planes beyond its own), so the pass takes about
// ceil(blocks / CUs) * (zc + 2) iteration times with blocks = tiles_xy *
// ceil(n2 / zc): the chunk is the zc <= 64 that minimises that (the largest
// on ties).  Large lattices get 64; small ones trade a little recomputation
// for a last round of blocks that is not nearly empty.
inline int fuse_zchunk(int tiles_xy, int n2) {
  const long long cus = device_cus();
  int best = 64;
  long long best_cost = -1;
  for (int zc = 64; zc >= 4; --zc) {
    const long long blocks = static_cast<long long>(tiles_xy) * ((n2 + zc - 1) / zc);
    const long long cost = (blocks + cus - 1) / cus * ((zc < n2 ? zc : n2) + 2);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = zc;
    }
  }
  return best;
}

// Tiles fill most of the 160 KB of LDS with one block per CU: SLOTS planes of
// (TX + 2) (TY + 2) values; a row of a tile is 256 B of one population plane.
template <class T, bool HALF>
struct FuseShape;
template <>
struct FuseShape<float, false> {
  static constexpr int TX = 64, TY = 13, NT = 1024, SLOTS = 38;
};
template <>
struct FuseShape<float, true> {
  static constexpr int TX = 64, TY = 11, NT = 896, SLOTS = 43;
};
template <>
struct FuseShape<double, false> {
  static constexpr int TX = 32, TY = 12, NT = 512, SLOTS = 38;
};
template <>
struct FuseShape<double, true> {
  static constexpr int TX = 32, TY = 12, NT = 512, SLOTS = 43;
};

// The forward pass with half-way x_1 walls needs, at an x_1-face node of
// output plane z - 1, the step-1 value f*_kbar of that node, for every kbar
// opposite an unknown k.  Of these only kbar = (-+1, 0, -1) has c_3 = -1,
// whose single plane slot the next plane overwrites, so the pass keeps that
// one value per face node in a side buffer (two faces x (TY + 2) rows x two
// plane parities) instead of a second slot for every c_3 = -1 population:
// its LDS has the full-way slots and tile.  (The split and adjoint passes
// keep the 43-slot layout of FuseShape<T, true>.)
template <class T, bool HALF>
struct FuseFwdShape : FuseShape<T, false> {
  static constexpr int SIDE = HALF ? 4 * (FuseShape<T, false>::TY + 2) : 0;
};

// index of population k among those with the same c_3
constexpr int cz_index(int k) {
  const int cz = vel_comp(3, k, 2);
  int idx = 0;
  for (int m = 0; m < k; ++m)
    if (vel_comp(3, m, 2) == cz) ++idx;
  return idx;
}

// LDS plane slot of population k for the step-1 plane produced at iteration it
// of a forward pass: step 2 on plane z reads k from plane z - c_3, so c_3 = +1
// values live three iterations, c_3 = 0 two and c_3 = -1 one (two with
// half-way walls, which also read the node's own opposite population).
template <bool HALF, int k>
__device__ __forceinline__ int fuse_slot(int it) {
  constexpr int cz = vel_comp(3, k, 2);
  constexpr int i = cz_index(k);
  if constexpr (cz == 0) return 2 * i + (it & 1);
  else if constexpr (cz == 1) return 18 + 3 * i + it % 3;
  else if constexpr (HALF) return 33 + 2 * i + (it & 1);
  else return 33 + i;
}

__device__ __forceinline__ int fuse_wrap(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// Region index (ry * (TX + 2) + rx, the tile and its halo of one) of phase-1
// work item t in [0, (TX + 2)(TY + 2)): the first TX * (TY + 2) items run along
// the interior columns 1..TX of each region row, so a wavefront's loads start
// on the tile's aligned x_1 origin instead of straddling two region rows; the
// last 2 (TY + 2) items are the halo columns 0 and TX + 1.  A bijection.
template <int TX, int TY>
__device__ __forceinline__ int fuse_region(int t) {
  constexpr int RX = TX + 2, RY = TY + 2;
  if (t < TX * RY) return (t / TX) * RX + 1 + t % TX;
  const int h = t - TX * RY;
  return (h >> 1) * RX + ((h & 1) ? TX + 1 : 0);
}

// Tile of this block.  Workgroups go to the 8 XCDs round-robin by index, so
// block b is given tile (b mod 8) * per + b / 8: each XCD walks a contiguous
// run of tiles in x_1-fastest order, and the tiles next to each other in x_1
// and x_2, whose halos read the same cache lines, run at the same time under
// one L2.
__device__ __forceinline__ void fuse_tile(const KParams& p, int TX, int TY, int& bx, int& by,
                                          int& bz) {
  const int gx = (p.n[0] + TX - 1) / TX, gy = (p.n[1] + TY - 1) / TY;
  const int nb = static_cast<int>(gridDim.x);
  const int per = nb / 8;
  const int b = static_cast<int>(blockIdx.x);
  const int t = (b < 8 * per) ? (b % 8) * per + b / 8 : b;
  bx = t % gx;
  by = (t / gx) % gy;
  bz = t / (gx * gy);
}

// The same for an adjoint pass, which reads k from plane z + c_3: the roles
// of c_3 = +1 and c_3 = -1 swap.
template <bool HALF, int k>
__device__ __forceinline__ int adj_slot(int it) {
  constexpr int cz = vel_comp(3, k, 2);
  constexpr int i = cz_index(k);
  if constexpr (cz == 0) return 2 * i + (it & 1);
  else if constexpr (cz == -1) return 18 + 3 * i + it % 3;
  else if constexpr (HALF) return 33 + 2 * i + (it & 1);
  else return 33 + i;
}

// ---- d = 2: 1-D tiles along x_1 marching along x_2 (the same plan with
// planes replaced by rows).  The c_2 classes of D2Q9 have three members each.
template <class T, bool HALF>
struct FuseShape2 {
  // 256 outputs (lattice sizes are often multiples); threads 0 and 1 also
  // take the two halo nodes of the step-1 row
  static constexpr int TX = 256, NT = 256, SLOTS = HALF ? 21 : 18;
};

constexpr int cy_index(int k) {
  const int cy = vel_comp(2, k, 1);
  int idx = 0;
  for (int m = 0; m < k; ++m)
    if (vel_comp(2, m, 1) == cy) ++idx;
  return idx;
}

template <bool HALF, int k>
__device__ __forceinline__ int fuse_slot2(int it) {
  constexpr int cy = vel_comp(2, k, 1);
  constexpr int i = cy_index(k);
  if constexpr (cy == 0) return 2 * i + (it & 1);
  else if constexpr (cy == 1) return 6 + 3 * i + it % 3;
  else if constexpr (HALF) return 15 + 2 * i + (it & 1);
  else return 15 + i;
}

// x_2 rows per block: 64, halved (down to 8) while the grid has fewer than
// four blocks per CU
__host__ __device__ constexpr int fuse_ychunk(int tiles_x, int n1) {
  int yc = 64;
  while (yc > 8 && tiles_x * ((n1 + yc - 1) / yc) < 4 * 256) yc /= 2;
  return yc;
}

// tile of this block for d = 2, in the XCD-aware order of fuse_tile
__device__ __forceinline__ void fuse_tile2(const KParams& p, int TX, int& bx, int& by) {
  const int gx = (p.n[0] + TX - 1) / TX;
  const int nb = static_cast<int>(gridDim.x);
  const int per = nb / 8;
  const int b = static_cast<int>(blockIdx.x);
  const int t = (b < 8 * per) ? (b % 8) * per + b / 8 : b;
  bx = t % gx;
  by = t / gx;
}

}  // namespace lbm
