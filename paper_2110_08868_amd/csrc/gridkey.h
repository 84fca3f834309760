// Neighbour-grid cell coordinates and keys, shared by the grid build and the
// clip kernel (both must place a point in the same cell).
#pragma once

#include "common.h"

namespace mak {

// Cell coordinate of a wrapped coordinate x in [0, L): floor(x / h), clamped.
__device__ __forceinline__ int cell_coord(double x, double h, int Gn) {
  int c = int(x / h);
  return c < 0 ? 0 : (c >= Gn ? Gn - 1 : c);
}

// Block-major key: the 4x4x4 cells of one block are contiguous, blocks in
// x-major order.  Gn = 4 * Gb.
__device__ __forceinline__ int64_t cell_key(int cx, int cy, int cz, int Gb) {
  const int64_t blk = (int64_t(cx >> 2) * Gb + (cy >> 2)) * Gb + (cz >> 2);
  return blk * 64 + (((cx & 3) << 4) | ((cy & 3) << 2) | (cz & 3));
}

__device__ __forceinline__ int64_t block_key(int bx, int by, int bz, int Gb) {
  return (int64_t(bx) * Gb + by) * Gb + bz;
}

}  // namespace mak
