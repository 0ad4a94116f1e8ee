// Order in which the persistent trailing updates walk the lower tiles of the
// trailing matrix.
//
// A persistent grid of kXcds * kSuperTile^2 (= 512) workgroups takes slots
// b, b + 512, ...; workgroup b runs on XCD b % kXcds (the round-robin
// placement of one launch).  In each round of 512 slots the 64 slots of one
// XCD cover one super-tile of kSuperTile x kSuperTile tiles, so the
// workgroups of an XCD working at the same time stage the same 8 row blocks
// of L and 8 column blocks of W, which then come from that XCD's L2 rather
// than from memory.  Super-tiles (SI >= SJ) are taken in row-major order of
// the lower triangle; slots of a super-tile above the diagonal or past the
// last tile hold no tile.  Any other grid size walks the tiles in plain
// row-major triangular order.
#pragma once

#include <hip/hip_runtime.h>

namespace mds {

constexpr int kXcds = 8;
constexpr int kSuperTile = 8;
constexpr int kTileGrid = kXcds * kSuperTile * kSuperTile;

// triangular index x -> (ti >= tj), x = ti (ti + 1) / 2 + tj
__device__ inline void tri_of(long x, int &ti, int &tj) {
  int t = (int)((sqrt(8.0 * (double)x + 1.0) - 1.0) * 0.5);
  while ((long)(t + 1) * (t + 2) / 2 <= x) ++t;
  while ((long)t * (t + 1) / 2 > x) --t;
  ti = t;
  tj = (int)(x - (long)t * (t + 1) / 2);
}

// number of slots the walk visits for nt x nt tiles
__device__ inline long tile_slots(int nt, bool xcd) {
  if (!xcd) return (long)nt * (nt + 1) / 2;
  const long ns = (nt + kSuperTile - 1) / kSuperTile;
  const long sup = ns * (ns + 1) / 2;
  return (sup + kXcds - 1) / kXcds * (long)kTileGrid;
}

// slot x -> tile (ti, tj); false when the slot holds no tile
__device__ inline bool tile_of(long x, int nt, bool xcd, int &ti, int &tj) {
  if (!xcd) {
    tri_of(x, ti, tj);
    return ti < nt;
  }
  const long round = x / kTileGrid;
  const int r = (int)(x - round * kTileGrid);
  const int q = r % kXcds, idx = r / kXcds;
  const long s = round * kXcds + q;
  const long ns = (nt + kSuperTile - 1) / kSuperTile;
  if (s >= ns * (ns + 1) / 2) return false;
  int SI, SJ;
  tri_of(s, SI, SJ);
  ti = SI * kSuperTile + idx / kSuperTile;
  tj = SJ * kSuperTile + idx % kSuperTile;
  return ti < nt && tj <= ti;
}

// Tiles of one launch: part 0 every lower tile (in the order above),
// part 1 the first tile column (the near strip of the look-ahead), part 2
// the tiles right of it (ti >= tj >= 1, row-major).
__device__ inline long part_slots(int part, int nt, bool xcd) {
  if (part == 1) return nt;
  if (part == 2) return (long)(nt - 1) * nt / 2;
  return tile_slots(nt, xcd);
}
__device__ inline bool part_tile(int part, long x, int nt, bool xcd, int &ti, int &tj) {
  if (part == 1) {
    ti = (int)x;
    tj = 0;
    return ti < nt;
  }
  if (part == 2) {
    tri_of(x, ti, tj);
    ++ti;
    ++tj;
    return ti < nt;
  }
  return tile_of(x, nt, xcd, ti, tj);
}

}  // namespace mds
