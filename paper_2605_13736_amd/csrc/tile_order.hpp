// Order in which the persistent trailing updates walk the lower tiles of the
// trailing matrix.
//
// A persistent grid whose size is a multiple of kXcds takes slots b,
// b + grid, ...; workgroup b runs on XCD b % kXcds (the round-robin placement
// of one launch), so slot x belongs to XCD x % kXcds and is entry x / kXcds
// of that XCD's queue.  The queue of XCD q holds the super-tiles q, q + kXcds,
// q + 2 kXcds, ... (kSuperTile x kSuperTile tiles each, super-tiles SI >= SJ
// in row-major order of the lower triangle), tile by tile, so the workgroups
// of an XCD working at the same time stage the same few row blocks of L and
// column blocks of W, which then come from that XCD's L2 rather than from
// memory.  Entries above the diagonal or past the last tile hold no tile.
// Any other grid size walks the tiles in plain row-major triangular order.
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
  return (sup + kXcds - 1) / kXcds * (long)(kXcds * kSuperTile * kSuperTile);
}

// slot x -> tile (ti, tj); false when the slot holds no tile
__device__ inline bool tile_of(long x, int nt, bool xcd, int &ti, int &tj) {
  if (!xcd) {
    tri_of(x, ti, tj);
    return ti < nt;
  }
  constexpr int kPer = kSuperTile * kSuperTile;
  const int q = (int)(x % kXcds);
  const long e = x / kXcds;  // entry of XCD q's queue
  const long s = (e / kPer) * kXcds + q;
  const int idx = (int)(e % kPer);
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
// the rest (part 2) walks the triangle of the tiles from (1, 1) on, in the
// order above.
__device__ inline long part_slots(int part, int nt, bool xcd) {
  if (part == 1) return nt;
  if (part == 2) return tile_slots(nt - 1, xcd);
  return tile_slots(nt, xcd);
}
__device__ inline bool part_tile(int part, long x, int nt, bool xcd, int &ti, int &tj) {
  if (part == 1) {
    ti = (int)x;
    tj = 0;
    return ti < nt;
  }
  if (part == 2) {
    const bool ok = tile_of(x, nt - 1, xcd, ti, tj);
    ++ti;
    ++tj;
    return ok;
  }
  return tile_of(x, nt, xcd, ti, tj);
}

}  // namespace mds
