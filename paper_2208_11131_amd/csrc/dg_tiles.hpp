// dg_tiles.hpp -- launch tiles chosen by the autotuner (dg_tiles.inc), as a
// compile-time table: the host runtime takes its default tiles from it, and
// the instantiation units build one fixed-tile volume and face kernel per
// entry.
#pragma once
#include <stddef.h>

namespace dgk {

struct TileEntry {
    int dim, order, prec, phys, forced, vol_C, vol_T, face_C, face_T;
};

constexpr TileEntry kTiles[] = {
#include "dg_tiles.inc"
    {0, 0, 0, 0, 0, 0, 0, 0, 0}};

constexpr size_t kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]) - 1;

// Fixed-tile volume or face kernel of one table entry (host stubs of the
// single-box and the grouped variant), or null.
struct FixedVol {
    int order, phys, C, NT, forced;
    const void *fn;
    const void *fnb;
};

}  // namespace dgk
