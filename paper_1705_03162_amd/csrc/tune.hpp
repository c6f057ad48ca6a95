// Table written by the autotuner (tune_gfx950.txt next to the library): per
// (scheme, floor(log2 n)) the fastest measured swept tile shape (width and
// work-group size; lines "scheme log2n width threads"), classic work-group size
// (lines "classic scheme log2n threads") and points per lane of batched one-wave
// tiles (lines "batch scheme log2n points").  Missing entries fall back to
// default_shape(), 256 and the most points per lane that divide n.
#pragma once

#include "swept.h"

namespace sw {

// Looks up (scheme, floor(log2 n)); returns false if absent or if the tuned
// width does not divide n.
bool tuned_shape(const sw_problem &p, int *width, int *threads);

// Classic work-group size of (scheme, floor(log2 n)), or of the nearest measured class.
bool tuned_classic_threads(const sw_problem &p, int *threads);

// Points per lane of batched tiles for (scheme, floor(log2 n)), or of the nearest measured class.
bool tuned_batch_points(const sw_problem &p, int *points);

}  // namespace sw
