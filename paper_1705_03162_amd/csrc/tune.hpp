// Tile-shape table written by the autotuner (tune_gfx950.txt next to the
// library): one line per (scheme, floor(log2 n)) with the fastest measured
// width and work-group size.  Missing entries fall back to default_shape().
#pragma once

#include "swept.h"

namespace sw {

// Looks up (scheme, floor(log2 n)); returns false if absent or if the tuned
// width does not divide n.
bool tuned_shape(const sw_problem &p, int *width, int *threads);

}  // namespace sw
