// Table written by the autotuner (tune_gfx950.txt next to the library): per
// (scheme, floor(log2 n)) the fastest measured swept tile shape (width and
// work-group size; lines "scheme log2n width threads") and classic work-group
// size (lines "classic scheme log2n threads").  Missing entries fall back to
// default_shape() and 256.
#pragma once

#include "swept.h"

namespace sw {

// Looks up (scheme, floor(log2 n)); returns false if absent or if the tuned
// width does not divide n.
bool tuned_shape(const sw_problem &p, int *width, int *threads);

// Classic work-group size of (scheme, floor(log2 n)), or of the nearest measured class.
bool tuned_classic_threads(const sw_problem &p, int *threads);

}  // namespace sw
