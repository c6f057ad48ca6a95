// Launchers of the HIP kernels in kernels.hip (host-callable).
#pragma once

#include <hip/hip_runtime.h>

#include "tile.hpp"

namespace sw {

// One swept phase: K work-groups of `threads` lanes, P points per lane.
hipError_t launch_swept_phase(int scheme, int P, int threads, const TileArgs &a, hipStream_t st);

// One classic sub-step over n points: src -> dst (in place on dst for a final RK2 stage).
hipError_t launch_classic_level(int scheme, const double *src, double *dst, int64_t n, int dirichlet,
                                int predictor, const Consts &c, hipStream_t st);

// Sets *flag to 1 if any of x[0..count) is not finite (flag must be zeroed first).
hipError_t launch_nonfinite_scan(const double *x, int64_t count, int *flag, hipStream_t st);

}  // namespace sw
