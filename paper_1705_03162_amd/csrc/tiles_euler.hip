// Swept tile kernels of the Euler equations (Sod): every points-per-lane variant of the
// single-solve kernel (one-wave and multi-wave work-groups) and of the batched kernel.
#include "swept_tile.hpp"

namespace sw {

template hipError_t swept_phase_for<Euler>(int, int, const TileArgs &, hipStream_t, int64_t);
template hipError_t batch_phase_for<Euler>(int, const SolveDesc *, const int2 *, int64_t, int, int, hipStream_t);
template int batch_blocks_for<Euler>(int);
template hipError_t persistent_phase_for<Euler>(int, const PersistArgs &, int, hipStream_t);
template int persistent_blocks_for<Euler>(int);

}  // namespace sw
