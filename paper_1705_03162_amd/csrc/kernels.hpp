// Launchers of the HIP kernels in kernels.hip and swept_tile.hpp (host-callable).
#pragma once

#include <hip/hip_runtime.h>

#include "tile.hpp"

namespace sw {

// One swept phase: tiles 0 .. tiles-1 (all K tiles when tiles < 0), one work-group of
// `threads` lanes each, P points per lane.
hipError_t launch_swept_phase(int scheme, int P, int threads, const TileArgs &a, hipStream_t st,
                              int64_t tiles = -1);

// One swept phase of the Shared variant (lds_tile.hpp): the tile's two rows in LDS,
// `threads` lanes striding over each level's points, one barrier per level.  The rows
// take 2 nv (w + 2 r) doubles of LDS, at most kLdsTileMaxBytes.
constexpr int64_t kLdsTileMaxBytes = 160 * 1024;
// LDS per work-group of the Shared variant: rows [nv][2][w + 2r] doubles, the r halo
// positions on each side holding the neighbouring triangles' tips.
constexpr int64_t lds_tile_bytes(int nv, int r, int w) { return (int64_t)2 * nv * (w + 2 * r) * 8; }
hipError_t launch_lds_phase(int scheme, int threads, const TileArgs &a, hipStream_t st, int64_t tiles = -1);
// Raise the Shared-variant kernel's dynamic LDS limit to kLdsTileMaxBytes; call before
// the first launch (not during stream capture).
hipError_t prepare_lds_phase(int scheme);

// One classic sub-step over n points: src -> dst (in place on dst for a final RK2 stage),
// in work-groups of `threads` lanes (a multiple of 64 in [64, 1024]).
hipError_t launch_classic_level(int scheme, const double *src, double *dst, int64_t n, int bc,
                                int predictor, const Consts &c, int threads, hipStream_t st);

// One phase of many independent solves: items[i] = (solve index into desc, tile).
// global_phase >= 0 runs that phase for every solve, -1 each solve's own phase.
// `grid` one-wave work-groups stride over the items.
hipError_t launch_batch_phase(int scheme, int P, const SolveDesc *desc, const int2 *items, int64_t nitems,
                              int global_phase, int grid, hipStream_t st);

// Per-scheme launchers of the swept tile kernels, defined in swept_tile.hpp and
// instantiated for Heat, KS and Euler in tiles_heat.hip, tiles_ks.hip and
// tiles_euler.hip (the dispatch above calls them).
template <class Sch>
hipError_t swept_phase_for(int P, int threads, const TileArgs &a, hipStream_t st, int64_t tiles);
template <class Sch>
hipError_t batch_phase_for(int P, const SolveDesc *desc, const int2 *items, int64_t nitems, int global_phase,
                           int grid, hipStream_t st);
template <class Sch>
int batch_blocks_for(int P);

// Persistent batched launch of one (scheme, points per lane) group: see batch_persistent.
struct PersistArgs {
    const SolveDesc *desc;        // the group's solves
    const int2 *items;            // (solve, tile), solve by solve
    const int64_t *phase_start;   // [max_phases + 1]: first queue entry of each phase
    int32_t *done;                // per items entry: phases completed (zeroed before the launch)
    int32_t *finished;            // per solve: tiles done with the last phase (zeroed)
    uint64_t *stamps;             // per solve: device clock when its last tile finished
    unsigned long long *next;     // queue counter (zeroed)
    int32_t *error;               // set if a dependency wait gave up (zeroed)
    int32_t max_phases;
    int64_t spin_limit;
};
hipError_t launch_persistent_batch(int scheme, int P, const PersistArgs &q, int grid, hipStream_t st);
// Resident persistent work-groups per CU for (scheme, P).
int persistent_blocks_per_cu(int scheme, int P);
template <class Sch>
hipError_t persistent_phase_for(int P, const PersistArgs &q, int grid, hipStream_t st);
template <class Sch>
int persistent_blocks_for(int P);
// Zero `count` 32-bit words (a kernel, so that it can sit inside a captured graph).
hipError_t launch_zero_words(void *p, int64_t count, hipStream_t st);

// desc[i].phase += 1 for every solve i < n that has phases left (served ticks).
hipError_t launch_advance_phases(SolveDesc *desc, int64_t n, hipStream_t st);

// Writes the device wall clock (constant-rate counter) to stamps[idx].
hipError_t launch_stamp(uint64_t *stamps, int idx, hipStream_t st);

// Resident one-wave batch work-groups per CU for (scheme, P).
int batch_blocks_per_cu(int scheme, int P);

// Sets *flag to 1 if any of x[0..count) is not finite (flag must be zeroed first).
hipError_t launch_nonfinite_scan(const double *x, int64_t count, int *flag, hipStream_t st);

}  // namespace sw
